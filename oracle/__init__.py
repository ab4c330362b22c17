"""CPU oracle for the LoRADS hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 numpy implementation of what the GPU library computes, written
from the paper ("A Low-Rank ADMM Splitting Approach for Semidefinite
Programming"): the sparse constraint operator and its adjoint (Section 1, the
definition of the linear map), the ADMM of Algorithm 1 with the CG subproblem
solves of eqs. (linU)/(linV) (Section 4.4), the Burer-Monteiro augmented
Lagrangian warm start with dynamic rank (Sections 4.1-4.3, 5.1), the two-phase
driver of Algorithm 2 and the error measures of Appendix B.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it, links it or reads its
output; the two share no code beyond the seeded instance generators in `sdpgen`.

Where the paper is silent the oracle follows the documented readings listed in
`oracle/options.py` (the same rules the GPU library implements independently).

Parity status: every function here is pinned by `tests/test_oracle_*.py`
(closed forms, brute-force dense evaluation, textbook solvers, exact identities);
there is no function marked "parity unpinned".
"""
from .options import Options  # noqa: F401
from . import operators, cg, admm, alm, lorads, metrics, rng, dense  # noqa: F401
