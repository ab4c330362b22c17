"""Per-family parameters of Section 5.1 used by callers of the library.

The switching tolerance of Phase I is 1e-3, the paper's setting for most
instances; the paper's lenient 1e-2 for MaxCut belongs to its stop on primal
infeasibility alone (1e-5), and under the full eq. (stop) at 1e-6 it leaves
slowly decaying factor columns to the ADMM.  The factor h applied to rho at the
switch depends on the family: MaxCut h = 10; matrix completion h = 5 below order
10000, 2.5 from there on; other problems h = 1.  The Lovasz theta family takes
the gamma rule on the cost's operator norm (gamma_rule 1).  The L-BFGS memory of Phase I
(left open by the paper) is 4.  The
initial rank is ceil(log2 n) for MaxCut (the rule of the MaxCut experiments),
round(ln m) for completion instances of order >= 10000 and round(2 ln m) otherwise.
"""
from __future__ import annotations

import math


def family_params(kind: str, n: int) -> dict:
    if kind == "maxcut":
        return dict(switch_tol=1e-3, h=10.0, lbfgs_mem=4)
    if kind == "mc":
        return dict(switch_tol=1e-3, h=5.0 if n < 10000 else 2.5, lbfgs_mem=4)
    if kind == "partition":  # graph partition and bisection: h = 10 (Section 5.1)
        return dict(switch_tol=1e-3, h=10.0, lbfgs_mem=4)
    if kind == "theta":  # Lovasz theta: gamma from the cost's operator norm (gamma_rule 1)
        return dict(switch_tol=1e-3, h=1.0, lbfgs_mem=4, gamma_rule=1)
    return dict(switch_tol=1e-3, h=1.0, lbfgs_mem=4)


def initial_rank(kind: str, n: int, m: int) -> int:
    if kind == "maxcut":
        return int(math.ceil(math.log2(n)))
    if kind == "mc" and n >= 10000:
        return int(round(math.log(m)))
    return int(round(2.0 * math.log(m)))


def solver_options(kind: str, n: int, r0: int, precision: int = 0, **kw):
    """lorads_options with the family's switch tolerance and h."""
    from .lorads import default_options
    fp = family_params(kind, n)
    fp.update(kw)
    return default_options(r0=r0, precision=precision, **fp)
