"""Error measures of Appendix B and related checks.

With the ALF sign convention (+lam^T (A(X) - b)) the dual multiplier of the
standard-form dual max b^T y s.t. C - A*(y) PSD is y = -lam, so the dual slack
is S = C + A*(lam).  The appendix writes the smallest singular value of the
slack; since min{0, .} of a singular value is always 0 the only meaningful
reading is the smallest eigenvalue, which is what is computed.

  primal infeasibility  ||A(X) - b||_2 / (1 + ||b||_1)
  dual infeasibility    |min(0, lambda_min(C - A*(y)))| / (1 + ||vec C||_1)
  primal-dual gap       (<C, X> - b^T y) / (1 + |<C, X>| + |b^T y|)

For the quadratic objective f(X) = <C, X> + (mu/2) ||X||_F^2 (Section 1's
convex f) the same measures are taken at the linearisation of f at X: C is
replaced by grad f(X) = C + mu X in the slack (S = grad f(X) + A*(lam)) and
<C, X> by <grad f(X), X> in the gap, which then measures the complementarity
<S, X> of the KKT conditions; the objective reported is f(X).  With mu = 0
these are the measures above.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import operators


def lambda_min(prob, lam, U=None) -> float:
    """Smallest eigenvalue of C + A*(lam), plus mu U U^T for the quadratic
    objective (U: the solution factor)."""
    S = operators.assemble(prob, lam, 1.0)
    mu = operators.mu_of(prob)
    if mu != 0.0 and U is None:
        raise ValueError("the quadratic objective's slack needs the solution factor")
    if prob.n <= 2500:
        Sd = S.toarray()
        if mu != 0.0:
            Sd = Sd + mu * (U @ U.T)
        return float(np.linalg.eigvalsh(Sd)[0])
    op = S
    if mu != 0.0:
        op = spla.LinearOperator((prob.n, prob.n), dtype=np.float64,
                                 matvec=lambda x: S @ x + mu * (U @ (U.T @ x)))
    vals = spla.eigsh(op, k=1, which="SA", tol=1e-10, maxiter=20000,
                      v0=np.ones(prob.n) / np.sqrt(prob.n))[0]
    return float(vals[0])


def appendix_b(prob, U, lam):
    nrm = operators.norms(prob)
    z = operators.forward(prob, U, U)
    obj = operators.objective(prob, U, U)
    # <grad f(X), X> = <C, X> + mu ||X||_F^2
    gx = operators.cost_inner(prob, U, U)
    mu = operators.mu_of(prob)
    if mu != 0.0:
        G = U.T @ U
        gx += mu * float(np.sum(G * G))
    y = -np.asarray(lam)
    by = float(prob.b @ y)
    lmin = lambda_min(prob, lam, U)
    return dict(
        obj=obj,
        dual_obj=by,
        pinf=float(np.linalg.norm(z - prob.b)) / (1.0 + nrm["b_1"]),
        pinf_inf=float(np.linalg.norm(z - prob.b)) / (1.0 + nrm["b_inf"]),
        dinf=abs(min(0.0, lmin)) / (1.0 + nrm["c_1"]),
        gap=(gx - by) / (1.0 + abs(gx) + abs(by)),
        lambda_min=lmin,
    )


def mc_recovery_error(prob, U, block: int = 1024):
    """||U1 U2^T - M||_F / ||M||_F with M = L R^T (the off-diagonal block of
    X = U U^T estimates M under the halved completion scaling).

    The definition written out: the difference U1 U2^T - L R^T is formed
    entry by entry, a block of rows at a time, and its squared entries summed,
    so no large quantity is subtracted from another."""
    n1 = prob.meta["n1"]
    L, R = prob.meta["L"], prob.meta["R"]
    U1, U2 = U[:n1], U[n1:]
    num = den = 0.0
    for j0 in range(0, n1, block):
        M = L[j0:j0 + block] @ R.T
        E = U1[j0:j0 + block] @ U2.T - M
        num += float(np.sum(E * E))
        den += float(np.sum(M * M))
    return float(np.sqrt(num / den))


def gram(A, B, block: int = 4096):
    """G = A^T B for tall factors A (n x ra), B (n x rb): the sum over rows j of
    the outer products A_j^T B_j, a block of rows at a time."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    G = np.zeros((A.shape[1], B.shape[1]))
    for j0 in range(0, A.shape[0], block):
        G += A[j0:j0 + block].T @ B[j0:j0 + block]
    return G
