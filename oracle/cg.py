"""Conjugate gradients on the n x r matrix space (Section 4.4).

The ADMM subproblems (linU)/(linV) are symmetric positive definite systems
(gamma I + rho sum_i a_i a_i^T) x = rhs with a_i = vec(A_i W).  Applied
matrix-free, the operator is

    M_W(P) = gamma P + rho A*(A(P W^T)) W,

because <a_i, vec P> = <A_i W, P> = <A_i, P W^T>.  The paper solves these systems
by unpreconditioned CG warm-started at the other factor; writing x = x0 + D, the
oracle runs textbook CG on M_W D = R0 from D = 0, where R0 = rhs - M_W(x0).
Inner product: Frobenius.  Stop: ||R||_F <= tol * ||R0||_F or maxit.
"""
from __future__ import annotations

import numpy as np

from . import operators


def cg_operator(prob, W: np.ndarray, rho: float, gamma: float):
    """M_W(P) = gamma P + rho A*(A(P W^T)) W, plus mu P (W^T W) for the
    quadratic objective (mu/2) ||X||_F^2."""
    mu = operators.mu_of(prob)
    G = W.T @ W if mu != 0.0 else None

    def apply(P):
        t = operators.forward(prob, P, W)
        out = gamma * P + operators.adjoint(prob, rho * t, 0.0, W)
        if G is not None:
            out = out + mu * (P @ G)
        return out
    return apply


def cg(apply_M, R0: np.ndarray, tol: float, maxit: int):
    """Textbook CG from D = 0.  Returns (D, iterations, ||R||/||R0||, residual
    norms)."""
    D = np.zeros_like(R0)
    R = R0.copy()
    rr = float(np.sum(R * R))
    rr0 = rr
    hist = [np.sqrt(rr)]
    if rr0 == 0.0:
        return D, 0, 0.0, hist
    P = R.copy()
    it = 0
    while it < maxit and rr > tol * tol * rr0:
        Q = apply_M(P)
        pq = float(np.sum(P * Q))
        if pq <= 0.0:
            break
        alpha = rr / pq
        D += alpha * P
        R -= alpha * Q
        rr_new = float(np.sum(R * R))
        beta = rr_new / rr
        rr = rr_new
        P = R + beta * P
        it += 1
        hist.append(np.sqrt(rr))
    return D, it, float(np.sqrt(rr / rr0)), hist
