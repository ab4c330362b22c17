"""Result measures computed with the library's Gram kernel (FP64 MFMA).

completion_recovery_error: for a planted completion M = L R^T and the solution
factor U_hat of order n1 + n2 (X = U_hat U_hat^T), the relative error
||U1 U2^T - M||_F / ||M||_F of the off-diagonal block, expanded into r x r and
r x k Gram products so that no n1 x n2 matrix is formed:
||U1 U2^T - L R^T||^2 = <U1^T U1, U2^T U2> - 2 <L^T U1, R^T U2> + <L^T L, R^T R>.
"""
from __future__ import annotations

import numpy as np


def completion_recovery_error(U_hat: np.ndarray, L: np.ndarray, R: np.ndarray) -> float:
    import torch
    from .lorads import gram
    dev = torch.device("cuda")
    n1 = L.shape[0]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    U1, U2, Ld, Rd = t(U_hat[:n1]), t(U_hat[n1:]), t(L), t(R)

    def g(A, B):
        G = torch.empty((A.shape[1], B.shape[1]), dtype=torch.float64, device=dev)
        gram(A, B, G)
        torch.cuda.synchronize()
        return G.cpu().numpy()

    e2 = np.sum(g(U1, U1) * g(U2, U2)) - 2.0 * np.sum(g(Ld, U1) * g(Rd, U2))
    m2 = np.sum(g(Ld, Ld) * g(Rd, Rd))
    # the identity subtracts quantities of size ||M||^2: errors below about
    # 1e-8 relative are not resolved (reported as 0)
    return float(np.sqrt(max(e2 + m2, 0.0) / m2))


def completion_recovery_error_sampled(U_hat: np.ndarray, L: np.ndarray, R: np.ndarray,
                                      cells: int = 1_000_000, seed: int = 0) -> float:
    """The same relative error estimated on `cells` uniformly drawn entries of M,
    each compared directly (no cancellation): sqrt(sum (X_jk - M_jk)^2 / sum M_jk^2)."""
    n1, n2 = L.shape[0], R.shape[0]
    rng = np.random.default_rng(seed)
    j = rng.integers(0, n1, cells)
    k = rng.integers(0, n2, cells)
    x = np.einsum("ij,ij->i", U_hat[j], U_hat[n1 + k])
    mv = np.einsum("ij,ij->i", L[j], R[k])
    return float(np.sqrt(np.sum((x - mv) ** 2) / np.sum(mv ** 2)))
