"""The constraint operator and its adjoint, from their definitions (FP64).

Section 1 defines A(X) = (<A_1, X>, ..., <A_m, X>).  For X = U V^T and a
symmetric A_i given by upper-triangle triplets (j, k, a):

    <A_i, U V^T> = sum_{j,k} (A_i)_{jk} <U_j, V_k>
                 = sum over triplets of a <U_j, V_k> + [j != k] a <U_k, V_j>.

The adjoint applied to a factor, (c C + A*(w)) V with A*(w) = sum_i w_i A_i,
assembles the symmetric sparse matrix c C + sum_i w_i A_i entry by entry
(off-diagonal triplets placed at (j, k) and (k, j), duplicates summed) and
multiplies it with V.  These are the products in eqs. (optU), (optV) and the
right-hand sides of (linU)/(linV).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_CHUNK = 1 << 20


def forward(prob, U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """z_i = <A_i, U V^T> for every constraint i."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    z = np.zeros(prob.m)
    nnz = prob.a_nnz
    for s in range(0, nnz, _CHUNK):
        e = slice(s, min(nnz, s + _CHUNK))
        j, k, a, i = prob.a_row[e], prob.a_col[e], prob.a_val[e], prob.a_con[e]
        d_jk = np.einsum("ij,ij->i", U[j], V[k])
        d_kj = np.einsum("ij,ij->i", U[k], V[j])
        t = a * np.where(j == k, d_jk, d_jk + d_kj)
        z += np.bincount(i, weights=t, minlength=prob.m)
    return z


def cost_inner(prob, U: np.ndarray, V: np.ndarray) -> float:
    """<C, U V^T> by the same triplet rule."""
    j, k, c = prob.c_row, prob.c_col, prob.c_val
    d_jk = np.einsum("ij,ij->i", U[j], V[k])
    d_kj = np.einsum("ij,ij->i", U[k], V[j])
    return float(np.sum(c * np.where(j == k, d_jk, d_jk + d_kj)))


def mu_of(prob) -> float:
    return float(getattr(prob, "mu", 0.0))


def objective(prob, U: np.ndarray, V: np.ndarray) -> float:
    """f(U V^T) for f(X) = <C, X> + (mu / 2) ||X||_F^2 (Section 1 allows any
    convex smooth f; this is the quadratic one), with
    ||U V^T||_F^2 = <U^T U, V^T V>."""
    mu = mu_of(prob)
    val = cost_inner(prob, U, V)
    if mu != 0.0:
        val += 0.5 * mu * float(np.sum((U.T @ U) * (V.T @ V)))
    return val


def grad_apply(prob, U: np.ndarray, V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """grad f(U V^T) W = C W + mu U (V^T W)."""
    out = cost_apply(prob, W)
    mu = mu_of(prob)
    if mu != 0.0:
        out = out + mu * (U @ (V.T @ W))
    return out


def assemble(prob, w: np.ndarray, c_scale: float) -> sp.csr_matrix:
    """The symmetric sparse matrix c_scale * C + sum_i w_i A_i."""
    w = np.asarray(w, dtype=np.float64)
    rows = [prob.c_row, prob.a_row]
    cols = [prob.c_col, prob.a_col]
    vals = [c_scale * prob.c_val, w[prob.a_con] * prob.a_val]
    off_c = prob.c_row != prob.c_col
    off_a = prob.a_row != prob.a_col
    rows += [prob.c_col[off_c], prob.a_col[off_a]]
    cols += [prob.c_row[off_c], prob.a_row[off_a]]
    vals += [c_scale * prob.c_val[off_c], (w[prob.a_con] * prob.a_val)[off_a]]
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    v = np.concatenate(vals)
    return sp.coo_matrix((v, (r, c)), shape=(prob.n, prob.n)).tocsr()


def adjoint(prob, w: np.ndarray, c_scale: float, V: np.ndarray) -> np.ndarray:
    """(c_scale * C + A*(w)) V."""
    S = assemble(prob, w, c_scale)
    return np.asarray(S @ np.asarray(V, dtype=np.float64))


def cost_apply(prob, V: np.ndarray) -> np.ndarray:
    """C V."""
    return adjoint(prob, np.zeros(prob.m), 1.0, V)


def cost_norm2(prob) -> float:
    """||C||_2, the largest eigenvalue magnitude of the dense symmetric C."""
    from .dense import dense_C
    C = dense_C(prob)
    return float(np.max(np.abs(np.linalg.eigvalsh(C)))) if prob.n else 0.0


def norms(prob):
    """||b||_inf, ||b||_1 and the Frobenius and entrywise-1 norms of C (full
    symmetric matrix: off-diagonal triplets count twice)."""
    twice = np.where(prob.c_row == prob.c_col, 1.0, 2.0)
    c_fro = float(np.sqrt(np.sum(twice * prob.c_val ** 2)))
    c_l1 = float(np.sum(twice * np.abs(prob.c_val)))
    b = prob.b
    return dict(b_inf=float(np.max(np.abs(b))) if b.size else 0.0,
                b_1=float(np.sum(np.abs(b))), b_2=float(np.linalg.norm(b)),
                c_fro=c_fro, c_1=c_l1)
