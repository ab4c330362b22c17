"""Pins of the oracle's CG on the subproblem systems (CPU only).

References: the dense nr x nr system of (linU) built from vec(A_i W) and
solved by LU (textbook); the MaxCut closed form (the system is block diagonal
with r x r blocks gamma I + rho a a^T, inverted by Sherman-Morrison); the
two-eigenvalue termination of CG; mutual orthogonality of CG residuals.
"""
import numpy as np
import pytest

import oracle
import sdpgen
from oracle import dense
from oracle.cg import cg, cg_operator


def _dense_system(p, W, rho, gamma):
    n, r = W.shape
    A = dense.dense_A(p)
    cols = np.stack([(A[i] @ W).ravel() for i in range(p.m)], axis=1)  # vec(A_i W), row-major
    return gamma * np.eye(n * r) + rho * cols @ cols.T


@pytest.mark.parametrize("name", ["generic", "mc"])
def test_cg_vs_dense_solve(name):
    p = sdpgen.generic_random(8, 10, 7) if name == "generic" else sdpgen.mc_planted(5, 4, 2, 8, count=14)
    rng = np.random.default_rng(9)
    W = rng.standard_normal((p.n, 3))
    R = rng.standard_normal((p.n, 3))
    rho, gamma = 2.0, 0.5
    M = _dense_system(p, W, rho, gamma)
    ref = np.linalg.solve(M, R.ravel()).reshape(R.shape)
    D, it, rel, _ = cg(cg_operator(p, W, rho, gamma), R, 1e-13, 1000)
    assert rel <= 1e-13
    assert np.allclose(D, ref, rtol=1e-10, atol=1e-12)
    # the matrix-free operator equals the dense matrix
    P = rng.standard_normal(W.shape)
    assert np.allclose(cg_operator(p, W, rho, gamma)(P).ravel(), M @ P.ravel(), rtol=1e-12)


def test_maxcut_sherman_morrison():
    p = sdpgen.maxcut_er(60, 0.1, 10)
    rng = np.random.default_rng(11)
    W = rng.standard_normal((p.n, 5))
    R = rng.standard_normal((p.n, 5))
    rho, gamma = 7.0, 1.3
    D, it, rel, _ = cg(cg_operator(p, W, rho, gamma), R, 1e-13, 1000)
    # (gamma I + rho w w^T)^-1 r = (r - rho w <w, r> / (gamma + rho |w|^2)) / gamma per row
    wr = np.sum(W * R, axis=1)
    ww = np.sum(W * W, axis=1)
    ref = (R - (rho * wr / (gamma + rho * ww))[:, None] * W) / gamma
    assert np.allclose(D, ref, rtol=1e-11, atol=1e-13)


def test_maxcut_two_iterations_equal_row_norms():
    """Rows of W with equal norms: the MaxCut system has exactly two distinct
    eigenvalues (gamma and gamma + rho |w|^2), so CG terminates in 2 steps."""
    p = sdpgen.maxcut_er(80, 0.1, 12)
    rng = np.random.default_rng(13)
    W = rng.standard_normal((p.n, 6))
    W /= np.linalg.norm(W, axis=1, keepdims=True)
    R = rng.standard_normal((p.n, 6))
    D, it, rel, _ = cg(cg_operator(p, W, 4.0, 0.9), R, 1e-12, 50)
    assert it == 2 and rel <= 1e-12


def test_cg_residuals_orthogonal():
    p = sdpgen.mc_planted(40, 35, 2, 14, count=500)
    rng = np.random.default_rng(15)
    W = rng.standard_normal((p.n, 4)) / 2
    R0 = rng.standard_normal((p.n, 4))
    M = cg_operator(p, W, 3.0, 1.0)
    residuals = []
    for k in range(6):
        D, it, _, _ = cg(M, R0, 0.0, k)
        residuals.append(R0 - M(D))
    G = np.array([[np.sum(a * b) for b in residuals] for a in residuals])
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) <= 1e-9 * np.max(np.diag(G))
