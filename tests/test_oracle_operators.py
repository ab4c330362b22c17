"""Pins of the oracle's constraint operator and adjoint (CPU only).

Each check uses something other than the oracle's own formula: dense matrices
built entry by entry (brute force), the structure's closed form (diagonal and
pair constraints), and the adjoint identity <A(P V^T), w> = <A*(w) V, P>.
"""
import numpy as np
import pytest

import oracle
import sdpgen
from oracle import dense


def _small_problems():
    return {
        "generic": sdpgen.generic_random(9, 7, 1),
        "maxcut": sdpgen.maxcut_er(12, 0.4, 2, "pm1"),
        "mc": sdpgen.mc_planted(6, 5, 2, 3, count=18),
    }


@pytest.mark.parametrize("name", ["generic", "maxcut", "mc"])
def test_forward_bruteforce(name):
    p = _small_problems()[name]
    rng = np.random.default_rng(0)
    U, V = rng.standard_normal((p.n, 4)), rng.standard_normal((p.n, 4))
    A = dense.dense_A(p)
    X = U @ V.T
    ref = np.array([np.sum(A[i] * X) for i in range(p.m)])
    assert np.allclose(oracle.operators.forward(p, U, V), ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("name", ["generic", "maxcut", "mc"])
@pytest.mark.parametrize("c_scale", [0.0, 1.0, -2.5])
def test_adjoint_bruteforce(name, c_scale):
    p = _small_problems()[name]
    rng = np.random.default_rng(1)
    V = rng.standard_normal((p.n, 3))
    w = rng.standard_normal(p.m)
    S = c_scale * dense.dense_C(p) + np.tensordot(w, dense.dense_A(p), axes=1)
    assert np.allclose(oracle.operators.adjoint(p, w, c_scale, V), S @ V, rtol=1e-13, atol=1e-13)


def test_cost_inner_bruteforce():
    p = _small_problems()["generic"]
    rng = np.random.default_rng(2)
    U, V = rng.standard_normal((p.n, 3)), rng.standard_normal((p.n, 3))
    assert np.isclose(oracle.operators.cost_inner(p, U, V), np.sum(dense.dense_C(p) * (U @ V.T)), rtol=1e-13)


def test_norms_bruteforce():
    p = _small_problems()["generic"]
    Cd = dense.dense_C(p)
    nrm = oracle.operators.norms(p)
    assert np.isclose(nrm["c_fro"], np.linalg.norm(Cd))
    assert np.isclose(nrm["c_1"], np.abs(Cd).sum())
    assert nrm["b_inf"] == np.abs(p.b).max()


def test_diag_closed_form():
    """MaxCut constraints X_ii = 1: A(U V^T)_i = <U_i, V_i>; A*(w) V = diag(w) V."""
    p = sdpgen.maxcut_er(50, 0.1, 3)
    rng = np.random.default_rng(3)
    U, V = rng.standard_normal((p.n, 5)), rng.standard_normal((p.n, 5))
    w = rng.standard_normal(p.m)
    assert np.allclose(oracle.operators.forward(p, U, V), np.sum(U * V, axis=1), rtol=1e-14)
    assert np.allclose(oracle.operators.adjoint(p, w, 0.0, V), w[:, None] * V, rtol=1e-14)


def test_pair_closed_form():
    """Completion constraints: A_i = (e_j e_{n1+k}^T + e_{n1+k} e_j^T)/2, so
    A(U V^T)_i = (<U_j, V_{n1+k}> + <U_{n1+k}, V_j>)/2."""
    p = sdpgen.mc_planted(20, 15, 2, 4, count=90)
    n1 = p.meta["n1"]
    rng = np.random.default_rng(4)
    U, V = rng.standard_normal((p.n, 3)), rng.standard_normal((p.n, 3))
    j, k = p.a_row, p.a_col
    ref = 0.5 * (np.sum(U[j] * V[k], axis=1) + np.sum(U[k] * V[j], axis=1))
    assert np.all(k >= n1)
    assert np.allclose(oracle.operators.forward(p, U, V), ref, rtol=1e-14)
    # feasibility of the planted matrix: X = [L; R][L; R]^T has X_{j, n1+k} = M_jk
    F = np.vstack([p.meta["L"], p.meta["R"]])
    assert np.allclose(oracle.operators.forward(p, F, F), p.b, rtol=1e-12)


def test_adjointness_identity():
    p = sdpgen.mc_planted(300, 250, 3, 5, count=9000)
    rng = np.random.default_rng(5)
    P, V = rng.standard_normal((p.n, 7)), rng.standard_normal((p.n, 7))
    w = rng.standard_normal(p.m)
    lhs = float(oracle.operators.forward(p, P, V) @ w)
    rhs = float(np.sum(oracle.operators.adjoint(p, w, 0.0, V) * P))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_maxcut_objective_is_cut():
    """For a +-1 vector x, <C, x x^T> with C = -L/4 is minus the cut weight."""
    p = sdpgen.maxcut_er(10, 0.5, 6, "pm1")
    ei, ej, w = p.meta["edges"]
    x = np.where(np.arange(10) % 3 == 0, 1.0, -1.0)
    cut = float(np.sum(w * (x[ei] != x[ej])))
    assert np.isclose(oracle.operators.cost_inner(p, x[:, None], x[:, None]), -cut)
