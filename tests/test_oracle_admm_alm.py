"""Pins of the oracle's ADMM and ALM steps (CPU only).

  * Proposition 1, first identity: the multiplier step raises L_rho by exactly
    ||lam+ - lam||^2 / rho.
  * Proposition 1, second statement: with exact subproblem solves, the U and
    V steps lower L_rho by at least gamma/2 (||dU||^2 + ||dV||^2).
  * Each half step satisfies its optimality condition, eq. (optU)/(optV).
  * ALM gradient against central finite differences; the quartic line-search
    coefficients reproduce L(U + a D) - L(U) exactly at several a; the chosen
    step is the minimiser over a fine grid; L decreases along inner iterations.
  * SplitMix64 against its published seed-0 outputs.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import sdpgen
from oracle import alm, admm, operators
from oracle.options import Options

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(seed=0):
    p = sdpgen.mc_planted(30, 25, 2, 20 + seed, count=300)
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((p.n, 4)) * 0.5
    V = rng.standard_normal((p.n, 4)) * 0.5
    lam = rng.standard_normal(p.m) * 0.1
    return p, U, V, lam


def test_prop1_multiplier_identity():
    p, U, V, lam = _setup()
    rho, gamma = 3.0, 2.0
    lam_new = lam + rho * (operators.forward(p, U, V) - p.b)
    lhs = admm.alf(p, U, V, lam_new, rho, gamma) - admm.alf(p, U, V, lam, rho, gamma)
    assert np.isclose(lhs, np.sum((lam_new - lam) ** 2) / rho, rtol=1e-11)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_prop1_descent_inequality(seed):
    p, U, V, lam = _setup(seed)
    rho, gamma = 2.0, 1.5
    maxit = p.n * 4
    U1, _ = admm.half_step(p, V, lam, rho, gamma, 1e-13, maxit)
    V1, _ = admm.half_step(p, U1, lam, rho, gamma, 1e-13, maxit)
    drop = admm.alf(p, U1, V1, lam, rho, gamma) - admm.alf(p, U, V, lam, rho, gamma)
    bound = -0.5 * gamma * (np.sum((V1 - V) ** 2) + np.sum((U1 - U) ** 2))
    assert drop <= bound + 1e-9 * abs(bound)


def test_half_step_optimality():
    """eq. (optU): C V + gamma (U+ - V) + A*(lam) V + rho A*(A(U+ V^T) - b) V = 0."""
    p, U, V, lam = _setup(3)
    rho, gamma = 4.0, 0.7
    U1, _ = admm.half_step(p, V, lam, rho, gamma, 1e-13, p.n * 4)
    z = operators.forward(p, U1, V) - p.b
    res = operators.adjoint(p, lam + rho * z, 1.0, V) + gamma * (U1 - V)
    scale = np.linalg.norm(operators.adjoint(p, lam, 1.0, V)) + gamma * np.linalg.norm(V)
    assert np.linalg.norm(res) <= 1e-10 * scale


def test_alm_gradient_finite_differences():
    p = sdpgen.maxcut_er(25, 0.3, 5, "pm1")
    rng = np.random.default_rng(6)
    U = rng.standard_normal((p.n, 3))
    lam = rng.standard_normal(p.m)
    rho = 1.7
    z = operators.forward(p, U, U)
    G = alm.gradient(p, U, z, lam, rho)
    D = rng.standard_normal(U.shape)
    h = 1e-5
    fd = (alm.objective_parts(p, U + h * D, lam, rho) - alm.objective_parts(p, U - h * D, lam, rho)) / (2 * h)
    assert np.isclose(fd, np.sum(G * D), rtol=1e-7)


def test_quartic_coefficients_exact():
    p, U, _, lam = _setup(4)
    rng = np.random.default_rng(7)
    D = rng.standard_normal(U.shape)
    rho = 2.5
    z = operators.forward(p, U, U)
    q1, q2, q3, q4 = alm.quartic_coefficients(p, U, D, z, lam, rho)
    f0 = alm.objective_parts(p, U, lam, rho)
    for a in (-1.3, -0.2, 0.35, 1.0, 2.7):
        direct = alm.objective_parts(p, U + a * D, lam, rho) - f0
        poly = q1 * a + q2 * a * a + q3 * a ** 3 + q4 * a ** 4
        assert np.isclose(direct, poly, rtol=1e-10, atol=1e-9 * abs(f0))


@pytest.mark.parametrize("coeffs", [(-3.0, 1.0, -2.0, 0.7), (-1.0, -4.0, 0.5, 0.2), (-0.5, 2.0, 0.0, 1e-3),
                                    (-2.0, 3.0, 0.0, 0.0)])
def test_quartic_step_is_grid_minimiser(coeffs):
    q1, q2, q3, q4 = coeffs
    a = alm.quartic_step(q1, q2, q3, q4)
    grid = np.linspace(1e-6, 50, 200001)
    vals = q1 * grid + q2 * grid ** 2 + q3 * grid ** 3 + q4 * grid ** 4
    best = grid[np.argmin(vals)]
    assert abs(a - best) <= 3e-4 * max(1.0, best)


def test_lbfgs_inner_monotone():
    p = sdpgen.maxcut_er(40, 0.2, 8)
    U = sdpgen.random_init_U(p.n, 4, 8)
    lam = np.zeros(p.m)
    rho = 1.0
    vals = [alm.objective_parts(p, U, lam, rho)]
    for _ in range(15):
        U, z, it, conv = alm.lbfgs_inner(p, U, lam, rho, 0.0, 1, 4, 1.0)
        vals.append(alm.objective_parts(p, U, lam, rho))
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(vals, vals[1:]))


def test_splitmix64_published_outputs():
    g = json.load(open(os.path.join(GOLDEN, "splitmix64_seed0.json")))
    got = [format(int(x), "016x") for x in oracle.rng.splitmix_output(0, np.arange(1, 4))]
    assert got == g["outputs"]


def test_normals_moments():
    x = oracle.rng.normals(123, 2, 200000)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1.0) < 0.01
    assert abs(np.mean(x ** 4) - 3.0) < 0.05  # Gaussian kurtosis


def test_rank_growth_keeps_columns():
    U = np.arange(12.0).reshape(4, 3)
    G = alm.grow_rank(U, 5, 0, 9)
    assert G.shape == (4, 5) and np.array_equal(G[:, :3], U)
    assert np.all(np.abs(G[:, 3:]) < 1e-2 * np.linalg.norm(U))


@pytest.mark.parametrize("v_after", [0.0, 10.0])
def test_rank_growth_only_while_phase_one_continues(monkeypatch, v_after):
    """An inner solve that stops at the iteration cap raises the rank only when
    the infeasibility after it is still above the switching tolerance."""
    p = sdpgen.mc_planted(12, 10, 2, 3, count=60)
    U0 = np.random.default_rng(1).standard_normal((p.n, 3))
    opts = Options(switch_tol=1e-3, rank_grow_iters=5, alm_outer_max=1)

    def capped(prob, U, lam, rho, tol, cap, mem, c_fro):
        # the cap is reached; the infeasibility afterwards is v_after (1 + ||b||_inf)
        z = prob.b.copy()
        z[0] += v_after * (1.0 + np.max(np.abs(prob.b)))
        return U, z, cap, False

    monkeypatch.setattr(alm, "lbfgs_inner", capped)
    out = alm.alm(p, U0, np.zeros(p.m), opts)
    if v_after == 0.0:
        assert out["growths"] == 0 and out["rank"] == 3
    else:
        assert out["growths"] >= 1 and out["rank"] > 3
