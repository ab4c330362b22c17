"""Pins of the oracle on the quadratic objective f(X) = <C, X> + (mu/2)||X||_F^2
(Section 1's convex f; CPU only).

Closed form: min <C, X> + (mu/2) ||X||_F^2 s.t. tr X = 1, X PSD has the
solution X* = sum_i x_i v_i v_i^T over the eigenpairs (c_i, v_i) of C with
x_i = max(0, (tau - c_i) / mu) and sum_i x_i = 1 (the KKT conditions
C + mu X - tau I = S, S PSD, <S, X> = 0 diagonalise with C).  The solve must
reach f(X*) and X* itself; the Appendix-B measures of the exact pair
(X*, lam = -tau) must vanish (gap 0, no negative slack eigenvalue), and
moving off it must show in them.
Derivatives: the Phase-I gradient against central differences of the
augmented Lagrangian, the quartic's coefficients against the Lagrangian at
five step lengths, and the CG operator against central differences of the
gradient of eq. (ALF) in the free factor (the subproblem is quadratic, so the
difference of gradients is the operator applied to the step).
"""
import math

import numpy as np
import pytest

import oracle
import sdpgen
from oracle import admm, alm, operators
from oracle.options import Options, paper_defaults


def _water_fill(n, mu, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) / math.sqrt(n)
    Cd = 0.5 * (G + G.T)
    ir, ic = np.triu_indices(n)
    ar = np.arange(n)
    p = sdpgen.Problem(n=n, m=1, c_row=ir, c_col=ic, c_val=Cd[ir, ic], a_con=np.zeros(n),
                       a_row=ar, a_col=ar, a_val=np.ones(n), b=np.ones(1), kind="generic", mu=mu)
    c, V = np.linalg.eigh(Cd)
    # water level: sum max(0, (tau - c_i) / mu) = 1, found on the sorted eigenvalues
    for k in range(1, n + 1):
        tau = (mu + c[:k].sum()) / k
        if k == n or tau <= c[k]:
            break
    x = np.maximum(0.0, (tau - c) / mu)
    X = (V * x) @ V.T
    f = float(c @ x + 0.5 * mu * x @ x)
    return p, X, f, tau, int((x > 0).sum())


@pytest.mark.parametrize("mu", [0.2, 1.0])
def test_water_filling_closed_form(mu):
    p, Xs, fs, tau, active = _water_fill(40, mu, 3)
    assert 2 <= active <= 6
    r0 = 8
    U0 = sdpgen.random_init_U(p.n, r0, 4)
    res = oracle.lorads.lorads(p, U0, Options(**paper_defaults(p.kind, p.n)))
    assert res["phase2"]["converged"]
    assert abs(res["metrics"]["obj"] - fs) <= 1e-6 * max(1.0, abs(fs))
    Uh = res["U_hat"]
    assert np.linalg.norm(Uh @ Uh.T - Xs) <= 1e-4 * np.linalg.norm(Xs)


def test_measures_vanish_at_the_exact_solution():
    mu = 0.5
    p, Xs, fs, tau, active = _water_fill(30, mu, 5)
    assert active == 3
    w, V = np.linalg.eigh(Xs)
    keep = w > 1e-12
    U = V[:, keep] * np.sqrt(w[keep])
    m = oracle.metrics.appendix_b(p, U, np.array([-tau]))
    assert abs(m["obj"] - fs) <= 1e-12 * max(1.0, abs(fs))
    assert m["pinf"] <= 1e-13 and abs(m["gap"]) <= 1e-12
    assert m["lambda_min"] >= -1e-12 and m["dinf"] <= 1e-14
    # a multiplier off the optimum shows a negative slack eigenvalue
    m2 = oracle.metrics.appendix_b(p, U, np.array([-tau - 0.05]))
    assert m2["dinf"] > 1e-4 and abs(m2["gap"]) > 1e-4


def _random_case(mu):
    p = sdpgen.generic_random(9, 6, 2)
    p.mu = mu
    rng = np.random.default_rng(1)
    return p, rng.standard_normal((9, 3)), rng.standard_normal((9, 3)), rng.standard_normal(p.m)


@pytest.mark.parametrize("mu", [0.0, 0.7])
def test_phase1_gradient_finite_differences(mu):
    p, U, D, lam = _random_case(mu)
    rho = 1.3
    z = operators.forward(p, U, U)
    g = alm.gradient(p, U, z, lam, rho)
    h = 1e-6
    fd = np.zeros_like(U)
    for i in range(U.shape[0]):
        for j in range(U.shape[1]):
            E = np.zeros_like(U)
            E[i, j] = h
            fd[i, j] = (alm.objective_parts(p, U + E, lam, rho) - alm.objective_parts(p, U - E, lam, rho)) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(g)


@pytest.mark.parametrize("mu", [0.0, 0.7])
def test_quartic_coefficients_reproduce_the_lagrangian(mu):
    p, U, D, lam = _random_case(mu)
    rho = 0.9
    z = operators.forward(p, U, U)
    q1, q2, q3, q4 = alm.quartic_coefficients(p, U, D, z, lam, rho)
    base = alm.objective_parts(p, U, lam, rho)
    for a in (-1.3, -0.2, 0.4, 1.0, 2.5):
        want = alm.objective_parts(p, U + a * D, lam, rho) - base
        got = q1 * a + q2 * a ** 2 + q3 * a ** 3 + q4 * a ** 4
        assert abs(got - want) <= 1e-9 * max(1.0, abs(want))


@pytest.mark.parametrize("mu", [0.0, 0.7])
def test_cg_operator_is_the_subproblem_hessian(mu):
    p, W, P, lam = _random_case(mu)
    rho, gamma = 1.7, 2.1
    M = oracle.cg.cg_operator(p, W, rho, gamma)

    def grad_u(U):
        # gradient of eq. (ALF) in U at fixed V = W, by central differences
        h = 1e-5
        g = np.zeros_like(U)
        for i in range(U.shape[0]):
            for j in range(U.shape[1]):
                E = np.zeros_like(U)
                E[i, j] = h
                g[i, j] = (admm.alf(p, U + E, W, lam, rho, gamma) - admm.alf(p, U - E, W, lam, rho, gamma)) / (2 * h)
        return g

    diff = grad_u(W + P) - grad_u(W)
    assert np.linalg.norm(M(P) - diff) <= 1e-6 * np.linalg.norm(diff)
    # and R0 is the negative gradient at x0 = W
    assert np.linalg.norm(-admm.grad_factor(p, W, lam, rho) + grad_u(W)) <= 1e-6 * np.linalg.norm(grad_u(W))


def _fully_observed(n1, n2, seed):
    """Completion with every cell observed and mu scaled to the planted matrix:
    X* = [U S U^T, M; M^T, V S V^T] (M = U S V^T) for every mu >= 0 (per
    singular pair, min (a + b)/2 + (mu/2)(a^2 + b^2) s.t. a b >= s^2 is at
    a = b = s), so f* = sum s + 2 mu sum s^2 (||X*||_F^2 = 4 sum s^2)."""
    p = sdpgen.mc_planted(n1, n2, 2, seed, count=n1 * n2)
    M = p.meta["L"] @ p.meta["R"].T
    s = np.linalg.svd(M, compute_uv=False)
    p.mu = 0.25 * s.sum() / (s ** 2).sum()
    return p, s.sum() + 2.0 * p.mu * (s ** 2).sum()


@pytest.mark.parametrize("n1,n2,seed", [(8, 6, 4), (30, 24, 7)])
def test_fully_observed_completion_with_mu(n1, n2, seed):
    p, want = _fully_observed(n1, n2, seed)
    out = oracle.lorads.lorads(p, sdpgen.random_init_U(p.n, sdpgen.rank_rule_2lnm(p.m), 3),
                               Options(**paper_defaults(p.kind, p.n)))
    assert out["phase2"]["converged"]
    assert abs(out["metrics"]["obj"] - want) <= 1e-6 * want
