"""Pins of the oracle on rank-one constraint families (CPU only).

Sensor network localization (Section 3): with exact distances on a network
that the anchors pin down, the relaxation's feasible set is the single point
Z = [I X; X^T X^T X] (X the true positions), so a solve recovers the sensors
and Z has rank d.  Graph bisection of an even cycle C_n: the relaxation
min <L/4, X> s.t. diag X = 1, <J, X> = 0 has value n lambda_2(L) / 4 =
n (1 - cos(2 pi / n)) / 2 (the second eigenspace of the circulant Laplacian
gives a feasible X with a constant diagonal).  Operator form: for A = c a a^T,
<A, U V^T> = c (a^T U)(a^T V)^T, checked with a taken from the generator.  Section 3's escape example: below.
"""
import math

import numpy as np
import pytest

import oracle
import sdpgen
from oracle.options import Options, paper_defaults


def _solve(p, r0, seed=3):
    o = Options(**paper_defaults(p.kind, p.n))
    return oracle.lorads.lorads(p, sdpgen.random_init_U(p.n, r0, seed), o)


def test_snl_recovers_sensors():
    p = sdpgen.snl(30, 4, 0.45, 7)
    out = _solve(p, sdpgen.rank_rule_2lnm(p.m))
    assert out["phase2"]["converged"]
    Z = out["U_hat"] @ out["U_hat"].T
    assert np.abs(Z[:2, :2] - np.eye(2)).max() <= 1e-5
    assert np.abs(Z[2:, :2] - p.meta["sensors"]).max() <= 1e-5
    ev = np.linalg.eigvalsh(Z)[::-1]
    assert ev[2] <= 1e-4 * ev[0]


@pytest.mark.parametrize("n", [8, 16, 30])
def test_cycle_bisection_closed_form(n):
    e = np.arange(n)
    p = sdpgen.min_bisection(n, e, (e + 1) % n, np.ones(n))
    out = _solve(p, 4)
    assert out["phase2"]["converged"]
    want = n * (1.0 - math.cos(2.0 * math.pi / n)) / 2.0
    assert abs(out["metrics"]["obj"] - want) <= 1e-6 * want


def test_rank_one_forward_identity():
    p = sdpgen.snl(12, 3, 0.6, 2)
    rng = np.random.default_rng(5)
    U, V = rng.standard_normal((p.n, 4)), rng.standard_normal((p.n, 4))
    z = oracle.operators.forward(p, U, V)
    X, A = p.meta["sensors"], p.meta["anchors"]
    # the generator's constraints in order: Z_00, Z_11, (e0 + e1), then sensor
    # pairs, then anchor-sensor pairs, each A = a a^T
    vecs = [np.eye(p.n)[0], np.eye(p.n)[1], np.eye(p.n)[0] + np.eye(p.n)[1]]
    for i in range(12):
        for j in range(i + 1, 12):
            if np.linalg.norm(X[i] - X[j]) < 0.6:
                a = np.zeros(p.n); a[2 + i], a[2 + j] = 1.0, -1.0
                vecs.append(a)
    for k in range(3):
        for j in range(12):
            if np.linalg.norm(A[k] - X[j]) < 0.6:
                a = np.zeros(p.n); a[:2] = A[k]; a[2 + j] = -1.0
                vecs.append(a)
    assert len(vecs) == p.m
    want = np.array([(a @ U) @ (a @ V) for a in vecs])
    assert np.linalg.norm(z - want) <= 1e-13 * np.linalg.norm(want)


# ---------------------------------------------------------------------------
# Section 3's escape example: one sensor, three anchors (self-made; each set
# was found by a multi-start search for a spurious local minimum of the
# rank-d penalty).  At rank d the factorised relaxation is the SNL problem
# itself, min_x sum_k (|a_k - x|^2 - d_k^2)^2, whose spurious minimum traps
# the Burer-Monteiro phase; the ADMM started from the trapped factor (its own
# rho rule, lambda = 0) moves off it to the unique feasible point
# Z = [I x*; x*^T |x*|^2].  Entries: anchors, true sensor, the spurious
# minimum to three decimals (refined by Newton's method in the test).
# ---------------------------------------------------------------------------
ESCAPE_CASES = [
    ([[-0.855, -0.964], [0.16, -0.618], [0.951, -0.785]], [-0.096, -0.211], [0.026, -1.345]),
    ([[-0.67, 0.754], [0.789, -0.903], [-0.604, 0.273]], [0.578, 0.213], [-0.311, -0.663]),
    ([[-0.766, -0.505], [0.613, -0.098], [0.754, 0.203]], [0.579, -0.625], [0.147, 0.456]),
    ([[0.635, -0.753], [0.696, -0.484], [-0.505, 0.545]], [0.515, 0.692], [-0.638, -0.425]),
    ([[-0.326, 0.333], [0.801, -0.497], [0.987, -0.924]], [-0.771, -0.039], [-0.048, 0.809]),
]
ESCAPE_PHASE1_OUTER = 8  # the trapped Burer-Monteiro run: rho grows to about 5e6


def escape_instance(case):
    A, xs, _ = (np.asarray(v, dtype=np.float64) for v in case)
    return sdpgen.snl_positions(xs[None, :], A)


def sensor_of(U, V=None):
    """Sensor position held by Z = U V^T (symmetrised) or U U^T."""
    Z = U @ (U if V is None else V).T
    return 0.5 * (Z[:2, 2] + Z[2, :2])


def _penalty_newton(A, xs, x):
    """Newton's method on f(x) = sum_k (|a_k - x|^2 - d_k^2)^2 from x; returns
    the point, |grad f|, the Hessian's smallest eigenvalue and f."""
    d2 = ((A - xs) ** 2).sum(1)
    for _ in range(30):
        res = ((A - x) ** 2).sum(1) - d2
        g = (4.0 * res[:, None] * (x - A)).sum(0)
        H = sum(8.0 * np.outer(x - a, x - a) + 4.0 * rk * np.eye(2) for a, rk in zip(A, res))
        x = x - np.linalg.solve(H, g)
    res = ((A - x) ** 2).sum(1) - d2
    g = (4.0 * res[:, None] * (x - A)).sum(0)
    H = sum(8.0 * np.outer(x - a, x - a) + 4.0 * rk * np.eye(2) for a, rk in zip(A, res))
    return x, float(np.linalg.norm(g)), float(np.linalg.eigvalsh(H)[0]), float((res ** 2).sum())


@pytest.mark.parametrize("case", range(len(ESCAPE_CASES)))
def test_escape_cases_have_spurious_minima(case):
    A, xs, xsp = (np.asarray(v, dtype=np.float64) for v in ESCAPE_CASES[case])
    x, gn, hmin, f = _penalty_newton(A, xs, xsp)
    assert gn <= 1e-10 and hmin > 0.0 and f > 1e-2  # a strict local minimum, not feasible
    assert np.linalg.norm(x - xsp) <= 2e-3 and np.linalg.norm(x - xs) > 0.5
    # the true sensor is the global one (f = 0) and the relaxation's feasible
    # point: the generator's b are met by Z = [I x*; x*^T |x*|^2]
    p = escape_instance(ESCAPE_CASES[case])
    U = np.array([[1.0, 0.0], [0.0, 1.0], list(xs)])
    assert np.abs(oracle.operators.forward(p, U, U) - p.b).max() <= 1e-14


@pytest.mark.parametrize("case", range(len(ESCAPE_CASES)))
def test_admm_escapes_where_burer_monteiro_is_trapped(case):
    A, xs, xsp = (np.asarray(v, dtype=np.float64) for v in ESCAPE_CASES[case])
    p = escape_instance(ESCAPE_CASES[case])
    U0 = np.array([[1.0, 0.0], [0.0, 1.0], list(xsp)])
    # Phase I at rank d from the spurious point: trapped (the sensor stays
    # far from x*, the infeasibility far from the switching tolerance)
    p1 = oracle.alm.alm(p, U0, np.zeros(p.m), Options(r_max=2, alm_outer_max=ESCAPE_PHASE1_OUTER))
    assert np.linalg.norm(sensor_of(p1["U"]) - xs) > 0.5 and p1["pinf"] > 1e-2
    # ADMM from the trapped factor at the same rank
    out = oracle.lorads.lorads(p, p1["U"], Options(r_max=2, phase1=False))
    assert out["phase2"]["converged"]
    assert np.linalg.norm(sensor_of(out["U_hat"]) - xs) <= 1e-4
