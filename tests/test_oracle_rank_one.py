"""Pins of the oracle on rank-one constraint families (CPU only).

Sensor network localization (Section 3): with exact distances on a network
that the anchors pin down, the relaxation's feasible set is the single point
Z = [I X; X^T X^T X] (X the true positions), so a solve recovers the sensors
and Z has rank d.  Graph bisection of an even cycle C_n: the relaxation
min <L/4, X> s.t. diag X = 1, <J, X> = 0 has value n lambda_2(L) / 4 =
n (1 - cos(2 pi / n)) / 2 (the second eigenspace of the circulant Laplacian
gives a feasible X with a constant diagonal).  Operator form: for A = c a a^T,
<A, U V^T> = c (a^T U)(a^T V)^T, checked with a taken from the generator.
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
