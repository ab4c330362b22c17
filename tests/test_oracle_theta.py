"""Oracle pins on a general-structure family with a dense cost: the Lovasz
theta SDP (min <-J, X>, tr X = 1, X_ij = 0 on edges, X PSD) has the closed
forms theta(C_5) = sqrt 5, theta(C_n) = n cos(pi/n) / (1 + cos(pi/n)) for odd
n, theta(K_n) = 1, theta of the empty graph = n and theta(Petersen) = 4.  The
two-phase method stops at eq. (stop) <= 1e-6, so the objective is held to a
few times that, relative.  The family takes gamma = 1 + ||C||_2 (its
defaults); ||-J||_2 = n is pinned by J's spectrum (n once, 0 otherwise), the
odd cycles C_15 and C_21 by the closed form, and a random graph's theta by a
dense interior-point solve (independent code).
"""
import math

import numpy as np
import pytest

import oracle
import sdpgen
from oracle import dense
from oracle.options import Options, paper_defaults
from tests.pins import ipm

THETA = {
    "C5": (5, sdpgen.cycle_edges(5), math.sqrt(5.0)),
    "C7": (7, sdpgen.cycle_edges(7), 7 * math.cos(math.pi / 7) / (1 + math.cos(math.pi / 7))),
    "K6": (6, sdpgen.complete_edges(6), 1.0),
    "empty6": (6, [], 6.0),
    "petersen": (10, sdpgen.petersen_edges(), 4.0),
}


def theta_instance(name):
    n, edges, theta = THETA[name]
    p = sdpgen.lovasz_theta(n, edges)
    r0 = max(2, sdpgen.rank_rule_2lnm(p.m))
    return p, r0, theta


@pytest.mark.parametrize("name", sorted(THETA))
def test_oracle_lovasz_theta(name):
    p, r0, theta = theta_instance(name)
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    res = oracle.lorads.lorads(p, U0, Options(**paper_defaults(p.kind, p.n)))
    assert res["phase2"]["kkt"] <= 1e-6
    assert abs(-res["metrics"]["obj"] - theta) <= 5e-6 * theta


def test_theta_cost_norm():
    for n, edges in ((21, sdpgen.cycle_edges(21)), (10, sdpgen.petersen_edges()), (6, [])):
        p = sdpgen.lovasz_theta(n, edges)
        assert abs(oracle.operators.cost_norm2(p) - n) <= 1e-10 * n
        o = Options(**paper_defaults(p.kind, p.n))
        assert o.gamma_rule == 1 and abs(o.gamma(0.0, n, float(n)) - (1.0 + n)) <= 1e-12


@pytest.mark.parametrize("n", [15, 21])
def test_oracle_theta_odd_cycles(n):
    p = sdpgen.lovasz_theta(n, sdpgen.cycle_edges(n))
    theta = n * math.cos(math.pi / n) / (1 + math.cos(math.pi / n))
    r0 = max(2, sdpgen.rank_rule_2lnm(p.m))
    res = oracle.lorads.lorads(p, sdpgen.random_init_U(p.n, r0, 3), Options(**paper_defaults(p.kind, p.n)))
    assert res["phase2"]["converged"]
    assert abs(-res["metrics"]["obj"] - theta) <= 5e-6 * theta


def random_theta(n, prob, seed):
    ei, ej = sdpgen.er_gnp_edges(n, prob, np.random.default_rng(seed))
    return sdpgen.lovasz_theta(n, list(zip(ei.tolist(), ej.tolist())))


def test_oracle_theta_random_graph_vs_ipm():
    p = random_theta(40, 0.15, 5)
    ref = ipm.solve(dense.dense_C(p), dense.dense_A(p), p.b)
    assert abs(ref["obj"] - ref["dobj"]) <= 1e-7 * abs(ref["obj"])
    r0 = max(2, sdpgen.rank_rule_2lnm(p.m))
    res = oracle.lorads.lorads(p, sdpgen.random_init_U(p.n, r0, 3), Options(**paper_defaults(p.kind, p.n)))
    assert res["phase2"]["converged"]
    assert abs(res["metrics"]["obj"] - ref["obj"]) <= 1e-6 * abs(ref["obj"])
