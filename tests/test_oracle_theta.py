"""Oracle pins on a general-structure family with a dense cost: the Lovasz
theta SDP (min <-J, X>, tr X = 1, X_ij = 0 on edges, X PSD) has the closed
forms theta(C_5) = sqrt 5, theta(C_n) = n cos(pi/n) / (1 + cos(pi/n)) for odd
n, theta(K_n) = 1, theta of the empty graph = n and theta(Petersen) = 4.  The
two-phase method stops at eq. (stop) <= 1e-6, so the objective is held to a
few times that, relative.
"""
import math

import pytest

import oracle
import sdpgen
from oracle.options import Options, paper_defaults

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
