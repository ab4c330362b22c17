"""End-to-end pins of the oracle's two-phase solve (CPU only).

Closed forms of the MaxCut relaxation (min form, C = -L/4):
  * complete graph K_n: -n^2/4;
  * bipartite graph, unit weights: -|E| (every edge cut, X = x x^T feasible);
  * odd cycle C_n: -n (1 + cos(pi/n)) / 2 (vertex-transitive: n lambda_max(L)/4).
Completion: fully observed M gives the nuclear norm; a planted low-rank M with
enough samples is recovered.  A dense interior-point solve (independent code)
cross-checks general instances; exhaustive enumeration brackets small MaxCut
values between the best cut and the best cut / 0.87856 (Goemans-Williamson).
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import sdpgen
from oracle import dense
from oracle.options import Options, paper_defaults
from tests.pins import ipm


def solve(p, r0, seed=3, **kw):
    o = Options(**{**paper_defaults(p.kind, p.n), **kw})
    return oracle.lorads.lorads(p, sdpgen.random_init_U(p.n, r0, seed), o)


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def test_complete_graph():
    n = 24
    iu, ju = np.triu_indices(n, 1)
    p = sdpgen.maxcut_from_edges(n, iu, ju, np.ones(iu.size))
    out = solve(p, 5)
    assert out["phase2"]["converged"]
    assert rel(out["metrics"]["obj"], -n * n / 4) <= 1e-6


@pytest.mark.parametrize("n", [9, 21])
def test_odd_cycle(n):
    ei = np.arange(n)
    p = sdpgen.maxcut_from_edges(n, ei, (ei + 1) % n, np.ones(n))
    out = solve(p, 4)
    assert out["phase2"]["converged"]
    assert rel(out["metrics"]["obj"], -n * (1 + math.cos(math.pi / n)) / 2) <= 1e-6


def test_bipartite_grid():
    p = sdpgen.maxcut_torus(6, 8, 1, "unit")  # even torus: bipartite
    out = solve(p, 4)
    assert out["phase2"]["converged"]
    assert rel(out["metrics"]["obj"], -96.0) <= 1e-6


def test_fully_observed_completion():
    p = sdpgen.mc_planted(8, 6, 2, 4, count=48)
    M = p.meta["L"] @ p.meta["R"].T
    out = solve(p, 6)
    assert out["phase2"]["converged"]
    assert rel(out["metrics"]["obj"], np.linalg.svd(M, compute_uv=False).sum()) <= 1e-6


def test_planted_completion_recovery():
    p = sdpgen.mc_planted(60, 50, 2, 5, count=1500)
    M = p.meta["L"] @ p.meta["R"].T
    out = solve(p, sdpgen.rank_rule_2lnm(p.m))
    assert out["phase2"]["converged"]
    assert rel(out["metrics"]["obj"], np.linalg.svd(M, compute_uv=False).sum()) <= 1e-6
    assert oracle.metrics.mc_recovery_error(p, out["U_hat"]) <= 1e-4


@pytest.mark.parametrize("which", ["generic", "maxcut"])
def test_dense_ipm_cross_check(which):
    p = sdpgen.generic_random(10, 8, 5) if which == "generic" else sdpgen.maxcut_er(40, 0.2, 6, "pm1")
    ref = ipm.solve(dense.dense_C(p), dense.dense_A(p), p.b)
    assert abs(ref["obj"] - ref["dobj"]) <= 1e-7 * (1 + abs(ref["obj"]))
    out = solve(p, 6)
    assert out["phase2"]["converged"]
    assert rel(out["metrics"]["obj"], ref["obj"]) <= 1e-6
    m = out["metrics"]
    assert m["pinf"] <= 1e-6 and m["dinf"] <= 1e-5 and abs(m["gap"]) <= 5e-5


def test_exhaustive_cut_sandwich():
    p = sdpgen.maxcut_er(12, 0.4, 7, "unit")
    ei, ej, w = p.meta["edges"]
    best = 0.0
    for bits in itertools.product([0, 1], repeat=11):
        x = np.array((0,) + bits)
        best = max(best, float(np.sum(w * (x[ei] != x[ej]))))
    out = solve(p, 4)
    sdp = -out["metrics"]["obj"]
    assert best - 1e-6 <= sdp <= best / 0.87856 + 1e-6


def test_certificates_er():
    p = sdpgen.maxcut_er(80, 0.1, 8, "pm1")
    out = solve(p, 7)
    m = out["metrics"]
    assert out["phase2"]["kkt"] < 1e-6
    assert m["pinf"] <= 1e-6 and m["dinf"] <= 1e-5 and abs(m["gap"]) <= 5e-5


def degenerate_instances():
    """Degenerate SDPs and their optimal values: a 1 x 1 SDP, whose feasible set
    is the single point X = b / a (optimum 3 * 2); MaxCut of one edge, where
    X = [[1, -1], [-1, 1]] cuts it (min form: -1); and MaxCut of graphs without
    edges, where C = 0 and every feasible X is optimal (0), down to a single
    vertex.  The 1 x 1 case starts Phase I next to the stationary point U = 0
    of its first subproblems, so it also exercises the growth of rho."""
    one = sdpgen.Problem(n=1, m=1, c_row=[0], c_col=[0], c_val=[3.0], a_con=[0], a_row=[0],
                         a_col=[0], a_val=[1.0], b=[2.0], kind="generic")
    return {
        "one_by_one": (one, 6.0),
        "single_edge": (sdpgen.maxcut_from_edges(2, [0], [1], [1.0]), -1.0),
        "edgeless5": (sdpgen.maxcut_from_edges(5, [], [], []), 0.0),
        "single_vertex": (sdpgen.maxcut_from_edges(1, [], [], []), 0.0),
    }


def degenerate_rank(p):
    return max(1, min(int(math.floor(math.sqrt(2.0 * p.m))), p.n))


@pytest.mark.parametrize("name", ["one_by_one", "single_edge", "edgeless5", "single_vertex"])
def test_degenerate_instances(name):
    p, want = degenerate_instances()[name]
    out = solve(p, degenerate_rank(p))
    assert out["phase2"]["converged"]
    assert abs(out["metrics"]["obj"] - want) <= 1e-6 * max(1.0, abs(want))
    assert out["metrics"]["pinf"] <= 1e-6
