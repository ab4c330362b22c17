"""Learned warm start as shipped (paper_2403_09133_amd/data/gnn_maxcut.npz):
prediction on graphs of the training range, the fallback rules, and a solve
started from the predicted multipliers reaching the cold solve's objective."""
import math

import numpy as np
import pytest

import sdpgen

pytestmark = pytest.mark.gpu


def test_predict_inside_and_outside_training_range():
    from paper_2403_09133_amd import warmstart as W
    ws = W.WarmStart.load()
    inside = W.instances(2, W.HELDOUT_SEED0 + 77)
    small = sdpgen.maxcut_er(300, 0.03, 5, "pm1")
    preds = ws.predict(inside + [small])
    for p, pr in zip(inside, preds[:2]):
        assert pr["reason"] == "learned"
        lam = pr["lambda0"]
        assert lam.shape == (p.m,) and np.all(np.isfinite(lam))
        assert pr["r0"] == math.ceil(math.log2(p.n))
        # MaxCut duals are negative multiples of the weighted degree scale:
        # lambda = -y with y < 0 on every node that has an edge
        assert np.median(lam) > 0
    assert preds[2]["lambda0"] is None and "training range" in preds[2]["reason"]


def test_warm_solve_matches_cold_objective():
    from paper_2403_09133_amd import Context, warmstart as W
    from paper_2403_09133_amd.params import solver_options
    ws = W.WarmStart.load()
    p = W.instances(6, W.HELDOUT_SEED0)[5]  # n = 2079
    pr = ws.predict([p])[0]
    r0 = W.rule_rank(p.n)
    U0 = W.random_start(p, r0)
    with Context(p) as ctx:
        cold = ctx.admm_solve([U0], solver_options("maxcut", p.n, r0))[0]
        warm = ctx.admm_solve([U0], solver_options("maxcut", p.n, r0), init_lambda=[pr["lambda0"]])[0]
        chk = ctx.admm_solve([U0], solver_options("maxcut", p.n, r0, warm_check=1),
                             init_lambda=[pr["lambda0"]])[0]
    for res in (cold, warm, chk):
        assert res["kkt"] < 1e-4 and abs(res["gap"]) < 1e-4
    assert abs(warm["obj"] - cold["obj"]) <= 2e-4 * abs(cold["obj"])
    # with the check on, a rejected learned start continues exactly as the cold start
    if chk["warm_fallback"]:
        assert chk["admm_iters"] == cold["admm_iters"] and chk["obj"] == cold["obj"]
