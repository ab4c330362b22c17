"""Batched persistent launch (many MaxCut SDPs of uneven order in one launch)
against the single-instance GPU path and the FP64 oracle.

Bar: each instance's objective within 1e-6 relative of the oracle's at KKT
residual (eq. stop) below 1e-6; the factors returned per instance reproduce the
reported objective and primal infeasibility when the oracle re-evaluates them.
"""
import math

import numpy as np
import pytest

import oracle
import sdpgen
from oracle.options import Options, paper_defaults

pytestmark = pytest.mark.gpu

BATCH = sdpgen.batch_maxcut(6, 5000, 50, 260, 3.0, 12.0, "pm1")
R0 = 6


def _opts(**kw):
    from paper_2403_09133_amd import default_options
    pd = paper_defaults("maxcut", 100)
    kw.setdefault("r0", R0)
    return default_options(**{**pd, **kw})


def _U0s():
    return [sdpgen.random_init_U(p.n, R0, 100 + i) for i, p in enumerate(BATCH)]


@pytest.fixture(scope="module")
def oracle_results():
    out = []
    for p, U0 in zip(BATCH, _U0s()):
        out.append(oracle.lorads.lorads(p, U0, Options(**paper_defaults(p.kind, p.n)), with_metrics=False))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_matches_oracle(device, oracle_results, precision):
    from paper_2403_09133_amd import Context
    with Context(BATCH) as ctx:
        res = ctx.admm_solve(_U0s(), _opts(precision=precision, batch_mode=1))
        sols = [ctx.get_solution(i, r["rank"]) for i, r in enumerate(res)]
    for p, r, ref, (U, V, lam) in zip(BATCH, res, oracle_results, sols):
        assert r["status"] == 0 and r["kkt"] < 1e-6, r
        Uh = 0.5 * (U + V)
        oobj = oracle.operators.cost_inner(p, ref["U_hat"], ref["U_hat"])
        assert abs(r["obj"] - oobj) <= 1e-6 * abs(oobj), (r["obj"], oobj)
        assert abs(oracle.operators.cost_inner(p, Uh, Uh) - r["obj"]) <= 1e-10 * abs(oobj)
        z = oracle.operators.forward(p, Uh, Uh)
        assert abs(np.linalg.norm(z - p.b) / (1 + np.abs(p.b).sum()) - r["pinf"]) <= 1e-12


def test_batch_matches_sequential_gpu(device):
    from paper_2403_09133_amd import Context
    with Context(BATCH) as ctx:
        rb = ctx.admm_solve(_U0s(), _opts(batch_mode=1))
        rs = ctx.admm_solve(_U0s(), _opts(batch_mode=2))
    # the two paths round differently (fused passes against separate
    # kernels); MaxCut iteration counts follow rounding in the slow tail (a
    # trajectory-level quantity), so they are held to 25% and the objective to
    # 1e-7
    for a, b in zip(rb, rs):
        assert a["rank"] == b["rank"]
        assert abs(a["obj"] - b["obj"]) <= 1e-7 * abs(b["obj"])
        assert abs(a["admm_iters"] - b["admm_iters"]) <= max(3, 0.25 * b["admm_iters"])


def test_batch_autotune(device):
    from paper_2403_09133_amd import Context
    with Context(BATCH) as ctx:
        best, times = ctx.batch_autotune(_U0s(), _opts(max_admm_iter=20), (64, 128, 256))
        assert best in (64, 128, 256) and all(t > 0 for t in times.values())
        res = ctx.admm_solve(_U0s(), _opts(batch_mode=1))
    assert all(r["status"] == 0 for r in res)


def test_batch_requires_diag(device):
    from paper_2403_09133_amd import Context, lorads
    probs = [BATCH[0], sdpgen.mc_planted(10, 8, 2, 3, count=40)]
    with Context(probs) as ctx:
        with pytest.raises(lorads.LoradsError):
            ctx.admm_solve([sdpgen.random_init_U(p.n, 3, 1) for p in probs],
                           _opts(batch_mode=1, r0=3))
