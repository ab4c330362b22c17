"""The quadratic objective f(X) = <C, X> + (mu/2)||X||_F^2 (Section 1's convex
f) on the GPU, against closed forms and the oracle.

  * min <C, X> + (mu/2)||X||^2 s.t. tr X = 1: the water-filling solution over
    the eigenpairs of C (objective to 1e-6, X to 1e-4), with a dense C
    (n = 400, the matrix-core products) and a sparse C (n = 300);
  * completion with every cell observed: f* = sum s + 2 mu sum s^2 over the
    singular values of the planted matrix (objective to 1e-6), in the FP64,
    FP32-CG and mixed forms, at n_X = 54 (the oracle recomputes the
    Appendix-B measures from the returned factors and multipliers) and at
    n_X = 220;
  * the batched form refuses mu != 0.
The closed forms are derived in tests/test_oracle_quadratic.py, which pins the
oracle to them.
"""
import math

import numpy as np
import pytest

import oracle
import sdpgen
from oracle.options import paper_defaults
from tests.test_oracle_quadratic import _fully_observed

pytestmark = pytest.mark.gpu


def _water_fill(n, seed, dense):
    rng = np.random.default_rng(seed)
    if dense:
        G = rng.standard_normal((n, n)) / math.sqrt(n)
        Cd = 0.5 * (G + G.T)
    else:
        Cd = np.zeros((n, n))
        k = 6 * n
        i, j = rng.integers(0, n, k), rng.integers(0, n, k)
        np.add.at(Cd, (i, j), rng.standard_normal(k) / 3.0)
        Cd = 0.5 * (Cd + Cd.T)
    c, V = np.linalg.eigh(Cd)
    # mu such that the water level covers exactly the three smallest
    # eigenvalues: tau = (mu + c0 + c1 + c2) / 3 lies in (c2, c3]
    lo = (c[2] - c[0]) + (c[2] - c[1])
    hi = (c[3] - c[0]) + (c[3] - c[1]) + (c[3] - c[2])
    mu = 0.5 * (lo + hi)
    for k in range(1, n + 1):
        tau = (mu + c[:k].sum()) / k
        if k == n or tau <= c[k]:
            break
    x = np.maximum(0.0, (tau - c) / mu)
    ir, ic = np.nonzero(np.triu(Cd) != 0)
    ar = np.arange(n)
    p = sdpgen.Problem(n=n, m=1, c_row=ir, c_col=ic, c_val=Cd[ir, ic], a_con=np.zeros(n),
                       a_row=ar, a_col=ar, a_val=np.ones(n), b=np.ones(1), kind="generic", mu=mu)
    return p, (V * x) @ V.T, float(c @ x + 0.5 * mu * x @ x), int((x > 0).sum())


@pytest.mark.parametrize("dense,n", [(True, 400), (False, 300)])
@pytest.mark.parametrize("precision", [0, 1])
def test_water_filling(device, dense, n, precision):
    from paper_2403_09133_amd import Context, default_options
    p, Xs, fs, active = _water_fill(n, 11, dense)
    assert active == 3
    r0 = 6
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    with Context(p) as ctx:
        assert ctx.problem_info()["c_dense"] == dense
        res = ctx.admm_solve([U0], default_options(r0=r0, precision=precision, time_limit=100.0,
                                                   **paper_defaults(p.kind, p.n)))[0]
        U, V, lam = ctx.get_solution(0, res["rank"])
    print(f"[test] water filling n={n} dense={dense}: obj {res['obj']:.10f} (closed form {fs:.10f}), "
          f"admm {res['admm_iters']}", flush=True)
    assert res["status"] == 0 and res["kkt"] < 1e-6, res
    assert abs(res["obj"] - fs) <= 1e-6 * abs(fs)
    Uh = 0.5 * (U + V)
    assert np.linalg.norm(Uh @ Uh.T - Xs) <= 1e-4 * np.linalg.norm(Xs)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_fully_observed_completion_small(device, precision):
    from paper_2403_09133_amd import Context, default_options
    p, want = _fully_observed(30, 24, 7)
    r0 = sdpgen.rank_rule_2lnm(p.m)
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    with Context(p) as ctx:
        res = ctx.admm_solve([U0], default_options(r0=r0, precision=precision,
                                                   **paper_defaults(p.kind, p.n)))[0]
        U, V, lam = ctx.get_solution(0, res["rank"])
    assert res["status"] == 0 and res["kkt"] < 1e-6, res
    assert abs(res["obj"] - want) <= 1e-6 * want, (res["obj"], want)
    m = oracle.metrics.appendix_b(p, 0.5 * (U + V), lam)
    assert abs(m["obj"] - res["obj"]) <= 1e-10 * abs(m["obj"])
    assert abs(m["pinf"] - res["pinf"]) <= 1e-9
    assert abs(m["gap"] - res["gap"]) <= 1e-9
    assert abs(m["dinf"] - res["dinf"]) <= 1e-8


@pytest.mark.parametrize("precision", [0, 2])
def test_fully_observed_completion_larger(device, precision):
    from paper_2403_09133_amd import Context, default_options
    p, want = _fully_observed(120, 100, 9)
    r0 = sdpgen.rank_rule_2lnm(p.m)
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    with Context(p) as ctx:
        assert ctx.problem_info()["structure"] == "pair"
        res = ctx.admm_solve([U0], default_options(r0=r0, precision=precision,
                                                   **paper_defaults(p.kind, p.n)))[0]
    print(f"[test] fully observed 120 x 100, mu {p.mu:.4g}: obj {res['obj']:.8f} (closed form {want:.8f}), "
          f"rank {res['rank']}, admm {res['admm_iters']}", flush=True)
    assert res["status"] == 0 and res["kkt"] < 1e-6, res
    assert abs(res["obj"] - want) <= 1e-6 * want, (res["obj"], want)


def test_batch_refuses_mu(device):
    from paper_2403_09133_amd import Context, default_options, lorads
    ps = [sdpgen.maxcut_er(40, 0.2, s) for s in (1, 2)]
    ps[1].mu = 0.1
    U0 = [sdpgen.random_init_U(p.n, 6, 3) for p in ps]
    with Context(ps) as ctx:
        with pytest.raises(lorads.LoradsError) as e:
            ctx.admm_solve(U0, default_options(r0=6, batch_mode=1))
    assert e.value.status == lorads.LORADS_EINVAL and "mu = 0" in str(e.value)
