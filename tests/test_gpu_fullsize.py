"""GPU parity at the full sizes of the benchmarked configurations.

The two completion instances (n_X = 20000, m = 4,605,170, r = 15, and the
headline n_X = 40000, m = 15,683,710, r = 17, whose rows the solver pads to 32
columns) and the two MaxCut instances of the FP32-CG configuration (the
100 x 100 torus and G(20000, 60000)): the forward map and the adjoint are
compared with the oracle element by element (the oracle forms them in a few
seconds at these sizes), in FP64 to the operator tests' bounds and in FP32 to
the FP32 bounds; the CG entry point, which runs the solver's CG layout and
kernels, is compared after a fixed number of iterations with the oracle's
textbook CG on the same system.
"""
import math

import numpy as np
import pytest

import oracle
import sdpgen

pytestmark = pytest.mark.gpu

_CACHE = {}


def _problem(name):
    if name not in _CACHE:
        _CACHE[name] = sdpgen.config_instance(name)
    return _CACHE[name]


def _rank(p):
    from paper_2403_09133_amd.params import initial_rank
    return initial_rank(p.kind, p.n, p.m)


def _abs_bound_forward(p, U, V):
    pa = sdpgen.Problem(n=p.n, m=p.m, c_row=p.c_row, c_col=p.c_col, c_val=p.c_val, a_con=p.a_con,
                        a_row=p.a_row, a_col=p.a_col, a_val=np.abs(p.a_val), b=p.b)
    return oracle.operators.forward(pa, np.abs(U), np.abs(V))


# ld 16: factors in rows of 16 columns (the solver's padded FP64 layout, on
# which the completion forward map runs its two-columns-per-lane kernel)
@pytest.mark.parametrize("name,ld", [("mc_10000", None), ("mc_10000", 16), ("mc_20000", None),
                                     ("mc_20000", 32), ("maxcut_torus100", None),
                                     ("maxcut_gnm20000", None)])
def test_fullsize_forward_adjoint_f64(device, name, ld):
    import torch
    from paper_2403_09133_amd import Context
    p = _problem(name)
    r = _rank(p)
    rng = np.random.default_rng(21)
    U, V = rng.standard_normal((p.n, r)), rng.standard_normal((p.n, r))
    w = rng.standard_normal(p.m)
    refz = oracle.operators.forward(p, U, V)
    refa = oracle.operators.adjoint(p, w, 1.0, V)

    def dev(a):
        if ld is None or a.ndim == 1:
            return torch.tensor(a, device=device)
        big = torch.zeros((a.shape[0], ld), dtype=torch.float64, device=device)
        big[:, :a.shape[1]] = torch.tensor(a, device=device)
        return big[:, :a.shape[1]]

    with Context(p) as ctx:
        Ud, Vd, wd = (dev(a) for a in (U, V, w))
        z = torch.zeros(p.m, dtype=torch.float64, device=device)
        out = dev(np.zeros((p.n, r)))  # the adjoint writes with V's row stride
        ctx.apply_A(Ud, Vd, z)
        ctx.apply_AT_V(wd, Vd, out)
        torch.cuda.synchronize()
        gz, ga = z.cpu().numpy(), out.cpu().numpy()
    assert np.linalg.norm(gz - refz) <= 1e-12 * np.linalg.norm(refz)
    assert np.all(np.abs(gz - refz) <= 1e-12 * _abs_bound_forward(p, U, V) + 1e-300)
    assert np.linalg.norm(ga - refa) <= 1e-12 * np.linalg.norm(refa)


@pytest.mark.parametrize("name", ["mc_10000", "mc_20000", "maxcut_gnm20000"])
def test_fullsize_forward_adjoint_f32(device, name):
    import torch
    from paper_2403_09133_amd import Context
    p = _problem(name)
    r = _rank(p)
    rng = np.random.default_rng(22)
    U32 = rng.standard_normal((p.n, r)).astype(np.float32)
    V32 = rng.standard_normal((p.n, r)).astype(np.float32)
    w32 = rng.standard_normal(p.m).astype(np.float32)
    U, V, w = (a.astype(np.float64) for a in (U32, V32, w32))
    refz = oracle.operators.forward(p, U, V)
    refa = oracle.operators.adjoint(p, w, 1.0, V)
    with Context(p) as ctx:
        Ud, Vd, wd = (torch.tensor(a, device=device) for a in (U32, V32, w32))
        z = torch.zeros(p.m, dtype=torch.float32, device=device)
        out = torch.zeros_like(Vd)
        ctx.apply_A(Ud, Vd, z)
        ctx.apply_AT_V(wd, Vd, out)
        torch.cuda.synchronize()
        gz, ga = z.cpu().numpy().astype(np.float64), out.cpu().numpy().astype(np.float64)
    bound = _abs_bound_forward(p, U, V)
    assert np.all(np.abs(gz - refz) <= 6e-8 * np.abs(refz) + 1.2e-7 * bound + 1e-30)
    assert np.linalg.norm(ga - refa) <= 1e-6 * np.linalg.norm(refa)


@pytest.mark.parametrize("name", ["mc_10000", "mc_20000", "maxcut_torus100"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fullsize_cg_iterations(device, name, dtype):
    import torch
    from paper_2403_09133_amd import Context
    p = _problem(name)
    r = _rank(p)
    rng = np.random.default_rng(23)
    W = rng.standard_normal((p.n, r)) / math.sqrt(r)
    R = rng.standard_normal((p.n, r))
    if dtype == "f32":
        W, R = (a.astype(np.float32).astype(np.float64) for a in (W, R))
    rho, gamma, K = 2.0, 1.5, 5
    apply_M = oracle.cg.cg_operator(p, W, rho, gamma)
    Xref, itref, _, _ = oracle.cg.cg(apply_M, R, 1e-14, K)
    assert itref == K
    tdt = torch.float64 if dtype == "f64" else torch.float32
    with Context(p) as ctx:
        Wd = torch.tensor(W, dtype=tdt, device=device)
        Rd = torch.tensor(R, dtype=tdt, device=device)
        Xd = torch.zeros_like(Wd)
        info = ctx.cg_solve(Wd, Rd, Xd, rho, gamma, 1e-14, K)
        X = Xd.cpu().numpy().astype(np.float64)
    assert info["iters"] == K
    tol = 1e-10 if dtype == "f64" else 1e-4
    assert np.linalg.norm(X - Xref) <= tol * np.linalg.norm(Xref)



def test_fullsize_batch_sampled(device):
    """The benchmarked batch (512 MaxCut SDPs, n in [50, 2000]) in one
    persistent launch, FP64: every instance either meets eq. (stop) or stops
    at the iteration cap, and nearly all meet it; on sampled instances (the
    first, the last, two in between and the largest) the oracle recomputes the
    Appendix-B measures from the returned factors and multipliers, and on three
    of them (the smallest, a middle one and the largest) an oracle solve from
    the same start, with the batched form's rank cap of 32, reaches the same
    objective to 1e-6 relative."""
    from oracle.options import Options, paper_defaults
    from paper_2403_09133_amd import Context, default_options, lorads
    from paper_2403_09133_amd.params import family_params
    probs = sdpgen.batch_maxcut(512, 2000, 50, 2000, 3.0, 20.0, "pm1")
    U0 = [sdpgen.random_init_U(p.n, int(math.ceil(math.log2(p.n))), 2000 + i)
          for i, p in enumerate(probs)]
    pd = family_params("maxcut", 1000)

    def opts(**kw):
        return default_options(r0=1, **{**pd, **kw})

    ns = [p.n for p in probs]
    big, small = int(np.argmax(ns)), int(np.argmin(ns))
    mid = int(np.argsort(ns)[len(ns) // 2])
    sample = sorted({0, 100, 255, 511, big, small, mid})
    with Context(probs) as ctx:
        res = ctx.admm_solve(U0, opts(batch_mode=1))
        sols = {i: ctx.get_solution(i, res[i]["rank"]) for i in sample}
    for r in res:
        assert r["status"] in (0, lorads.LORADS_MAXITER), r
        assert r["status"] == lorads.LORADS_MAXITER or r["kkt"] < 1e-6, r
    conv = sum(r["status"] == 0 for r in res)
    print(f"[test] batch: {conv}/512 meet eq. (stop)", flush=True)
    assert conv >= 500
    for i in sample:
        p, r = probs[i], res[i]
        U, V, lam = sols[i]
        m = oracle.metrics.appendix_b(p, 0.5 * (U + V), lam)
        assert abs(m["obj"] - r["obj"]) <= 1e-10 * max(1.0, abs(m["obj"])), (i, m["obj"], r["obj"])
        assert abs(m["pinf"] - r["pinf"]) <= 1e-9, (i, m["pinf"], r["pinf"])
        assert abs(m["gap"] - r["gap"]) <= 1e-9, (i, m["gap"], r["gap"])
    for i in (small, mid, big):
        p, r = probs[i], res[i]
        assert r["status"] == 0, (i, r)
        o = Options(**paper_defaults(p.kind, p.n), r_limit=32)
        ref = oracle.lorads.lorads(p, U0[i], o, with_metrics=False)
        oobj = oracle.operators.cost_inner(p, ref["U_hat"], ref["U_hat"])
        assert ref["phase2"]["converged"], i
        assert abs(r["obj"] - oobj) <= 1e-6 * abs(oobj), (i, p.n, r["obj"], oobj)


def _nuclear_norm_planted(L, R):
    # M = L R^T = Q_L (T_L T_R^T) Q_R^T with L = Q_L T_L, R = Q_R T_R: the
    # singular values of M are those of the k x k core
    tl = np.linalg.qr(L, mode="r")
    tr = np.linalg.qr(R, mode="r")
    return float(np.linalg.svd(tl @ tr.T, compute_uv=False).sum())


@pytest.mark.parametrize("name", ["mc_10000", "mc_20000"])
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_fullsize_completion_solve(device, name, precision):
    """The completion solves of the benchmark (n_X = 20000, m = 4,605,170,
    r = 15, and the headline n_X = 40000, m = 15,683,710, r = 17; ranks
    round(ln m)), with the benchmarked options and start, FP64, FP32-CG and
    mixed (FP32 Phase-I maps as well): it meets eq. (stop); the oracle recomputes the objective, the
    primal infeasibility and the gap (Appendix B) from the returned factors and
    multipliers at full size; the objective equals the nuclear norm of the
    planted matrix (the completion SDP's value at exact recovery) and the
    planted matrix is recovered."""
    from paper_2403_09133_amd import Context, lorads
    from paper_2403_09133_amd.params import initial_rank, solver_options
    p = _problem(name)
    r0 = initial_rank(p.kind, p.n, p.m)
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    print(f"[test] {name} precision {precision}: n={p.n} m={p.m} r0={r0}", flush=True)
    with Context(p) as ctx:
        res = ctx.admm_solve([U0], solver_options(p.kind, p.n, r0, precision))[0]
        U, V, lam = ctx.get_solution(0, res["rank"])
    assert res["status"] == lorads.LORADS_OK and res["kkt"] < 1e-6, res
    Uh = 0.5 * (U + V)
    nrm = oracle.operators.norms(p)
    obj = oracle.operators.cost_inner(p, Uh, Uh)
    pinf = float(np.linalg.norm(oracle.operators.forward(p, Uh, Uh) - p.b)) / (1.0 + nrm["b_1"])
    by = float(p.b @ -lam)
    gap = (obj - by) / (1.0 + abs(obj) + abs(by))
    assert abs(obj - res["obj"]) <= 1e-10 * abs(obj), (obj, res["obj"])
    assert abs(pinf - res["pinf"]) <= 1e-9, (pinf, res["pinf"])
    assert abs(gap - res["gap"]) <= 1e-9, (gap, res["gap"])
    nuc = _nuclear_norm_planted(p.meta["L"], p.meta["R"])
    assert abs(res["obj"] - nuc) <= 1e-6 * nuc, (res["obj"], nuc)
    assert oracle.metrics.mc_recovery_error(p, Uh) < 1e-6


@pytest.mark.parametrize("name", ["maxcut_torus100", "maxcut_gnm20000"])
@pytest.mark.parametrize("precision", [0, 1])
def test_fullsize_maxcut_solve(device, name, precision):
    """The MaxCut instances of the FP32-CG configuration (100 x 100 torus with
    +-1 weights; G(20000, 60000) with unit weights), FP64 and FP32-CG, rank
    from ceil(log2 n) and grown in Phase I: the solve meets eq. (stop) at 1e-6,
    and the oracle recomputes every Appendix-B measure from the returned
    factors and multipliers (its own Lanczos for the smallest eigenvalue of the
    dual slack): each agrees with the library's, and primal infeasibility,
    dual infeasibility and gap are all below 2e-6."""
    from paper_2403_09133_amd import Context, lorads
    from paper_2403_09133_amd.params import initial_rank, solver_options
    p = _problem(name)
    r0 = initial_rank(p.kind, p.n, p.m)
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    print(f"[test] {name} precision {precision}: n={p.n} r0={r0}", flush=True)
    with Context(p) as ctx:
        res = ctx.admm_solve([U0], solver_options(p.kind, p.n, r0, precision))[0]
        U, V, lam = ctx.get_solution(0, res["rank"])
    assert res["status"] == lorads.LORADS_OK and res["kkt"] < 1e-6, res
    m = oracle.metrics.appendix_b(p, 0.5 * (U + V), lam)
    assert abs(m["obj"] - res["obj"]) <= 1e-10 * abs(m["obj"]), (m["obj"], res["obj"])
    assert abs(m["pinf"] - res["pinf"]) <= 1e-9
    assert abs(m["gap"] - res["gap"]) <= 1e-9
    assert abs(m["dinf"] - res["dinf"]) <= 1e-8, (m["dinf"], res["dinf"])
    for k in ("pinf", "dinf"):
        assert m[k] <= 2e-6, (k, m[k])
    assert abs(m["gap"]) <= 2e-6, m["gap"]


_SMALL_C2 = {}


def _small_c2(name):
    # the C2 graph families at sizes the oracle solves in seconds
    if name not in _SMALL_C2:
        p = (sdpgen.maxcut_torus(20, 20, 1002, "pm1") if name == "torus20"
             else sdpgen.maxcut_gnm(2000, 6000, 1003, "unit"))
        r0 = int(math.ceil(math.log2(p.n)))
        U0 = sdpgen.random_init_U(p.n, r0, 3)
        from oracle.options import Options, paper_defaults
        _SMALL_C2[name] = (p, U0, oracle.lorads.lorads(p, U0, Options(**paper_defaults(p.kind, p.n))))
    return _SMALL_C2[name]


def _certified_interval(p, Uh, lam):
    """[lower, upper] around the SDP optimum from a MaxCut result: the cost of
    the (nearly feasible) X = U U^T is an upper bound, and y + lambda_min 1
    (y = -lam) is dual feasible because the constraints sum to the identity, so
    b^T y + n min(0, lambda_min) is a lower bound."""
    obj = oracle.operators.cost_inner(p, Uh, Uh)
    lmin = oracle.metrics.lambda_min(p, lam)
    lower = float(p.b @ -lam) + p.n * min(0.0, lmin)
    return lower, obj


@pytest.mark.parametrize("name", ["torus20", "gnm2000"])
@pytest.mark.parametrize("precision", [0, 1])
def test_c2_family_matches_oracle(device, name, precision):
    """The two C2 graph families at oracle-sized orders (20 x 20 torus, +-1
    weights; G(2000, 6000), unit weights) from the same start: both meet
    eq. (stop) at 1e-6.  On the torus both reach the optimum and the
    objectives agree to 1e-6 relative.  On G(2000, 6000) at rank 11 (below the
    Barvinok-Pataki bound of 63) a first-order stationary point of the
    factored problem need not be optimal, and which one a run stops at follows
    its rounding: the oracle's own result has lambda_min(S) = -7e-3 there, a
    certified interval 2.8e-3 wide, which Appendix B reports as a dual
    infeasibility of 1.2e-6 (it divides by 1 + ||C||_1).  There both results
    must meet Appendix B to 2e-6, each certified interval (primal cost above,
    a dual-feasible shift of the multipliers below) must be narrower than
    1e-2 relative, and the two intervals must overlap (both hold the
    optimum)."""
    from paper_2403_09133_amd import Context
    from paper_2403_09133_amd.params import solver_options
    p, U0, ref = _small_c2(name)
    assert ref["phase2"]["converged"]
    with Context(p) as ctx:
        res = ctx.admm_solve([U0], solver_options(p.kind, p.n, U0.shape[1], precision))[0]
        U, V, lam = ctx.get_solution(0, res["rank"])
    assert res["status"] == 0 and res["kkt"] < 1e-6, res
    oobj = ref["metrics"]["obj"]
    if name == "torus20":
        assert abs(res["obj"] - oobj) <= 1e-6 * abs(oobj), (res["obj"], oobj)
        return
    lo_g, hi_g = _certified_interval(p, 0.5 * (U + V), lam)
    lo_o, hi_o = _certified_interval(p, ref["U_hat"], ref["lam"])
    scale = abs(oobj)
    print(f"[test] {name}: gpu [{lo_g:.6f}, {hi_g:.6f}] oracle [{lo_o:.6f}, {hi_o:.6f}]", flush=True)
    for lo, hi in ((lo_g, hi_g), (lo_o, hi_o)):
        assert hi - lo <= 1e-2 * scale, (lo, hi)
    assert res["pinf"] <= 2e-6 and res["dinf"] <= 2e-6 and abs(res["gap"]) <= 2e-6, res
    mo = ref["metrics"]
    assert mo["pinf"] <= 2e-6 and mo["dinf"] <= 2e-6 and abs(mo["gap"]) <= 2e-6, mo
    # the primal costs are upper bounds only up to the 1e-6 infeasibility
    assert max(lo_g, lo_o) <= min(hi_g, hi_o) + 1e-6 * scale
