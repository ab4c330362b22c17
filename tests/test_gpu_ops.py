"""GPU parity of the operator entry points against the FP64 oracle.

Tolerances: FP64 results within 1e-12 relative (norm-wise) plus the
componentwise rounding bound 1e-12 * sum |a| |U| |V|; FP32 results within 2e-5
relative (about 100 unit roundoffs of float accumulated over short sums).
"""
import math

import numpy as np
import pytest

import oracle
import sdpgen

pytestmark = pytest.mark.gpu


def _problems():
    out = {}
    out["diag_er200"] = sdpgen.config_instance("maxcut_er200")
    p = sdpgen.mc_planted(70, 55, 3, 11, count=1800)
    # shuffle the caller order to exercise the internal permutation
    rng = np.random.default_rng(5)
    perm = rng.permutation(p.m)
    p.a_con = np.argsort(perm).astype(np.int32)[p.a_con]
    p.b = p.b[perm]
    out["pair_mc_perm"] = p
    q = sdpgen.mc_planted(40, 30, 2, 12, count=500)
    q.a_val = np.random.default_rng(3).uniform(0.2, 1.0, q.m)  # non-uniform pair coefficients
    out["pair_nonuniform"] = q
    out["generic_small"] = sdpgen.generic_random(14, 9, 4)
    return out


PROBS = _problems()


def _rand(n, r, seed):
    return np.random.default_rng(seed).standard_normal((n, r))


def _abs_bound_forward(p, U, V):
    Ua, Va = np.abs(U), np.abs(V)
    pa = sdpgen.Problem(n=p.n, m=p.m, c_row=p.c_row, c_col=p.c_col, c_val=p.c_val, a_con=p.a_con,
                        a_row=p.a_row, a_col=p.a_col, a_val=np.abs(p.a_val), b=p.b)
    return oracle.operators.forward(pa, Ua, Va)


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("r", [1, 7, 15, 33])
def test_forward_f64(device, name, r):
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS[name]
    U, V = _rand(p.n, r, 1), _rand(p.n, r, 2)
    ref = oracle.operators.forward(p, U, V)
    with Context(p) as ctx:
        Ud = torch.tensor(U, device=device)
        Vd = torch.tensor(V, device=device)
        z = torch.zeros(p.m, dtype=torch.float64, device=device)
        ctx.apply_A(Ud, Vd, z)
        torch.cuda.synchronize()
        got = z.cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    bound = _abs_bound_forward(p, U, V)
    assert np.all(np.abs(got - ref) <= 1e-12 * bound + 1e-300)


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("r", [1, 8, 15, 40])
@pytest.mark.parametrize("c_scale", [0.0, 1.0, -0.5])
def test_adjoint_f64(device, name, r, c_scale):
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS[name]
    V = _rand(p.n, r, 3)
    w = np.random.default_rng(4).standard_normal(p.m)
    ref = oracle.operators.adjoint(p, w, c_scale, V)
    with Context(p) as ctx:
        Vd = torch.tensor(V, device=device)
        wd = torch.tensor(w, device=device)
        out = torch.zeros_like(Vd)
        ctx.apply_AT_V(wd, Vd, out, c_scale=c_scale)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-12 * max(np.linalg.norm(ref), 1e-300)


@pytest.mark.parametrize("name", sorted(PROBS))
def test_forward_adjoint_f32(device, name):
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS[name]
    r = 12
    U, V = _rand(p.n, r, 5), _rand(p.n, r, 6)
    w = np.random.default_rng(7).standard_normal(p.m)
    U32, V32, w32 = U.astype(np.float32), V.astype(np.float32), w.astype(np.float32)
    refz = oracle.operators.forward(p, U32.astype(np.float64), V32.astype(np.float64))
    refa = oracle.operators.adjoint(p, w32.astype(np.float64), 1.0, V32.astype(np.float64))
    with Context(p) as ctx:
        Ud, Vd, wd = (torch.tensor(a, device=device) for a in (U32, V32, w32))
        z = torch.zeros(p.m, dtype=torch.float32, device=device)
        out = torch.zeros_like(Vd)
        ctx.apply_A(Ud, Vd, z)
        ctx.apply_AT_V(wd, Vd, out)
        torch.cuda.synchronize()
        gz, ga = z.cpu().numpy().astype(np.float64), out.cpu().numpy().astype(np.float64)
    # FP32 path: coefficients stored in float (relative error <= 2^-24 each),
    # FP64 accumulation, one float rounding of the result
    bound = _abs_bound_forward(p, U32.astype(np.float64), V32.astype(np.float64))
    assert np.all(np.abs(gz - refz) <= 6e-8 * np.abs(refz) + 1.2e-7 * bound + 1e-30)
    assert np.linalg.norm(ga - refa) <= 1e-6 * np.linalg.norm(refa)


# (r, ld): odd stride; even stride shorter than the 16-column lane group
# (the two-column form must not be used: its last row would read past the
# buffer); padded rows with nonzero padding on the two-column form (16 and 8
# columns), whose masks must keep the padding out of every sum
@pytest.mark.parametrize("r,ld", [(9, 13), (9, 10), (15, 16), (6, 8)])
def test_leading_dimension(device, r, ld):
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS["pair_mc_perm"]
    big = torch.tensor(_rand(p.n, ld, 8), device=device)
    U = big[:, :r]
    ref = oracle.operators.forward(p, U.cpu().numpy(), U.cpu().numpy())
    with Context(p) as ctx:
        z = torch.zeros(p.m, dtype=torch.float64, device=device)
        ctx.apply_A(U, U, z)
        w = torch.tensor(np.random.default_rng(1).standard_normal(p.m), device=device)
        out = torch.full((p.n, ld), 7.0, dtype=torch.float64, device=device)
        ctx.apply_AT_V(w, U, out[:, :r])
        torch.cuda.synchronize()
    assert np.linalg.norm(z.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    refa = oracle.operators.adjoint(p, w.cpu().numpy(), 1.0, U.cpu().numpy())
    o = out.cpu().numpy()
    assert np.linalg.norm(o[:, :r] - refa) <= 1e-12 * np.linalg.norm(refa)
    assert np.all(o[:, r:] == 7.0)  # padding never written


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("r", [3, 10, 37])
def test_cg_parity(device, name, dtype, r):
    """Ranks 3, 10 and 37 put 1, 4 and 16 lanes on a factor row (4 columns per
    lane, the last ones partly masked)."""
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS[name]
    W = _rand(p.n, r, 9) / math.sqrt(r)
    R = _rand(p.n, r, 10)
    rho, gamma = 3.0, 1.5
    tol = 1e-10 if dtype == "f64" else 1e-5
    apply_M = oracle.cg.cg_operator(p, W, rho, gamma)
    Xref, itref, relref, _ = oracle.cg.cg(apply_M, R, tol, 500)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    with Context(p) as ctx:
        Wd = torch.tensor(W, dtype=tdt, device=device)
        Rd = torch.tensor(R, dtype=tdt, device=device)
        Xd = torch.zeros_like(Wd)
        info = ctx.cg_solve(Wd, Rd, Xd, rho, gamma, tol, 500)
        X = Xd.cpu().numpy().astype(np.float64)
    # the system residual of the GPU solution, evaluated by the oracle
    res = np.linalg.norm(R - apply_M(X)) / np.linalg.norm(R)
    if dtype == "f64":
        assert info["status"] == 0 and info["relres"] <= tol
        assert abs(info["iters"] - itref) <= 1
        assert np.linalg.norm(X - Xref) <= 1e-8 * np.linalg.norm(Xref)
        assert res <= 10 * tol
    else:
        assert res <= 1e-4
        assert np.linalg.norm(X - Xref) <= 1e-3 * np.linalg.norm(Xref)


def test_cg_warm_start(device):
    """x0 != 0: the solve continues from x0 (same solution as from zero)."""
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS["pair_mc_perm"]
    r = 6
    W = _rand(p.n, r, 11) / math.sqrt(r)
    R = _rand(p.n, r, 12)
    apply_M = oracle.cg.cg_operator(p, W, 2.0, 0.7)
    Xref, _, _, _ = oracle.cg.cg(apply_M, R, 1e-12, 1000)
    x0 = Xref + 1e-3 * _rand(p.n, r, 13)
    with Context(p) as ctx:
        Wd = torch.tensor(W, device=device)
        Rd = torch.tensor(R, device=device)
        Xd = torch.tensor(x0, device=device)
        info = ctx.cg_solve(Wd, Rd, Xd, 2.0, 0.7, 1e-6, 1000)
        X = Xd.cpu().numpy()
    assert np.linalg.norm(R - apply_M(X)) <= 1e-6 * np.linalg.norm(R - apply_M(x0)) * 1.01


@pytest.mark.parametrize("shape", [(1000, 7, 7), (4099, 15, 15), (333, 20, 5), (16, 1, 3)])
def test_gram_mfma(device, shape):
    import torch
    from paper_2403_09133_amd import gram
    n, ra, rb = shape
    A = _rand(n, ra, 14)
    B = _rand(n, rb, 15)
    Ad = torch.tensor(A, device=device)
    Bd = torch.tensor(B, device=device)
    G = torch.zeros((ra, rb), dtype=torch.float64, device=device)
    gram(Ad, Bd, G)
    ref = oracle.metrics.gram(A, B)
    assert np.linalg.norm(G.cpu().numpy() - ref) <= 1e-13 * n * np.linalg.norm(ref) / 10 + 1e-12


@pytest.mark.parametrize("d", [1e-3, 0.3])
def test_recovery_error_path_matches_oracle(device, d):
    """The library's recovery error (Gram products on the device, expanded
    norm) against the oracle's entry-by-entry definition, on factors whose
    error is known: U1 = (1 + d) L + a small perturbation, U2 = R."""
    from paper_2403_09133_amd.report import completion_recovery_error
    p = sdpgen.mc_planted(700, 500, 5, 9, count=5000)
    L, R = p.meta["L"], p.meta["R"]
    rng = np.random.default_rng(3)
    U = np.vstack([(1.0 + d) * L, R]) + 1e-4 * rng.standard_normal((p.n, 5))
    ref = oracle.metrics.mc_recovery_error(p, U)
    got = completion_recovery_error(U, L, R)
    assert abs(ref - d) <= 0.05 * d
    assert abs(got - ref) <= 1e-7 * ref, (got, ref)


@pytest.mark.parametrize("name", ["diag_er200", "pair_mc_perm", "generic_small"])
def test_dual_lambda_min(device, name):
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS[name]
    lam = np.random.default_rng(16).standard_normal(p.m) * 0.3
    ref = oracle.metrics.lambda_min(p, lam)
    with Context(p) as ctx:
        got = ctx.dual_lambda_min(torch.tensor(lam, device=device), max_steps=400)
    scale = max(1.0, abs(ref))
    assert abs(got - ref) <= 1e-8 * scale


def _lane_group(r):
    g = 1
    while g < r:
        g *= 2
    return g


# rows of 200 incident entries: two staging passes of 128 per row
_LONG_ROWS = sdpgen.mc_planted(300, 300, 2, 13, count=60000)


@pytest.mark.parametrize("name", ["pair_mc_perm", "pair_nonuniform", "long_rows"])
@pytest.mark.parametrize("r", [5, 16, 17, 23, 24, 30])
@pytest.mark.parametrize("c_scale", [0.0, -0.5])
def test_adjoint_two_column_layout(device, name, r, c_scale):
    """The FP64 adjoint on rows padded to the lane group (the two-columns-per-
    lane form; ranks 17..24 add a third column per lane) against the oracle to
    1e-12, with nonzero padding in V that the masks must keep out and padding
    in the output that must stay unwritten."""
    import torch
    from paper_2403_09133_amd import Context
    p = _LONG_ROWS if name == "long_rows" else PROBS[name]
    ld = max(_lane_group(r), 8 * ((r + 7) // 8))
    big = torch.tensor(_rand(p.n, ld, 21), device=device)
    V = big[:, :r]
    w = np.random.default_rng(22).standard_normal(p.m)
    ref = oracle.operators.adjoint(p, w, c_scale, V.cpu().numpy())
    with Context(p) as ctx:
        out = torch.full((p.n, ld), 7.0, dtype=torch.float64, device=device)
        ctx.apply_AT_V(torch.tensor(w, device=device), V, out[:, :r], c_scale=c_scale)
        torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.linalg.norm(o[:, :r] - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.all(o[:, r:] == 7.0)


@pytest.mark.parametrize("name", ["pair_mc_perm", "pair_nonuniform", "long_rows"])
@pytest.mark.parametrize("r", [3, 12, 15, 17, 30, 33])
def test_forward_f32_four_column_layout(device, name, r):
    """The FP32 forward map on rows padded to four columns per lane (G =
    pow2(ceil(r / 4)) >= 4 lanes, 16-byte loads; nonzero padding that the
    masks must keep out) against the oracle's FP64 map of the same FP32
    inputs.  Bound: a lane's chain of 8 fused multiply-adds, log2 G levels of
    the group tree and the final rounding each add at most 2^-24 of the sum of
    the terms' magnitudes (the coefficient's FP32 storage one more)."""
    import math
    import torch
    from paper_2403_09133_amd import Context
    p = _LONG_ROWS if name == "long_rows" else PROBS[name]
    g = max(4, _lane_group((r + 3) // 4))
    ld = 4 * g
    big = _rand(p.n, ld, 31).astype(np.float32)
    big2 = _rand(p.n, ld, 32).astype(np.float32)
    U, V = big[:, :r].astype(np.float64), big2[:, :r].astype(np.float64)
    ref = oracle.operators.forward(p, U, V)
    with Context(p) as ctx:
        Ud, Vd = torch.tensor(big, device=device)[:, :r], torch.tensor(big2, device=device)[:, :r]
        z = torch.zeros(p.m, dtype=torch.float32, device=device)
        ctx.apply_A(Ud, Vd, z)
        torch.cuda.synchronize()
        got = z.cpu().numpy().astype(np.float64)
    u = 2.0 ** -24
    bound = _abs_bound_forward(p, U, V)
    assert np.all(np.abs(got - ref) <= (10 + math.log2(g)) * u * bound + u * np.abs(ref) + 1e-30)


@pytest.mark.parametrize("name", ["pair_mc_perm", "pair_nonuniform", "long_rows"])
@pytest.mark.parametrize("r", [3, 15, 17, 33])
@pytest.mark.parametrize("c_scale", [0.0, 1.0])
def test_adjoint_f32_four_column_layout(device, name, r, c_scale):
    """The FP32 adjoint on rows padded to four columns per lane (nonzero
    padding in V, output padding unwritten) against the oracle's FP64 product
    of the same FP32 inputs, norm-wise to 1e-6 as the one-column FP32 form."""
    import torch
    from paper_2403_09133_amd import Context
    p = _LONG_ROWS if name == "long_rows" else PROBS[name]
    g = max(4, _lane_group((r + 3) // 4))
    ld = 4 * g
    big = _rand(p.n, ld, 41).astype(np.float32)
    w = np.random.default_rng(42).standard_normal(p.m).astype(np.float32)
    ref = oracle.operators.adjoint(p, w.astype(np.float64), c_scale, big[:, :r].astype(np.float64))
    with Context(p) as ctx:
        Vd = torch.tensor(big, device=device)[:, :r]
        out = torch.full((p.n, ld), 7.0, dtype=torch.float32, device=device)
        ctx.apply_AT_V(torch.tensor(w, device=device), Vd, out[:, :r], c_scale=c_scale)
        torch.cuda.synchronize()
    o = out.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(o[:, :r] - ref) <= 1e-6 * np.linalg.norm(ref)
    assert np.all(o[:, r:] == 7.0)
