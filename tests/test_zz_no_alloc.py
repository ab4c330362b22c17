"""lorads_cg_solve_noalloc, the CG entry point that allocates nothing, against
lorads_cg_solve on the same inputs: the same kernels and launches, so the
solution, iteration count and residual agree bit for bit.  Two calls in a row,
the second with a smaller factor (the workspace keeps the first call's
contents, which the second must not see), for each structure class and both
precisions; a call whose workspace exceeds the 64 MiB static array is rejected
with EINVAL, and the entry point works again after it."""
import math

import numpy as np
import pytest

import sdpgen

pytestmark = pytest.mark.gpu

PROBS = {
    "pair": sdpgen.mc_planted(300, 250, 3, 5, count=12000),
    "diag": sdpgen.maxcut_er(400, 0.03, 7, "pm1"),
    "generic": sdpgen.generic_random(40, 30, 5),
}
# (structure, rank of the first call, rank of the second, smaller, call)
CASES = [("pair", 13, 5), ("diag", 9, 4), ("generic", 8, 3)]


def _inputs(p, r, seed, tdt, device):
    import torch
    rng = np.random.default_rng(seed)
    W = torch.tensor(rng.standard_normal((p.n, r)) / math.sqrt(r), dtype=tdt, device=device)
    R = torch.tensor(rng.standard_normal((p.n, r)), dtype=tdt, device=device)
    X0 = torch.tensor(0.1 * rng.standard_normal((p.n, r)), dtype=tdt, device=device)
    return W, R, X0


@pytest.mark.parametrize("kind,r1,r2", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_cg_solve(device, kind, r1, r2, dtype):
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS[kind]
    tdt = torch.float64 if dtype == "f64" else torch.float32
    print(f"[test] noalloc {kind} {dtype} r={r1},{r2} n={p.n} m={p.m}", flush=True)
    with Context(p) as ctx:
        for call, r in enumerate((r1, r2)):
            W, R, X0 = _inputs(p, r, 100 + call, tdt, device)
            Xa, Xb = X0.clone(), X0.clone()
            a = ctx.cg_solve(W, R, Xa, 2.0, 1.5, 1e-10, 30)
            b = ctx.cg_solve_noalloc(W, R, Xb, 2.0, 1.5, 1e-10, 30)
            torch.cuda.synchronize()
            assert a["iters"] == b["iters"] > 0, (a, b)
            assert a["status"] == b["status"]
            assert a["relres"] == b["relres"]
            assert torch.equal(Xa, Xb), float((Xa - Xb).abs().max())


def test_noalloc_rejects_oversized_workspace(device):
    import torch
    from paper_2403_09133_amd import Context, lorads
    # completion rows of 256 FP64 columns: six buffers of 30000 x 256 doubles
    # (61 MB each) do not fit the 64 MiB workspace
    p = sdpgen.mc_planted(15000, 15000, 2, 3, count=20000)
    print(f"[test] noalloc oversized: n={p.n} r=256", flush=True)
    with Context(p) as ctx:
        W, R, X0 = _inputs(p, 256, 7, torch.float64, device)
        with pytest.raises(lorads.LoradsError) as e:
            ctx.cg_solve_noalloc(W, R, X0, 2.0, 1.5, 1e-8, 5)
        assert e.value.status == lorads.LORADS_EINVAL
        assert "static workspace" in str(e.value)
        # a call that fits still runs afterwards
        W, R, X0 = _inputs(p, 4, 8, torch.float64, device)
        Xa, Xb = X0.clone(), X0.clone()
        a = ctx.cg_solve(W, R, Xa, 2.0, 1.5, 1e-10, 20)
        b = ctx.cg_solve_noalloc(W, R, Xb, 2.0, 1.5, 1e-10, 20)
        torch.cuda.synchronize()
        assert a["iters"] == b["iters"] and torch.equal(Xa, Xb)
