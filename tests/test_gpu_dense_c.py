"""Dense cost matrices on the matrix cores (the general SDP families of the
paper's SDPLIB experiments with a dense C, such as the Lovasz theta SDP).

A C with at least n^2 / 4 entries and n >= 256 is also kept dense, and every
product with C runs as an MFMA product over 16-row tiles of C and ranges of
its columns (partials added in a fixed order).  Checks:
  * the layout flag, set on the dense cases and not on a sparse C of the
    same order;
  * lorads_apply_AT_V against the oracle's (c_scale C + A*(w)) V, FP64 to
    1e-12 and FP32 to 2e-5 relative, for a random dense symmetric C with
    general constraints (any transposed or misplaced tile fails) and for the
    theta cost -J, ranks 1 .. 64 (one to four column tiles, ragged ones);
  * min <C, X> s.t. tr X = 1 with a random dense symmetric C: the optimum
    is the smallest eigenvalue of C (numpy's eigvalsh, independent code), to
    1e-6 relative, at n = 400 and at n = 2048, where the dense C (4.2M
    entries, 32 MB) is the solve's whole operator work.
Solves of the Lovasz theta SDP beyond the small closed forms (odd cycles up
to C_21, random graphs of order 40 and 60 against an interior-point solve)
are in tests/test_gpu_solve.py; they take the family's gamma rule
(gamma = 1 + ||C||_2).
"""
import math

import numpy as np
import pytest

import oracle
import sdpgen
from oracle.options import Options, paper_defaults

pytestmark = pytest.mark.gpu


def _problems():
    return {
        # random dense symmetric C (G G^T + noise, shifted), 12 sparse constraints
        "generic_dense_300": sdpgen.generic_random(300, 12, 5, density=0.01),
        # Lovasz theta of G(260, 0.05): C = -J
        "theta_er260": sdpgen.lovasz_theta(
            260, [tuple(e) for e in zip(*sdpgen.er_gnp_edges(260, 0.05, np.random.default_rng(8)))]),
    }


PROBS = _problems()


def test_dense_flag(device):
    from paper_2403_09133_amd import Context
    for name, p in PROBS.items():
        with Context(p) as ctx:
            assert ctx.problem_info()["c_dense"], name
    sparse = sdpgen.mc_planted(200, 150, 2, 3, count=3000)  # C = I/2 of order 350
    with Context(sparse) as ctx:
        assert not ctx.problem_info()["c_dense"]


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("r", [1, 5, 16, 23, 40, 50, 64])
@pytest.mark.parametrize("c_scale", [1.0, -0.5])
def test_dense_adjoint_f64(device, name, r, c_scale):
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS[name]
    rng = np.random.default_rng(r)
    V = rng.standard_normal((p.n, r))
    for w in (rng.standard_normal(p.m), np.zeros(p.m)):
        ref = oracle.operators.adjoint(p, w, c_scale, V)
        with Context(p) as ctx:
            Vd, wd = torch.tensor(V, device=device), torch.tensor(w, device=device)
            out = torch.full_like(Vd, float("nan"))
            ctx.apply_AT_V(wd, Vd, out, c_scale=c_scale)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), (name, r)


@pytest.mark.parametrize("name", sorted(PROBS))
@pytest.mark.parametrize("r", [19, 64])
def test_dense_adjoint_f32(device, name, r):
    import torch
    from paper_2403_09133_amd import Context
    p = PROBS[name]
    rng = np.random.default_rng(2)
    V = rng.standard_normal((p.n, r)).astype(np.float32)
    w = rng.standard_normal(p.m).astype(np.float32)
    ref = oracle.operators.adjoint(p, w.astype(np.float64), 1.0, V.astype(np.float64))
    with Context(p) as ctx:
        Vd, wd = torch.tensor(V, device=device), torch.tensor(w, device=device)
        out = torch.zeros_like(Vd)
        ctx.apply_AT_V(wd, Vd, out, c_scale=1.0)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 2e-5 * np.linalg.norm(ref)


def _min_eig_problem(n, seed):
    """min <C, X> s.t. tr X = 1, X PSD: C random dense symmetric of order n."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) / math.sqrt(n)
    Cd = 0.5 * (G + G.T)
    ir, ic = np.triu_indices(n)
    ar = np.arange(n)
    return sdpgen.Problem(n=n, m=1, c_row=ir, c_col=ic, c_val=Cd[ir, ic], a_con=np.zeros(n),
                          a_row=ar, a_col=ar, a_val=np.ones(n), b=np.ones(1), kind="generic"), Cd


@pytest.mark.parametrize("n", [400, 2048])
@pytest.mark.parametrize("precision", [0, 1])
def test_dense_min_eigenvalue_solve(device, n, precision):
    from paper_2403_09133_amd import Context, default_options
    p, Cd = _min_eig_problem(n, 21)
    want = float(np.linalg.eigvalsh(Cd)[0])
    r0 = 4
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    print(f"[test] min eigenvalue n={n} precision {precision}", flush=True)
    with Context(p) as ctx:
        assert ctx.problem_info()["c_dense"]
        res = ctx.admm_solve([U0], default_options(r0=r0, precision=precision, time_limit=100.0,
                                                   **paper_defaults(p.kind, p.n)))[0]
    print(f"[test] obj {res['obj']:.10f} (lambda_min {want:.10f}), kkt {res['kkt']:.2e}, "
          f"admm {res['admm_iters']}, {res['t_phase1'] + res['t_phase2']:.2f} s", flush=True)
    assert res["status"] == 0 and res["kkt"] < 1e-6, res
    assert abs(res["obj"] - want) <= 1e-6 * abs(want), (res["obj"], want)


@pytest.mark.parametrize("precision", [0, 1])
def test_dense_theta_solve_certified(device, precision):
    """theta(G(260, 0.05)): C = -J kept dense (every product with it on the
    matrix cores), the family's gamma = 1 + ||C||_2, and an initial rank of 30
    (the rank rule's 15 grows to 23 in Phase I, below the optimum's rank, where
    the run stops at a stationary point with a negative dual slack eigenvalue).
    The oracle recomputes the Appendix-B measures from the returned factors
    and multipliers: P-infeasibility, dual infeasibility and gap all below
    1e-6 certify the objective."""
    from paper_2403_09133_amd import Context, default_options
    p = PROBS["theta_er260"]
    r0 = 30
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    print(f"[test] dense theta precision {precision}", flush=True)
    with Context(p) as ctx:
        assert ctx.problem_info()["c_dense"]
        res = ctx.admm_solve([U0], default_options(r0=r0, precision=precision, time_limit=100.0,
                                                   **paper_defaults(p.kind, p.n)))[0]
        U, V, lam = ctx.get_solution(0, res["rank"])
    print(f"[test] obj {res['obj']:.10f} admm {res['admm_iters']} gamma {res['gamma']:.3f}", flush=True)
    assert res["status"] == 0 and res["kkt"] < 1e-6, res
    assert abs(res["gamma"] - (1.0 + p.n)) <= 1e-9 * p.n
    m = oracle.metrics.appendix_b(p, 0.5 * (U + V), lam)
    assert m["pinf"] <= 1e-6 and m["dinf"] <= 1e-6 and abs(m["gap"]) <= 1e-6, m
    assert abs(m["obj"] - res["obj"]) <= 1e-10 * abs(m["obj"])
