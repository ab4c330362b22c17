#!/usr/bin/env python
"""Benchmark of the LoRADS hot path on one MI355X.

Workload: the planted rank-5 matrix-completion SDP with M of order 10000 x 10000
(X of order 20000), 4,605,170 observed entries, C = I/2, solved by the
two-phase method (warm start + ADMM with CG subproblems) to KKT residual 1e-6,
CG in FP32 with FP64 right-hand sides, dual updates and residuals.

One step = one full two-phase solve from the same random start, the instance
already resident in HBM (setup is outside the timed region).

value  = algorithmic bytes of every constraint-operator application of the
         solves (forward map, adjoint product, fused CG operator; indices,
         coefficients, inputs and outputs counted once) / wall time, in GB/s.
roofline: the dominant kernel's algorithmic bytes per launch / its mean launch
         time from HIP events recorded on the solver's stream during the timed
         steps, against the 8 TB/s HBM peak.
cpu_baseline: the FP64 numpy oracle's forward map and adjoint product at the
         same size on the host, one thread, in the same unit.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources that determine the operator kernels; hardware-counter traffic recorded
# under profiles/ applies only while their hash is unchanged
KERNEL_SOURCES = ["paper_2403_09133_amd/csrc/kernels_struct.hpp", "paper_2403_09133_amd/csrc/kernels.hpp",
                  "paper_2403_09133_amd/csrc/ops.hip", "paper_2403_09133_amd/csrc/common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(symbol: str):
    """HBM bytes per launch of `symbol` from the recorded FETCH_SIZE / WRITE_SIZE
    passes (already scaled by the copy-kernel calibration), or None when no
    record exists or the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    if rec.get("sources_sha256") != kernel_sources_hash():
        return None
    ent = rec.get("kernels", {}).get(symbol)
    return None if ent is None else int(round(ent["hbm_bytes_per_launch"]))
# kernel classes timed by the library (lorads_result.prof_*), with the kernel
# each one runs on the completion workload
KERNEL_CLASSES = {
    "fused CG operator": "kpair_cg_vec<float, 4>",
    "forward map A(UV^T)": "k1_pair_v2<8, 0>",
    "adjoint (C + A*(w))V, gradient form": "kpair_grad_v2<8>",
    "line-search maps A(UD^T+DU^T), A(DD^T)": "k1_pair_v2<8, 3>",
}
WORKLOADS = {
    # name -> (generator key, precision code, description)
    "mc_10000": ("mc_10000", 1, "matrix completion 10000x10000, rank 5, |Omega|=4605170, X of order 20000"),
    "mc_20000": ("mc_20000", 1, "matrix completion 20000x20000, rank 5, 800*d draws deduplicated, X of order 40000"),
    "maxcut_torus100": ("maxcut_torus100", 1, "MaxCut 100x100 torus, +-1 weights, n=m=10000"),
    "maxcut_gnm20000": ("maxcut_gnm20000", 1, "MaxCut G(20000, M=60000), unit weights"),
}


def initial_rank(p) -> int:
    from paper_2403_09133_amd.params import initial_rank as rule
    return rule(p.kind, p.n, p.m)


def lib_options(p, r0, precision, **kw):
    from paper_2403_09133_amd.params import solver_options
    return solver_options(p.kind, p.n, r0, precision, **kw)


def cpu_baseline(p, r: int, budget_s: float = 20.0):
    """Time the oracle's forward map and adjoint product (FP64, numpy) on the
    host, single thread, for a bounded number of applications."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    import oracle
    rng = np.random.default_rng(0)
    U = rng.standard_normal((p.n, r))
    V = rng.standard_normal((p.n, r))
    w = rng.standard_normal(p.m)
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        reps, t = 0, 0.0
        t0 = time.perf_counter()
        while True:
            oracle.operators.forward(p, U, V)
            oracle.operators.adjoint(p, w, 1.0, V)
            reps += 1
            t = time.perf_counter() - t0
            if t > budget_s / 2 or reps >= 8:
                break
    finally:
        if ctx is not None:
            ctx.unregister() if hasattr(ctx, "unregister") else None
    bytes_pair = 2 * (8.0 * p.m + 8.0 * p.m + 2.0 * p.n * r * 8)
    return dict(value=round(reps * bytes_pair / t / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                sample=f"{reps} x (A(UV^T) + (C + A*(y))V) at full size, r={r}, FP64 numpy, "
                       f"{t:.1f} s on the host")


def batch_leg(count: int = 512, sample: int = 16):
    """Batched form: `count` MaxCut SDPs, n ~ U{50..2000}, average degree ~ U[3, 20],
    +-1 weights, rank ceil(log2 n) each, in one persistent launch (workgroup size
    autotuned), FP64 and FP32 CG; against `sample` instances solved one after the
    other by the single-instance path, extrapolated to `count`."""
    import sdpgen
    from paper_2403_09133_amd import Context, default_options
    t = time.time()
    probs = sdpgen.batch_maxcut(count, 2000, 50, 2000, 3.0, 20.0, "pm1")
    U0 = [sdpgen.random_init_U(p.n, int(math.ceil(math.log2(p.n))), 2000 + i) for i, p in enumerate(probs)]
    t_gen = time.time() - t
    from paper_2403_09133_amd.params import family_params
    pd = family_params("maxcut", 1000)

    def opts(**kw):
        return default_options(r0=1, switch_tol=pd["switch_tol"], h=pd["h"], **kw)

    out = dict(instances=count, sum_n=int(sum(p.n for p in probs)),
               sum_edges=int(sum(len(p.meta["edges"][0]) for p in probs)), gen_s=round(t_gen, 2))
    t = time.time()
    ctx = Context(probs)
    out["setup_s"] = round(time.time() - t, 2)
    best, times = ctx.batch_autotune(U0, opts(max_admm_iter=30), (64, 128, 192, 256))
    out["autotune"] = {"block": best, "ms_short_run": {k: round(v, 2) for k, v in times.items()}}
    for name, prec in (("fp64", 0), ("fp32", 1)):
        t = time.perf_counter()
        res = ctx.admm_solve(U0, opts(precision=prec, batch_mode=1))
        dt = time.perf_counter() - t
        out[name] = dict(s=round(dt, 4), converged=int(sum(r["status"] == 0 for r in res)),
                         max_admm_iters=int(max(r["admm_iters"] for r in res)),
                         median_admm_iters=float(np.median([r["admm_iters"] for r in res])),
                         max_kkt=float(max(r["kkt"] for r in res)))
        print(f"[bench] batch {name}: {dt:.3f}s, {out[name]['converged']}/{count} converged",
              file=sys.stderr, flush=True)
    ctx.close()
    sub = probs[:sample]
    ctx = Context(sub)
    t = time.perf_counter()
    res = ctx.admm_solve(U0[:sample], opts(batch_mode=2))
    dt = time.perf_counter() - t
    ctx.close()
    share = sum(p.n for p in sub) / sum(p.n for p in probs)
    out["sequential_sample"] = dict(instances=sample, s=round(dt, 3),
                                    extrapolated_s=round(dt / share, 2),
                                    note="first instances of the batch solved one after the other "
                                         "(single-instance path, FP64); extrapolated by their share of sum n")
    out["speedup_vs_sequential_fp64"] = round(out["sequential_sample"]["extrapolated_s"] / out["fp64"]["s"], 1)
    return out


def learned_leg(count: int = 6):
    """Learned warm start (the shipped MaxCut network) against the cold start on
    `count` held-out graphs shaped like its training set (n ~ U{2000..5000},
    average degree ~ U[4, 16], +-1 weights), FP64 solves to eq. (stop) <= 1e-6
    from the same random U0: mean time-to-KKT, ADMM iterations and the App. B gap."""
    from paper_2403_09133_amd import Context, warmstart as W
    from paper_2403_09133_amd.params import solver_options
    ws = W.WarmStart.load()
    probs = W.instances(count, W.HELDOUT_SEED0 + 500)
    t = time.perf_counter()
    preds = ws.predict(probs)
    t_pred = time.perf_counter() - t
    rows = []
    for p, pr in zip(probs, preds):
        r0 = W.rule_rank(p.n)
        U0 = W.random_start(p, r0)
        with Context(p) as ctx:
            cold = ctx.admm_solve([U0], solver_options("maxcut", p.n, r0))[0]
            warm = ctx.admm_solve([U0], solver_options("maxcut", p.n, r0),
                                  init_lambda=[pr["lambda0"]])[0]
        rows.append((cold, warm))
        print(f"[bench] learned leg n={p.n}: cold {cold['t_total']:.2f}s {cold['admm_iters']} it, "
              f"learned {warm['t_total']:.2f}s {warm['admm_iters']} it", file=sys.stderr, flush=True)
    mean = lambda k, i: float(np.mean([r[i][k] for r in rows]))
    col = lambda k, i: [r[i][k] for r in rows]
    return dict(instances=count, predict_s=round(t_pred, 3),
                cold_admm=col("admm_iters", 0), learned_admm=col("admm_iters", 1),
                cold_gap=[float(f"{g:.2e}") for g in col("gap", 0)],
                learned_gap=[float(f"{g:.2e}") for g in col("gap", 1)],
                caution="a solve that meets eq. (stop) after very few ADMM iterations at a large rho can be "
                        "off by its App. B gap (listed); compare times only together with the gaps",
                cold_mean_s=round(mean("t_total", 0), 3), learned_mean_s=round(mean("t_total", 1), 3),
                cold_mean_admm=mean("admm_iters", 0), learned_mean_admm=mean("admm_iters", 1),
                cold_converged=int(sum(r[0]["status"] == 0 for r in rows)),
                learned_converged=int(sum(r[1]["status"] == 0 for r in rows)),
                max_gap=float(max(max(abs(r[0]["gap"]), abs(r[1]["gap"])) for r in rows)),
                note="held-out evaluation over 48 graphs: profiles/warmstart_maxcut_c5a_eval.md")


def ops_profile(key: str, reps: int):
    """Operator calls only: REPS x (forward map, adjoint product, 20-iteration CG
    solve) in FP32 at r0 columns, then one 256 MiB device-to-device copy whose
    known size calibrates the HBM byte counters."""
    import torch
    import sdpgen
    from paper_2403_09133_amd import Context
    dev = torch.device("cuda")
    p = sdpgen.config_instance(key)
    r = initial_rank(p)
    ctx = Context(p)
    g = torch.Generator().manual_seed(7)
    U = torch.randn(p.n, r, generator=g).to(dev)
    V = torch.randn(p.n, r, generator=g).to(dev) / math.sqrt(r)
    z = torch.empty(p.m, device=dev)
    out = torch.empty_like(V)
    X = torch.empty_like(V)
    for i in range(reps):
        ctx.apply_A(U, V, z)
        ctx.apply_AT_V(z, V, out)
        ctx.cg_solve(V, out, X.zero_(), 2.0, 1.5, 0.0, 20)
        torch.cuda.synchronize()
        print(f"[bench] ops rep {i} done", file=sys.stderr, flush=True)
    calibration_copy()
    ctx.close()


def calibration_copy():
    """One 256 MiB device-to-device copy: its FETCH_SIZE / WRITE_SIZE readings
    against the known size give the scale of the byte counters."""
    import torch
    a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    a.copy_(b)
    torch.cuda.synchronize()
    print(f"[bench] copy of {a.numel() * 4} bytes done", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mc_10000", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-warm-start leg")
    ap.add_argument("--ops-profile", type=int, default=0, metavar="REPS",
                    help="only run REPS applications of each operator at the workload's size (FP32, "
                         "r0 columns) and a 256 MiB device copy, for hardware-counter runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 256 MiB device copy (byte-counter calibration in counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the single-instance and batched paths are measured "
              "on one GPU and there is no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import sdpgen
    from paper_2403_09133_amd import Context

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    key, prec, desc = WORKLOADS[args.workload]
    if args.ops_profile:
        ops_profile(key, args.ops_profile)
        return
    t = time.time()
    p = sdpgen.config_instance(key)
    t_gen = time.time() - t
    r0 = initial_rank(p)
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    print(f"[bench] {args.workload}: n={p.n} m={p.m} r0={r0} (generated in {t_gen:.1f}s)", file=sys.stderr, flush=True)
    t = time.time()
    ctx = Context(p)
    torch.cuda.synchronize()
    t_setup = time.time() - t
    print(f"[bench] setup {t_setup:.2f}s {ctx.problem_info()}", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        res = ctx.admm_solve([U0], lib_options(p, r0, prec))[0]
        print(f"[bench] warmup {i}: {res['t_total']:.3f}s status {res['status']} kkt {res['kkt']:.2e}",
              file=sys.stderr, flush=True)

    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        # profile 2: the CG operator's launches carry their own HIP events; the
        # other launches run unrecorded (their classes are timed below)
        res = ctx.admm_solve([U0], lib_options(p, r0, prec, profile=2))[0]
        results.append(res)
        print(f"[bench] step {i}: {res['t_total']:.3f}s status {res['status']} kkt {res['kkt']:.2e} "
              f"obj {res['obj']:.10g} admm {res['admm_iters']} cg {res['cg_iters']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    op_bytes = sum(r["op_bytes"] for r in results)
    value = op_bytes / wall / 1e9

    # every kernel class timed on one more solve after the timed region; the
    # dominant class's figures come from the timed steps (live HIP-event
    # timings) when it is the one timed there
    names = list(KERNEL_CLASSES)
    K = len(names)
    full = ctx.admm_solve([U0], lib_options(p, r0, prec, profile=1))[0]
    ms = [full["prof_ms"][k] for k in range(K)]
    launches = [full["prof_launches"][k] for k in range(K)]
    kbytes = [full["prof_bytes"][k] for k in range(K)]
    dom = int(np.argmax(ms))
    kernels = {names[k]: dict(launches=int(launches[k]), total_ms=round(ms[k], 3),
                              mean_us=round(ms[k] * 1e3 / max(1, launches[k]), 2),
                              gbs=round(kbytes[k] / (ms[k] * 1e-3) / 1e9, 1) if ms[k] > 0 else None)
               for k in range(K)}
    timed_live = dom == 0
    if timed_live:
        ms = [sum(r["prof_ms"][k] for r in results) for k in range(K)]
        launches = [sum(r["prof_launches"][k] for r in results) for k in range(K)]
        kbytes = [sum(r["prof_bytes"][k] for r in results) for k in range(K)]
    else:
        print(f"[bench] dominant class {names[dom]} is not the one timed in the timed steps; "
              "its figures come from the extra profiled solve", file=sys.stderr, flush=True)
    achieved = kbytes[dom] / (ms[dom] * 1e-3) / 1e9 if ms[dom] > 0 else 0.0
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=recorded_traffic(KERNEL_CLASSES[names[dom]]),
                    kernel=names[dom], symbol=KERNEL_CLASSES[names[dom]], launches=int(launches[dom]),
                    mean_launch_us=round(ms[dom] * 1e3 / max(1, launches[dom]), 2),
                    bytes_per_launch=round(kbytes[dom] / max(1, launches[dom])),
                    timed_in="timed steps" if timed_live else "extra profiled solve")

    last = results[-1]
    extra = dict(
        time_to_kkt_s={"fp32_cg": round(wall / args.steps, 4)},
        solve=dict(status=last["status"], kkt=last["kkt"], obj=last["obj"], pinf=last["pinf"],
                   dinf=last["dinf"], gap=last["gap"], rank=last["rank"], admm_iters=last["admm_iters"],
                   cg_iters=last["cg_iters"], alm_outer=last["alm_outer"], alm_inner=last["alm_inner"],
                   t_phase1=round(last["t_phase1"], 4), t_phase2=round(last["t_phase2"], 4)),
        kernels=kernels, setup_s=round(t_setup, 3),
    )
    if p.kind == "mc":
        from paper_2403_09133_amd.report import (completion_recovery_error,
                                                 completion_recovery_error_sampled)
        U, V, lam = ctx.get_solution(0, last["rank"])
        Uh = 0.5 * (U + V)
        extra["mc_recovery_error"] = dict(
            gram_identity=completion_recovery_error(Uh, p.meta["L"], p.meta["R"]),
            sampled_1e6_cells=completion_recovery_error_sampled(Uh, p.meta["L"], p.meta["R"]),
            note="||U1 U2^T - M||_F / ||M||_F; the Gram identity resolves about 1e-8, the sample is exact per cell")
    if not args.no_fp64:
        t = time.perf_counter()
        r64 = ctx.admm_solve([U0], lib_options(p, r0, 0))[0]
        extra["time_to_kkt_s"]["fp64"] = round(time.perf_counter() - t, 4)
        extra["fp64_solve"] = dict(status=r64["status"], kkt=r64["kkt"], obj=r64["obj"],
                                   admm_iters=r64["admm_iters"], cg_iters=r64["cg_iters"])
        extra["fp32_vs_fp64_obj_rel"] = abs(last["obj"] - r64["obj"]) / max(1.0, abs(r64["obj"]))
    ctx.close()
    if args.copy_calibration:
        calibration_copy()

    line = {
        "metric": "A(UV^T)+A^*(y)V as HBM GB/s; time-to-1e-6 KKT residual, FP32/batched vs FP64",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "n_X": p.n, "m": p.m, "r0": r0,
                   "kkt_tol": 1e-6},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, r0)
    line.update(extra)
    if not args.no_learned:
        line["learned_warm_start"] = learned_leg()
        line["time_to_kkt_s"]["learned_fp64_mean"] = line["learned_warm_start"]["learned_mean_s"]
        line["time_to_kkt_s"]["cold_fp64_mean_same_instances"] = line["learned_warm_start"]["cold_mean_s"]
    if not args.no_batch:
        line["batched_maxcut"] = batch_leg()
        line["time_to_kkt_s"]["batched_512_fp64"] = line["batched_maxcut"]["fp64"]["s"]
        line["time_to_kkt_s"]["batched_512_fp32"] = line["batched_maxcut"]["fp32"]["s"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
