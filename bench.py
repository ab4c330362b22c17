#!/usr/bin/env python
"""Benchmark of the LoRADS hot path on one MI355X.

Headline workload: the planted rank-5 matrix-completion SDP with M of order
20000 x 20000 (X of order 40000), 15,683,710 observed entries drawn as the
paper's completion generator draws them (800 d uniform cells, duplicates
merged), C = I/2, solved by the two-phase method (Burer-Monteiro warm start,
then ADMM with CG subproblem solves) to KKT residual eq. (stop) <= 1e-6; the
initial rank round(ln m) = 17.  The timed form is the mixed one: CG iterations
and the two maps of Phase I's exact line search in FP32, the gradient, the
quartic's sums, right-hand sides, dual updates and residuals in FP64
(--precision selects another).  The FP32-CG form (line search in FP64) and the
plain FP64 form are solved from the same starts beside it.  A second entry
repeats the timed form on the completion instance of order 10000 (4,605,170
entries, rank 15).

One step = one full two-phase solve, the instance already resident in HBM
(setup is outside the timed region); timed step i starts from its own random
U0 (seed i + 1), so the mean time covers the spread of Phase-I trajectories.

value  = algorithmic bytes of every constraint-operator application of the
         solves (forward map, adjoint product, fused CG operator, the gradient
         form as a forward map plus an adjoint, the line-search pass as the two
         forward maps it computes; indices, coefficients, inputs and outputs
         counted once) / wall time of the timed steps, in GB/s.
roofline: the dominant kernel class of the timed steps (all classes carry HIP
         events on the solver's stream during the timed steps): algorithmic
         bytes per launch x launches / summed event time, against the 8 TB/s
         HBM peak; `traffic` is the measured HBM bytes per launch of that class
         on this workload (FETCH_SIZE + WRITE_SIZE, profiles/hbm_traffic.json)
         while the kernel sources are unchanged, else null.
roofline_fp64, roofline_fp32_cg: the same for the comparison solves.
ops_cold_warm: forward map and adjoint product alone at the solve's rank, FP32
         and FP64, warm (back to back) and cold (a 1 GiB buffer written before
         each call, flushing the 256 MB Infinity Cache and the L2s).
dense_cost: C V alone for a random dense symmetric C of order 8192 kept dense
         (the matrix-core product), FP64 and FP32, ranks 4, 16, 32, warm and
         cold, against the HBM and MFMA peaks.
cpu_baseline: the FP64 numpy oracle's forward map and adjoint product at the
         same size on the host, one thread, in the same unit; beside it
         per-operator medians on other configurations, the same loops with
         numpy's thread pools unrestricted, and the oracle's end-to-end time
         to eq. (stop) <= 1e-6 on the MaxCut instance of order 200.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
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
# solver forms (lorads_options.precision)
PREC_NAMES = {0: "fp64", 1: "fp32_cg", 2: "mixed"}

# kernel classes timed by the library (lorads_result.prof_*)
CLASSES = ["fused CG operator", "forward map A(UV^T)", "adjoint (C + A*(w))V", "line search A(UD^T+DU^T), A(DD^T)"]


def pow2_group(k: int) -> int:
    g = 1
    while g < k and g < 64:
        g <<= 1
    return g


def class_kernels(structure: str, r: int, cg_dtype: str, n=None, mixed=False) -> list:
    """The kernel each class runs for a structure and rank (the names rocprofv3
    reports), so that a line names what was timed; mixed: the line search's
    maps on FP32 copies."""
    G = pow2_group(r)
    if structure == "pair":
        # the CG layout pads rows to 64 bytes; the vector form needs its lane
        # group's columns inside the row
        esz = 4 if cg_dtype == "float" else 8
        vw = 16 // esz
        ld = (r + 64 // esz - 1) // (64 // esz) * (64 // esz)
        # FP64 at ranks 17..24: 8 lanes with an extra 8-byte vector each
        x3 = 1 if esz == 8 and 16 < r <= 24 and ld >= 24 else 0
        gv = 16 // vw if x3 else pow2_group((r + vw - 1) // vw)
        if x3 or (gv * vw <= ld and gv <= 16):
            # rows of [W | P] above one XCD's 4 MiB L2: split by partner block
            if n is not None and n * 2 * ld * esz > (4 << 20):
                cg = f"kpair_cg_xvec<{cg_dtype}, {gv}, {x3}> + xcg_combine<{cg_dtype}>"
            else:
                cg = f"kpair_cg_vec<{cg_dtype}, {gv}, {x3}>"
        else:
            cg = f"kpair_rows<{cg_dtype}, {G}, 1>"
        # FP64 maps: G / 2 lanes of two columns; 8 lanes of three for r = 17..24
        X3 = 1 if 16 < r <= 24 else 0
        GV = 8 if X3 else max(1, G // 2)
        ls = f"k1_pair_ls<{GV}, {X3}>"
        if mixed and r >= 9:
            ls = f"k1_pair_ls_f32<{max(4, pow2_group((r + 3) // 4))}>"
        return [cg, f"k1_pair_v2<{GV}, 0, {X3}>", f"kpair_grad_v2<{GV}, {X3}>", ls]
    if structure == "diag":
        # the line search's two maps run as forward maps (counted in that class)
        return [f"k3_diag<{cg_dtype}, {G}>", f"k1_diag<double, {G}, 0|1>", f"k2_diag<double, {G}, 0>",
                "(none: two forward maps)"]
    return [f"k1_generic<{cg_dtype}, {G}, 2> + k2_generic<{cg_dtype}, {G}, 1>", f"k1_generic<double, {G}, 1>",
            f"k2_generic<double, {G}, 0>", f"k1_generic<double, {G}, 0>"]


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload: str, precision: str, klass: str):
    """HBM bytes per launch of a kernel class on a workload, from the recorded
    FETCH_SIZE / WRITE_SIZE passes (already scaled by the copy-kernel
    calibration), or None when no record exists for that workload, precision
    and class, or the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    if rec.get("sources_sha256") != kernel_sources_hash():
        return None
    ent = rec.get("workloads", {}).get(workload, {}).get(precision, {}).get(klass)
    return None if ent is None else int(round(ent["hbm_bytes_per_launch"]))


WORKLOADS = {
    # name -> description
    "mc_20000": "matrix completion 20000x20000, rank 5, 800*d draws deduplicated, X of order 40000",
    "mc_10000": "matrix completion 10000x10000, rank 5, |Omega|=4605170, X of order 20000",
    "maxcut_torus100": "MaxCut 100x100 torus, +-1 weights, n=m=10000",
    "maxcut_gnm20000": "MaxCut G(20000, M=60000), unit weights",
}


def initial_rank(p) -> int:
    from paper_2403_09133_amd.params import initial_rank as rule
    return rule(p.kind, p.n, p.m)


def lib_options(p, r0, precision, **kw):
    from paper_2403_09133_amd.params import solver_options
    return solver_options(p.kind, p.n, r0, precision, **kw)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu() -> dict:
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(model=model, nproc=os.cpu_count())


def per_operator(q, rq: int, reps: int, rng):
    """Median time of the oracle's forward map and adjoint product on one
    instance at rank rq (random factors and multipliers)."""
    import oracle
    Uq = rng.standard_normal((q.n, rq))
    Vq = rng.standard_normal((q.n, rq))
    wq = rng.standard_normal(q.m)
    tf, ta = [], []
    for _ in range(reps):
        t1 = time.perf_counter()
        oracle.operators.forward(q, Uq, Vq)
        t2 = time.perf_counter()
        oracle.operators.adjoint(q, wq, 1.0, Vq)
        t3 = time.perf_counter()
        tf.append(t2 - t1)
        ta.append(t3 - t2)
    return dict(rank=rq, reps=reps, forward_s=round(float(np.median(tf)), 5),
                adjoint_s=round(float(np.median(ta)), 5))


def cpu_baseline(p, r: int, budget_s: float = 20.0, e2e=("maxcut_er200",), workload: str = "mc_20000",
                 per_op=(("maxcut_torus100", 5), ("mc_10000", 5)), per_op_all=(("mc_10000", 5),)):
    """The oracle's forward map and adjoint product (FP64, numpy) on the host,
    one thread, for a bounded number of applications; per-operator medians on
    other configurations, one thread and with numpy's thread pools
    unrestricted (per_op, per_op_all: configuration names and repetitions;
    workload: the timed workload's name); plus the oracle's end-to-end
    solves to eq. (stop) of the named instances (by default the MaxCut
    instance of order 200), one thread, from the library's initial rank."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    import oracle
    import sdpgen
    from oracle.options import Options, paper_defaults
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
        # per-operator medians at full size on the other configurations
        per_op_1 = {}
        for name, reps_ in per_op:
            q = sdpgen.config_instance(name)
            per_op_1[name] = per_operator(q, initial_rank(q), reps_, rng)
        solves = []
        for name in e2e:
            q = sdpgen.config_instance(name)
            r0 = initial_rank(q)
            U0 = sdpgen.random_init_U(q.n, r0, 3)
            log(f"oracle end-to-end solve of {name} (n = {q.n}, m = {q.m}, r0 = {r0})")
            t1 = time.perf_counter()
            out = oracle.lorads.lorads(q, U0, Options(**paper_defaults(q.kind, q.n)), with_metrics=False,
                                       progress=lambda msg, nm=name: log(f"oracle {nm}: {msg}"))
            t_e2e = time.perf_counter() - t1
            log(f"oracle {name}: {t_e2e:.1f} s")
            solves.append(dict(workload=f"{name} (n = {q.n}, m = {q.m}, r0 = {r0}), FP64 numpy, 1 thread",
                               s=round(t_e2e, 3), admm_iters=int(out["phase2"]["iters"]),
                               converged=bool(out["phase2"]["converged"])))
    finally:
        if ctx is not None and hasattr(ctx, "unregister"):
            ctx.unregister()
    # the same per-operator loops with numpy's thread pools unrestricted
    all_threads = dict(threads=os.cpu_count())
    if threadpool_limits is not None:
        from threadpoolctl import threadpool_info
        all_threads["threads"] = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    for name, reps_ in per_op_all:
        q = sdpgen.config_instance(name)
        all_threads[name] = per_operator(q, initial_rank(q), reps_, rng)
    all_threads[workload] = per_operator(p, r, 3, rng)
    bytes_pair = 2 * (8.0 * p.m + 8.0 * p.m + 2.0 * p.n * r * 8)
    return dict(value=round(reps * bytes_pair / t / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                sample=f"{reps} x (A(UV^T) + (C + A*(y))V) at full size, r={r}, FP64 numpy, "
                       f"{t:.1f} s on the host",
                host=host_cpu(),
                per_operator_median=per_op_1,
                per_operator_median_all_threads=all_threads,
                oracle_time_to_kkt_s=solves)


def starts(p, r0, steps, warmup):
    """Random starts U0 ~ N(0, 1/r0): warm-up starts from seeds 1000.., timed
    step i from seed i + 1 (the time to eq. (stop) depends on the start through
    the Phase-I trajectory, so the timed steps average over K starts)."""
    import sdpgen
    return ([sdpgen.random_init_U(p.n, r0, 1000 + i) for i in range(warmup)],
            [sdpgen.random_init_U(p.n, r0, 1 + i) for i in range(steps)])


def timed_solves(ctx, p, r0, prec, warm_starts, timed_starts):
    """Untimed solves from `warm_starts`, then one timed solve from each of
    `timed_starts` with every kernel class carrying HIP events (profile
    level 1)."""
    import torch
    for i, U0 in enumerate(warm_starts):
        res = ctx.admm_solve([U0], lib_options(p, r0, prec))[0]
        log(f"warmup {i}: {res['t_total']:.3f}s status {res['status']} kkt {res['kkt']:.2e}")
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, U0 in enumerate(timed_starts):
        res = ctx.admm_solve([U0], lib_options(p, r0, prec, profile=1))[0]
        results.append(res)
        log(f"step {i}: {res['t_total']:.3f}s status {res['status']} kkt {res['kkt']:.2e} "
            f"obj {res['obj']:.10g} admm {res['admm_iters']} cg {res['cg_iters']} "
            f"(phase I {res['t_phase1']:.3f}s, II {res['t_phase2']:.3f}s)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return results, wall


def roofline_of(results, workload, structure, prec, n):
    """Dominant class over the timed solves and its figures."""
    K = len(CLASSES)
    ms = [sum(r["prof_ms"][k] for r in results) for k in range(K)]
    launches = [sum(r["prof_launches"][k] for r in results) for k in range(K)]
    kbytes = [sum(r["prof_bytes"][k] for r in results) for k in range(K)]
    rank = results[-1]["rank"]
    names = class_kernels(structure, rank, "float" if prec != 0 else "double", n, mixed=prec == 2)
    kernels = {CLASSES[k]: dict(kernel=names[k], launches=int(launches[k]), total_ms=round(ms[k], 3),
                                mean_us=round(ms[k] * 1e3 / max(1, launches[k]), 2),
                                gbs=round(kbytes[k] / (ms[k] * 1e-3) / 1e9, 1) if ms[k] > 0 else None)
               for k in range(K)}
    dom = int(np.argmax(ms))
    achieved = kbytes[dom] / (ms[dom] * 1e-3) / 1e9 if ms[dom] > 0 else 0.0
    pname = PREC_NAMES[prec]
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4),
                traffic=recorded_traffic(workload, pname, CLASSES[dom]),
                kernel=CLASSES[dom], symbol=names[dom], launches=int(launches[dom]),
                mean_launch_us=round(ms[dom] * 1e3 / max(1, launches[dom]), 2),
                bytes_per_launch=round(kbytes[dom] / max(1, launches[dom])),
                timed_in="timed steps (HIP events on the solver's stream)")
    return roof, kernels


def padded_ld(r: int, elem: int) -> int:
    """The library's fast factor layout for the completion kernels: rows of
    whole 64-byte sectors and at least the lane group (the power of two >= r)."""
    g = 1
    while g < r:
        g *= 2
    per = 64 // elem
    return max(g, -(-r // per) * per)


def ops_cold_warm(ctx, p, r: int, reps: int = 10, flush_bytes: int = 1 << 30):
    """Forward map and adjoint product alone, FP32 and FP64, warm (back to
    back) and cold (a 1 GiB write before each call).  Median of `reps`.  The
    factors are n x r (ld = r) and, for the completion kernels, also in the
    padded layout (ld = padded_ld; the two-column FP64 forward map needs it);
    the algorithmic bytes count r columns either way."""
    import torch
    from paper_2403_09133_amd.lorads import F32
    dev = torch.device("cuda")
    flush = torch.empty(flush_bytes // 4, dtype=torch.float32, device=dev)
    out = {}
    g = torch.Generator().manual_seed(11)
    layouts = [(dt, pad) for dt in (torch.float32, torch.float64)
               for pad in ((False, True) if p.kind == "mc" else (False,))]
    for dt, pad in layouts:
        s = 4 if dt == torch.float32 else 8
        ld = padded_ld(r, s) if pad else r
        U = torch.zeros(p.n, ld, dtype=dt, device=dev)[:, :r]
        V = torch.zeros(p.n, ld, dtype=dt, device=dev)[:, :r]
        U.copy_(torch.randn(p.n, r, generator=g, dtype=torch.float64).to(dev, dt))
        V.copy_(torch.randn(p.n, r, generator=g, dtype=torch.float64).to(dev, dt))
        w = torch.randn(p.m, generator=g, dtype=torch.float64).to(dev, dt)
        z = torch.empty(p.m, dtype=dt, device=dev)
        o = torch.zeros(p.n, ld, dtype=dt, device=dev)[:, :r]
        if p.kind == "mc":
            fwd_b = 8.0 * p.m + p.m * s + 2.0 * p.n * r * s
            adj_b = 8.0 * p.m + p.m * s + 2.0 * p.n * r * s + p.n * (4 + s) + (p.n + 1) * 4
        else:
            fwd_b = p.m * (4 + s) + 2.0 * p.n * r * s + p.m * s
            adj_b = p.m * (4 + 2 * s) + 2.0 * p.n * r * s + p.c_val.size * 2 * (4 + s) + (p.n + 1) * 4
        ops = {"K1 forward A(UV^T)": (lambda: ctx.apply_A(U, V, z), fwd_b),
               "K2 adjoint (C + A*(w))V": (lambda: ctx.apply_AT_V(w, V, o), adj_b)}
        for name, (fn, nbytes) in ops.items():
            fn()
            torch.cuda.synchronize()
            res = {}
            for mode in ("warm", "cold"):
                ts = []
                for _ in range(reps):
                    if mode == "cold":
                        flush.fill_(1.0)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    fn()
                    e1.record()
                    e1.synchronize()
                    ts.append(e0.elapsed_time(e1) * 1e3)
                us = float(np.median(ts))
                res[mode] = dict(us=round(us, 2), gbs=round(nbytes / (us * 1e-6) / 1e9, 1),
                                 frac=round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))
            key = f"{name} {'fp32' if s == 4 else 'fp64'}" + (f" ld={ld}" if pad else "")
            out[key] = dict(bytes=int(nbytes), ld=ld, **res)
        del U, V, w, z, o
    del flush
    torch.cuda.empty_cache()
    return dict(rank=r, reps=reps, flush="1 GiB fill before each cold call", **out)


def theta_leg():
    """The Lovasz theta SDP of G(260, 0.05) (seed 8): C = -J kept dense (the
    matrix-core products), the family's gamma = 1 + ||C||_2, initial rank 30,
    FP64 and FP32-CG; time to eq. (stop) <= 1e-6 and the Appendix-B measures."""
    import sdpgen
    from paper_2403_09133_amd import Context
    from paper_2403_09133_amd.params import solver_options
    ei, ej = sdpgen.er_gnp_edges(260, 0.05, np.random.default_rng(8))
    p = sdpgen.lovasz_theta(260, list(zip(ei.tolist(), ej.tolist())))
    r0 = 30
    U0 = sdpgen.random_init_U(p.n, r0, 3)
    out = dict(workload="Lovasz theta of G(260, 0.05), seed 8: n = 260, m = %d, dense C, r0 = 30" % p.m)
    with Context(p) as ctx:
        out["c_dense"] = bool(ctx.problem_info()["c_dense"])
        for name, prec in (("fp64", 0), ("fp32_cg", 1)):
            res = ctx.admm_solve([U0], solver_options(p.kind, p.n, r0, prec))[0]
            out[name] = dict(s=round(res["t_total"], 3), status=res["status"], kkt=res["kkt"],
                             admm_iters=res["admm_iters"], obj=res["obj"], pinf=res["pinf"],
                             dinf=res["dinf"], gap=res["gap"], gamma=res["gamma"])
            log(f"theta G(260, 0.05) {name}: {res['t_total']:.2f}s status {res['status']} obj {res['obj']:.9f}")
    return out


def dense_cost_leg(n: int = 8192, ranks=(4, 16, 32), reps: int = 10, flush_bytes: int = 1 << 30):
    """C V alone (lorads_apply_AT_V with a zero multiplier) for a random dense
    symmetric C of order n, kept dense by the library (the matrix-core
    product), FP64 and FP32, warm and cold (a 1 GiB write before each call),
    median of `reps`.  The constraint is tr X = 1.  Algorithmic bytes:
    C once (n^2 s), V in and C V out (2 n r s); flops 2 n^2 r."""
    import torch
    import sdpgen
    from paper_2403_09133_amd import Context
    rng = np.random.default_rng(21)
    G = rng.standard_normal((n, n)) / math.sqrt(n)
    ir, ic = np.triu_indices(n)
    cv = 0.5 * (G[ir, ic] + G[ic, ir])
    del G
    ar = np.arange(n)
    p = sdpgen.Problem(n=n, m=1, c_row=ir, c_col=ic, c_val=cv, a_con=np.zeros(n), a_row=ar,
                       a_col=ar, a_val=np.ones(n), b=np.ones(1), kind="generic")
    del ir, ic, cv
    dev = torch.device("cuda")
    g = torch.Generator().manual_seed(12)
    out = dict(workload=f"random dense symmetric C of order {n} (seed 21), tr X = 1", n=n, reps=reps,
               flush="1 GiB fill before each cold call")
    with Context(p) as ctx:
        out["c_dense"] = bool(ctx.problem_info()["c_dense"])
        flush = torch.empty(flush_bytes // 4, dtype=torch.float32, device=dev)
        for dt, tag, peak_tf in ((torch.float64, "fp64", 78.6), (torch.float32, "fp32", 157.3)):
            sz = 8 if dt == torch.float64 else 4
            for r in ranks:
                V = torch.randn(n, r, generator=g, dtype=torch.float64).to(dev, dt)
                w = torch.zeros(1, dtype=dt, device=dev)
                o = torch.zeros(n, r, dtype=dt, device=dev)
                ctx.apply_AT_V(w, V, o)
                torch.cuda.synchronize()
                nbytes = float(n) * n * sz + 2.0 * n * r * sz
                flops = 2.0 * n * n * r
                res = {}
                for mode in ("warm", "cold"):
                    ts = []
                    for _ in range(reps):
                        if mode == "cold":
                            flush.fill_(1.0)
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record()
                        ctx.apply_AT_V(w, V, o)
                        e1.record()
                        e1.synchronize()
                        ts.append(e0.elapsed_time(e1) * 1e3)
                    us = float(np.median(ts))
                    res[mode] = dict(us=round(us, 2), gbs=round(nbytes / (us * 1e-6) / 1e9, 1),
                                     frac=round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                                     tflops=round(flops / (us * 1e-6) / 1e12, 2),
                                     mfma_frac=round(flops / (us * 1e-6) / 1e12 / peak_tf, 4))
                out[f"CV {tag} r={r}"] = dict(bytes=int(nbytes), flops=int(flops), **res)
                log(f"dense C V n={n} {tag} r={r}: cold {res['cold']['us']:.1f} us "
                    f"({res['cold']['gbs']:.0f} GB/s), warm {res['warm']['us']:.1f} us")
                del V, w, o
        del flush
    torch.cuda.empty_cache()
    return out


def batch_leg(count: int = 512, sequential: bool = True):
    """Batched form: `count` MaxCut SDPs, n ~ U{50..2000}, average degree ~ U[3, 20],
    +-1 weights, rank ceil(log2 n) each, in one persistent launch (workgroup size
    autotuned on short runs), FP64 and FP32 CG; against the same instances solved
    one after the other by the single-instance path (measured, FP64)."""
    import sdpgen
    from paper_2403_09133_amd import Context, default_options
    from paper_2403_09133_amd.params import family_params
    t = time.time()
    probs = sdpgen.batch_maxcut(count, 2000, 50, 2000, 3.0, 20.0, "pm1")
    U0 = [sdpgen.random_init_U(p.n, int(math.ceil(math.log2(p.n))), 2000 + i) for i, p in enumerate(probs)]
    t_gen = time.time() - t
    pd = family_params("maxcut", 1000)

    def opts(**kw):
        return default_options(r0=1, **{**pd, **kw})

    out = dict(instances=count, sum_n=int(sum(p.n for p in probs)),
               sum_edges=int(sum(len(p.meta["edges"][0]) for p in probs)), gen_s=round(t_gen, 2))
    t = time.time()
    ctx = Context(probs)
    out["setup_s"] = round(time.time() - t, 2)
    t = time.perf_counter()
    best, times = ctx.batch_autotune(U0, opts(max_admm_iter=10, alm_outer_max=2), (64, 128, 256))
    out["autotune"] = {"block": best, "s": round(time.perf_counter() - t, 2),
                       "ms_short_run": {k: round(v, 2) for k, v in times.items()},
                       "short_run": "2 ALM outer and 10 ADMM iterations per instance"}
    for name, prec in (("fp64", 0), ("fp32", 1)):
        t = time.perf_counter()
        res = ctx.admm_solve(U0, opts(precision=prec, batch_mode=1))
        dt = time.perf_counter() - t
        out[name] = dict(s=round(dt, 4), converged=int(sum(r["status"] == 0 for r in res)),
                         max_admm_iters=int(max(r["admm_iters"] for r in res)),
                         median_admm_iters=float(np.median([r["admm_iters"] for r in res])),
                         max_kkt=float(max(r["kkt"] for r in res)), max_rank=int(max(r["rank"] for r in res)))
        log(f"batch {name}: {dt:.3f}s, {out[name]['converged']}/{count} converged")
    ctx.close()
    if sequential:
        t = time.perf_counter()
        conv = 0
        for i, p in enumerate(probs):
            with Context(p) as one:
                r = one.admm_solve([U0[i]], opts(batch_mode=2))[0]
            conv += r["status"] == 0
            if i % 64 == 63:
                log(f"sequential {i + 1}/{count}: {time.perf_counter() - t:.1f}s")
        dt = time.perf_counter() - t
        out["sequential_fp64"] = dict(s=round(dt, 3), converged=int(conv),
                                      note="every instance solved one after the other by the single-instance "
                                           "path (context setup per instance included)")
        out["speedup_vs_sequential_fp64"] = round(dt / out["fp64"]["s"], 1)
    return out


def learned_leg(count: int = 6):
    """Learned warm start (the shipped MaxCut network) against the cold start on
    `count` held-out graphs shaped like its training set (n ~ U{2000..5000},
    average degree ~ U[4, 16], +-1 weights), FP64 solves to eq. (stop) <= 1e-6
    from the same random U0: time-to-KKT, ADMM iterations and the App. B gap."""
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
        log(f"learned leg n={p.n}: cold {cold['t_total']:.2f}s {cold['admm_iters']} it, "
            f"learned {warm['t_total']:.2f}s {warm['admm_iters']} it")
    col = lambda k, i: [r[i][k] for r in rows]
    med = lambda k, i: float(np.median(col(k, i)))
    return dict(instances=count, predict_s=round(t_pred, 3),
                cold_s=[round(v, 3) for v in col("t_total", 0)], learned_s=[round(v, 3) for v in col("t_total", 1)],
                cold_admm=col("admm_iters", 0), learned_admm=col("admm_iters", 1),
                cold_gap=[float(f"{g:.2e}") for g in col("gap", 0)],
                learned_gap=[float(f"{g:.2e}") for g in col("gap", 1)],
                cold_median_s=round(med("t_total", 0), 3), learned_median_s=round(med("t_total", 1), 3),
                cold_converged=int(sum(r[0]["status"] == 0 for r in rows)),
                learned_converged=int(sum(r[1]["status"] == 0 for r in rows)),
                gaps_above_1e_6=int(sum(abs(r[i]["gap"]) > 1e-6 for r in rows for i in (0, 1))),
                note="medians with every solve's App. B gap; held-out evaluation: "
                     "profiles/warmstart_maxcut_c5a_eval.md")


def ops_profile(key: str, reps: int):
    """Operator calls only: REPS x (forward map, adjoint product, 20-iteration CG
    solve) in FP32 at the initial rank, then one 256 MiB device-to-device copy
    whose known size calibrates the HBM byte counters."""
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
        log(f"ops rep {i} done")
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
    log(f"copy of {a.numel() * 4} bytes done")


def workload_leg(key, steps, warmup, prec, compare=(0,), with_ops=True):
    """Timed solves of one workload: the given form with its roofline, each
    form in `compare` from the same starts with its roofline, and the
    operators alone."""
    import torch
    import sdpgen
    from paper_2403_09133_amd import Context
    t = time.time()
    p = sdpgen.config_instance(key)
    t_gen = time.time() - t
    r0 = initial_rank(p)
    warm_starts, timed_starts = starts(p, r0, steps, warmup)
    log(f"{key}: n={p.n} m={p.m} r0={r0} (generated in {t_gen:.1f}s)")
    t = time.time()
    ctx = Context(p)
    torch.cuda.synchronize()
    t_setup = time.time() - t
    info = ctx.problem_info()
    log(f"setup {t_setup:.2f}s {info}")
    results, wall = timed_solves(ctx, p, r0, prec, warm_starts, timed_starts)
    op_bytes = sum(r["op_bytes"] for r in results)
    roof, kernels = roofline_of(results, key, info["structure"], prec, p.n)
    last = results[-1]
    leg = dict(p=p, r0=r0, wall=wall, value=op_bytes / wall / 1e9, roofline=roof, kernels=kernels,
               setup_s=round(t_setup, 3), structure=info["structure"],
               steps=dict(s=[round(r["t_total"], 4) for r in results], status=[r["status"] for r in results],
                          admm_iters=[r["admm_iters"] for r in results],
                          alm_inner=[r["alm_inner"] for r in results],
                          starts="U0 ~ N(0, 1/r0), seeds 1..K (one per timed step)"),
               solve=dict(status=last["status"], kkt=last["kkt"], obj=last["obj"], pinf=last["pinf"],
                          dinf=last["dinf"], gap=last["gap"], rank=last["rank"],
                          admm_iters=last["admm_iters"], cg_iters=last["cg_iters"],
                          alm_outer=last["alm_outer"], alm_inner=last["alm_inner"],
                          rank_growths=last["rank_growths"], t_phase1=round(last["t_phase1"], 4),
                          t_phase2=round(last["t_phase2"], 4)))
    if p.kind == "mc":
        from paper_2403_09133_amd.report import completion_recovery_error_sampled
        U, V, lam = ctx.get_solution(0, last["rank"])
        leg["mc_recovery_error"] = dict(
            sampled_1e6_cells=completion_recovery_error_sampled(0.5 * (U + V), p.meta["L"], p.meta["R"]),
            note="||U1 U2^T - M||_F / ||M||_F on 10^6 uniformly drawn cells")
    for cp in compare:
        if cp == prec:
            continue
        # the same solves in another form, from the same starts
        rcs, wallc = timed_solves(ctx, p, r0, cp, [], timed_starts)
        rc = rcs[-1]
        roofc, kernc = roofline_of(rcs, key, info["structure"], cp, p.n)
        leg.setdefault("compare", {})[PREC_NAMES[cp]] = dict(
            s=round(wallc / len(rcs), 4), status=[r["status"] for r in rcs], kkt=max(r["kkt"] for r in rcs),
            obj=rc["obj"], admm_iters=[r["admm_iters"] for r in rcs], cg_iters=[r["cg_iters"] for r in rcs],
            alm_inner=[r["alm_inner"] for r in rcs], steps_s=[round(r["t_total"], 4) for r in rcs],
            roofline=roofc, kernels=kernc)
        if cp == 0:
            leg["obj_rel_diff_vs_fp64"] = max(abs(a["obj"] - b["obj"]) / max(1.0, abs(b["obj"]))
                                              for a, b in zip(results, rcs))
    if with_ops:
        leg["ops_cold_warm"] = ops_cold_warm(ctx, p, last["rank"])
    ctx.close()
    return leg


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mc_20000", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-e2e", default="maxcut_er200", metavar="NAMES",
                    help="comma-separated instances the oracle solves end to end in the CPU baseline "
                         "(maxcut_er200, maxcut_torus100, maxcut_gnm20000; the larger ones take minutes)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the second completion workload and the theta leg")
    ap.add_argument("--no-ops", action="store_true", help="skip the cold / warm operator timings")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the one-at-a-time solve of the 512 batched instances")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-warm-start leg")
    ap.add_argument("--fp64-only", action="store_true", help="time the plain FP64 form in the timed steps")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp32_cg", "fp64"],
                    help="form of the timed steps (mixed: FP32 CG and FP32 line-search maps)")
    ap.add_argument("--no-fp32-cg", action="store_true", help="skip the FP32-CG comparison solve")
    ap.add_argument("--ops-profile", type=int, default=0, metavar="REPS",
                    help="only run REPS applications of each operator at the workload's size (FP32, "
                         "initial rank) and a 256 MiB device copy, for hardware-counter runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with a 256 MiB device copy (byte-counter calibration in counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the single-instance and batched paths are measured "
              "on one GPU and there is no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.ops_profile:
        ops_profile(args.workload, args.ops_profile)
        return
    prec = 0 if args.fp64_only else {"mixed": 2, "fp32_cg": 1, "fp64": 0}[args.precision]
    compare = [c for c, off in ((0, args.no_fp64), (1, args.no_fp32_cg)) if not off and c != prec]
    leg = workload_leg(args.workload, args.steps, args.warmup, prec, compare=compare,
                       with_ops=not args.no_ops)
    p = leg["p"]
    tkey = PREC_NAMES[prec]
    cmp_ = leg.get("compare", {})
    line = {
        "metric": "A(UV^T)+A^*(y)V as HBM GB/s; time-to-1e-6 KKT residual, FP32/batched vs FP64",
        "value": round(leg["value"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(leg["wall"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec != 0 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "n_X": p.n, "m": p.m,
                   "r0": leg["r0"], "kkt_tol": 1e-6},
        "roofline": leg["roofline"],
    }
    for name, c in cmp_.items():
        line[f"roofline_{name}"] = c["roofline"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p, leg["r0"], e2e=[x for x in args.oracle_e2e.split(",") if x],
                                             workload=args.workload)
    line["time_to_kkt_s"] = {tkey: round(leg["wall"] / args.steps, 4)}
    for name, c in cmp_.items():
        line["time_to_kkt_s"][name] = c["s"]
    if "obj_rel_diff_vs_fp64" in leg:
        line["obj_rel_diff_vs_fp64"] = leg["obj_rel_diff_vs_fp64"]
    line["steps_detail"] = leg["steps"]
    line["solve"] = leg["solve"]
    line["kernels"] = leg["kernels"]
    for name, c in cmp_.items():
        line[f"{name}_solve"] = {k: v for k, v in c.items() if k != "roofline"}
    line["setup_s"] = leg["setup_s"]
    if "mc_recovery_error" in leg:
        line["mc_recovery_error"] = leg["mc_recovery_error"]
    if "ops_cold_warm" in leg:
        line["ops_cold_warm"] = {args.workload: leg["ops_cold_warm"]}
    if not args.no_secondary and args.workload != "mc_10000":
        sec = workload_leg("mc_10000", 5, 1, prec, compare=(), with_ops=not args.no_ops)
        line["secondary"] = {"mc_10000": dict(ms_per_step=round(sec["wall"] / 5 * 1e3, 3), steps=sec["steps"],
                                              value=round(sec["value"], 2), roofline=sec["roofline"],
                                              solve=sec["solve"], kernels=sec["kernels"])}
        if "ops_cold_warm" in sec:
            line.setdefault("ops_cold_warm", {})["mc_10000"] = sec["ops_cold_warm"]
    if not args.no_secondary:
        line["theta_dense"] = theta_leg()
        line["time_to_kkt_s"]["theta_g260_fp64"] = line["theta_dense"]["fp64"]["s"]
        line["dense_cost"] = dense_cost_leg()
    if not args.no_learned:
        line["learned_warm_start"] = learned_leg()
        line["time_to_kkt_s"]["learned_fp64_median"] = line["learned_warm_start"]["learned_median_s"]
        line["time_to_kkt_s"]["cold_fp64_median_same_instances"] = line["learned_warm_start"]["cold_median_s"]
    if not args.no_batch:
        line["batched_maxcut"] = batch_leg(sequential=not args.no_sequential)
        line["time_to_kkt_s"]["batched_512_fp64"] = line["batched_maxcut"]["fp64"]["s"]
        line["time_to_kkt_s"]["batched_512_fp32"] = line["batched_maxcut"]["fp32"]["s"]
        if "sequential_fp64" in line["batched_maxcut"]:
            line["time_to_kkt_s"]["sequential_512_fp64"] = line["batched_maxcut"]["sequential_fp64"]["s"]
    if args.copy_calibration:
        calibration_copy()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
