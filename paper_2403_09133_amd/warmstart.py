"""Learned Phase-I warm start for MaxCut SDPs (driver around the lorads_gnn_* calls).

The paper names better warm starts as future work (Section 6).  Here a
message-passing network reads the MaxCut graph and predicts the optimal dual
multiplier of every diag(X) = 1 constraint and a rank factor; the solve then
starts Phase I (Section 4.1, the Burer-Monteiro ALM) from lambda0 = -yhat
instead of lambda = 0.

Stages, all on the device through the library:
  labels    cold FP64 solves to eq. (stop) <= 1e-6 in the batched launch;
            y* = -lambda* per node, r* = numerical rank of X_hat (eigenvalues
            of U_hat^T U_hat above 1e-6 of the largest)
  train     Adam on the resident graph set, minibatches of consecutive graphs
            in a shuffled order
  predict   lambda0 = -y_scale * yhat; cold start (no lambda0) when the graph is
            outside the training range of n or an output is not finite; the
            solver adds the third rule (options.warm_check): back to the cold
            start if the first Phase-I outer iteration does not lower the
            infeasibility
  evaluate  cold vs learned on held-out instances, one solve at a time, with
            per-instance time, ADMM and CG iterations, KKT residual and a
            paired sign test

Graph of a problem: the off-diagonal entries of C, with w_jk = 4 C_jk (MaxCut
C = -L/4, so the entries of C off the diagonal are w/4).

Usage: python -m paper_2403_09133_amd.warmstart all --out DIR [--train N ...]
       python -m paper_2403_09133_amd.warmstart eval --out DIR [--eval N]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import pathlib
import sys
import time
from typing import List, Optional, Sequence

import numpy as np

MODEL_PATH = pathlib.Path(__file__).resolve().parent / "data" / "gnn_maxcut.npz"
N_RANGE = (2000, 5000)
DEG_RANGE = (4.0, 16.0)
TRAIN_SEED0 = 100_000
HELDOUT_SEED0 = 900_000
R_SCALE = 10.0
LAYERS = 3


def log(msg: str):
    print(f"[warmstart] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# graphs
# ---------------------------------------------------------------------------
def problem_graph(p):
    """Undirected weighted edges (i < j) of a MaxCut problem's C."""
    off = p.c_row != p.c_col
    return p.c_row[off].astype(np.int64), p.c_col[off].astype(np.int64), 4.0 * p.c_val[off]


def graph_set(problems):
    """Symmetric COO over global node ids plus node offsets."""
    node_off = [0]
    rows, cols, ws = [], [], []
    for p in problems:
        i, j, w = problem_graph(p)
        o = node_off[-1]
        rows += [i + o, j + o]
        cols += [j + o, i + o]
        ws += [w, w]
        node_off.append(o + p.n)
    return (np.asarray(node_off, dtype=np.int64), np.concatenate(rows).astype(np.int32),
            np.concatenate(cols).astype(np.int32), np.concatenate(ws).astype(np.float32))


def rule_rank(n: int) -> int:
    from .params import initial_rank
    return initial_rank("maxcut", n, n)


def instances(count: int, seed0: int):
    import sdpgen
    return sdpgen.batch_maxcut(count, seed0, N_RANGE[0], N_RANGE[1], DEG_RANGE[0], DEG_RANGE[1], "pm1")


def random_start(p, r: int):
    import sdpgen
    return sdpgen.random_init_U(p.n, r, int(p.meta.get("seed", 0)))


def node_of_constraint(p):
    """Node (diagonal index) of every constraint of a diag(X) = 1 problem."""
    out = np.empty(p.m, dtype=np.int64)
    out[p.a_con] = p.a_row
    return out


# ---------------------------------------------------------------------------
# labels
# ---------------------------------------------------------------------------
def numerical_rank(U: np.ndarray, rel: float = 1e-6) -> int:
    ev = np.linalg.eigvalsh(U.T @ U)
    return int(np.sum(ev > rel * ev.max()))


def make_labels(problems, chunk: int = 512, eps: float = 1e-6):
    """Cold FP64 solves in the batched launch; returns per-problem dicts."""
    from .lorads import Context
    from .params import solver_options
    out = []
    for c0 in range(0, len(problems), chunk):
        sub = problems[c0:c0 + chunk]
        t = time.perf_counter()
        ctx = Context(sub)
        U0 = [random_start(p, rule_rank(p.n)) for p in sub]
        opts = solver_options("maxcut", 1000, 1, eps=eps, batch_mode=1 if len(sub) > 1 else 2)
        res = ctx.admm_solve(U0, opts)
        for i, (p, r) in enumerate(zip(sub, res)):
            U, V, lam = ctx.get_solution(i, r["rank"])
            y = np.empty(p.n)
            y[node_of_constraint(p)] = -lam
            out.append(dict(y=y, r=numerical_rank(0.5 * (U + V)), status=r["status"],
                            kkt=r["kkt"], admm_iters=r["admm_iters"], rank=r["rank"]))
        ctx.close()
        log(f"labels {c0 + len(sub)}/{len(problems)}: {time.perf_counter() - t:.1f}s, "
            f"converged {sum(r['status'] == 0 for r in res)}/{len(sub)}")
    return out


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def init_params(layers: int, seed: int) -> np.ndarray:
    """He-scaled normal weights, zero biases, in the library's flat layout."""
    from .lorads import load
    rng = np.random.default_rng(seed)
    H, F = 64, 5
    parts = [rng.standard_normal(H * F) * math.sqrt(2.0 / F), np.zeros(H)]
    for _ in range(layers):
        parts += [rng.standard_normal(H * H) * math.sqrt(1.0 / H),
                  rng.standard_normal(H * H) * math.sqrt(1.0 / H), np.zeros(H)]
    parts += [rng.standard_normal(H) * math.sqrt(1.0 / H), np.zeros(1),
              rng.standard_normal(H) * math.sqrt(1.0 / H), np.zeros(1)]
    theta = np.concatenate(parts).astype(np.float32)
    if theta.size != load().lorads_gnn_param_count(layers):
        raise RuntimeError("parameter layout mismatch")
    return theta


def train(problems, labels, epochs: int = 40, batch_graphs: int = 16, lr: float = 2e-3,
          omega: float = 1.0, seed: int = 0, y_scale: float = 1.0, val=None):
    """Train on the converged instances; returns (theta, history)."""
    from .lorads import Gnn
    keep = [i for i, l in enumerate(labels) if l["status"] == 0]
    rng = np.random.default_rng(seed)
    order = rng.permutation(keep)
    probs = [problems[i] for i in order]
    node_off, rows, cols, w = graph_set(probs)
    y = np.concatenate([labels[i]["y"] for i in order]) / y_scale
    r = np.array([labels[i]["r"] for i in order], dtype=np.float64) / R_SCALE
    net = Gnn(LAYERS)
    net.load_graphs(node_off, rows, cols, w)
    net.set_targets(y, r)
    net.set_params(init_params(LAYERS, seed))
    G = len(probs)
    starts = list(range(0, G, batch_graphs))
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        lr_ep = lr * 0.5 * (1.0 + math.cos(math.pi * ep / epochs))
        tot = 0.0
        for s in rng.permutation(len(starts)):
            g0 = starts[s]
            g1 = min(G, g0 + batch_graphs)
            loss, _ = net.loss_grad(g0, g1, omega, want_grad=False)
            net.adam_step(lr_ep)
            tot += loss * (g1 - g0)
        entry = dict(epoch=ep, train_loss=tot / G, s=round(time.perf_counter() - t0, 2))
        if val is not None and (ep % 5 == 4 or ep == epochs - 1):
            entry.update(evaluate_loss(net.get_params(), *val, y_scale=y_scale))
        hist.append(entry)
        log(json.dumps(entry))
    ms, launches, flops = net.layer_time()
    theta = net.get_params()
    net.close()
    return theta, hist, dict(layer_ms=ms, layer_launches=launches, layer_flops=flops,
                             train_s=time.perf_counter() - t0, graphs=G,
                             nodes=int(node_off[-1]), directed_edges=int(rows.size))


def evaluate_loss(theta, problems, labels, y_scale=1.0):
    """Held-out relative error of yhat and mean absolute rank error, beside the
    relative error of a per-set least-squares fit y ~ a * sum_k |w_jk| + b (the
    degree-only predictor the network has to beat)."""
    from .lorads import Gnn
    ev = Gnn(LAYERS)
    node_off, rows, cols, w = graph_set(problems)
    ev.load_graphs(node_off, rows, cols, w)
    ev.set_params(theta)
    yh, rh = ev.forward(0, len(problems))
    ev.close()
    y = np.concatenate([l["y"] for l in labels])
    r = np.array([l["r"] for l in labels], dtype=np.float64)
    yh = yh.astype(np.float64) * y_scale
    rel = float(np.linalg.norm(yh - y) / np.linalg.norm(y))
    deg = np.zeros(node_off[-1])
    np.add.at(deg, rows, np.abs(w))
    Amat = np.stack([deg, np.ones_like(deg)], 1)
    coef, *_ = np.linalg.lstsq(Amat, y, rcond=None)
    rel_deg = float(np.linalg.norm(Amat @ coef - y) / np.linalg.norm(y))
    return dict(val_y_rel=rel, val_y_rel_degree_fit=rel_deg,
                val_r_mae=float(np.mean(np.abs(rh * R_SCALE - r))))


# ---------------------------------------------------------------------------
# inference
# ---------------------------------------------------------------------------
class WarmStart:
    """Trained network plus its training range; predicts lambda0 and a rank."""

    def __init__(self, theta: np.ndarray, n_range=N_RANGE, y_scale: float = 1.0,
                 rank_margin: Optional[int] = None):
        self.theta = np.asarray(theta, dtype=np.float32)
        self.n_range = tuple(int(v) for v in n_range)
        self.y_scale = float(y_scale)
        self.rank_margin = rank_margin

    @classmethod
    def load(cls, path=MODEL_PATH):
        z = np.load(path, allow_pickle=False)
        rm = int(z["rank_margin"]) if "rank_margin" in z.files and int(z["rank_margin"]) >= 0 else None
        return cls(z["theta"], tuple(z["n_range"]), float(z["y_scale"]), rm)

    def save(self, path):
        path = pathlib.Path(path)
        path.parent.mkdir(parents=True, exist_ok=True)
        np.savez(path, theta=self.theta, n_range=np.array(self.n_range), y_scale=self.y_scale,
                 rank_margin=-1 if self.rank_margin is None else self.rank_margin)

    def predict(self, problems) -> List[dict]:
        """Per problem: lambda0 (caller constraint order) or None, r0, reason."""
        from .lorads import Gnn
        out: List[Optional[dict]] = [None] * len(problems)
        inside = []
        for k, p in enumerate(problems):
            if not (self.n_range[0] <= p.n <= self.n_range[1]):
                out[k] = dict(lambda0=None, r0=rule_rank(p.n), reason="n outside the training range")
            else:
                inside.append(k)
        if inside:
            sub = [problems[k] for k in inside]
            net = Gnn(LAYERS)
            node_off, rows, cols, w = graph_set(sub)
            net.load_graphs(node_off, rows, cols, w)
            net.set_params(self.theta)
            yh, rh = net.forward(0, len(sub))
            net.close()
            for q, k in enumerate(inside):
                p = problems[k]
                y = yh[node_off[q]:node_off[q + 1]].astype(np.float64) * self.y_scale
                rr = float(rh[q]) * R_SCALE
                if not (np.all(np.isfinite(y)) and math.isfinite(rr)):
                    out[k] = dict(lambda0=None, r0=rule_rank(p.n), reason="non-finite prediction")
                    continue
                lam = -y[node_of_constraint(p)]
                r0 = rule_rank(p.n)
                if self.rank_margin is not None:
                    r0 = int(min(r0, max(2, math.ceil(rr) + self.rank_margin)))
                out[k] = dict(lambda0=lam, r0=r0, reason="learned", rhat=rr)
        return out


# ---------------------------------------------------------------------------
# evaluation
# ---------------------------------------------------------------------------
def sign_test(wins: int, losses: int) -> float:
    """Two-sided exact binomial p-value of wins vs losses (ties dropped)."""
    n = wins + losses
    if n == 0:
        return 1.0
    k = min(wins, losses)
    p = sum(math.comb(n, i) for i in range(k + 1)) / 2.0 ** n
    return float(min(1.0, 2.0 * p))


def evaluate(ws: WarmStart, problems, eps: float = 1e-6, checked: bool = True):
    """Cold and learned start on each problem (same random U0).  With `checked`
    the learned start also runs under options.warm_check ("warm_checked")."""
    from .lorads import Context
    from .params import solver_options
    preds = ws.predict(problems)
    rows, ys = [], []
    for k, (p, pr) in enumerate(zip(problems, preds)):
        ctx = Context([p])
        r_rule = rule_rank(p.n)
        cold = ctx.admm_solve([random_start(p, r_rule)], solver_options("maxcut", p.n, r_rule, eps=eps))[0]
        _, _, lam = ctx.get_solution(0, cold["rank"])
        y = np.empty(p.n)
        y[node_of_constraint(p)] = -lam
        ys.append(y)
        row = dict(n=p.n, reason=pr["reason"], r0=pr["r0"], cold=_summ(cold))
        for name, chk in (("warm", 0), ("warm_checked", 1)):
            if name == "warm_checked" and not checked:
                continue
            if pr["lambda0"] is None:
                row[name] = row["cold"]
                continue
            res = ctx.admm_solve([random_start(p, pr["r0"])],
                                 solver_options("maxcut", p.n, pr["r0"], eps=eps, warm_check=chk),
                                 init_lambda=[pr["lambda0"]])[0]
            row[name] = _summ(res)
        ctx.close()
        rows.append(row)
        log(f"eval {k + 1}/{len(problems)} n={p.n}: cold {row['cold']['t']:.2f}s "
            f"{row['cold']['admm']} it, learned {row['warm']['t']:.2f}s {row['warm']['admm']} it")
    out = {"warm": _compare(rows, "warm")}
    if checked:
        out["warm_checked"] = _compare(rows, "warm_checked")
    # solves whose Appendix-B gap misses the 1e-6 bar, per arm
    for name in ["cold"] + list(out):
        out.setdefault("gap_above_1e-6", {})[name] = int(sum(abs(r[name]["gap"]) > 1e-6 for r in rows))
    # what the network predicts: y_hat against the converged cold solves' y*,
    # beside the degree-only least-squares fit
    keep = [k for k, r in enumerate(rows) if r["cold"]["status"] == 0 and r["reason"] == "learned"]
    if keep:
        labs = [dict(y=ys[k], r=0) for k in keep]
        out["prediction"] = evaluate_loss(ws.theta, [problems[k] for k in keep], labs, ws.y_scale)
    return rows, out


def _summ(r):
    return dict(t=r["t_total"], t1=r["t_phase1"], admm=r["admm_iters"], cg=r["cg_iters"],
                kkt=r["kkt"], status=r["status"], obj=r["obj"], alm_outer=r["alm_outer"],
                alm_inner=r["alm_inner"], fallback=r.get("warm_fallback", 0), rank=r["rank"],
                pinf=r["pinf"], dinf=r["dinf"], gap=r["gap"])


def _compare(rows, name="warm"):
    out = {}
    for key in ("t", "t1", "admm", "cg", "kkt", "alm_inner", "gap", "dinf"):
        c = np.array([abs(r["cold"][key]) for r in rows], dtype=np.float64)
        w = np.array([abs(r[name][key]) for r in rows], dtype=np.float64)
        q = lambda a: [float(np.percentile(a, 25)), float(np.median(a)), float(np.percentile(a, 75))]
        wins, losses = int(np.sum(w < c)), int(np.sum(w > c))
        out[key] = dict(cold_q25_med_q75=q(c), warm_q25_med_q75=q(w), warm_better=wins,
                        warm_worse=losses, sign_test_p=sign_test(wins, losses),
                        median_ratio=float(np.median(w / np.maximum(c, 1e-300))))
    out["instances"] = len(rows)
    out["fallbacks"] = int(sum(r[name]["fallback"] or r["reason"] != "learned" for r in rows))
    out["converged_cold"] = int(sum(r["cold"]["status"] == 0 for r in rows))
    out["converged_learned"] = int(sum(r[name]["status"] == 0 for r in rows))
    out["max_obj_rel_diff"] = float(max(abs(r["cold"]["obj"] - r[name]["obj"]) /
                                        max(1.0, abs(r["cold"]["obj"])) for r in rows))
    return out


# ---------------------------------------------------------------------------
def main(argv: Optional[Sequence[str]] = None):
    ap = argparse.ArgumentParser()
    ap.add_argument("stage", choices=["all", "eval"],
                    help="all: labels, training and evaluation; eval: the shipped network on "
                         "--eval held-out instances")
    ap.add_argument("--out", required=True)
    ap.add_argument("--train", type=int, default=2048)
    ap.add_argument("--heldout", type=int, default=128)
    ap.add_argument("--eval", type=int, default=64, help="held-out instances solved cold and warm")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch-graphs", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--omega", type=float, default=1.0)
    ap.add_argument("--rank-margin", type=int, default=-1, help="-1: keep the rank rule")
    ap.add_argument("--label-chunk", type=int, default=256, help="instances per batched label solve")
    a = ap.parse_args(argv)
    out = pathlib.Path(a.out)
    out.mkdir(parents=True, exist_ok=True)
    report = dict(config=vars(a))
    if a.stage == "eval":
        ws = WarmStart.load()
        rows, cmp = evaluate(ws, instances(a.eval, HELDOUT_SEED0))
        report["evaluation"] = cmp
        report["evaluation_rows"] = rows
        log(json.dumps(cmp))
        (out / "report.json").write_text(json.dumps(report, indent=1))
        return
    t = time.perf_counter()
    tr = instances(a.train, TRAIN_SEED0)
    ho = instances(a.heldout, HELDOUT_SEED0)
    log(f"generated {len(tr)} + {len(ho)} instances in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    lab_tr = make_labels(tr, a.label_chunk)
    lab_ho = make_labels(ho, a.label_chunk)
    report["labels"] = dict(s=round(time.perf_counter() - t, 1),
                            train_converged=sum(l["status"] == 0 for l in lab_tr),
                            heldout_converged=sum(l["status"] == 0 for l in lab_ho),
                            r_star_hist=np.bincount([l["r"] for l in lab_tr]).tolist(),
                            final_rank_hist=np.bincount([l["rank"] for l in lab_tr]).tolist(),
                            admm_median=float(np.median([l["admm_iters"] for l in lab_tr])))
    log(json.dumps(report["labels"]))
    ys = float(np.std(np.concatenate([l["y"] for l in lab_tr])))
    hk = [i for i, l in enumerate(lab_ho) if l["status"] == 0]
    theta, hist, perf = train(tr, lab_tr, a.epochs, a.batch_graphs, a.lr, a.omega, 0, ys,
                              val=([ho[i] for i in hk], [lab_ho[i] for i in hk]))
    report["train"] = dict(history=hist, perf=perf, y_scale=ys)
    ws = WarmStart(theta, N_RANGE, ys, None if a.rank_margin < 0 else a.rank_margin)
    ws.save(out / "gnn_maxcut.npz")
    rows, cmp = evaluate(ws, ho[:a.eval])
    report["evaluation"] = cmp
    report["evaluation_rows"] = rows
    log(json.dumps(cmp))
    (out / "report.json").write_text(json.dumps(report, indent=1))


if __name__ == "__main__":
    main()
