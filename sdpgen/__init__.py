"""Seeded synthetic SDP instances shaped like the paper's workloads.

This module only *builds problem data* (C, the constraint matrices A_i, b) and
random starting points; it performs none of the solver's arithmetic, so both the
CPU oracle and the GPU library consume it.

Problem form (linear SDP of the paper's problem statement, Section 1):

    min <C, X>  s.t.  <A_i, X> = b_i (i < m),  X PSD,  X of order n.

Sparse symmetric matrices are given as upper-triangle COO triplets (row <= col).
An off-diagonal triplet (j, k, v) stands for both (j, k) and (k, j).

Workload families (Section 5.3 MaxCut, Section 5.4 matrix completion):

* MaxCut: C = -L(G, w)/4 with L the weighted Laplacian, A_i = e_i e_i^T, b = 1.
  Minimising <C, X> is the paper's max-form relaxation with the sign flipped.
* Matrix completion: X of order n1 + n2, C = I/2, one constraint per observed
  entry (j, k): A = (e_j e_{n1+k}^T + e_{n1+k} e_j^T)/2, b = M_jk.  This is the
  paper's formulation with C and A halved; the feasible set is the same and the
  optimal value equals the nuclear norm of M at exact recovery.

Every generator takes an integer seed and draws from numpy's PCG64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Problem", "maxcut_from_edges", "er_gnp_edges", "gnm_edges", "torus_edges",
    "maxcut_er", "maxcut_gnm", "maxcut_torus", "mc_planted", "mc_sample_count",
    "mc_paper_sample", "random_init_U", "batch_maxcut", "generic_random",
    "rank_rule_2lnm", "rank_rule_sqrt2m", "config_instance", "CONFIGS",
]


@dataclasses.dataclass
class Problem:
    """Host-side SDP instance in upper-triangle COO form."""
    n: int
    m: int
    c_row: np.ndarray  # int32
    c_col: np.ndarray  # int32
    c_val: np.ndarray  # float64
    a_con: np.ndarray  # int32, constraint id of each triplet
    a_row: np.ndarray  # int32
    a_col: np.ndarray  # int32
    a_val: np.ndarray  # float64
    b: np.ndarray      # float64, length m
    kind: str = "generic"           # "maxcut" | "mc" | "generic"
    meta: dict = dataclasses.field(default_factory=dict)
    # objective f(X) = <C, X> + (mu / 2) ||X||_F^2 (mu = 0: the linear SDP)
    mu: float = 0.0

    def __post_init__(self):
        self.c_row = np.ascontiguousarray(self.c_row, dtype=np.int32)
        self.c_col = np.ascontiguousarray(self.c_col, dtype=np.int32)
        self.c_val = np.ascontiguousarray(self.c_val, dtype=np.float64)
        self.a_con = np.ascontiguousarray(self.a_con, dtype=np.int32)
        self.a_row = np.ascontiguousarray(self.a_row, dtype=np.int32)
        self.a_col = np.ascontiguousarray(self.a_col, dtype=np.int32)
        self.a_val = np.ascontiguousarray(self.a_val, dtype=np.float64)
        self.b = np.ascontiguousarray(self.b, dtype=np.float64)

    @property
    def c_nnz(self) -> int:
        return int(self.c_row.size)

    @property
    def a_nnz(self) -> int:
        return int(self.a_row.size)


# ----------------------------------------------------------------------------
# graphs
# ----------------------------------------------------------------------------

def _dedupe_pairs(i: np.ndarray, j: np.ndarray, n: int):
    lo = np.minimum(i, j).astype(np.int64)
    hi = np.maximum(i, j).astype(np.int64)
    keep = lo != hi
    key = np.unique(lo[keep] * n + hi[keep])
    return key


def gnm_edges(n: int, M: int, rng: np.random.Generator):
    """Exactly M distinct non-loop edges drawn uniformly (Erdos-Renyi G(n, M))."""
    total = n * (n - 1) // 2
    if M > total:
        raise ValueError("too many edges")
    keys = np.empty(0, dtype=np.int64)
    while keys.size < M:
        need = M - keys.size
        draw = int(need * 1.2) + 16
        i = rng.integers(0, n, size=draw)
        j = rng.integers(0, n, size=draw)
        keys = np.union1d(keys, _dedupe_pairs(i, j, n))
    if keys.size > M:
        keys = np.sort(rng.choice(keys, size=M, replace=False))
    return (keys // n).astype(np.int32), (keys % n).astype(np.int32)


def er_gnp_edges(n: int, p: float, rng: np.random.Generator):
    """G(n, p): every pair present independently with probability p.

    The edge count is Binomial(n(n-1)/2, p); given the count the edge set is a
    uniform subset, which is the same law as independent coin flips.
    """
    total = n * (n - 1) // 2
    if total <= 200_000:
        iu, ju = np.triu_indices(n, 1)
        flips = rng.random(total) < p
        return iu[flips].astype(np.int32), ju[flips].astype(np.int32)
    M = int(rng.binomial(total, p))
    return gnm_edges(n, M, rng)


def torus_edges(a: int, b: int):
    """2D toroidal grid a x b: node (x, y) ~ (x+-1 mod a, y) and (x, y+-1 mod b)."""
    ei, ej = [], []
    for x in range(a):
        for y in range(b):
            u = x * b + y
            ei.append(u); ej.append(((x + 1) % a) * b + y)
            ei.append(u); ej.append(x * b + (y + 1) % b)
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    lo, hi = np.minimum(ei, ej), np.maximum(ei, ej)
    key = np.unique(lo * (a * b) + hi)
    return (key // (a * b)).astype(np.int32), (key % (a * b)).astype(np.int32)


def maxcut_from_edges(n: int, ei, ej, w, meta: Optional[dict] = None) -> Problem:
    """MaxCut relaxation in min form: C = -L/4, diag(X) = 1 (Section 5.3)."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    lo, hi = np.minimum(ei, ej), np.maximum(ei, ej)
    deg = np.bincount(lo, weights=w, minlength=n) + np.bincount(hi, weights=w, minlength=n)
    # L_jj = sum_k w_jk, L_jk = -w_jk  =>  C_jj = -deg_j/4, C_jk = +w_jk/4
    c_row = np.concatenate([np.arange(n), lo])
    c_col = np.concatenate([np.arange(n), hi])
    c_val = np.concatenate([-deg / 4.0, w / 4.0])
    ar = np.arange(n)
    md = {"edges": (lo.astype(np.int32), hi.astype(np.int32), w)}
    if meta:
        md.update(meta)
    return Problem(n=n, m=n, c_row=c_row, c_col=c_col, c_val=c_val,
                   a_con=ar, a_row=ar, a_col=ar, a_val=np.ones(n), b=np.ones(n),
                   kind="maxcut", meta=md)


def maxcut_er(n: int, p: float, seed: int, weights: str = "unit") -> Problem:
    rng = np.random.default_rng(seed)
    ei, ej = er_gnp_edges(n, p, rng)
    w = _weights(ei.size, weights, rng)
    return maxcut_from_edges(n, ei, ej, w, {"seed": seed, "family": f"G({n},p={p})"})


def maxcut_gnm(n: int, M: int, seed: int, weights: str = "unit") -> Problem:
    rng = np.random.default_rng(seed)
    ei, ej = gnm_edges(n, M, rng)
    w = _weights(ei.size, weights, rng)
    return maxcut_from_edges(n, ei, ej, w, {"seed": seed, "family": f"G({n},M={M})"})


def maxcut_torus(a: int, b: int, seed: int, weights: str = "pm1") -> Problem:
    rng = np.random.default_rng(seed)
    ei, ej = torus_edges(a, b)
    w = _weights(ei.size, weights, rng)
    return maxcut_from_edges(a * b, ei, ej, w, {"seed": seed, "family": f"torus{a}x{b}"})


def _weights(k: int, kind: str, rng: np.random.Generator) -> np.ndarray:
    if kind == "unit":
        return np.ones(k)
    if kind == "pm1":
        return rng.choice(np.array([-1.0, 1.0]), size=k)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# matrix completion
# ----------------------------------------------------------------------------

def mc_sample_count(d: int, draws: int) -> float:
    """Expected number of distinct cells after `draws` uniform draws (with
    replacement) from a d x d grid."""
    cells = float(d) * d
    return cells * (1.0 - math.exp(draws * math.log1p(-1.0 / cells)))


def mc_planted(n1: int, n2: int, rank: int, seed: int, count: Optional[int] = None,
               draws: Optional[int] = None) -> Problem:
    """Planted low-rank completion: M = L R^T with L, R ~ N(0, 1).

    Either `count` distinct observed cells drawn uniformly without replacement,
    or `draws` uniform draws with replacement, deduplicated.  Observed cells are
    listed in lexicographic (row, column) order.
    """
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((n1, rank))
    R = rng.standard_normal((n2, rank))
    cells = n1 * n2
    if count is not None:
        keys = np.empty(0, dtype=np.int64)
        while keys.size < count:
            need = count - keys.size
            keys = np.union1d(keys, rng.integers(0, cells, size=int(need * 1.05) + 64))
        if keys.size > count:
            keys = np.sort(rng.choice(keys, size=count, replace=False))
    elif draws is not None:
        keys = np.unique(rng.integers(0, cells, size=draws))
    else:
        raise ValueError("count or draws")
    j = (keys // n2).astype(np.int64)
    k = (keys % n2).astype(np.int64)
    m = keys.size
    bvals = np.einsum("ij,ij->i", L[j], R[k])
    n = n1 + n2
    ar = np.arange(n)
    return Problem(n=n, m=m, c_row=ar, c_col=ar, c_val=np.full(n, 0.5),
                   a_con=np.arange(m), a_row=j, a_col=n1 + k, a_val=np.full(m, 0.5),
                   b=bvals, kind="mc",
                   meta={"n1": n1, "n2": n2, "L": L, "R": R, "seed": seed,
                         "family": f"MC {n1}x{n2} rank{rank}"})


def mc_paper_sample(n_x: int, seed: int, rank: int = 5) -> Problem:
    """MC_n_x of Table 5 shape: X of order n_x, M of order n_x/2, 800 * (n_x/2)
    uniform draws with replacement, deduplicated."""
    d = n_x // 2
    return mc_planted(d, d, rank, seed, draws=800 * d)


# ----------------------------------------------------------------------------
# small generic SDPs (for brute-force cross-checks)
# ----------------------------------------------------------------------------

def generic_random(n: int, m: int, seed: int, density: float = 0.3) -> Problem:
    """Random sparse symmetric A_i, b = A(X0) for a random X0 PSD, C = G G^T + I
    (so the dual is strictly feasible and the primal is feasible: the optimum
    is attained)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) / math.sqrt(n)
    Cd = G @ G.T + 0.5 * np.eye(n) + 0.3 * (rng.standard_normal((n, n)))
    Cd = (Cd + Cd.T) / 2
    # make C PSD-ish but indefinite parts allowed; shift keeps the dual feasible
    w = np.linalg.eigvalsh(Cd)
    if w[0] < 0.1:
        Cd += (0.1 - w[0]) * np.eye(n)
    ir, ic = np.triu_indices(n)
    c_row, c_col, c_val = ir, ic, Cd[ir, ic]
    cons, rows, cols, vals = [], [], [], []
    for i in range(m):
        mask = rng.random(ir.size) < density
        if not mask.any():
            mask[rng.integers(0, ir.size)] = True
        sel = np.nonzero(mask)[0]
        cons.append(np.full(sel.size, i)); rows.append(ir[sel]); cols.append(ic[sel])
        vals.append(rng.standard_normal(sel.size))
    F = rng.standard_normal((n, n))
    X0 = F @ F.T / n + np.eye(n) * 0.1
    con = np.concatenate(cons); row = np.concatenate(rows); col = np.concatenate(cols)
    val = np.concatenate(vals)
    # b_i = <A_i, X0>, off-diagonal triplets count twice
    contrib = val * X0[row, col] * np.where(row == col, 1.0, 2.0)
    b = np.bincount(con, weights=contrib, minlength=m)
    return Problem(n=n, m=m, c_row=c_row, c_col=c_col, c_val=c_val, a_con=con,
                   a_row=row, a_col=col, a_val=val, b=b, kind="generic",
                   meta={"seed": seed, "X0": X0})


# ----------------------------------------------------------------------------
# starting points and rank rules
# ----------------------------------------------------------------------------

def random_init_U(n: int, r: int, seed: int) -> np.ndarray:
    """Random start for the warm-start phase: i.i.d. N(0, 1/r) entries."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5EED]))
    return rng.standard_normal((n, r)) / math.sqrt(r)


def rank_rule_2lnm(m: int) -> int:
    """Initial rank 2 log m of Section 5.1 (natural log, rounded)."""
    return int(round(2.0 * math.log(m)))


def rank_rule_sqrt2m(m: int) -> int:
    return int(round(math.sqrt(2.0 * m)))


# ----------------------------------------------------------------------------
# batches and the named workloads
# ----------------------------------------------------------------------------

def batch_maxcut(count: int, seed0: int, n_lo: int, n_hi: int, deg_lo: float, deg_hi: float,
                 weights: str = "pm1"):
    """Ragged batch of ER MaxCut instances: n ~ U{n_lo..n_hi}, average degree
    ~ U[deg_lo, deg_hi], p = deg/(n-1)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(rng.integers(n_lo, n_hi + 1))
        d = float(rng.uniform(deg_lo, deg_hi))
        p = min(1.0, d / (n - 1))
        ei, ej = er_gnp_edges(n, p, rng)
        w = _weights(ei.size, weights, rng)
        out.append(maxcut_from_edges(n, ei, ej, w, {"seed": seed0 + i, "avg_degree": d}))
    return out


CONFIGS = {
    # small FP64 MaxCut: G(200, 0.05), unit weights, r0 = ceil(log2 n)
    "maxcut_er200": dict(kind="maxcut", seed=1001),
    # 100 x 100 torus, +-1 weights
    "maxcut_torus100": dict(kind="maxcut", seed=1002),
    # G(20000, M=60000), unit weights (average degree 6)
    "maxcut_gnm20000": dict(kind="maxcut", seed=1003),
    # planted rank-5 completion, 10000 x 10000 with 4,605,170 observed cells
    "mc_10000": dict(kind="mc", seed=1004),
    # planted rank-5 completion, 20000 x 20000, 800 d draws deduplicated
    "mc_20000": dict(kind="mc", seed=1005),
}


def config_instance(name: str) -> Problem:
    if name == "maxcut_er200":
        return maxcut_er(200, 0.05, 1001, "unit")
    if name == "maxcut_torus100":
        return maxcut_torus(100, 100, 1002, "pm1")
    if name == "maxcut_gnm20000":
        return maxcut_gnm(20000, 60000, 1003, "unit")
    if name == "mc_10000":
        return mc_planted(10000, 10000, 5, 1004, count=4_605_170)
    if name == "mc_20000":
        return mc_paper_sample(40000, 1005)
    raise KeyError(name)


# ----------------------------------------------------------------------------
# Lovasz theta SDPs: min <-J, X> s.t. tr X = 1, X_ij = 0 on the graph's edges,
# X PSD; the optimal value is -theta(G) (a general-structure family with a
# dense cost)
# ----------------------------------------------------------------------------

def lovasz_theta(n: int, edges) -> Problem:
    ei = np.array([min(a, b) for a, b in edges], dtype=np.int64)
    ej = np.array([max(a, b) for a, b in edges], dtype=np.int64)
    ir, ic = np.triu_indices(n)
    c_row, c_col, c_val = ir, ic, np.full(ir.size, -1.0)
    m = 1 + ei.size
    con = np.concatenate([np.zeros(n, dtype=np.int64), 1 + np.arange(ei.size)])
    row = np.concatenate([np.arange(n), ei])
    col = np.concatenate([np.arange(n), ej])
    # an off-diagonal triplet counts twice in <A_i, X>: 0.5 gives X_ij itself
    val = np.concatenate([np.ones(n), np.full(ei.size, 0.5)])
    b = np.zeros(m)
    b[0] = 1.0
    return Problem(n=n, m=m, c_row=c_row, c_col=c_col, c_val=c_val, a_con=con,
                   a_row=row, a_col=col, a_val=val, b=b, kind="theta",
                   meta={"graph_edges": len(edges)})


def cycle_edges(n: int):
    return [(i, (i + 1) % n) for i in range(n)]


def complete_edges(n: int):
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def petersen_edges():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return outer + spokes + inner


# ----------------------------------------------------------------------------
# Rank-one constraints: every A_i = a_i a_i^T (Section 3's sensor network
# localization relaxation; the balance constraint of graph bisection)
# ----------------------------------------------------------------------------

def _rank_one_triplets(con: int, idx, val):
    """Upper-triangle triplets of a a^T for a sparse a (indices ascending):
    diagonal a_k^2, off-diagonal a_j a_k (one triplet stands for both sides)."""
    idx = np.asarray(idx, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    order = np.argsort(idx)
    idx, val = idx[order], val[order]
    iu, ju = np.triu_indices(idx.size)
    return (np.full(iu.size, con, dtype=np.int64), idx[iu], idx[ju], val[iu] * val[ju])


def snl(n_sensors: int, n_anchors: int, radius: float, seed: int, d: int = 2) -> Problem:
    """SDP relaxation of sensor network localization (Section 3) with exact
    distances, sensors and anchors uniform in [-0.5, 0.5]^d (see
    snl_positions)."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(-0.5, 0.5, (n_sensors, d))
    A = rng.uniform(-0.5, 0.5, (n_anchors, d))
    p = snl_positions(X, A, radius)
    p.meta.update(seed=seed, family=f"SNL({n_sensors}, {n_anchors}, r={radius})")
    return p


def snl_positions(X, A, radius: float = np.inf) -> Problem:
    """SDP relaxation of sensor network localization (Section 3) for given
    sensor positions X (n_s x d) and anchors A (n_a x d), exact distances:
    Z of order d + n_s, Z[:d, :d] = I written with rank-one constraints
    (Z_kk = 1 and <(e_k + e_l)(e_k + e_l)^T, Z> = 2), one constraint
    <(0; e_i - e_j)(0; e_i - e_j)^T, Z> = |x_i - x_j|^2 per sensor pair closer
    than `radius` and <(a_k; -e_j)(a_k; -e_j)^T, Z> = |a_k - x_j|^2 per
    anchor-sensor pair closer than `radius`; C = 0.  The true positions are
    kept in meta."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    n_sensors, d = X.shape
    n_anchors = A.shape[0]
    parts, b = [], []

    def add(idx, val, rhs):
        parts.append(_rank_one_triplets(len(b), idx, val))
        b.append(rhs)

    for k in range(d):
        add([k], [1.0], 1.0)
    for k in range(d):
        for l in range(k + 1, d):
            add([k, l], [1.0, 1.0], 2.0)
    ss = 0
    for i in range(n_sensors):
        dist = np.linalg.norm(X[i + 1:] - X[i], axis=1)
        for j in np.nonzero(dist < radius)[0] + i + 1:
            add([d + i, d + j], [1.0, -1.0], float(np.sum((X[i] - X[j]) ** 2)))
            ss += 1
    sa = 0
    for k in range(n_anchors):
        dist = np.linalg.norm(X - A[k], axis=1)
        for j in np.nonzero(dist < radius)[0]:
            add(list(range(d)) + [d + j], list(A[k]) + [-1.0], float(np.sum((A[k] - X[j]) ** 2)))
            sa += 1
    con, row, col, val = (np.concatenate([p[t] for p in parts]) for t in range(4))
    n = d + n_sensors
    return Problem(n=n, m=len(b), c_row=np.zeros(0), c_col=np.zeros(0), c_val=np.zeros(0),
                   a_con=con, a_row=row, a_col=col, a_val=val, b=np.asarray(b), kind="snl",
                   meta={"d": d, "sensors": X, "anchors": A, "sensor_pairs": ss,
                         "anchor_pairs": sa, "family": f"SNL({n_sensors}, {n_anchors})"})


def min_bisection(n: int, ei, ej, w, meta: Optional[dict] = None) -> Problem:
    """Graph bisection relaxation: min <L/4, X> s.t. diag(X) = 1 and
    <J / n, X> = 0 (x in {-1, 1}^n with sum x = 0), J / n = a a^T with
    a = 1 / sqrt(n) the one dense rank-one constraint (scaled like the diagonal
    ones: ||a|| = 1).  The value bounds the minimum bisection width from below."""
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    lo, hi = np.minimum(ei, ej), np.maximum(ei, ej)
    deg = np.bincount(lo, weights=w, minlength=n) + np.bincount(hi, weights=w, minlength=n)
    c_row = np.concatenate([np.arange(n), lo])
    c_col = np.concatenate([np.arange(n), hi])
    c_val = np.concatenate([deg / 4.0, -w / 4.0])
    ar = np.arange(n)
    jc, jr, jcol, jv = _rank_one_triplets(n, ar, np.full(n, 1.0 / np.sqrt(n)))
    md = {"edges": (lo.astype(np.int32), hi.astype(np.int32), w)}
    if meta:
        md.update(meta)
    return Problem(n=n, m=n + 1, c_row=c_row, c_col=c_col, c_val=c_val,
                   a_con=np.concatenate([ar, jc]), a_row=np.concatenate([ar, jr]),
                   a_col=np.concatenate([ar, jcol]), a_val=np.concatenate([np.ones(n), jv]),
                   b=np.concatenate([np.ones(n), [0.0]]), kind="partition", meta=md)


def min_bisection_er(n: int, p: float, seed: int, weights: str = "unit") -> Problem:
    rng = np.random.default_rng(seed)
    ei, ej = er_gnp_edges(n, p, rng)
    w = _weights(ei.size, weights, rng)
    return min_bisection(n, ei, ej, w, {"seed": seed, "family": f"bisection G({n},p={p})"})
