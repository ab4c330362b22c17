// LoRADS driver: Phase I (Burer-Monteiro ALM with L-BFGS, exact quartic line
// search and dynamic rank), the switch, Phase II (ADMM with CG subproblem
// solves) and the Appendix-B error measures.  Host code orchestrates device
// kernels; every vector operation of the path runs on the GPU, the host only
// keeps scalars (rho, gamma, tolerances, iteration counts) and makes the decisions.
#include <algorithm>
#include <chrono>
#include <complex>

#include "kernels.hpp"
#include "kernels_quad.hpp"
#include "solver.hpp"

namespace lorads {

namespace {

using Clock = std::chrono::steady_clock;
double secs(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

inline int gridN(size_t N) { return grid_for(N, 2048); }

// Real roots of c3 x^3 + c2 x^2 + c1 x + c0 (c3 may be 0).
std::vector<double> real_roots_cubic(double c3, double c2, double c1, double c0) {
  std::vector<double> out;
  if (c3 == 0.0) {
    if (c2 == 0.0) {
      if (c1 != 0.0) out.push_back(-c0 / c1);
      return out;
    }
    const double disc = c1 * c1 - 4 * c2 * c0;
    if (disc >= 0) {
      const double q = -0.5 * (c1 + std::copysign(std::sqrt(disc), c1));
      if (q != 0.0) out.push_back(q / c2);
      if (q != 0.0) out.push_back(c0 / q); else out.push_back(0.0);
    }
    return out;
  }
  // depressed cubic via the trigonometric / Cardano formulas, then two Newton
  // polish steps per root on the original polynomial
  const double a = c2 / c3, b = c1 / c3, c = c0 / c3;
  const double Q = (a * a - 3 * b) / 9.0;
  const double R = (2 * a * a * a - 9 * a * b + 27 * c) / 54.0;
  const double Q3 = Q * Q * Q;
  if (R * R < Q3) {
    const double th = std::acos(std::max(-1.0, std::min(1.0, R / std::sqrt(Q3))));
    const double sq = -2.0 * std::sqrt(Q);
    out.push_back(sq * std::cos(th / 3.0) - a / 3.0);
    out.push_back(sq * std::cos((th + 2 * M_PI) / 3.0) - a / 3.0);
    out.push_back(sq * std::cos((th - 2 * M_PI) / 3.0) - a / 3.0);
  } else {
    const double A = -std::copysign(std::cbrt(std::fabs(R) + std::sqrt(R * R - Q3)), R);
    const double B = (A != 0.0) ? Q / A : 0.0;
    out.push_back((A + B) - a / 3.0);
  }
  for (double& x : out) {
    for (int it = 0; it < 2; ++it) {
      const double f = ((c3 * x + c2) * x + c1) * x + c0;
      const double df = (3 * c3 * x + 2 * c2) * x + c1;
      if (df != 0.0) x -= f / df;
    }
  }
  return out;
}

}  // namespace

// minimiser over a > 0 of q1 a + q2 a^2 + q3 a^3 + q4 a^4
double quartic_step(double q1, double q2, double q3, double q4) {
  const auto roots = real_roots_cubic(4 * q4, 3 * q3, 2 * q2, q1);
  double best = 0.0, bestv = 0.0;
  for (double a : roots) {
    if (!(a > 0.0)) continue;
    const double v = (((q4 * a + q3) * a + q2) * a + q1) * a;
    if (v < bestv) { best = a; bestv = v; }
  }
  return best;
}

// gamma_rule 1 reads ||C||_2, which phase2 estimates before its first use
double gamma_of(const Problem& P, const lorads_options& o, double rho) {
  (void)rho;
  if (o.gamma_fixed > 0) return o.gamma_fixed;
  if (o.gamma_rule == 1) {
    if (P.c_norm2 < 0.0) fail(LORADS_EINVAL, "gamma rule 1 before the estimate of ||C||_2");
    return o.gamma_scale * (1.0 + P.c_norm2);
  }
  return o.gamma_scale * (1.0 + P.c_fro / std::sqrt((double)P.n));
}

// ===========================================================================
// Phase I: augmented Lagrangian on the factorised problem
//   L(U) = <C, U U^T> + lam^T (A(U U^T) - b) + rho/2 ||A(U U^T) - b||^2
//   grad = 2 (C + A*(lam + rho (A(U U^T) - b))) U
// ===========================================================================
// Factor-shaped work arrays have row stride ld: for PAIR problems rows are
// padded to whole 64-byte sectors (zero padding, the layout of the CG work
// buffers), so a gathered row of U or D is one aligned cache line; other
// structures use ld = r.  Zero padding is kept by every update (the vector
// updates are linear and the operators write columns < r only).
struct AlmState {
  int n, m, r, ld;
  DevBuf<double> G, Gn, D, Q, CD, p1, p2, Sn, Yn;
  // quadratic objective: U^T U (at the last gradient), U^T D, D^T D
  DevBuf<double> gUU, gUD, gDD;
  DevBuf<double> lsp;  // block partials of the fused line-search pass
  std::vector<DevBuf<double>> S, Y;
  // slot of sc holding <S, Y> of each pair buffer (it travels with the buffer)
  std::vector<int> sy;
  int sy_n = 0;
  int head = 0, count = 0;
};

// FP64 factor rows of PAIR problems: whole 64-byte sectors, and at least the
// lane group G (up to 32) so the two-column kernels apply (r = 17..24 gets 32
// columns rather than 24)
static int alm_ld(const Problem& P, int r) {
  if (P.structure != LORADS_STRUCT_PAIR) return r;
  const int ld = cg_ld(P, r, (int)sizeof(double));
  const int G = lane_group(r);
  return G <= 32 ? std::max(ld, G) : ld;
}

static void alm_alloc(AlmState& A, int n, int m, int r, int ld, int mem, hipStream_t s) {
  A.n = n; A.m = m; A.r = r; A.ld = ld;
  const size_t N = (size_t)n * ld;
  // every array starts zeroed (padding columns must stay zero; no kernel may
  // meet a stale value)
  for (DevBuf<double>* b : {&A.G, &A.Gn, &A.D, &A.Q, &A.CD, &A.Sn, &A.Yn}) {
    b->alloc(N);
    b->zero(s);
  }
  A.p1.alloc(m); A.p2.alloc(m);
  A.gUU.alloc((size_t)r * r); A.gUD.alloc((size_t)r * r); A.gDD.alloc((size_t)r * r);

  A.S.resize(mem); A.Y.resize(mem);
  A.sy.resize(mem);
  for (int i = 0; i < mem; ++i) A.sy[i] = S_PAIRS + i;
  A.sy_n = S_PAIRS + mem;
  for (int i = 0; i < mem; ++i) {
    A.S[i].alloc(N);
    A.Y[i].alloc(N);
    A.S[i].zero(s);
    A.Y[i].zero(s);
  }
  A.head = A.count = 0;
}

// G = 2 (C + A*(lam + rho (z - b))) U with z = A(U U^T) recomputed, plus
// 2 mu U (U^T U) for the quadratic objective (U^T U kept for the line search)
static void alm_gradient(Problem& P, AlmState& A, const double* U, double* G, double rho,
                         hipStream_t s, double& bytes);
static void alm_gradient_linear(Problem& P, AlmState& A, const double* U, double* G, double rho,
                                hipStream_t s, double& bytes) {
  if (grad_pair_ready(P)) {
    // the gradient forms w per entry and returns z = A(U U^T) for the line
    // search and the infeasibility
    op_grad_pair(P, U, A.r, A.ld, rho, G, A.ld, 2.0, s, P.zbuf.p);
    bytes += bytes_grad_pair(P, A.r);
  } else {
    op_forward_w(P, U, U, A.r, A.ld, P.zbuf.p, P.wbuf.p, P.lam.p, rho, s);
    op_adjoint<double>(P, P.wbuf.p, 1.0, U, A.r, A.ld, G, A.ld, 2.0, s);
    bytes += bytes_forward(P, A.r, 8) + bytes_adjoint(P, A.r, 8, true);
  }
}

static void alm_gradient(Problem& P, AlmState& A, const double* U, double* G, double rho,
                         hipStream_t s, double& bytes) {
  alm_gradient_linear(P, A, U, G, rho, s, bytes);
  if (P.mu != 0.0) {
    gram_small<double>(P, A.n, A.r, A.r, U, A.ld, U, A.ld, A.gUU.p, s);
    add_xg<double, double><<<grid_for((size_t)A.n * A.r), kBlock, 0, s>>>(A.n, A.r, A.r, U, A.ld, A.gUU.p,
                                                                         2.0 * P.mu, G, A.ld);
    HIPCHK(hipGetLastError());
  }
}

// Phase I's copy of U in the working layout (the master P.U stays n x r)
struct AlmFactor {
  DevBuf<double> buf;
  double* U = nullptr;
  int ld = 0;
  void load(Problem& P, int r, int ld_, hipStream_t s) {
    ld = ld_;
    if (ld == r) { U = P.U.p; return; }
    buf.alloc((size_t)P.n * ld);
    buf.zero(s);
    copy_rows<double, double><<<gridN((size_t)P.n * r), kBlock, 0, s>>>(P.n, r, P.U.p, r, buf.p, ld);
    HIPCHK(hipGetLastError());
    U = buf.p;
  }
  void store(Problem& P, int r, hipStream_t s) {
    if (ld == r) return;
    copy_rows<double, double><<<gridN((size_t)P.n * r), kBlock, 0, s>>>(P.n, r, buf.p, ld, P.U.p, r);
    HIPCHK(hipGetLastError());
  }
};

static double host_norm_zb(Problem& P, hipStream_t s) {
  // ||z - b||_2 via dual_update with rho = 0 (lam unchanged)
  dual_update_slot(P, P.zbuf.p, 0.0, P.lam.p, S_GEN, s);
  double v;
  read_slots(P, S_GEN, &v, 1, s);
  return std::sqrt(v);
}

void phase1(Problem& P, const lorads_options& o, SolveInfo& info, hipStream_t s) {
  const int n = P.n, m = P.m;
  int r = P.rank;
  const int r_cap = rank_cap(P, o);
  const double c_fro = P.c_fro;
  double rho = o.rho0 > 0 ? o.rho0 : 1.0 / std::max(1.0, P.b_inf);
  AlmState A;
  AlmFactor F;
  refresh_inc_lam(P, s);
  F.load(P, r, alm_ld(P, r), s);
  alm_alloc(A, n, m, r, F.ld, o.lbfgs_mem, s);
  double* U = F.U;
  // mixed form: FP32 copies of U and of the direction for the line search's
  // maps (same row stride, zero padding); gf = lanes per constraint
  DevBuf<float> U32, D32;
  int gf = 0;
  auto cast_rows = [&](const double* X, float* Y) {
    copy_rows<double, float><<<gridN((size_t)n * r), kBlock, 0, s>>>(n, r, X, F.ld, Y, F.ld);
    HIPCHK(hipGetLastError());
  };
  auto setup_mixed = [&]() {
    gf = o.precision == LORADS_MIXED ? pair_f32_lanes(P, r, F.ld) : 0;
    if (!gf) return;
    U32.alloc((size_t)n * F.ld);
    U32.zero(s);
    D32.alloc((size_t)n * F.ld);
    D32.zero(s);
    cast_rows(U, U32.p);
  };
  setup_mixed();
  // factor dots in the compact summation order whatever the row stride
  auto adot = [&](const double* X, const double* Y, double scale, int slot, hipStream_t st) {
    dot_rows_to_slot(P, n, r, F.ld, X, Y, scale, slot, st);
  };
  op_forward<double>(P, U, U, r, F.ld, P.zbuf.p, 1.0, s);
  info.op_bytes += bytes_forward(P, r, 8);
  double v = host_norm_zb(P, s) / (1.0 + P.b_inf);
  double v_ref = INFINITY;
  int outer = 0, inner_total = 0, growths = 0;
  double h[16];
  // a caller multiplier is kept only if the first outer iteration lowers the
  // infeasibility; otherwise Phase I restarts cold from the same U
  const double v_start = v, rho_start = rho;
  bool warm_pending = info.warm;
  DevBuf<double> U_start;
  if (warm_pending) {
    U_start.alloc((size_t)n * F.ld);
    HIPCHK(hipMemcpyAsync(U_start.p, U, (size_t)n * F.ld * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  while (v > o.switch_tol && outer < o.alm_outer_max) {
    const int cap = (r < r_cap) ? o.rank_grow_iters : o.alm_inner_max;
    const double tol = std::max(o.alm_inner_rel * v, o.alm_inner_floor);
    const size_t N = (size_t)n * F.ld;
    // ---------------- inner L-BFGS ----------------
    A.head = A.count = 0;
    alm_gradient(P, A, U, A.G.p, rho, s, info.op_bytes);
    adot(A.G.p, A.G.p, 1.0, S_GEN, s);
    read_slots(P, S_GEN, h, 1, s);
    double gnorm2 = h[0];  // ||G||^2 of the current gradient
    int it = 0;
    bool conv = false;
    const unsigned Nc = (unsigned)((size_t)n * r);
    const int rg = grid_for((size_t)n * r, kRedBlocks);
    const int mem = o.lbfgs_mem;
    double* part = P.part.p;
    // Each pass of the two-loop finishes the previous pass's sums itself
    // (PrevSums), so the passes write their partials to two alternating
    // regions of P.part; the last pass's <G, D> partials go above the
    // line-search partials and are summed by the line search's finishing
    // launch.  1 / <S, Y> of a pair is formed on the device from the pair's
    // own slot, exactly as the host would form it.
    double* pbuf[2] = {part, part + kLbfgsPartStride};
    double* part_gd = part + 3 * kLbfgsPartStride;
    // the pair kernel's four sums (read by its finish and, while its pair is
    // the newest in memory, by the next two-loop's first pass)
    double* part_pair = pbuf[1];
    static_assert(4 * kRedBlocks <= kLbfgsPartStride, "pair sums exceed their region");
    bool fresh_pair = false;
    P.ensure_part((size_t)4 * kLbfgsPartStride);
    // two-loop recursion, newest pair first, in fused passes (each pass
    // updates q and forms the next dot; q = G until the first update).  The
    // scalars stay on the device: alphas in slots S_GEN+16+t, <S,Y> and
    // <Y,Y> of the newest pair in S_GEN+1, S_GEN+2, beta in S_GEN+6.  The
    // last pass forms D = -q and <G, D> (S_GEN+10) for the descent check.
    auto two_loop = [&]() {
      std::vector<int> order;
      for (int t = 0; t < A.count; ++t) order.push_back((A.head - 1 - t + mem) % mem);
      const int mc = (int)order.size();
      int cur = 0;
      PrevSums prev{};
      auto chain = [&](int k, int dv0, int q0, int q1 = 0, int q2 = 0) {
        prev = PrevSums{pbuf[cur], rg, k, {1.0, 1.0, 1.0}, {q0, q1, q2}, {dv0, -1, -1}};
        cur ^= 1;
      };
      if (mc > 0) {
        const int k0 = order[0];
        if (fresh_pair) {
          // the newest pair and G came from the last step: its pair kernel left
          // the three starting sums in part_pair (cur stays 0: the first pass
          // writes pbuf[0])
          prev = PrevSums{part_pair, rg, 3, {1.0, 1.0, 1.0}, {S_GEN + 16, S_GEN + 1, S_GEN + 2},
                          {A.sy[k0], -1, -1}};
        } else {
          dots3_kernel<<<rg, kBlock, 0, s>>>(Nc, r, F.ld, A.S[k0].p, A.G.p, A.S[k0].p, A.Y[k0].p,
                                             A.Y[k0].p, A.Y[k0].p, 3, pbuf[cur]);
          chain(3, A.sy[k0], S_GEN + 16, S_GEN + 1, S_GEN + 2);
        }
        for (int t = 0; t < mc; ++t) {
          // q = -alpha_t Y_t + q; on the last pass q *= <S,Y>/<Y,Y> of the newest pair
          const bool last = t == mc - 1;
          const double* u = last ? A.Y[order[mc - 1]].p : A.S[order[t + 1]].p;
          lbfgs_first_kernel<<<rg, kBlock, 0, s>>>(Nc, r, F.ld, P.sc.p, S_GEN + 16 + t, -1.0,
                                                   A.Y[order[t]].p, t == 0 ? A.G.p : A.Q.p, A.Q.p,
                                                   last ? 1 : 0, S_GEN + 1, S_GEN + 2, u, pbuf[cur],
                                                   prev);
          if (last) chain(1, A.sy[order[mc - 1]], S_GEN + 6);
          else chain(1, A.sy[order[t + 1]], S_GEN + 16 + t + 1);
        }
        for (int t = mc - 1; t >= 0; --t) {
          // q += (alpha_t - beta_t) S_t, then the next beta's dot, or D = -q
          if (t > 0) {
            lbfgs_second_kernel<<<rg, kBlock, 0, s>>>(Nc, r, F.ld, P.sc.p, S_GEN + 16 + t, S_GEN + 6,
                                                      A.S[order[t]].p, A.Q.p, A.Q.p,
                                                      A.Y[order[t - 1]].p, nullptr, nullptr,
                                                      pbuf[cur], prev);
            chain(1, A.sy[order[t - 1]], S_GEN + 6);
          } else {
            lbfgs_second_kernel<<<rg, kBlock, 0, s>>>(Nc, r, F.ld, P.sc.p, S_GEN + 16, S_GEN + 6,
                                                      A.S[order[0]].p, A.Q.p, A.Q.p, nullptr,
                                                      A.D.p, A.G.p, part_gd, prev);
          }
        }
      } else {
        lbfgs_second_kernel<<<rg, kBlock, 0, s>>>(Nc, r, F.ld, P.sc.p, 0, 0, nullptr, A.G.p, nullptr,
                                                  nullptr, A.D.p, A.G.p, part_gd, prev);
      }
      HIPCHK(hipGetLastError());
    };
    // the exact line search's maps and sums; one host read (slots S_GEN+1 ..
    // S_GEN+nread)
    // PAIR with a diagonal C: C D is formed inside the sums pass
    const double* cdiag =
        (P.structure == LORADS_STRUCT_PAIR && P.cdiag.n > 0) ? P.cdiag.p : nullptr;
    // PAIR: the two maps and their seven m-vector sums in one pass (nothing
    // m-sized written); otherwise the maps, then the sums
    double hq[4] = {0.0, 0.0, 0.0, 0.0};  // quadratic objective's quartic terms
    const int nls = gf ? ls_blocks_f32(P, r, F.ld) : ls_blocks(P, r);
    if (A.lsp.n < (size_t)7 * nls) A.lsp.alloc((size_t)7 * nls);
    auto line_search = [&](int nread) {
      bool fused;
      if (gf) {
        // the direction's FP32 copy (D changes before every search)
        cast_rows(A.D.p, D32.p);
        op_linesearch_pair_f32(P, U32.p, D32.p, r, F.ld, P.zbuf.p, P.lam.p, A.lsp.p, s);
        fused = true;
      } else {
        fused = op_linesearch_pair(P, U, A.D.p, r, F.ld, P.zbuf.p, P.lam.p, A.lsp.p, s);
      }
      if (!fused) op_forward_pair(P, U, A.D.p, r, F.ld, A.p1.p, A.p2.p, s);
      if (!cdiag)
        op_adjoint<double>(P, (const double*)nullptr, 1.0, A.D.p, r, F.ld, A.CD.p, F.ld, 1.0, s);
      // the two maps, and C D (a product with C alone)
      info.op_bytes += 2 * bytes_forward(P, r, gf ? 4 : 8) + bytes_cprod(P, r, 8);
      if (P.mu != 0.0) {
        // the quadratic objective's quartic terms (U^T U is the last gradient's)
        gram_small<double>(P, n, r, r, U, F.ld, A.D.p, F.ld, A.gUD.p, s);
        gram_small<double>(P, n, r, r, A.D.p, F.ld, A.D.p, F.ld, A.gDD.p, s);
        quad_coefs<<<1, kBlock, 0, s>>>(r, A.gUU.p, A.gUD.p, A.gDD.p, P.sc.p, S_QUAD);
        HIPCHK(hipGetLastError());
      }
      linesearch_slots(P, n, r, F.ld, A.CD.p, U, A.D.p, P.zbuf.p, A.p1.p, A.p2.p, P.lam.p,
                       S_GEN + 1, s, part_gd, cdiag, h, nread, fused ? A.lsp.p : nullptr,
                       fused ? nls : 0);
      if (P.mu != 0.0) read_slots(P, S_QUAD, hq, 4, s);
    };
    // A step's curvature pair enters the memory at once, before its <S, Y>
    // is known on the host, so the next direction and line search are queued
    // without waiting for it.  The host reads <S, Y> and ||G||^2 (slots
    // S_GEN+11, S_GEN+12) with the line search's sums: a pair with
    // <S, Y> <= 0 is taken out again (the buffers it displaced are untouched
    // until the next step) and the direction recomputed, so the iterates are
    // those of the plain order.
    bool pending = false;
    int undo_head = 0, undo_count = 0;
    // applies the pending pair's test; true when the pair was taken out
    auto resolve = [&](double sy, double gg) {
      pending = false;
      gnorm2 = gg;
      if (sy > 0.0) return false;
      fresh_pair = false;
      A.head = undo_head;
      A.count = undo_count;
      std::swap(A.S[undo_head], A.Sn);
      std::swap(A.Y[undo_head], A.Yn);
      std::swap(A.sy[undo_head], A.sy_n);
      return true;
    };
    // top-of-iteration test: true when the inner loop ends here
    auto stop_test = [&]() {
      const double gnorm = std::sqrt(gnorm2);
      if (!std::isfinite(gnorm)) fail(LORADS_ENUMERIC, "non-finite gradient in phase I");
      if (gnorm / (1.0 + c_fro) <= tol) { conv = true; return true; }
      return it >= cap;
    };
    while (true) {
      if (pending && it >= cap) {
        read_slots(P, S_GEN + 11, h, 2, s);
        resolve(h[0], h[1]);
      }
      if (!pending && stop_test()) break;
      two_loop();
      line_search(12);
      if (pending) {
        const bool out = resolve(h[10], h[11]);
        if (stop_test()) break;
        if (out) {
          two_loop();
          line_search(10);
        }
      }
      // The line search also returns <G, D>: a direction that is not a
      // descent direction is replaced by -G (memory cleared) and the search
      // repeated, as is a quasi-Newton step whose exact minimiser is not
      // positive.
      double alpha = 0.0;
      bool checked = false;
      for (int attempt = 0; attempt < 3; ++attempt) {
        if (attempt > 0) line_search(checked ? 9 : 10);
        if (!checked) {
          checked = true;
          if (!(h[9] < 0.0)) {
            axpby<double, double><<<gridN(N), kBlock, 0, s>>>(N, -1.0, A.G.p, 0.0, A.D.p);
            A.head = A.count = 0;
            continue;
          }
        }
        const double c1 = h[0], c2 = h[1];
        const double p22 = h[2], p12 = h[3], p11 = h[4], p02 = h[5], p01 = h[6], l1 = h[7],
                     l2 = h[8];
        const double mu = P.mu;
        const double q4 = 0.5 * rho * p22 + 0.5 * mu * hq[3];
        const double q3 = rho * p12 + mu * hq[2];
        const double q2 = c2 + l2 + 0.5 * rho * (p11 + 2.0 * p02) + 0.5 * mu * hq[1];
        const double q1 = c1 + l1 + rho * p01 + mu * hq[0];
        alpha = quartic_step(q1, q2, q3, q4);
        if (alpha > 0.0 || A.count == 0) break;
        // retry along steepest descent with a cleared memory
        axpby<double, double><<<gridN(N), kBlock, 0, s>>>(N, -1.0, A.G.p, 0.0, A.D.p);
        A.head = A.count = 0;
      }
      if (!(alpha > 0.0)) break;
      // S = alpha D; U += S; new gradient; Y = G_new - G; <S, Y> into the
      // pair's own slot (and S_GEN+11), ||G_new||^2 into S_GEN+12.  The pair
      // enters the memory now (the oldest pair is dropped when full) and
      // leaves it again at the next read if <S, Y> <= 0.
      lbfgs_step_kernel<<<gridN(N), kBlock, 0, s>>>(N, alpha, A.D.p, A.Sn.p, U);
      if (gf) cast_rows(U, U32.p);
      alm_gradient(P, A, U, A.Gn.p, rho, s, info.op_bytes);
      lbfgs_pair_kernel<<<rg, kBlock, 0, s>>>(Nc, r, F.ld, A.Gn.p, A.G.p, A.Yn.p, A.Sn.p,
                                              part_pair);
      pair_finish<<<1, kBlock, 0, s>>>(rg, part_pair, P.sc.p, A.sy_n, S_GEN + 11, S_GEN + 12);
      HIPCHK(hipGetLastError());
      undo_head = A.head;
      undo_count = A.count;
      std::swap(A.S[A.head], A.Sn);
      std::swap(A.Y[A.head], A.Yn);
      std::swap(A.sy[A.head], A.sy_n);
      A.head = (A.head + 1) % mem;
      A.count = std::min(A.count + 1, mem);
      pending = true;
      fresh_pair = true;
      std::swap(A.G, A.Gn);
      ++it;
    }
    inner_total += it;
    // z of the current U is in zbuf (from the last gradient evaluation)
    v = host_norm_zb(P, s) / (1.0 + P.b_inf);
    if (o.verbose > 1)
      fprintf(stderr, "[lorads] ALM outer %d: r=%d rho=%.3g inner=%d conv=%d v=%.3e\n", outer, r,
              rho, it, (int)conv, v);
    if (warm_pending) {
      warm_pending = false;
      if (!(v < v_start)) {
        HIPCHK(hipMemcpyAsync(U, U_start.p, (size_t)n * F.ld * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (gf) cast_rows(U, U32.p);
        P.lam.zero(s);
        refresh_inc_lam(P, s);
        rho = rho_start;
        info.warm_fallback = 1;
        op_forward<double>(P, U, U, r, F.ld, P.zbuf.p, 1.0, s);
        info.op_bytes += bytes_forward(P, r, 8);
        v = host_norm_zb(P, s) / (1.0 + P.b_inf);
        continue;
      }
    }
    // a hard inner solve raises the rank only while Phase I goes on: once the
    // infeasibility meets the switching tolerance the phase ends
    if (!conv && r < r_cap && it >= cap && v > o.switch_tol) {
      const int r_new = std::min((int)std::ceil(o.rank_factor * r), r_cap);
      adot(U, U, 1.0, S_GEN, s);
      read_slots(P, S_GEN, h, 1, s);
      const double sigma = 1e-3 * std::sqrt(h[0]) / std::sqrt((double)n * r);
      // the kernel reads the compact n x r master that F.store has just
      // written (the working copy U may have padded rows)
      F.store(P, r, s);
      DevBuf<double> Unew;
      Unew.alloc((size_t)n * r_new);
      grow_rank_kernel<<<gridN((size_t)n * r_new), kBlock, 0, s>>>(n, r, r_new, P.U.p, Unew.p, sigma,
                                                                   o.seed, (uint64_t)growths);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
      P.U = std::move(Unew);
      r = r_new;
      P.rank = r;
      F.load(P, r, alm_ld(P, r), s);
      U = F.U;
      alm_alloc(A, n, m, r, F.ld, o.lbfgs_mem, s);
      setup_mixed();
      ++growths;
      op_forward<double>(P, U, U, r, F.ld, P.zbuf.p, 1.0, s);
      info.op_bytes += bytes_forward(P, r, 8);
      v = host_norm_zb(P, s) / (1.0 + P.b_inf);
      continue;
    }
    if (v <= o.alm_eta * v_ref) {
      dual_update_slot(P, P.zbuf.p, rho, P.lam.p, S_GEN, s);
      refresh_inc_lam(P, s);
      v_ref = v;
    } else {
      rho *= o.alm_rho_factor;
    }
    ++outer;
  }
  F.store(P, r, s);
  info.alm_outer = outer;
  info.alm_inner = inner_total;
  info.growths = growths;
  info.rho_alm = rho;
  info.pinf_alm = v;
}

// ===========================================================================
// Phase II: ADMM (Algorithm 1) with CG subproblem solves
// ===========================================================================
// CG work buffers in the CG layout (leading dimension ld = cg_ld(P, r), zero
// padding that no kernel writes)
// For PAIR problems W holds rows [W_t | P_t] (stride ldw = 2 ld) so that the
// CG operator reads both factors of a partner from one line; P2 points at the
// direction's half.
template <typename T>
struct CgBufs {
  DevBuf<T> R, X, Pd, Q, W, t;
  DevBuf<char> xparts;  // per-XCD partials of the split CG operator (large factors)
  int ld = 0, ldw = 0;
  T* P2 = nullptr;
  void alloc(const Problem& P, int n, int m, int ld_, bool interleave, hipStream_t s) {
    ld = ld_;
    ldw = interleave ? 2 * ld : ld;
    const size_t N = (size_t)n * ld;
    R.alloc(N); X.alloc(N); Pd.alloc(N); Q.alloc(N); W.alloc((size_t)n * ldw); t.alloc(m);
    R.zero(s); X.zero(s); Pd.zero(s); Q.zero(s); W.zero(s);
    P2 = interleave ? W.p + ld : nullptr;
    const size_t xb = cg_xparts_bytes(P, ld, (int)sizeof(typename OpAcc<T>::type));
    if (xb) xparts.alloc(xb);
  }
};

// new = W + argmin-correction: solves M_W D = -(C + A*(lam + rho (A(W W^T) - b))) W
template <typename T>
static int half_step(Problem& P, const double* W, double* out, int r, double rho, double gamma,
                     double tol, int maxit, CgBufs<T>& B, DevBuf<double>& R64, hipStream_t s,
                     SolveInfo& info, const double* Wp = nullptr, double* outp = nullptr,
                     int ldp = 0, double* gW = nullptr) {
  const int ld = B.ld;
  const size_t N = (size_t)P.n * ld;  // CG layout
  double* R = std::is_same<T, double>::value ? reinterpret_cast<double*>(B.R.p) : R64.p;
  if (grad_pair_ready(P)) {
    // the gradient form needs no forward map here (z is recomputed after the
    // step); it reads the zero-padded copy of W when there is one
    if (Wp) op_grad_pair(P, Wp, r, ldp, rho, R, ld, -1.0, s);
    else op_grad_pair(P, W, r, r, rho, R, ld, -1.0, s);
    info.op_bytes += bytes_grad_pair(P, r);
  } else {
    op_forward_w(P, W, W, r, r, P.zbuf.p, P.wbuf.p, P.lam.p, rho, s);
    op_adjoint<double>(P, P.wbuf.p, 1.0, W, r, r, R, ld, -1.0, s);
    info.op_bytes += bytes_forward(P, r, 8) + bytes_adjoint(P, r, 8, true);
  }
  if (P.mu != 0.0) {
    // quadratic objective: grad f(W W^T) W gains mu W (W^T W); the operator
    // gains mu P (W^T W)
    gram_small<double>(P, P.n, r, r, W, r, W, r, gW, s);
    add_xg<double, double><<<grid_for((size_t)P.n * r), kBlock, 0, s>>>(P.n, r, r, W, r, gW, -P.mu, R, ld);
    HIPCHK(hipGetLastError());
  }
  if constexpr (!std::is_same<T, double>::value)
    convert_kernel<double, float><<<gridN(N), kBlock, 0, s>>>(N, R64.p, B.R.p);
  copy_rows<double, T><<<gridN((size_t)P.n * r), kBlock, 0, s>>>(P.n, r, W, r, B.W.p, B.ldw);
  HIPCHK(hipMemsetAsync(B.X.p, 0, N * sizeof(T), s));
  double rel;
  int it;
  {
    CgXpartsScope xs(P, B.xparts.n ? B.xparts.p : nullptr);
    it = cg_run<T>(P, B.W.p, B.ldw, r, ld, rho, gamma, B.R.p, B.X.p, B.Pd.p, B.P2, B.Q.p, B.t.p,
                   tol, maxit, s, &rel, &info.op_bytes, P.mu != 0.0 ? gW : nullptr);
  }
  add_rows<double, T><<<gridN((size_t)P.n * r), kBlock, 0, s>>>(P.n, r, W, r, B.X.p, ld, out);
  if (outp)
    copy_rows<double, double><<<gridN((size_t)P.n * r), kBlock, 0, s>>>(P.n, r, out, r, outp, ldp);
  HIPCHK(hipGetLastError());
  return it;
}

template <typename T>
static void phase2_t(Problem& P, const lorads_options& o, double rho, SolveInfo& info,
                     hipStream_t s, Clock::time_point t_start) {
  const int n = P.n, m = P.m, r = P.rank;
  const size_t N = (size_t)n * r;
  // U and V start equal to the phase-I factor
  P.V.alloc(N);
  HIPCHK(hipMemcpyAsync(P.V.p, P.U.p, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  DevBuf<double> Vold, R64;
  Vold.alloc(N);
  const int ldc = cg_ld(P, r, (int)sizeof(T));
  const size_t Nc = (size_t)n * ldc;
  if constexpr (!std::is_same<T, double>::value) {
    R64.alloc(Nc);
    R64.zero(s);
  }
  CgBufs<T> B;
  B.alloc(P, n, m, ldc, P.structure == LORADS_STRUCT_PAIR, s);
  DevBuf<double> gW;  // W^T W of the quadratic objective
  if (P.mu != 0.0) gW.alloc((size_t)r * r);
  refresh_inc_lam(P, s);
  // PAIR: zero-padded FP64 copies of U and V (rows of whole 64-byte sectors),
  // kept equal to the masters, for the gradient form and the dual update's
  // forward map (the same results as on the compact masters)
  const int ldp = alm_ld(P, r);
  DevBuf<double> Up, Vp;
  const bool padded = ldp != r;
  if (padded) {
    Up.alloc((size_t)n * ldp);
    Vp.alloc((size_t)n * ldp);
    Up.zero(s);
    Vp.zero(s);
    copy_rows<double, double><<<gridN(N), kBlock, 0, s>>>(n, r, P.U.p, r, Up.p, ldp);
    copy_rows<double, double><<<gridN(N), kBlock, 0, s>>>(n, r, P.V.p, r, Vp.p, ldp);
    HIPCHK(hipGetLastError());
  }
  const int maxit = (int)std::min<long long>((long long)N, o.cg_maxit);
  const double floor = (std::is_same<T, double>::value) ? o.cg_tol_floor : std::max(o.cg_tol_floor, 1e-6);
  double kkt = INFINITY, pinf = INFINITY, dres = INFINITY, gamma = gamma_of(P, o, rho);
  int k = 0;
  long long cg_total = 0;
  double h[4];
  info.status = LORADS_MAXITER;
  while (k < o.max_admm_iter) {
    gamma = gamma_of(P, o, rho);
    const double tol = std::min(o.cg_tol_max, std::max(floor, o.cg_tol_kkt * kkt));
    HIPCHK(hipMemcpyAsync(Vold.p, P.V.p, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    dot_to_slot<double, double>(P, N, Vold.p, Vold.p, 1.0, S_GEN + 2, s);
    const int iu = half_step<T>(P, P.V.p, P.U.p, r, rho, gamma, tol, maxit, B, R64, s, info,
                                padded ? Vp.p : nullptr, padded ? Up.p : nullptr, ldp, gW.p);
    const int iv = half_step<T>(P, P.U.p, P.V.p, r, rho, gamma, tol, maxit, B, R64, s, info,
                                padded ? Up.p : nullptr, padded ? Vp.p : nullptr, ldp, gW.p);
    cg_total += iu + iv;
    // z = A(U V^T); lam += rho (z - b); residual norms
    if (padded) op_forward<double>(P, Up.p, Vp.p, r, ldp, P.zbuf.p, 1.0, s);
    else op_forward<double>(P, P.U.p, P.V.p, r, r, P.zbuf.p, 1.0, s);
    info.op_bytes += bytes_forward(P, r, 8);
    dual_update_slot(P, P.zbuf.p, rho, P.lam.p, S_GEN, s);
    refresh_inc_lam(P, s);
    axpby<double, double><<<gridN(N), kBlock, 0, s>>>(N, 1.0, P.V.p, -1.0, Vold.p);  // V+ - V
    dot_to_slot<double, double>(P, N, Vold.p, Vold.p, 1.0, S_GEN + 1, s);
    HIPCHK(hipGetLastError());
    read_slots(P, S_GEN, h, 3, s);
    pinf = std::sqrt(h[0]) / (1.0 + P.b_inf);
    dres = gamma * std::sqrt(h[1]) / (1.0 + std::sqrt(h[2]));
    if (!std::isfinite(pinf) || !std::isfinite(dres)) fail(LORADS_ENUMERIC, "non-finite residual in ADMM");
    kkt = std::max(pinf, dres);
    ++k;
    if (o.verbose > 1)
      fprintf(stderr, "[lorads] ADMM %d: rho=%.4g gamma=%.4g cg=%d+%d pinf=%.3e dres=%.3e\n", k,
              rho, gamma, iu, iv, pinf, dres);
    if (kkt < o.eps) { info.status = LORADS_OK; break; }
    if (k % o.rho_every == 0 && rho < o.rho_max) rho = std::min(o.rho_growth * rho, o.rho_max);
    if (o.time_limit > 0 && secs(t_start, Clock::now()) > o.time_limit) {
      info.status = LORADS_TIMELIMIT;
      break;
    }
  }
  info.admm_iters = k;
  info.cg_iters = cg_total;
  info.kkt = kkt;
  info.pinf_stop = pinf;
  info.dres_stop = dres;
  info.rho = rho;
  info.gamma = gamma;
}

void phase2(Problem& P, const lorads_options& o, double rho, SolveInfo& info, hipStream_t s,
            std::chrono::steady_clock::time_point t_start) {
  if (o.gamma_rule == 1 && !(o.gamma_fixed > 0)) cost_norm2(P, s);
  if (o.precision != LORADS_F64)
    phase2_t<float>(P, o, rho, info, s, t_start);
  else
    phase2_t<double>(P, o, rho, info, s, t_start);
}

int rank_cap(const Problem& P, const lorads_options& o) {
  int cap = o.r_max > 0 ? o.r_max : (int)std::floor(std::sqrt(2.0 * P.m));
  cap = std::min(cap, P.n);
  cap = std::min(cap, 256);
  return std::max(cap, 1);
}

}  // namespace lorads
