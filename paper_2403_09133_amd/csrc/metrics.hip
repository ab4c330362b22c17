// End-of-solve measures (Appendix B): primal infeasibility, dual infeasibility
// through the smallest eigenvalue of the dual slack (Lanczos on the adjoint
// kernel), duality gap; and the tall-skinny Gram products A^T B on FP64 MFMA.
#include <algorithm>

#include "kernels.hpp"
#include "kernels_quad.hpp"
#include "solver.hpp"

namespace lorads {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Gram G = A^T B.  One wave accumulates a 16 x 16 output tile over a strided
// set of 4-row slabs with v_mfma_f64_16x16x4f64: lane l supplies
// A[row0 + l/16][i0 + l%16] as the (M x K) operand and B[row0 + l/16][j0 + l%16]
// as the (K x N) operand; accumulator element v of lane l holds
// D[l/16 + 4 v][l%16] (layout checked against A^T B on the host).
// Per-block tiles are reduced in LDS, blocks write partial tiles, and a
// second kernel sums them in block order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) gram_partial(const double* __restrict__ A,
                                                    const double* __restrict__ B, int64_t n,
                                                    int ra, int rb, int lda, int ldb,
                                                    double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ti = blockIdx.y / ((rb + 15) / 16), tj = blockIdx.y % ((rb + 15) / 16);
  const int ia = ti * 16 + (lane & 15), jb = tj * 16 + (lane & 15);
  const int krow = lane >> 4;
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  const int64_t slabs = (n + 3) / 4;
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t sl = (int64_t)blockIdx.x * 4 + wid; sl < slabs; sl += stride) {
    const int64_t row = sl * 4 + krow;
    const double a = (row < n && ia < ra) ? A[row * lda + ia] : 0.0;
    const double b = (row < n && jb < rb) ? B[row * ldb + jb] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  __shared__ double tile[4][16][16];
  for (int v = 0; v < 4; ++v) tile[wid][(lane >> 4) + 4 * v][lane & 15] = acc[v];
  __syncthreads();
  const int t = threadIdx.x;  // 256 threads = one 16 x 16 tile
  const int i = t / 16, j = t % 16;
  const double s = tile[0][i][j] + tile[1][i][j] + tile[2][i][j] + tile[3][i][j];
  const int gi = ti * 16 + i, gj = tj * 16 + j;
  if (gi < ra && gj < rb) part[((size_t)blockIdx.x * ra + gi) * rb + gj] = s;
}

__global__ void gram_finish(const double* __restrict__ part, int nblk, int ra, int rb,
                            double* __restrict__ G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ra * rb) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * ra * rb + t];
  G[t] = s;
}

void gram(const double* A, const double* B, int64_t n, int ra, int rb, int lda, int ldb,
          double* G, hipStream_t s) {
  if (ra < 1 || rb < 1 || n < 0) fail(LORADS_EINVAL, "gram: bad sizes");
  const int tiles = ((ra + 15) / 16) * ((rb + 15) / 16);
  int nblk = (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + 15) / 16));
  DevBuf<double> part;
  part.alloc((size_t)nblk * ra * rb);
  gram_partial<<<dim3(nblk, tiles), 256, 0, s>>>(A, B, n, ra, rb, lda, ldb, part.p);
  gram_finish<<<(ra * rb + 255) / 256, 256, 0, s>>>(part.p, nblk, ra, rb, G);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Lanczos with full reorthogonalisation for lambda_min(C + A*(lam)).
// ---------------------------------------------------------------------------
// c[i] = <Q_i, y>, i < k (one block per basis vector)
__global__ void __launch_bounds__(256) basis_dots(int n, int k, const double* __restrict__ Qb,
                                                  const double* __restrict__ y,
                                                  double* __restrict__ c) {
  __shared__ double sh[4];
  const int i = blockIdx.x;
  if (i >= k) return;
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += 256) s += Qb[(size_t)i * n + t] * y[t];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) c[i] = s;
}

// y -= sum_{i<k} c[i] Q_i
__global__ void __launch_bounds__(256) basis_sub(int n, int k, const double* __restrict__ Qb,
                                                 const double* __restrict__ c,
                                                 double* __restrict__ y) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  double s = y[t];
  for (int i = 0; i < k; ++i) s -= c[i] * Qb[(size_t)i * n + t];
  y[t] = s;
}

__global__ void start_vector(int n, double* __restrict__ q) {
  // deterministic pseudo-random start (SplitMix64 finaliser of the index)
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const uint64_t z = splitmix_mix(0x243F6A8885A308D3ull + (uint64_t)(t + 1) * 0x9E3779B97F4A7C15ull);
  q[t] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
}

// number of eigenvalues of the tridiagonal (a, b) below x (Sturm sequence)
static int sturm_count(const std::vector<double>& a, const std::vector<double>& b, int k, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    const double bb = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
    d = a[i] - x - ((i > 0) ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0) ++cnt;
  }
  return cnt;
}

static double tridiag_min(const std::vector<double>& a, const std::vector<double>& b, int k) {
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < k; ++i) {
    const double rad = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - rad);
    hi = std::max(hi, a[i] + rad);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(lo)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(a, b, k, mid) >= 1) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Residual bound of the smallest Ritz pair: beta_k |s_k|, with s_k the last
// component of the unit eigenvector of T for theta (inverse iteration on the
// tridiagonal, shifted just below theta).  The smallest eigenvalue of the
// operator lies within this bound of a Ritz value.
static double ritz_residual(const std::vector<double>& a, const std::vector<double>& b, int k,
                            double theta, double beta) {
  if (k == 1) return std::fabs(beta);
  double scale = 0.0;
  for (int i = 0; i < k; ++i) scale = std::max(scale, std::fabs(a[i]) + 2.0 * (i < k - 1 ? std::fabs(b[i]) : 0.0));
  const double shift = theta - 1e-13 * std::max(1.0, scale);
  std::vector<double> x(k, 1.0), d(k), u(k), rhs(k);
  for (int it = 0; it < 3; ++it) {
    // Thomas algorithm on (T - shift I) x_new = x
    for (int i = 0; i < k; ++i) {
      const double sub = i > 0 ? b[i - 1] : 0.0;
      double di = a[i] - shift - (i > 0 ? sub * u[i - 1] : 0.0);
      if (di == 0.0) di = 1e-300;
      d[i] = di;
      u[i] = i < k - 1 ? b[i] / di : 0.0;
      rhs[i] = (x[i] - (i > 0 ? sub * rhs[i - 1] : 0.0)) / di;
    }
    for (int i = k - 1; i >= 0; --i) x[i] = rhs[i] - (i < k - 1 ? u[i] * x[i + 1] : 0.0);
    double nrm = 0.0;
    for (double v : x) nrm += v * v;
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return INFINITY;
    for (double& v : x) v /= nrm;
  }
  return std::fabs(beta * x[k - 1]);
}

// ||C||_2 by the power method: v <- C v / ||C v|| from a fixed start (entries
// 1 + ((i 2654435761) mod 1024) / 1024, normalised), the estimate ||C v|| with
// ||v|| = 1 rising to max |eig(C)|; stops when it changes by less than 1e-12
// relative, at C v = 0, or after 1000 products.  The products are the adjoint
// with no multiplier (c_scale C V at rank 1).
double cost_norm2(Problem& P, hipStream_t s) {
  if (P.c_norm2 >= 0.0) return P.c_norm2;
  const int n = P.n;
  std::vector<double> h0(n);
  double nn = 0.0;
  for (int i = 0; i < n; ++i) {
    h0[i] = 1.0 + (double)(((uint64_t)i * 2654435761ull) % 1024ull) / 1024.0;
    nn += h0[i] * h0[i];
  }
  nn = std::sqrt(nn);
  for (int i = 0; i < n; ++i) h0[i] /= nn;
  DevBuf<double> v, w;
  v.upload(h0, s);
  w.alloc(n);
  double est = 0.0, h[1];
  for (int it = 0; it < 1000; ++it) {
    op_adjoint<double>(P, (const double*)nullptr, 1.0, v.p, 1, 1, w.p, 1, 1.0, s);
    dot_to_slot<double, double>(P, (size_t)n, w.p, w.p, 1.0, S_GEN, s);
    read_slots(P, S_GEN, h, 1, s);
    const double nrm = std::sqrt(h[0]);
    if (!std::isfinite(nrm)) fail(LORADS_ENUMERIC, "non-finite product in the estimate of ||C||_2");
    if (nrm == 0.0) { est = 0.0; break; }
    axpby<double, double><<<grid_for((size_t)n), kBlock, 0, s>>>((size_t)n, 1.0 / nrm, w.p, 0.0, v.p);
    HIPCHK(hipGetLastError());
    const bool done = it > 0 && std::fabs(nrm - est) <= 1e-12 * nrm;
    est = nrm;
    if (done) break;
  }
  P.c_norm2 = est;
  return est;
}

double dual_lambda_min(Problem& P, const double* lam, int max_steps, hipStream_t s,
                       const double* Uh, int r) {
  const int n = P.n;
  const int kmax = std::max(2, std::min(max_steps, n));
  const bool quad = Uh != nullptr && P.mu != 0.0 && r > 0;
  DevBuf<double> Qb, y, c, tq;
  if (quad) tq.alloc(r);
  Qb.alloc((size_t)kmax * n);
  y.alloc(n);
  c.alloc(kmax + 1);
  Qb.zero(s);
  const int gridn = (n + 255) / 256;
  start_vector<<<gridn, 256, 0, s>>>(n, Qb.p);
  dot_to_slot<double, double>(P, n, Qb.p, Qb.p, 1.0, S_GEN, s);
  double h[2];
  read_slots(P, S_GEN, h, 1, s);
  axpby<double, double><<<gridn, 256, 0, s>>>(n, 0.0, Qb.p, 1.0 / std::sqrt(h[0]), Qb.p);
  std::vector<double> al, be;
  double theta = 0.0, anorm = 0.0;
  int k = 0;
  for (; k < kmax; ++k) {
    double* qk = Qb.p + (size_t)k * n;
    op_adjoint<double>(P, lam, 1.0, qk, 1, 1, y.p, 1, 1.0, s);
    if (quad) {
      // + mu Uh (Uh^T q_k)
      gram_small<double>(P, n, r, 1, Uh, r, qk, 1, tq.p, s);
      add_xg<double, double><<<grid_for((size_t)n), kBlock, 0, s>>>(n, r, 1, Uh, r, tq.p, P.mu, y.p, 1);
    }
    // full reorthogonalisation, twice (classical Gram-Schmidt); the first
    // pass's coefficient on q_k is alpha_k = <q_k, S q_k>
    double ak = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      basis_dots<<<k + 1, 256, 0, s>>>(n, k + 1, Qb.p, y.p, c.p);
      if (pass == 0)
        HIPCHK(hipMemcpyAsync(&ak, c.p + k, sizeof(double), hipMemcpyDeviceToHost, s));
      basis_sub<<<gridn, 256, 0, s>>>(n, k + 1, Qb.p, c.p, y.p);
    }
    dot_to_slot<double, double>(P, n, y.p, y.p, 1.0, S_GEN, s);
    read_slots(P, S_GEN, h, 1, s);
    h[1] = ak;
    al.push_back(ak);
    const double beta = std::sqrt(h[0]);
    theta = tridiag_min(al, be, k + 1);
    anorm = std::max(anorm, std::fabs(ak) + beta + (k > 0 ? be[k - 1] : 0.0));
    // stop once the smallest Ritz value is within 1e-12 of the operator's
    // scale of an eigenvalue (checked every 5 steps), or on an invariant
    // subspace
    if (k % 5 == 4 && ritz_residual(al, be, k + 1, theta, beta) <= 1e-12 * std::max(1.0, anorm)) {
      ++k;
      break;
    }
    if (!(beta > 1e-13 * std::max(1.0, anorm))) { ++k; break; }
    be.push_back(beta);
    if (k + 1 < kmax)
      axpby<double, double><<<gridn, 256, 0, s>>>(n, 1.0 / beta, y.p, 0.0, Qb.p + (size_t)(k + 1) * n);
  }
  HIPCHK(hipGetLastError());
  return theta;
}

// ---------------------------------------------------------------------------
void final_metrics(Problem& P, lorads_result& res, hipStream_t s, int lanczos_steps) {
  const int n = P.n, m = P.m, r = P.rank;
  const size_t N = (size_t)n * r;
  DevBuf<double> Uh, CU;
  Uh.alloc(N);
  CU.alloc(N);
  // U_hat = (U + V)/2
  add_kernel<double, double, double><<<grid_for(N), kBlock, 0, s>>>(N, P.U.p, P.V.p, Uh.p);
  axpby<double, double><<<grid_for(N), kBlock, 0, s>>>(N, 0.0, Uh.p, 0.5, Uh.p);
  op_forward<double>(P, Uh.p, Uh.p, r, r, P.zbuf.p, 1.0, s);
  dual_update_slot(P, P.zbuf.p, 0.0, P.lam.p, S_GEN, s);
  op_adjoint<double>(P, (const double*)nullptr, 1.0, Uh.p, r, r, CU.p, r, 1.0, s);
  dot_to_slot<double, double>(P, N, CU.p, Uh.p, 1.0, S_GEN + 1, s);
  dot_to_slot<double, double>(P, m, P.b.p, P.lam.p, -1.0, S_GEN + 2, s);
  HIPCHK(hipGetLastError());
  double h[3];
  read_slots(P, S_GEN, h, 3, s);
  const double zb = std::sqrt(h[0]);
  // quadratic objective: f(X) = <C, X> + (mu/2) ||X||^2 with ||X||^2 = ||Uh^T Uh||^2;
  // the measures are taken at grad f(X) = C + mu X (<grad f(X), X> in the gap)
  double xx = 0.0;
  if (P.mu != 0.0) {
    DevBuf<double> g;
    g.alloc((size_t)r * r);
    gram_small<double>(P, n, r, r, Uh.p, r, Uh.p, r, g.p, s);
    std::vector<double> gh((size_t)r * r);
    HIPCHK(hipMemcpyAsync(gh.data(), g.p, gh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (double v : gh) xx += v * v;
  }
  res.obj = h[1] + 0.5 * P.mu * xx;
  const double gx = h[1] + P.mu * xx;
  res.dual_obj = h[2];
  res.pinf = zb / (1.0 + P.b_1);
  res.lambda_min = lanczos_steps > 0 ? dual_lambda_min(P, P.lam.p, lanczos_steps, s, Uh.p, r) : NAN;
  res.dinf = std::fabs(std::min(0.0, res.lambda_min)) / (1.0 + P.c_1);
  res.gap = (gx - res.dual_obj) / (1.0 + std::fabs(gx) + std::fabs(res.dual_obj));
}

}  // namespace lorads
