// Batched two-phase solve of many diagonal-constraint SDPs (MaxCut) in one
// persistent launch: workgroup b runs the whole method on instance b -- the
// Burer-Monteiro augmented Lagrangian warm start with L-BFGS, exact quartic
// line search and rank growth, the switch, and the ADMM of Algorithm 1 with CG
// subproblem solves -- using only workgroup-level synchronisation.  Instances
// of different order share one launch through per-instance descriptors into
// concatenated pools (factor rows strided by the instance's rank capacity).
// The decisions and tolerances are those of the single-instance path.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "batch.hpp"
#include "kernels.hpp"
#include "solver.hpp"

namespace lorads {

// ---------------------------------------------------------------------------
// workgroup reductions
// ---------------------------------------------------------------------------
__device__ double wg_sum(double v) {
  __shared__ double buf[16];
  __shared__ double result;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) buf[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += buf[i];
    result = s;
  }
  __syncthreads();
  return result;
}

// two workgroup sums with one set of barriers (each summed as wg_sum sums it)
__device__ void wg_sum2(double& a, double& b) {
  __shared__ double buf[2][16];
  __shared__ double result[2];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    buf[0][wid] = a;
    buf[1][wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) sa += buf[0][i];
    for (int i = 0; i < nw; ++i) sb += buf[1][i];
    result[0] = sa;
    result[1] = sb;
  }
  __syncthreads();
  a = result[0];
  b = result[1];
}

// Instance view: pointers already offset to the instance.
template <typename T>
struct Inst {
  int n, m, ld, r;
  const int *cptr, *ccol, *dptr, *drow;
  const double *cval, *dcoef, *dsq, *b;
  double c_fro, b_inf, b_1;
};

#define FOR_ROWS(j) for (int j = threadIdx.x; j < I.n; j += blockDim.x)
#define FOR_CONS(i) for (int i = threadIdx.x; i < I.m; i += blockDim.x)
// Factor rows are served by groups of kBG lanes (lane l holds columns l and
// l + kBG; the rank capacity is at most 2 kBG), so the loads of a row are
// contiguous and a row's inner product is a DPP reduction inside the group.
constexpr int kBG = 16;
// workgroup size limit of the batched launch (keeps the kernel's registers
// free of spills)
constexpr int kBatchMaxBlock = 256;
#define FOR_GROUPS(j, cnt) for (int j = (int)threadIdx.x / kBG; j < (cnt); j += (int)blockDim.x / kBG)
#define FOR_RC(j, c) FOR_GROUPS(j, I.n) for (int c = (int)threadIdx.x % kBG; c < I.r; c += kBG)

// Element passes over the active block visit kBU rows per group at a time and
// issue every load of those rows before the first store, so a workgroup keeps
// kBU * blockDim / kBG rows in flight.  Out-of-range rows and columns load from
// a clamped in-row position and are masked.
constexpr int kBU = 4;
struct PassSlots {
  int q[kBU][2];
  bool on[kBU][2];
};
__device__ __forceinline__ void pass_slots(int it, int n, int r, int ld, PassSlots& S) {
  const int l = threadIdx.x % kBG, ng = blockDim.x / kBG;
  const int c0 = min(l, ld - 1), c1 = min(l + kBG, ld - 1);
#pragma unroll
  for (int u = 0; u < kBU; ++u) {
    const int j = it + u * ng;
    const bool rok = j < n;
    const int base = (rok ? j : n - 1) * ld;
    S.q[u][0] = base + c0;
    S.q[u][1] = base + c1;
    S.on[u][0] = rok && l < r;
    S.on[u][1] = rok && l + kBG < r;
  }
}
#define FOR_PASS(it) \
  for (int it = (int)threadIdx.x / kBG; it < I.n; it += kBU * ((int)blockDim.x / kBG))
#define FOR_UH(u, h) _Pragma("unroll") for (int u = 0; u < kBU; ++u) _Pragma("unroll") for (int h = 0; h < 2; ++h)

// Row inner products <X_j, Y_j> of the rows of kBU constraints, it + u * ng
// (ng groups per workgroup), every load issued before the reductions; rows of
// constraints past m repeat the last constraint's row.
template <typename T>
__device__ __forceinline__ void b_row_dots(const Inst<T>& I, int it, const double* X, const double* Y,
                                           double (&s)[kBU]) {
  const int l = threadIdx.x % kBG, ng = blockDim.x / kBG;
  const int c0 = min(l, I.ld - 1), c1 = min(l + kBG, I.ld - 1);
  int base[kBU];
#pragma unroll
  for (int u = 0; u < kBU; ++u) base[u] = I.drow[min(it + u * ng, I.m - 1)] * I.ld;
  double x[kBU][2], y[kBU][2];
#pragma unroll
  for (int u = 0; u < kBU; ++u) {
    x[u][0] = X[base[u] + c0];
    x[u][1] = X[base[u] + c1];
    y[u][0] = Y[base[u] + c0];
    y[u][1] = Y[base[u] + c1];
  }
#pragma unroll
  for (int u = 0; u < kBU; ++u) {
    double t = 0.0;
    if (l < I.r) t += x[u][0] * y[u][0];
    if (l + kBG < I.r) t += x[u][1] * y[u][1];
    s[u] = group_sum<kBG>(t);
  }
}
#define FOR_CPASS(it) \
  for (int it = (int)threadIdx.x / kBG; it < I.m; it += kBU * ((int)blockDim.x / kBG))

// z_i = scale a_i <X_row, Y_row>
template <typename T>
__device__ void b_forward(const Inst<T>& I, const double* X, const double* Y, double* z, double scale) {
  const int l = threadIdx.x % kBG, ng = blockDim.x / kBG;
  FOR_CPASS(it) {
    double s[kBU];
    b_row_dots(I, it, X, Y, s);
#pragma unroll
    for (int u = 0; u < kBU; ++u) {
      const int i = it + u * ng;
      if (l == 0 && i < I.m) z[i] = scale * I.dcoef[i] * s[u];
    }
  }
}

// out_j = os (cs (C V)_j + (sum_{i on row j} w_i a_i) V_j), w may be null
// A group serves kBU rows at once: the lanes load up to kBG entries of each
// row's cost list together, then every step gathers one partner row for each
// of the kBU rows (entry broadcast inside the group), so kBU partner rows are
// in flight per step.
// GRAD: gradient form with V = U: z_i = a_i <U_j, U_j> (the row's inner
// product summed as b_row_dots sums it) and w_i = lam_i + rho (z_i - b_i) of
// the row's constraints are formed in the same pass and z is written, so out
// equals the forward map of w followed by the plain adjoint bit for bit.
template <typename T, bool GRAD = false>
__device__ void b_adjoint(const Inst<T>& I, const double* w, double cs, const double* V,
                          double* out, double os, double* zo = nullptr,
                          const double* lam = nullptr, double rho = 0.0) {
  const int l = threadIdx.x % kBG, ng = blockDim.x / kBG;
  const int c0 = min(l, I.ld - 1), c1 = min(l + kBG, I.ld - 1);
  FOR_PASS(it) {
    int j[kBU], e0[kBU], e1[kBU];
#pragma unroll
    for (int u = 0; u < kBU; ++u) j[u] = min(it + u * ng, I.n - 1);
    int span = 0;
#pragma unroll
    for (int u = 0; u < kBU; ++u) {
      e0[u] = cs != 0.0 ? I.cptr[j[u]] : 0;
      e1[u] = cs != 0.0 ? I.cptr[j[u] + 1] : 0;
      span = max(span, e1[u] - e0[u]);
    }
    double acc[kBU][2] = {};
    for (int base = 0; base < span; base += kBG) {
      int col[kBU];
      double a[kBU];
#pragma unroll
      for (int u = 0; u < kBU; ++u) {
        const int e = e0[u] + base + l;
        const bool ok = e < e1[u];
        col[u] = ok ? I.ccol[e] : j[u];
        a[u] = ok ? cs * I.cval[e] : 0.0;
      }
      const int cnt = min(kBG, span - base);
      for (int t = 0; t < cnt; ++t) {
        double v[kBU][2], au[kBU];
#pragma unroll
        for (int u = 0; u < kBU; ++u) {
          const int q = __shfl(col[u], t, kBG) * I.ld;
          v[u][0] = V[q + c0];
          v[u][1] = V[q + c1];
        }
#pragma unroll
        for (int u = 0; u < kBU; ++u) au[u] = __shfl(a[u], t, kBG);
#pragma unroll
        for (int u = 0; u < kBU; ++u) {
          acc[u][0] += au[u] * v[u][0];
          acc[u][1] += au[u] * v[u][1];
        }
      }
    }
    double d[kBU], vj[kBU][2];
#pragma unroll
    for (int u = 0; u < kBU; ++u) {
      double t = 0.0;
      vj[u][0] = V[j[u] * I.ld + c0];
      vj[u][1] = V[j[u] * I.ld + c1];
      if (GRAD) {
        double q = 0.0;
        if (l < I.r) q += vj[u][0] * vj[u][0];
        if (l + kBG < I.r) q += vj[u][1] * vj[u][1];
        const double srow = group_sum<kBG>(q);
        const bool live = it + u * ng < I.n;
        for (int i = I.dptr[j[u]] + l; i < I.dptr[j[u] + 1]; i += kBG) {
          const double v = srow * I.dcoef[i];
          const double wv = lam[i] + rho * (v - I.b[i]);
          if (live) zo[i] = v;
          t += wv * I.dcoef[i];
        }
      } else if (w) {
        for (int i = I.dptr[j[u]] + l; i < I.dptr[j[u] + 1]; i += kBG) t += w[i] * I.dcoef[i];
      }
      d[u] = group_sum<kBG>(t);
    }
#pragma unroll
    for (int u = 0; u < kBU; ++u) {
      if (it + u * ng >= I.n) continue;
      const int q = j[u] * I.ld;
      if (l < I.r) out[q + l] = os * (acc[u][0] + d[u] * vj[u][0]);
      if (l + kBG < I.r) out[q + l + kBG] = os * (acc[u][1] + d[u] * vj[u][1]);
    }
  }
}

template <typename T>
__device__ double b_dot(const Inst<T>& I, const double* X, const double* Y) {
  double s = 0.0;
  FOR_PASS(it) {
    PassSlots S;
    pass_slots(it, I.n, I.r, I.ld, S);
    double xv[kBU][2], yv[kBU][2];
    FOR_UH(u, h) { xv[u][h] = X[S.q[u][h]]; yv[u][h] = Y[S.q[u][h]]; }
    FOR_UH(u, h) if (S.on[u][h]) s += xv[u][h] * yv[u][h];
  }
  return wg_sum(s);
}

template <typename T>
__device__ double b_mdot(const Inst<T>& I, const double* x, const double* y) {
  double s = 0.0;
  FOR_CONS(i) s += x[i] * y[i];
  return wg_sum(s);
}

// y = a x + b y over the active block (x may alias y)
template <typename T, typename TX, typename TY>
__device__ void b_axpby(const Inst<T>& I, double a, const TX* x, double bb, TY* y) {
  FOR_PASS(it) {
    PassSlots S;
    pass_slots(it, I.n, I.r, I.ld, S);
    double xv[kBU][2], yv[kBU][2];
    FOR_UH(u, h) { xv[u][h] = (double)x[S.q[u][h]]; yv[u][h] = (double)y[S.q[u][h]]; }
    FOR_UH(u, h) if (S.on[u][h]) y[S.q[u][h]] = (TY)(a * xv[u][h] + bb * yv[u][h]);
  }
  __syncthreads();
}

// y = a x + b y, then <y, y>, in one pass: the arithmetic and summation order
// of b_axpby followed by b_dot(y, y)
template <typename T>
__device__ double b_axpby_norm2(const Inst<T>& I, double a, const double* x, double bb, double* y) {
  double s = 0.0;
  FOR_PASS(it) {
    PassSlots S;
    pass_slots(it, I.n, I.r, I.ld, S);
    double xv[kBU][2], yv[kBU][2];
    FOR_UH(u, h) { xv[u][h] = x[S.q[u][h]]; yv[u][h] = y[S.q[u][h]]; }
    FOR_UH(u, h) if (S.on[u][h]) {
      const double v = (double)(a * xv[u][h] + bb * yv[u][h]);
      y[S.q[u][h]] = v;
      s += v * v;
    }
  }
  return wg_sum(s);
}

template <typename T>
__device__ double b_norm_zb(const Inst<T>& I, const double* z) {
  double s = 0.0;
  FOR_CONS(i) {
    const double d = z[i] - I.b[i];
    s += d * d;
  }
  return sqrt(wg_sum(s));
}

// ---------------------------------------------------------------------------
// quartic line search (same formulas as the single-instance path)
// ---------------------------------------------------------------------------
__device__ int d_real_roots_cubic(double c3, double c2, double c1, double c0, double* out) {
  int k = 0;
  if (c3 == 0.0) {
    if (c2 == 0.0) {
      if (c1 != 0.0) out[k++] = -c0 / c1;
      return k;
    }
    const double disc = c1 * c1 - 4 * c2 * c0;
    if (disc >= 0) {
      const double q = -0.5 * (c1 + copysign(sqrt(disc), c1));
      if (q != 0.0) { out[k++] = q / c2; out[k++] = c0 / q; } else { out[k++] = 0.0; }
    }
    return k;
  }
  const double a = c2 / c3, b = c1 / c3, c = c0 / c3;
  const double Q = (a * a - 3 * b) / 9.0;
  const double R = (2 * a * a * a - 9 * a * b + 27 * c) / 54.0;
  const double Q3 = Q * Q * Q;
  if (R * R < Q3) {
    const double th = acos(fmax(-1.0, fmin(1.0, R / sqrt(Q3))));
    const double sq = -2.0 * sqrt(Q);
    out[k++] = sq * cos(th / 3.0) - a / 3.0;
    out[k++] = sq * cos((th + 2 * M_PI) / 3.0) - a / 3.0;
    out[k++] = sq * cos((th - 2 * M_PI) / 3.0) - a / 3.0;
  } else {
    const double A = -copysign(cbrt(fabs(R) + sqrt(R * R - Q3)), R);
    const double B = (A != 0.0) ? Q / A : 0.0;
    out[k++] = (A + B) - a / 3.0;
  }
  for (int t = 0; t < k; ++t) {
    double x = out[t];
    for (int it = 0; it < 2; ++it) {
      const double f = ((c3 * x + c2) * x + c1) * x + c0;
      const double df = (3 * c3 * x + 2 * c2) * x + c1;
      if (df != 0.0) x -= f / df;
    }
    out[t] = x;
  }
  return k;
}

__device__ double d_quartic_step(double q1, double q2, double q3, double q4) {
  double roots[3];
  const int k = d_real_roots_cubic(4 * q4, 3 * q3, 2 * q2, q1, roots);
  double best = 0.0, bestv = 0.0;
  for (int t = 0; t < k; ++t) {
    const double a = roots[t];
    if (!(a > 0.0)) continue;
    const double v = (((q4 * a + q3) * a + q2) * a + q1) * a;
    if (v < bestv) { best = a; bestv = v; }
  }
  return best;
}

// ---------------------------------------------------------------------------
// the per-instance solver
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBatchMaxBlock) batch_solve_kernel(const BatchDesc* __restrict__ descs,
                                                           BatchArrays A, BatchOpts o) {
  const BatchDesc d = descs[blockIdx.x];
  Inst<T> I;
  I.n = d.n; I.m = d.m; I.ld = d.rcap; I.r = d.r0;
  I.cptr = A.cptr + d.cptr_off;
  I.ccol = A.ccol + d.ccol_off;
  I.cval = A.cval + d.ccol_off;
  I.dptr = A.dptr + d.dptr_off;
  I.drow = A.drow + d.con_off;
  I.dcoef = A.dcoef + d.con_off;
  I.dsq = A.dsq + d.row_off;
  I.b = A.b + d.con_off;
  I.c_fro = d.c_fro; I.b_inf = d.b_inf; I.b_1 = d.b_1;
  const size_t F = (size_t)A.fac_total;
  double* U = A.U + d.fac_off;
  double* V = A.V + d.fac_off;
  double* Vold = A.Vold + d.fac_off;
  double* G = A.G + d.fac_off;
  double* Gn = A.Gn + d.fac_off;
  double* D = A.D + d.fac_off;
  double* Sn = A.Sn + d.fac_off;
  double* Yn = A.Yn + d.fac_off;
  double* CD = A.CD + d.fac_off;
  double* R64 = A.R64 + d.fac_off;
  double* z = A.z + d.con_off;
  double* lam = A.lam + d.con_off;
  double* p1 = A.p1 + d.con_off;
  double* p2 = A.p2 + d.con_off;
  T* X = (T*)A.X + d.fac_off;
  T* R = (T*)A.R + d.fac_off;
  T* Pd = (T*)A.P + d.fac_off;
  T* Q = (T*)A.Q + d.fac_off;
  T* Wt = (T*)A.W + d.fac_off;
  BatchResult res;
  memset(&res, 0, sizeof(res));
  const int mem = o.lbfgs_mem;

  // ================= Phase I: ALM =================
  const int r_cap = o.r_max > 0 ? min(d.rcap, o.r_max) : d.rcap;
  double rho = o.rho0 > 0 ? o.rho0 : 1.0 / fmax(1.0, I.b_inf);
  b_forward(I, U, U, z, 1.0);
  __syncthreads();
  double v = b_norm_zb(I, z) / (1.0 + I.b_inf);
  double v_ref = INFINITY;
  int outer = 0, inner_total = 0, growths = 0;
  double rhoh[8];
  int slot_of[8];
  while (o.phase1 && v > o.switch_tol && outer < o.alm_outer_max) {
    const int cap = (I.r < r_cap) ? o.rank_grow_iters : o.alm_inner_max;
    const double tol = fmax(o.alm_inner_rel * v, o.alm_inner_floor);
    int head = 0, count = 0;
    for (int t = 0; t < mem; ++t) slot_of[t] = t;
    // gradient G = 2 (C + A*(lam + rho (z - b))) U
    b_adjoint<T, true>(I, nullptr, 1.0, U, G, 2.0, z, lam, rho);
    __syncthreads();
    int it = 0;
    bool conv = false;
    while (true) {
      const double gnorm = sqrt(b_dot(I, G, G));
      if (!(gnorm == gnorm)) { res.status = LORADS_ENUMERIC; goto finish; }
      if (gnorm / (1.0 + I.c_fro) <= tol) { conv = true; break; }
      if (it >= cap) break;
      // two-loop recursion, q in D
      b_axpby(I, 1.0, G, 0.0, D);
      double al[8];
      for (int t = 0; t < count; ++t) {
        const int k = slot_of[(head - 1 - t + mem) % mem];
        double* Sk = A.S + (size_t)k * F + d.fac_off;
        double* Yk = A.Y + (size_t)k * F + d.fac_off;
        al[t] = rhoh[k] * b_dot(I, Sk, D);
        b_axpby(I, -al[t], Yk, 1.0, D);
      }
      if (count > 0) {
        const int k = slot_of[(head - 1 + mem) % mem];
        double* Sk = A.S + (size_t)k * F + d.fac_off;
        double* Yk = A.Y + (size_t)k * F + d.fac_off;
        const double sy = b_dot(I, Sk, Yk), yy = b_dot(I, Yk, Yk);
        b_axpby(I, 0.0, D, sy / yy, D);
      }
      for (int t = count - 1; t >= 0; --t) {
        const int k = slot_of[(head - 1 - t + mem) % mem];
        double* Sk = A.S + (size_t)k * F + d.fac_off;
        double* Yk = A.Y + (size_t)k * F + d.fac_off;
        const double bt = rhoh[k] * b_dot(I, Yk, D);
        b_axpby(I, al[t] - bt, Sk, 1.0, D);
      }
      b_axpby(I, 0.0, D, -1.0, D);
      if (!(b_dot(I, G, D) < 0.0)) {
        b_axpby(I, -1.0, G, 0.0, D);
        head = count = 0;
      }
      double alpha = 0.0;
      for (int attempt = 0; attempt < 2; ++attempt) {
        b_forward(I, U, D, p1, 2.0);
        b_forward(I, D, D, p2, 1.0);
        b_adjoint(I, (const double*)nullptr, 1.0, D, CD, 1.0);
        __syncthreads();
        const double c1 = 2.0 * b_dot(I, CD, U), c2 = b_dot(I, CD, D);
        double s7[7] = {0, 0, 0, 0, 0, 0, 0};
        FOR_CONS(i) {
          const double a0 = z[i] - I.b[i], a1 = p1[i], a2 = p2[i], l = lam[i];
          s7[0] += a2 * a2; s7[1] += a1 * a2; s7[2] += a1 * a1; s7[3] += a0 * a2;
          s7[4] += a0 * a1; s7[5] += l * a1; s7[6] += l * a2;
        }
        for (int t = 0; t < 7; ++t) s7[t] = wg_sum(s7[t]);
        const double q4 = 0.5 * rho * s7[0];
        const double q3 = rho * s7[1];
        const double q2 = c2 + s7[6] + 0.5 * rho * (s7[2] + 2.0 * s7[3]);
        const double q1 = c1 + s7[5] + rho * s7[4];
        alpha = d_quartic_step(q1, q2, q3, q4);
        if (alpha > 0.0 || count == 0) break;
        b_axpby(I, -1.0, G, 0.0, D);
        head = count = 0;
      }
      if (!(alpha > 0.0)) break;
      b_axpby(I, alpha, D, 0.0, Sn);
      b_axpby(I, 1.0, Sn, 1.0, U);
      b_adjoint<T, true>(I, nullptr, 1.0, U, Gn, 2.0, z, lam, rho);
      __syncthreads();
      b_axpby(I, 1.0, Gn, 0.0, Yn);
      b_axpby(I, -1.0, G, 1.0, Yn);
      const double sy = b_dot(I, Sn, Yn);
      if (sy > 0.0) {
        // the pair goes to the oldest slot when the memory is full
        const int pos = head;
        const int k = slot_of[pos];
        double* Sk = A.S + (size_t)k * F + d.fac_off;
        double* Yk = A.Y + (size_t)k * F + d.fac_off;
        b_axpby(I, 1.0, Sn, 0.0, Sk);
        b_axpby(I, 1.0, Yn, 0.0, Yk);
        rhoh[k] = 1.0 / sy;
        head = (head + 1) % mem;
        count = min(count + 1, mem);
      }
      {
        double* t = G; G = Gn; Gn = t;
      }
      ++it;
    }
    inner_total += it;
    v = b_norm_zb(I, z) / (1.0 + I.b_inf);
    if (!conv && I.r < r_cap && it >= cap && v > o.switch_tol) {
      const int r_new = min((int)ceil(o.rank_factor * I.r), r_cap);
      const double sigma = 1e-3 * sqrt(b_dot(I, U, U)) / sqrt((double)I.n * I.r);
      const int add = r_new - I.r;
      FOR_GROUPS(j, I.n) for (int c = I.r + (int)threadIdx.x % kBG; c < r_new; c += kBG) {
        const uint64_t t = (uint64_t)j * add + (uint64_t)(c - I.r);
        const uint64_t k1 = ((uint64_t)growths << 40) + 2ull * t + 1ull, k2 = k1 + 1ull;
        const uint64_t gg = 0x9E3779B97F4A7C15ull;
        const double u1 = ((double)(splitmix_mix(o.seed + k1 * gg) >> 11) + 1.0) * 0x1.0p-53;
        const double u2 = (double)(splitmix_mix(o.seed + k2 * gg) >> 11) * 0x1.0p-53;
        U[(size_t)j * I.ld + c] = sigma * sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
      }
      __syncthreads();
      I.r = r_new;
      ++growths;
      b_forward(I, U, U, z, 1.0);
      __syncthreads();
      v = b_norm_zb(I, z) / (1.0 + I.b_inf);
      continue;
    }
    if (v <= o.alm_eta * v_ref) {
      FOR_CONS(i) lam[i] += rho * (z[i] - I.b[i]);
      __syncthreads();
      v_ref = v;
    } else {
      rho *= o.alm_rho_factor;
    }
    ++outer;
  }
  res.alm_outer = outer;
  res.alm_inner = inner_total;
  res.growths = growths;
  res.rho_alm = rho;

  {
    // ================= Phase II: ADMM =================
    rho *= o.h;
    const double gamma = o.gamma_fixed > 0 ? o.gamma_fixed
                                           : o.gamma_scale * (1.0 + I.c_fro / sqrt((double)I.n));
    b_axpby(I, 1.0, U, 0.0, V);
    const int maxit = (int)min((long long)I.n * I.r, (long long)o.cg_maxit);
    const double floor_tol = (sizeof(T) == 8) ? o.cg_tol_floor : fmax(o.cg_tol_floor, 1e-6);
    double kkt = INFINITY, pinf = INFINITY, dres = INFINITY;
    long long cg_total = 0;
    int k = 0;
    res.status = LORADS_MAXITER;
    while (k < o.max_admm_iter) {
      const double tol = fmin(o.cg_tol_max, fmax(floor_tol, o.cg_tol_kkt * kkt));
      const double vnorm2 = b_axpby_norm2(I, 1.0, V, 0.0, Vold);
      for (int half = 0; half < 2; ++half) {
        const double* W = half == 0 ? V : U;
        double* out = half == 0 ? U : V;
        // R = -(C + A*(lam + rho (A(W W^T) - b))) W, CG on M_W D = R from D = 0
        b_adjoint<T, true>(I, nullptr, 1.0, W, R64, -1.0, z, lam, rho);
        __syncthreads();
        // CG set-up, and the first operator application Q = M(P) with P = R in
        // the same pass (row-local); its <P, Q> is used if the loop runs
        double rr = 0.0, pq0 = 0.0;
        FOR_PASS(it) {
          PassSlots S;
          pass_slots(it, I.n, I.r, I.ld, S);
          const int ng = blockDim.x / kBG;
          double rv[kBU][2], wv[kBU][2], pv[kBU][2], wt[kBU][2], ds[kBU];
          FOR_UH(u, h) { rv[u][h] = R64[S.q[u][h]]; wv[u][h] = W[S.q[u][h]]; }
          FOR_UH(u, h) {
            const int q = S.q[u][h];
            const T t = (T)rv[u][h];
            const T tw = (T)wv[u][h];
            pv[u][h] = (double)t;
            wt[u][h] = (double)tw;
            if (S.on[u][h]) {
              R[q] = t;
              Wt[q] = tw;
              X[q] = (T)0;
              Pd[q] = t;
              rr += (double)t * (double)t;
            }
          }
#pragma unroll
          for (int u = 0; u < kBU; ++u) {
            const int j = min(it + u * ng, I.n - 1);
            double dd = 0.0;
#pragma unroll
            for (int h = 0; h < 2; ++h)
              if (S.on[u][h]) dd += pv[u][h] * wt[u][h];
            ds[u] = group_sum<kBG>(dd) * rho * I.dsq[j];
          }
          FOR_UH(u, h) if (S.on[u][h]) {
            const T qv = (T)(gamma * pv[u][h] + ds[u] * wt[u][h]);
            Q[S.q[u][h]] = qv;
            pq0 += pv[u][h] * (double)qv;
          }
        }
        wg_sum2(rr, pq0);
        const double rr0 = rr;
        int cgi = 0;
        double beta = 0.0;
        while (rr0 > 0.0 && cgi < maxit && rr > tol * tol * rr0) {
          // from the second iteration on, the direction P = R + beta P is formed
          // in the same pass (row-local), then Q = gamma P + rho dsq <P_j, W_j> W_j
          double pq = pq0;
          if (cgi > 0) {
            pq = 0.0;
            FOR_PASS(it) {
              PassSlots S;
              pass_slots(it, I.n, I.r, I.ld, S);
              const int ng = blockDim.x / kBG;
              double pv[kBU][2], wv[kBU][2], ds[kBU];
              {
                double rv[kBU][2];
                FOR_UH(u, h) {
                  pv[u][h] = (double)Pd[S.q[u][h]];
                  rv[u][h] = (double)R[S.q[u][h]];
                  wv[u][h] = (double)Wt[S.q[u][h]];
                }
                FOR_UH(u, h) {
                  const T pt = (T)(rv[u][h] + beta * pv[u][h]);
                  if (S.on[u][h]) Pd[S.q[u][h]] = pt;
                  pv[u][h] = (double)pt;
                }
              }
#pragma unroll
              for (int u = 0; u < kBU; ++u) {
                const int j = min(it + u * ng, I.n - 1);
                double dd = 0.0;
#pragma unroll
                for (int h = 0; h < 2; ++h)
                  if (S.on[u][h]) dd += pv[u][h] * wv[u][h];
                ds[u] = group_sum<kBG>(dd) * rho * I.dsq[j];
              }
              FOR_UH(u, h) if (S.on[u][h]) {
                const T qv = (T)(gamma * pv[u][h] + ds[u] * wv[u][h]);
                Q[S.q[u][h]] = qv;
                pq += pv[u][h] * (double)qv;
              }
            }
            pq = wg_sum(pq);
          }
          if (!(pq > 0.0)) break;
          const double alpha = rr / pq;
          double rn = 0.0;
          FOR_PASS(it) {
            PassSlots S;
            pass_slots(it, I.n, I.r, I.ld, S);
            double xv[kBU][2], pv[kBU][2], rv[kBU][2], qv[kBU][2];
            FOR_UH(u, h) {
              const int q = S.q[u][h];
              xv[u][h] = (double)X[q];
              pv[u][h] = (double)Pd[q];
              rv[u][h] = (double)R[q];
              qv[u][h] = (double)Q[q];
            }
            FOR_UH(u, h) if (S.on[u][h]) {
              const int q = S.q[u][h];
              X[q] = (T)(xv[u][h] + alpha * pv[u][h]);
              const T rt = (T)(rv[u][h] - alpha * qv[u][h]);
              R[q] = rt;
              rn += (double)rt * (double)rt;
            }
          }
          rn = wg_sum(rn);
          beta = rn / rr;
          rr = rn;
          ++cgi;
        }
        cg_total += cgi;
        FOR_RC(j, c) {
          const size_t q = (size_t)j * I.ld + c;
          out[q] = W[q] + (double)X[q];
        }
        __syncthreads();
      }
      // dual update and residuals
      b_forward(I, U, V, z, 1.0);
      __syncthreads();
      double s = 0.0;
      FOR_CONS(i) {
        const double dz = z[i] - I.b[i];
        lam[i] += rho * dz;
        s += dz * dz;
      }
      s = wg_sum(s);
      const double dv2 = b_axpby_norm2(I, 1.0, V, -1.0, Vold);
      pinf = sqrt(s) / (1.0 + I.b_inf);
      dres = gamma * sqrt(dv2) / (1.0 + sqrt(vnorm2));
      if (!(pinf == pinf) || !(dres == dres)) { res.status = LORADS_ENUMERIC; break; }
      kkt = fmax(pinf, dres);
      ++k;
      if (kkt < o.eps) { res.status = LORADS_OK; break; }
      if (k % o.rho_every == 0 && rho < o.rho_max) rho = fmin(o.rho_growth * rho, o.rho_max);
    }
    res.admm_iters = k;
    res.cg_iters = cg_total;
    res.kkt = kkt;
    res.pinf_stop = pinf;
    res.dres_stop = dres;
    res.rho = rho;
    res.gamma = gamma;
  }
  {
    // ================= output measures =================
    b_axpby(I, 0.5, U, 0.0, D);
    b_axpby(I, 0.5, V, 1.0, D);  // D = U_hat
    b_forward(I, D, D, z, 1.0);
    b_adjoint(I, (const double*)nullptr, 1.0, D, CD, 1.0);
    __syncthreads();
    const double zb = b_norm_zb(I, z);
    res.obj = b_dot(I, CD, D);
    res.dual_obj = -b_mdot(I, I.b, lam);
    res.pinf = zb / (1.0 + I.b_1);
    res.gap = (res.obj - res.dual_obj) / (1.0 + fabs(res.obj) + fabs(res.dual_obj));
  }
finish:
  res.rank = I.r;
  if (threadIdx.x == 0) A.res[blockIdx.x] = res;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
bool batch_eligible(const std::vector<std::unique_ptr<Problem>>& probs) {
  if (probs.size() < 2) return false;
  for (auto& p : probs)
    if (p->structure != LORADS_STRUCT_DIAG || p->mu != 0.0) return false;
  return true;
}

void Batch::build(const std::vector<std::unique_ptr<Problem>>& probs, hipStream_t s) {
  const int np = (int)probs.size();
  std::vector<BatchDesc> h(np);
  long long cp = 0, cc = 0, dp = 0, con = 0, row = 0, fac = 0;
  for (int i = 0; i < np; ++i) {
    const Problem& P = *probs[i];
    BatchDesc& d = h[i];
    d.n = P.n;
    d.m = P.m;
    d.cptr_off = (int)cp; cp += P.n + 1;
    d.ccol_off = (int)cc; cc += P.cval.n;
    d.dptr_off = (int)dp; dp += P.n + 1;
    d.con_off = (int)con; con += P.m;
    d.row_off = (int)row; row += P.n;
    d.c_fro = P.c_fro; d.b_inf = P.b_inf; d.b_1 = P.b_1;
    d.rcap = std::max(1, std::min({32, (int)std::floor(std::sqrt(2.0 * P.m)), P.n}));
    d.fac_off = fac;
    fac += (long long)P.n * d.rcap;
  }
  host_desc = h;
  n_cptr = cp; n_ccol = cc; n_con = con; n_row = row; fac_total = fac;
  cptr.alloc(cp); ccol.alloc(std::max<long long>(cc, 1)); cval.alloc(std::max<long long>(cc, 1));
  dptr.alloc(dp); drow.alloc(con); dcoef.alloc(con); dsq.alloc(row); b.alloc(con);
  for (int i = 0; i < np; ++i) {
    const Problem& P = *probs[i];
    const BatchDesc& d = h[i];
    HIPCHK(hipMemcpyAsync(cptr.p + d.cptr_off, P.cptr.p, (P.n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (P.cval.n) {
      HIPCHK(hipMemcpyAsync(ccol.p + d.ccol_off, P.ccol.p, P.ccol.n * sizeof(int), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(cval.p + d.ccol_off, P.cval.p, P.cval.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipMemcpyAsync(dptr.p + d.dptr_off, P.dptr.p, (P.n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(drow.p + d.con_off, P.drow.p, P.m * sizeof(int), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(dcoef.p + d.con_off, P.dcoef.p, P.m * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(dsq.p + d.row_off, P.dsq.p, P.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(b.p + d.con_off, P.b.p, P.m * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  const size_t F = (size_t)fac;
  for (DevBuf<double>* buf : {&U, &V, &Vold, &G, &Gn, &D, &Sn, &Yn, &CD, &R64}) buf->alloc(F);
  z.alloc(con); lam.alloc(con); p1.alloc(con); p2.alloc(con);
  res.alloc(np);
  desc.alloc(np);
  HIPCHK(hipStreamSynchronize(s));
  built = true;
}

void batch_solve(std::vector<std::unique_ptr<Problem>>& probs, Batch& B, const lorads_options& o,
                 lorads_result* results, hipStream_t s, int block) {
  const int np = (int)probs.size();
  if (!B.built) B.build(probs, s);
  if (o.lbfgs_mem > 8) fail(LORADS_EINVAL, "batched solve supports lbfgs_mem <= 8");
  std::vector<BatchDesc> h = B.host_desc;
  for (int i = 0; i < np; ++i) {
    if (!o.init_U[i]) fail(LORADS_EINVAL, "init_U missing for problem " + std::to_string(i));
    const int r0 = o.init_rank ? o.init_rank[i] : o.r0;
    if (r0 > h[i].rcap) fail(LORADS_EINVAL, "initial rank above the batched rank capacity of problem " + std::to_string(i));
    h[i].r0 = r0;
  }
  HIPCHK(hipMemcpyAsync(B.desc.p, h.data(), np * sizeof(BatchDesc), hipMemcpyHostToDevice, s));
  // starting points: U (strided by the rank capacity) and lambda
  B.U.zero(s);
  std::vector<double> stage;
  for (int i = 0; i < np; ++i) {
    const Problem& P = *probs[i];
    stage.assign((size_t)P.n * h[i].rcap, 0.0);
    for (int j = 0; j < P.n; ++j)
      for (int c = 0; c < h[i].r0; ++c)
        stage[(size_t)j * h[i].rcap + c] = o.init_U[i][(size_t)j * h[i].r0 + c];
    HIPCHK(hipMemcpy(B.U.p + h[i].fac_off, stage.data(), stage.size() * sizeof(double), hipMemcpyHostToDevice));
    if (o.init_lambda && o.init_lambda[i]) {
      DevBuf<double> tmp;
      tmp.upload(o.init_lambda[i], P.m, s);
      if (P.perm_identity)
        HIPCHK(hipMemcpyAsync(B.lam.p + h[i].con_off, tmp.p, P.m * sizeof(double), hipMemcpyDeviceToDevice, s));
      else
        gather_kernel<double><<<grid_for(P.m), kBlock, 0, s>>>(P.m, P.perm.p, tmp.p, B.lam.p + h[i].con_off);
      HIPCHK(hipStreamSynchronize(s));
    } else {
      HIPCHK(hipMemsetAsync(B.lam.p + h[i].con_off, 0, P.m * sizeof(double), s));
    }
  }
  BatchOpts bo;
  bo.phase1 = o.phase1; bo.switch_tol = o.switch_tol; bo.h = o.h; bo.eps = o.eps;
  bo.rho_growth = o.rho_growth; bo.rho_every = o.rho_every; bo.rho_max = o.rho_max;
  bo.max_admm_iter = o.max_admm_iter; bo.gamma_fixed = o.gamma_fixed; bo.gamma_scale = o.gamma_scale;
  bo.cg_tol_max = o.cg_tol_max; bo.cg_tol_floor = o.cg_tol_floor; bo.cg_tol_kkt = o.cg_tol_kkt;
  bo.cg_maxit = o.cg_maxit; bo.lbfgs_mem = o.lbfgs_mem; bo.alm_inner_max = o.alm_inner_max;
  bo.rank_grow_iters = o.rank_grow_iters; bo.rank_factor = o.rank_factor;
  bo.alm_inner_rel = o.alm_inner_rel; bo.alm_inner_floor = o.alm_inner_floor;
  bo.alm_eta = o.alm_eta; bo.alm_rho_factor = o.alm_rho_factor; bo.alm_outer_max = o.alm_outer_max;
  bo.rho0 = o.rho0; bo.seed = o.seed; bo.r_max = o.r_max;
  BatchArrays a;
  a.cptr = B.cptr.p; a.ccol = B.ccol.p; a.cval = B.cval.p; a.dptr = B.dptr.p; a.drow = B.drow.p;
  a.dcoef = B.dcoef.p; a.dsq = B.dsq.p; a.b = B.b.p;
  a.U = B.U.p; a.V = B.V.p; a.Vold = B.Vold.p; a.G = B.G.p; a.Gn = B.Gn.p; a.D = B.D.p;
  a.Sn = B.Sn.p; a.Yn = B.Yn.p; a.CD = B.CD.p; a.R64 = B.R64.p;
  a.z = B.z.p; a.lam = B.lam.p; a.p1 = B.p1.p; a.p2 = B.p2.p;
  a.res = B.res.p;
  a.fac_total = B.fac_total;
  const size_t F = (size_t)B.fac_total;
  B.S.alloc(F * o.lbfgs_mem);
  B.Y.alloc(F * o.lbfgs_mem);
  a.S = B.S.p; a.Y = B.Y.p;
  const bool f32 = o.precision != LORADS_F64;
  const size_t esz = f32 ? sizeof(float) : sizeof(double);
  for (DevBuf<char>* buf : {&B.X, &B.R, &B.P, &B.Q, &B.W}) buf->alloc(F * esz);
  a.X = B.X.p; a.R = B.R.p; a.P = B.P.p; a.Q = B.Q.p; a.W = B.W.p;
  if (block < 64 || block > kBatchMaxBlock || block % 64)
    fail(LORADS_EINVAL, "batch block size must be a multiple of 64 in [64, 256]");
  if (f32)
    batch_solve_kernel<float><<<np, block, 0, s>>>(B.desc.p, a, bo);
  else
    batch_solve_kernel<double><<<np, block, 0, s>>>(B.desc.p, a, bo);
  HIPCHK(hipGetLastError());
  std::vector<BatchResult> hr(np);
  HIPCHK(hipMemcpyAsync(hr.data(), B.res.p, np * sizeof(BatchResult), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // hand each instance's factors and multipliers to its problem object
  for (int i = 0; i < np; ++i) {
    Problem& P = *probs[i];
    const BatchResult& q = hr[i];
    lorads_result& R = results[i];
    std::memset(&R, 0, sizeof(R));
    R.status = q.status; R.rank = q.rank; R.alm_outer = q.alm_outer; R.alm_inner = q.alm_inner;
    R.rank_growths = q.growths; R.admm_iters = q.admm_iters; R.cg_iters = q.cg_iters;
    R.obj = q.obj; R.dual_obj = q.dual_obj; R.pinf = q.pinf; R.gap = q.gap; R.kkt = q.kkt;
    R.pinf_stop = q.pinf_stop; R.dres_stop = q.dres_stop; R.rho = q.rho; R.gamma = q.gamma;
    R.dinf = NAN; R.lambda_min = NAN;
    const int rr = std::max(1, q.rank);
    P.rank = rr;
    P.U.alloc((size_t)P.n * rr);
    P.V.alloc((size_t)P.n * rr);
    P.lam.alloc(P.m);
    copy_rows<double, double><<<grid_for((size_t)P.n * rr), kBlock, 0, s>>>(P.n, rr, B.U.p + h[i].fac_off, h[i].rcap, P.U.p, rr);
    copy_rows<double, double><<<grid_for((size_t)P.n * rr), kBlock, 0, s>>>(P.n, rr, B.V.p + h[i].fac_off, h[i].rcap, P.V.p, rr);
    HIPCHK(hipMemcpyAsync(P.lam.p, B.lam.p + h[i].con_off, P.m * sizeof(double), hipMemcpyDeviceToDevice, s));
    P.solved = true;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
}

}  // namespace lorads
