// Structure-specialised kernels: DIAG (A_i = a_i e_j e_j^T, MaxCut) and PAIR
// (A_i = a_i (e_j e_k^T + e_k e_j^T), matrix completion).  Same group-per-row
// mapping and deterministic reductions as the generic kernels.
#pragma once

#include "kernels.hpp"

namespace lorads {

// ===========================================================================
// K1 forward map, shared MODE convention:
//   0: z = scale * A(U V^T)
//   1: z = A(U V^T), w = lam + rho (z - b)   (FP64)
//   2: z = sc[S_RHO] * A(U V^T), skipped once the CG has converged
// ===========================================================================
template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) k1_diag(
    int m, const int* __restrict__ drow, const T* __restrict__ dcoef, const T* __restrict__ U,
    const T* __restrict__ V, int r, int ld, T* __restrict__ z, double scale,
    const double* __restrict__ lam, const double* __restrict__ b, double rho,
    double* __restrict__ w, const double* __restrict__ sc, int parity) {
  if (MODE == 2 && sc[S_DONE + parity] != 0.0) return;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (i >= m) return;
  const int j = drow[i];
  double s = 0.0;
  for (int c = lane; c < r; c += G) s += (double)U[(size_t)j * ld + c] * (double)V[(size_t)j * ld + c];
  s = group_sum<G>(s) * (double)dcoef[i];
  if (lane == 0) {
    if (MODE == 1) {
      z[i] = (T)s;
      w[i] = lam[i] + rho * (s - b[i]);
    } else if (MODE == 2) {
      z[i] = (T)(sc[S_RHO] * s);
    } else {
      z[i] = (T)(scale * s);
    }
  }
}

template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) k1_pair(
    int m, const int* __restrict__ pj, const int* __restrict__ pk, const T* __restrict__ pcoef,
    double pair_coef, const T* __restrict__ U, const T* __restrict__ V, int r, int ld,
    T* __restrict__ z, double scale, const double* __restrict__ lam,
    const double* __restrict__ b, double rho, double* __restrict__ w,
    const double* __restrict__ sc, int parity) {
  if (MODE == 2 && sc[S_DONE + parity] != 0.0) return;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (i >= m) return;
  const int j = pj[i], k = pk[i];
  double s = 0.0;
  for (int c = lane; c < r; c += G)
    s += (double)U[(size_t)j * ld + c] * (double)V[(size_t)k * ld + c] +
         (double)U[(size_t)k * ld + c] * (double)V[(size_t)j * ld + c];
  const double a = pcoef ? (double)pcoef[i] : pair_coef;
  s = group_sum<G>(s) * a;
  if (lane == 0) {
    if (MODE == 1) {
      z[i] = (T)s;
      w[i] = lam[i] + rho * (s - b[i]);
    } else if (MODE == 2) {
      z[i] = (T)(sc[S_RHO] * s);
    } else {
      z[i] = (T)(scale * s);
    }
  }
}

// ===========================================================================
// K2 DIAG: out_j = out_scale (c_scale (C V)_j + (sum_{i on row j} w_i a_i) V_j)
// ===========================================================================
template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) k2_diag(
    int n, const int* __restrict__ cptr, const int* __restrict__ ccol,
    const T* __restrict__ cval, double c_scale, const int* __restrict__ dptr,
    const T* __restrict__ dcoef, const T* __restrict__ unused, const T* __restrict__ w,
    const T* __restrict__ V, int r, int ld, T* __restrict__ out, int ldo, double out_scale,
    const T* __restrict__ P, double* __restrict__ sc, int parity, double* __restrict__ part,
    int* __restrict__ counter) {
  const int row = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (row >= n) return;
  constexpr int MAXC = 4;
  double acc[MAXC];
#pragma unroll
  for (int t = 0; t < MAXC; ++t) acc[t] = 0.0;
  if (c_scale != 0.0) {
    for (int e = cptr[row]; e < cptr[row + 1]; ++e) {
      const int k = ccol[e];
      const double a = c_scale * (double)cval[e];
#pragma unroll
      for (int t = 0; t < MAXC; ++t) {
        const int c = lane + t * G;
        if (c < r) acc[t] += a * (double)V[(size_t)k * ld + c];
      }
    }
  }
  double d = 0.0;
  if (w != nullptr)
    for (int i = dptr[row]; i < dptr[row + 1]; ++i) d += (double)w[i] * (double)dcoef[i];
#pragma unroll
  for (int t = 0; t < MAXC; ++t) {
    const int c = lane + t * G;
    if (c < r) out[(size_t)row * ldo + c] = (T)(out_scale * (acc[t] + d * (double)V[(size_t)row * ld + c]));
  }
}

// ===========================================================================
// K3 DIAG (fused CG operator, row-local):
//   Q_j = gamma P_j + rho (sum_i a_i^2) <P_j, W_j> W_j,   plus <P, Q>.
// ===========================================================================
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k3_diag(int n, const T* __restrict__ dsq,
                                                  const T* __restrict__ W,
                                                  const T* __restrict__ P, T* __restrict__ Q,
                                                  int r, double* __restrict__ sc, int parity,
                                                  double* __restrict__ part,
                                                  int* __restrict__ counter) {
  __shared__ double sh[kBlock / 64];
  if (sc[S_DONE + parity] != 0.0) return;
  const int row = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  const double gamma = sc[S_GAMMA], rho = sc[S_RHO];
  double pq = 0.0;
  if (row < n) {
    double d = 0.0;
    for (int c = lane; c < r; c += G) d += (double)P[(size_t)row * r + c] * (double)W[(size_t)row * r + c];
    d = group_sum<G>(d) * rho * (double)dsq[row];
    for (int c = lane; c < r; c += G) {
      const double p = (double)P[(size_t)row * r + c];
      const T q = (T)(gamma * p + d * (double)W[(size_t)row * r + c]);
      Q[(size_t)row * r + c] = q;
      pq += p * (double)q;
    }
  }
  const double bs = block_sum(pq, sh);
  if (last_block(bs, part, counter)) {
    const double s = sum_parts(part, gridDim.x);
    sc[S_PQ] = s;
    if (!(s > 0.0)) {
      sc[S_BRK] = 1.0;
    } else {
      sc[S_BRK] = 0.0;
      sc[S_ALPHA] = sc[S_RR + parity] / s;
    }
    *counter = 0;
  }
}

// ===========================================================================
// K2 PAIR, row-owner over both views (no atomics):
//   MODE 0: out_t = out_scale (c_scale (C V)_t + sum_{i incident to t} w_i a_i V_partner)
//   MODE 1: fused CG operator.  For every constraint incident to row t with
//           partner p: d_i = <Pm_t, V_p> + <Pm_p, V_t>, and
//           Q_t = gamma Pm_t + rho sum_i a_i^2 d_i V_p;  accumulates <Pm, Q>.
//           (V = the fixed factor W, Pm = the CG direction.)
// ===========================================================================
template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) k2_pair(
    int n, const int* __restrict__ cptr, const int* __restrict__ ccol,
    const T* __restrict__ cval, double c_scale, const int* __restrict__ rptr,
    const int* __restrict__ pk, const int* __restrict__ cvptr, const int* __restrict__ cvj,
    const int* __restrict__ cvid, const T* __restrict__ pcoef, double pair_coef,
    const T* __restrict__ w, const T* __restrict__ V, const T* __restrict__ Pm, int r, int ld,
    T* __restrict__ out, int ldo, double out_scale, double* __restrict__ sc, int parity,
    double* __restrict__ part, int* __restrict__ counter) {
  __shared__ double sh[kBlock / 64];
  if (MODE == 1 && sc[S_DONE + parity] != 0.0) return;
  const int row = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  constexpr int MAXC = 4;
  double acc[MAXC], pt[MAXC], vt[MAXC];
#pragma unroll
  for (int t = 0; t < MAXC; ++t) acc[t] = pt[t] = vt[t] = 0.0;
  double pq = 0.0;
  if (row < n) {
    if (MODE == 1) {
#pragma unroll
      for (int t = 0; t < MAXC; ++t) {
        const int c = lane + t * G;
        if (c < r) {
          pt[t] = (double)Pm[(size_t)row * ld + c];
          vt[t] = (double)V[(size_t)row * ld + c];
        }
      }
    }
    if (MODE == 0 && c_scale != 0.0) {
      for (int e = cptr[row]; e < cptr[row + 1]; ++e) {
        const int k = ccol[e];
        const double a = c_scale * (double)cval[e];
#pragma unroll
        for (int t = 0; t < MAXC; ++t) {
          const int c = lane + t * G;
          if (c < r) acc[t] += a * (double)V[(size_t)k * ld + c];
        }
      }
    }
    // view R (row is j, partner k = pk[i]) then view C (row is k, partner j)
    const int r0 = rptr[row], r1 = rptr[row + 1];
    const int c0 = cvptr[row], c1 = cvptr[row + 1];
    const int total = (MODE == 0 && w == nullptr) ? 0 : (r1 - r0) + (c1 - c0);
    for (int q = 0; q < total; ++q) {
      int id, p;
      if (q < r1 - r0) {
        id = r0 + q;
        p = pk[id];
      } else {
        const int e = c0 + (q - (r1 - r0));
        id = cvid[e];
        p = cvj[e];
      }
      const double a = pcoef ? (double)pcoef[id] : pair_coef;
      double coef;
      if (MODE == 1) {
        double d = 0.0;
#pragma unroll
        for (int t = 0; t < MAXC; ++t) {
          const int c = lane + t * G;
          if (c < r)
            d += pt[t] * (double)V[(size_t)p * ld + c] + (double)Pm[(size_t)p * ld + c] * vt[t];
        }
        d = group_sum<G>(d);
        coef = a * a * d;
      } else {
        coef = (double)w[id] * a;
      }
#pragma unroll
      for (int t = 0; t < MAXC; ++t) {
        const int c = lane + t * G;
        if (c < r) acc[t] += coef * (double)V[(size_t)p * ld + c];
      }
    }
    if (MODE == 1) {
      const double gamma = sc[S_GAMMA], rho = sc[S_RHO];
#pragma unroll
      for (int t = 0; t < MAXC; ++t) {
        const int c = lane + t * G;
        if (c < r) {
          const T qv = (T)(gamma * pt[t] + rho * acc[t]);
          out[(size_t)row * ldo + c] = qv;
          pq += pt[t] * (double)qv;
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < MAXC; ++t) {
        const int c = lane + t * G;
        if (c < r) out[(size_t)row * ldo + c] = (T)(out_scale * acc[t]);
      }
    }
  }
  if (MODE == 1) {
    const double bs = block_sum(pq, sh);
    if (last_block(bs, part, counter)) {
      const double s = sum_parts(part, gridDim.x);
      sc[S_PQ] = s;
      if (!(s > 0.0)) {
        sc[S_BRK] = 1.0;
      } else {
        sc[S_BRK] = 0.0;
        sc[S_ALPHA] = sc[S_RR + parity] / s;
      }
      *counter = 0;
    }
  }
}

}  // namespace lorads
