// Structure-specialised kernels: DIAG (A_i = a_i e_j e_j^T, MaxCut) and PAIR
// (A_i = a_i (e_j e_k^T + e_k e_j^T), matrix completion).  Same group-per-row
// mapping and deterministic reductions as the generic kernels.
#pragma once

#include "kernels.hpp"

namespace lorads {

constexpr int kMaxCols = 4;  // factor columns per lane held in registers (r <= 4 G)
constexpr int kUnroll = 4;   // incident constraints gathered per step (memory-level parallelism)

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

// PAIR forward map: a group takes a chunk of at most kPairChunk constraints
// (j, k) of one row j (contiguous in the internal order), keeps U_j, V_j in
// registers and gathers the partners kUnroll at a time:
//   z_i = a_i (<U_j, V_k> + <U_k, V_j>).
template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) k1_pair(
    int nchunks, const int* __restrict__ chunk_row, const int* __restrict__ chunk_start,
    const int* __restrict__ rptr, const int* __restrict__ pk, const T* __restrict__ pcoef,
    double pair_coef, const T* __restrict__ U, const T* __restrict__ V, int r, int ld,
    T* __restrict__ z, double scale, const double* __restrict__ lam,
    const double* __restrict__ b, double rho, double* __restrict__ w,
    const double* __restrict__ sc, int parity) {
  if (MODE == 2 && sc[S_DONE + parity] != 0.0) return;
  const int chunk = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (chunk >= nchunks) return;
  const int row = chunk_row[chunk];
  const int i0 = chunk_start[chunk], i1 = min(i0 + kPairChunk, rptr[row + 1]);
  double uj[kMaxCols], vj[kMaxCols];
#pragma unroll
  for (int t = 0; t < kMaxCols; ++t) {
    const int c = lane + t * G;
    uj[t] = c < r ? (double)U[(size_t)row * ld + c] : 0.0;
    vj[t] = c < r ? (double)V[(size_t)row * ld + c] : 0.0;
  }
  const double mult = (MODE == 2) ? sc[S_RHO] : (MODE == 0 ? scale : 1.0);
  for (int i = i0; i < i1; i += kUnroll) {
    const int cnt = min(kUnroll, i1 - i);
    int k[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) k[u] = u < cnt ? pk[i + u] : row;
    double d[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < kMaxCols; ++t) {
        const int c = lane + t * G;
        if (c < r)
          s += uj[t] * (double)V[(size_t)k[u] * ld + c] + (double)U[(size_t)k[u] * ld + c] * vj[t];
      }
      d[u] = s;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<G>(d[u]);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      // every lane holds the reduced d[u]; lane u mod G stores it
      if (lane == (u & (G - 1)) && u < cnt) {
        const int id = i + u;
        const double val = d[u] * (pcoef ? (double)pcoef[id] : pair_coef);
        if (MODE == 1) {
          z[id] = (T)val;
          w[id] = lam[id] + rho * (val - b[id]);
        } else {
          z[id] = (T)(mult * val);
        }
      }
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
    const T* __restrict__ P, double* __restrict__ sc, int parity, double* __restrict__ part) {
  const int row = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (row >= n) return;
  double acc[kMaxCols];
#pragma unroll
  for (int t = 0; t < kMaxCols; ++t) acc[t] = 0.0;
  if (c_scale != 0.0) {
    for (int e = cptr[row]; e < cptr[row + 1]; ++e) {
      const int k = ccol[e];
      const double a = c_scale * (double)cval[e];
#pragma unroll
      for (int t = 0; t < kMaxCols; ++t) {
        const int c = lane + t * G;
        if (c < r) acc[t] += a * (double)V[(size_t)k * ld + c];
      }
    }
  }
  double d = 0.0;
  if (w != nullptr)
    for (int i = dptr[row]; i < dptr[row + 1]; ++i) d += (double)w[i] * (double)dcoef[i];
#pragma unroll
  for (int t = 0; t < kMaxCols; ++t) {
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
                                                  double* __restrict__ part) {
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
  publish_partial(block_sum(pq, sh), part);
}

// ===========================================================================
// K2 PAIR, row-owner over both views (no atomics).  Row t's incident
// constraints are its view-R entries (t is the smaller index, partner pk) and
// its view-C entries (t is the larger index, partner cvj, id cvid).
//   MODE 0: out_t = out_scale (c_scale (C V)_t + sum_i w_i a_i V_partner)
//   MODE 1: fused CG operator.  For each incident constraint with partner p:
//           d_i = <Pm_t, V_p> + <Pm_p, V_t>  (= <A_i, Pm V^T>), and
//           Q_t = gamma Pm_t + rho sum_i a_i^2 d_i V_p;  accumulates <Pm, Q>.
//           (V = the fixed factor W, Pm = the CG direction.)
//   MODE 2: CG operator from precomputed w = rho A(Pm V^T):
//           Q_t = gamma Pm_t + sum_i w_i a_i V_p;  accumulates <Pm, Q>.
//           (each constraint's inner product is formed once, by the forward
//           kernel, instead of once per view)
// kUnroll incident constraints are gathered per step.
// ===========================================================================
template <typename T, int G, int MODE>
__device__ __forceinline__ void pair_batch(int cnt, const int* id, const int* p,
                                           const T* __restrict__ pcoef, double pair_coef,
                                           const T* __restrict__ w, const T* __restrict__ V,
                                           const T* __restrict__ Pm, int r, int ld, int lane,
                                           const double* pt, const double* vt, double* acc) {
  double vp[kUnroll][kMaxCols];
  double coef[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
    for (int t = 0; t < kMaxCols; ++t) {
      const int c = lane + t * G;
      vp[u][t] = (c < r) ? (double)V[(size_t)p[u] * ld + c] : 0.0;
    }
  }
  if (MODE == 1) {
    double d[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < kMaxCols; ++t) {
        const int c = lane + t * G;
        if (c < r) s += pt[t] * vp[u][t] + (double)Pm[(size_t)p[u] * ld + c] * vt[t];
      }
      d[u] = s;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<G>(d[u]);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const double a = pcoef ? (double)pcoef[id[u]] : pair_coef;
      coef[u] = u < cnt ? a * a * d[u] : 0.0;
    }
  } else {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const double a = pcoef ? (double)pcoef[id[u]] : pair_coef;
      coef[u] = u < cnt ? (double)w[id[u]] * a : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u)
#pragma unroll
    for (int t = 0; t < kMaxCols; ++t) acc[t] += coef[u] * vp[u][t];
}

template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) k2_pair(
    int n, const int* __restrict__ cptr, const int* __restrict__ ccol,
    const T* __restrict__ cval, double c_scale, const int* __restrict__ rptr,
    const int* __restrict__ pk, const int* __restrict__ cvptr, const int* __restrict__ cvj,
    const int* __restrict__ cvid, const T* __restrict__ pcoef, double pair_coef,
    const T* __restrict__ w, const T* __restrict__ V, const T* __restrict__ Pm, int r, int ld,
    T* __restrict__ out, int ldo, double out_scale, double* __restrict__ sc, int parity,
    double* __restrict__ part) {
  // one block per output row; its kBlock/G groups split the row's incident
  // constraints (kUnroll at a time) and their partial rows are summed in LDS
  // in group order
  constexpr bool kCg = (MODE == 1 || MODE == 2);
  constexpr int kBatch = (MODE == 1) ? 1 : 0;  // MODE 2 gathers like MODE 0
  constexpr int NGR = kBlock / G;
  __shared__ double sh[kBlock / 64];
  __shared__ double red[kBlock * kMaxCols];
  if (kCg && sc[S_DONE + parity] != 0.0) return;
  const int row = blockIdx.x;
  const int grp = threadIdx.x / G;
  const int lane = threadIdx.x & (G - 1);
  double acc[kMaxCols], pt[kMaxCols], vt[kMaxCols];
#pragma unroll
  for (int t = 0; t < kMaxCols; ++t) acc[t] = pt[t] = vt[t] = 0.0;
  if (kCg) {
#pragma unroll
    for (int t = 0; t < kMaxCols; ++t) {
      const int c = lane + t * G;
      if (c < r) {
        pt[t] = (double)Pm[(size_t)row * ld + c];
        if (MODE == 1) vt[t] = (double)V[(size_t)row * ld + c];
      }
    }
  }
  if (MODE == 0 && c_scale != 0.0) {
    for (int e = cptr[row] + grp; e < cptr[row + 1]; e += NGR) {
      const int k = ccol[e];
      const double a = c_scale * (double)cval[e];
#pragma unroll
      for (int t = 0; t < kMaxCols; ++t) {
        const int c = lane + t * G;
        if (c < r) acc[t] += a * (double)V[(size_t)k * ld + c];
      }
    }
  }
  if (MODE != 0 || w != nullptr) {
    const int r0 = rptr[row], nR = rptr[row + 1] - r0;
    const int c0 = cvptr[row], total = nR + (cvptr[row + 1] - c0);
    for (int q = grp * kUnroll; q < total; q += NGR * kUnroll) {
      const int cnt = min(kUnroll, total - q);
      int id[kUnroll], p[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int qq = u < cnt ? q + u : q;  // padding repeats a valid entry
        if (qq < nR) {
          id[u] = r0 + qq;
          p[u] = pk[id[u]];
        } else {
          const int e = c0 + (qq - nR);
          id[u] = cvid[e];
          p[u] = cvj[e];
        }
      }
      pair_batch<T, G, kBatch>(cnt, id, p, pcoef, pair_coef, w, V, Pm, r, ld, lane, pt, vt, acc);
    }
  }
#pragma unroll
  for (int t = 0; t < kMaxCols; ++t) red[grp * (kMaxCols * G) + t * G + lane] = acc[t];
  __syncthreads();
  double pq = 0.0;
  if (grp == 0) {
#pragma unroll
    for (int t = 0; t < kMaxCols; ++t) {
      double s = 0.0;
      for (int g = 0; g < NGR; ++g) s += red[g * (kMaxCols * G) + t * G + lane];
      acc[t] = s;
    }
    if (kCg) {
      const double gamma = sc[S_GAMMA], rho = (MODE == 1) ? sc[S_RHO] : 1.0;
#pragma unroll
      for (int t = 0; t < kMaxCols; ++t) {
        const int c = lane + t * G;
        if (c < r) {
          const T qv = (T)(gamma * pt[t] + rho * acc[t]);
          out[(size_t)row * ldo + c] = qv;
          pq += pt[t] * (double)qv;
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < kMaxCols; ++t) {
        const int c = lane + t * G;
        if (c < r) out[(size_t)row * ldo + c] = (T)(out_scale * acc[t]);
      }
    }
  }
  if (kCg) publish_partial(block_sum(pq, sh), part);
}

}  // namespace lorads
