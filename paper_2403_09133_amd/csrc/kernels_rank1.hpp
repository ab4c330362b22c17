// Rank-one constraints: A_i = c_i a_i a_i^T with a sparse a_i (the sensor
// network localization relaxation of Section 3; the balance constraint of graph
// bisection, a = 1).  With A_i of this form
//   <A_i, U V^T> = c_i <a_i^T U, a_i^T V>,   (A*(w) V)_t = sum_i w_i c_i a_{i,t} a_i^T V,
// so every operator runs through the r-vectors a_i^T U: a segment pass (one
// lane group per segment of at most kR1Seg entries of a_i, so a dense a_i is
// shared out), a per-constraint pass that adds its segments in order, and, for
// the adjoint and the CG operator, a row pass over the constraints that touch
// each row.  Every sum has a fixed order.
#pragma once

#include "kernels.hpp"

namespace lorads {

constexpr int kR1Cols = 4;  // columns per lane held in registers (r <= 4 G)

// su[s] = sum_{e in segment s} a_e U_{idx_e}, and with TWO the same of V into sv
template <typename T, int G, int TWO>
__global__ void __launch_bounds__(kBlock) r1_seg(
    int nseg, const int* __restrict__ sstart, const int* __restrict__ idx,
    const T* __restrict__ val, const T* __restrict__ U, const T* __restrict__ V, int r, int ld,
    typename OpAcc<T>::type* __restrict__ su, typename OpAcc<T>::type* __restrict__ sv,
    const double* __restrict__ sc, int parity) {
  using A = typename OpAcc<T>::type;
  if (sc && sc[S_DONE + parity] != 0.0) return;
  const int seg = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (seg >= nseg) return;
  A au[kR1Cols], av[kR1Cols];
#pragma unroll
  for (int t = 0; t < kR1Cols; ++t) au[t] = av[t] = 0;
  for (int e = sstart[seg]; e < sstart[seg + 1]; ++e) {
    const size_t k = (size_t)idx[e] * ld;
    const A a = (A)val[e];
#pragma unroll
    for (int t = 0; t < kR1Cols; ++t) {
      const int c = lane + t * G;
      if (c < r) {
        au[t] += a * (A)U[k + c];
        if (TWO) av[t] += a * (A)V[k + c];
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kR1Cols; ++t) {
    const int c = lane + t * G;
    if (c < r) {
      su[(size_t)seg * r + c] = au[t];
      if (TWO) sv[(size_t)seg * r + c] = av[t];
    }
  }
}

// Per constraint i (segments cseg[i] .. cseg[i + 1] - 1 added in order into
// the r-vectors u = a_i^T U, v = a_i^T V):
//   MODE 0: z_i = scale c_i <u, v>
//   MODE 1: z_i = c_i <u, v> and w_i = lam_i + rho (z_i - b_i)        (FP64)
//   MODE 2: S_i = u and coef_i = c_i w_i                 (adjoint; V unused)
//   MODE 3: S_i = v (of W) and coef_i = sc[S_RHO] c_i^2 <u, v> (u of the
//           direction): the CG operator's weight of row S_i
template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) r1_con(
    int m, const int* __restrict__ cseg, const double* __restrict__ cc,
    const typename OpAcc<T>::type* __restrict__ su, const typename OpAcc<T>::type* __restrict__ sv,
    int r, T* __restrict__ z, double scale, const double* __restrict__ lam,
    const double* __restrict__ b, double rho, double* __restrict__ wout, const T* __restrict__ w,
    typename OpAcc<T>::type* __restrict__ S, typename OpAcc<T>::type* __restrict__ coef,
    const double* __restrict__ sc, int parity) {
  using A = typename OpAcc<T>::type;
  if (MODE == 3 && sc[S_DONE + parity] != 0.0) return;
  const int i = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (i >= m) return;
  A u[kR1Cols], v[kR1Cols];
#pragma unroll
  for (int t = 0; t < kR1Cols; ++t) u[t] = v[t] = 0;
  for (int g = cseg[i]; g < cseg[i + 1]; ++g) {
#pragma unroll
    for (int t = 0; t < kR1Cols; ++t) {
      const int c = lane + t * G;
      if (c < r) {
        u[t] += su[(size_t)g * r + c];
        if (MODE != 2) v[t] += sv[(size_t)g * r + c];
      }
    }
  }
  if (MODE == 2) {
#pragma unroll
    for (int t = 0; t < kR1Cols; ++t) {
      const int c = lane + t * G;
      if (c < r) S[(size_t)i * r + c] = u[t];
    }
    if (lane == 0) coef[i] = (A)(cc[i] * (double)w[i]);
    return;
  }
  double d = 0.0;
#pragma unroll
  for (int t = 0; t < kR1Cols; ++t) d += (double)u[t] * (double)v[t];
  d = group_sum<G>(d);
  if (MODE == 3) {
#pragma unroll
    for (int t = 0; t < kR1Cols; ++t) {
      const int c = lane + t * G;
      if (c < r) S[(size_t)i * r + c] = v[t];
    }
    if (lane == 0) coef[i] = (A)(sc[S_RHO] * cc[i] * cc[i] * d);
    return;
  }
  if (lane == 0) {
    const double zi = cc[i] * d;
    if (MODE == 1) {
      z[i] = (T)zi;
      wout[i] = lam[i] + rho * (zi - b[i]);
    } else {
      z[i] = (T)(scale * zi);
    }
  }
}

// Row pass: acc_t = c_scale (C V)_t + sum_{i touching t} coef_i a_{i,t} S_i
//   MODE 0: out_t = out_scale acc_t               (adjoint; coef null: C alone)
//   MODE 1: Q_t = gamma P_t + acc_t, with the block partials of <P, Q> (CG)
template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) r1_rows(
    int n, const int* __restrict__ cptr, const int* __restrict__ ccol,
    const T* __restrict__ cval, double c_scale, const int* __restrict__ tptr,
    const int* __restrict__ tcon, const T* __restrict__ tval,
    const typename OpAcc<T>::type* __restrict__ coef, const typename OpAcc<T>::type* __restrict__ S,
    const T* __restrict__ V, int r, int ld, T* __restrict__ out, int ldo, double out_scale,
    const T* __restrict__ P, const double* __restrict__ sc, int parity, double* __restrict__ part) {
  using A = typename OpAcc<T>::type;
  __shared__ double sh[kBlock / 64];
  if (MODE == 1 && sc[S_DONE + parity] != 0.0) return;
  const int row = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  double acc[kR1Cols];
#pragma unroll
  for (int t = 0; t < kR1Cols; ++t) acc[t] = 0.0;
  double pq = 0.0;
  if (row < n) {
    if (MODE == 0 && c_scale != 0.0) {
      for (int e = cptr[row]; e < cptr[row + 1]; ++e) {
        const size_t k = (size_t)ccol[e] * ld;
        const double a = c_scale * (double)cval[e];
#pragma unroll
        for (int t = 0; t < kR1Cols; ++t) {
          const int c = lane + t * G;
          if (c < r) acc[t] += a * (double)V[k + c];
        }
      }
    }
    if (coef != nullptr) {
      for (int e = tptr[row]; e < tptr[row + 1]; ++e) {
        const int i = tcon[e];
        const double a = (double)coef[i] * (double)tval[e];
#pragma unroll
        for (int t = 0; t < kR1Cols; ++t) {
          const int c = lane + t * G;
          if (c < r) acc[t] += a * (double)S[(size_t)i * r + c];
        }
      }
    }
    if (MODE == 1) {
      const double gamma = sc[S_GAMMA];
#pragma unroll
      for (int t = 0; t < kR1Cols; ++t) {
        const int c = lane + t * G;
        if (c < r) {
          const double p = (double)P[(size_t)row * ld + c];
          const T q = (T)(gamma * p + acc[t]);
          out[(size_t)row * ldo + c] = q;
          pq += p * (double)q;
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < kR1Cols; ++t) {
        const int c = lane + t * G;
        if (c < r) out[(size_t)row * ldo + c] = (T)(out_scale * acc[t]);
      }
    }
  }
  if (MODE == 1) publish_partial(block_sum(pq, sh), part);
}

}  // namespace lorads
