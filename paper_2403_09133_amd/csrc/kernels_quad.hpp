// The quadratic objective f(X) = <C, X> + (mu / 2) ||X||_F^2 (Section 1's
// convex f).  With X = U V^T its gradient applied to a factor is
// C W + mu U (V^T W), so every extra term is a product with an r x r Gram
// matrix: the Phase I gradient gains 2 mu U (U^T U), the exact line search's
// quartic gains the terms of ||A0 + a A1 + a^2 A2||_F^2 (A0 = U^T U,
// A1 = U^T D + D^T U, A2 = D^T D), and the ADMM subproblem operator gains
// mu P (W^T W) with -mu W (W^T W) in its right-hand side.  Every sum has a
// fixed order.
#pragma once

#include "kernels.hpp"

namespace lorads {

constexpr int kGramBlocks = 256;  // row blocks of the Gram partials

// part[b][k][c] = sum over rows i = b, b + B, ... of X[i][k] Y[i][c]
// (X: n x ra, Y: n x rb)
template <typename T>
__global__ void __launch_bounds__(kBlock) gram_rr_partial(int n, int ra, int rb, const T* __restrict__ X,
                                                          int ldx, const T* __restrict__ Y, int ldy,
                                                          double* __restrict__ part) {
  const int rr = ra * rb;
  for (int kc = threadIdx.x; kc < rr; kc += kBlock) {
    const int k = kc / rb, c = kc % rb;
    double s = 0.0;
    for (int i = blockIdx.x; i < n; i += gridDim.x)
      s += (double)X[(size_t)i * ldx + k] * (double)Y[(size_t)i * ldy + c];
    part[(size_t)blockIdx.x * rr + kc] = s;
  }
}

// G[k][c] = sum_b part[b][k][c] (b in order), G of rr = ra rb entries
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) gram_rr_finish(int rr, int nb, const double* __restrict__ part,
                                                         double* __restrict__ G) {
  for (int kc = blockIdx.x * kBlock + threadIdx.x; kc < rr; kc += gridDim.x * kBlock) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * rr + kc];
    G[kc] = s;
  }
}

// out[i][c] += alpha sum_{k < r} X[i][k] G[k][c] for the first rc columns
// (G: r x rc row-major)
template <typename TX, typename TO>
__global__ void __launch_bounds__(kBlock) add_xg(int n, int r, int rc, const TX* __restrict__ X, int ldx,
                                                 const double* __restrict__ G, double alpha,
                                                 TO* __restrict__ out, int ldo) {
  const size_t total = (size_t)n * rc;
  for (size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * kBlock) {
    const size_t i = idx / rc;
    const int c = (int)(idx % rc);
    double s = 0.0;
    for (int k = 0; k < r; ++k) s += (double)X[i * ldx + k] * G[k * rc + c];
    out[i * ldo + c] = (TO)((double)out[i * ldo + c] + alpha * s);
  }
}

// CG operator term: Q += mu P G (G = W^T W), with the block partials of
// <P, mu P G> after the operator's own (the caller adds their count); skipped
// once the CG has converged
template <typename T>
__global__ void __launch_bounds__(kBlock) cg_quad(int n, int r, int ld, const T* __restrict__ Pd,
                                                  const double* __restrict__ G, double mu,
                                                  T* __restrict__ Q, const double* __restrict__ sc,
                                                  int parity, double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  if (sc[S_DONE + parity] != 0.0) return;  // block-uniform
  const size_t total = (size_t)n * r;
  double acc = 0.0;
  for (size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * kBlock) {
    const size_t i = idx / r;
    const int c = (int)(idx % r);
    double s = 0.0;
    for (int k = 0; k < r; ++k) s += (double)Pd[i * ld + k] * G[k * r + c];
    const double q = mu * s;
    Q[i * ld + c] = (T)((double)Q[i * ld + c] + q);
    acc += (double)Pd[i * ld + c] * q;
  }
  publish_partial(block_sum(acc, sh), part);
}

// The quartic's Gram terms from A0 = U^T U, B = U^T D and A2 = D^T D
// (A1 = B + B^T): sc[slot + 0..3] = <A0, A1>, ||A1||^2 + 2 <A0, A2>,
// <A1, A2>, ||A2||^2.  One block.
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) quad_coefs(int r, const double* __restrict__ A0,
                                                     const double* __restrict__ B,
                                                     const double* __restrict__ A2,
                                                     double* __restrict__ sc, int slot) {
  __shared__ double sh[kBlock / 64];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int kc = threadIdx.x; kc < r * r; kc += kBlock) {
    const int k = kc / r, c = kc % r;
    const double a0 = A0[kc], a1 = B[kc] + B[c * r + k], a2 = A2[kc];
    s[0] += a0 * a1;
    s[1] += a1 * a1 + 2.0 * a0 * a2;
    s[2] += a1 * a2;
    s[3] += a2 * a2;
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double v = block_sum(s[t], sh);
    if (threadIdx.x == 0) sc[slot + t] = v;
  }
}

}  // namespace lorads
