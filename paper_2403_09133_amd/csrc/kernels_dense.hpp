// Dense cost matrix: out = alpha C V + beta out over the first r columns, with
// C stored dense (n x ldc, row-major, ldc a multiple of 64, zero padding) and
// the products on the matrix cores (v_mfma_f64_16x16x4f64 in FP64,
// v_mfma_f32_16x16x4f32 in FP32).  With r small against n the product reads
// C once and is bound by that stream (r / 4 flop per byte of C in FP64), so
// the work is cut into many waves: wave (t, s) takes the 16-row tile t of C
// and the s-th range of columns k, stages 16 x 64 blocks of C in its LDS with
// 16-byte loads, and accumulates its 16 x r partial product; cdense_finish
// adds the partials of the ranges in range order (a fixed order).
#pragma once

#include "kernels.hpp"

namespace lorads {

constexpr int kDenseK = 64;     // columns of C staged per step
constexpr int kDenseNT = 4;     // 16-column tiles of V per wave (r <= 64)

template <typename T>
struct DenseMfma;
template <>
struct DenseMfma<double> {
  typedef double acc4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc4 op(double a, double b, acc4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 output tile held by accumulator element v of lane l
  static __device__ __forceinline__ int row(int l, int v) { return l / 16 + 4 * v; }
};
template <>
struct DenseMfma<float> {
  typedef float acc4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc4 op(float a, float b, acc4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l / 16) + v; }
};

// part[(s n + i) r + c] = sum over the k of range s of C[i][k] V[k][c]
template <typename T>
__global__ void __launch_bounds__(kBlock) cdense_partial(int n, int ldc, const T* __restrict__ C,
                                                         const T* __restrict__ V, int r, int ld,
                                                         int tiles, int splits, int kchunk,
                                                         T* __restrict__ part) {
  using M = DenseMfma<T>;
  typedef T vec __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int VW = 16 / (int)sizeof(T);
  constexpr int SK = kDenseK + 1;  // padded LDS row
  __shared__ T sa[kBlock / 64][16 * SK];
  const int l = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int gw = blockIdx.x * (kBlock / 64) + wid;
  if (gw >= tiles * splits) return;  // wave-uniform; no block-wide synchronisation follows
  const int t = gw / splits, sp = gw % splits;
  const int i0 = 16 * t;
  const int k0 = sp * kchunk, k1 = min(ldc, k0 + kchunk);
  const int nt = min(kDenseNT, (r + 15) / 16);
  T* a_lds = sa[wid];
  typename M::acc4 acc[kDenseNT];
#pragma unroll
  for (int q = 0; q < kDenseNT; ++q) acc[q] = typename M::acc4{0, 0, 0, 0};
  for (int kb = k0; kb < k1; kb += kDenseK) {
    // stage C[i0 .. i0 + 15][kb .. kb + 63] (rows past n read as zero)
#pragma unroll
    for (int q = 0; q < 16 * kDenseK / (64 * VW); ++q) {
      const int e = (q * 64 + l) * VW;
      const int row = e / kDenseK, kofs = e % kDenseK;
      vec v;
#pragma unroll
      for (int w = 0; w < VW; ++w) v[w] = (T)0;
      if (i0 + row < n) v = *reinterpret_cast<const vec*>(C + (size_t)(i0 + row) * ldc + kb + kofs);
#pragma unroll
      for (int w = 0; w < VW; ++w) a_lds[row * SK + kofs + w] = v[w];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
    for (int kk = 0; kk < kDenseK; kk += 4) {
      const T a = a_lds[(l & 15) * SK + kk + (l >> 4)];
      const int krow = kb + kk + (l >> 4);
#pragma unroll
      for (int q = 0; q < kDenseNT; ++q) {
        if (q < nt) {
          const int col = 16 * q + (l & 15);
          const T b = (krow < n && col < r) ? V[(size_t)krow * ld + col] : (T)0;
          acc[q] = M::op(a, b, acc[q]);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
#pragma unroll
  for (int q = 0; q < kDenseNT; ++q) {
    if (q >= nt) break;
    const int col = 16 * q + (l & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = i0 + M::row(l, v);
      if (row < n && col < r) part[((size_t)sp * n + row) * r + col] = acc[q][v];
    }
  }
}

// out[i][c] = alpha sum_s part[s][i][c] (s in order) + beta out[i][c]
template <typename T>
__global__ void __launch_bounds__(kBlock) cdense_finish(int n, int r, int splits,
                                                        const T* __restrict__ part, double alpha,
                                                        double beta, T* __restrict__ out, int ldo) {
  const size_t total = (size_t)n * r;
  for (size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * kBlock) {
    const size_t i = idx / r, c = idx % r;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += (double)part[(size_t)sp * total + idx];
    double v = alpha * s;
    if (beta != 0.0) v += beta * (double)out[i * ldo + c];
    out[i * ldo + c] = (T)v;
  }
}

}  // namespace lorads
