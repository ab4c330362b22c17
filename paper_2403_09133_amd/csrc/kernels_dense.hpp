// Dense cost matrix: out = alpha C V + beta out over the first r columns, with
// C stored dense in 16 x 64 tiles (each tile one contiguous run of 1024
// entries, row-major inside; the tiles of a 16-row band in column order, ldc
// a multiple of 64, zero padding) and
// the products on the matrix cores (v_mfma_f64_16x16x4f64 in FP64,
// v_mfma_f32_16x16x4f32 in FP32).  With r small against n the product reads
// C once and is bound by that stream (r / 4 flop per byte of C in FP64), so
// the work is cut into many blocks: block (g, s) takes four or eight 16-row tiles of C
// and the s-th range of columns k, and accumulates their 16 x r partial
// products; cdense_finish adds the partials of the ranges in range order (a
// fixed order).
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

// part[(s n + i) r + c] = sum over the k of range s of C[i][k] V[k][c].
// A block of WPB waves takes WPB consecutive 16-row tiles of C (wave w the
// tile WPB g + w) and the s-th range of columns k, in 64-column steps.  Each
// step stages the 64 x (16 NT) block of V once for the WPB waves and each wave's
// 16 x 64 tile of C in LDS (one contiguous 8 KB or 4 KB run), and the loads of the
// next step are issued before this step's MFMAs, so the stream of C overlaps
// the products.  NT = ceil(r / 16) column tiles of V; a lane's operands are
// A[m][k] = C[i0 + (l & 15)][k] and B[k][j] = V[k][16 q + (l & 15)] with
// k = kb + kk + (l >> 4), the k's of a step taken in order.
template <typename T, int NT, int WPB>
__global__ void __launch_bounds__(64 * WPB) cdense_partial(int n, int ldc, const T* __restrict__ C,
                                                         const T* __restrict__ V, int r, int ld,
                                                         int tiles, int splits, int kchunk,
                                                         T* __restrict__ part) {
  using M = DenseMfma<T>;
  typedef T vec __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int VW = 16 / (int)sizeof(T);
  constexpr int SK = kDenseK + 1;        // padded LDS row of the C block
  constexpr int RC = 16 * NT;            // V columns staged
  constexpr int SV = RC + 1;             // padded LDS row of the V block
  constexpr int CQ = 16 * kDenseK / (64 * VW);   // 16-byte C loads per lane and step
  constexpr int BT = 64 * WPB;           // threads per block
  constexpr int VQ = kDenseK * RC / BT;          // V elements per thread and step
  static_assert(kDenseK * RC % BT == 0, "whole V elements per thread");
  __shared__ T sa[WPB][16 * SK];
  __shared__ T sv[kDenseK * SV];
  const int l = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int sp = blockIdx.x % splits, tg = blockIdx.x / splits;
  const int t = WPB * tg + wid;
  const bool live = t < tiles;           // wave-uniform; every wave still takes the barriers
  const int i0 = 16 * t;
  const int k0 = sp * kchunk, k1 = min(ldc, k0 + kchunk);
  // this wave's row band of tiles: a step reads one contiguous 16 x 64 tile
  const T* ctile = C + (size_t)t * 16 * ldc;
  T* a_lds = sa[wid];
  typename M::acc4 acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = typename M::acc4{0, 0, 0, 0};
  vec cr[CQ];
  T vr[VQ];
  // loads of the step at column kb into registers (rows of C past n and
  // V entries outside n x r read as zero)
  auto load_step = [&](int kb) {
#pragma unroll
    for (int q = 0; q < CQ; ++q) {
      const int e = (q * 64 + l) * VW;
      const int row = e / kDenseK, kofs = e % kDenseK;
#pragma unroll
      for (int w = 0; w < VW; ++w) cr[q][w] = (T)0;
      if (live && i0 + row < n) cr[q] = *reinterpret_cast<const vec*>(ctile + (size_t)(kb / kDenseK) * (16 * kDenseK) + e);
    }
#pragma unroll
    for (int q = 0; q < VQ; ++q) {
      const int e = q * BT + (int)threadIdx.x;
      const int row = e / RC, col = e % RC;
      vr[q] = (kb + row < n && col < r) ? V[(size_t)(kb + row) * ld + col] : (T)0;
    }
  };
  if (k0 < k1) load_step(k0);
  for (int kb = k0; kb < k1; kb += kDenseK) {
#pragma unroll
    for (int q = 0; q < CQ; ++q) {
      const int e = (q * 64 + l) * VW;
      const int row = e / kDenseK, kofs = e % kDenseK;
#pragma unroll
      for (int w = 0; w < VW; ++w) a_lds[row * SK + kofs + w] = cr[q][w];
    }
#pragma unroll
    for (int q = 0; q < VQ; ++q) {
      const int e = q * BT + (int)threadIdx.x;
      sv[(e / RC) * SV + e % RC] = vr[q];
    }
    __syncthreads();
    if (kb + kDenseK < k1) load_step(kb + kDenseK);  // in flight during the products
    if (live) {
#pragma unroll
      for (int kk = 0; kk < kDenseK; kk += 4) {
        const T a = a_lds[(l & 15) * SK + kk + (l >> 4)];
        const T* brow = sv + (kk + (l >> 4)) * SV + (l & 15);
#pragma unroll
        for (int q = 0; q < NT; ++q) acc[q] = M::op(a, brow[16 * q], acc[q]);
      }
    }
    __syncthreads();  // the blocks are read before the next step stages over them
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
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
