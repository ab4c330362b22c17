// Device kernels of the LoRADS hot path for gfx950 (wave64).
//
// Factor matrices are row-major (row j = the r-vector of node j).  A row is
// handled by a group of G lanes (G = power of two >= r, at most 64); lane c of
// the group owns columns c, c + G, ...  Reductions inside a group use wave
// shuffles (xor butterflies never leave an aligned group), reductions across a
// grid use per-block partial sums finished by a one-block kernel, so every sum
// has a fixed order and results are bitwise reproducible run to run.
#pragma once

#include "common.hpp"

namespace lorads {

// Lane exchange inside a 16-lane row by a DPP move (a VALU operation, so it
// does not queue on the CU's LDS pipeline the way a bpermute shuffle does).
// CTRL: 0xB1 swaps lanes 2k <-> 2k+1, 0x4E swaps pairs inside a quad,
// 0x141 mirrors each half-row (i <-> 7 - i), 0x140 mirrors the row (i <-> 15 - i).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over an aligned group of G lanes (G a power of two <= 64); every lane of
// the group receives the same value.  Up to 16 lanes: DPP swaps and mirrors
// (after each step a lane holds the sum of its aligned block, and a mirror
// pairs every lane with one in the other half of the doubled block; a + b and
// b + a round alike, so all lanes agree bit for bit).  Wider groups finish
// with xor shuffles across rows.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if (G >= 2) v += dpp_move<0xB1>(v);
  if (G >= 4) v += dpp_move<0x4E>(v);
  if (G >= 8) v += dpp_move<0x141>(v);
  if (G >= 16) v += dpp_move<0x140>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Arithmetic type of the per-constraint products of the operator kernels:
// the element type itself (the FP32 form computes its operator in FP32;
// the scalars of CG and every solver decision stay FP64).
template <typename T> struct OpAcc { using type = double; };
template <> struct OpAcc<float> { using type = float; };

template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if (G >= 2) v += dpp_move<0xB1>(v);
  if (G >= 4) v += dpp_move<0x4E>(v);
  if (G >= 8) v += dpp_move<0x141>(v);
  if (G >= 16) v += dpp_move<0x140>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Every reduction kernel runs in blocks of kBlock = 256 threads (4 waves).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  // wave reduction then across the 4 waves of the block
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) t += sh[i];
  }
  return t;  // valid in thread 0
}

// Position of element i of a row-major (stride ld) array inside rows of stride
// 2 ld (32-bit division whenever the index fits).
__device__ __forceinline__ size_t interleaved_index(size_t i, int ld) {
  if (i <= 0xffffffffu) {
    const unsigned iu = (unsigned)i, lu = (unsigned)ld;
    return (size_t)(iu / lu) * 2u * lu + iu % lu;
  }
  return (i / ld) * 2 * ld + i % ld;
}

// Grid reductions are two-stage: every block stores its partial (plain store,
// thread 0 holds the block's value) and a one-block finishing kernel sums the
// partials in index order.  The kernel boundary makes the partials visible
// across XCDs without device-scope fences in the producing kernels.
__device__ __forceinline__ void publish_partial(double partial, double* part) {
  if (threadIdx.x == 0) part[blockIdx.x] = partial;
}

// Sum of part[0..n) by the whole block (strided per thread, then the block
// tree): a fixed order for a given n and block size.  Result in thread 0.
// A thread issues the loads of eight of its strided elements before adding
// them in index order, so a long partial array costs few memory round trips.
__device__ __forceinline__ double block_sum_parts(const double* part, int n, double* sh) {
  double s = 0.0;
  constexpr int bs = kBlock;
  int i = threadIdx.x;
  for (; i + 7 * bs < n; i += 8 * bs) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[i + u * bs];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  if (i + 3 * bs < n) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = part[i + u * bs];
#pragma unroll
    for (int u = 0; u < 4; ++u) s += v[u];
    i += 4 * bs;
  }
  for (; i < n; i += bs) s += part[i];
  return block_sum(s, sh);
}

// The value block_sum_parts returns in a block of kBlock = 256 threads,
// computed by one wave (so the waves of a block can finish several arrays at
// once): lane l plays threads l, l + 64, l + 128 and l + 192, each summing its
// strided elements in index order, then each virtual wave's xor tree, then the
// four wave totals in wave order.  Same operations in the same order, so the
// same bits; every lane returns the value.
__device__ __forceinline__ double wave_sum_parts(const double* part, int n) {
  static_assert(kBlock == 256, "emulates a block of four waves");
  const int l = threadIdx.x & 63;
  double w[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double s = 0.0;
    for (int i = 64 * v + l; i < n; i += kBlock) s += part[i];
    w[v] = s;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w[v] += __shfl_xor(w[v], o, 64);
  }
  double t = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) t += w[v];
  return t;
}

// wave_sum_parts for n <= 2 kBlock in two steps, so that a wave can issue the
// loads of several arrays before it sums any: load_parts2 fetches a lane's
// (at most) two elements of each virtual thread, sum_parts2 adds them in
// index order and finishes as wave_sum_parts does.
struct Parts2 {
  double x[4][2];
};
__device__ __forceinline__ Parts2 load_parts2(const double* part, int n) {
  const int l = threadIdx.x & 63;
  Parts2 q;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 64 * v + l;
    q.x[v][0] = i < n ? part[i] : 0.0;
    q.x[v][1] = i + kBlock < n ? part[i + kBlock] : 0.0;
  }
  return q;
}
__device__ __forceinline__ double sum_parts2(const Parts2& q, int n) {
  const int l = threadIdx.x & 63;
  double w[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 64 * v + l;
    double s = 0.0;
    if (i < n) s += q.x[v][0];
    if (i + kBlock < n) s += q.x[v][1];
    w[v] = s;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) w[v] += __shfl_xor(w[v], o, 64);
  }
  double t = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) t += w[v];
  return t;
}

// block_sum_parts for n <= kWideParts kBlock with all of a thread's loads
// issued before its additions (one memory round trip; the same additions in
// the same order, so the same value)
constexpr int kWideParts = 24;
__device__ __forceinline__ double block_sum_parts_wide(const double* part, int n, double* sh) {
  double v[kWideParts];
#pragma unroll
  for (int u = 0; u < kWideParts; ++u) {
    const int i = threadIdx.x + u * kBlock;
    v[u] = i < n ? part[i] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kWideParts; ++u)
    if ((int)threadIdx.x + u * kBlock < n) s += v[u];
  return block_sum(s, sh);
}

// Copies count (<= 64) slot values to host-mapped words 1 .. count, then,
// after a system-scope fence, the sequence number to word 0; the host waits
// for that number instead of for the stream.
[[maybe_unused]] static __global__ void __launch_bounds__(64) publish_slots(
    const double* __restrict__ src, int count, double* dst, long long seq) {
  const int i = threadIdx.x;
  if (i < count) dst[1 + i] = src[i];
  __threadfence_system();
  __syncthreads();
  if (i == 0) __atomic_store_n(reinterpret_cast<long long*>(dst), seq, __ATOMIC_RELEASE);
}

// sc[slot + t] = scale * sum of partial array t (t < k), arrays of length np
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) finish_slots(int np, int k, const double* __restrict__ part,
                                                       double scale, double* __restrict__ sc, int slot) {
  __shared__ double sh[kBlock / 64];
  for (int t = 0; t < k; ++t) {
    const double v = block_sum_parts(part + (size_t)t * np, np, sh);
    if (threadIdx.x == 0) sc[slot + t] = scale * v;
  }
}

// CG step length from the operator's <P, Q> partials: alpha = ||R||^2 / <P, Q>,
// or the breakdown flag when <P, Q> <= 0.  Skipped once converged.
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) cg_alpha_finish(int np, const double* __restrict__ part,
                                                          double* __restrict__ sc, int parity) {
  __shared__ double sh[kBlock / 64];
  if (sc[S_DONE + parity] != 0.0) return;
  const double s = np <= kWideParts * kBlock ? block_sum_parts_wide(part, np, sh)
                                             : block_sum_parts(part, np, sh);
  if (threadIdx.x == 0) {
    sc[S_PQ] = s;
    if (!(s > 0.0)) {
      sc[S_BRK] = 1.0;
    } else {
      sc[S_BRK] = 0.0;
      sc[S_ALPHA] = sc[S_RR + parity] / s;
    }
  }
}

// ===========================================================================
// K1 (generic): forward map z_i = <A_i, U V^T> over the constraint-CSR.
//   MODE 0: z = scale * A(U V^T)
//   MODE 1: z = A(U V^T), w = lam + rho (z - b)          (FP64 z, w)
//   MODE 2: z = sc[S_RHO] * A(U V^T), skipped once the CG has converged
// One group of G lanes per constraint; lanes split the r columns.
// ===========================================================================
template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) k1_generic(
    int m, const int* __restrict__ kptr, const int* __restrict__ krow,
    const int* __restrict__ kcol, const T* __restrict__ kval, const T* __restrict__ U,
    const T* __restrict__ V, int r, int ld, T* __restrict__ z, double scale,
    const double* __restrict__ lam, const double* __restrict__ b, double rho,
    double* __restrict__ w, const double* __restrict__ sc, int parity) {
  if (MODE == 2 && sc[S_DONE + parity] != 0.0) return;
  const int gid = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (gid >= m) return;
  double acc = 0.0;
  const int e0 = kptr[gid], e1 = kptr[gid + 1];
  // a long constraint (the trace row of a theta SDP, a dense a_i) takes its
  // triplets eight at a time with every load of the eight issued first; the
  // sums are formed triplet by triplet in the order of the one-at-a-time loop
  constexpr int B = 8;
  int e = e0;
  for (; e + B <= e1; e += B) {
    int j[B], k[B];
    double a[B], sv[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      j[u] = krow[e + u];
      k[u] = kcol[e + u];
      a[u] = (double)kval[e + u];
      sv[u] = 0.0;
    }
    for (int c = lane; c < r; c += G) {
      double x1[B], y1[B], x2[B], y2[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        x1[u] = (double)U[(size_t)j[u] * ld + c];
        y1[u] = (double)V[(size_t)k[u] * ld + c];
        x2[u] = (double)U[(size_t)k[u] * ld + c];
        y2[u] = (double)V[(size_t)j[u] * ld + c];
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        sv[u] += x1[u] * y1[u];
        if (j[u] != k[u]) sv[u] += x2[u] * y2[u];
      }
    }
#pragma unroll
    for (int u = 0; u < B; ++u) acc += a[u] * sv[u];
  }
  for (; e < e1; ++e) {
    const int j = krow[e], k = kcol[e];
    const double a = (double)kval[e];
    double s = 0.0;
    for (int c = lane; c < r; c += G) {
      s += (double)U[(size_t)j * ld + c] * (double)V[(size_t)k * ld + c];
      if (j != k) s += (double)U[(size_t)k * ld + c] * (double)V[(size_t)j * ld + c];
    }
    acc += a * s;
  }
  acc = group_sum<G>(acc);
  if (lane == 0) {
    if (MODE == 0) {
      z[gid] = (T)(scale * acc);
    } else if (MODE == 1) {
      z[gid] = (T)acc;
      w[gid] = lam[gid] + rho * (acc - b[gid]);
    } else {
      z[gid] = (T)(sc[S_RHO] * acc);
    }
  }
}

// ===========================================================================
// K2 (generic): out = out_scale * (c_scale C + A*(w)) V over row-CSRs of C and of
// the adjoint (entries (col, constraint, coef)).  One group per output row.
//   MODE 0: plain adjoint product
//   MODE 1: CG operator epilogue: out = gamma P + A*(w) V (w already holds
//           rho * A(P W^T)); per-block partials of <P, out> for the step
//           length (cg_alpha_finish).
// ===========================================================================
template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock) k2_generic(
    int n, const int* __restrict__ cptr, const int* __restrict__ ccol,
    const T* __restrict__ cval, double c_scale, const int* __restrict__ aptr,
    const int* __restrict__ acol, const int* __restrict__ acon, const T* __restrict__ aval,
    const T* __restrict__ w, const T* __restrict__ V, int r, int ld, T* __restrict__ out,
    int ldo, double out_scale,
    // MODE 1
    const T* __restrict__ P, double* __restrict__ sc, int parity, double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  if (MODE == 1 && sc[S_DONE + parity] != 0.0) return;
  const int row = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  constexpr int MAXC = 4;  // columns per lane held in registers (r <= 4 G)
  double acc[MAXC];
#pragma unroll
  for (int t = 0; t < MAXC; ++t) acc[t] = 0.0;
  double pq = 0.0;
  if (row < n) {
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
    for (int e = aptr[row]; w != nullptr && e < aptr[row + 1]; ++e) {
      const int k = acol[e];
      const double a = (double)w[acon[e]] * (double)aval[e];
#pragma unroll
      for (int t = 0; t < MAXC; ++t) {
        const int c = lane + t * G;
        if (c < r) acc[t] += a * (double)V[(size_t)k * ld + c];
      }
    }
    if (MODE == 1) {
      const double gamma = sc[S_GAMMA];
#pragma unroll
      for (int t = 0; t < MAXC; ++t) {
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
      for (int t = 0; t < MAXC; ++t) {
        const int c = lane + t * G;
        if (c < r) out[(size_t)row * ldo + c] = (T)(out_scale * acc[t]);
      }
    }
  }
  if (MODE == 1) publish_partial(block_sum(pq, sh), part);
}

// ===========================================================================
// CG vector steps on dense N = n r element buffers.
// ===========================================================================
// P = R, ||R||^2 -> S_RR0, S_RR(parity 0); clears the flags.
template <typename T>
__global__ void __launch_bounds__(kBlock) cg_init(size_t N, const T* __restrict__ R,
                                                  T* __restrict__ P, double* __restrict__ part,
                                                  T* __restrict__ P2, int ld) {
  // P2 (optional): second copy of P in rows of stride 2 ld (interleaved with W)
  __shared__ double sh[kBlock / 64];
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
    const T v = R[i];
    P[i] = v;
    if (P2) P2[interleaved_index(i, ld)] = v;
    s += (double)v * (double)v;
  }
  publish_partial(block_sum(s, sh), part);
}

[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) cg_init_finish(int np, const double* __restrict__ part,
                                                         double tol2, double* __restrict__ sc) {
  __shared__ double sh[kBlock / 64];
  const double rr = block_sum_parts(part, np, sh);
  if (threadIdx.x == 0) {
    sc[S_RR0] = rr;
    sc[S_RR + 0] = rr;
    sc[S_RR + 1] = rr;
    sc[S_DONE + 0] = (rr <= 0.0) ? 1.0 : 0.0;
    sc[S_DONE + 1] = sc[S_DONE + 0];
    sc[S_BRK] = 0.0;
    sc[S_ITERS] = 0.0;
    sc[S_TOL2] = tol2;
  }
}

// X += alpha P; R -= alpha Q; ||R||^2 -> next parity slot; convergence flag.
template <typename T>
__global__ void __launch_bounds__(kBlock) cg_update(size_t N, T* __restrict__ X,
                                                    T* __restrict__ R, const T* __restrict__ P,
                                                    const T* __restrict__ Q,
                                                    const double* __restrict__ sc, int parity,
                                                    double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  // the first element is loaded before the flags and the step length arrive
  const size_t i0 = (size_t)blockIdx.x * kBlock + threadIdx.x, stride = (size_t)gridDim.x * kBlock;
  T x0 = 0, r0 = 0, p0 = 0, q0 = 0;
  if (i0 < N) {
    x0 = X[i0];
    r0 = R[i0];
    p0 = P[i0];
    q0 = Q[i0];
  }
  const bool skip = sc[S_DONE + parity] != 0.0 || sc[S_BRK] != 0.0;
  double s = 0.0;
  if (!skip) {
    const double alpha = sc[S_ALPHA];
    auto step = [&](size_t i, T xv, T rv0, T pv, T qv) {
      X[i] = (T)((double)xv + alpha * (double)pv);
      const T rv = (T)((double)rv0 - alpha * (double)qv);
      R[i] = rv;
      s += (double)rv * (double)rv;
    };
    if (i0 < N) step(i0, x0, r0, p0, q0);
    for (size_t i = i0 + stride; i < N; i += stride) step(i, X[i], R[i], P[i], Q[i]);
  }
  if (!skip) publish_partial(block_sum(s, sh), part);
}

// P = R + beta P (skipped once converged).  Every block sums the np partials
// of ||R||^2 left by cg_update (block_sum_parts: one fixed order), so all
// blocks hold the same beta = ||R_new||^2 / ||R||^2.  Block 0 also records
// ||R_new||^2 in the next parity slot, beta, the iteration count and the
// convergence flag; a converged or broken-down solve carries its flag forward.
// Block 0 writes only slots of the next parity, which no block here reads.
template <typename T>
__global__ void __launch_bounds__(kBlock) cg_direction(size_t N, const T* __restrict__ R,
                                                       T* __restrict__ P,
                                                       double* __restrict__ sc,
                                                       int parity, T* __restrict__ P2, int ld,
                                                       int np, const double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  __shared__ double s_beta;
  const int q = parity ^ 1;
  // the first element is loaded while beta is being formed
  const size_t i0 = (size_t)blockIdx.x * kBlock + threadIdx.x, stride = (size_t)gridDim.x * kBlock;
  T r0 = 0, p0 = 0;
  if (i0 < N) {
    r0 = R[i0];
    p0 = P[i0];
  }
  if (sc[S_DONE + parity] != 0.0 || sc[S_BRK] != 0.0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[S_DONE + q] = 1.0;
      sc[S_RR + q] = sc[S_RR + parity];
    }
    return;
  }
  const double rr = block_sum_parts(part, np, sh);
  if (threadIdx.x == 0) {
    const double b = rr / sc[S_RR + parity];
    s_beta = b;
    if (blockIdx.x == 0) {
      sc[S_BETA] = b;
      sc[S_RR + q] = rr;
      sc[S_ITERS] += 1.0;
      sc[S_DONE + q] = (rr <= sc[S_TOL2] * sc[S_RR0]) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  const double beta = s_beta;
  auto step = [&](size_t i, T rv, T pv) {
    const T v = (T)((double)rv + beta * (double)pv);
    P[i] = v;
    if (P2) P2[interleaved_index(i, ld)] = v;
  };
  if (i0 < N) step(i0, r0, p0);
  for (size_t i = i0 + stride; i < N; i += stride) step(i, R[i], P[i]);
}

// ===========================================================================
// generic dense helpers
// ===========================================================================
// per-block partials of <X, Y> over N elements (fixed grid -> fixed order)
template <typename TX, typename TY>
__global__ void __launch_bounds__(kBlock) dot_kernel(size_t N, const TX* __restrict__ X,
                                                     const TY* __restrict__ Y,
                                                     double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock)
    s += (double)X[i] * (double)Y[i];
  publish_partial(block_sum(s, sh), part);
}

// per-block partials of <X, Y> over the first r columns of n rows stored with
// stride ld: element i of the compact order is visited by the thread that
// visits it in dot_kernel over n r elements, so for the same grid the partials
// (and the finished dot) equal those of the compact layout bit for bit
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) dot_rows_kernel(unsigned N, int r, int ld,
                                                          const double* __restrict__ X,
                                                          const double* __restrict__ Y,
                                                          double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double s = 0.0;
  for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    const size_t q = (size_t)(i / (unsigned)r) * ld + i % (unsigned)r;
    s += X[q] * Y[q];
  }
  publish_partial(block_sum(s, sh), part);
}

// ---------------------------------------------------------------------------
// Fused passes of the L-BFGS two-loop recursion and step.  Each visits the
// first r columns of n rows (stride ld) in the compact order of
// dot_rows_kernel (same grid), evaluates the same elementwise expressions as
// axpby / axpby_dev / axpby_slots / add_kernel, and writes the block partials
// of its dots to part + t * gridDim.x, so every value equals that of the
// unfused sequence bit for bit.  Padding columns are not touched (they are
// zero in every factor-shaped array and stay zero).
// ---------------------------------------------------------------------------
__device__ __forceinline__ size_t compact_to_row(unsigned i, int r, int ld) {
  return (size_t)(i / (unsigned)r) * ld + i % (unsigned)r;
}

// partials of <X_t, Y_t>, t < k <= 3
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) dots3_kernel(
    unsigned N, int r, int ld, const double* __restrict__ X0, const double* __restrict__ Y0,
    const double* __restrict__ X1, const double* __restrict__ Y1, const double* __restrict__ X2,
    const double* __restrict__ Y2, int k, double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    const size_t q = compact_to_row(i, r, ld);
    s0 += X0[q] * Y0[q];
    if (k > 1) s1 += X1[q] * Y1[q];
    if (k > 2) s2 += X2[q] * Y2[q];
  }
  publish_partial(block_sum(s0, sh), part);
  if (k > 1) publish_partial(block_sum(s1, sh), part + gridDim.x);
  if (k > 2) publish_partial(block_sum(s2, sh), part + 2 * gridDim.x);
}

// The previous pass's sums, finished by every block of the next pass instead
// of a one-block finishing launch: sum t (t < k <= 3) of the np partials at
// part + t * np, times its scale, belongs in slot q[t].  The scale is s[t], or
// 1 / sc[dv[t]] when dv[t] >= 0 (the reciprocal of a stored sum, rounded as a
// division on the host would round it).
struct PrevSums {
  const double* part;
  int np, k;
  double s[3];
  int q[3];
  int dv[3];
};

// Every block sums the partials with block_sum_parts (one fixed order), so
// all blocks hold the same values; block 0 stores them in their slots for
// later passes and the host.  The values are returned in vals (LDS).
__device__ __forceinline__ void prev_finish(const PrevSums& p, double* __restrict__ sc,
                                            double* vals, double* sh) {
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (t < p.k) {
      const double v = block_sum_parts(p.part + (size_t)t * p.np, p.np, sh);
      if (threadIdx.x == 0) {
        const double scale = p.dv[t] >= 0 ? 1.0 / sc[p.dv[t]] : p.s[t];
        const double val = scale * v;
        vals[t] = val;
        if (blockIdx.x == 0) sc[p.q[t]] = val;
      }
    }
  }
  __syncthreads();
}

// a slot's value: the previous pass's sum when it produces that slot (block 0
// may be writing it during this launch), else the stored value
__device__ __forceinline__ double slot_value(const PrevSums& p, const double* vals,
                                             const double* __restrict__ sc, int slot) {
#pragma unroll
  for (int t = 0; t < 3; ++t)
    if (t < p.k && p.q[t] == slot) return vals[t];
  return sc[slot];  // not written during this launch
}

// first loop: y = (sign sc[slot]) x + 1.0 yin (yin = y, or G before q exists);
// with scale, then y = (sc[sa] / sc[sb]) y + 0.0 y; partials of <u, y>
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) lbfgs_first_kernel(
    unsigned N, int r, int ld, double* __restrict__ sc, int slot, double sign,
    const double* __restrict__ x, const double* yin, double* y, int scale, int sa, int sb,
    const double* __restrict__ u, double* __restrict__ part, PrevSums prev) {
  __shared__ double sh[kBlock / 64];
  __shared__ double vals[3];
  // the first element's operands are loaded while the previous pass's sums
  // are being finished
  const unsigned i0 = blockIdx.x * kBlock + threadIdx.x, stride = gridDim.x * kBlock;
  size_t q0 = 0;
  double x0 = 0.0, y0 = 0.0, u0 = 0.0;
  if (i0 < N) {
    q0 = compact_to_row(i0, r, ld);
    x0 = x[q0];
    y0 = yin[q0];
    u0 = u[q0];
  }
  prev_finish(prev, sc, vals, sh);
  const double a = sign * slot_value(prev, vals, sc, slot);
  const double a2 = scale ? slot_value(prev, vals, sc, sa) / slot_value(prev, vals, sc, sb) : 0.0;
  const double b = 1.0;
  double s = 0.0;
  auto step = [&](size_t q, double xv, double yv, double uv) {
    double v = (double)(a * xv + b * yv);
    if (scale) v = (double)(a2 * v + 0.0 * v);
    y[q] = v;
    s += uv * v;
  };
  if (i0 < N) step(q0, x0, y0, u0);
  for (unsigned i = i0 + stride; i < N; i += stride) {
    const size_t q = compact_to_row(i, r, ld);
    step(q, x[q], yin[q], u[q]);
  }
  publish_partial(block_sum(s, sh), part);
}

// second loop: y = (sc[sa] - sc[sb]) x + 1.0 y (x == null: y unchanged); then
// either partials of <u, y>, or (d given) d = -1.0 y + 0.0 d and partials of <g, d>
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) lbfgs_second_kernel(
    unsigned N, int r, int ld, double* __restrict__ sc, int sa, int sb,
    const double* __restrict__ x, const double* yin, double* y, const double* __restrict__ u,
    double* __restrict__ d, const double* __restrict__ g, double* __restrict__ part,
    PrevSums prev) {
  __shared__ double sh[kBlock / 64];
  __shared__ double vals[3];
  // the first element's operands are loaded while the previous pass's sums
  // are being finished (o: u's element, or g's when d is formed)
  const unsigned i0 = blockIdx.x * kBlock + threadIdx.x, stride = gridDim.x * kBlock;
  size_t q0 = 0;
  double x0 = 0.0, y0 = 0.0, o0 = 0.0;
  if (i0 < N) {
    q0 = compact_to_row(i0, r, ld);
    y0 = yin[q0];
    if (x) x0 = x[q0];
    o0 = d ? g[q0] : u[q0];
  }
  prev_finish(prev, sc, vals, sh);
  const double a = x ? slot_value(prev, vals, sc, sa) - slot_value(prev, vals, sc, sb) : 0.0;
  const double b = 1.0;
  double s = 0.0;
  auto step = [&](size_t q, double xv, double yv, double ov) {
    double v = yv;
    if (x) {
      v = (double)(a * xv + b * v);
      y[q] = v;
    }
    // the dot's operands are chosen first so that its multiply-add is one
    // fused operation, as in dot_rows_kernel
    double fa, fb;
    if (d) {
      // D = -q; D's old contents are not read (a stale NaN must not leak in)
      const double dv = (double)(-1.0 * v + 0.0);
      d[q] = dv;
      fa = ov;
      fb = dv;
    } else {
      fa = ov;
      fb = v;
    }
    s += fa * fb;
  };
  if (i0 < N) step(q0, x0, y0, o0);
  for (unsigned i = i0 + stride; i < N; i += stride) {
    const size_t q = compact_to_row(i, r, ld);
    step(q, x ? x[q] : 0.0, yin[q], d ? g[q] : u[q]);
  }
  publish_partial(block_sum(s, sh), part);
}

// step and curvature pair: Sn = alpha D, U = U + Sn (all N entries)
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) lbfgs_step_kernel(
    size_t N, double alpha, const double* __restrict__ D, double* __restrict__ Sn,
    double* __restrict__ U) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
    const double sn = (double)(alpha * (double)D[i] + 0.0);  // Sn's old contents unread
    Sn[i] = sn;
    U[i] = (double)((double)U[i] + (double)sn);
  }
}

// Yn = Gn - G; partials of <Sn, Yn> and <Gn, Gn>
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) lbfgs_pair_kernel(
    unsigned N, int r, int ld, const double* __restrict__ Gn, const double* __restrict__ G,
    double* __restrict__ Yn, const double* __restrict__ Sn, double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  // also the three sums the next two-loop starts from when this pair is the
  // newest in memory (those of dots3_kernel over Sn, Gn and Yn: same products,
  // same order, same grid); arrays: <Sn, Gn>, <Sn, Yn>, <Yn, Yn>, ||Gn||^2
  double s_sy = 0.0, s_gg = 0.0, s_sg = 0.0, s_yy = 0.0;
  for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    const size_t q = compact_to_row(i, r, ld);
    const double gv = Gn[q], sv = Sn[q];
    double y = (double)(1.0 * gv + 0.0);  // Yn's old contents unread
    y = (double)(-1.0 * (double)G[q] + 1.0 * y);
    Yn[q] = y;
    s_sy += sv * y;
    s_gg += gv * gv;
    s_sg += sv * gv;
    s_yy += y * y;
  }
  publish_partial(block_sum(s_sg, sh), part);
  publish_partial(block_sum(s_sy, sh), part + gridDim.x);
  publish_partial(block_sum(s_yy, sh), part + 2 * gridDim.x);
  publish_partial(block_sum(s_gg, sh), part + 3 * gridDim.x);
}

// the curvature pair's sums: sc[q_sy] = sc[q_mirror] = <Sn, Yn> (array 1),
// sc[q_gg] = ||Gn||^2 (array 3), arrays of length np
// (waves 0 and 1 each finish one array)
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) pair_finish(
    int np, const double* __restrict__ part, double* __restrict__ sc, int q_sy, int q_mirror,
    int q_gg) {
  const int wid = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (wid == 0) {
    const double v0 = wave_sum_parts(part + np, np);
    if (l == 0) {
      sc[q_sy] = 1.0 * v0;
      sc[q_mirror] = 1.0 * v0;
    }
  } else if (wid == 1) {
    const double v1 = wave_sum_parts(part + 3 * (size_t)np, np);
    if (l == 0) sc[q_gg] = 1.0 * v1;
  }
}

// Several dots over m-vectors for the quartic line search, in one pass: block
// bid of nblk (stride nblk blocks) leaves partials at part + t * nblk + bid:
//   [0] = p2.p2, [1] = p1.p2, [2] = p1.p1, [3] = p0.p2, [4] = p0.p1,
//   [5] = lam.p1, [6] = lam.p2,   with p0 = z - b.
__device__ __forceinline__ void linesearch_partials(int bid, int nblk, int m,
                                                    const double* __restrict__ z,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ p1,
                                                    const double* __restrict__ p2,
                                                    const double* __restrict__ lam,
                                                    double* __restrict__ part, double* sh) {
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  // four of a thread's strided elements are loaded before they are summed in
  // index order (same sums as one element at a time, four times the loads in flight)
  const int stride = nblk * kBlock;
  int i = bid * kBlock + threadIdx.x;
  for (; i + 3 * stride < m; i += 4 * stride) {
    double zz[4], bb[4], q1[4], q2[4], ll[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = i + u * stride;
      zz[u] = z[e];
      bb[u] = b[e];
      q1[u] = p1[e];
      q2[u] = p2[e];
      ll[u] = lam[e];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double a0 = zz[u] - bb[u], a1 = q1[u], a2 = q2[u], l = ll[u];
      s[0] += a2 * a2; s[1] += a1 * a2; s[2] += a1 * a1; s[3] += a0 * a2;
      s[4] += a0 * a1; s[5] += l * a1;  s[6] += l * a2;
    }
  }
  for (; i < m; i += stride) {
    const double a0 = z[i] - b[i], a1 = p1[i], a2 = p2[i], l = lam[i];
    s[0] += a2 * a2; s[1] += a1 * a2; s[2] += a1 * a1; s[3] += a0 * a2;
    s[4] += a0 * a1; s[5] += l * a1;  s[6] += l * a2;
  }
  for (int t = 0; t < 7; ++t) {
    const double bs = block_sum(s[t], sh);
    if (threadIdx.x == 0) part[(size_t)t * nblk + bid] = bs;
  }
}

// All sums of the exact line search in one launch: blocks below rg form the
// partials of <CD, U> and <CD, D> over the first r columns of n rows (stride
// ld; the element order and grouping of dots3_kernel with rg blocks) at
// part_f + t * rg, blocks below gl the m-vector sums of linesearch_partials
// with gl blocks at part_m (with lsp, those sums from the nls block partials
// the fused line-search map left, summed in a fixed order).  With cdiag (a diagonal C by row), each element
// of C D is formed here as the PAIR adjoint's C part forms it (c D + 0: the
// product, then the other lane groups' zero sums) instead of read from CD.
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) linesearch_all(
    unsigned N, int r, int ld, const double* __restrict__ CD, const double* __restrict__ U,
    const double* __restrict__ D, int rg, double* __restrict__ part_f, int m,
    const double* __restrict__ z, const double* __restrict__ b, const double* __restrict__ p1,
    const double* __restrict__ p2, const double* __restrict__ lam, int gl,
    double* __restrict__ part_m, const double* __restrict__ cdiag,
    const double* __restrict__ lsp, int nls) {
  __shared__ double sh[kBlock / 64];
  const int bid = blockIdx.x;
  if (bid < rg) {  // uniform over the block
    double s0 = 0.0, s1 = 0.0;
    for (unsigned i = bid * kBlock + threadIdx.x; i < N; i += rg * kBlock) {
      const size_t q = compact_to_row(i, r, ld);
      const double dq = D[q];
      const double cd = cdiag ? cdiag[i / (unsigned)r] * dq + 0.0 : CD[q];
      s0 += cd * U[q];
      s1 += cd * dq;
    }
    const double b0 = block_sum(s0, sh);
    if (threadIdx.x == 0) part_f[bid] = b0;
    const double b1 = block_sum(s1, sh);
    if (threadIdx.x == 0) part_f[rg + bid] = b1;
  }
  if (bid < gl) {
    if (lsp) {
      // the seven sums already formed per block of the fused line-search map
      // (nls partials each): block bid adds partials bid, bid + gl, ...
      for (int t = 0; t < 7; ++t) {
        double v = 0.0;
        for (int j = bid + (int)threadIdx.x * gl; j < nls; j += gl * kBlock) v += lsp[(size_t)t * nls + j];
        const double bs = block_sum(v, sh);
        if (threadIdx.x == 0) part_m[(size_t)t * gl + bid] = bs;
      }
    } else {
      linesearch_partials(bid, gl, m, z, b, p1, p2, lam, part_m, sh);
    }
  }
}

// sc[slot] = 2 <CD, U>, sc[slot + 1] = <CD, D>, sc[slot + 2 + t] = line-search
// sum t; with part_gd, also sc[slot + 9] = the sum of its rg partials
//
// host (optional): also publish slots slot .. slot + npub - 1 (npub <= 64) to
// host-mapped words 1 .. npub and then seq to word 0, as publish_slots does
// (sums not formed here are copied from sc, written by earlier launches).
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) linesearch_finish(
    int rg, const double* __restrict__ part_f, int gl, const double* __restrict__ part_m,
    const double* __restrict__ part_gd, double* __restrict__ sc, int slot, double* host,
    long long seq, int npub) {
  // ten sums (rg, gl <= 2 kBlock), wave w finishes sums w, w + 4, w + 8: 0 and
  // 1 over part_f, 2 .. 8 over part_m, 9 over part_gd; a wave loads all of
  // its arrays before it sums them
  const int wid = threadIdx.x >> 6, l = threadIdx.x & 63;
  constexpr int kW = kBlock / 64;
  Parts2 q[3];
  int na[3];
  bool on[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int a = wid + kW * j;
    on[j] = a < 9 || (a == 9 && part_gd != nullptr);
    const double* p = a < 2 ? part_f + (size_t)a * rg
                            : (a < 9 ? part_m + (size_t)(a - 2) * gl : part_gd);
    na[j] = (a < 2 || a == 9) ? rg : gl;
    if (on[j]) q[j] = load_parts2(p, na[j]);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int a = wid + kW * j;
    if (!on[j]) continue;
    const double v = sum_parts2(q[j], na[j]);
    if (l == 0) {
      const double val = (a == 0 ? 2.0 : 1.0) * v;
      sc[slot + a] = val;
      if (host && a < npub) host[1 + a] = val;
    }
  }
  if (host) {
    const int t = threadIdx.x;
    if (t < npub && (t >= 10 || (t == 9 && part_gd == nullptr))) host[1 + t] = sc[slot + t];
    __threadfence_system();
    __syncthreads();
    if (t == 0) __atomic_store_n(reinterpret_cast<long long*>(host), seq, __ATOMIC_RELEASE);
  }
}

// Dual update lam += rho (z - b) and per-block partials of ||z - b||^2.
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) dual_update(int m, const double* __restrict__ z,
                                                      const double* __restrict__ b,
                                                      double rho, double* __restrict__ lam,
                                                      double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double s = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
    const double d = z[i] - b[i];
    lam[i] += rho * d;
    s += d * d;
  }
  publish_partial(block_sum(s, sh), part);
}

// y = a * x + b * y  (elementwise, mixed types allowed); with b = 0 the old y
// is not read (uninitialised memory may hold NaN patterns)
template <typename TX, typename TY>
__global__ void __launch_bounds__(kBlock) axpby(size_t N, double a, const TX* __restrict__ x,
                                                double b, TY* __restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock)
    y[i] = (TY)(a * (double)x[i] + (b != 0.0 ? b * (double)y[i] : 0.0));
}

// y = a * x + b * y with a = sc[sa] - sc[sb] (ratio == 0) or sc[sa] / sc[sb]
// (ratio == 1): device-resident coefficients, same arithmetic as axpby
template <typename T>
__global__ void __launch_bounds__(kBlock) axpby_slots(size_t N, const double* __restrict__ sc,
                                                      int sa, int sb, int ratio,
                                                      const T* __restrict__ x, double b,
                                                      T* __restrict__ y) {
  const double a = ratio ? sc[sa] / sc[sb] : sc[sa] - sc[sb];
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock)
    y[i] = (T)(a * (double)x[i] + (b != 0.0 ? b * (double)y[i] : 0.0));
}

// y = a * x + b * y with a = sign * sc[slot] (device-resident coefficient)
template <typename T>
__global__ void __launch_bounds__(kBlock) axpby_dev(size_t N, const double* __restrict__ sc,
                                                    int slot, double sign, const T* __restrict__ x,
                                                    double b, T* __restrict__ y) {
  const double a = sign * sc[slot];
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock)
    y[i] = (T)(a * (double)x[i] + (b != 0.0 ? b * (double)y[i] : 0.0));
}

// z = x + y (z may alias x or y), with conversion
template <typename TX, typename TY, typename TZ>
__global__ void __launch_bounds__(kBlock) add_kernel(size_t N, const TX* __restrict__ x,
                                                     const TY* __restrict__ y, TZ* __restrict__ z) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock)
    z[i] = (TZ)((double)x[i] + (double)y[i]);
}

template <typename TS, typename TD>
__global__ void __launch_bounds__(kBlock) convert_kernel(size_t N, const TS* __restrict__ s,
                                                         TD* __restrict__ d) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock)
    d[i] = (TD)s[i];
}

// strided copy between row-major layouts (n rows, r columns)
// out = x + y row by row: x, out with leading dimension ldx, y with ldy
template <typename TX, typename TY>
__global__ void __launch_bounds__(kBlock) add_rows(int n, int r, const TX* __restrict__ x, int ldx,
                                                   const TY* __restrict__ y, int ldy,
                                                   TX* __restrict__ out) {
  const size_t N = (size_t)n * r;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
    const size_t j = i / r, c = i % r;
    out[j * ldx + c] = x[j * ldx + c] + (TX)y[j * ldy + c];
  }
}

template <typename TS, typename TD>
__global__ void __launch_bounds__(kBlock) copy_rows(int n, int r, const TS* __restrict__ s,
                                                    int lds, TD* __restrict__ d, int ldd) {
  const size_t N = (size_t)n * r;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
    const size_t j = i / r, c = i % r;
    d[j * ldd + c] = (TD)s[j * lds + c];
  }
}

// permutations of constraint-indexed vectors: dst[idx[i]] = src[i] / dst[i] = src[idx[i]]
template <typename T>
__global__ void __launch_bounds__(kBlock) scatter_kernel(int m, const int* __restrict__ idx,
                                                         const T* __restrict__ src, T* __restrict__ dst) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) dst[idx[i]] = src[i];
}
// lb[2 t] = lam[id[t]] (the multiplier half of the interleaved [lam, b]
// entries of the incident lists)
[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) gather_lam_lb(
    int E, const int* __restrict__ id, const double* __restrict__ lam, double* __restrict__ lb) {
  for (int t = blockIdx.x * kBlock + threadIdx.x; t < E; t += gridDim.x * kBlock)
    lb[2 * (size_t)t] = lam[id[t]];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) gather_kernel(int m, const int* __restrict__ idx,
                                                        const T* __restrict__ src, T* __restrict__ dst) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) dst[i] = src[idx[i]];
}

// rank growth: new row-major layout with r_new columns; the first r_old copy
// U, the rest are sigma * N(0,1) from the counter-based SplitMix64 stream
// (Steele-Lea-Flood 2014) with Box-Muller, element t = j (r_new - r_old) + c'.
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

[[maybe_unused]] static __global__ void __launch_bounds__(kBlock) grow_rank_kernel(int n, int r_old, int r_new,
                                                           const double* __restrict__ U,
                                                           double* __restrict__ Unew,
                                                           double sigma, uint64_t seed,
                                                           uint64_t event) {
  const size_t N = (size_t)n * r_new;
  const int add = r_new - r_old;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
    const size_t j = i / r_new;
    const int c = (int)(i % r_new);
    if (c < r_old) {
      Unew[i] = U[j * r_old + c];
    } else {
      const uint64_t t = (uint64_t)j * add + (uint64_t)(c - r_old);
      const uint64_t k1 = (event << 40) + 2ull * t + 1ull;
      const uint64_t k2 = k1 + 1ull;
      const uint64_t g = 0x9E3779B97F4A7C15ull;
      const double u1 = ((double)(splitmix_mix(seed + k1 * g) >> 11) + 1.0) * 0x1.0p-53;
      const double u2 = (double)(splitmix_mix(seed + k2 * g) >> 11) * 0x1.0p-53;
      Unew[i] = sigma * sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    }
  }
}

}  // namespace lorads
