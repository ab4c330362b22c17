// Structure-specialised kernels: DIAG (A_i = a_i e_j e_j^T, MaxCut) and PAIR
// (A_i = a_i (e_j e_k^T + e_k e_j^T), matrix completion).  Same group-per-row
// mapping and deterministic reductions as the generic kernels.
#pragma once

#include "kernels.hpp"

namespace lorads {

constexpr int kMaxCols = 4;  // factor columns per lane held in registers (r <= 4 G)
#ifndef LORADS_UNROLL
#define LORADS_UNROLL 4
#endif
constexpr int kUnroll = LORADS_UNROLL;  // constraints gathered per step (memory-level parallelism)
#ifndef LORADS_GRAD_UNROLL
#define LORADS_GRAD_UNROLL 4
#endif
// entries gathered per group and step in the FP64 gradient form (a group's
// entries are summed in list order whatever the value)
constexpr int kGU = LORADS_GRAD_UNROLL;
constexpr int kPairStage = 256;         // PAIR incident entries staged in LDS per wave and pass
// word 3 of a raw buffer resource on gfx9 parts (32-bit data format, no
// swizzle, no index stride)
constexpr int kBufferRsrcWord3 = 0x00020000;

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
// MODE 0 z = scale * A(U V^T); MODE 1 also w = lam + rho (z - b); MODE 2 the
// CG form; MODE 3 the two maps of the exact line search in one pass with
// V = D:  z = A(U D^T + D U^T) = 2 A(U D^T),  w = A(D D^T).
template <typename T, int G, int MODE, int KC = kMaxCols>
__global__ void __launch_bounds__(kBlock) k1_pair(
    int nchunks, const int* __restrict__ chunk_row, const int* __restrict__ chunk_start,
    const int* __restrict__ rptr, const int* __restrict__ pk, const T* __restrict__ pcoef,
    double pair_coef, const T* __restrict__ U, const T* __restrict__ V, int r, int ld,
    T* __restrict__ z, double scale, const double* __restrict__ lam,
    const double* __restrict__ b, double rho, double* __restrict__ w,
    const double* __restrict__ sc, int parity) {
  // results of a chunk are collected in the group's LDS slots and written as
  // contiguous runs at the end (groups of at least 4 lanes)
  constexpr bool kStage = G >= 4;
  constexpr bool kTwo = (MODE == 1 || MODE == 3);
  __shared__ T sz[kStage ? (kBlock / G) * kPairChunk : 1];
  __shared__ double sw[(kStage && kTwo) ? (kBlock / G) * kPairChunk : 1];
  if (MODE == 2 && sc[S_DONE + parity] != 0.0) return;
  const int chunk = (blockIdx.x * kBlock + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  const int gslot = (threadIdx.x / G) * kPairChunk;
  if (chunk >= nchunks) return;
  const int row = chunk_row[chunk];
  const int i0 = chunk_start[chunk], i1 = min(i0 + kPairChunk, rptr[row + 1]);
  using A = typename OpAcc<T>::type;
  A uj[KC], vj[KC];
#pragma unroll
  for (int t = 0; t < KC; ++t) {
    const int c = lane + t * G;
    uj[t] = c < r ? (A)U[row * ld + c] : (A)0;
    vj[t] = c < r ? (A)V[row * ld + c] : (A)0;
  }
  const double mult = (MODE == 2) ? sc[S_RHO] : (MODE == 0 ? scale : 1.0);
  for (int i = i0; i < i1; i += kUnroll) {
    const int cnt = min(kUnroll, i1 - i);
    int k[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) k[u] = u < cnt ? pk[i + u] : row;
    A d[kUnroll], d2[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      A s = 0, s2 = 0;
      const int base = k[u] * ld;
#pragma unroll
      for (int t = 0; t < KC; ++t) {
        const int c = lane + t * G;
        if (c < r) {
          const A vk = (A)V[base + c];
          s += uj[t] * vk + (A)U[base + c] * vj[t];
          if (MODE == 3) s2 += vj[t] * vk;
        }
      }
      d[u] = s;
      d2[u] = s2;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<G>(d[u]);
    if (MODE == 3) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) d2[u] = group_sum<G>(d2[u]);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      // every lane holds the reduced d[u]; lane u mod G stores it
      if (lane == (u & (G - 1)) && u < cnt) {
        const int id = i + u;
        const double val = (double)d[u] * (pcoef ? (double)pcoef[id] : pair_coef);
        T zv;
        double wv = 0.0;
        if (MODE == 1) {
          zv = (T)val;
          wv = lam[id] + rho * (val - b[id]);
        } else if (MODE == 3) {
          const double a = pcoef ? (double)pcoef[id] : pair_coef;
          zv = (T)(2.0 * val);
          wv = 2.0 * a * (double)d2[u];
        } else {
          zv = (T)(mult * val);
        }
        if (kStage) {
          sz[gslot + (id - i0)] = zv;
          if (kTwo) sw[gslot + (id - i0)] = wv;
        } else {
          z[id] = zv;
          if (kTwo) w[id] = wv;
        }
      }
    }
  }
  if (kStage) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q = lane; q < i1 - i0; q += G) {
      z[i0 + q] = sz[gslot + q];
      if (kTwo) w[i0 + q] = sw[gslot + q];
    }
  }
}

// FP64 forward maps (MODE 0, 1 and 3 of k1_pair) with two columns per lane
// loaded as one 16-byte vector: GV = G / 2 lanes per constraint, so a wave
// keeps twice the constraints of the one-column form in flight.  The sums are
// those of the one-column form bit for bit: a lane adds its two columns' terms
// (columns 2l and 2l + 1, exactly the first level of the G-lane tree), then the
// remaining levels run over GV lanes, and every term is evaluated by the same
// expression.  Needs rows aligned to 16 bytes (ld even) and r <= 2 GV.
// X3 = 1 (ranks 17 .. 24 with GV = 8): each lane also holds column 2 GV + lane,
// so 8 lanes cover 24 columns instead of 16 lanes covering 32 (a third fewer
// bytes gathered per partner row, twice the constraints per wave in flight);
// a lane's sum is (pair sum) + third term, the same expression in every map
// of this form, so the forward maps, the line search and the gradient form
// agree bit for bit with each other (not with the one-column form).  Needs
// ld >= 3 GV.
// Chunks come from the XCD lists: workgroup b serves list b mod kXcds, whose
// partners all lie in one block of rows, so the partner rows one XCD gathers
// stay in its L2.
__device__ __forceinline__ int xchunk_of(const int* __restrict__ xoff, int GV) {
  const int x = blockIdx.x % kXcds;
  const int local = (blockIdx.x / kXcds) * (kBlock / GV) + (int)threadIdx.x / GV;
  const int c = xoff[x] + local;
  return c < xoff[x + 1] ? c : -1;
}

template <int GV, int MODE, int X3 = 0>
__global__ void __launch_bounds__(kBlock) k1_pair_v2(
    const int* __restrict__ xoff, const int* __restrict__ chunk_row,
    const int* __restrict__ chunk_start, const int* __restrict__ chunk_end,
    const int* __restrict__ pk, const double* __restrict__ pcoef,
    double pair_coef, const double* __restrict__ U, const double* __restrict__ V, int r, int ld,
    double* __restrict__ z, double scale, const double* __restrict__ lam,
    const double* __restrict__ b, double rho, double* __restrict__ w) {
  constexpr bool kStage = GV >= 4;
  constexpr bool kTwo = (MODE == 1 || MODE == 3);
  typedef double d2 __attribute__((ext_vector_type(2)));
  __shared__ double sz[kStage ? (kBlock / GV) * kPairChunk : 1];
  __shared__ double sw[(kStage && kTwo) ? (kBlock / GV) * kPairChunk : 1];
  const int chunk = xchunk_of(xoff, GV);
  const int lane = threadIdx.x & (GV - 1);
  const int gslot = (threadIdx.x / GV) * kPairChunk;
  if (chunk < 0) return;
  const int row = chunk_row[chunk];
  const int i0 = chunk_start[chunk], i1 = chunk_end[chunk];
  const int c0 = 2 * lane, c2 = 2 * GV + lane;
  const bool on0 = c0 < r, on1 = c0 + 1 < r, on2 = X3 && c2 < r;
  const d2 uj = *reinterpret_cast<const d2*>(U + row * ld + c0);
  const d2 vj = *reinterpret_cast<const d2*>(V + row * ld + c0);
  const double uj2 = X3 ? U[row * ld + c2] : 0.0, vj2 = X3 ? V[row * ld + c2] : 0.0;
  const double mult = MODE == 0 ? scale : 1.0;
  for (int i = i0; i < i1; i += kUnroll) {
    const int cnt = min(kUnroll, i1 - i);
    int k[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) k[u] = u < cnt ? pk[i + u] : row;
    d2 vk[kUnroll], uk[kUnroll];
    double vk2[kUnroll], uk2[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      vk[u] = *reinterpret_cast<const d2*>(V + k[u] * ld + c0);
      uk[u] = *reinterpret_cast<const d2*>(U + k[u] * ld + c0);
      if (X3) {
        vk2[u] = V[k[u] * ld + c2];
        uk2[u] = U[k[u] * ld + c2];
      }
    }
    double d[kUnroll], d2s[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      double s0 = 0.0, s1 = 0.0, q0 = 0.0, q1 = 0.0;
      if (on0) {
        s0 += uj[0] * vk[u][0] + uk[u][0] * vj[0];
        if (MODE == 3) q0 += vj[0] * vk[u][0];
      }
      if (on1) {
        s1 += uj[1] * vk[u][1] + uk[u][1] * vj[1];
        if (MODE == 3) q1 += vj[1] * vk[u][1];
      }
      d[u] = s0 + s1;
      d2s[u] = q0 + q1;
      if (X3) {
        double s2 = 0.0, q2 = 0.0;
        if (on2) {
          s2 += uj2 * vk2[u] + uk2[u] * vj2;
          if (MODE == 3) q2 += vj2 * vk2[u];
        }
        d[u] = d[u] + s2;
        d2s[u] = d2s[u] + q2;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<GV>(d[u]);
    if (MODE == 3) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) d2s[u] = group_sum<GV>(d2s[u]);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (lane == (u & (GV - 1)) && u < cnt) {
        const int id = i + u;
        const double val = d[u] * (pcoef ? pcoef[id] : pair_coef);
        double zv, wv = 0.0;
        if (MODE == 1) {
          zv = val;
          wv = lam[id] + rho * (val - b[id]);
        } else if (MODE == 3) {
          const double a = pcoef ? pcoef[id] : pair_coef;
          zv = 2.0 * val;
          wv = 2.0 * a * d2s[u];
        } else {
          zv = mult * val;
        }
        if (kStage) {
          sz[gslot + (id - i0)] = zv;
          if (kTwo) sw[gslot + (id - i0)] = wv;
        } else {
          z[id] = zv;
          if (kTwo) w[id] = wv;
        }
      }
    }
  }
  if (kStage) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q = lane; q < i1 - i0; q += GV) {
      z[i0 + q] = sz[gslot + q];
      if (kTwo) w[i0 + q] = sw[gslot + q];
    }
  }
}

// The exact line search of Phase I in one pass (PAIR, FP64, two columns per
// lane, XCD chunk lists): the loop of k1_pair_v2 MODE 3, which collects a chunk's
//   p1_i = A(U D^T + D U^T)_i = 2 a (<U_j, D_k> + <U_k, D_j>),
//   p2_i = A(D D^T)_i = 2 a <D_j, D_k>
// in the group's LDS slots (the same expressions, so the same values), ends by
// reading z, b and lam of the chunk's constraints as contiguous runs and adding
// the seven sums of the quartic (the order of linesearch_partials):
//   p2.p2, p1.p2, p1.p1, p0.p2, p0.p1, lam.p1, lam.p2,   p0 = z - b.
// Nothing m-sized is written: each block leaves its seven partials at
// part[t * gridDim.x + block].  Groups of at least 4 lanes (GV >= 4); X3 as
// in k1_pair_v2.
template <int GV, int X3 = 0>
__global__ void __launch_bounds__(kBlock) k1_pair_ls(
    const int* __restrict__ xoff, const int* __restrict__ chunk_row,
    const int* __restrict__ chunk_start, const int* __restrict__ chunk_end,
    const int* __restrict__ pk, const double* __restrict__ pcoef,
    double pair_coef, const double* __restrict__ U, const double* __restrict__ D, int r, int ld,
    const double* __restrict__ z, const double* __restrict__ b, const double* __restrict__ lam,
    double* __restrict__ part) {
  static_assert(GV >= 4, "the chunk results are staged per group");
  typedef double d2 __attribute__((ext_vector_type(2)));
  __shared__ double s1[(kBlock / GV) * kPairChunk];
  __shared__ double s2[(kBlock / GV) * kPairChunk];
  __shared__ double sh[kBlock / 64];
  const int chunk = xchunk_of(xoff, GV);
  const int lane = threadIdx.x & (GV - 1);
  const int gslot = (threadIdx.x / GV) * kPairChunk;
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (chunk >= 0) {
    const int row = chunk_row[chunk];
    const int i0 = chunk_start[chunk], i1 = chunk_end[chunk];
    const int c0 = 2 * lane, c2 = 2 * GV + lane;
    const bool on0 = c0 < r, on1 = c0 + 1 < r, on2 = X3 && c2 < r;
    const d2 uj = *reinterpret_cast<const d2*>(U + row * ld + c0);
    const d2 dj = *reinterpret_cast<const d2*>(D + row * ld + c0);
    const double uj2 = X3 ? U[row * ld + c2] : 0.0, dj2 = X3 ? D[row * ld + c2] : 0.0;
    for (int i = i0; i < i1; i += kUnroll) {
      const int cnt = min(kUnroll, i1 - i);
      int k[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) k[u] = u < cnt ? pk[i + u] : row;
      d2 dk[kUnroll], uk[kUnroll];
      double dk2[kUnroll], uk2[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        dk[u] = *reinterpret_cast<const d2*>(D + k[u] * ld + c0);
        uk[u] = *reinterpret_cast<const d2*>(U + k[u] * ld + c0);
        if (X3) {
          dk2[u] = D[k[u] * ld + c2];
          uk2[u] = U[k[u] * ld + c2];
        }
      }
      double d[kUnroll], dd[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        double sa = 0.0, sb = 0.0, qa = 0.0, qb = 0.0;
        if (on0) {
          sa += uj[0] * dk[u][0] + uk[u][0] * dj[0];
          qa += dj[0] * dk[u][0];
        }
        if (on1) {
          sb += uj[1] * dk[u][1] + uk[u][1] * dj[1];
          qb += dj[1] * dk[u][1];
        }
        d[u] = sa + sb;
        dd[u] = qa + qb;
        if (X3) {
          double sc2 = 0.0, qc2 = 0.0;
          if (on2) {
            sc2 += uj2 * dk2[u] + uk2[u] * dj2;
            qc2 += dj2 * dk2[u];
          }
          d[u] = d[u] + sc2;
          dd[u] = dd[u] + qc2;
        }
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<GV>(d[u]);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) dd[u] = group_sum<GV>(dd[u]);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (lane == (u & (GV - 1)) && u < cnt) {
          const int id = i + u;
          const double a = pcoef ? pcoef[id] : pair_coef;
          s1[gslot + (id - i0)] = 2.0 * (d[u] * a);
          s2[gslot + (id - i0)] = 2.0 * a * dd[u];
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q = lane; q < i1 - i0; q += GV) {
      const double p1 = s1[gslot + q], p2 = s2[gslot + q];
      const double p0 = z[i0 + q] - b[i0 + q], l = lam[i0 + q];
      acc[0] += p2 * p2;
      acc[1] += p1 * p2;
      acc[2] += p1 * p1;
      acc[3] += p0 * p2;
      acc[4] += p0 * p1;
      acc[5] += l * p1;
      acc[6] += l * p2;
    }
  }
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    const double bs = block_sum(acc[t], sh);
    if (threadIdx.x == 0) part[(size_t)t * gridDim.x + blockIdx.x] = bs;
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
// PAIR, one wave per row over the row's incident list: every constraint
// a (e_j e_k^T + e_k e_j^T) appears in the list of row j (partner k) and of
// row k (partner j), partners ascending.  The wave's 64/G lane groups take
// interleaved entries (so the index loads of a step are contiguous) and
// kUnroll entries per step; each lane holds KC columns (c = lane + t G; KC = 1
// whenever r <= G).
// The group partials are summed by a fixed xor butterfly across the wave.
// A wave first loads a pass of kPairStage entries (partners and coefficients,
// every load of the pass in flight at once) into its own LDS slots, so the
// gathers of a step wait on one memory latency instead of an index chain.
//   MODE 0 (adjoint):  out_t = out_scale (c_scale (C V)_t + sum_e a_e w_{id(e)} V_p);
//                      w == nullptr drops the sum (the solver's C D and C U products)
//   MODE 1 (CG operator, V = the fixed factor, Pm = the direction):
//     Q_t = gamma Pm_t + rho sum_e a_e^2 (<Pm_t, V_p> + <Pm_p, V_t>) V_p,
//     i.e. (gamma I + rho A* A(. V^T) V) applied to Pm; block partials of <Pm, Q>.
//     Each constraint's inner product is formed by both of its rows, so no
//     per-constraint buffer is written or gathered.
//   MODE 2 (gradient form of MODE 0 with V = U, uniform a): the multiplier-side
//     weight of each entry is formed in place, w = lam + rho (a <U_t, U_p> - b),
//     from lam and b stored per incident entry (streamed, not gathered); the
//     entry's inner product and w are evaluated exactly as the forward map
//     (MODE 1 of k1_pair) evaluates them, so out equals MODE 0 fed with that
//     map's w bit for bit.
// ===========================================================================
template <typename T, int G, int MODE, int KC = kMaxCols>
__global__ void __launch_bounds__(kBlock) kpair_rows(
    int n, const int* __restrict__ cptr, const int* __restrict__ ccol,
    const T* __restrict__ cval, double c_scale, const int* __restrict__ inc_ptr,
    const int* __restrict__ inc_nb, const int* __restrict__ inc_id, const T* __restrict__ pcoef,
    double pair_coef, const T* __restrict__ w, const T* __restrict__ V, const T* __restrict__ Pm,
    int r, int ld, T* __restrict__ out, int ldo, double out_scale, double* __restrict__ sc,
    int parity, double* __restrict__ part, const double* __restrict__ lb_inc, double rho_w) {
  constexpr int NG = 64 / G;
  constexpr int CH = kPairStage;  // incident entries staged per wave and pass
  __shared__ double sh[kBlock / 64];
  __shared__ int s_nb[kBlock / 64][CH];
  using A = typename OpAcc<T>::type;
  __shared__ A s_cf[kBlock / 64][CH];
  __shared__ double s_bi[MODE == 2 ? kBlock / 64 : 1][MODE == 2 ? CH : 1];
  if (MODE == 1 && sc[S_DONE + parity] != 0.0) return;
  const int wl = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = wl / G, lane = wl & (G - 1);
  const int row = blockIdx.x * (kBlock / 64) + wid;
  int* nbw = s_nb[wid];
  A* cfw = s_cf[wid];
  double pq = 0.0;
  if (row < n) {  // wave-uniform
    A acc[KC], pt[KC], vt[KC];
#pragma unroll
    for (int t = 0; t < KC; ++t) {
      const int c = lane + t * G;
      acc[t] = 0;
      pt[t] = (MODE == 1 && c < r) ? (A)Pm[row * ld + c] : (A)0;
      vt[t] = (MODE != 0 && c < r) ? (A)V[row * ld + c] : (A)0;
    }
    if (MODE != 1 && c_scale != 0.0) {
      for (int e = cptr[row] + grp; e < cptr[row + 1]; e += NG) {
        const int k = ccol[e];
        const A a = (A)(c_scale * (double)cval[e]);
#pragma unroll
        for (int t = 0; t < KC; ++t) {
          const int c = lane + t * G;
          if (c < r) acc[t] += a * (A)V[k * ld + c];
        }
      }
    }
    // MODE 0 with w == nullptr is the C part alone (c_scale C V)
    const int e0 = inc_ptr[row];
    const int e1 = (MODE == 0 && w == nullptr) ? e0 : inc_ptr[row + 1];
    for (int base = e0; base < e1; base += CH) {
      const int cnt = min(CH, e1 - base);
      // stage: partners and per-entry coefficients (a w_id for the adjoint,
      // a^2 for the CG operator), all loads of the pass in flight together
#pragma unroll
      for (int q = 0; q < CH / 64; ++q) {
        const int j = wl + 64 * q;
        if (MODE == 2) {
          if (j < cnt) {
            nbw[j] = inc_nb[base + j];
            cfw[j] = (A)lb_inc[2 * (size_t)(base + j)];
            s_bi[wid][j] = lb_inc[2 * (size_t)(base + j) + 1];
          }
        } else if (j < cnt) {
          nbw[j] = inc_nb[base + j];
          double a = pair_coef;
          if (pcoef != nullptr || MODE == 0) {
            const int id = inc_id[base + j];
            if (pcoef != nullptr) a = (double)pcoef[id];
            if (MODE == 0) a *= (double)w[id];
            else a *= a;
          } else if (MODE == 1) {
            a *= a;
          }
          cfw[j] = (A)a;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int j = grp; j < cnt; j += NG * kUnroll) {
        int p[kUnroll];
        A coef[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int ju = j + u * NG;
          const bool ok = ju < cnt;
          p[u] = (ok ? nbw[ju] : row) * ld;
          coef[u] = ok ? cfw[ju] : (A)0;
        }
        if (MODE == 0) {
#pragma unroll
          for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int t = 0; t < KC; ++t) {
              const int c = lane + t * G;
              if (c < r) acc[t] += coef[u] * (A)V[p[u] + c];
            }
        } else if (MODE == 2) {
          // coef holds lam of the entry (0 past the list); w and a w as in
          // the forward map and the adjoint's staging
          A vp[kUnroll][KC], d[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            A s = 0;
#pragma unroll
            for (int t = 0; t < KC; ++t) {
              const int c = lane + t * G;
              vp[u][t] = c < r ? (A)V[p[u] + c] : (A)0;
              s += vt[t] * vp[u][t] + vp[u][t] * vt[t];
            }
            d[u] = s;
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<G>(d[u]);
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const int ju = j + u * NG;
            const bool ok = ju < cnt;
            const double val = (double)d[u] * pair_coef;
            const double wv = (double)coef[u] + rho_w * (val - s_bi[wid][min(ju, CH - 1)]);
            coef[u] = ok ? (A)(pair_coef * wv) : (A)0;
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int t = 0; t < KC; ++t) {
              const int c = lane + t * G;
              if (c < r) acc[t] += coef[u] * vp[u][t];
            }
        } else {
          A vp[kUnroll][KC], d[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            A s = 0;
#pragma unroll
            for (int t = 0; t < KC; ++t) {
              const int c = lane + t * G;
              vp[u][t] = c < r ? (A)V[p[u] + c] : (A)0;
              const A pp = c < r ? (A)Pm[p[u] + c] : (A)0;
              s += pt[t] * vp[u][t] + pp * vt[t];
            }
            d[u] = s;
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<G>(d[u]) * coef[u];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int t = 0; t < KC; ++t) acc[t] += d[u] * vp[u][t];
        }
      }
      // the next pass overwrites this wave's staging slots
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int t = 0; t < KC; ++t)
      for (int o = G; o < 64; o <<= 1) acc[t] += __shfl_xor(acc[t], o, 64);
    if (grp == 0) {
      if (MODE == 1) {
        const double gamma = sc[S_GAMMA], rho = sc[S_RHO];
#pragma unroll
        for (int t = 0; t < KC; ++t) {
          const int c = lane + t * G;
          if (c < r) {
            const T qv = (T)(gamma * (double)pt[t] + rho * (double)acc[t]);
            out[row * ldo + c] = qv;
            pq += (double)pt[t] * (double)qv;
          }
        }
      } else {
#pragma unroll
        for (int t = 0; t < KC; ++t) {
          const int c = lane + t * G;
          if (c < r) out[row * ldo + c] = (T)(out_scale * (double)acc[t]);
        }
      }
    }
  }
  if (MODE == 1) publish_partial(block_sum(pq, sh), part);
}

// ===========================================================================
// Gradient form (MODE 2 of kpair_rows) with two columns per lane in 16-byte
// loads and two rows per wave: each half-wave serves one row with NG groups of
// GV = G / 2 lanes, so a group takes the same entries in the same order as a
// G-lane group of the one-column form, the within-entry sums follow the same
// tree (a lane adds its two columns first) and the cross-group sums pair the
// same groups.  The output equals MODE 2's bit for bit.  X3 = 1 (ranks
// 17 .. 24, GV = 8) adds column 2 GV + lane per lane as in k1_pair_v2, with
// the entry sums of that form (then 4 groups serve a row, and the output
// equals the X3 forward map fed to the adjoint, not MODE 2).
//
// z (optional): the forward map A(V V^T) as a by-product.  Each entry's inner
// product is the forward map's expression in the forward map's order, so the
// value is the forward map's bit for bit; a row writes the entries of its
// upper part (partners above the row), which in the incident list follow the
// lower ones and are the row-view constraints rptr[row] .. rptr[row + 1] in
// order.  The values are collected in the entries' LDS slots and written as
// one contiguous run per staged pass.
// ===========================================================================
template <int GV, int X3 = 0>
__global__ void __launch_bounds__(kBlock) kpair_grad_v2(
    int n, const int* __restrict__ cptr, const int* __restrict__ ccol,
    const double* __restrict__ cval, double c_scale, const int* __restrict__ inc_ptr,
    const int* __restrict__ inc_nb, double pair_coef, const double* __restrict__ V, int r,
    int ld, double* __restrict__ out, int ldo, double out_scale,
    const double* __restrict__ lb_inc, double rho_w,
    const int* __restrict__ rptr, double* __restrict__ z) {
  constexpr int HW = 32;              // lanes per row
  constexpr int NG = HW / GV;         // groups per row
  constexpr int CH = kPairStage / 2;  // entries staged per row and pass (a multiple of NG kGU)
  typedef double d2 __attribute__((ext_vector_type(2)));
  __shared__ int s_nb[kBlock / HW][CH];
  __shared__ double s_cf[kBlock / HW][CH];
  __shared__ double s_bi[kBlock / HW][CH];
  const int hl = threadIdx.x & (HW - 1), hid = threadIdx.x / HW;
  const int grp = hl / GV, lane = hl & (GV - 1);
  const int row = blockIdx.x * (kBlock / HW) + hid;
  int* nbw = s_nb[hid];
  double* cfw = s_cf[hid];
  double* biw = s_bi[hid];
  if (row < n) {  // uniform over the half-wave
    const int c0 = 2 * lane, c2 = 2 * GV + lane;
    const bool on0 = c0 < r, on1 = c0 + 1 < r, on2 = X3 && c2 < r;
    double vt0 = 0.0, vt1 = 0.0, vt2 = 0.0;
    {
      const d2 v = *reinterpret_cast<const d2*>(V + row * ld + c0);
      if (on0) vt0 = v[0];
      if (on1) vt1 = v[1];
      if (on2) vt2 = V[row * ld + c2];
    }
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    if (c_scale != 0.0) {
      for (int e = cptr[row] + grp; e < cptr[row + 1]; e += NG) {
        const int k = ccol[e];
        const double a = c_scale * cval[e];
        if (on0) acc0 += a * V[k * ld + c0];
        if (on1) acc1 += a * V[k * ld + c0 + 1];
        if (on2) acc2 += a * V[k * ld + c2];
      }
    }
    const int e0 = inc_ptr[row], e1 = inc_ptr[row + 1];
    // z: the upper part starts at list position zlow and maps to rptr[row] on
    const int zrow = z ? rptr[row] : 0;
    const int zlow = z ? (e1 - e0) - (rptr[row + 1] - zrow) : 0;
    for (int base = e0; base < e1; base += CH) {
      const int cnt = min(CH, e1 - base);
#pragma unroll
      for (int q = 0; q < CH / HW; ++q) {
        const int j = hl + HW * q;
        if (j < cnt) {
          nbw[j] = inc_nb[base + j];
          const d2 lb = *reinterpret_cast<const d2*>(lb_inc + 2 * (size_t)(base + j));
          cfw[j] = lb[0];
          biw[j] = lb[1];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int j = grp; j < cnt; j += NG * kGU) {
        int p[kGU];
        double coef[kGU];
#pragma unroll
        for (int u = 0; u < kGU; ++u) {
          const int ju = j + u * NG;
          const bool ok = ju < cnt;
          p[u] = (ok ? nbw[ju] : row) * ld;
          coef[u] = ok ? cfw[ju] : 0.0;
        }
        double vp0[kGU], vp1[kGU], vp2[kGU], d[kGU];
#pragma unroll
        for (int u = 0; u < kGU; ++u) {
          const d2 v = *reinterpret_cast<const d2*>(V + p[u] + c0);
          vp0[u] = on0 ? v[0] : 0.0;
          vp1[u] = on1 ? v[1] : 0.0;
          if (X3) {
            const double v2 = V[p[u] + c2];
            vp2[u] = on2 ? v2 : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < kGU; ++u) {
          double s0 = 0.0, s1 = 0.0;
          s0 += vt0 * vp0[u] + vp0[u] * vt0;
          s1 += vt1 * vp1[u] + vp1[u] * vt1;
          d[u] = s0 + s1;
          if (X3) {
            double s2 = 0.0;
            s2 += vt2 * vp2[u] + vp2[u] * vt2;
            d[u] = d[u] + s2;
          }
        }
#pragma unroll
        for (int u = 0; u < kGU; ++u) d[u] = group_sum<GV>(d[u]);
#pragma unroll
        for (int u = 0; u < kGU; ++u) {
          const int ju = j + u * NG;
          const bool ok = ju < cnt;
          const double val = d[u] * pair_coef;
          const double wv = coef[u] + rho_w * (val - biw[min(ju, CH - 1)]);
          coef[u] = ok ? pair_coef * wv : 0.0;
          // the entry's lam slot (already read by the whole group) takes z
          if (z && ok && lane == (u & (GV - 1))) cfw[ju] = val;
        }
#pragma unroll
        for (int u = 0; u < kGU; ++u) {
          if (on0) acc0 += coef[u] * vp0[u];
          if (on1) acc1 += coef[u] * vp1[u];
          if (on2) acc2 += coef[u] * vp2[u];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (z) {
        // slots read by the lanes that stage them next
        const int off = base - e0 - zlow;  // z index of slot q: zrow + off + q
#pragma unroll
        for (int q = 0; q < CH / HW; ++q) {
          const int j = hl + HW * q;
          if (j < cnt && off + j >= 0) z[zrow + off + j] = cfw[j];
        }
      }
    }
    for (int o = GV; o < HW; o <<= 1) {
      acc0 += __shfl_xor(acc0, o, 64);
      acc1 += __shfl_xor(acc1, o, 64);
      if (X3) acc2 += __shfl_xor(acc2, o, 64);
    }
    if (grp == 0) {
      if (on0) out[row * ldo + c0] = out_scale * acc0;
      if (on1) out[row * ldo + c0 + 1] = out_scale * acc1;
      if (on2) out[row * ldo + c2] = out_scale * acc2;
    }
  }
}

// ===========================================================================
// The adjoint product (MODE 0 of kpair_rows) in the FP64 two-columns-per-lane
// layout of kpair_grad_v2: half a wave per row (two rows per wave), GV lanes
// per entry holding columns 2 lane and 2 lane + 1 (one 16-byte load), with X3
// (ranks 17 .. 24) also column 2 GV + lane; NG = 32 / GV groups take the
// row's entries in turn, kGU entries per step.  A pass stages the partners and
// the coefficients a_e w_id(e) of CH entries in the half-wave's LDS slots.
//   out_t = out_scale (c_scale (C V)_t + sum_e a_e w_id(e) V_p)
// (w == nullptr: the C part alone).  The group partials are summed by the xor
// butterfly of kpair_grad_v2.  Needs ld >= the lane group of r and 16-byte
// aligned rows (pair_v2_ok).
// ===========================================================================
template <int GV, int X3 = 0>
__global__ void __launch_bounds__(kBlock) kpair_adj_v2(
    int n, const int* __restrict__ cptr, const int* __restrict__ ccol,
    const double* __restrict__ cval, double c_scale, const int* __restrict__ inc_ptr,
    const int* __restrict__ inc_nb, const int* __restrict__ inc_id,
    const double* __restrict__ pcoef, double pair_coef, const double* __restrict__ w,
    const double* __restrict__ V, int r, int ld, double* __restrict__ out, int ldo,
    double out_scale) {
  constexpr int HW = 32;              // lanes per row
  constexpr int NG = HW / GV;         // groups per row
  constexpr int CH = kPairStage / 2;  // entries staged per row and pass
  typedef double d2 __attribute__((ext_vector_type(2)));
  __shared__ int s_nb[kBlock / HW][CH];
  __shared__ double s_cf[kBlock / HW][CH];
  const int hl = threadIdx.x & (HW - 1), hid = threadIdx.x / HW;
  const int grp = hl / GV, lane = hl & (GV - 1);
  const int row = blockIdx.x * (kBlock / HW) + hid;
  int* nbw = s_nb[hid];
  double* cfw = s_cf[hid];
  if (row < n) {  // uniform over the half-wave
    const int c0 = 2 * lane, c2 = 2 * GV + lane;
    const bool on0 = c0 < r, on1 = c0 + 1 < r, on2 = X3 && c2 < r;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    if (c_scale != 0.0) {
      for (int e = cptr[row] + grp; e < cptr[row + 1]; e += NG) {
        const int k = ccol[e];
        const double a = c_scale * cval[e];
        if (on0) acc0 += a * V[k * ld + c0];
        if (on1) acc1 += a * V[k * ld + c0 + 1];
        if (on2) acc2 += a * V[k * ld + c2];
      }
    }
    const int e0 = inc_ptr[row];
    const int e1 = w != nullptr ? inc_ptr[row + 1] : e0;
    for (int base = e0; base < e1; base += CH) {
      const int cnt = min(CH, e1 - base);
#pragma unroll
      for (int q = 0; q < CH / HW; ++q) {
        const int j = hl + HW * q;
        if (j < cnt) {
          nbw[j] = inc_nb[base + j];
          const int id = inc_id[base + j];
          const double a = pcoef != nullptr ? pcoef[id] : pair_coef;
          cfw[j] = a * w[id];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int j = grp; j < cnt; j += NG * kGU) {
        int p[kGU];
        double coef[kGU];
#pragma unroll
        for (int u = 0; u < kGU; ++u) {
          const int ju = j + u * NG;
          const bool ok = ju < cnt;
          p[u] = (ok ? nbw[ju] : row) * ld;
          coef[u] = ok ? cfw[ju] : 0.0;
        }
        double vp0[kGU], vp1[kGU], vp2[kGU];
#pragma unroll
        for (int u = 0; u < kGU; ++u) {
          const d2 v = *reinterpret_cast<const d2*>(V + p[u] + c0);
          vp0[u] = on0 ? v[0] : 0.0;
          vp1[u] = on1 ? v[1] : 0.0;
          if (X3) {
            const double v2 = V[p[u] + c2];
            vp2[u] = on2 ? v2 : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < kGU; ++u) {
          acc0 += coef[u] * vp0[u];
          acc1 += coef[u] * vp1[u];
          if (X3) acc2 += coef[u] * vp2[u];
        }
      }
      // the slots are read before the next pass stages over them
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int o = GV; o < HW; o <<= 1) {
      acc0 += __shfl_xor(acc0, o, 64);
      acc1 += __shfl_xor(acc1, o, 64);
      if (X3) acc2 += __shfl_xor(acc2, o, 64);
    }
    if (grp == 0) {
      if (on0) out[row * ldo + c0] = out_scale * acc0;
      if (on1) out[row * ldo + c0 + 1] = out_scale * acc1;
      if (on2) out[row * ldo + c2] = out_scale * acc2;
    }
  }
}

// ===========================================================================
// FP32 forward map (MODE 0 of k1_pair) over the XCD chunk lists with four
// columns per lane loaded as one 16-byte vector: G = pow2(ceil(r / 4)) >= 4
// lanes per constraint, FP32 products and sums (the FP32 form's operator
// arithmetic), z_i = scale a_i (<U_j, V_k> + <U_k, V_j>) rounded once to
// FP32, staged per group and written as contiguous runs.  Columns at or past
// r are masked (padding may hold anything).  Needs ld a multiple of 4,
// ld >= 4 G and 16-byte aligned U and V.
// ===========================================================================
template <int G>
__global__ void __launch_bounds__(kBlock) k1_pair_f4(
    const int* __restrict__ xoff, const int* __restrict__ chunk_row,
    const int* __restrict__ chunk_start, const int* __restrict__ chunk_end,
    const int* __restrict__ pk, const float* __restrict__ pcoef, double pair_coef,
    const float* __restrict__ U, const float* __restrict__ V, int r, int ld,
    float* __restrict__ z, double scale) {
  static_assert(G >= 4, "the chunk results are staged per group");
  typedef float f4 __attribute__((ext_vector_type(4)));
  __shared__ float sz[(kBlock / G) * kPairChunk];
  const int chunk = xchunk_of(xoff, G);
  const int lane = threadIdx.x & (G - 1);
  const int gslot = (threadIdx.x / G) * kPairChunk;
  if (chunk < 0) return;
  const int row = chunk_row[chunk];
  const int i0 = chunk_start[chunk], i1 = chunk_end[chunk];
  const int c0 = 4 * lane;
  f4 uj = *reinterpret_cast<const f4*>(U + row * ld + c0);
  f4 vj = *reinterpret_cast<const f4*>(V + row * ld + c0);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (c0 + v >= r) {  // the row's own padding: zero, so the partner's drops out
      uj[v] = 0.0f;
      vj[v] = 0.0f;
    }
  }
  for (int i = i0; i < i1; i += kUnroll) {
    const int cnt = min(kUnroll, i1 - i);
    int k[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) k[u] = u < cnt ? pk[i + u] : row;
    f4 vk[kUnroll], uk[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      vk[u] = *reinterpret_cast<const f4*>(V + k[u] * ld + c0);
      uk[u] = *reinterpret_cast<const f4*>(U + k[u] * ld + c0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (c0 + v >= r) {
          vk[u][v] = 0.0f;
          uk[u][v] = 0.0f;
        }
      }
    }
    float d[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      float sa = uj[0] * vk[u][0];
      sa = fmaf(uk[u][0], vj[0], sa);
#pragma unroll
      for (int v = 1; v < 4; ++v) {
        sa = fmaf(uj[v], vk[u][v], sa);
        sa = fmaf(uk[u][v], vj[v], sa);
      }
      d[u] = sa;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<G>(d[u]);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (lane == (u & (G - 1)) && u < cnt) {
        const int id = i + u;
        const double a = pcoef ? (double)pcoef[id] : pair_coef;
        sz[gslot + (id - i0)] = (float)(scale * (a * (double)d[u]));
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int q = lane; q < i1 - i0; q += G) z[i0 + q] = sz[gslot + q];
}

// ===========================================================================
// FP32 adjoint product (MODE 0 of kpair_rows) with four columns per lane as
// one 16-byte vector: half a wave per row, G = pow2(ceil(r / 4)) >= 4 lanes per
// entry, NG = 32 / G groups taking the row's entries in turn, kGU entries per
// step; FP32 products and sums (the FP32 form's operator arithmetic), the
// group partials summed by an xor butterfly.  Otherwise as kpair_adj_v2.
// Needs ld a multiple of 4, ld >= 4 G and a 16-byte aligned V.
// ===========================================================================
template <int G>
__global__ void __launch_bounds__(kBlock) kpair_adj_f4(
    int n, const int* __restrict__ cptr, const int* __restrict__ ccol,
    const float* __restrict__ cval, double c_scale, const int* __restrict__ inc_ptr,
    const int* __restrict__ inc_nb, const int* __restrict__ inc_id,
    const float* __restrict__ pcoef, double pair_coef, const float* __restrict__ w,
    const float* __restrict__ V, int r, int ld, float* __restrict__ out, int ldo,
    double out_scale) {
  static_assert(G >= 4 && G <= 32, "four to thirty-two lanes per entry");
  constexpr int HW = 32;              // lanes per row
  constexpr int NG = HW / G;          // groups per row
  constexpr int CH = kPairStage / 2;  // entries staged per row and pass
  typedef float f4 __attribute__((ext_vector_type(4)));
  __shared__ int s_nb[kBlock / HW][CH];
  __shared__ float s_cf[kBlock / HW][CH];
  const int hl = threadIdx.x & (HW - 1), hid = threadIdx.x / HW;
  const int grp = hl / G, lane = hl & (G - 1);
  const int row = blockIdx.x * (kBlock / HW) + hid;
  int* nbw = s_nb[hid];
  float* cfw = s_cf[hid];
  if (row < n) {  // uniform over the half-wave
    const int c0 = 4 * lane;
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if (c_scale != 0.0) {
      for (int e = cptr[row] + grp; e < cptr[row + 1]; e += NG) {
        const int k = ccol[e];
        const float a = (float)(c_scale * (double)cval[e]);
        const f4 v = *reinterpret_cast<const f4*>(V + k * ld + c0);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] += a * v[t];
      }
    }
    const int e0 = inc_ptr[row];
    const int e1 = w != nullptr ? inc_ptr[row + 1] : e0;
    for (int base = e0; base < e1; base += CH) {
      const int cnt = min(CH, e1 - base);
#pragma unroll
      for (int q = 0; q < CH / HW; ++q) {
        const int j = hl + HW * q;
        if (j < cnt) {
          nbw[j] = inc_nb[base + j];
          const int id = inc_id[base + j];
          const double a = pcoef != nullptr ? (double)pcoef[id] : pair_coef;
          cfw[j] = (float)(a * (double)w[id]);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int j = grp; j < cnt; j += NG * kGU) {
        int p[kGU];
        float coef[kGU];
#pragma unroll
        for (int u = 0; u < kGU; ++u) {
          const int ju = j + u * NG;
          const bool ok = ju < cnt;
          p[u] = (ok ? nbw[ju] : row) * ld;
          coef[u] = ok ? cfw[ju] : 0.0f;
        }
        f4 vp[kGU];
#pragma unroll
        for (int u = 0; u < kGU; ++u) vp[u] = *reinterpret_cast<const f4*>(V + p[u] + c0);
#pragma unroll
        for (int u = 0; u < kGU; ++u)
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[t] += coef[u] * vp[u][t];
      }
      // the slots are read before the next pass stages over them
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      for (int o = G; o < HW; o <<= 1) acc[t] += __shfl_xor(acc[t], o, 64);
    if (grp == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (c0 + t < r) out[row * ldo + c0 + t] = (float)(out_scale * (double)acc[t]);
    }
  }
}

// ===========================================================================
// Line search of the mixed form on FP32 copies of U and D (PAIR, uniform
// coefficient, XCD chunk lists as k1_pair_ls): four columns per lane loaded as
// one 16-byte vector, G = pow2(ceil(r / 4)) >= 4 lanes per constraint.  The
// inner products are formed in FP32; p1 = 2 a (<U_j, D_k> + <U_k, D_j>) and
// p2 = 2 a <D_j, D_k> are rounded to FP64 in the group's LDS slots and the
// seven sums of the quartic run in FP64 with z, b and lam (all FP64) read as
// contiguous runs.  Rows need ld >= 4 G (zero padding).
template <int G>
__global__ void __launch_bounds__(kBlock) k1_pair_ls_f32(
    const int* __restrict__ xoff, const int* __restrict__ chunk_row,
    const int* __restrict__ chunk_start, const int* __restrict__ chunk_end,
    const int* __restrict__ pk, double pair_coef, const float* __restrict__ U,
    const float* __restrict__ D, int ld, const double* __restrict__ z,
    const double* __restrict__ b, const double* __restrict__ lam, double* __restrict__ part) {
  static_assert(G >= 4, "the chunk results are staged per group");
  typedef float f4 __attribute__((ext_vector_type(4)));
  __shared__ double s1[(kBlock / G) * kPairChunk];
  __shared__ double s2[(kBlock / G) * kPairChunk];
  __shared__ double sh[kBlock / 64];
  const int chunk = xchunk_of(xoff, G);
  const int lane = threadIdx.x & (G - 1);
  const int gslot = (threadIdx.x / G) * kPairChunk;
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (chunk >= 0) {
    const int row = chunk_row[chunk];
    const int i0 = chunk_start[chunk], i1 = chunk_end[chunk];
    const int c0 = 4 * lane;
    const f4 uj = *reinterpret_cast<const f4*>(U + row * ld + c0);
    const f4 dj = *reinterpret_cast<const f4*>(D + row * ld + c0);
    for (int i = i0; i < i1; i += kUnroll) {
      const int cnt = min(kUnroll, i1 - i);
      int k[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) k[u] = u < cnt ? pk[i + u] : row;
      f4 dk[kUnroll], uk[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        dk[u] = *reinterpret_cast<const f4*>(D + k[u] * ld + c0);
        uk[u] = *reinterpret_cast<const f4*>(U + k[u] * ld + c0);
      }
      float d[kUnroll], dd[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        float sa = uj[0] * dk[u][0];
        sa = fmaf(uk[u][0], dj[0], sa);
        float qa = dj[0] * dk[u][0];
#pragma unroll
        for (int v = 1; v < 4; ++v) {
          sa = fmaf(uj[v], dk[u][v], sa);
          sa = fmaf(uk[u][v], dj[v], sa);
          qa = fmaf(dj[v], dk[u][v], qa);
        }
        d[u] = sa;
        dd[u] = qa;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<G>(d[u]);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) dd[u] = group_sum<G>(dd[u]);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (lane == (u & (G - 1)) && u < cnt) {
          const int id = i + u;
          s1[gslot + (id - i0)] = 2.0 * ((double)d[u] * pair_coef);
          s2[gslot + (id - i0)] = 2.0 * pair_coef * (double)dd[u];
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q = lane; q < i1 - i0; q += G) {
      const double p1 = s1[gslot + q], p2 = s2[gslot + q];
      const double p0 = z[i0 + q] - b[i0 + q], l = lam[i0 + q];
      acc[0] += p2 * p2;
      acc[1] += p1 * p2;
      acc[2] += p1 * p1;
      acc[3] += p0 * p2;
      acc[4] += p0 * p1;
      acc[5] += l * p1;
      acc[6] += l * p2;
    }
  }
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    const double bs = block_sum(acc[t], sh);
    if (threadIdx.x == 0) part[(size_t)t * gridDim.x + blockIdx.x] = bs;
  }
}

// ===========================================================================
// PAIR CG operator on the CG layout (rows padded to 64 bytes, W and the
// direction interleaved: row p = [W_p | P_p], stride ldw = 2 ld, zero padding).
// A lane holds VW = 16 / sizeof(T) contiguous columns loaded as one 16-byte
// vector, so a constraint occupies G = pow2(ceil(r / VW)) lanes (4 for r <= 16
// in FP32) and its inner product needs log2 G lane moves; a wave serves 64 / G
// constraints per step.  Otherwise as kpair_rows MODE 1 (incident lists staged
// per wave in LDS, fixed-order sums, block partials of <P, Q>).
// Partner rows are read with buffer loads: the staged entry is the partner's
// byte offset (32-bit), the direction half sits at a scalar offset of ld
// elements, and reads past the buffer return zero.  The staged list of a chunk
// is padded to a whole number of steps with entries (own row, coefficient 0),
// so the step loop runs without lane guards.  The FP32 form's launch bound
// asks for 7 waves per SIMD (at most 72 VGPRs; the unbounded allocation gives
// 6), which measured 3% faster on the completion solves; the FP64 form and
// the X3 forms keep their natural allocation (7 waves would spill).
// X3 = 1 (ranks 17 .. 24, G VW = 16): each lane also holds VW / 2 columns
// from G VW + lane VW / 2 on, loaded as one 8-byte vector, so G lanes cover
// 24 columns (a quarter fewer bytes gathered than 32-column groups, twice the
// constraints per wave); the lane's chain runs on over those columns.  Needs
// ld >= 24.  The solver uses it in FP64 (whose 64-byte rows hold 24 columns
// at these ranks, too few for 16 lanes of two).
// ===========================================================================
template <typename T, int G, int X3 = 0>
__global__ void __launch_bounds__(kBlock, (sizeof(T) == 4 && !X3 ? 7 : 1)) kpair_cg_vec(
    int n, const int* __restrict__ inc_ptr, const int* __restrict__ inc_nb,
    const int* __restrict__ inc_id, const T* __restrict__ pcoef, double pair_coef,
    const T* __restrict__ WP, int ld, int r, T* __restrict__ Q, double* __restrict__ sc,
    int parity, double* __restrict__ part) {
  using A = typename OpAcc<T>::type;
  constexpr int VW = 16 / (int)sizeof(T);
  constexpr int VH = X3 ? VW / 2 : 1;  // columns of the lane's extra 8-byte vector
  constexpr int NG = 64 / G;
  constexpr int CH = kPairStage;
  constexpr int STEP = NG * kUnroll;  // entries per step of a wave (divides CH)
  static_assert(CH % STEP == 0, "staging chunk must hold whole steps");
  typedef T vec __attribute__((ext_vector_type(16 / sizeof(T))));
  typedef T hvec __attribute__((ext_vector_type(8 / sizeof(T))));
  __shared__ double sh[kBlock / 64];
  __shared__ int s_nb[kBlock / 64][CH];
  __shared__ A s_cf[kBlock / 64][CH];
  if (sc[S_DONE + parity] != 0.0) return;
  const int wl = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = wl / G, lane = wl & (G - 1);
  const int row = blockIdx.x * (kBlock / 64) + wid;
  const int ldw = 2 * ld;
  const int c0 = lane * VW;  // first column of this lane (c0 < ld: G * VW <= ld)
  const int rowb = ldw * (int)sizeof(T);  // bytes per row
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)WP, 0, n * rowb, kBufferRsrcWord3);
  const int pofs = ld * (int)sizeof(T);  // direction half of a row
  int* nbw = s_nb[wid];
  A* cfw = s_cf[wid];
  double pq = 0.0;
  if (row < n) {  // wave-uniform
    A acc[VW], pt[VW], vt[VW];
    {
      const vec w = *reinterpret_cast<const vec*>(WP + row * ldw + c0);
      const vec p = *reinterpret_cast<const vec*>(WP + row * ldw + ld + c0);
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        vt[v] = (A)w[v];
        pt[v] = (A)p[v];
        acc[v] = 0;
      }
    }
    const int cx = G * VW + lane * VH;  // first extra column (X3)
    const int xsh = (cx - c0) * (int)sizeof(T);
    A accx[VH], ptx[VH], vtx[VH];
#pragma unroll
    for (int h = 0; h < VH; ++h) {
      vtx[h] = X3 ? (A)WP[row * ldw + cx + h] : (A)0;
      ptx[h] = X3 ? (A)WP[row * ldw + ld + cx + h] : (A)0;
      accx[h] = 0;
    }
    const A a2u = (A)(pair_coef * pair_coef);
    const int own = row * rowb;
    const int e0 = inc_ptr[row], e1 = inc_ptr[row + 1];
    for (int base = e0; base < e1; base += CH) {
      const int cnt = min(CH, e1 - base);
      const int cntp = (cnt + STEP - 1) / STEP * STEP;
#pragma unroll
      for (int q = 0; q < CH / 64; ++q) {
        const int j = wl + 64 * q;
        if (j < cntp) {
          int off = own;
          A a2 = 0;
          if (j < cnt) {
            off = inc_nb[base + j] * rowb;
            a2 = a2u;
            if (pcoef != nullptr) {
              const A a = (A)pcoef[inc_id[base + j]];
              a2 = a * a;
            }
          }
          nbw[j] = off;
          cfw[j] = a2;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int j = grp; j < cntp; j += STEP) {
        int off[kUnroll];
        A coef[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          off[u] = nbw[j + u * NG] + c0 * (int)sizeof(T);
          coef[u] = cfw[j + u * NG];
        }
        vec wv[kUnroll], pv[kUnroll];
        hvec wx[kUnroll], px[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          wv[u] = __builtin_bit_cast(vec, __builtin_amdgcn_raw_buffer_load_b128(rs, off[u], 0, 0));
          pv[u] = __builtin_bit_cast(vec, __builtin_amdgcn_raw_buffer_load_b128(rs, off[u], pofs, 0));
          if (X3) {
            wx[u] = __builtin_bit_cast(hvec, __builtin_amdgcn_raw_buffer_load_b64(rs, off[u] + xsh, 0, 0));
            px[u] = __builtin_bit_cast(hvec, __builtin_amdgcn_raw_buffer_load_b64(rs, off[u] + xsh, pofs, 0));
          }
        }
        A d[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          // one fused multiply-add chain over the lane's columns
          A s = pt[0] * (A)wv[u][0];
          s = fma((A)pv[u][0], vt[0], s);
#pragma unroll
          for (int v = 1; v < VW; ++v) {
            s = fma(pt[v], (A)wv[u][v], s);
            s = fma((A)pv[u][v], vt[v], s);
          }
          if (X3) {
#pragma unroll
            for (int h = 0; h < VH; ++h) {
              s = fma(ptx[h], (A)wx[u][h], s);
              s = fma((A)px[u][h], vtx[h], s);
            }
          }
          d[u] = s;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<G>(d[u]) * coef[u];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
          for (int v = 0; v < VW; ++v) acc[v] += d[u] * (A)wv[u][v];
          if (X3) {
#pragma unroll
            for (int h = 0; h < VH; ++h) accx[h] += d[u] * (A)wx[u][h];
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int v = 0; v < VW; ++v)
      for (int o = G; o < 64; o <<= 1) acc[v] += __shfl_xor(acc[v], o, 64);
    if (X3) {
#pragma unroll
      for (int h = 0; h < VH; ++h)
        for (int o = G; o < 64; o <<= 1) accx[h] += __shfl_xor(accx[h], o, 64);
    }
    if (grp == 0) {
      const double gamma = sc[S_GAMMA], rho = sc[S_RHO];
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        const int c = c0 + v;
        if (c < r) {
          const T qv = (T)(gamma * (double)pt[v] + rho * (double)acc[v]);
          Q[row * ld + c] = qv;
          pq += (double)pt[v] * (double)qv;
        }
      }
      if (X3) {
#pragma unroll
        for (int h = 0; h < VH; ++h) {
          const int c = cx + h;
          if (c < r) {
            const T qv = (T)(gamma * (double)ptx[h] + rho * (double)accx[h]);
            Q[row * ld + c] = qv;
            pq += (double)ptx[h] * (double)qv;
          }
        }
      }
    }
  }
  publish_partial(block_sum(pq, sh), part);
}

// ===========================================================================
// The PAIR CG operator split by XCD (factor arrays larger than one XCD's L2):
// workgroup b serves partner block x = b mod kXcds.  A wave takes one row's
// incident entries whose partners lie in block x (the row's list is sorted by
// partner, so they are the run inc_xptr[row (kXcds + 1) + x] ..
// inc_xptr[row (kXcds + 1) + x + 1]) and writes that run's part of
// rho^-1 (Q - gamma P) for the row, sum_e a^2 (<P_row, W_p> + <P_p, W_row>) W_p,
// to xparts[(x n + row) ld + c]; an XCD thus gathers the [W | P] rows of one
// block only.  Otherwise the computation of kpair_cg_vec (same staging,
// buffer loads, per-group order within the run and X3 form).  xcg_combine then forms
// Q = gamma P + rho sum_x xparts[x] in block order and the partials of <P, Q>.
// ===========================================================================
template <typename T, int G, int X3 = 0>
__global__ void __launch_bounds__(kBlock, (sizeof(T) == 4 && !X3 ? 7 : 1)) kpair_cg_xvec(
    int n, const int* __restrict__ inc_xptr, const int* __restrict__ inc_nb,
    const int* __restrict__ inc_id, const T* __restrict__ pcoef, double pair_coef,
    const T* __restrict__ WP, int ld, int r, typename OpAcc<T>::type* __restrict__ xparts,
    const double* __restrict__ sc, int parity) {
  using A = typename OpAcc<T>::type;
  constexpr int VW = 16 / (int)sizeof(T);
  constexpr int VH = X3 ? VW / 2 : 1;  // columns of the lane's extra 8-byte vector
  constexpr int NG = 64 / G;
  constexpr int CH = kPairStage;
  constexpr int STEP = NG * kUnroll;
  static_assert(CH % STEP == 0, "staging chunk must hold whole steps");
  typedef T vec __attribute__((ext_vector_type(16 / sizeof(T))));
  typedef T hvec __attribute__((ext_vector_type(8 / sizeof(T))));
  __shared__ int s_nb[kBlock / 64][CH];
  __shared__ A s_cf[kBlock / 64][CH];
  if (sc[S_DONE + parity] != 0.0) return;
  const int wl = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = wl / G, lane = wl & (G - 1);
  const int x = blockIdx.x % kXcds;
  const int row = (blockIdx.x / kXcds) * (kBlock / 64) + wid;
  if (row >= n) return;  // wave-uniform; no block-wide synchronisation follows
  const int ldw = 2 * ld;
  const int c0 = lane * VW;
  const int rowb = ldw * (int)sizeof(T);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)WP, 0, n * rowb, kBufferRsrcWord3);
  const int pofs = ld * (int)sizeof(T);
  int* nbw = s_nb[wid];
  A* cfw = s_cf[wid];
  A acc[VW], pt[VW], vt[VW];
  {
    const vec w = *reinterpret_cast<const vec*>(WP + row * ldw + c0);
    const vec p = *reinterpret_cast<const vec*>(WP + row * ldw + ld + c0);
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      vt[v] = (A)w[v];
      pt[v] = (A)p[v];
      acc[v] = 0;
    }
  }
  const int cx = G * VW + lane * VH;  // first extra column (X3)
  const int xsh = (cx - c0) * (int)sizeof(T);
  A accx[VH], ptx[VH], vtx[VH];
#pragma unroll
  for (int h = 0; h < VH; ++h) {
    vtx[h] = X3 ? (A)WP[row * ldw + cx + h] : (A)0;
    ptx[h] = X3 ? (A)WP[row * ldw + ld + cx + h] : (A)0;
    accx[h] = 0;
  }
  const A a2u = (A)(pair_coef * pair_coef);
  const int own = row * rowb;
  const int e0 = inc_xptr[row * (kXcds + 1) + x], e1 = inc_xptr[row * (kXcds + 1) + x + 1];
  for (int base = e0; base < e1; base += CH) {
    const int cnt = min(CH, e1 - base);
    const int cntp = (cnt + STEP - 1) / STEP * STEP;
#pragma unroll
    for (int q = 0; q < CH / 64; ++q) {
      const int j = wl + 64 * q;
      if (j < cntp) {
        int off = own;
        A a2 = 0;
        if (j < cnt) {
          off = inc_nb[base + j] * rowb;
          a2 = a2u;
          if (pcoef != nullptr) {
            const A a = (A)pcoef[inc_id[base + j]];
            a2 = a * a;
          }
        }
        nbw[j] = off;
        cfw[j] = a2;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int j = grp; j < cntp; j += STEP) {
      int off[kUnroll];
      A coef[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        off[u] = nbw[j + u * NG] + c0 * (int)sizeof(T);
        coef[u] = cfw[j + u * NG];
      }
      vec wv[kUnroll], pv[kUnroll];
      hvec wx[kUnroll], px[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        wv[u] = __builtin_bit_cast(vec, __builtin_amdgcn_raw_buffer_load_b128(rs, off[u], 0, 0));
        pv[u] = __builtin_bit_cast(vec, __builtin_amdgcn_raw_buffer_load_b128(rs, off[u], pofs, 0));
        if (X3) {
          wx[u] = __builtin_bit_cast(hvec, __builtin_amdgcn_raw_buffer_load_b64(rs, off[u] + xsh, 0, 0));
          px[u] = __builtin_bit_cast(hvec, __builtin_amdgcn_raw_buffer_load_b64(rs, off[u] + xsh, pofs, 0));
        }
      }
      A d[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        A sm = pt[0] * (A)wv[u][0];
        sm = fma((A)pv[u][0], vt[0], sm);
#pragma unroll
        for (int v = 1; v < VW; ++v) {
          sm = fma(pt[v], (A)wv[u][v], sm);
          sm = fma((A)pv[u][v], vt[v], sm);
        }
        if (X3) {
#pragma unroll
          for (int h = 0; h < VH; ++h) {
            sm = fma(ptx[h], (A)wx[u][h], sm);
            sm = fma((A)px[u][h], vtx[h], sm);
          }
        }
        d[u] = sm;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) d[u] = group_sum<G>(d[u]) * coef[u];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[v] += d[u] * (A)wv[u][v];
        if (X3) {
#pragma unroll
          for (int h = 0; h < VH; ++h) accx[h] += d[u] * (A)wx[u][h];
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
#pragma unroll
  for (int v = 0; v < VW; ++v)
    for (int o = G; o < 64; o <<= 1) acc[v] += __shfl_xor(acc[v], o, 64);
  if (X3) {
#pragma unroll
    for (int h = 0; h < VH; ++h)
      for (int o = G; o < 64; o <<= 1) accx[h] += __shfl_xor(accx[h], o, 64);
  }
  if (grp == 0) {
    A* dst = xparts + ((size_t)x * n + row) * ld;
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      const int c = c0 + v;
      if (c < r) dst[c] = acc[v];
    }
    if (X3) {
#pragma unroll
      for (int h = 0; h < VH; ++h) {
        const int c = cx + h;
        if (c < r) dst[c] = accx[h];
      }
    }
  }
}

// Q = gamma P + rho sum_x xparts[x] (x = 0 .. kXcds - 1 in order) over the
// first r columns of each row, with the block partials of <P, Q>; P is the
// direction half of the interleaved rows [W | P] (stride 2 ld).
template <typename T>
__global__ void __launch_bounds__(kBlock) xcg_combine(
    int n, int r, int ld, const typename OpAcc<T>::type* __restrict__ xparts,
    const T* __restrict__ WP, T* __restrict__ Q, const double* __restrict__ sc, int parity,
    double* __restrict__ part) {
  using A = typename OpAcc<T>::type;
  __shared__ double sh[kBlock / 64];
  if (sc[S_DONE + parity] != 0.0) return;
  const double gamma = sc[S_GAMMA], rho = sc[S_RHO];
  const size_t N = (size_t)n * r, plane = (size_t)n * ld;
  double pq = 0.0;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
    const size_t row = i / (unsigned)r;
    const int c = (int)(i - row * (unsigned)r);
    const size_t q = row * ld + c;
    A acc = xparts[q];
#pragma unroll
    for (int x = 1; x < kXcds; ++x) acc += xparts[x * plane + q];
    const A pt = (A)WP[row * 2 * ld + ld + c];
    const T qv = (T)(gamma * (double)pt + rho * (double)acc);
    Q[q] = qv;
    pq += (double)pt * (double)qv;
  }
  publish_partial(block_sum(pq, sh), part);
}

}  // namespace lorads
