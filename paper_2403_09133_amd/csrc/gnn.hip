// Learned Phase-I warm start: a message-passing network over the constraint
// graph (for MaxCut, the graph itself) that predicts a dual multiplier per node
// and a graph-level rank factor.  The paper lists better warm starts as future
// work (Section 6); the network and its training are an addition.
//
// Everything is FP32 and resident on the device: the graph set, its features,
// all activations, parameters, gradient and Adam moments.  A training step is
// a short chain of kernels over a contiguous range of graphs:
//
//   input layer   H0 = relu(x W_in^T + b_in)                 (row-wise)
//   layer l       M = A H_{l-1}  (one wave per row, lane = channel)
//                 H_l = relu([H_{l-1} | M] [W_s | W_n]^T + b) (FP32 MFMA 16x16x4)
//   heads         yhat, per-graph mean pool, rhat, loss, head gradients
//   layer l bwd   dZ = dH o [H_l > 0]; [dM | dH_self] = dZ [W_n | W_s] (MFMA);
//                 [gW_s | gW_n] += dZ^T [H_{l-1} | M]  (MFMA, split over blocks)
//                 dH_{l-1} = dH_self + A^T dM  (A^T through the symmetric rows)
//   Adam
//
// Reductions are deterministic: blocks write partials in a fixed grid and a
// finishing kernel sums them in block order.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <numeric>

#include "common.hpp"

namespace lorads {
namespace {

constexpr int kH = 64;        // hidden width
constexpr int kF = 8;         // padded feature count (5 used)
constexpr int kFUsed = 5;
constexpr int kTile = 64;     // rows per MFMA tile
constexpr int kBwdBlocks = 512;
constexpr int kHeadBlocks = 512;

typedef float flt4 __attribute__((ext_vector_type(4)));

// accumulator element v of lane l of v_mfma_f32_16x16x4f32 holds D[4 (l/16) + v][l % 16];
// operand A of lane l is A[l % 16][l / 16] (M x K), operand B is B[l / 16][l % 16] (K x N)
__device__ __forceinline__ int drow(int lane, int v) { return 4 * (lane >> 4) + v; }

struct Offsets {
  int64_t w_in, b_in, vy, cy, vr, cr, total;
  int64_t ws(int l) const { return 384 + (int64_t)l * (2 * kH * kH + kH); }
  int64_t wn(int l) const { return ws(l) + kH * kH; }
  int64_t b(int l) const { return ws(l) + 2 * kH * kH; }
  explicit Offsets(int layers) {
    w_in = 0;
    b_in = kH * kFUsed;
    vy = 384 + (int64_t)layers * (2 * kH * kH + kH);
    cy = vy + kH;
    vr = cy + 1;
    cr = vr + kH;
    total = cr + 1;
  }
};

__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// features and normalised edge weights (once per graph set)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) features_kernel(int64_t N, const int64_t* __restrict__ rptr,
                                                       const float* __restrict__ w,
                                                       const int* __restrict__ gid,
                                                       const int64_t* __restrict__ node_off,
                                                       float* __restrict__ x,
                                                       float* __restrict__ inv_rs,
                                                       float* __restrict__ an) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double deg = 0, sw = 0, sa = 0, s2 = 0;
  for (int64_t e = rptr[j]; e < rptr[j + 1]; ++e) {
    const double v = w[e];
    deg += 1.0; sw += v; sa += fabs(v); s2 += v * v;
  }
  const int g = gid[j];
  const double ng = (double)(node_off[g + 1] - node_off[g]);
  float* xj = x + j * kF;
  xj[0] = (float)(deg / 10.0);
  xj[1] = (float)(sw / 10.0);
  xj[2] = (float)(sa / 10.0);
  xj[3] = (float)(s2 / 10.0);
  xj[4] = (float)(log(ng) / 10.0);
  xj[5] = xj[6] = xj[7] = 0.0f;
  const double inv = 1.0 / (1.0 + sa);
  inv_rs[j] = (float)inv;
  for (int64_t e = rptr[j]; e < rptr[j + 1]; ++e) an[e] = (float)(w[e] * inv);
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) input_fwd(int64_t n0, int64_t n1, const float* __restrict__ x,
                                                 const float* __restrict__ theta,
                                                 float* __restrict__ H0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = n0 + t / kH;
  const int c = (int)(t % kH);
  if (j >= n1) return;
  const float* W = theta;  // W_in (64 x 5), then b_in
  float z = theta[kH * kFUsed + c];
  for (int f = 0; f < kFUsed; ++f) z += W[c * kFUsed + f] * x[j * kF + f];
  H0[j * kH + c] = fmaxf(z, 0.0f);
}

// sum over the adjacency row of row j of coef[e] * X[col[e], lane]
__device__ __forceinline__ float row_gather(int64_t j, const int64_t* __restrict__ rptr,
                                            const int* __restrict__ col,
                                            const float* __restrict__ coef,
                                            const float* __restrict__ X, int lane) {
  const int64_t e0 = rptr[j], e1 = rptr[j + 1];
  float acc = 0.0f;
  for (int64_t base = e0; base < e1; base += 64) {
    const int cnt = (int)min<int64_t>(64, e1 - base);
    int myc = 0;
    float myw = 0.0f;
    if (lane < cnt) { myc = col[base + lane]; myw = coef[base + lane]; }
    int u = 0;
    for (; u + 4 <= cnt; u += 4) {
      const int c0 = __shfl(myc, u, 64), c1 = __shfl(myc, u + 1, 64);
      const int c2 = __shfl(myc, u + 2, 64), c3 = __shfl(myc, u + 3, 64);
      const float w0 = __shfl(myw, u, 64), w1 = __shfl(myw, u + 1, 64);
      const float w2 = __shfl(myw, u + 2, 64), w3 = __shfl(myw, u + 3, 64);
      const float h0 = X[(size_t)c0 * kH + lane], h1 = X[(size_t)c1 * kH + lane];
      const float h2 = X[(size_t)c2 * kH + lane], h3 = X[(size_t)c3 * kH + lane];
      acc += w0 * h0;
      acc += w1 * h1;
      acc += w2 * h2;
      acc += w3 * h3;
    }
    for (; u < cnt; ++u) {
      const int c = __shfl(myc, u, 64);
      const float wv = __shfl(myw, u, 64);
      acc += wv * X[(size_t)c * kH + lane];
    }
  }
  return acc;
}

// One block = 64 rows.  M rows by message aggregation, then
// Z = [H_prev | M] [W_s | W_n]^T + b on MFMA, H = relu(Z).
__global__ void __launch_bounds__(256) layer_fwd(int64_t n0, int64_t n1,
                                                 const int64_t* __restrict__ rptr,
                                                 const int* __restrict__ col,
                                                 const float* __restrict__ an,
                                                 const float* __restrict__ Hp,
                                                 const float* __restrict__ Ws,
                                                 const float* __restrict__ Wn,
                                                 const float* __restrict__ bias,
                                                 float* __restrict__ M, float* __restrict__ Ho) {
  constexpr int SA = 2 * kH + 4;  // [H_prev | M] tile, row stride
  constexpr int SB = kH + 4;      // B operand [k][j] = W[j][k], row stride
  __shared__ float sA[kTile * SA];
  __shared__ float sB[2 * kH * SB];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t row0 = n0 + (int64_t)blockIdx.x * kTile;
  // weights: sB[k][j] = Ws[j][k] (k < 64), Wn[j][k - 64] (k >= 64)
  for (int idx = tid; idx < kH * kH; idx += 256) {
    const int j = idx / kH, k = idx % kH;
    sB[k * SB + j] = Ws[idx];
    sB[(k + kH) * SB + j] = Wn[idx];
  }
  // H_prev tile
  for (int idx = tid; idx < kTile * (kH / 4); idx += 256) {
    const int r = idx / (kH / 4), q = idx % (kH / 4);
    const int64_t j = row0 + r;
    flt4 v = {0.f, 0.f, 0.f, 0.f};
    if (j < n1) v = *reinterpret_cast<const flt4*>(Hp + j * kH + 4 * q);
    float* d = sA + r * SA + 4 * q;
    d[0] = v[0]; d[1] = v[1]; d[2] = v[2]; d[3] = v[3];
  }
  // aggregation: wave wid owns tile rows wid*16 .. wid*16+15
  for (int rr = 0; rr < 16; ++rr) {
    const int r = wid * 16 + rr;
    const int64_t j = row0 + r;
    float acc = 0.0f;
    if (j < n1) {
      acc = row_gather(j, rptr, col, an, Hp, lane);
      M[j * kH + lane] = acc;
    }
    sA[r * SA + kH + lane] = acc;
  }
  __syncthreads();
  flt4 acc[4];
  for (int ct = 0; ct < 4; ++ct) acc[ct] = flt4{0.f, 0.f, 0.f, 0.f};
  const int ar = wid * 16 + (lane & 15), kk = lane >> 4;
#pragma unroll 4
  for (int s = 0; s < 2 * kH / 4; ++s) {
    const float a = sA[ar * SA + 4 * s + kk];
    const float* brow = sB + (4 * s + kk) * SB + (lane & 15);
    acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, brow[0], acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, brow[16], acc[1], 0, 0, 0);
    acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, brow[32], acc[2], 0, 0, 0);
    acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, brow[48], acc[3], 0, 0, 0);
  }
  for (int ct = 0; ct < 4; ++ct) {
    const int c = ct * 16 + (lane & 15);
    const float bc = bias[c];
    for (int v = 0; v < 4; ++v) {
      const int64_t j = row0 + wid * 16 + drow(lane, v);
      if (j < n1) Ho[j * kH + c] = fmaxf(acc[ct][v] + bc, 0.0f);
    }
  }
}

// yhat_j = <H_L[j], v_y> + c_y.  With targets: dy_j = 2 (yhat_j - y_j) / Nr and
// per-block partials of sum e^2, sum dy and sum dy_j H_L[j] (layout kH + 2 per block).
__global__ void __launch_bounds__(256) head_nodes(int64_t n0, int64_t n1,
                                                  const float* __restrict__ HL,
                                                  const float* __restrict__ theta, int64_t vy,
                                                  const float* __restrict__ y,
                                                  float* __restrict__ yhat,
                                                  float* __restrict__ dy,
                                                  double* __restrict__ part) {
  __shared__ double red[4][kH + 2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const float vyc = theta[vy + lane], cy = theta[vy + kH];
  const double inv_n = 1.0 / (double)(n1 - n0);
  double g = 0.0, e2 = 0.0, sdy = 0.0;
  for (int64_t j = n0 + (int64_t)blockIdx.x * 4 + wid; j < n1; j += (int64_t)gridDim.x * 4) {
    const float h = HL[j * kH + lane];
    const float yh = wave_sum(h * vyc) + cy;
    if (lane == 0) yhat[j] = yh;
    if (y) {
      const double e = (double)yh - (double)y[j];
      const float d = (float)(2.0 * e * inv_n);
      if (lane == 0) dy[j] = d;
      g += (double)d * h;
      e2 += e * e;
      sdy += d;
    }
  }
  if (!y) return;
  red[wid][lane] = g;
  if (lane == 0) { red[wid][kH] = e2; red[wid][kH + 1] = sdy; }
  __syncthreads();
  if (wid == 0) {
    for (int q = lane; q < kH + 2; q += 64) {
      const double s = red[0][q] + red[1][q] + red[2][q] + red[3][q];
      part[(size_t)blockIdx.x * (kH + 2) + q] = s;
    }
  }
}

// one block per graph: pool = mean of H_L rows, rhat = <pool, v_r> + c_r;
// with targets: dr = 2 omega (rhat - r) / Gr and er2 = (rhat - r)^2
__global__ void __launch_bounds__(256) pool_graphs(int g0, const int64_t* __restrict__ node_off,
                                                   const float* __restrict__ HL,
                                                   const float* __restrict__ theta, int64_t vr,
                                                   const float* __restrict__ r, float omega,
                                                   int Gr, float* __restrict__ pool,
                                                   float* __restrict__ rhat,
                                                   float* __restrict__ dr,
                                                   double* __restrict__ er2) {
  __shared__ float red[4][kH];
  const int g = g0 + blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t a = node_off[g], b = node_off[g + 1];
  float s = 0.0f;
  for (int64_t j = a + wid; j < b; j += 4) s += HL[j * kH + lane];
  red[wid][lane] = s;
  __syncthreads();
  if (wid != 0) return;
  const float p = (red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane]) / (float)(b - a);
  pool[(size_t)g * kH + lane] = p;
  const float rh = wave_sum(p * theta[vr + lane]) + theta[vr + kH];
  if (lane == 0) {
    rhat[g] = rh;
    if (r) {
      const double e = (double)rh - (double)r[g];
      dr[g] = (float)(2.0 * omega * e / Gr);
      er2[g] = e * e;
    }
  }
}

// head gradients and the loss, one block of 256 threads:
// grad[v_y] = sum_blocks part, grad[c_y] = sum dy, grad[v_r] = sum_g dr_g pool_g,
// grad[c_r] = sum dr; loss = sum e^2 / Nr + omega sum er^2 / Gr
__global__ void __launch_bounds__(256) head_finish(int nblk, const double* __restrict__ part,
                                                   int g0, int g1,
                                                   const float* __restrict__ pool,
                                                   const float* __restrict__ dr,
                                                   const double* __restrict__ er2,
                                                   int64_t Nr, float omega,
                                                   int64_t vy, int64_t vr,
                                                   float* __restrict__ grad,
                                                   double* __restrict__ loss) {
  const int t = threadIdx.x;
  if (t < kH + 2) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * (kH + 2) + t];
    if (t < kH) grad[vy + t] = (float)s;
    else if (t == kH + 1) grad[vy + kH] = (float)s;
    else loss[1] = s / (double)Nr;  // t == kH: sum e^2
  } else if (t >= 128 && t < 128 + kH) {
    const int c = t - 128;
    double s = 0.0;
    for (int g = g0; g < g1; ++g) s += (double)dr[g] * pool[(size_t)g * kH + c];
    grad[vr + c] = (float)s;
  } else if (t == 192) {
    double s = 0.0, e = 0.0;
    for (int g = g0; g < g1; ++g) { s += dr[g]; e += er2[g]; }
    grad[vr + kH] = (float)s;
    loss[2] = (double)omega * e / (double)(g1 - g0);
  }
}

__global__ void loss_total(double* loss) { loss[0] = loss[1] + loss[2]; }

// ---------------------------------------------------------------------------
// backward through one message-passing layer.  Persistent blocks walk the
// 64-row tiles; each block accumulates its share of [gW_s | gW_n] and gb in
// MFMA accumulators and writes one partial (kH x 2kH + kH floats).
// head != 0: dH of the last layer comes from the heads,
//   dH[j][c] = dy_j v_y[c] + dr_{g(j)} v_r[c] / n_{g(j)}.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) layer_bwd(int64_t n0, int64_t n1, int head,
                                                 const float* __restrict__ dH,
                                                 const float* __restrict__ dy,
                                                 const float* __restrict__ dr,
                                                 const int* __restrict__ gid,
                                                 const int64_t* __restrict__ node_off,
                                                 const float* __restrict__ theta, int64_t vy,
                                                 int64_t vr, const float* __restrict__ Hl,
                                                 const float* __restrict__ Hp,
                                                 const float* __restrict__ M,
                                                 const float* __restrict__ Ws,
                                                 const float* __restrict__ Wn,
                                                 const float* __restrict__ inv_rs,
                                                 float* __restrict__ dHs,
                                                 float* __restrict__ dMs,
                                                 float* __restrict__ part) {
  constexpr int SZ = kH + 4;
  constexpr int SW = 2 * kH + 4;
  __shared__ float sZ[kTile * SZ];
  __shared__ float sW[kH * SW];  // B operand [k = out][j]: Wn[out][in] (j < 64), Ws[out][in] (j >= 64)
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int idx = tid; idx < kH * kH; idx += 256) {
    const int o = idx / kH, i = idx % kH;
    sW[o * SW + i] = Wn[idx];
    sW[o * SW + kH + i] = Ws[idx];
  }
  flt4 gw[4][2];
  for (int a = 0; a < 4; ++a) gw[a][0] = gw[a][1] = flt4{0.f, 0.f, 0.f, 0.f};
  float gb = 0.0f;
  const int64_t ntiles = (n1 - n0 + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = n0 + tile * kTile;
    __syncthreads();  // previous tile's readers of sZ are done (and sW is ready)
    for (int idx = tid; idx < kTile * kH; idx += 256) {
      const int r = idx / kH, c = idx % kH;
      const int64_t j = row0 + r;
      float d = 0.0f;
      if (j < n1) {
        float g;
        if (head) {
          const int q = gid[j];
          const float cnt = (float)(node_off[q + 1] - node_off[q]);
          g = dy[j] * theta[vy + c] + dr[q] * theta[vr + c] / cnt;
        } else {
          g = dH[j * kH + c];
        }
        d = Hl[j * kH + c] > 0.0f ? g : 0.0f;
      }
      sZ[r * SZ + c] = d;
    }
    __syncthreads();
    if (tid < kH) {
      float s = 0.0f;
      for (int r = 0; r < kTile; ++r) s += sZ[r * SZ + tid];
      gb += s;
    }
    // [dM | dH_self] = dZ [W_n | W_s]: wave rows wid*16.., 8 column tiles
    {
      flt4 acc[8];
      for (int ct = 0; ct < 8; ++ct) acc[ct] = flt4{0.f, 0.f, 0.f, 0.f};
      const int ar = wid * 16 + (lane & 15), kk = lane >> 4;
#pragma unroll 2
      for (int s = 0; s < kH / 4; ++s) {
        const float a = sZ[ar * SZ + 4 * s + kk];
        const float* brow = sW + (4 * s + kk) * SW + (lane & 15);
#pragma unroll
        for (int ct = 0; ct < 8; ++ct)
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, brow[16 * ct], acc[ct], 0, 0, 0);
      }
      for (int ct = 0; ct < 8; ++ct) {
        const int c = (ct & 3) * 16 + (lane & 15);
        for (int v = 0; v < 4; ++v) {
          const int64_t j = row0 + wid * 16 + drow(lane, v);
          if (j < n1) {
            if (ct < 4) dMs[j * kH + c] = acc[ct][v] * inv_rs[j];
            else dHs[j * kH + c] = acc[ct][v];
          }
        }
      }
    }
    // [gW_s | gW_n] += dZ^T [H_prev | M]: wave wid owns input columns
    // wid*32 .. wid*32+31 of the 128 (waves 0,1: H_prev; 2,3: M)
    {
      const float* src = (wid < 2) ? Hp : M;
      const int cbase = (wid & 1) * 32;
      const int kk = lane >> 4;
      for (int s = 0; s < kTile / 4; ++s) {
        const int r = 4 * s + kk;
        const int64_t j = row0 + r;
        float b0 = 0.0f, b1 = 0.0f;
        if (j < n1) {
          b0 = src[j * kH + cbase + (lane & 15)];
          b1 = src[j * kH + cbase + 16 + (lane & 15)];
        }
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
          const float a = sZ[r * SZ + ot * 16 + (lane & 15)];
          gw[ot][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b0, gw[ot][0], 0, 0, 0);
          gw[ot][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b1, gw[ot][1], 0, 0, 0);
        }
      }
    }
  }
  // partial layout: [out][128] then gb[64]
  float* P = part + (size_t)blockIdx.x * (kH * 2 * kH + kH);
  for (int ot = 0; ot < 4; ++ot)
    for (int h = 0; h < 2; ++h) {
      const int in = wid * 32 + h * 16 + (lane & 15);
      for (int v = 0; v < 4; ++v) P[(ot * 16 + drow(lane, v)) * 2 * kH + in] = gw[ot][h][v];
    }
  if (tid < kH) P[kH * 2 * kH + tid] = gb;
}

// gW_s, gW_n, gb of one layer: sums of the block partials in block order
__global__ void __launch_bounds__(256) layer_grad_finish(int nblk, const float* __restrict__ part,
                                                         float* __restrict__ gWs,
                                                         float* __restrict__ gWn,
                                                         float* __restrict__ gb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int per = kH * 2 * kH + kH;
  if (t >= per) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * per + t];
  if (t < kH * 2 * kH) {
    const int o = t / (2 * kH), i = t % (2 * kH);
    if (i < kH) gWs[o * kH + i] = (float)s;
    else gWn[o * kH + i - kH] = (float)s;
  } else {
    gb[t - kH * 2 * kH] = (float)s;
  }
}

// dH_prev[k] = dH_self[k] + sum_{j in row k} w_kj dMs[j]   (dMs = dM / (1 + sum |w|))
__global__ void __launch_bounds__(256) spmm_bwd(int64_t n0, int64_t n1,
                                                const int64_t* __restrict__ rptr,
                                                const int* __restrict__ col,
                                                const float* __restrict__ w,
                                                const float* __restrict__ dHs,
                                                const float* __restrict__ dMs,
                                                float* __restrict__ dH) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t k = n0 + (int64_t)blockIdx.x * 4 + wid;
  if (k >= n1) return;
  dH[k * kH + lane] = dHs[k * kH + lane] + row_gather(k, rptr, col, w, dMs, lane);
}

// input layer gradient partials: per block [gW_in (64 x 5) | gb_in (64)]
__global__ void __launch_bounds__(256) input_bwd(int64_t n0, int64_t n1,
                                                 const float* __restrict__ dH0,
                                                 const float* __restrict__ H0,
                                                 const float* __restrict__ x,
                                                 float* __restrict__ part) {
  __shared__ float red[4][kH][kFUsed + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float s[kFUsed + 1] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int64_t j = n0 + (int64_t)blockIdx.x * 4 + wid; j < n1; j += (int64_t)gridDim.x * 4) {
    const float d = H0[j * kH + lane] > 0.0f ? dH0[j * kH + lane] : 0.0f;
    for (int f = 0; f < kFUsed; ++f) s[f] += d * x[j * kF + f];
    s[kFUsed] += d;
  }
  for (int f = 0; f <= kFUsed; ++f) red[wid][lane][f] = s[f];
  __syncthreads();
  if (wid != 0) return;
  float* P = part + (size_t)blockIdx.x * kH * (kFUsed + 1);
  for (int f = 0; f <= kFUsed; ++f)
    P[lane * (kFUsed + 1) + f] = red[0][lane][f] + red[1][lane][f] + red[2][lane][f] + red[3][lane][f];
}

__global__ void __launch_bounds__(256) input_grad_finish(int nblk, const float* __restrict__ part,
                                                         float* __restrict__ grad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int per = kH * (kFUsed + 1);
  if (t >= per) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * per + t];
  const int c = t / (kFUsed + 1), f = t % (kFUsed + 1);
  if (f < kFUsed) grad[c * kFUsed + f] = (float)s;
  else grad[kH * kFUsed + c] = (float)s;
}

__global__ void __launch_bounds__(256) adam_kernel(int64_t P, float* __restrict__ theta,
                                                   const float* __restrict__ g,
                                                   float* __restrict__ m1,
                                                   float* __restrict__ m2, float lr, float b1,
                                                   float b2, float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  theta[i] -= lr * (a / bc1) / (sqrtf(b / bc2) + eps);
}

}  // namespace
}  // namespace lorads

using namespace lorads;

struct lorads_gnn {
  int layers = 0;
  Offsets off{1};
  hipStream_t stream = nullptr;
  DevBuf<float> theta, grad, m1, m2;
  int64_t adam_t = 0;
  bool have_grad = false;
  // graph set
  int G = 0;
  int64_t N = 0, E = 0;
  std::vector<int64_t> h_node_off;
  DevBuf<int64_t> node_off, rptr;
  DevBuf<int> gid, col;
  DevBuf<float> w, an, inv_rs, x;
  DevBuf<float> y, r;
  bool have_targets = false;
  // activations
  DevBuf<float> H, M, dH, dHs, dMs, yhat, dy, pool, rhat, dr;
  DevBuf<double> er2, hpart, loss;
  DevBuf<float> wpart;
  // layer timing (events recycled through a free list)
  std::vector<hipEvent_t> ev, free_ev;
  double t_ms = 0, flops = 0;
  int64_t launches = 0;
  lorads_gnn(int L) : layers(L), off(L) {}
  ~lorads_gnn() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : free_ev) (void)hipEventDestroy(e);
  }
  float* Hl(int l) { return H.p + (size_t)l * N * kH; }
  float* Ml(int l) { return M.p + (size_t)(l - 1) * N * kH; }
};

namespace {

template <typename F>
lorads_status gguard(F&& f) {
  try {
    f();
    return LORADS_OK;
  } catch (const lorads::Error& e) {
    lorads::set_global_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    lorads::set_global_error("host allocation failed");
    return LORADS_ENOMEM;
  } catch (const std::exception& e) {
    lorads::set_global_error(e.what());
    return LORADS_EDEVICE;
  }
}

lorads_gnn& chk(lorads_gnn* g) {
  if (!g) fail(LORADS_EINVAL, "null network");
  return *g;
}

void check_range(const lorads_gnn& g, int g0, int g1) {
  if (g.G == 0) fail(LORADS_ESTATE, "no graph set loaded");
  if (g0 < 0 || g1 > g.G || g0 >= g1) fail(LORADS_EINVAL, "graph range out of bounds");
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void resolve_timing(lorads_gnn& g);

hipEvent_t take_event(lorads_gnn& g) {
  hipEvent_t e;
  if (!g.free_ev.empty()) {
    e = g.free_ev.back();
    g.free_ev.pop_back();
  } else {
    HIPCHK(hipEventCreate(&e));
  }
  return e;
}

// time a launch on the network's stream (message-passing layer kernels only)
template <typename L>
void timed(lorads_gnn& g, double flops, L&& launch) {
  if (g.ev.size() >= 4096) resolve_timing(g);
  hipEvent_t a = take_event(g), b = take_event(g);
  HIPCHK(hipEventRecord(a, g.stream));
  launch();
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(b, g.stream));
  g.ev.push_back(a);
  g.ev.push_back(b);
  g.flops += flops;
  ++g.launches;
}

void resolve_timing(lorads_gnn& g) {
  if (g.ev.empty()) return;
  HIPCHK(hipEventSynchronize(g.ev.back()));
  for (size_t i = 0; i + 1 < g.ev.size(); i += 2) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, g.ev[i], g.ev[i + 1]));
    g.t_ms += ms;
  }
  g.free_ev.insert(g.free_ev.end(), g.ev.begin(), g.ev.end());
  g.ev.clear();
}

void forward(lorads_gnn& g, int g0, int g1, bool train, float omega) {
  const int64_t n0 = g.h_node_off[g0], n1 = g.h_node_off[g1], Nr = n1 - n0;
  const int L = g.layers;
  hipStream_t s = g.stream;
  const float* th = g.theta.p;
  input_fwd<<<blocks_for(Nr * kH, 256), 256, 0, s>>>(n0, n1, g.x.p, th, g.Hl(0));
  HIPCHK(hipGetLastError());
  for (int l = 1; l <= L; ++l) {
    const unsigned tiles = blocks_for(Nr, kTile);
    timed(g, 2.0 * Nr * kH * 2 * kH, [&] {
      layer_fwd<<<tiles, 256, 0, s>>>(n0, n1, g.rptr.p, g.col.p, g.an.p, g.Hl(l - 1),
                                      th + g.off.ws(l - 1), th + g.off.wn(l - 1),
                                      th + g.off.b(l - 1), g.Ml(l), g.Hl(l));
    });
  }
  const int hb = (int)std::min<int64_t>(kHeadBlocks, blocks_for(Nr, 4));
  head_nodes<<<hb, 256, 0, s>>>(n0, n1, g.Hl(L), th, g.off.vy, train ? g.y.p : nullptr,
                                g.yhat.p, g.dy.p, g.hpart.p);
  HIPCHK(hipGetLastError());
  pool_graphs<<<g1 - g0, 256, 0, s>>>(g0, g.node_off.p, g.Hl(L), th, g.off.vr,
                                      train ? g.r.p : nullptr, omega, g1 - g0, g.pool.p,
                                      g.rhat.p, g.dr.p, g.er2.p);
  HIPCHK(hipGetLastError());
  if (train) {
    head_finish<<<1, 256, 0, s>>>(hb, g.hpart.p, g0, g1, g.pool.p, g.dr.p, g.er2.p, Nr, omega,
                                  g.off.vy, g.off.vr, g.grad.p, g.loss.p);
    loss_total<<<1, 1, 0, s>>>(g.loss.p);
    HIPCHK(hipGetLastError());
  }
}

void backward(lorads_gnn& g, int g0, int g1) {
  const int64_t n0 = g.h_node_off[g0], n1 = g.h_node_off[g1], Nr = n1 - n0;
  const int L = g.layers;
  hipStream_t s = g.stream;
  const float* th = g.theta.p;
  const int nb = (int)std::min<int64_t>(kBwdBlocks, blocks_for(Nr, kTile));
  for (int l = L; l >= 1; --l) {
    timed(g, 2.0 * 2.0 * Nr * kH * 2 * kH, [&] {
      layer_bwd<<<nb, 256, 0, s>>>(n0, n1, l == L ? 1 : 0, g.dH.p, g.dy.p, g.dr.p, g.gid.p,
                                   g.node_off.p, th, g.off.vy, g.off.vr, g.Hl(l), g.Hl(l - 1),
                                   g.Ml(l), th + g.off.ws(l - 1), th + g.off.wn(l - 1),
                                   g.inv_rs.p, g.dHs.p, g.dMs.p, g.wpart.p);
    });
    layer_grad_finish<<<blocks_for(kH * 2 * kH + kH, 256), 256, 0, s>>>(
        nb, g.wpart.p, g.grad.p + g.off.ws(l - 1), g.grad.p + g.off.wn(l - 1),
        g.grad.p + g.off.b(l - 1));
    HIPCHK(hipGetLastError());
    timed(g, 0.0, [&] {
      spmm_bwd<<<blocks_for(Nr, 4), 256, 0, s>>>(n0, n1, g.rptr.p, g.col.p, g.w.p, g.dHs.p,
                                                  g.dMs.p, g.dH.p);
    });
  }
  const int ib = (int)std::min<int64_t>(kHeadBlocks, blocks_for(Nr, 4));
  input_bwd<<<ib, 256, 0, s>>>(n0, n1, g.dH.p, g.Hl(0), g.x.p, g.wpart.p);
  input_grad_finish<<<blocks_for(kH * (kFUsed + 1), 256), 256, 0, s>>>(ib, g.wpart.p, g.grad.p);
  HIPCHK(hipGetLastError());
}

}  // namespace

extern "C" {

int64_t lorads_gnn_param_count(int32_t layers) {
  if (layers < 1 || layers > 8) return -1;
  return Offsets(layers).total;
}

lorads_status lorads_gnn_create(int32_t layers, lorads_gnn** out) {
  return gguard([&] {
    if (!out) fail(LORADS_EINVAL, "null output pointer");
    *out = nullptr;
    if (layers < 1 || layers > 8) fail(LORADS_EINVAL, "layers must be in [1, 8]");
    auto g = std::make_unique<lorads_gnn>(layers);
    const size_t P = (size_t)g->off.total;
    g->theta.alloc(P); g->grad.alloc(P); g->m1.alloc(P); g->m2.alloc(P);
    g->theta.zero(); g->grad.zero(); g->m1.zero(); g->m2.zero();
    g->loss.alloc(3);
    g->loss.zero();
    g->hpart.alloc((size_t)kHeadBlocks * (kH + 2));
    g->wpart.alloc((size_t)std::max(kBwdBlocks * (kH * 2 * kH + kH), kHeadBlocks * kH * (kFUsed + 1)));
    HIPCHK(hipDeviceSynchronize());
    *out = g.release();
  });
}

lorads_status lorads_gnn_set_params(lorads_gnn* gp, const float* theta, int64_t count) {
  return gguard([&] {
    lorads_gnn& g = chk(gp);
    if (!theta || count != g.off.total) fail(LORADS_EINVAL, "parameter count mismatch");
    for (int64_t i = 0; i < count; ++i)
      if (!std::isfinite(theta[i])) fail(LORADS_EINVAL, "non-finite parameter");
    g.theta.upload(theta, (size_t)count, g.stream);
    g.m1.zero(g.stream);
    g.m2.zero(g.stream);
    g.adam_t = 0;
    g.have_grad = false;
    HIPCHK(hipStreamSynchronize(g.stream));
  });
}

lorads_status lorads_gnn_get_params(const lorads_gnn* gp, float* theta, int64_t count) {
  return gguard([&] {
    lorads_gnn& g = chk(const_cast<lorads_gnn*>(gp));
    if (!theta || count != g.off.total) fail(LORADS_EINVAL, "parameter count mismatch");
    HIPCHK(hipMemcpyAsync(theta, g.theta.p, count * sizeof(float), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
  });
}

lorads_status lorads_gnn_load_graphs(lorads_gnn* gp, int32_t n_graphs, const int64_t* node_off,
                                     int64_t nnz, const int32_t* row, const int32_t* col,
                                     const float* w) {
  return gguard([&] {
    lorads_gnn& g = chk(gp);
    if (n_graphs < 1 || !node_off) fail(LORADS_EINVAL, "need at least one graph");
    if (nnz < 0 || (nnz > 0 && (!row || !col || !w))) fail(LORADS_EINVAL, "null edge arrays");
    if (node_off[0] != 0) fail(LORADS_EINVAL, "node_off[0] must be 0");
    for (int q = 0; q < n_graphs; ++q)
      if (node_off[q + 1] <= node_off[q]) fail(LORADS_EINVAL, "every graph needs at least one node");
    const int64_t N = node_off[n_graphs];
    if (N > INT32_MAX) fail(LORADS_EINVAL, "too many nodes");
    std::vector<int> gid(N);
    for (int q = 0; q < n_graphs; ++q)
      for (int64_t j = node_off[q]; j < node_off[q + 1]; ++j) gid[j] = q;
    // rows by counting sort, each row sorted by column
    std::vector<int64_t> rp(N + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) {
      const int a = row[e], b = col[e];
      if (a < 0 || a >= N || b < 0 || b >= N) fail(LORADS_EINVAL, "edge endpoint out of range");
      if (a == b) fail(LORADS_EINVAL, "self loop");
      if (gid[a] != gid[b]) fail(LORADS_EINVAL, "edge joins two graphs");
      if (!std::isfinite(w[e])) fail(LORADS_EINVAL, "non-finite edge weight");
      ++rp[a + 1];
    }
    for (int64_t j = 0; j < N; ++j) rp[j + 1] += rp[j];
    std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
    std::vector<std::pair<int, float>> adj(nnz);
    for (int64_t e = 0; e < nnz; ++e) adj[fill[row[e]]++] = {col[e], w[e]};
    for (int64_t j = 0; j < N; ++j) {
      std::sort(adj.begin() + rp[j], adj.begin() + rp[j + 1],
                [](const auto& p, const auto& q) { return p.first < q.first; });
      for (int64_t e = rp[j] + 1; e < rp[j + 1]; ++e)
        if (adj[e].first == adj[e - 1].first) fail(LORADS_EINVAL, "duplicate edge");
    }
    // symmetry: (j, k, w) needs (k, j, w)
    for (int64_t j = 0; j < N; ++j)
      for (int64_t e = rp[j]; e < rp[j + 1]; ++e) {
        const int k = adj[e].first;
        auto lo = adj.begin() + rp[k], hi = adj.begin() + rp[k + 1];
        auto it = std::lower_bound(lo, hi, (int)j,
                                   [](const auto& p, int v) { return p.first < v; });
        if (it == hi || it->first != (int)j || it->second != adj[e].second)
          fail(LORADS_EINVAL, "adjacency is not symmetric");
      }
    std::vector<int> hc(nnz);
    std::vector<float> hw(nnz);
    for (int64_t e = 0; e < nnz; ++e) { hc[e] = adj[e].first; hw[e] = adj[e].second; }
    hipStream_t s = g.stream;
    g.G = n_graphs;
    g.N = N;
    g.E = nnz;
    g.h_node_off.assign(node_off, node_off + n_graphs + 1);
    g.node_off.upload(g.h_node_off, s);
    g.rptr.upload(rp, s);
    g.gid.upload(gid, s);
    g.col.upload(hc, s);
    g.w.upload(hw, s);
    g.an.alloc(std::max<int64_t>(nnz, 1));
    g.inv_rs.alloc(N);
    g.x.alloc((size_t)N * kF);
    g.H.alloc((size_t)(g.layers + 1) * N * kH);
    g.M.alloc((size_t)g.layers * N * kH);
    g.dH.alloc((size_t)N * kH);
    g.dHs.alloc((size_t)N * kH);
    g.dMs.alloc((size_t)N * kH);
    g.yhat.alloc(N); g.dy.alloc(N);
    g.pool.alloc((size_t)n_graphs * kH);
    g.rhat.alloc(n_graphs); g.dr.alloc(n_graphs);
    g.er2.alloc(n_graphs);
    g.have_targets = false;
    g.have_grad = false;
    features_kernel<<<blocks_for(N, 256), 256, 0, s>>>(N, g.rptr.p, g.w.p, g.gid.p, g.node_off.p,
                                                       g.x.p, g.inv_rs.p, g.an.p);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  });
}

lorads_status lorads_gnn_set_targets(lorads_gnn* gp, const float* y, const float* r) {
  return gguard([&] {
    lorads_gnn& g = chk(gp);
    if (g.G == 0) fail(LORADS_ESTATE, "no graph set loaded");
    if (!y || !r) fail(LORADS_EINVAL, "null targets");
    for (int64_t j = 0; j < g.N; ++j)
      if (!std::isfinite(y[j])) fail(LORADS_EINVAL, "non-finite node target");
    for (int q = 0; q < g.G; ++q)
      if (!std::isfinite(r[q])) fail(LORADS_EINVAL, "non-finite graph target");
    g.y.upload(y, g.N, g.stream);
    g.r.upload(r, g.G, g.stream);
    HIPCHK(hipStreamSynchronize(g.stream));
    g.have_targets = true;
  });
}

lorads_status lorads_gnn_forward(lorads_gnn* gp, int32_t g0, int32_t g1, float* yhat, float* rhat) {
  return gguard([&] {
    lorads_gnn& g = chk(gp);
    check_range(g, g0, g1);
    forward(g, g0, g1, false, 0.0f);
    const int64_t n0 = g.h_node_off[g0], n1 = g.h_node_off[g1];
    if (yhat)
      HIPCHK(hipMemcpyAsync(yhat, g.yhat.p + n0, (n1 - n0) * sizeof(float), hipMemcpyDeviceToHost, g.stream));
    if (rhat)
      HIPCHK(hipMemcpyAsync(rhat, g.rhat.p + g0, (g1 - g0) * sizeof(float), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
  });
}

lorads_status lorads_gnn_loss_grad(lorads_gnn* gp, int32_t g0, int32_t g1, float omega,
                                   double* loss, float* grad, int64_t count) {
  return gguard([&] {
    lorads_gnn& g = chk(gp);
    check_range(g, g0, g1);
    if (!g.have_targets) fail(LORADS_ESTATE, "no targets set");
    if (!std::isfinite(omega) || omega < 0) fail(LORADS_EINVAL, "omega must be finite and >= 0");
    if (grad && count != g.off.total) fail(LORADS_EINVAL, "parameter count mismatch");
    forward(g, g0, g1, true, omega);
    backward(g, g0, g1);
    if (loss) HIPCHK(hipMemcpyAsync(loss, g.loss.p, sizeof(double), hipMemcpyDeviceToHost, g.stream));
    if (grad)
      HIPCHK(hipMemcpyAsync(grad, g.grad.p, count * sizeof(float), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    g.have_grad = true;
  });
}

lorads_status lorads_gnn_adam_step(lorads_gnn* gp, float lr, float beta1, float beta2, float eps) {
  return gguard([&] {
    lorads_gnn& g = chk(gp);
    if (!g.have_grad) fail(LORADS_ESTATE, "no gradient yet");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
      fail(LORADS_EINVAL, "invalid Adam hyper-parameters");
    ++g.adam_t;
    const float bc1 = 1.0f - std::pow(beta1, (float)g.adam_t);
    const float bc2 = 1.0f - std::pow(beta2, (float)g.adam_t);
    const int64_t P = g.off.total;
    adam_kernel<<<blocks_for(P, 256), 256, 0, g.stream>>>(P, g.theta.p, g.grad.p, g.m1.p, g.m2.p,
                                                         lr, beta1, beta2, eps, bc1, bc2);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(g.stream));
  });
}

lorads_status lorads_gnn_layer_time(lorads_gnn* gp, double* ms, int64_t* launches, double* flops) {
  return gguard([&] {
    lorads_gnn& g = chk(gp);
    resolve_timing(g);
    if (ms) *ms = g.t_ms;
    if (launches) *launches = g.launches;
    if (flops) *flops = g.flops;
    g.t_ms = 0;
    g.launches = 0;
    g.flops = 0;
  });
}

void lorads_gnn_destroy(lorads_gnn* g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  delete g;
}

}  // extern "C"
