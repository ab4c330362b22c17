// Shared definitions of the gfx950 LoRADS library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/lorads.h"

namespace lorads {

// ---------------------------------------------------------------------------
// error handling: every HIP call in host code goes through HIPCHK, which turns a
// failure into a thrown DeviceError caught at the C ABI boundary.
// ---------------------------------------------------------------------------
struct Error {
  lorads_status status;
  std::string msg;
};

[[noreturn]] void fail(lorads_status s, const std::string& msg);

// message returned by lorads_last_error(NULL) (calls without a context)
void set_global_error(const std::string& msg);

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      ::lorads::fail(e_ == hipErrorOutOfMemory ? LORADS_ENOMEM : LORADS_EDEVICE,  \
                     std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

// device buffer owned by the library
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count == 0) return;
    HIPCHK(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
  void upload(const T* h, size_t count, hipStream_t s = nullptr) {
    alloc(count);
    if (count) HIPCHK(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void upload(const std::vector<T>& v, hipStream_t s = nullptr) { upload(v.data(), v.size(), s); }
  void zero(hipStream_t s = nullptr) {
    if (n) HIPCHK(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
};

// scalar slots of the device-resident solver state (FP64 array `sc`)
enum Slot : int {
  S_RR0 = 0,   // CG: ||R0||^2
  S_RR = 1,    // CG: ||R||^2, two parity slots (1, 2)
  S_DONE = 3,  // CG: converged flag, two parity slots (3, 4)
  S_ALPHA = 5,
  S_BETA = 6,
  S_BRK = 7,    // CG breakdown (pq <= 0)
  S_ITERS = 8,  // CG iterations completed
  S_TOL2 = 9,   // CG tol^2
  S_GAMMA = 10,
  S_RHO = 11,
  S_PQ = 12,
  S_GEN = 16,  // 16..63 general-purpose reduction outputs
  S_PAIRS = 64,  // 64..80: <S, Y> of each L-BFGS pair buffer (memory <= 16, plus one)
  S_QUAD = 84,   // 84..87: the quartic's Gram terms of the quadratic objective
  S_COUNT = 96
};

constexpr int kBlock = 256;        // threads per block of the row / element kernels
constexpr int kRedBlocks = 512;    // grid of the fixed-grid reductions
constexpr int kMaxPart = 8192;     // capacity of a partial-sum buffer
// L-BFGS passes: two alternating regions of three partial arrays, the line
// search's nine arrays, then the descent check's array above them
constexpr int kLbfgsPartStride = 2048;
static_assert(3 * kRedBlocks <= kLbfgsPartStride, "L-BFGS partial region too small");
static_assert(9 * kRedBlocks <= 3 * kLbfgsPartStride, "line-search partials reach the descent-check array");
static_assert(4 * kLbfgsPartStride <= kMaxPart, "partial-sum buffer too small");
constexpr int kPairChunk = 32;     // PAIR forward map: constraints per work item
// XCDs of the part: consecutive workgroups of a launch are dealt to them in
// turn, so workgroup b runs on XCD b mod kXcds (each with its own L2)
constexpr int kXcds = 8;
constexpr int kR1Seg = 64;
constexpr int kDenseCMinN = 256;  // smallest order for which a dense C is stored dense         // RANK1: entries of a_i per segment (one lane group)

inline int pow2_group(int r) {
  int g = 1;
  while (g < r && g < 64) g <<= 1;
  return g;
}

// lanes per factor row of the row kernels: a lane holds up to
// LORADS_COLS_PER_LANE columns of a row in registers (c = lane + t G), so a
// wave covers 64 / G rows at once.  One column per lane keeps every gathered
// row inside a single load instruction.
#ifndef LORADS_COLS_PER_LANE
#define LORADS_COLS_PER_LANE 1
#endif
inline int lane_group(int r) {
  return pow2_group((r + LORADS_COLS_PER_LANE - 1) / LORADS_COLS_PER_LANE);
}

}  // namespace lorads
