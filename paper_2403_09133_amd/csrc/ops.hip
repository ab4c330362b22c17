// Operator dispatch (generic / DIAG / PAIR layouts) and the device-resident CG.
#include <hip/hip_ext.h>

#include <atomic>
#include <chrono>

#include "kernels.hpp"
#include "kernels_dense.hpp"
#include "kernels_quad.hpp"
#include "kernels_rank1.hpp"
#include "kernels_struct.hpp"
#include "problem.hpp"

namespace lorads {

#define LORADS_DISPATCH_G(Gval, CALL)                   \
  switch (Gval) {                                       \
    case 1: { constexpr int G = 1; CALL; } break;       \
    case 2: { constexpr int G = 2; CALL; } break;       \
    case 4: { constexpr int G = 4; CALL; } break;       \
    case 8: { constexpr int G = 8; CALL; } break;       \
    case 16: { constexpr int G = 16; CALL; } break;     \
    case 32: { constexpr int G = 32; CALL; } break;     \
    default: { constexpr int G = 64; CALL; } break;     \
  }

template <typename T> static const T* kv(const Problem& P);
template <> const double* kv<double>(const Problem& P) { return P.kval.p; }
template <> const float* kv<float>(const Problem& P) { return P.kvalf.p; }
template <typename T> static const T* av(const Problem& P);
template <> const double* av<double>(const Problem& P) { return P.aval.p; }
template <> const float* av<float>(const Problem& P) { return P.avalf.p; }
template <typename T> static const T* cv(const Problem& P);
template <> const double* cv<double>(const Problem& P) { return P.cval.p; }
template <> const float* cv<float>(const Problem& P) { return P.cvalf.p; }
template <typename T> static const T* dc(const Problem& P);
template <> const double* dc<double>(const Problem& P) { return P.dcoef.p; }
template <> const float* dc<float>(const Problem& P) { return P.dcoeff.p; }
template <typename T> static const T* ds(const Problem& P);
template <> const double* ds<double>(const Problem& P) { return P.dsq.p; }
template <> const float* ds<float>(const Problem& P) { return P.dsqf.p; }
template <typename T> static const T* pc(const Problem& P);
template <> const double* pc<double>(const Problem& P) { return P.pcoef.p; }
template <> const float* pc<float>(const Problem& P) { return P.pcoeff.p; }
template <typename T> static const T* r1v(const Problem& P);
template <> const double* r1v<double>(const Problem& P) { return P.r1val.p; }
template <> const float* r1v<float>(const Problem& P) { return P.r1valf.p; }
template <typename T> static const T* r1t(const Problem& P);
template <> const double* r1t<double>(const Problem& P) { return P.r1tval.p; }
template <> const float* r1t<float>(const Problem& P) { return P.r1tvalf.p; }

// RANK1 work vectors at rank r (segment partials of two factors, per-constraint
// r-vectors and weights), in the operator's accumulation type
template <typename T>
struct R1Work {
  using A = typename OpAcc<T>::type;
  A *su, *sv, *S, *coef;
};
template <typename T>
static R1Work<T> r1_work(Problem& P, int r) {
  using A = typename OpAcc<T>::type;
  const size_t nseg = (size_t)P.r1nseg, m = (size_t)P.m;
  const size_t need = (2 * nseg * r + m * r + m) * sizeof(double);
  if (P.r1work_bytes < need) {
    P.r1work.alloc(need);
    P.r1work_bytes = need;
  }
  A* base = reinterpret_cast<A*>(P.r1work.p);
  return R1Work<T>{base, base + nseg * r, base + 2 * nseg * r, base + 2 * nseg * r + m * r};
}

// G as above, plus KC = the factor columns a lane holds: 1 when r <= G
#define LORADS_DISPATCH_GK(G, r, CALL)                          \
  do {                                                           \
    if ((r) <= (G)) {                                            \
      constexpr int KC = 1;                                      \
      LORADS_DISPATCH_G(G, CALL);                                \
    } else {                                                     \
      constexpr int KC = kMaxCols;                               \
      LORADS_DISPATCH_G(G, CALL);                                \
    }                                                            \
  } while (0)

// the PAIR kernels index factor rows with 32-bit offsets
static void check_pair_offsets(const Problem& P, int ld) {
  if ((long long)P.n * ld >= (1LL << 31)) fail(LORADS_EINVAL, "n * ld exceeds the 32-bit offset range");
}

// one wave (64 lanes) per row, 4 rows per block
static int waves_grid(int rows) { return std::max(1, (rows + kBlock / 64 - 1) / (kBlock / 64)); }

static int rows_grid(int rows, int G) {
  const long long threads = (long long)rows * G;
  return (int)std::max<long long>(1, (threads + kBlock - 1) / kBlock);
}

// The two-columns-per-lane FP64 forms (k1_pair_v2, kpair_grad_v2) serve
// factors with 16-byte aligned rows of at least G entries: every lane loads
// its two columns unguarded, so all G columns a group covers must lie inside
// the row (ld >= G), or the last row's loads would run past the buffer.  Their
// results equal the one-column form's bit for bit.
static bool pair_v2_ok(const Problem& P, const void* U, const void* V, int r, int ld) {
  const int G = lane_group(r);
  return P.structure == LORADS_STRUCT_PAIR && G >= 2 && G <= 32 && r <= G && ld >= G &&
         ld % 2 == 0 && (reinterpret_cast<uintptr_t>(U) % 16) == 0 &&
         (reinterpret_cast<uintptr_t>(V) % 16) == 0;
}

// GV lanes per constraint (pair_v2_lanes) and the third-column form X3 for
// ranks 17 .. 24 (G = lane_group(r) = 32 there, so ld >= 32 >= 3 GV)
#define LORADS_DISPATCH_V2(G, r, CALL)                                   \
  do {                                                                   \
    switch (G) {                                                         \
      case 2: { constexpr int GV = 1, X3 = 0; CALL; } break;             \
      case 4: { constexpr int GV = 2, X3 = 0; CALL; } break;             \
      case 8: { constexpr int GV = 4, X3 = 0; CALL; } break;             \
      case 16: { constexpr int GV = 8, X3 = 0; CALL; } break;            \
      default:                                                           \
        if ((r) <= 24) { constexpr int GV = 8, X3 = 1; CALL; }           \
        else { constexpr int GV = 16, X3 = 0; CALL; }                    \
        break;                                                           \
    }                                                                    \
  } while (0)

// groups of at least 4 lanes (the fused line search stages per group)
#define LORADS_DISPATCH_LS(G, r, CALL)                                   \
  do {                                                                   \
    switch (G) {                                                         \
      case 8: { constexpr int GV = 4, X3 = 0; CALL; } break;             \
      case 16: { constexpr int GV = 8, X3 = 0; CALL; } break;            \
      default:                                                           \
        if ((r) <= 24) { constexpr int GV = 8, X3 = 1; CALL; }           \
        else { constexpr int GV = 16, X3 = 0; CALL; }                    \
        break;                                                           \
    }                                                                    \
  } while (0)

// ---------------------------------------------------------------------------
// FP32 forward maps with four columns per lane (k1_pair_f4): PAIR structure
// with the XCD chunk lists, rows of a multiple of 4 floats holding the whole
// lane group (ld >= 4 G), 16-byte aligned factors; G lanes, or 0 when the
// layout does not allow the form
static int pair_f4_lanes(const Problem& P, const void* U, const void* V, int r, int ld) {
  if (P.structure != LORADS_STRUCT_PAIR || P.nxchunks == 0 || r < 1 || r > 128) return 0;
  const int g = std::max(4, pow2_group((r + 3) / 4));
  if (g > 32 || ld % 4 != 0 || ld < 4 * g) return 0;
  if ((reinterpret_cast<uintptr_t>(U) % 16) != 0 || (reinterpret_cast<uintptr_t>(V) % 16) != 0) return 0;
  return g;
}

#define LORADS_DISPATCH_F32(Gv, CALL)                  \
  do {                                                 \
    switch (Gv) {                                      \
      case 4: { constexpr int GF = 4; CALL; } break;   \
      case 8: { constexpr int GF = 8; CALL; } break;   \
      case 16: { constexpr int GF = 16; CALL; } break; \
      default: { constexpr int GF = 32; CALL; } break; \
    }                                                  \
  } while (0)

template <typename T>
static void op_forward_impl(Problem& P, const T* U, const T* V, int r, int ld, T* z, double scale,
                            hipStream_t s) {
  const int G = lane_group(r);
  if (P.structure == LORADS_STRUCT_RANK1) {
    const R1Work<T> wk = r1_work<T>(P, r);
    LORADS_DISPATCH_G(G, (r1_seg<T, G, 1><<<rows_grid(P.r1nseg, G), kBlock, 0, s>>>(
                             P.r1nseg, P.r1sstart.p, P.r1idx.p, r1v<T>(P), U, V, r, ld, wk.su,
                             wk.sv, nullptr, 0)));
    LORADS_DISPATCH_G(G, (r1_con<T, G, 0><<<rows_grid(P.m, G), kBlock, 0, s>>>(
                             P.m, P.r1cseg.p, P.r1c.p, wk.su, wk.sv, r, z, scale, nullptr, nullptr,
                             0.0, nullptr, nullptr, nullptr, nullptr, nullptr, 0)));
  } else if (P.structure == LORADS_STRUCT_DIAG) {
    LORADS_DISPATCH_G(G, (k1_diag<T, G, 0><<<rows_grid(P.m, G), kBlock, 0, s>>>(
                             P.m, P.drow.p, dc<T>(P), U, V, r, ld, z, scale, nullptr, nullptr,
                             0.0, nullptr, nullptr, 0)));
  } else if (P.structure == LORADS_STRUCT_PAIR && std::is_same<T, double>::value &&
             pair_v2_ok(P, U, V, r, ld)) {
    check_pair_offsets(P, ld);
    LORADS_DISPATCH_V2(G, r, (k1_pair_v2<GV, 0, X3><<<xchunk_grid(P, GV), kBlock, 0, s>>>(
                              P.xchunk_off.p, P.xchunk_row.p, P.xchunk_start.p, P.xchunk_end.p, P.pk.p,
                              P.pcoef.p, P.pair_coef, (const double*)U, (const double*)V, r, ld,
                              (double*)z, scale, nullptr, nullptr, 0.0, nullptr)));
  } else if (P.structure == LORADS_STRUCT_PAIR && std::is_same<T, float>::value &&
             pair_f4_lanes(P, U, V, r, ld) > 0) {
    check_pair_offsets(P, ld);
    LORADS_DISPATCH_F32(pair_f4_lanes(P, U, V, r, ld), (k1_pair_f4<GF><<<xchunk_grid(P, GF), kBlock, 0, s>>>(
                             P.xchunk_off.p, P.xchunk_row.p, P.xchunk_start.p, P.xchunk_end.p, P.pk.p,
                             (const float*)pc<T>(P), P.pair_coef, (const float*)U, (const float*)V,
                             r, ld, (float*)z, scale)));
  } else if (P.structure == LORADS_STRUCT_PAIR) {
    check_pair_offsets(P, ld);
    LORADS_DISPATCH_GK(G, r, (k1_pair<T, G, 0, KC><<<rows_grid(P.nfchunks, G), kBlock, 0, s>>>(
                             P.nfchunks, P.fchunk_row.p, P.fchunk_start.p, P.rptr.p, P.pk.p,
                             pc<T>(P), P.pair_coef, U, V, r, ld, z, scale,
                             nullptr, nullptr, 0.0, nullptr, nullptr, 0)));
  } else {
    LORADS_DISPATCH_G(G, (k1_generic<T, G, 0><<<rows_grid(P.m, G), kBlock, 0, s>>>(
                             P.m, P.kptr.p, P.krow.p, P.kcol.p, kv<T>(P), U, V, r, ld, z, scale,
                             nullptr, nullptr, 0.0, nullptr, nullptr, 0)));
  }
  HIPCHK(hipGetLastError());
}

template <typename T>
void op_forward(Problem& P, const T* U, const T* V, int r, int ld, T* z, double scale,
                hipStream_t s) {
  P.prof.run(1, bytes_forward(P, r, sizeof(T)), s,
             [&] { op_forward_impl<T>(P, U, V, r, ld, z, scale, s); });
}

static void op_forward_w_impl(Problem& P, const double* U, const double* V, int r, int ld,
                              double* z, double* w, const double* lam, double rho, hipStream_t s);

void op_forward_w(Problem& P, const double* U, const double* V, int r, int ld, double* z,
                  double* w, const double* lam, double rho, hipStream_t s) {
  // the extra w output is an m-vector write beyond the plain forward map
  P.prof.run(1, bytes_forward(P, r, 8) + 16.0 * P.m, s,
             [&] { op_forward_w_impl(P, U, V, r, ld, z, w, lam, rho, s); });
}

static void op_forward_w_impl(Problem& P, const double* U, const double* V, int r, int ld,
                              double* z, double* w, const double* lam, double rho, hipStream_t s) {
  const int G = lane_group(r);
  if (P.structure == LORADS_STRUCT_RANK1) {
    const R1Work<double> wk = r1_work<double>(P, r);
    LORADS_DISPATCH_G(G, (r1_seg<double, G, 1><<<rows_grid(P.r1nseg, G), kBlock, 0, s>>>(
                             P.r1nseg, P.r1sstart.p, P.r1idx.p, P.r1val.p, U, V, r, ld, wk.su,
                             wk.sv, nullptr, 0)));
    LORADS_DISPATCH_G(G, (r1_con<double, G, 1><<<rows_grid(P.m, G), kBlock, 0, s>>>(
                             P.m, P.r1cseg.p, P.r1c.p, wk.su, wk.sv, r, z, 1.0, lam, P.b.p, rho, w,
                             nullptr, nullptr, nullptr, nullptr, 0)));
  } else if (P.structure == LORADS_STRUCT_DIAG) {
    LORADS_DISPATCH_G(G, (k1_diag<double, G, 1><<<rows_grid(P.m, G), kBlock, 0, s>>>(
                             P.m, P.drow.p, P.dcoef.p, U, V, r, ld, z, 1.0, lam, P.b.p, rho, w,
                             nullptr, 0)));
  } else if (pair_v2_ok(P, U, V, r, ld)) {
    check_pair_offsets(P, ld);
    LORADS_DISPATCH_V2(G, r, (k1_pair_v2<GV, 1, X3><<<xchunk_grid(P, GV), kBlock, 0, s>>>(
                              P.xchunk_off.p, P.xchunk_row.p, P.xchunk_start.p, P.xchunk_end.p, P.pk.p,
                              P.pcoef.p, P.pair_coef, U, V, r, ld, z, 1.0, lam, P.b.p, rho, w)));
  } else if (P.structure == LORADS_STRUCT_PAIR) {
    check_pair_offsets(P, ld);
    LORADS_DISPATCH_GK(G, r, (k1_pair<double, G, 1, KC><<<rows_grid(P.nfchunks, G), kBlock, 0, s>>>(
                             P.nfchunks, P.fchunk_row.p, P.fchunk_start.p, P.rptr.p, P.pk.p,
                             P.pcoef.p, P.pair_coef, U, V, r, ld, z, 1.0,
                             lam, P.b.p, rho, w, nullptr, 0)));
  } else {
    LORADS_DISPATCH_G(G, (k1_generic<double, G, 1><<<rows_grid(P.m, G), kBlock, 0, s>>>(
                             P.m, P.kptr.p, P.krow.p, P.kcol.p, P.kval.p, U, V, r, ld, z, 1.0,
                             lam, P.b.p, rho, w, nullptr, 0)));
  }
  HIPCHK(hipGetLastError());
}

// p1 = A(U D^T + D U^T), p2 = A(D D^T) (FP64): one pass for PAIR, two forward maps otherwise
void op_forward_pair(Problem& P, const double* U, const double* D, int r, int ld, double* p1,
                     double* p2, hipStream_t s) {
  if (P.structure != LORADS_STRUCT_PAIR) {
    op_forward<double>(P, U, D, r, ld, p1, 2.0, s);
    op_forward<double>(P, D, D, r, ld, p2, 1.0, s);
    return;
  }
  P.prof.run(3, bytes_forward(P, r, 8) + 8.0 * P.m, s, [&] {
    check_pair_offsets(P, ld);
    const int G = lane_group(r);
    if (pair_v2_ok(P, U, D, r, ld)) {
      LORADS_DISPATCH_V2(G, r, (k1_pair_v2<GV, 3, X3><<<xchunk_grid(P, GV), kBlock, 0, s>>>(
                                P.xchunk_off.p, P.xchunk_row.p, P.xchunk_start.p, P.xchunk_end.p,
                                P.pk.p, P.pcoef.p, P.pair_coef, U, D, r, ld, p1, 1.0, nullptr, nullptr,
                                0.0, p2)));
    } else {
      LORADS_DISPATCH_GK(G, r, (k1_pair<double, G, 3, KC><<<rows_grid(P.nfchunks, G), kBlock, 0, s>>>(
                               P.nfchunks, P.fchunk_row.p, P.fchunk_start.p, P.rptr.p, P.pk.p,
                               P.pcoef.p, P.pair_coef, U, D, r, ld, p1, 1.0, nullptr, nullptr, 0.0,
                               p2, nullptr, 0)));
    }
    HIPCHK(hipGetLastError());
  });
}

// The fused line-search pass (PAIR, FP64 two-column layout): the seven sums
// of the quartic as block partials in part (7 * ls_blocks doubles), nothing
// m-sized written.  Returns false (nothing launched) where the layout does not
// allow it; the caller then runs op_forward_pair and the m-vector sums.
bool op_linesearch_pair(Problem& P, const double* U, const double* D, int r, int ld,
                        const double* z, const double* lam, double* part, hipStream_t s) {
  const int G = lane_group(r);
  if (!pair_v2_ok(P, U, D, r, ld) || G < 8) return false;
  if (xchunk_grid(P, pair_v2_lanes(r)) != ls_blocks(P, r)) fail(LORADS_EINVAL, "line-search grid mismatch");
  check_pair_offsets(P, ld);
  P.prof.run(3, bytes_linesearch_pair(P, r), s, [&] {
    LORADS_DISPATCH_LS(G, r, (k1_pair_ls<GV, X3><<<ls_blocks(P, r), kBlock, 0, s>>>(
                              P.xchunk_off.p, P.xchunk_row.p, P.xchunk_start.p, P.xchunk_end.p,
                              P.pk.p, P.pcoef.p, P.pair_coef, U, D, r, ld, z, P.b.p, lam, part)));
    HIPCHK(hipGetLastError());
  });
  return true;
}

template <typename T>
static void op_adjoint_impl(Problem& P, const T* w, double c_scale, const T* V, int r, int ld,
                            T* out, int ldo, double out_scale, hipStream_t s);

template <typename T>
void op_adjoint(Problem& P, const T* w, double c_scale, const T* V, int r, int ld, T* out,
                int ldo, double out_scale, hipStream_t s) {
  // products with the cost matrix alone (w == null) are not timed: the class
  // covers the adjoint with multiplier weights
  if (w == nullptr) {
    op_adjoint_impl<T>(P, w, c_scale, V, r, ld, out, ldo, out_scale, s);
    return;
  }
  P.prof.run(2, bytes_adjoint(P, r, sizeof(T), c_scale != 0.0), s,
             [&] { op_adjoint_impl<T>(P, w, c_scale, V, r, ld, out, ldo, out_scale, s); });
}

template <typename T>
static void op_adjoint_impl(Problem& P, const T* w, double c_scale, const T* V, int r, int ld,
                            T* out, int ldo, double out_scale, hipStream_t s) {
  const int G = lane_group(r);
  if (r > 4 * G) fail(LORADS_EINVAL, "rank above 256 is not supported");
  if (P.cdense.n && c_scale != 0.0 && r <= 16 * kDenseNT) {
    // dense C on the matrix cores: the A* part alone, then C V added to it
    if (w == nullptr) {
      cdense_apply<T>(P, V, r, ld, out, ldo, out_scale * c_scale, 0.0, s);
      return;
    }
    op_adjoint_impl<T>(P, w, 0.0, V, r, ld, out, ldo, out_scale, s);
    cdense_apply<T>(P, V, r, ld, out, ldo, out_scale * c_scale, 1.0, s);
    return;
  }
  if (P.structure == LORADS_STRUCT_RANK1) {
    // S_i = a_i^T V with weight c_i w_i, then the row pass (C alone without w)
    const R1Work<T> wk = r1_work<T>(P, r);
    if (w != nullptr) {
      LORADS_DISPATCH_G(G, (r1_seg<T, G, 0><<<rows_grid(P.r1nseg, G), kBlock, 0, s>>>(
                               P.r1nseg, P.r1sstart.p, P.r1idx.p, r1v<T>(P), V, V, r, ld, wk.su,
                               nullptr, nullptr, 0)));
      LORADS_DISPATCH_G(G, (r1_con<T, G, 2><<<rows_grid(P.m, G), kBlock, 0, s>>>(
                               P.m, P.r1cseg.p, P.r1c.p, wk.su, nullptr, r, nullptr, 1.0, nullptr,
                               nullptr, 0.0, nullptr, w, wk.S, wk.coef, nullptr, 0)));
    }
    LORADS_DISPATCH_G(G, (r1_rows<T, G, 0><<<rows_grid(P.n, G), kBlock, 0, s>>>(
                             P.n, P.cptr.p, P.ccol.p, cv<T>(P), c_scale, P.r1tptr.p, P.r1tcon.p,
                             r1t<T>(P), w != nullptr ? wk.coef : nullptr, wk.S, V, r, ld, out, ldo,
                             out_scale, nullptr, nullptr, 0, nullptr)));
  } else if (P.structure == LORADS_STRUCT_DIAG) {
    LORADS_DISPATCH_G(G, (k2_diag<T, G, 0><<<rows_grid(P.n, G), kBlock, 0, s>>>(
                             P.n, P.cptr.p, P.ccol.p, cv<T>(P), c_scale, P.dptr.p, dc<T>(P),
                             nullptr, w, V, r, ld, out, ldo, out_scale, nullptr, nullptr, 0,
                             nullptr)));
  } else if (P.structure == LORADS_STRUCT_PAIR && std::is_same<T, double>::value &&
             pair_v2_ok(P, V, V, r, ld) && ldo >= r) {
    check_pair_offsets(P, std::max(ld, ldo));
    const int grid = std::max(1, (P.n + kBlock / 32 - 1) / (kBlock / 32));  // two rows per wave
    LORADS_DISPATCH_V2(G, r, (kpair_adj_v2<GV, X3><<<grid, kBlock, 0, s>>>(
                              P.n, P.cptr.p, P.ccol.p, (const double*)cv<T>(P), c_scale,
                              P.inc_ptr.p, P.inc_nb.p, P.inc_id.p, (const double*)pc<T>(P),
                              P.pair_coef, (const double*)w, (const double*)V, r, ld,
                              (double*)out, ldo, out_scale)));
  } else if (P.structure == LORADS_STRUCT_PAIR && std::is_same<T, float>::value &&
             pair_f4_lanes(P, V, V, r, ld) > 0 && ldo >= r) {
    check_pair_offsets(P, std::max(ld, ldo));
    const int grid = std::max(1, (P.n + kBlock / 32 - 1) / (kBlock / 32));  // two rows per wave
    LORADS_DISPATCH_F32(pair_f4_lanes(P, V, V, r, ld), (kpair_adj_f4<GF><<<grid, kBlock, 0, s>>>(
                             P.n, P.cptr.p, P.ccol.p, (const float*)cv<T>(P), c_scale, P.inc_ptr.p,
                             P.inc_nb.p, P.inc_id.p, (const float*)pc<T>(P), P.pair_coef,
                             (const float*)w, (const float*)V, r, ld, (float*)out, ldo, out_scale)));
  } else if (P.structure == LORADS_STRUCT_PAIR) {
    check_pair_offsets(P, std::max(ld, ldo));
    LORADS_DISPATCH_GK(G, r, (kpair_rows<T, G, 0, KC><<<waves_grid(P.n), kBlock, 0, s>>>(
                             P.n, P.cptr.p, P.ccol.p, cv<T>(P), c_scale, P.inc_ptr.p, P.inc_nb.p,
                             P.inc_id.p, pc<T>(P), P.pair_coef, w, V, nullptr, r, ld, out, ldo,
                             out_scale, nullptr, 0, nullptr, nullptr, 0.0)));
  } else {
    LORADS_DISPATCH_G(G, (k2_generic<T, G, 0><<<rows_grid(P.n, G), kBlock, 0, s>>>(
                             P.n, P.cptr.p, P.ccol.p, cv<T>(P), c_scale, P.aptr.p, P.acol.p,
                             P.acon.p, av<T>(P), w, V, r, ld, out, ldo, out_scale, nullptr,
                             nullptr, 0, nullptr)));
  }
  HIPCHK(hipGetLastError());
}

bool grad_pair_ready(const Problem& P) {
  return P.structure == LORADS_STRUCT_PAIR && P.inc_lb.n > 0 && P.inc_lb_lam;
}

void refresh_inc_lam(Problem& P, hipStream_t s) {
  if (P.structure != LORADS_STRUCT_PAIR || P.inc_lb.n == 0) return;
  const int E = (int)(P.inc_lb.n / 2);
  gather_lam_lb<<<grid_for(E), kBlock, 0, s>>>(E, P.inc_id.p, P.lam.p, P.inc_lb.p);
  HIPCHK(hipGetLastError());
  P.inc_lb_lam = true;
}

void op_grad_pair(Problem& P, const double* U, int r, int ld, double rho, double* out, int ldo,
                  double out_scale, hipStream_t s, double* z) {
  if (!grad_pair_ready(P)) fail(LORADS_EINVAL, "gradient form needs per-entry lam and b");
  const bool v2 = pair_v2_ok(P, U, U, r, ld);
  if (z && !(v2 && P.inc_upper_view)) {
    op_forward<double>(P, U, U, r, ld, z, 1.0, s);
    z = nullptr;
  }
  // dense C: the kernels take the sparse part as empty and C U is added after
  const bool dense = P.cdense.n && r <= 16 * kDenseNT;
  const double cs = dense ? 0.0 : 1.0;
  P.prof.run(2, bytes_grad_pair(P, r), s, [&] {
    check_pair_offsets(P, std::max(ld, ldo));
    const int G = lane_group(r);
    if (r > 4 * G) fail(LORADS_EINVAL, "rank above 256 is not supported");
    if (v2) {
      const int grid = std::max(1, (P.n + kBlock / 32 - 1) / (kBlock / 32));  // two rows per wave
      LORADS_DISPATCH_V2(G, r, (kpair_grad_v2<GV, X3><<<grid, kBlock, 0, s>>>(
                                P.n, P.cptr.p, P.ccol.p, P.cval.p, cs, P.inc_ptr.p, P.inc_nb.p,
                                P.pair_coef, U, r, ld, out, ldo, out_scale, P.inc_lb.p, rho,
                                P.rptr.p, z)));
    } else {
      LORADS_DISPATCH_GK(G, r, (kpair_rows<double, G, 2, KC><<<waves_grid(P.n), kBlock, 0, s>>>(
                               P.n, P.cptr.p, P.ccol.p, P.cval.p, cs, P.inc_ptr.p, P.inc_nb.p,
                               P.inc_id.p, nullptr, P.pair_coef, nullptr, U, nullptr, r, ld, out, ldo,
                               out_scale, nullptr, 0, nullptr, P.inc_lb.p, rho)));
    }
    HIPCHK(hipGetLastError());
    if (dense) cdense_apply<double>(P, U, r, ld, out, ldo, out_scale, 1.0, s);
  });
}

#ifndef LORADS_DENSE_BLOCKS
#define LORADS_DENSE_BLOCKS 1024
#endif

template <typename T>
void cdense_apply(Problem& P, const T* V, int r, int ld, T* out, int ldo, double alpha, double beta,
                  hipStream_t s) {
  if (P.cdense.n == 0 || r < 1 || r > 16 * kDenseNT || ld < r || ldo < r)
    fail(LORADS_EINVAL, "dense C product: unsupported shape");
  const T* C = sizeof(T) == 8 ? (const T*)(const void*)P.cdense.p : (const T*)(const void*)P.cdensef.p;
  const int tiles = (P.n + 15) / 16;
  const int nt = (r + 15) / 16;
  // eight tiles per block at one column tile (the staged V block is small, so
  // two blocks of eight waves fit a CU), else four
  const int wpb = nt == 1 ? 8 : 4;
  const int groups = (tiles + wpb - 1) / wpb;
  const int kblocks = P.ldc / kDenseK;
  // about LORADS_DENSE_BLOCKS blocks: ranges of whole 64-column blocks
  const int want = std::max(1, std::min(kblocks, (LORADS_DENSE_BLOCKS + groups - 1) / groups));
  const int kchunk = (kblocks + want - 1) / want * kDenseK;
  const int splits = (P.ldc + kchunk - 1) / kchunk;
  const size_t need = (size_t)splits * P.n * r * sizeof(T);
  if (P.cdpart.n < need) P.cdpart.alloc(need);
  T* part = reinterpret_cast<T*>(P.cdpart.p);
  const int blocks = groups * splits;
  switch (nt) {
    case 1: cdense_partial<T, 1, 8><<<blocks, 512, 0, s>>>(P.n, P.ldc, C, V, r, ld, tiles, splits, kchunk, part); break;
    case 2: cdense_partial<T, 2, 4><<<blocks, 256, 0, s>>>(P.n, P.ldc, C, V, r, ld, tiles, splits, kchunk, part); break;
    case 3: cdense_partial<T, 3, 4><<<blocks, 256, 0, s>>>(P.n, P.ldc, C, V, r, ld, tiles, splits, kchunk, part); break;
    default: cdense_partial<T, 4, 4><<<blocks, 256, 0, s>>>(P.n, P.ldc, C, V, r, ld, tiles, splits, kchunk, part); break;
  }
  cdense_finish<T><<<grid_for((size_t)P.n * r), kBlock, 0, s>>>(P.n, r, splits, part, alpha, beta,
                                                                out, ldo);
  HIPCHK(hipGetLastError());
}
template void cdense_apply<double>(Problem&, const double*, int, int, double*, int, double, double,
                                   hipStream_t);
template void cdense_apply<float>(Problem&, const float*, int, int, float*, int, double, double,
                                  hipStream_t);

template <typename T>
void gram_small(Problem& P, int n, int ra, int rb, const T* X, int ldx, const T* Y, int ldy, double* G,
                hipStream_t s) {
  if (ra < 1 || rb < 1 || ra > 256 || rb > 256) fail(LORADS_EINVAL, "small Gram: bad shape");
  const int rr = ra * rb;
  // at most 2^21 partial entries (16 MB)
  const int nb = std::max(1, std::min(kGramBlocks, (1 << 21) / rr));
  const size_t need = (size_t)nb * rr;
  if (P.qpart.n < need) P.qpart.alloc(need);
  gram_rr_partial<T><<<nb, kBlock, 0, s>>>(n, ra, rb, X, ldx, Y, ldy, P.qpart.p);
  gram_rr_finish<<<std::max(1, (rr + kBlock - 1) / kBlock), kBlock, 0, s>>>(rr, nb, P.qpart.p, G);
  HIPCHK(hipGetLastError());
}
template void gram_small<double>(Problem&, int, int, int, const double*, int, const double*, int, double*,
                                 hipStream_t);
template void gram_small<float>(Problem&, int, int, int, const float*, int, const float*, int, double*,
                                hipStream_t);

int pair_f32_lanes(const Problem& P, int r, int ld) {
  if (P.structure != LORADS_STRUCT_PAIR || P.pcoef.n != 0 || P.nxchunks == 0 || r < 1 || r > 128)
    return 0;
  const int g = std::max(4, pow2_group((r + 3) / 4));
  return (ld % 4 == 0 && ld >= 4 * g && g <= 32) ? g : 0;
}



void op_linesearch_pair_f32(Problem& P, const float* U32, const float* D32, int r, int ld,
                            const double* z, const double* lam, double* part, hipStream_t s) {
  const int g = pair_f32_lanes(P, r, ld);
  if (g == 0 || (reinterpret_cast<uintptr_t>(U32) % 16) != 0 ||
      (reinterpret_cast<uintptr_t>(D32) % 16) != 0)
    fail(LORADS_EINVAL, "mixed line search: layout not supported");
  check_pair_offsets(P, ld);
  P.prof.run(3, bytes_linesearch_pair_f32(P, r), s, [&] {
    LORADS_DISPATCH_F32(g, (k1_pair_ls_f32<GF><<<xchunk_grid(P, GF), kBlock, 0, s>>>(
                               P.xchunk_off.p, P.xchunk_row.p, P.xchunk_start.p, P.xchunk_end.p,
                               P.pk.p, P.pair_coef, U32, D32, ld, z, P.b.p, lam, part)));
    HIPCHK(hipGetLastError());
  });
}

int cg_ld(const Problem& P, int r, int elem_bytes) {
  if (P.structure != LORADS_STRUCT_PAIR) return r;
  const int per_line = 64 / elem_bytes;  // 64-byte rows: a gathered row never straddles a line
  return (r + per_line - 1) / per_line * per_line;
}

template <typename T>
int op_cg(Problem& P, const T* W, int ldw, int r, int ld, const T* Pd, const T* P2, T* Q, T* t,
          int parity, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const int G = lane_group(r);
  if (r > 4 * G) fail(LORADS_EINVAL, "rank above 256 is not supported");
  double* sc = P.sc.p;
  int np = 0;  // block partials of <P, Q> written to P.part
  if (P.structure != LORADS_STRUCT_PAIR && (ld != r || ldw != r || P2))
    fail(LORADS_EINVAL, "CG buffers must be compact");
  // PAIR on the CG layout: one kernel with 16-byte column vectors per lane
  // (FP64 at ranks 17 .. 24: 8 lanes with an extra 8-byte vector each, 24
  // columns; in FP32 the 8-lane 32-column form measured faster than 4 lanes
  // with the extra vector, 327 against 483 us at m = 15.7M)
  constexpr int VW = 16 / (int)sizeof(T);
  const bool x3 = sizeof(T) == 8 && r > 16 && r <= 24 && ld >= 24;
  const int gv = x3 ? 16 / VW : pow2_group((r + VW - 1) / VW);
  const bool vec = P.structure == LORADS_STRUCT_PAIR && P2 && P2 == W + ld && ldw == 2 * ld &&
                   ld % VW == 0 && (x3 || (gv * VW <= ld && gv <= 16)) &&
                   (size_t)P.n * ldw * sizeof(T) < ((size_t)1 << 31);
  // factor arrays larger than one XCD's L2 (with the caller's partials): the
  // operator split by partner block, then the combining pass
  using Acc = typename OpAcc<T>::type;
  const bool xcd = vec && P.cg_xparts != nullptr && cg_xparts_bytes(P, ld, (int)sizeof(Acc)) > 0;
  // events: attached to that kernel's launch (its own start and end), else
  // recorded around the operator's launches
  const bool ext = ev0 != nullptr && vec && !xcd;
  if (ev0 && !ext) HIPCHK(hipEventRecord(ev0, s));
  if (P.structure == LORADS_STRUCT_RANK1) {
    // u_i = a_i^T P, S_i = a_i^T W, weight rho c_i^2 <u_i, S_i>; then
    // Q_t = gamma P_t + sum_i weight_i a_{i,t} S_i
    if (ld != r || ldw != r || P2) fail(LORADS_EINVAL, "CG buffers must be compact");
    const R1Work<T> wk = r1_work<T>(P, r);
    LORADS_DISPATCH_G(G, (r1_seg<T, G, 1><<<rows_grid(P.r1nseg, G), kBlock, 0, s>>>(
                             P.r1nseg, P.r1sstart.p, P.r1idx.p, r1v<T>(P), Pd, W, r, ld, wk.su,
                             wk.sv, sc, parity)));
    LORADS_DISPATCH_G(G, (r1_con<T, G, 3><<<rows_grid(P.m, G), kBlock, 0, s>>>(
                             P.m, P.r1cseg.p, P.r1c.p, wk.su, wk.sv, r, nullptr, 1.0, nullptr,
                             nullptr, 0.0, nullptr, nullptr, wk.S, wk.coef, sc, parity)));
    const int grid = rows_grid(P.n, G);
    P.ensure_part(grid);
    LORADS_DISPATCH_G(G, (r1_rows<T, G, 1><<<grid, kBlock, 0, s>>>(
                             P.n, nullptr, nullptr, nullptr, 0.0, P.r1tptr.p, P.r1tcon.p, r1t<T>(P),
                             wk.coef, wk.S, W, r, ld, Q, ld, 1.0, Pd, sc, parity, P.part.p)));
    np = grid;
  } else if (P.structure == LORADS_STRUCT_DIAG) {
    const int grid = rows_grid(P.n, G);
    P.ensure_part(grid);
    LORADS_DISPATCH_G(G, (k3_diag<T, G><<<grid, kBlock, 0, s>>>(
                             P.n, ds<T>(P), W, Pd, Q, r, sc, parity, P.part.p)));
    np = grid;
  } else if (P.structure == LORADS_STRUCT_PAIR) {
    // one wave per row over its incident constraints, G lanes per constraint.
    // With P2 the direction is read from its copy interleaved with W (row p:
    // [W_p | P_p], stride ldw = 2 ld), so one gathered line holds both rows.
    const T* Pg = P2 ? P2 : Pd;
    check_pair_offsets(P, ldw);
    const int grid = waves_grid(P.n);
    P.ensure_part(grid);
    if (xcd) {
      Acc* xp = static_cast<Acc*>(P.cg_xparts);
      const int xgrid = kXcds * ((P.n + kBlock / 64 - 1) / (kBlock / 64));
#define LORADS_CG_XVEC(GG, X)                                                                      \
  kpair_cg_xvec<T, GG, X><<<xgrid, kBlock, 0, s>>>(P.n, P.inc_xptr.p, P.inc_nb.p, P.inc_id.p,      \
                                                   pc<T>(P), P.pair_coef, W, ld, r, xp, sc, parity)
      if (x3) {
        if constexpr (sizeof(T) == 8) LORADS_CG_XVEC(8, 1);
      } else switch (gv) {
        case 1: LORADS_CG_XVEC(1, 0); break;
        case 2: LORADS_CG_XVEC(2, 0); break;
        case 4: LORADS_CG_XVEC(4, 0); break;
        case 8: LORADS_CG_XVEC(8, 0); break;
        default: LORADS_CG_XVEC(16, 0); break;
      }
#undef LORADS_CG_XVEC
      const int cgrid = grid_for((size_t)P.n * r, 1024);
      P.ensure_part(cgrid);
      xcg_combine<T><<<cgrid, kBlock, 0, s>>>(P.n, r, ld, xp, W, Q, sc, parity, P.part.p);
    } else if (vec) {
#define LORADS_CG_VEC(GG, X)                                                                       \
  do {                                                                                             \
    if (ext)                                                                                       \
      hipExtLaunchKernelGGL(kpair_cg_vec<T, GG, X>, dim3(grid), dim3(kBlock), 0, s, ev0, ev1, 0u,   \
                            P.n, P.inc_ptr.p, P.inc_nb.p, P.inc_id.p, pc<T>(P), P.pair_coef, W, ld, \
                            r, Q, sc, parity, P.part.p);                                           \
    else                                                                                           \
      kpair_cg_vec<T, GG, X><<<grid, kBlock, 0, s>>>(P.n, P.inc_ptr.p, P.inc_nb.p, P.inc_id.p,     \
                                                     pc<T>(P), P.pair_coef, W, ld, r, Q, sc,        \
                                                     parity, P.part.p);                             \
  } while (0)
      if (x3) {
        if constexpr (sizeof(T) == 8) LORADS_CG_VEC(8, 1);
      } else switch (gv) {
        case 1: LORADS_CG_VEC(1, 0); break;
        case 2: LORADS_CG_VEC(2, 0); break;
        case 4: LORADS_CG_VEC(4, 0); break;
        case 8: LORADS_CG_VEC(8, 0); break;
        default: LORADS_CG_VEC(16, 0); break;
      }
#undef LORADS_CG_VEC
    } else {
      LORADS_DISPATCH_GK(G, r, (kpair_rows<T, G, 1, KC><<<grid, kBlock, 0, s>>>(
                               P.n, nullptr, nullptr, nullptr, 0.0, P.inc_ptr.p, P.inc_nb.p,
                               P.inc_id.p, pc<T>(P), P.pair_coef, nullptr, W, Pg, r, ldw, Q, ld,
                               1.0, sc, parity, P.part.p, nullptr, 0.0)));
    }
    np = xcd ? grid_for((size_t)P.n * r, 1024) : grid;
  } else {
    LORADS_DISPATCH_G(G, (k1_generic<T, G, 2><<<rows_grid(P.m, G), kBlock, 0, s>>>(
                             P.m, P.kptr.p, P.krow.p, P.kcol.p, kv<T>(P), Pd, W, r, r, t, 1.0,
                             nullptr, nullptr, 0.0, nullptr, sc, parity)));
    const int grid = rows_grid(P.n, G);
    P.ensure_part(grid);
    LORADS_DISPATCH_G(G, (k2_generic<T, G, 1><<<grid, kBlock, 0, s>>>(
                             P.n, nullptr, nullptr, nullptr, 0.0, P.aptr.p, P.acol.p, P.acon.p,
                             av<T>(P), t, W, r, r, Q, r, 1.0, Pd, sc, parity, P.part.p)));
    np = grid;
  }
  HIPCHK(hipGetLastError());
  if (ev1 && !ext) HIPCHK(hipEventRecord(ev1, s));
  return np;
}

// ---------------------------------------------------------------------------
// algorithmic bytes (indices, coefficients, inputs and outputs once each)
// ---------------------------------------------------------------------------
double bytes_forward(const Problem& P, int r, int s) {
  const double nr = (double)P.n * r * s;
  if (P.structure == LORADS_STRUCT_DIAG) return (double)P.m * (4 + s) + 2.0 * nr + (double)P.m * s;
  if (P.structure == LORADS_STRUCT_PAIR)
    return (double)P.m * 8 + (double)P.m * s + 2.0 * nr + (P.pcoef.n ? (double)P.m * s : 0.0);
  if (P.structure == LORADS_STRUCT_RANK1)  // a's entries, segment bounds, c, both factors, z
    return (double)P.r1idx.n * (4 + s) + (double)(P.r1nseg + P.m + 1) * 4 + (double)P.m * 8 + 2.0 * nr +
           (double)P.m * s;
  return (double)P.a_nnz * (8 + s) + (double)(P.m + 1) * 4 + 2.0 * nr + (double)P.m * s;
}

double bytes_linesearch_pair(const Problem& P, int r) {
  return (double)P.m * 8 + 3.0 * P.m * 8 + 2.0 * P.n * r * 8 + (P.pcoef.n ? (double)P.m * 8 : 0.0);
}

double bytes_adjoint(const Problem& P, int r, int s, bool with_c) {
  const double nr = (double)P.n * r * s;
  const double cbytes = !with_c ? 0.0
                        : P.cdense.n ? (double)P.n * P.ldc * s
                                     : (double)P.cval.n * (4 + s) + (double)(P.n + 1) * 4;
  if (P.structure == LORADS_STRUCT_DIAG) return (double)P.m * (4 + 2 * s) + 2.0 * nr + cbytes;
  if (P.structure == LORADS_STRUCT_RANK1)  // a by constraint and by row, w, c, V, out
    return 2.0 * (double)P.r1idx.n * (4 + s) + (double)(P.r1nseg + P.m + P.n + 2) * 4 +
           (double)P.m * (8 + s) + 2.0 * nr + cbytes;
  if (P.structure == LORADS_STRUCT_PAIR)
    return (double)P.m * 8 + (double)P.m * s + 2.0 * nr + cbytes + (P.pcoef.n ? (double)P.m * s : 0.0);
  return (double)P.acol.n * (8 + s) + (double)(P.n + 1) * 4 + (double)P.m * s + 2.0 * nr + cbytes;
}

double bytes_cprod(const Problem& P, int r, int s) {
  if (P.cdense.n) return (double)P.n * P.ldc * s + 2.0 * (double)P.n * r * s;
  return (double)P.cval.n * (4 + s) + (double)(P.n + 1) * 4 + 2.0 * (double)P.n * r * s;
}

double bytes_grad_pair(const Problem& P, int r) {
  // the gradient form applies both maps: A(U U^T) entry by entry and the adjoint
  return bytes_forward(P, r, 8) + bytes_adjoint(P, r, 8, true);
}

// mixed-form line search: the factor reads at 4 bytes
double bytes_linesearch_pair_f32(const Problem& P, int r) {
  return (double)P.m * 8 + 3.0 * P.m * 8 + 2.0 * P.n * r * 4;
}

double bytes_cg_op(const Problem& P, int r, int s) {
  const double nr = (double)P.n * r * s;
  if (P.structure == LORADS_STRUCT_DIAG) return (double)P.n * s + 3.0 * nr;
  if (P.structure == LORADS_STRUCT_PAIR) return (double)P.m * 8 + 3.0 * nr + (P.pcoef.n ? (double)P.m * s : 0.0);
  return bytes_forward(P, r, s) + bytes_adjoint(P, r, s, false) + nr;
}

// ---------------------------------------------------------------------------
__global__ void set_slots_kernel(double* sc, int slot, double v0, double v1, double v2, double v3,
                                 int count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double v[4] = {v0, v1, v2, v3};
    for (int i = 0; i < count; ++i) sc[slot + i] = v[i];
  }
}

void set_slots(Problem& P, int slot, const double* vals, int count, hipStream_t s) {
  for (int i = 0; i < count; i += 4) {
    const int c = std::min(4, count - i);
    double v[4] = {0, 0, 0, 0};
    for (int t = 0; t < c; ++t) v[t] = vals[i + t];
    set_slots_kernel<<<1, 64, 0, s>>>(P.sc.p, slot + i, v[0], v[1], v[2], v[3], c);
  }
  HIPCHK(hipGetLastError());
}

#ifndef LORADS_HOST_PUBLISH
#define LORADS_HOST_PUBLISH 1
#endif
// Waits until the device has published sequence number seq (a kernel wrote
// the values to the pinned words, then seq after a system-scope fence) and
// copies count values out: the host spins on the number for a short while,
// then waits for the stream (which also reports a failed launch).
static void wait_published(Problem& P, long long seq, double* vals, int count, hipStream_t s) {
  volatile long long* flag = reinterpret_cast<volatile long long*>(P.hs.h);
  const auto t0 = std::chrono::steady_clock::now();
  bool seen = false;
  for (unsigned spin = 1; !(seen = (*flag == seq)); ++spin) {
    if ((spin & 1023) == 0 &&
        std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000))
      break;
  }
  if (!seen) {
    HIPCHK(hipStreamSynchronize(s));
    if (*flag != seq) fail(LORADS_EDEVICE, "device did not publish the solver scalars");
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  const volatile double* hv = P.hs.h + 1;
  for (int i = 0; i < count; ++i) vals[i] = hv[i];
  if (P.prof.on) {  // the stream has passed these timings: finished forward / adjoint
    P.prof.resolve(1);
    P.prof.resolve(2);
  }
}

void read_slots(Problem& P, int slot, double* vals, int count, hipStream_t s) {
  if (LORADS_HOST_PUBLISH && !P.hs.h) P.hs.init();  // first read of this problem
  if (LORADS_HOST_PUBLISH && count <= 64) {
    const long long seq = ++P.hs.seq;
    publish_slots<<<1, 64, 0, s>>>(P.sc.p + slot, count, P.hs.d, seq);
    HIPCHK(hipGetLastError());
    wait_published(P, seq, vals, count, s);
    return;
  }
  HIPCHK(hipMemcpyAsync(vals, P.sc.p + slot, count * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (P.prof.on) {  // the stream is idle: finished forward / adjoint timings
    P.prof.resolve(1);
    P.prof.resolve(2);
  }
}

template <typename TX, typename TY>
void dot_to_slot(Problem& P, size_t N, const TX* X, const TY* Y, double scale, int slot,
                 hipStream_t s) {
  const int grid = grid_for(N, kRedBlocks);
  dot_kernel<TX, TY><<<grid, kBlock, 0, s>>>(N, X, Y, P.part.p);
  finish_slots<<<1, kBlock, 0, s>>>(grid, 1, P.part.p, scale, P.sc.p, slot);
  HIPCHK(hipGetLastError());
}

void dot_rows_to_slot(Problem& P, int n, int r, int ld, const double* X, const double* Y,
                      double scale, int slot, hipStream_t s) {
  const size_t N = (size_t)n * r;
  if (ld == r || N >= ((size_t)1 << 32)) {
    if (ld != r) fail(LORADS_EINVAL, "padded factor too large for the row-strided dot");
    dot_to_slot<double, double>(P, N, X, Y, scale, slot, s);
    return;
  }
  const int grid = grid_for(N, kRedBlocks);
  dot_rows_kernel<<<grid, kBlock, 0, s>>>((unsigned)N, r, ld, X, Y, P.part.p);
  finish_slots<<<1, kBlock, 0, s>>>(grid, 1, P.part.p, scale, P.sc.p, slot);
  HIPCHK(hipGetLastError());
}

void dual_update_slot(Problem& P, const double* z, double rho, double* lam, int slot, hipStream_t s) {
  const int grid = grid_for(P.m, kRedBlocks);
  dual_update<<<grid, kBlock, 0, s>>>(P.m, z, P.b.p, rho, lam, P.part.p);
  finish_slots<<<1, kBlock, 0, s>>>(grid, 1, P.part.p, 1.0, P.sc.p, slot);
  HIPCHK(hipGetLastError());
}

void linesearch_slots(Problem& P, int n, int r, int ld, const double* CD, const double* U,
                      const double* D, const double* z, const double* p1, const double* p2,
                      const double* lam, int slot, hipStream_t s, const double* part_gd,
                      const double* cdiag, double* vals, int nread, const double* lsp, int nls) {
  const size_t N = (size_t)n * r;
  if (N >= ((size_t)1 << 32)) fail(LORADS_EINVAL, "factor too large for the line-search dots");
  const int rg = grid_for(N, kRedBlocks), gl = grid_for(P.m, kRedBlocks);
  P.ensure_part((size_t)2 * rg + (size_t)7 * gl);
  double* part_f = P.part.p;
  double* part_m = P.part.p + 2 * rg;
  linesearch_all<<<std::max(rg, gl), kBlock, 0, s>>>((unsigned)N, r, ld, CD, U, D, rg, part_f, P.m, z,
                                                     P.b.p, p1, p2, lam, gl, part_m, cdiag, lsp, nls);
  if (part_gd && part_gd < part_m + (size_t)7 * gl)
    fail(LORADS_EINVAL, "descent-check partials overlap the line-search partials");
  if (rg > 2 * kBlock || gl > 2 * kBlock) fail(LORADS_EINVAL, "line-search partials exceed the finishing layout");
  // with vals, the finishing launch also publishes slot .. slot + nread - 1
  // to the host and the call returns them (no separate read launch)
  if (vals && LORADS_HOST_PUBLISH && !P.hs.h) P.hs.init();
  const bool pub = vals && LORADS_HOST_PUBLISH && nread <= 64;
  const long long seq = pub ? ++P.hs.seq : 0;
  linesearch_finish<<<1, kBlock, 0, s>>>(rg, part_f, gl, part_m, part_gd, P.sc.p, slot,
                                         pub ? P.hs.d : nullptr, seq, nread);
  HIPCHK(hipGetLastError());
  if (pub) wait_published(P, seq, vals, nread, s);
  else if (vals) read_slots(P, slot, vals, nread, s);
}

// ---------------------------------------------------------------------------
// CG: solve M_W D = R from D = X (normally 0).  The loop runs in chunks of
// device-resident iterations; after each chunk one flag is read back.
// ---------------------------------------------------------------------------
template <typename T>
int cg_run(Problem& P, const T* W, int ldw, int r, int ld, double rho, double gamma, T* R, T* X,
           T* Pd, T* P2, T* Q, T* t, double tol, int maxit, hipStream_t s, double* relres,
           double* op_bytes, const double* quadG) {
  const size_t N = (size_t)P.n * ld;  // padding entries are zero and stay zero
  const double sv[2] = {gamma, rho};
  set_slots(P, S_GAMMA, sv, 2, s);
  const int gridv = grid_for(N, 1024);
  cg_init<T><<<gridv, kBlock, 0, s>>>(N, R, Pd, P.part.p, P2, ld);
  cg_init_finish<<<1, kBlock, 0, s>>>(gridv, P.part.p, tol * tol, P.sc.p);
  HIPCHK(hipGetLastError());
  int k = 0;
  // Launch schedule (results do not depend on it: iterations queued after the
  // device-side convergence flag is set return at once).  The first chunk is
  // the previous solve's iteration count; later chunks aim at the iteration
  // where the residual, decaying at its observed rate, meets the tolerance.
  int chunk = P.cg_last_iters > 0 ? std::min(P.cg_last_iters, 32) : 2;
  constexpr int kRead = S_ITERS + 1;  // slots 0 .. S_ITERS
  double h[kRead];
  int iters = 0;
  bool done = false;
  double rr_prev = -1.0;
  while (!done && k < maxit) {
    const int steps = std::min(chunk, maxit - k);
    const int iters_before = iters;
    for (int i = 0; i < steps; ++i, ++k) {
      const int par = k & 1;
      int np = 0;
      P.prof.run_ext(0, bytes_cg_op(P, r, sizeof(T)), [&](hipEvent_t e0, hipEvent_t e1) {
        np = op_cg<T>(P, W, ldw, r, ld, Pd, P2, Q, t, par, s, e0, e1);
      });
      if (quadG) {
        // the quadratic objective's term mu P (W^T W), its partials after the operator's
        const int gq = grid_for((size_t)P.n * r, 512);
        P.ensure_part((size_t)np + gq);
        cg_quad<T><<<gq, kBlock, 0, s>>>(P.n, r, ld, Pd, quadG, P.mu, Q, P.sc.p, par, P.part.p + np);
        np += gq;
      }
      cg_alpha_finish<<<1, kBlock, 0, s>>>(np, P.part.p, P.sc.p, par);
      cg_update<T><<<gridv, kBlock, 0, s>>>(N, X, R, Pd, Q, P.sc.p, par, P.part.p);
      cg_direction<T><<<gridv, kBlock, 0, s>>>(N, R, Pd, P.sc.p, par, P2, ld, gridv, P.part.p);
    }
    HIPCHK(hipGetLastError());
    // earlier chunks' timings are read while the device runs this one
    if (P.prof.on) P.prof.settle(0);
    read_slots(P, 0, h, kRead, s);
    iters = (int)h[S_ITERS];
    // launches after convergence returned at once: time only the live ones
    if (P.prof.on) P.prof.mark(0, iters - iters_before);
    done = h[S_DONE + (k & 1)] != 0.0;
    const double rr = h[S_RR + (k & 1)], rr0 = h[S_RR0];
    const double rr_ref = rr_prev > 0.0 ? rr_prev : rr0;
    const int ran = iters - iters_before;
    int next = std::min(chunk * 2, 32);
    if (!done && ran > 0 && rr > 0.0 && rr < rr_ref) {
      const double per_it = std::log(rr / rr_ref) / ran;  // log decay per iteration (< 0)
      const double need = std::log(tol * tol * rr0 / rr) / per_it;
      if (std::isfinite(need)) next = std::max(1, std::min(32, (int)std::ceil(need)));
    }
    rr_prev = rr;
    chunk = next;
  }
  P.cg_last_iters = k > 0 ? (int)h[S_ITERS] : P.cg_last_iters;
  read_slots(P, 0, h, kRead, s);
  iters = (int)h[S_ITERS];
  if (relres) *relres = h[S_RR0] > 0 ? std::sqrt(h[S_RR + (k & 1)] / h[S_RR0]) : 0.0;
  if (op_bytes) *op_bytes += (double)iters * bytes_cg_op(P, r, sizeof(T));
  return iters;
}

// explicit instantiations
template void op_forward<double>(Problem&, const double*, const double*, int, int, double*, double, hipStream_t);
template void op_forward<float>(Problem&, const float*, const float*, int, int, float*, double, hipStream_t);
template void op_adjoint<double>(Problem&, const double*, double, const double*, int, int, double*, int, double, hipStream_t);
template void op_adjoint<float>(Problem&, const float*, double, const float*, int, int, float*, int, double, hipStream_t);
template int op_cg<double>(Problem&, const double*, int, int, int, const double*, const double*, double*, double*, int, hipStream_t, hipEvent_t, hipEvent_t);
template int op_cg<float>(Problem&, const float*, int, int, int, const float*, const float*, float*, float*, int, hipStream_t, hipEvent_t, hipEvent_t);
template void dot_to_slot<double, double>(Problem&, size_t, const double*, const double*, double, int, hipStream_t);
template void dot_to_slot<float, float>(Problem&, size_t, const float*, const float*, double, int, hipStream_t);
template int cg_run<double>(Problem&, const double*, int, int, int, double, double, double*, double*, double*, double*, double*, double*, double, int, hipStream_t, double*, double*, const double*);
template int cg_run<float>(Problem&, const float*, int, int, int, double, double, float*, float*, float*, float*, float*, float*, double, int, hipStream_t, double*, double*, const double*);

}  // namespace lorads
