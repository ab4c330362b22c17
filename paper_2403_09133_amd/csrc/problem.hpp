// Host-side problem state of the library: ingest, device layouts, operators.
#pragma once

#include <memory>

#include "common.hpp"

namespace lorads {

// Live timing of the operator launches with HIP events recorded on the stream
// the kernels run on.  Kinds: 0 CG operator, 1 forward map, 2 adjoint product.
// Pairs are resolved at the solver's existing synchronisation points; CG
// launches that the device skipped after convergence are not counted.
// kernel classes: 0 CG operator, 1 forward map, 2 adjoint product,
// 3 the warm start's line-search pair A(U D^T + D U^T), A(D D^T)
constexpr int kProfKinds = 4;
struct KernelProfile {
  bool on = false;
  unsigned kinds = ~0u;  // bit k: time class k
  struct Pair { hipEvent_t a, b; double bytes; };
  std::vector<hipEvent_t> all, free_;
  std::vector<Pair> pending[kProfKinds];
  double ms[kProfKinds] = {0, 0, 0, 0}, bytes[kProfKinds] = {0, 0, 0, 0};
  long long count[kProfKinds] = {0, 0, 0, 0};

  hipEvent_t get() {
    if (free_.empty()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      all.push_back(e);
      return e;
    }
    hipEvent_t e = free_.back();
    free_.pop_back();
    return e;
  }
  template <typename F>
  void run(int kind, double b, hipStream_t s, F&& launch) {
    if (!on || !((kinds >> kind) & 1u)) { launch(); return; }
    hipEvent_t e0 = get(), e1 = get();
    HIPCHK(hipEventRecord(e0, s));
    launch();
    HIPCHK(hipEventRecord(e1, s));
    pending[kind].push_back({e0, e1, b});
  }
  // as run, for launch sites that take the two events themselves (a kernel
  // launched with start / stop events is timed from its own dispatch)
  template <typename F>
  void run_ext(int kind, double b, F&& launch) {
    if (!on || !((kinds >> kind) & 1u)) { launch((hipEvent_t) nullptr, (hipEvent_t) nullptr); return; }
    hipEvent_t e0 = get(), e1 = get();
    launch(e0, e1);
    pending[kind].push_back({e0, e1, b});
  }
  // the first `marked` pending pairs of each kind have finished and the first
  // `live` of them are counted; settle() reads them later, so that a launch
  // site can have the host read them while the device runs newer work
  size_t marked[kProfKinds] = {0, 0, 0, 0}, live[kProfKinds] = {0, 0, 0, 0};
  // the pairs of `kind` not yet marked have finished (the caller has seen
  // later work on the stream end); count the first `keep` of them (all when
  // keep < 0)
  void mark(int kind, long long keep = -1) {
    auto& v = pending[kind];
    const size_t fresh = v.size() - marked[kind];
    const size_t k = keep < 0 ? fresh : std::min<size_t>(fresh, (size_t)keep);
    if (k > 0) {
      // counted pairs form a prefix: settle a batch that ends uncounted first
      if (live[kind] != marked[kind]) settle(kind);
      live[kind] = marked[kind] + k;
    }
    marked[kind] = v.size();
  }
  // accumulate the counted marked pairs and return every marked pair's events
  void settle(int kind) {
    auto& v = pending[kind];
    for (size_t i = 0; i < live[kind]; ++i) {
      float t = 0.f;
      HIPCHK(hipEventSynchronize(v[i].b));  // complete already
      HIPCHK(hipEventElapsedTime(&t, v[i].a, v[i].b));
      ms[kind] += t;
      bytes[kind] += v[i].bytes;
      count[kind] += 1;
    }
    for (size_t i = 0; i < marked[kind]; ++i) { free_.push_back(v[i].a); free_.push_back(v[i].b); }
    v.erase(v.begin(), v.begin() + (long)marked[kind]);
    marked[kind] = live[kind] = 0;
  }
  // mark and settle at once; the caller has synchronised the stream
  void resolve(int kind, long long keep = -1) {
    mark(kind, keep);
    settle(kind);
  }
  void resolve_all() {
    for (int k = 0; k < kProfKinds; ++k) resolve(k);
  }
  void reset() {
    for (int k = 0; k < kProfKinds; ++k) {
      for (auto& pr : pending[k]) { free_.push_back(pr.a); free_.push_back(pr.b); }
      pending[k].clear();
      marked[k] = live[k] = 0;
      ms[k] = bytes[k] = 0;
      count[k] = 0;
    }
  }
  ~KernelProfile() {
    for (auto e : all) (void)hipEventDestroy(e);
  }
};

// Device layout of one SDP instance.
//
// Internal constraint order: the order in which constraint-indexed vectors
// (b, z, w, lambda) live on the device.  `perm[i]` is the caller's id of
// internal constraint i; when the caller's order is kept perm_identity is set
// and no permutation is ever applied.
// Pinned, device-mapped host words that read_slots has the device publish
// into: word 0 a sequence number written last, words 1 .. 64 slot values.
struct HostSlots {
  double* h = nullptr;  // host address
  double* d = nullptr;  // device address of the same memory
  long long seq = 0;
  HostSlots() = default;
  HostSlots(const HostSlots&) = delete;
  HostSlots& operator=(const HostSlots&) = delete;
  ~HostSlots() {
    if (h) (void)hipHostFree(h);
  }
  void init() {
    if (h) return;
    HIPCHK(hipHostMalloc((void**)&h, 65 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void**)&d, h, 0));
    *(volatile long long*)h = 0;
  }
};

struct Problem {
  int n = 0, m = 0;
  int structure = LORADS_STRUCT_GENERIC;
  bool perm_identity = true;
  double b_inf = 0, b_1 = 0, b_2 = 0, c_fro = 0, c_1 = 0;
  double c_norm2 = -1.0;  // ||C||_2 once estimated (cost_norm2), else negative
  // objective f(X) = <C, X> + (mu / 2) ||X||_F^2 (mu = 0: the linear SDP)
  double mu = 0;
  int64_t a_nnz = 0, c_nnz = 0;

  DevBuf<int> perm;  // internal -> caller id
  DevBuf<double> b;  // internal order

  // K1 generic: constraint-CSR of the upper-triangle triplets
  DevBuf<int> kptr, krow, kcol;
  DevBuf<double> kval;
  DevBuf<float> kvalf;
  // K2 generic: adjoint row-CSR (both triangles): entries (col, constraint, coef)
  DevBuf<int> aptr, acol, acon;
  DevBuf<double> aval;
  DevBuf<float> avalf;
  // cost matrix C, row-CSR of the full symmetric matrix
  DevBuf<int> cptr, ccol;
  DevBuf<double> cval;
  DevBuf<double> cdiag;  // diagonal C only: C_jj by row (zero where absent), else empty
  DevBuf<float> cvalf;
  // partials of the small Gram products of the quadratic objective
  DevBuf<double> qpart;
  // dense C (at least a quarter of the n^2 entries, n >= kDenseCMinN): also
  // stored in 16 x 64 tiles, each one contiguous run (row bands of 16 rows,
  // ldc a multiple of 64 columns, zero padding), FP64 and FP32; products with
  // C then run on the matrix cores (cdense_apply), with
  // their split partials in cdpart
  DevBuf<double> cdense;
  DevBuf<float> cdensef;
  int ldc = 0;
  DevBuf<char> cdpart;

  // RANK1 structure: A_i = r1c[i] a_i a_i^T.  a_i's entries (index, value) in
  // constraint CSR r1ptr / r1idx / r1val, cut into segments of at most
  // kR1Seg entries (segment s: entries r1sstart[s] .. r1sstart[s + 1] - 1 of
  // constraint r1scon[s]; constraint i owns segments r1cseg[i] ..
  // r1cseg[i + 1] - 1); row view: row t meets constraints r1tcon[e] with
  // a_{i,t} = r1tval[e], e in r1tptr[t] .. r1tptr[t + 1] - 1.  Work vectors
  // (segment partials, per-constraint r-vectors and coefficients) grow with
  // the rank on first use.
  DevBuf<int> r1ptr, r1idx, r1scon, r1sstart, r1cseg, r1tptr, r1tcon;
  DevBuf<double> r1val, r1c, r1tval;
  DevBuf<float> r1valf, r1cf, r1tvalf;
  int r1nseg = 0;
  DevBuf<char> r1work;
  size_t r1work_bytes = 0;

  // DIAG structure: constraint i (internal order) sits on row drow[i] with
  // coefficient dcoef[i]; rows own contiguous constraint ranges dptr.
  DevBuf<int> drow, dptr;
  DevBuf<double> dcoef, dsq;  // dsq[j] = sum of coef^2 of the row's constraints
  DevBuf<float> dcoeff, dsqf;

  // PAIR structure: constraint i = (j, k), j < k, coefficient a (uniform when
  // pcoef is empty: pair_coef).  Two row-owner views for the fused CG operator:
  //   view R: rows j, entries sorted by (j, k) == internal order (ptr: rptr)
  //   incident lists: every constraint in the list of both of its rows,
  //   partners ascending (ptr: inc_ptr)
  DevBuf<int> pj, pk;          // internal order
  DevBuf<double> pcoef;
  DevBuf<float> pcoeff;
  double pair_coef = 0;        // used when pcoef is empty
  DevBuf<int> rptr;            // n+1: view R row pointers (rows owning entries as j)
  // forward-map work list: chunks of at most kPairChunk consecutive view-R
  // constraints of one row (row, first constraint); the chunk ends at the
  // next chunk's start or the row's end
  DevBuf<int> fchunk_row, fchunk_start;
  int nfchunks = 0;
  // XCD chunk lists of the two-column FP64 maps (row, first and last + 1
  // constraint of each chunk; list x at [xchunk_off[x], xchunk_off[x + 1]),
  // all of its partners in partner block x)
  DevBuf<int> xchunk_row, xchunk_start, xchunk_end, xchunk_off;
  int nxchunks = 0, xchunk_maxlen = 0;
  // the incident lists cut by partner block: row t's entries with partners in
  // block x are inc_xptr[t (kXcds + 1) + x] .. inc_xptr[t (kXcds + 1) + x + 1]
  DevBuf<int> inc_xptr;
  // per-XCD partial outputs of the CG operator (kXcds planes of n x ld of the
  // operator's accumulation type), provided by the caller of a CG run whose
  // factor array exceeds one XCD's L2 (nullptr: the single-pass operator)
  void* cg_xparts = nullptr;
  DevBuf<int> inc_ptr, inc_nb, inc_id;  // incident lists: row pointers, partner, internal id
  // uniform coefficient only: [lam, b] per incident entry (interleaved, 16
  // bytes), so the gradient form streams them instead of gathering w by id;
  // lam is filled by refresh_inc_lam
  DevBuf<double> inc_lb;
  bool inc_lb_lam = false;
  // every row's incident entries with partners above the row are, in list
  // order, the view-R constraints rptr[row] .. rptr[row + 1] (checked at setup)
  bool inc_upper_view = false;

  // solver scratch
  DevBuf<double> sc;
  HostSlots hs;
  DevBuf<double> part;
  size_t part_cap = 0;

  // last solution
  int rank = 0;
  bool solved = false;
  DevBuf<double> U, V, lam;  // lam in internal order

  // scratch m-vectors
  DevBuf<double> zbuf, wbuf, tbuf, ubuf;
  DevBuf<float> tbuff;

  KernelProfile prof;
  int cg_last_iters = 0;  // iterations of the last CG solve (launch schedule only)

  // The partial-sum buffer is sized once at setup (kernels may still read it,
  // so it is never reallocated); launches that would need more are refused.
  void ensure_part(size_t need) {
    if (need > part_cap) fail(LORADS_EINVAL, "partial-sum buffer too small for this launch");
  }
};

// host-only validation (throws EINVAL); ingest() validates and uploads
void validate(const lorads_problem& p);
std::unique_ptr<Problem> ingest(const lorads_problem& p, hipStream_t s);

// ---------------------------------------------------------------------------
// operators (enqueued on stream s; vectors in internal constraint order)
// ---------------------------------------------------------------------------
// z = scale * A(U V^T)
template <typename T>
void op_forward(Problem& P, const T* U, const T* V, int r, int ld, T* z, double scale, hipStream_t s);
// z = A(U V^T) and w = lam + rho (z - b)   (FP64)
void op_forward_w(Problem& P, const double* U, const double* V, int r, int ld, double* z,
                  double* w, const double* lam, double rho, hipStream_t s);
// out = out_scale * (c_scale C + A*(w)) V
template <typename T>
void op_adjoint(Problem& P, const T* w, double c_scale, const T* V, int r, int ld, T* out,
                int ldo, double out_scale, hipStream_t s);
// CG operator Q = gamma P + rho A*(A(P W^T)) W with device scalars in sc;
// records the CG step length in sc (see cg_update).  t: m-vector scratch.
template <typename T>
// Q = M_W(Pd) (+ block partials of <Pd, Q> in P.part; returns their count)
// W with row stride ldw; the direction Pd (stride ld), or its copy P2 in the
// rows of W (stride ldw) when P2 is given.  ev0 / ev1 (optional): events that
// receive the operator's start and end (attached to the kernel launch itself
// where the operator is one kernel, else recorded around its launches)
int op_cg(Problem& P, const T* W, int ldw, int r, int ld, const T* Pd, const T* P2, T* Q, T* t,
          int parity, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// p1 = A(U D^T + D U^T) and p2 = A(D D^T) in FP64 (the exact line search),
// U and D with row stride ld
void op_forward_pair(Problem& P, const double* U, const double* D, int r, int ld, double* p1,
                     double* p2, hipStream_t s);
// the fused line-search pass (PAIR): the seven m-vector sums of the quartic
// (p0 = z - b, p1, p2 and lam, the order of linesearch_slots) as
// 7 x ls_blocks(P) block partials in part, without writing p1 and p2; false
// (nothing launched) where the two-column layout does not apply
bool op_linesearch_pair(Problem& P, const double* U, const double* D, int r, int ld,
                        const double* z, const double* lam, double* part, hipStream_t s);
// grid of the two-column maps over the XCD chunk lists for groups of GV
// lanes: kXcds x the blocks the longest list needs (block b serves list
// b mod kXcds)
inline int xchunk_grid(const Problem& P, int GV) {
  const long long per = ((long long)P.xchunk_maxlen * GV + kBlock - 1) / kBlock;
  return (int)std::max<long long>(kXcds, kXcds * std::max<long long>(1, per));
}
// the CG operator runs split by XCD when the interleaved [W | P] rows exceed
// one XCD's L2 (4 MiB): bytes of its per-XCD partials, else 0
inline size_t cg_xparts_bytes(const Problem& P, int ld, int elem) {
  if (P.structure != LORADS_STRUCT_PAIR || P.inc_xptr.n == 0) return 0;
  if ((size_t)P.n * 2 * ld * elem <= ((size_t)4 << 20)) return 0;
  return (size_t)kXcds * P.n * ld * elem;
}
// sets the CG operator's per-XCD partials for the life of a CG run
struct CgXpartsScope {
  Problem& P;
  CgXpartsScope(Problem& P_, void* p) : P(P_) { P.cg_xparts = p; }
  ~CgXpartsScope() { P.cg_xparts = nullptr; }
};
// grid of the fused line-search pass at rank r (groups of G/2 lanes), i.e. its
// count of block partials
// lanes per constraint of the FP64 two-column maps at rank r: half the
// power-of-two group, except 8 lanes with a third column each for r = 17 .. 24
inline int pair_v2_lanes(int r) {
  if (r > 16 && r <= 24) return 8;
  int g = 1;
  while (g < r && g < 64) g <<= 1;
  return std::max(1, g / 2);
}
inline int ls_blocks(const Problem& P, int r) { return xchunk_grid(P, pair_v2_lanes(r)); }
// gradient form for PAIR problems with a uniform coefficient:
//   out = out_scale (C + A*(lam + rho (A(U U^T) - b))) U
// with lam and b read per incident entry (refresh_inc_lam after lam changes);
// bit-identical to op_forward_w followed by op_adjoint.  z (optional) receives
// A(U U^T), bit-identical to op_forward with scale 1 (the gradient kernel
// writes it when it can, otherwise a forward map runs first)
bool grad_pair_ready(const Problem& P);
void refresh_inc_lam(Problem& P, hipStream_t s);
void op_grad_pair(Problem& P, const double* U, int r, int ld, double rho, double* out, int ldo,
                  double out_scale, hipStream_t s, double* z = nullptr);
// line search of the mixed form on FP32 copies U32, D32 of U and D (same row
// stride ld, zero padding): lanes per constraint at rank r, 0 where the form
// does not apply (needs PAIR with a uniform coefficient, ld >= 4 lanes and
// groups of at least 4 lanes)
int pair_f32_lanes(const Problem& P, int r, int ld);
// the fused line search from U32, D32: 7 x ls_blocks_f32 block partials in part
void op_linesearch_pair_f32(Problem& P, const float* U32, const float* D32, int r, int ld,
                            const double* z, const double* lam, double* part, hipStream_t s);
inline int ls_blocks_f32(const Problem& P, int r, int ld) {
  const int g = pair_f32_lanes(P, r, ld);
  return g ? xchunk_grid(P, g) : 0;
}
double bytes_linesearch_pair_f32(const Problem& P, int r);
// G = X^T Y (ra x rb, FP64, row-major) for n-row factors X (ra columns, row
// stride ldx) and Y (rb, ldy), in a fixed order; partials in P.qpart
template <typename T>
void gram_small(Problem& P, int n, int ra, int rb, const T* X, int ldx, const T* Y, int ldy, double* G,
                hipStream_t s);
// out = alpha C V + beta out (first r columns) with the dense copy of C
template <typename T>
void cdense_apply(Problem& P, const T* V, int r, int ld, T* out, int ldo, double alpha, double beta,
                  hipStream_t s);
// leading dimension of the CG work buffers: PAIR problems pad rows to a
// multiple of 64 bytes (zero padding), so every row the CG operator gathers
// sits in whole, aligned 64-byte sectors; other structures use r
int cg_ld(const Problem& P, int r, int elem_bytes);

// algorithmic bytes of one application (for throughput accounting)
double bytes_forward(const Problem& P, int r, int s);
double bytes_adjoint(const Problem& P, int r, int s, bool with_c);
double bytes_cg_op(const Problem& P, int r, int s);
double bytes_grad_pair(const Problem& P, int r);  // gradient form: forward + adjoint (FP64)
double bytes_cprod(const Problem& P, int r, int s);  // C V alone: C's entries, V and the output
// fused line-search pass: indices, z, b and lam once, U and D once (FP64)
double bytes_linesearch_pair(const Problem& P, int r);

// ---------------------------------------------------------------------------
// reductions / small helpers
// ---------------------------------------------------------------------------
void set_slots(Problem& P, int slot, const double* vals, int count, hipStream_t s);
void read_slots(Problem& P, int slot, double* vals, int count, hipStream_t s);  // synchronises
// ||C||_2 by the power method on C (cached in P.c_norm2); synchronises
double cost_norm2(Problem& P, hipStream_t s);
// lam += rho (z - b) and sc[slot] = ||z - b||^2 (rho = 0: norm only)
void dual_update_slot(Problem& P, const double* z, double rho, double* lam, int slot, hipStream_t s);
// the sums of the quartic line search in one pass: sc[slot] = 2 <CD, U>,
// sc[slot + 1] = <CD, D> (first r columns of n rows of stride ld) and the seven
// m-vector inner products of p0 = z - b, p1, p2 and lam -> sc[slot + 2 .. slot + 8];
// part_gd (optional, above the line-search partials in P.part): partials of a
// dot over the same factor grid, summed into sc[slot + 9]
// cdiag (optional, PAIR): C's diagonal by row; then C D is formed in the pass
// as the PAIR adjoint's C part rounds it, and CD is not read
// vals (optional): also read slot .. slot + nread - 1 back to the host (the
// finishing launch publishes them; synchronises like read_slots)
void linesearch_slots(Problem& P, int n, int r, int ld, const double* CD, const double* U,
                      const double* D, const double* z, const double* p1, const double* p2,
                      const double* lam, int slot, hipStream_t s, const double* part_gd = nullptr,
                      const double* cdiag = nullptr, double* vals = nullptr, int nread = 0,
                      const double* lsp = nullptr, int nls = 0);
template <typename TX, typename TY>
void dot_to_slot(Problem& P, size_t N, const TX* X, const TY* Y, double scale, int slot, hipStream_t s);
// the same for n x r factors stored with row stride ld (bit-identical to the
// compact dot_to_slot over n r elements)
void dot_rows_to_slot(Problem& P, int n, int r, int ld, const double* X, const double* Y,
                      double scale, int slot, hipStream_t s);

inline int grid_for(size_t N, int cap = 2048) {
  size_t g = (N + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > (size_t)cap) g = cap;
  return (int)g;
}

// CG on M_W D = R from D = X (X holds x0 = 0 normally; R holds R0 - M x0).
// Buffers dense n x r of type T.  Returns iterations; *relres = ||R||/||R0||.
// quadG (r x r, FP64, optional): W^T W of the quadratic objective, whose term
// P.mu P (W^T W) the operator then includes.
template <typename T>
int cg_run(Problem& P, const T* W, int ldw, int r, int ld, double rho, double gamma, T* R, T* X,
           T* Pd, T* P2, T* Q, T* t, double tol, int maxit, hipStream_t s, double* relres,
           double* op_bytes, const double* quadG = nullptr);

}  // namespace lorads
