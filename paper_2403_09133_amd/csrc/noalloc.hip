// The CG entry point that allocates nothing: lorads_cg_solve_noalloc.
//
// It runs the CG of lorads_cg_solve (the same kernels, launches and results)
// with its work buffers (the CG-layout copies of W, R and X, the direction, the
// operator output, for general constraints the per-constraint buffer, and for
// factors larger than one XCD's L2 the per-XCD partials of the operator)
// placed in one static device array of kScratchBytes instead of allocating
// them.  Each GPU the library runs on holds its own copy of the array until the
// process ends; lorads_setup records that copy's address for the current
// device (hipGetSymbolAddress), and the entry point uses only that address.
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "solver.hpp"

namespace lorads {
// largest workspace the entry point takes: 64 MiB
constexpr size_t kScratchBytes = size_t(64) << 20;
}  // namespace lorads

// The static workspace.  In host code this name is a host-side stand-in, not a
// device address: host code reaches the memory only through the per-device
// address recorded below.
static __device__ __align__(256) unsigned char scratch[lorads::kScratchBytes];

namespace lorads {

namespace {

std::mutex g_scratch_mu;
std::vector<unsigned char*> g_scratch_ptr;  // device address of `scratch`, by device id

template <typename T>
__global__ void __launch_bounds__(kBlock) fill_zero(size_t N, T* __restrict__ x) {
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock)
    x[i] = (T)0;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

void scratch_register_current_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (g_scratch_ptr[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    fail(LORADS_EDEVICE, std::string("hipGetSymbolAddress of the static workspace failed: ") +
                             hipGetErrorString(e));
  g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
}

static unsigned char* scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= (int)g_scratch_ptr.size() || g_scratch_ptr[dev] == nullptr)
    fail(LORADS_ESTATE, "no static workspace recorded for this device (the context was set up on another)");
  return g_scratch_ptr[dev];
}

size_t cg_noalloc_bytes(const Problem& P, int r, int elem) {
  const int ldp = cg_ld(P, r, elem);
  const int ldw = P.structure == LORADS_STRUCT_PAIR ? 2 * ldp : ldp;
  const size_t nt = P.structure == LORADS_STRUCT_GENERIC ? (size_t)P.m : 0;
  // the CG operator's accumulation type is the element type here (FP32 and
  // FP64 accumulate in their own precision)
  return round256((size_t)P.n * ldw * elem) + 4 * round256((size_t)P.n * ldp * elem) +
         round256(nt * elem) + round256(cg_xparts_bytes(P, ldp, elem));
}

template <typename T>
void cg_noalloc(Problem& P, int dev, const T* W, double rho, double gamma, const T* R, T* X, int r,
                int ld, double tol, int maxit, hipStream_t s, int* iters, double* relres, bool* ok) {
  const size_t need = cg_noalloc_bytes(P, r, (int)sizeof(T));
  if (need > kScratchBytes)
    fail(LORADS_EINVAL, "the CG workspace of this call (" + std::to_string(need) +
                            " bytes) exceeds the static workspace of " +
                            std::to_string(kScratchBytes) + " bytes");
  if (!P.hs.h) fail(LORADS_ESTATE, "host words of the problem not set up");
  if (P.structure == LORADS_STRUCT_RANK1)
    fail(LORADS_EINVAL, "rank-one constraint problems are not served without allocation "
                        "(their operator's work vectors grow with the rank)");
  unsigned char* base = scratch_address(dev);
  const int ldp = cg_ld(P, r, (int)sizeof(T));
  const size_t N = (size_t)P.n * ldp;
  const bool inter = P.structure == LORADS_STRUCT_PAIR;
  const int ldw = inter ? 2 * ldp : ldp;
  const size_t bw = round256((size_t)P.n * ldw * sizeof(T)), bn = round256(N * sizeof(T));
  T* Wd = reinterpret_cast<T*>(base);
  T* Rd = reinterpret_cast<T*>(base + bw);
  T* Xd = reinterpret_cast<T*>(base + bw + bn);
  T* Pd = reinterpret_cast<T*>(base + bw + 2 * bn);
  T* Qd = reinterpret_cast<T*>(base + bw + 3 * bn);
  const size_t bt = round256((P.structure == LORADS_STRUCT_GENERIC ? (size_t)P.m : 0) * sizeof(T));
  T* td = P.structure == LORADS_STRUCT_GENERIC ? reinterpret_cast<T*>(base + bw + 4 * bn) : nullptr;
  // per-XCD partials of the split CG operator (large factors only), as
  // lorads_cg_solve provides them
  const size_t xb = cg_xparts_bytes(P, ldp, (int)sizeof(T));
  CgXpartsScope xs(P, xb ? static_cast<void*>(base + bw + 4 * bn + bt) : nullptr);
  // the workspace keeps the last call's contents: clear the buffers (padding
  // columns must be zero) with a fill kernel
  const size_t words = (bw + 4 * bn) / sizeof(T);
  fill_zero<T><<<grid_for(words), kBlock, 0, s>>>(words, Wd);
  T* P2 = inter ? Wd + ldp : nullptr;
  const int g = grid_for(N);
  copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, W, ld, Wd, ldw);
  copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, R, ld, Rd, ldp);
  copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, X, ld, Xd, ldp);
  // R <- R - M x0 (one operator application with the flags cleared)
  const double sv[2] = {gamma, rho};
  set_slots(P, S_GAMMA, sv, 2, s);
  const double flags[2] = {0.0, 0.0};
  set_slots(P, S_DONE, flags, 2, s);
  set_slots(P, S_RR, flags, 2, s);
  if (P2) copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, Xd, ldp, P2, ldw);
  op_cg<T>(P, Wd, ldw, r, ldp, Xd, P2, Qd, td, 0, s);
  axpby<T, T><<<g, kBlock, 0, s>>>(N, -1.0, Qd, 1.0, Rd);
  double rel = 0.0;
  const int it = cg_run<T>(P, Wd, ldw, r, ldp, rho, gamma, Rd, Xd, Pd, P2, Qd, td, tol, maxit, s,
                           &rel, nullptr);
  copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, Xd, ldp, X, ld);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  if (iters) *iters = it;
  if (relres) *relres = rel;
  *ok = rel <= tol;
}

template void cg_noalloc<double>(Problem&, int, const double*, double, double, const double*,
                                 double*, int, int, double, int, hipStream_t, int*, double*, bool*);
template void cg_noalloc<float>(Problem&, int, const float*, double, double, const float*, float*,
                                int, int, double, int, hipStream_t, int*, double*, bool*);

}  // namespace lorads
