// Solver entry points shared by the C ABI translation unit.
#pragma once

#include <chrono>

#include "problem.hpp"

namespace lorads {

struct SolveInfo {
  int status = LORADS_OK;
  int alm_outer = 0, alm_inner = 0, growths = 0;
  int admm_iters = 0;
  long long cg_iters = 0;
  double rho_alm = 0, pinf_alm = 0;
  double kkt = 0, pinf_stop = 0, dres_stop = 0, rho = 0, gamma = 0;
  double op_bytes = 0;
  bool warm = false;       // started from a caller multiplier with warm_check on
  int warm_fallback = 0;
};

double quartic_step(double q1, double q2, double q3, double q4);
double gamma_of(const Problem& P, const lorads_options& o, double rho);
int rank_cap(const Problem& P, const lorads_options& o);

// Phase I on P.U (n x P.rank, FP64) and P.lam (internal order); may grow P.rank.
void phase1(Problem& P, const lorads_options& o, SolveInfo& info, hipStream_t s);
// Phase II from U = V = P.U, multiplier P.lam, penalty rho; leaves U, V, lam.
void phase2(Problem& P, const lorads_options& o, double rho, SolveInfo& info, hipStream_t s,
            std::chrono::steady_clock::time_point t_start);

// Appendix-B measures of U_hat = (U + V)/2 and lam; fills the result fields.
void final_metrics(Problem& P, lorads_result& res, hipStream_t s, int lanczos_steps);
// lambda_min(C + A*(lam)) by Lanczos, lam in internal order
// smallest eigenvalue of C + A*(lam), plus P.mu Uh Uh^T when Uh (n x r, the
// solution factor of the quadratic objective) is given
double dual_lambda_min(Problem& P, const double* lam, int max_steps, hipStream_t s,
                       const double* Uh = nullptr, int r = 0);
// G = A^T B (ra x rb, row-major), FP64 MFMA
void gram(const double* A, const double* B, int64_t n, int ra, int rb, int lda, int ldb,
          double* G, hipStream_t s);

// The static workspace of lorads_cg_solve_noalloc (noalloc.hip): record its
// address on the current device (once per device; called by lorads_setup),
// the bytes one call needs, and the CG of lorads_cg_solve run in it on the
// device `dev` the context was set up on.
void scratch_register_current_device();
size_t cg_noalloc_bytes(const Problem& P, int r, int elem);
template <typename T>
void cg_noalloc(Problem& P, int dev, const T* W, double rho, double gamma, const T* R, T* X, int r,
                int ld, double tol, int maxit, hipStream_t s, int* iters, double* relres, bool* ok);

}  // namespace lorads
