// Batched persistent solve of many diagonal-constraint SDPs (see batch.hip).
#pragma once

#include <memory>

#include "problem.hpp"

namespace lorads {

// Per-instance view into the concatenated pools.
struct BatchDesc {
  int n, m, r0, rcap;  // rcap: factor row stride = rank capacity in the batch
  int cptr_off, ccol_off, dptr_off, con_off, row_off;
  long long fac_off;   // first element of the instance's n x rcap factor block
  double c_fro, b_inf, b_1;
};

struct BatchResult {
  int status, rank, alm_outer, alm_inner, growths, admm_iters;
  long long cg_iters;
  double kkt, pinf_stop, dres_stop, rho, gamma, rho_alm;
  double obj, dual_obj, pinf, gap;
};

struct BatchOpts {
  int phase1, rho_every, max_admm_iter, cg_maxit, lbfgs_mem, alm_inner_max, rank_grow_iters,
      alm_outer_max, r_max;
  double switch_tol, h, eps, rho_growth, rho_max, gamma_fixed, gamma_scale, cg_tol_max,
      cg_tol_floor, cg_tol_kkt, rank_factor, alm_inner_rel, alm_inner_floor, alm_eta,
      alm_rho_factor, rho0;
  uint64_t seed;
};

struct BatchArrays {
  const int *cptr, *ccol, *dptr, *drow;
  const double *cval, *dcoef, *dsq, *b;
  double *U, *V, *Vold, *G, *Gn, *D, *Sn, *Yn, *CD, *R64, *S, *Y;
  double *z, *lam, *p1, *p2;
  void *X, *R, *P, *Q, *W;  // CG vectors in the CG precision
  BatchResult* res;
  long long fac_total;
};

struct Batch {
  bool built = false;
  std::vector<BatchDesc> host_desc;
  long long n_cptr = 0, n_ccol = 0, n_con = 0, n_row = 0, fac_total = 0;
  DevBuf<int> cptr, ccol, dptr, drow;
  DevBuf<double> cval, dcoef, dsq, b;
  DevBuf<double> U, V, Vold, G, Gn, D, Sn, Yn, CD, R64, S, Y;
  DevBuf<double> z, lam, p1, p2;
  DevBuf<char> X, R, P, Q, W;
  DevBuf<BatchResult> res;
  DevBuf<BatchDesc> desc;
  int block = 256;     // workgroup size of the persistent launch (autotuned)
  void build(const std::vector<std::unique_ptr<Problem>>& probs, hipStream_t s);
};

// every problem of the context has diagonal constraints (and there are >= 2)
bool batch_eligible(const std::vector<std::unique_ptr<Problem>>& probs);
// one persistent launch over all problems; fills results and each problem's
// solution (U, V, lambda) for lorads_get_solution
void batch_solve(std::vector<std::unique_ptr<Problem>>& probs, Batch& B, const lorads_options& o,
                 lorads_result* results, hipStream_t s, int block);

}  // namespace lorads
