// extern "C" boundary of the library (declared in include/lorads.h).
#include <chrono>
#include <cstring>
#include <memory>

#include "batch.hpp"
#include "kernels.hpp"
#include "solver.hpp"

struct lorads_ctx {
  std::vector<std::unique_ptr<lorads::Problem>> probs;
  lorads::Batch batch;
  std::string err;
  hipStream_t stream = nullptr;
  int device = 0;
};

namespace {

thread_local std::string g_setup_err;

lorads_status record(lorads_ctx* ctx, const lorads::Error& e) {
  if (ctx) ctx->err = e.msg; else g_setup_err = e.msg;
  return e.status;
}

template <typename F>
lorads_status guarded(lorads_ctx* ctx, F&& f) {
  try {
    f();
    return LORADS_OK;
  } catch (const lorads::Error& e) {
    return record(ctx, e);
  } catch (const std::bad_alloc&) {
    return record(ctx, {LORADS_ENOMEM, "host allocation failed"});
  } catch (const std::exception& e) {
    return record(ctx, {LORADS_EDEVICE, e.what()});
  }
}

lorads::Problem& get(lorads_ctx* ctx, int prob) {
  if (!ctx) lorads::fail(LORADS_EINVAL, "null context");
  if (prob < 0 || prob >= (int)ctx->probs.size()) lorads::fail(LORADS_EINVAL, "problem index out of range");
  return *ctx->probs[prob];
}

void check_factor(const void* p, int r, int ld) {
  if (!p) lorads::fail(LORADS_EINVAL, "null factor pointer");
  if (r < 1 || r > 256) lorads::fail(LORADS_EINVAL, "rank must be in [1, 256]");
  if (ld < r) lorads::fail(LORADS_EINVAL, "ld must be >= r");
}

void check_dtype(int dtype) {
  if (dtype != LORADS_F64 && dtype != LORADS_F32) lorads::fail(LORADS_EINVAL, "unknown dtype");
}

}  // namespace

using namespace lorads;

void lorads::set_global_error(const std::string& msg) { g_setup_err = msg; }

extern "C" {

const char* lorads_version(void) { return "lorads-gfx950 0.1"; }

const char* lorads_last_error(const lorads_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_setup_err.c_str();
}

void lorads_default_options(lorads_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = LORADS_F64;
  o->eps = 1e-6;
  o->switch_tol = 1e-3;
  o->h = 1.0;
  o->rho_growth = 1.2;
  o->rho_every = 5;
  o->rho_max = 5000.0;
  o->max_admm_iter = 5000;
  o->time_limit = 0.0;
  o->gamma_fixed = 0.0;
  o->gamma_scale = 1.0;
  o->cg_tol_max = 0.1;
  o->cg_tol_floor = 1e-12;
  o->cg_tol_kkt = 1e-2;
  o->cg_maxit = 2000;
  o->lbfgs_mem = 4;
  o->alm_inner_max = 2000;
  o->rank_grow_iters = 1000;
  o->rank_factor = 1.5;
  o->r0 = 0;
  o->r_max = 0;
  o->alm_inner_rel = 0.1;
  o->alm_inner_floor = 1e-8;
  o->alm_eta = 0.25;
  o->alm_rho_factor = 10.0;
  o->alm_outer_max = 200;
  o->rho0 = 0.0;
  o->seed = 0;
  o->phase1 = 1;
  o->verbose = 0;
  o->profile = 0;
  o->batch_mode = 0;
  o->batch_block = 0;
  o->init_U = nullptr;
  o->init_lambda = nullptr;
  o->init_rank = nullptr;
  o->warm_check = 0;
  o->gamma_rule = 0;
}

lorads_status lorads_setup(const lorads_problem* probs, int32_t nprob, lorads_ctx** out) {
  if (!out) return record(nullptr, {LORADS_EINVAL, "null output pointer"});
  *out = nullptr;
  if (!probs || nprob < 1) return record(nullptr, {LORADS_EINVAL, "need at least one problem"});
  auto ctx = std::make_unique<lorads_ctx>();
  // validate every problem on the host before any device call
  lorads_status st = guarded(nullptr, [&] {
    for (int i = 0; i < nprob; ++i) {
      try {
        validate(probs[i]);
      } catch (Error& e) {
        e.msg = "problem " + std::to_string(i) + ": " + e.msg;
        throw;
      }
    }
  });
  if (st != LORADS_OK) return st;
  st = guarded(nullptr, [&] {
    HIPCHK(hipGetDevice(&ctx->device));
    HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
    for (int i = 0; i < nprob; ++i) {
      try {
        ctx->probs.push_back(ingest(probs[i], ctx->stream));
      } catch (Error& e) {
        e.msg = "problem " + std::to_string(i) + ": " + e.msg;
        throw;
      }
      // the pinned words the solver reads its scalars through, made here so
      // that lorads_cg_solve_noalloc never allocates
      ctx->probs.back()->hs.init();
    }
    scratch_register_current_device();
  });
  if (st != LORADS_OK) {
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    return st;
  }
  *out = ctx.release();
  return LORADS_OK;
}

lorads_status lorads_problem_info(const lorads_ctx* ctx, int32_t prob, int32_t* structure,
                                  int32_t* n, int32_t* m) {
  return guarded(const_cast<lorads_ctx*>(ctx), [&] {
    Problem& P = get(const_cast<lorads_ctx*>(ctx), prob);
    if (structure) *structure = P.structure;
    if (n) *n = P.n;
    if (m) *m = P.m;
  });
}

lorads_status lorads_problem_flags(const lorads_ctx* ctx, int32_t prob, int32_t* flags) {
  return guarded(const_cast<lorads_ctx*>(ctx), [&] {
    Problem& P = get(const_cast<lorads_ctx*>(ctx), prob);
    if (!flags) fail(LORADS_EINVAL, "flags");
    *flags = P.cdense.n ? LORADS_FLAG_DENSE_C : 0;
  });
}

void lorads_destroy(lorads_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->probs.clear();
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

lorads_status lorads_apply_A(lorads_ctx* ctx, int32_t prob, const void* U, const void* V,
                             int32_t r, int32_t ld, void* z, int32_t dtype, void* stream) {
  return guarded(ctx, [&] {
    Problem& P = get(ctx, prob);
    check_factor(U, r, ld);
    check_factor(V, r, ld);
    check_dtype(dtype);
    if (!z) fail(LORADS_EINVAL, "null output");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == LORADS_F64) {
      double* dst = P.perm_identity ? (double*)z : P.tbuf.p;
      op_forward<double>(P, (const double*)U, (const double*)V, r, ld, dst, 1.0, s);
      if (!P.perm_identity)
        scatter_kernel<double><<<grid_for(P.m), kBlock, 0, s>>>(P.m, P.perm.p, dst, (double*)z);
    } else {
      float* dst = P.perm_identity ? (float*)z : P.tbuff.p;
      op_forward<float>(P, (const float*)U, (const float*)V, r, ld, dst, 1.0, s);
      if (!P.perm_identity)
        scatter_kernel<float><<<grid_for(P.m), kBlock, 0, s>>>(P.m, P.perm.p, dst, (float*)z);
    }
    HIPCHK(hipGetLastError());
  });
}

lorads_status lorads_apply_AT_V(lorads_ctx* ctx, int32_t prob, const void* w, double c_scale,
                                const void* V, int32_t r, int32_t ld, void* out, int32_t dtype,
                                void* stream) {
  return guarded(ctx, [&] {
    Problem& P = get(ctx, prob);
    check_factor(V, r, ld);
    check_factor(out, r, ld);
    check_dtype(dtype);
    if (!w) fail(LORADS_EINVAL, "null w");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == LORADS_F64) {
      const double* wi = (const double*)w;
      if (!P.perm_identity) {
        gather_kernel<double><<<grid_for(P.m), kBlock, 0, s>>>(P.m, P.perm.p, wi, P.tbuf.p);
        wi = P.tbuf.p;
      }
      op_adjoint<double>(P, wi, c_scale, (const double*)V, r, ld, (double*)out, ld, 1.0, s);
    } else {
      const float* wi = (const float*)w;
      if (!P.perm_identity) {
        gather_kernel<float><<<grid_for(P.m), kBlock, 0, s>>>(P.m, P.perm.p, wi, P.tbuff.p);
        wi = P.tbuff.p;
      }
      op_adjoint<float>(P, wi, c_scale, (const float*)V, r, ld, (float*)out, ld, 1.0, s);
    }
    HIPCHK(hipGetLastError());
  });
}

}  // extern "C"

namespace {

template <typename T>
void cg_api(Problem& P, const T* W, double rho, double gamma, const T* R, T* X, int r, int ld,
            double tol, int maxit, hipStream_t s, int* iters, double* relres, bool* ok) {
  // internal buffers in the CG layout (zero padding beyond column r)
  const int ldp = cg_ld(P, r, (int)sizeof(T));
  const size_t N = (size_t)P.n * ldp;
  // PAIR: W and a copy of the direction share rows (stride 2 ldp)
  const bool inter = P.structure == LORADS_STRUCT_PAIR;
  const int ldw = inter ? 2 * ldp : ldp;
  DevBuf<T> Wd, Rd, Xd, Pd, Qd, td;
  Wd.alloc((size_t)P.n * ldw); Rd.alloc(N); Xd.alloc(N); Pd.alloc(N); Qd.alloc(N); td.alloc(P.m);
  Wd.zero(s); Rd.zero(s); Xd.zero(s); Pd.zero(s); Qd.zero(s);
  T* P2 = inter ? Wd.p + ldp : nullptr;
  // per-XCD partials of the split CG operator when the factors exceed one L2
  DevBuf<char> xparts;
  const size_t xb = cg_xparts_bytes(P, ldp, (int)sizeof(typename OpAcc<T>::type));
  if (xb) xparts.alloc(xb);
  CgXpartsScope xs(P, xb ? xparts.p : nullptr);
  const int g = grid_for(N);
  copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, W, ld, Wd.p, ldw);
  copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, R, ld, Rd.p, ldp);
  copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, X, ld, Xd.p, ldp);
  // R <- R - M x0 (one operator application with the flags cleared)
  const double sv[4] = {gamma, rho, 0.0, 0.0};
  set_slots(P, S_GAMMA, sv, 2, s);
  const double flags[2] = {0.0, 0.0};
  set_slots(P, S_DONE, flags, 2, s);
  set_slots(P, S_RR, flags, 2, s);
  if (P2) copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, Xd.p, ldp, P2, ldw);
  op_cg<T>(P, Wd.p, ldw, r, ldp, Xd.p, P2, Qd.p, td.p, 0, s);
  axpby<T, T><<<g, kBlock, 0, s>>>(N, -1.0, Qd.p, 1.0, Rd.p);
  double rel = 0.0;
  const int it = cg_run<T>(P, Wd.p, ldw, r, ldp, rho, gamma, Rd.p, Xd.p, Pd.p, P2, Qd.p, td.p, tol,
                           maxit, s, &rel, nullptr);
  copy_rows<T, T><<<g, kBlock, 0, s>>>(P.n, r, Xd.p, ldp, X, ld);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  if (iters) *iters = it;
  if (relres) *relres = rel;
  *ok = rel <= tol;
}

}  // namespace

extern "C" {

lorads_status lorads_cg_solve(lorads_ctx* ctx, int32_t prob, const void* W, double rho,
                              double gamma, const void* R, void* X, int32_t r, int32_t ld,
                              double tol, int32_t maxit, int32_t dtype, int32_t* iters,
                              double* relres, void* stream) {
  bool ok = true;
  lorads_status st = guarded(ctx, [&] {
    Problem& P = get(ctx, prob);
    check_factor(W, r, ld);
    check_factor(R, r, ld);
    check_factor(X, r, ld);
    check_dtype(dtype);
    if (!(rho >= 0.0) || !(gamma > 0.0)) fail(LORADS_EINVAL, "need rho >= 0 and gamma > 0");
    if (!(tol >= 0.0) || maxit < 0) fail(LORADS_EINVAL, "need tol >= 0 and maxit >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == LORADS_F64)
      cg_api<double>(P, (const double*)W, rho, gamma, (const double*)R, (double*)X, r, ld, tol,
                     maxit, s, iters, relres, &ok);
    else
      cg_api<float>(P, (const float*)W, rho, gamma, (const float*)R, (float*)X, r, ld, tol, maxit,
                    s, iters, relres, &ok);
  });
  if (st == LORADS_OK && !ok) return LORADS_MAXITER;
  return st;
}

lorads_status lorads_cg_solve_noalloc(lorads_ctx* ctx, int32_t prob, const void* W, double rho,
                                      double gamma, const void* R, void* X, int32_t r, int32_t ld,
                                      double tol, int32_t maxit, int32_t dtype, int32_t* iters,
                                      double* relres, void* stream) {
  bool ok = true;
  lorads_status st = guarded(ctx, [&] {
    Problem& P = get(ctx, prob);
    check_factor(W, r, ld);
    check_factor(R, r, ld);
    check_factor(X, r, ld);
    check_dtype(dtype);
    if (!(rho >= 0.0) || !(gamma > 0.0)) fail(LORADS_EINVAL, "need rho >= 0 and gamma > 0");
    if (!(tol >= 0.0) || maxit < 0) fail(LORADS_EINVAL, "need tol >= 0 and maxit >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == LORADS_F64)
      cg_noalloc<double>(P, ctx->device, (const double*)W, rho, gamma, (const double*)R, (double*)X,
                         r, ld, tol, maxit, s, iters, relres, &ok);
    else
      cg_noalloc<float>(P, ctx->device, (const float*)W, rho, gamma, (const float*)R, (float*)X, r,
                        ld, tol, maxit, s, iters, relres, &ok);
  });
  if (st == LORADS_OK && !ok) return LORADS_MAXITER;
  return st;
}

lorads_status lorads_admm_solve(lorads_ctx* ctx, const lorads_options* opt, lorads_result* res) {
  lorads_status worst = LORADS_OK;
  lorads_status st = guarded(ctx, [&] {
    if (!ctx || !opt || !res) fail(LORADS_EINVAL, "null argument");
    const lorads_options& o = *opt;
    if (o.precision != LORADS_F64 && o.precision != LORADS_F32 && o.precision != LORADS_MIXED)
      fail(LORADS_EINVAL, "precision");
    if (!(o.eps > 0) || o.max_admm_iter < 0 || o.lbfgs_mem < 1 || o.lbfgs_mem > 16 ||
        o.rho_every < 1 || o.profile < 0 || o.profile > 2 || o.gamma_rule < 0 || o.gamma_rule > 1)
      fail(LORADS_EINVAL, "invalid options");
    if (!o.init_U) fail(LORADS_EINVAL, "init_U is required (the random start is an input)");
    for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
      const int r0 = o.init_rank ? o.init_rank[pi] : o.r0;
      if (r0 < 1 || r0 > 256 || r0 > ctx->probs[pi]->n)
        fail(LORADS_EINVAL, "initial rank of problem " + std::to_string(pi) + " must be in [1, min(256, n)]");
    }
    hipStream_t s = ctx->stream;
    bool warm_checked = false;
    if (o.warm_check && o.init_lambda)
      for (size_t pi = 0; pi < ctx->probs.size(); ++pi) warm_checked |= o.init_lambda[pi] != nullptr;
    if (o.batch_mode == 1 && warm_checked)
      fail(LORADS_EINVAL, "warm_check with a given init_lambda needs the sequential path");
    const bool batch_ok = batch_eligible(ctx->probs) && (o.gamma_rule == 0 || o.gamma_fixed > 0);
    if (o.batch_mode != 2 && !warm_checked && batch_ok) {
      // all problems in one persistent launch
      const auto t0 = std::chrono::steady_clock::now();
      batch_solve(ctx->probs, ctx->batch, o, res, s,
                  o.batch_block > 0 ? o.batch_block : ctx->batch.block);
      const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
        res[pi].t_total = t;
        res[pi].t_phase2 = t;
        if (res[pi].status > worst) worst = (lorads_status)res[pi].status;
      }
      return;
    }
    if (o.batch_mode == 1)
      fail(LORADS_EINVAL, "batched solve needs >= 2 problems, all with diagonal constraints and mu = 0, "
                          "and gamma rule 0");
    for (size_t pi = 0; pi < ctx->probs.size(); ++pi) {
      Problem& P = *ctx->probs[pi];
      if (!o.init_U[pi]) fail(LORADS_EINVAL, "init_U missing for problem " + std::to_string(pi));
      const int r0 = o.init_rank ? o.init_rank[pi] : o.r0;
      lorads_result& R = res[pi];
      std::memset(&R, 0, sizeof(R));
      const auto t0 = std::chrono::steady_clock::now();
      P.rank = r0;
      P.U.upload(o.init_U[pi], (size_t)P.n * r0, s);
      P.lam.alloc(P.m);
      if (o.init_lambda && o.init_lambda[pi]) {
        DevBuf<double> tmp;
        tmp.upload(o.init_lambda[pi], P.m, s);
        if (P.perm_identity)
          HIPCHK(hipMemcpyAsync(P.lam.p, tmp.p, P.m * sizeof(double), hipMemcpyDeviceToDevice, s));
        else
          gather_kernel<double><<<grid_for(P.m), kBlock, 0, s>>>(P.m, P.perm.p, tmp.p, P.lam.p);
        HIPCHK(hipStreamSynchronize(s));
      } else {
        P.lam.zero(s);
      }
      SolveInfo info;
      info.warm = o.warm_check && o.init_lambda && o.init_lambda[pi];
      P.prof.reset();
      P.prof.on = o.profile != 0;
      P.prof.kinds = o.profile == 2 ? 1u : ~0u;
      double rho;
      if (o.phase1) {
        phase1(P, o, info, s);
        rho = info.rho_alm;
      } else {
        rho = o.rho0 > 0 ? o.rho0 : 1.0 / std::max(1.0, P.b_inf);
      }
      HIPCHK(hipStreamSynchronize(s));
      const auto t1 = std::chrono::steady_clock::now();
      phase2(P, o, o.h * rho, info, s, t0);
      HIPCHK(hipStreamSynchronize(s));
      const auto t2 = std::chrono::steady_clock::now();
      P.prof.resolve_all();
      P.prof.on = false;
      for (int k = 0; k < kProfKinds; ++k) {
        R.prof_ms[k] = P.prof.ms[k];
        R.prof_bytes[k] = P.prof.bytes[k];
        R.prof_launches[k] = P.prof.count[k];
      }
      P.solved = true;
      final_metrics(P, R, s, 300);
      HIPCHK(hipStreamSynchronize(s));
      const auto t3 = std::chrono::steady_clock::now();
      R.status = info.status;
      R.rank = P.rank;
      R.alm_outer = info.alm_outer;
      R.alm_inner = info.alm_inner;
      R.rank_growths = info.growths;
      R.warm_fallback = info.warm_fallback;
      R.admm_iters = info.admm_iters;
      R.cg_iters = info.cg_iters;
      R.kkt = info.kkt;
      R.pinf_stop = info.pinf_stop;
      R.dres_stop = info.dres_stop;
      R.rho = info.rho;
      R.gamma = info.gamma;
      R.op_bytes = info.op_bytes;
      R.t_phase1 = std::chrono::duration<double>(t1 - t0).count();
      R.t_phase2 = std::chrono::duration<double>(t2 - t1).count();
      R.t_metrics = std::chrono::duration<double>(t3 - t2).count();
      R.t_total = std::chrono::duration<double>(t2 - t0).count();
      if (o.verbose > 0)
        fprintf(stderr,
                "[lorads] problem %zu: r=%d alm %d/%d admm %d cg %lld kkt %.2e obj %.10g "
                "(%.3fs + %.3fs)\n",
                pi, R.rank, R.alm_outer, R.alm_inner, R.admm_iters, (long long)R.cg_iters, R.kkt,
                R.obj, R.t_phase1, R.t_phase2);
      if (R.status > worst) worst = (lorads_status)R.status;
    }
  });
  return st != LORADS_OK ? st : worst;
}

lorads_status lorads_batch_autotune(lorads_ctx* ctx, const lorads_options* opt, const int32_t* cand,
                                    int32_t ncand, int32_t* best, double* times_ms) {
  return guarded(ctx, [&] {
    if (!ctx || !opt || !cand || ncand < 1 || !best) fail(LORADS_EINVAL, "null argument");
    if (!batch_eligible(ctx->probs)) fail(LORADS_EINVAL, "context is not eligible for the batched launch");
    hipStream_t s = ctx->stream;
    std::vector<lorads_result> res(ctx->probs.size());
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    double best_ms = INFINITY;
    int best_b = 0;
    for (int i = 0; i < ncand; ++i) {
      HIPCHK(hipEventRecord(e0, s));
      batch_solve(ctx->probs, ctx->batch, *opt, res.data(), s, cand[i]);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (times_ms) times_ms[i] = ms;
      if (ms < best_ms) { best_ms = ms; best_b = cand[i]; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->batch.block = best_b;
    *best = best_b;
  });
}

lorads_status lorads_get_solution(const lorads_ctx* cctx, int32_t prob, double* U, double* V,
                                  double* lambda) {
  lorads_ctx* ctx = const_cast<lorads_ctx*>(cctx);
  return guarded(ctx, [&] {
    Problem& P = get(ctx, prob);
    if (!P.solved) fail(LORADS_ESTATE, "no solution yet");
    hipStream_t s = ctx->stream;
    const size_t N = (size_t)P.n * P.rank;
    if (U) HIPCHK(hipMemcpyAsync(U, P.U.p, N * sizeof(double), hipMemcpyDeviceToHost, s));
    if (V) HIPCHK(hipMemcpyAsync(V, P.V.p, N * sizeof(double), hipMemcpyDeviceToHost, s));
    if (lambda) {
      if (P.perm_identity) {
        HIPCHK(hipMemcpyAsync(lambda, P.lam.p, P.m * sizeof(double), hipMemcpyDeviceToHost, s));
      } else {
        scatter_kernel<double><<<grid_for(P.m), kBlock, 0, s>>>(P.m, P.perm.p, P.lam.p, P.tbuf.p);
        HIPCHK(hipMemcpyAsync(lambda, P.tbuf.p, P.m * sizeof(double), hipMemcpyDeviceToHost, s));
      }
    }
    HIPCHK(hipStreamSynchronize(s));
  });
}

lorads_status lorads_gram(const void* A, const void* B, int64_t n, int32_t ra, int32_t rb,
                          int32_t lda, int32_t ldb, void* G, void* stream) {
  return guarded(nullptr, [&] {
    if (!A || !B || !G) fail(LORADS_EINVAL, "null pointer");
    if (lda < ra || ldb < rb) fail(LORADS_EINVAL, "leading dimension too small");
    gram((const double*)A, (const double*)B, n, ra, rb, lda, ldb, (double*)G, (hipStream_t)stream);
  });
}

lorads_status lorads_dual_lambda_min(lorads_ctx* ctx, int32_t prob, const void* lambda,
                                     int32_t max_steps, double* out) {
  return guarded(ctx, [&] {
    Problem& P = get(ctx, prob);
    if (!lambda || !out) fail(LORADS_EINVAL, "null pointer");
    if (max_steps < 2) fail(LORADS_EINVAL, "max_steps must be >= 2");
    hipStream_t s = ctx->stream;
    const double* li = (const double*)lambda;
    DevBuf<double> tmp;
    if (!P.perm_identity) {
      tmp.alloc(P.m);
      gather_kernel<double><<<grid_for(P.m), kBlock, 0, s>>>(P.m, P.perm.p, li, tmp.p);
      li = tmp.p;
    }
    *out = dual_lambda_min(P, li, max_steps, s);
    HIPCHK(hipStreamSynchronize(s));
  });
}

}  // extern "C"
