"""ctypes binding of liblorads.so (argument marshalling only).

Every computation happens in the gfx950 library; this module converts numpy
arrays and torch device tensors into the pointers, sizes and structs of the C
ABI declared in include/lorads.h.  Loading fails loudly when the library has
not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import pathlib
from typing import Optional, Sequence

import numpy as np

_LIB_PATH = pathlib.Path(__file__).resolve().parent / "liblorads.so"
_lib = None

LORADS_OK, LORADS_MAXITER, LORADS_TIMELIMIT = 0, 1, 2
LORADS_EINVAL, LORADS_ENOMEM, LORADS_EDEVICE, LORADS_ENUMERIC, LORADS_ESTATE = -1, -2, -3, -4, -5
F64, F32 = 0, 1
MIXED = 2  # solver precision: FP32 CG and FP32 line-search maps
LORADS_FLAG_DENSE_C = 1
STRUCT_NAMES = {0: "generic", 1: "diag", 2: "pair", 3: "rank1"}


class LoradsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lorads status {status}: {msg}")
        self.status = status


class Problem_(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("m", C.c_int32),
        ("c_nnz", C.c_int64), ("c_row", C.c_void_p), ("c_col", C.c_void_p), ("c_val", C.c_void_p),
        ("a_nnz", C.c_int64), ("a_con", C.c_void_p), ("a_row", C.c_void_p), ("a_col", C.c_void_p),
        ("a_val", C.c_void_p), ("b", C.c_void_p), ("mu", C.c_double),
    ]


class Options_(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("eps", C.c_double), ("switch_tol", C.c_double), ("h", C.c_double),
        ("rho_growth", C.c_double), ("rho_every", C.c_int32), ("rho_max", C.c_double),
        ("max_admm_iter", C.c_int32), ("time_limit", C.c_double), ("gamma_fixed", C.c_double),
        ("gamma_scale", C.c_double), ("cg_tol_max", C.c_double), ("cg_tol_floor", C.c_double),
        ("cg_tol_kkt", C.c_double), ("cg_maxit", C.c_int32), ("lbfgs_mem", C.c_int32),
        ("alm_inner_max", C.c_int32), ("rank_grow_iters", C.c_int32), ("rank_factor", C.c_double),
        ("r0", C.c_int32), ("r_max", C.c_int32), ("alm_inner_rel", C.c_double),
        ("alm_inner_floor", C.c_double), ("alm_eta", C.c_double), ("alm_rho_factor", C.c_double),
        ("alm_outer_max", C.c_int32), ("rho0", C.c_double), ("seed", C.c_uint64),
        ("phase1", C.c_int32), ("verbose", C.c_int32), ("profile", C.c_int32),
        ("batch_mode", C.c_int32), ("batch_block", C.c_int32),
        ("init_U", C.c_void_p), ("init_lambda", C.c_void_p), ("init_rank", C.c_void_p),
        ("warm_check", C.c_int32), ("gamma_rule", C.c_int32),
    ]


class Result_(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("rank", C.c_int32), ("alm_outer", C.c_int32), ("alm_inner", C.c_int32),
        ("rank_growths", C.c_int32), ("admm_iters", C.c_int32), ("cg_iters", C.c_int64),
        ("obj", C.c_double), ("dual_obj", C.c_double), ("pinf", C.c_double), ("dinf", C.c_double),
        ("gap", C.c_double), ("lambda_min", C.c_double), ("kkt", C.c_double),
        ("pinf_stop", C.c_double), ("dres_stop", C.c_double), ("rho", C.c_double),
        ("gamma", C.c_double), ("t_phase1", C.c_double), ("t_phase2", C.c_double),
        ("t_metrics", C.c_double), ("t_total", C.c_double), ("op_bytes", C.c_double),
        ("prof_ms", C.c_double * 4), ("prof_bytes", C.c_double * 4), ("prof_launches", C.c_int64 * 4),
        ("warm_fallback", C.c_int32),
    ]


EXPORTED = [
    "lorads_default_options", "lorads_setup", "lorads_problem_info", "lorads_problem_flags",
    "lorads_apply_A",
    "lorads_apply_AT_V", "lorads_cg_solve", "lorads_cg_solve_noalloc", "lorads_admm_solve",
    "lorads_get_solution",
    "lorads_gram", "lorads_dual_lambda_min", "lorads_destroy", "lorads_last_error",
    "lorads_version", "lorads_batch_autotune",
    "lorads_gnn_param_count", "lorads_gnn_create", "lorads_gnn_set_params",
    "lorads_gnn_get_params", "lorads_gnn_load_graphs", "lorads_gnn_set_targets",
    "lorads_gnn_forward", "lorads_gnn_loss_grad", "lorads_gnn_adam_step",
    "lorads_gnn_layer_time", "lorads_gnn_destroy",
]


def library_path() -> pathlib.Path:
    return _LIB_PATH


def load():
    """Load liblorads.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -m paper_2403_09133_amd.build`")
    lib = C.CDLL(str(_LIB_PATH))
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.lorads_default_options.argtypes = [C.POINTER(Options_)]
    lib.lorads_default_options.restype = None
    lib.lorads_setup.argtypes = [C.POINTER(Problem_), i32, C.POINTER(vp)]
    lib.lorads_problem_info.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.lorads_apply_A.argtypes = [vp, i32, vp, vp, i32, i32, vp, i32, vp]
    lib.lorads_apply_AT_V.argtypes = [vp, i32, vp, dbl, vp, i32, i32, vp, i32, vp]
    lib.lorads_cg_solve.argtypes = [vp, i32, vp, dbl, dbl, vp, vp, i32, i32, dbl, i32, i32,
                                    C.POINTER(i32), C.POINTER(dbl), vp]
    lib.lorads_cg_solve_noalloc.argtypes = lib.lorads_cg_solve.argtypes
    lib.lorads_admm_solve.argtypes = [vp, C.POINTER(Options_), C.POINTER(Result_)]
    lib.lorads_get_solution.argtypes = [vp, i32, vp, vp, vp]
    lib.lorads_gram.argtypes = [vp, vp, i64, i32, i32, i32, i32, vp, vp]
    lib.lorads_dual_lambda_min.argtypes = [vp, i32, vp, i32, C.POINTER(dbl)]
    lib.lorads_batch_autotune.argtypes = [vp, C.POINTER(Options_), C.POINTER(i32), i32,
                                          C.POINTER(i32), C.POINTER(dbl)]
    lib.lorads_destroy.argtypes = [vp]
    lib.lorads_destroy.restype = None
    lib.lorads_last_error.argtypes = [vp]
    lib.lorads_last_error.restype = C.c_char_p
    lib.lorads_version.restype = C.c_char_p
    flt = C.c_float
    lib.lorads_gnn_param_count.argtypes = [i32]
    lib.lorads_gnn_param_count.restype = i64
    lib.lorads_gnn_create.argtypes = [i32, C.POINTER(vp)]
    lib.lorads_gnn_set_params.argtypes = [vp, vp, i64]
    lib.lorads_gnn_get_params.argtypes = [vp, vp, i64]
    lib.lorads_gnn_load_graphs.argtypes = [vp, i32, vp, i64, vp, vp, vp]
    lib.lorads_gnn_set_targets.argtypes = [vp, vp, vp]
    lib.lorads_gnn_forward.argtypes = [vp, i32, i32, vp, vp]
    lib.lorads_gnn_loss_grad.argtypes = [vp, i32, i32, flt, C.POINTER(dbl), vp, i64]
    lib.lorads_gnn_adam_step.argtypes = [vp, flt, flt, flt, flt]
    lib.lorads_gnn_layer_time.argtypes = [vp, C.POINTER(dbl), C.POINTER(i64), C.POINTER(dbl)]
    lib.lorads_gnn_destroy.argtypes = [vp]
    lib.lorads_gnn_destroy.restype = None
    for name in ("lorads_setup", "lorads_problem_info", "lorads_apply_A", "lorads_apply_AT_V",
                 "lorads_cg_solve", "lorads_cg_solve_noalloc", "lorads_admm_solve", "lorads_get_solution", "lorads_gram",
                 "lorads_dual_lambda_min", "lorads_batch_autotune", "lorads_gnn_create",
                 "lorads_gnn_set_params", "lorads_gnn_get_params", "lorads_gnn_load_graphs",
                 "lorads_gnn_set_targets", "lorads_gnn_forward", "lorads_gnn_loss_grad",
                 "lorads_gnn_adam_step", "lorads_gnn_layer_time"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _ptr(a) -> int:
    if a is None:
        return 0
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _stream(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:  # pragma: no cover
            pass
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


def _dtype_code(t) -> int:
    name = str(t.dtype)
    if name.endswith("float64"):
        return F64
    if name.endswith("float32"):
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _factor_shape(t):
    if t.dim() != 2:
        raise ValueError("factor must be 2-D (n x r)")
    if t.stride(1) != 1:
        raise ValueError("factor must be row-major with unit column stride")
    return int(t.shape[1]), int(t.stride(0))


def default_options(**kw) -> Options_:
    o = Options_()
    load().lorads_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Context:
    """Owns a lorads_ctx: the device copies of one or more SDP instances."""

    def __init__(self, problems):
        lib = load()
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self._keep = []
        arr = (Problem_ * len(problems))()
        for i, p in enumerate(problems):
            cols = {}
            for name, dt in (("c_row", np.int32), ("c_col", np.int32), ("c_val", np.float64),
                             ("a_con", np.int32), ("a_row", np.int32), ("a_col", np.int32),
                             ("a_val", np.float64), ("b", np.float64)):
                a = np.ascontiguousarray(getattr(p, name), dtype=dt)
                self._keep.append(a)
                cols[name] = a
            arr[i] = Problem_(int(p.n), int(p.m), int(cols["c_row"].size), _ptr(cols["c_row"]),
                              _ptr(cols["c_col"]), _ptr(cols["c_val"]), int(cols["a_row"].size),
                              _ptr(cols["a_con"]), _ptr(cols["a_row"]), _ptr(cols["a_col"]),
                              _ptr(cols["a_val"]), _ptr(cols["b"]), float(getattr(p, "mu", 0.0)))
        h = C.c_void_p()
        st = lib.lorads_setup(arr, len(problems), C.byref(h))
        self._keep = []
        if st != LORADS_OK:
            raise LoradsError(st, lib.lorads_last_error(None).decode())
        self.h = h
        self.nprob = len(problems)
        self.problems = list(problems)

    # -- helpers -----------------------------------------------------------
    def _check(self, st):
        if st not in (LORADS_OK, LORADS_MAXITER, LORADS_TIMELIMIT):
            raise LoradsError(st, load().lorads_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            load().lorads_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- entry points ------------------------------------------------------
    def problem_info(self, prob: int = 0):
        s, n, m, f = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        self._check(load().lorads_problem_info(self.h, prob, C.byref(s), C.byref(n), C.byref(m)))
        self._check(load().lorads_problem_flags(self.h, prob, C.byref(f)))
        return dict(structure=STRUCT_NAMES[s.value], n=n.value, m=m.value,
                    c_dense=bool(f.value & LORADS_FLAG_DENSE_C))

    def apply_A(self, U, V, z, prob: int = 0, stream=None):
        """z = A(U V^T) on device tensors (n x r row-major, z of length m)."""
        r, ld = _factor_shape(U)
        self._check(load().lorads_apply_A(self.h, prob, _ptr(U), _ptr(V), r, ld, _ptr(z),
                                          _dtype_code(U), _stream(stream)))
        return z

    def apply_AT_V(self, w, V, out, c_scale: float = 1.0, prob: int = 0, stream=None):
        """out = (c_scale C + A*(w)) V on device tensors."""
        r, ld = _factor_shape(V)
        self._check(load().lorads_apply_AT_V(self.h, prob, _ptr(w), float(c_scale), _ptr(V), r, ld,
                                             _ptr(out), _dtype_code(V), _stream(stream)))
        return out

    def cg_solve(self, W, R, X, rho: float, gamma: float, tol: float, maxit: int, prob: int = 0,
                 stream=None):
        """Solve gamma X + rho A*(A(X W^T)) W = R by CG from the content of X."""
        r, ld = _factor_shape(W)
        it, rel = C.c_int32(), C.c_double()
        st = self._check(load().lorads_cg_solve(self.h, prob, _ptr(W), float(rho), float(gamma),
                                                _ptr(R), _ptr(X), r, ld, float(tol), int(maxit),
                                                _dtype_code(W), C.byref(it), C.byref(rel),
                                                _stream(stream)))
        return dict(status=st, iters=it.value, relres=rel.value)

    def cg_solve_noalloc(self, W, R, X, rho: float, gamma: float, tol: float, maxit: int,
                         prob: int = 0, stream=None):
        """cg_solve with the work buffers in the library's static workspace (no
        device allocation)."""
        r, ld = _factor_shape(W)
        it, rel = C.c_int32(), C.c_double()
        st = self._check(load().lorads_cg_solve_noalloc(self.h, prob, _ptr(W), float(rho), float(gamma),
                                                        _ptr(R), _ptr(X), r, ld, float(tol), int(maxit),
                                                        _dtype_code(W), C.byref(it), C.byref(rel),
                                                        _stream(stream)))
        return dict(status=st, iters=it.value, relres=rel.value)

    def admm_solve(self, init_U: Sequence[np.ndarray], options: Options_,
                   init_lambda: Optional[Sequence[Optional[np.ndarray]]] = None):
        """Two-phase LoRADS solve of every problem; returns a list of dicts."""
        lib = load()
        keep = [np.ascontiguousarray(u, dtype=np.float64) for u in init_U]
        ptrs = (C.c_void_p * self.nprob)(*[_ptr(u) for u in keep])
        options.init_U = C.cast(ptrs, C.c_void_p)
        ranks = (C.c_int32 * self.nprob)(*[int(u.shape[1]) for u in keep])
        options.init_rank = C.cast(ranks, C.c_void_p)
        if init_lambda is not None:
            keepl = [None if l is None else np.ascontiguousarray(l, dtype=np.float64) for l in init_lambda]
            lptrs = (C.c_void_p * self.nprob)(*[_ptr(l) if l is not None else 0 for l in keepl])
            options.init_lambda = C.cast(lptrs, C.c_void_p)
        else:
            options.init_lambda = None
        res = (Result_ * self.nprob)()
        st = lib.lorads_admm_solve(self.h, C.byref(options), res)
        options.init_U = None
        options.init_lambda = None
        options.init_rank = None
        if st < 0:
            raise LoradsError(st, lib.lorads_last_error(self.h).decode())
        out = []
        for i in range(self.nprob):
            d = {}
            for f, _ in Result_._fields_:
                v = getattr(res[i], f)
                d[f] = list(v) if f.startswith("prof_") else v
            out.append(d)
        return out

    def batch_autotune(self, init_U: Sequence[np.ndarray], options: Options_,
                       candidates: Sequence[int] = (64, 128, 192, 256)):
        """Time the batched launch per workgroup size; the context keeps the
        fastest.  Returns (best, {size: ms})."""
        lib = load()
        keep = [np.ascontiguousarray(u, dtype=np.float64) for u in init_U]
        ptrs = (C.c_void_p * self.nprob)(*[_ptr(u) for u in keep])
        options.init_U = C.cast(ptrs, C.c_void_p)
        options.init_lambda = None
        ranks = (C.c_int32 * self.nprob)(*[int(u.shape[1]) for u in keep])
        options.init_rank = C.cast(ranks, C.c_void_p)
        cand = (C.c_int32 * len(candidates))(*candidates)
        times = (C.c_double * len(candidates))()
        best = C.c_int32()
        st = lib.lorads_batch_autotune(self.h, C.byref(options), cand, len(candidates), C.byref(best), times)
        options.init_U = None
        options.init_rank = None
        self._check(st)
        return best.value, {int(c): float(t) for c, t in zip(candidates, times)}

    def get_solution(self, prob: int = 0, rank: Optional[int] = None):
        info = self.problem_info(prob)
        if rank is None:
            raise ValueError("rank required (take it from the solve result)")
        n, m = info["n"], info["m"]
        U = np.empty((n, rank)); V = np.empty((n, rank)); lam = np.empty(m)
        self._check(load().lorads_get_solution(self.h, prob, _ptr(U), _ptr(V), _ptr(lam)))
        return U, V, lam

    def dual_lambda_min(self, lam, prob: int = 0, max_steps: int = 300) -> float:
        out = C.c_double()
        self._check(load().lorads_dual_lambda_min(self.h, prob, _ptr(lam), int(max_steps), C.byref(out)))
        return out.value


def gram(A, B, G, stream=None):
    """G = A^T B for FP64 device tensors A (n x ra), B (n x rb), G (ra x rb)."""
    ra, lda = _factor_shape(A)
    rb, ldb = _factor_shape(B)
    st = load().lorads_gram(_ptr(A), _ptr(B), int(A.shape[0]), ra, rb, lda, ldb, _ptr(G), _stream(stream))
    if st != LORADS_OK:
        raise LoradsError(st, load().lorads_last_error(None).decode())
    return G


def version() -> str:
    return load().lorads_version().decode()


def _gcheck(st: int):
    if st != LORADS_OK:
        raise LoradsError(st, load().lorads_last_error(None).decode())


class Gnn:
    """Owns a lorads_gnn: the warm-start network, its parameters, Adam state and
    a resident graph set (host numpy arrays in, host numpy arrays out)."""

    def __init__(self, layers: int = 3):
        lib = load()
        h = C.c_void_p()
        _gcheck(lib.lorads_gnn_create(int(layers), C.byref(h)))
        self._h = h
        self.layers = int(layers)
        self.n_params = int(lib.lorads_gnn_param_count(int(layers)))
        self.node_off = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lorads_gnn_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        _gcheck(load().lorads_gnn_set_params(self._h, _ptr(t), t.size))

    def get_params(self) -> np.ndarray:
        t = np.empty(self.n_params, dtype=np.float32)
        _gcheck(load().lorads_gnn_get_params(self._h, _ptr(t), t.size))
        return t

    def load_graphs(self, node_off, row, col, w):
        no = np.ascontiguousarray(node_off, dtype=np.int64)
        r = np.ascontiguousarray(row, dtype=np.int32)
        c = np.ascontiguousarray(col, dtype=np.int32)
        ww = np.ascontiguousarray(w, dtype=np.float32)
        _gcheck(load().lorads_gnn_load_graphs(self._h, len(no) - 1, _ptr(no), r.size, _ptr(r),
                                              _ptr(c), _ptr(ww)))
        self.node_off = no

    def set_targets(self, y, r):
        yy = np.ascontiguousarray(y, dtype=np.float32)
        rr = np.ascontiguousarray(r, dtype=np.float32)
        if yy.size != self.node_off[-1] or rr.size != len(self.node_off) - 1:
            raise ValueError("target sizes do not match the graph set")
        _gcheck(load().lorads_gnn_set_targets(self._h, _ptr(yy), _ptr(rr)))

    def forward(self, g0: int, g1: int):
        yh = np.empty(int(self.node_off[g1] - self.node_off[g0]), dtype=np.float32)
        rh = np.empty(g1 - g0, dtype=np.float32)
        _gcheck(load().lorads_gnn_forward(self._h, g0, g1, _ptr(yh), _ptr(rh)))
        return yh, rh

    def loss_grad(self, g0: int, g1: int, omega: float, want_grad: bool = True):
        loss = C.c_double()
        grad = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        _gcheck(load().lorads_gnn_loss_grad(self._h, g0, g1, float(omega), C.byref(loss),
                                            _ptr(grad), self.n_params if want_grad else 0))
        return loss.value, grad

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _gcheck(load().lorads_gnn_adam_step(self._h, lr, beta1, beta2, eps))

    def layer_time(self):
        ms, n, fl = C.c_double(), C.c_int64(), C.c_double()
        _gcheck(load().lorads_gnn_layer_time(self._h, C.byref(ms), C.byref(n), C.byref(fl)))
        return ms.value, n.value, fl.value
