"""Python binding of the fmmbem C ABI (include/fmmbem.h): argument marshalling only.

Every computation runs in the HIP library libfmmbem.so; if it is missing this module raises
instead of falling back to anything else.  Function names mirror the C entry points.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmmbem.so")

FMMBEM_OK, FMMBEM_ENOCONV = 0, 1
FMMBEM_EINVAL, FMMBEM_ENOMEM, FMMBEM_EDEVICE, FMMBEM_ENOTREADY, FMMBEM_EBREAKDOWN, FMMBEM_ENAN = -1, -2, -3, -4, -5, -6
FMMBEM_DIRECT, FMMBEM_DIRECT_DPSI, FMMBEM_DIRECT_BM, FMMBEM_INDIRECT = 0, 1, 2, 3
FMMBEM_FP64, FMMBEM_MIXED = 0, 1
FMMBEM_PC_NONE, FMMBEM_PC_DIAG, FMMBEM_PC_NEARBLOCK, FMMBEM_PC_LEARNED = 0, 1, 2, 3


class FmmbemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fmmbem error {code}: {msg}")
        self.code = code


class c64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("rc_factor", ctypes.c_double), ("rc", ctypes.c_double), ("leaf_max", ctypes.c_int),
                ("p_min", ctypes.c_int), ("p_excess", ctypes.c_double), ("ktau_switch", ctypes.c_double),
                ("max_depth", ctypes.c_int), ("lds_budget", ctypes.c_int), ("graphs", ctypes.c_int),
                ("autotune", ctypes.c_int), ("lane_tiles", ctypes.c_int), ("streams", ctypes.c_int),
                ("mfma", ctypes.c_int), ("fused", ctypes.c_int), ("kd_leaf_min", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("precond", ctypes.c_int), ("precision", ctypes.c_int), ("diag_shift", ctypes.c_double),
                ("use_x0", ctypes.c_int), ("inner_iters", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("inner_precision", ctypes.c_int), ("basis_fp32", ctypes.c_int), ("inner_p_min", ctypes.c_int),
                ("inner_p_excess", ctypes.c_double), ("reorth", ctypes.c_int)]


class SolveReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("t_setup_s", ctypes.c_double), ("t_solve_s", ctypes.c_double), ("status", ctypes.c_int),
                ("matvecs_fp64", ctypes.c_int64), ("matvecs_mixed", ctypes.c_int64), ("inner_iters", ctypes.c_int64),
                ("pc_fallback_at", ctypes.c_int32), ("matvecs_coarse", ctypes.c_int64)]


class BatchShape(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("kind", ctypes.c_int32), ("lane", ctypes.c_int32),
                ("whole", ctypes.c_int32), ("jt", ctypes.c_int32), ("mfma", ctypes.c_int32), ("jobs", ctypes.c_int64),
                ("ms", ctypes.c_double)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_pairs", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class TrainReport(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int64), ("pairs", ctypes.c_int32), ("solve_iters", ctypes.c_int32),
                ("solve_rel_res", ctypes.c_double), ("loss_zero", ctypes.c_double), ("loss_first", ctypes.c_double),
                ("loss_last", ctypes.c_double), ("t_data_s", ctypes.c_double), ("t_train_s", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rc", ctypes.c_double), ("root_side", ctypes.c_double),
                ("root_lo", ctypes.c_double * 3), ("depth", ctypes.c_int), ("nleaf", ctypes.c_int64),
                ("leaf_max_occ", ctypes.c_int), ("near_nnz", ctypes.c_int64), ("p2p_pairs", ctypes.c_int64),
                ("p", ctypes.c_int * 24), ("nbox", ctypes.c_int64 * 24), ("m2l_pairs", ctypes.c_int64 * 24),
                ("flops_m2l", ctypes.c_double), ("flops_m2m_l2l", ctypes.c_double),
                ("flops_p2m_l2p", ctypes.c_double), ("bytes_p2p", ctypes.c_double), ("lds_max", ctypes.c_int64)]


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


EXPORTS = {
    "fmmbem_default_options": (None, [ctypes.POINTER(Options)]),
    "fmmbem_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(Options)]),
    "fmmbem_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "fmmbem_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "fmmbem_set_mesh": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "fmmbem_set_wavenumber": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "fmmbem_set_admittance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_set_sources": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_set_formulation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fmmbem_setup": (ctypes.c_int, [ctypes.c_void_p]),
    "fmmbem_num_unknowns": (ctypes.c_int64, [ctypes.c_void_p]),
    "fmmbem_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_rhs_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_solve_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(SolveOpts), ctypes.c_void_p,
                                        ctypes.POINTER(SolveReport), ctypes.c_void_p]),
    "fmmbem_eval_field_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_eval_field_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_solve_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(SolveOpts),
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_release_workspace": (ctypes.c_int, [ctypes.c_void_p]),
    "fmmbem_batch_shapes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_int32)]),
    "fmmbem_set_batch_shapes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "fmmbem_solve_many": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "fmmbem_near_entries_n": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "fmmbem_default_train_opts": (None, [ctypes.c_void_p]),
    "fmmbem_learned_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_mlp_param_count": (ctypes.c_int64, []),
    "fmmbem_mlp_init": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "fmmbem_mlp_get_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_mlp_set_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_mlp_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_solve_history": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_int32)]),
    "fmmbem_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "fmmbem_matvec_dev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "fmmbem_default_solve_opts": (None, [ctypes.POINTER(SolveOpts)]),
    "fmmbem_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(SolveOpts), ctypes.c_void_p, ctypes.POINTER(SolveReport)]),
    "fmmbem_eval_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "fmmbem_near_entries": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_coaxial_table": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "fmmbem_rotation_table": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "fmmbem_last_timings": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fmmbem_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fmmbem_kernel_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FmmbemError(FMMBEM_EDEVICE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # PyTorch (device memory and streams for the *_dev entry points) ships its own HIP
        # runtime; it has to come up before this library's runtime touches the device, or it
        # finds no GPU afterwards.
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _c(a):
    return np.ascontiguousarray(a, np.complex128)


def default_options() -> Options:
    o = Options()
    lib().fmmbem_default_options(ctypes.byref(o))
    return o


def default_solve_opts() -> SolveOpts:
    o = SolveOpts()
    lib().fmmbem_default_solve_opts(ctypes.byref(o))
    return o


class Context:
    """One fmmbem context (one HIP device).  Methods map 1:1 onto the C calls."""

    def __init__(self, device: int = 0, options: Options | None = None, **opt):
        if options is None:
            options = default_options()
        for k, v in opt.items():
            setattr(options, k, v)
        h = ctypes.c_void_p()
        self._check(lib().fmmbem_create(ctypes.byref(h), device, ctypes.byref(options)), h)
        self.h = h
        self._n = 0

    def _check(self, rc, h=None):
        if rc < 0:
            msg = lib().fmmbem_last_error(h if h is not None else self.h)
            raise FmmbemError(rc, msg.decode() if msg else "")
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().fmmbem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inputs
    def fmmbem_set_mesh(self, V, T):
        V = np.ascontiguousarray(V, np.float64)
        T = np.ascontiguousarray(T, np.int64)
        self._check(lib().fmmbem_set_mesh(self.h, V.shape[0], _ptr(V), T.shape[0], _ptr(T)))
        self._n = T.shape[0]

    def fmmbem_set_wavenumber(self, k):
        self._check(lib().fmmbem_set_wavenumber(self.h, float(k)))

    def fmmbem_set_admittance(self, beta, beta_plus=None):
        b = _c(beta)
        bp = None if beta_plus is None else _c(beta_plus)
        self._check(lib().fmmbem_set_admittance(self.h, _ptr(b), None if bp is None else _ptr(bp)))

    def fmmbem_set_sources(self, rs, amp=None):
        rs = np.ascontiguousarray(np.atleast_2d(rs), np.float64)
        a = None if amp is None else _c(amp)
        self._check(lib().fmmbem_set_sources(self.h, rs.shape[0], _ptr(rs), None if a is None else _ptr(a)))
        self._ns = rs.shape[0]

    def fmmbem_set_formulation(self, f):
        self._check(lib().fmmbem_set_formulation(self.h, int(f)))

    def fmmbem_setup(self):
        self._check(lib().fmmbem_setup(self.h))

    def fmmbem_num_unknowns(self):
        return int(lib().fmmbem_num_unknowns(self.h))

    # ---- products and solve
    def fmmbem_rhs(self):
        n = self.fmmbem_num_unknowns()
        b = np.empty((self._ns, n), np.complex128)
        self._check(lib().fmmbem_rhs(self.h, _ptr(b)))
        return b

    def fmmbem_matvec(self, x, precision=FMMBEM_FP64, exact_far=False):
        x = _c(np.atleast_2d(x))
        y = np.empty_like(x)
        self._check(lib().fmmbem_matvec(self.h, x.shape[0], _ptr(x), _ptr(y), int(precision), int(bool(exact_far))))
        return y

    def fmmbem_matvec_dev(self, x_ptr: int, y_ptr: int, nrhs=1, precision=FMMBEM_FP64, stream: int = 0):
        self._check(lib().fmmbem_matvec_dev(self.h, nrhs, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr),
                                            int(precision), ctypes.c_void_p(stream)))

    def fmmbem_rhs_dev(self, b_ptr: int, stream: int = 0):
        self._check(lib().fmmbem_rhs_dev(self.h, ctypes.c_void_p(b_ptr), ctypes.c_void_p(stream)))

    def fmmbem_solve_dev(self, isrc, x_ptr: int, use_x0=False, stream: int = 0, **kw):
        o = default_solve_opts()
        for k, v in kw.items():
            setattr(o, k, v)
        o.use_x0 = int(bool(use_x0))
        rep = SolveReport()
        rc = self._check(lib().fmmbem_solve_dev(self.h, isrc, ctypes.byref(o), ctypes.c_void_p(x_ptr),
                                                ctypes.byref(rep), ctypes.c_void_p(stream)))
        return rep, rc

    def fmmbem_eval_field_dev(self, isrc, nr, r_ptr: int, x_ptr: int, psi_ptr: int, stream: int = 0):
        self._check(lib().fmmbem_eval_field_dev(self.h, isrc, int(nr), ctypes.c_void_p(r_ptr), ctypes.c_void_p(x_ptr),
                                                ctypes.c_void_p(psi_ptr), ctypes.c_void_p(stream)))

    def fmmbem_eval_field_noalloc(self, isrc, nr, r_ptr: int, x_ptr: int, psi_ptr: int, stream: int = 0):
        self._check(lib().fmmbem_eval_field_noalloc(self.h, isrc, int(nr), ctypes.c_void_p(r_ptr),
                                                    ctypes.c_void_p(x_ptr), ctypes.c_void_p(psi_ptr),
                                                    ctypes.c_void_p(stream)))

    def fmmbem_solve(self, isrc=0, x0=None, **kw):
        o = default_solve_opts()
        for k, v in kw.items():
            setattr(o, k, v)
        n = self.fmmbem_num_unknowns()
        x = np.zeros(n, np.complex128) if x0 is None else _c(x0).copy()
        if x0 is not None:
            o.use_x0 = 1
        rep = SolveReport()
        rc = self._check(lib().fmmbem_solve(self.h, isrc, ctypes.byref(o), _ptr(x), ctypes.byref(rep)))
        return x, rep, rc

    def fmmbem_solve_batch(self, isrc, x0=None, **kw):
        o = default_solve_opts()
        for k, v in kw.items():
            setattr(o, k, v)
        n = self.fmmbem_num_unknowns()
        src = np.ascontiguousarray(isrc, np.int32)
        ns = src.shape[0]
        x = np.zeros((ns, n), np.complex128) if x0 is None else _c(x0).reshape(ns, n).copy()
        if x0 is not None:
            o.use_x0 = 1
        reps = (SolveReport * ns)()
        rc = self._check(lib().fmmbem_solve_batch(self.h, ns, _ptr(src), ctypes.byref(o), _ptr(x), reps))
        return x, list(reps), rc

    # ---- learned preconditioner
    def fmmbem_learned_train(self, isrc=0, **kw):
        o = TrainOpts()
        lib().fmmbem_default_train_opts(ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        rep = TrainReport()
        self._check(lib().fmmbem_learned_train(self.h, isrc, ctypes.byref(o), ctypes.byref(rep)))
        return rep

    @staticmethod
    def fmmbem_mlp_param_count():
        return int(lib().fmmbem_mlp_param_count())

    def fmmbem_mlp_init(self, seed=1):
        self._check(lib().fmmbem_mlp_init(self.h, seed))

    def fmmbem_mlp_get_weights(self):
        w = np.empty(self.fmmbem_mlp_param_count(), np.float32)
        self._check(lib().fmmbem_mlp_get_weights(self.h, _ptr(w)))
        return w

    def fmmbem_mlp_set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        assert w.shape == (self.fmmbem_mlp_param_count(),)
        self._check(lib().fmmbem_mlp_set_weights(self.h, _ptr(w)))

    def fmmbem_mlp_forward(self, X):
        X = np.ascontiguousarray(X, np.float32)
        Y = np.empty((X.shape[0], 128), np.float32)
        self._check(lib().fmmbem_mlp_forward(self.h, X.shape[0], _ptr(X), _ptr(Y)))
        return Y

    def fmmbem_mlp_loss_grad(self, X, T):
        X = np.ascontiguousarray(X, np.float32)
        T = np.ascontiguousarray(T, np.float32)
        loss = np.zeros(1, np.float32)
        g = np.empty(self.fmmbem_mlp_param_count(), np.float32)
        self._check(lib().fmmbem_mlp_loss_grad(self.h, X.shape[0], _ptr(X), _ptr(T), _ptr(loss), _ptr(g)))
        return float(loss[0]), g

    def fmmbem_near_entries_n(self):
        nnz = ctypes.c_int64()
        self._check(lib().fmmbem_near_entries_n(self.h, ctypes.byref(nnz), None, None))
        Lp = np.empty(nnz.value, np.complex128)
        Mp = np.empty(nnz.value, np.complex128)
        self._check(lib().fmmbem_near_entries_n(self.h, ctypes.byref(nnz), _ptr(Lp), _ptr(Mp)))
        return Lp, Mp

    def fmmbem_batch_shapes(self):
        cnt = ctypes.c_int32()
        self._check(lib().fmmbem_batch_shapes(self.h, 0, None, ctypes.byref(cnt)))
        arr = (BatchShape * max(1, cnt.value))()
        self._check(lib().fmmbem_batch_shapes(self.h, cnt.value, arr, ctypes.byref(cnt)))
        return [{"level": s.level, "kind": ("m2l", "m2m", "l2l")[s.kind], "lane": s.lane, "whole": s.whole,
                 "jt": s.jt, "mfma": s.mfma, "jobs": s.jobs, "ms": s.ms} for s in arr[:cnt.value]]

    def fmmbem_set_batch_shapes(self, shapes):
        """shapes: dicts as returned by fmmbem_batch_shapes (level, kind, lane, whole, jt, mfma)."""
        kinds = {"m2l": 0, "m2m": 1, "l2l": 2}
        arr = (BatchShape * max(1, len(shapes)))()
        for q, d in enumerate(shapes):
            kind = kinds[d["kind"]] if isinstance(d["kind"], str) else int(d["kind"])
            arr[q] = BatchShape(d["level"], kind, d["lane"], d["whole"], d["jt"], d["mfma"], d.get("jobs", 0), 0.0)
        self._check(lib().fmmbem_set_batch_shapes(self.h, len(shapes), arr))

    def fmmbem_release_workspace(self):
        self._check(lib().fmmbem_release_workspace(self.h))

    def fmmbem_solve_history(self):
        cnt = ctypes.c_int32()
        self._check(lib().fmmbem_solve_history(self.h, 0, None, ctypes.byref(cnt)))
        out = np.empty(cnt.value, np.float64)
        self._check(lib().fmmbem_solve_history(self.h, cnt.value, _ptr(out), ctypes.byref(cnt)))
        return out

    def fmmbem_eval_field(self, isrc, pts, x):
        pts = np.ascontiguousarray(np.atleast_2d(pts), np.float64)
        x = _c(x)
        out = np.empty(pts.shape[0], np.complex128)
        self._check(lib().fmmbem_eval_field(self.h, isrc, pts.shape[0], _ptr(pts), _ptr(x), _ptr(out)))
        return out

    # ---- inspection
    def fmmbem_get_info(self) -> Info:
        info = Info()
        self._check(lib().fmmbem_get_info(self.h, ctypes.byref(info)))
        return info

    def fmmbem_near_entries(self):
        nnz = ctypes.c_int64()
        self._check(lib().fmmbem_near_entries(self.h, ctypes.byref(nnz), None, None, None, None))
        z = nnz.value
        r = np.empty(z, np.int64)
        c = np.empty(z, np.int64)
        L = np.empty(z, np.complex128)
        M = np.empty(z, np.complex128)
        self._check(lib().fmmbem_near_entries(self.h, ctypes.byref(nnz), _ptr(r), _ptr(c), _ptr(L), _ptr(M)))
        return r, c, L, M

    def fmmbem_profile(self, enable=True):
        self._check(lib().fmmbem_profile(self.h, int(bool(enable))))

    def fmmbem_kernel_stats(self):
        arr = (KStat * 128)()
        cnt = ctypes.c_int()
        self._check(lib().fmmbem_kernel_stats(self.h, 128, arr, ctypes.byref(cnt)))
        return [dict(name=arr[i].name.decode(), launches=arr[i].launches, ms=arr[i].ms, flops=arr[i].flops,
                     bytes=arr[i].bytes) for i in range(cnt.value)]

    def fmmbem_last_timings(self):
        t = np.zeros(8)
        self._check(lib().fmmbem_last_timings(self.h, _ptr(t)))
        return t


def fmmbem_solve_many(ctxs, isrc, threads=0, **kw):
    """Solve source isrc[i] of context ctxs[i] for every i, all systems in flight together from the
    calling thread (systems of one context in lock step with batched products).  Returns
    (solutions, reports, per-system codes, overall code)."""
    count = len(ctxs)
    o = default_solve_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    opts = (SolveOpts * max(1, count))(*([o] * count))
    hs = (ctypes.c_void_p * max(1, count))(*[c.h.value for c in ctxs])
    src = np.ascontiguousarray(isrc, np.int32)
    xs = [np.zeros(c.fmmbem_num_unknowns(), np.complex128) for c in ctxs]
    xp = (ctypes.c_void_p * max(1, count))(*[x.ctypes.data for x in xs])
    reps = (SolveReport * max(1, count))()
    status = np.zeros(max(1, count), np.int32)
    rc = lib().fmmbem_solve_many(count, hs, _ptr(src), opts, xp, reps, _ptr(status), int(threads))
    if rc < 0:
        msgs = [lib().fmmbem_last_error(c.h) for c, st in zip(ctxs, status[:count]) if st < 0]
        raise FmmbemError(rc, "; ".join(m.decode() for m in msgs if m) or "bad arguments")
    return xs, list(reps[:count]), status[:count].tolist(), rc


def fmmbem_coaxial_table(kind, ktau, p, method=-1, device=0):
    """Blocks m = 0..p-1 as a list of (p-m)x(p-m) complex arrays (rows n', cols n)."""
    from math import prod  # noqa: F401
    size = sum((p - m) ** 2 for m in range(p))
    out = np.empty(size, np.complex128)
    rc = lib().fmmbem_coaxial_table(device, int(kind), float(ktau), int(p), int(method), _ptr(out))
    if rc != 0:
        raise FmmbemError(rc, "coaxial table")
    blocks, off = [], 0
    for m in range(p):
        b = p - m
        blocks.append(out[off:off + b * b].reshape(b, b))
        off += b * b
    return blocks


def fmmbem_rotation_table(p, device=0):
    """List of Delta^n (2n+1)x(2n+1) for n < p."""
    size = sum((2 * n + 1) ** 2 for n in range(p))
    out = np.empty(size, np.float64)
    rc = lib().fmmbem_rotation_table(device, int(p), _ptr(out))
    if rc != 0:
        raise FmmbemError(rc, "rotation table")
    blocks, off = [], 0
    for n in range(p):
        w = 2 * n + 1
        blocks.append(out[off:off + w * w].reshape(w, w))
        off += w * w
    return blocks
