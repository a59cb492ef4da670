"""Thin ctypes binding of libfmmlm.so (include/fmmlm.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream; the binding
raises when the library is missing, and has no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmmlm.so")

FMMLM_FP64 = 0
FMMLM_FP32_COMPENSATED = 1
FREE = 1
REACTION = 2

_ERRORS = {
    -1: ValueError, -2: ValueError, -3: ValueError, -4: ValueError, -5: ValueError,
    -6: RuntimeError, -7: MemoryError, -8: NotImplementedError, -9: RuntimeError,
}


class Opts(ctypes.Structure):
    _fields_ = [("leaf_cap", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("fp64_top_levels", ctypes.c_int32), ("max_rhs", ctypes.c_int32),
                ("mac_d2", ctypes.c_int32), ("graph", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2),
                ("surrogate", ctypes.c_void_p)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("nsamples", ctypes.c_int64), ("steps", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("lr", ctypes.c_double), ("seed", ctypes.c_uint64), ("reserved", ctypes.c_int32 * 4)]


class TrainReport(ctypes.Structure):
    _fields_ = [("n_train", ctypes.c_int64), ("n_val", ctypes.c_int64), ("n_params", ctypes.c_int64),
                ("n_components", ctypes.c_int32), ("n_outputs", ctypes.c_int32),
                ("sample_seconds", ctypes.c_double), ("train_seconds", ctypes.c_double),
                ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("val_rms", ctypes.c_double), ("val_max", ctypes.c_double),
                ("yscale", ctypes.c_double), ("ladder_fit", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("tol", ctypes.c_double),
                ("zero_guess", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("matvecs", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("relres", ctypes.c_double), ("relres_est", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_tree_points", ctypes.c_int64),
                ("n_trees", ctypes.c_int32), ("p", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("n_boxes", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("m2l_free_pairs", ctypes.c_int64),
                ("m2l_reaction_pairs", ctypes.c_int64), ("p2p_free_pairs", ctypes.c_int64),
                ("p2p_reaction_pairs", ctypes.c_int64), ("n_free_ops", ctypes.c_int64),
                ("n_reaction_ops", ctypes.c_int64), ("n_sommerfeld_tasks", ctypes.c_int64),
                ("root_side", ctypes.c_double), ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("plan_seconds", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("tree_seconds", ctypes.c_double), ("lists_seconds", ctypes.c_double),
                ("ops_seconds", ctypes.c_double), ("table_seconds", ctypes.c_double),
                ("nearfield_seconds", ctypes.c_double), ("surrogate_tasks", ctypes.c_int64),
                ("surrogate_pairs", ctypes.c_int64), ("surrogate_check", ctypes.c_double),
                ("m2l_steps", ctypes.c_int64), ("m2l_tile_cols", ctypes.c_int32),
                ("m2l_variant", ctypes.c_int32), ("m2l_top_pairs", ctypes.c_int64),
                ("m2l_variant_ms", ctypes.c_double * 6), ("batch_variant", ctypes.c_int32),
                ("surrogate_rejected", ctypes.c_int32), ("batch_variant_ms", ctypes.c_double * 10),
                ("m2l_eval_ms", ctypes.c_double * 6), ("p2p_split_ms", ctypes.c_double * 5),
                ("p2p_split_pct", ctypes.c_int32), ("batch_min_rhs", ctypes.c_int32),
                ("p2p_lds_reserve", ctypes.c_int32), ("p2p_reserve_ms", ctypes.c_double * 3),
                ("m2l_chunks", ctypes.c_int64)]


EXPORTS = ["fmmlm_default_opts", "fmm_layered_plan", "fmm_layered_eval", "fmm_layered_destroy",
           "fmm_layered_strerror", "fmm_layered_plan_stats", "fmm_layered_plan_tree",
           "fmm_layered_sommerfeld", "fmm_layered_density", "fmm_layered_profile_begin",
           "fmm_layered_profile_end", "fmm_layered_density_asymptotic",
           "fmmlm_default_train_opts", "fmm_layered_surrogate_create",
           "fmm_layered_surrogate_create_for_plan", "fmm_layered_surrogate_train",
           "fmm_layered_surrogate_destroy", "fmm_layered_surrogate_params",
           "fmm_layered_surrogate_grad", "fmm_layered_surrogate_eval",
           "fmm_layered_surrogate_samples", "fmm_layered_plan_set_variants", "fmm_layered_solve",
           "fmm_layered_plan_general", "fmm_layered_sommerfeld_noalloc",
           "fmm_layered_surrogate_forward", "fmm_layered_surrogate_adam", "fmm_layered_plan_lists",
           "fmm_layered_tables_create", "fmm_layered_tables_create_for_plan", "fmm_layered_tables_info",
           "fmm_layered_interp2d"]
STAGES = ["gather", "p2m", "m2m", "m2l_top", "m2l", "m2l_reduce", "l2l", "l2p", "p2p_free", "p2p_reaction",
          "combine"]

_lib = None


def lib():
    """Load libfmmlm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    # torch brings its own HIP runtime: load it first so that the library and
    # torch share one runtime (and one device context) in this process
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    L.fmmlm_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.fmmlm_default_opts.restype = None
    L.fmm_layered_plan.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int64, vp, vp, vp, vp,
                                   ctypes.c_int32, ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
    L.fmm_layered_plan.restype = ctypes.c_int
    L.fmm_layered_eval.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int64, vp, ctypes.c_int64,
                                   ctypes.c_uint32, vp]
    L.fmm_layered_eval.restype = ctypes.c_int
    L.fmm_layered_plan_general.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int64, vp, vp, vp, vp,
                                           ctypes.c_int32, ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
    L.fmm_layered_plan_general.restype = ctypes.c_int
    L.fmm_layered_solve.argtypes = [vp, vp, vp, vp, ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveInfo)]
    L.fmm_layered_solve.restype = ctypes.c_int
    L.fmm_layered_destroy.argtypes = [vp]
    L.fmm_layered_destroy.restype = ctypes.c_int
    L.fmm_layered_strerror.argtypes = [ctypes.c_int]
    L.fmm_layered_strerror.restype = ctypes.c_char_p
    L.fmm_layered_plan_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.fmm_layered_plan_stats.restype = ctypes.c_int
    L.fmm_layered_plan_tree.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int64), vp, vp]
    L.fmm_layered_plan_tree.restype = ctypes.c_int
    L.fmm_layered_plan_lists.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), vp]
    L.fmm_layered_plan_lists.restype = ctypes.c_int
    L.fmm_layered_sommerfeld.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_int64, vp, vp, ctypes.c_int32, vp, vp]
    L.fmm_layered_sommerfeld.restype = ctypes.c_int
    L.fmm_layered_sommerfeld_noalloc.argtypes = L.fmm_layered_sommerfeld.argtypes
    L.fmm_layered_sommerfeld_noalloc.restype = ctypes.c_int
    L.fmm_layered_density.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, vp, vp, vp,
                                      vp, vp]
    L.fmm_layered_density.restype = ctypes.c_int
    L.fmm_layered_density_asymptotic.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32,
                                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                  dp, dp]
    L.fmm_layered_density_asymptotic.restype = ctypes.c_int
    L.fmmlm_default_train_opts.argtypes = [ctypes.POINTER(TrainOpts)]
    L.fmmlm_default_train_opts.restype = None
    L.fmm_layered_surrogate_create.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(vp)]
    L.fmm_layered_surrogate_create.restype = ctypes.c_int
    L.fmm_layered_surrogate_create_for_plan.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp)]
    L.fmm_layered_surrogate_create_for_plan.restype = ctypes.c_int
    L.fmm_layered_surrogate_train.argtypes = [vp, ctypes.POINTER(TrainOpts), vp, ctypes.POINTER(TrainReport)]
    L.fmm_layered_surrogate_train.restype = ctypes.c_int
    L.fmm_layered_surrogate_destroy.argtypes = [vp]
    L.fmm_layered_surrogate_destroy.restype = ctypes.c_int
    L.fmm_layered_surrogate_params.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_int64)]
    L.fmm_layered_surrogate_params.restype = ctypes.c_int
    L.fmm_layered_surrogate_grad.argtypes = [vp, ctypes.c_int64, vp, vp, vp, dp, vp, vp]
    L.fmm_layered_surrogate_grad.restype = ctypes.c_int
    L.fmm_layered_surrogate_eval.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_double, ctypes.c_int64, vp, vp,
                                             ctypes.c_int32, vp, vp, vp]
    L.fmm_layered_surrogate_eval.restype = ctypes.c_int
    L.fmm_layered_surrogate_samples.argtypes = [vp, ctypes.c_int64, ctypes.c_uint64, vp, vp, vp, vp, vp, vp]
    L.fmm_layered_surrogate_samples.restype = ctypes.c_int
    L.fmm_layered_tables_create.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_double,
                                            ctypes.c_double, vp, ctypes.POINTER(vp)]
    L.fmm_layered_tables_create.restype = ctypes.c_int
    L.fmm_layered_tables_create_for_plan.argtypes = [vp, vp, ctypes.POINTER(vp)]
    L.fmm_layered_tables_create_for_plan.restype = ctypes.c_int
    L.fmm_layered_tables_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    L.fmm_layered_tables_info.restype = ctypes.c_int
    L.fmm_layered_interp2d.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int32, vp, ctypes.c_int64, vp, vp, vp, vp]
    L.fmm_layered_interp2d.restype = ctypes.c_int
    L.fmm_layered_surrogate_forward.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp]
    L.fmm_layered_surrogate_forward.restype = ctypes.c_int
    L.fmm_layered_surrogate_adam.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp]
    L.fmm_layered_surrogate_adam.restype = ctypes.c_int
    L.fmm_layered_plan_set_variants.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.fmm_layered_plan_set_variants.restype = ctypes.c_int
    L.fmm_layered_profile_begin.argtypes = [vp, ctypes.c_int32]
    L.fmm_layered_profile_begin.restype = ctypes.c_int
    L.fmm_layered_profile_end.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64)]
    L.fmm_layered_profile_end.restype = ctypes.c_int
    _lib = L
    return L


def check(rc: int):
    if rc != 0:
        msg = lib().fmm_layered_strerror(rc).decode()
        raise _ERRORS.get(rc, RuntimeError)(f"fmmlm error {rc}: {msg}")


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """fmm_layered_plan over host geometry; eval on torch CUDA tensors.

    interface_a: the a coefficients of the general interface conditions
    (fmm_layered_plan_general); eps then holds the b coefficients."""

    def __init__(self, d, eps, x, y, z, layer, p, leaf_cap=64, precision=FMMLM_FP64,
                 fp64_top_levels=3, max_rhs=1, mac_d2=None, stream=None, surrogate=None, graph=False,
                 interface_a=None):
        self.d = _host(d, np.float64)
        self.eps = _host(eps, np.float64)
        x, y, z = _host(x, np.float64), _host(y, np.float64), _host(z, np.float64)
        layer = _host(layer, np.int32)
        self.n = len(x)
        o = Opts()
        lib().fmmlm_default_opts(ctypes.byref(o))
        o.leaf_cap = leaf_cap
        o.precision = precision
        o.fp64_top_levels = fp64_top_levels
        o.max_rhs = max_rhs
        if mac_d2 is not None:
            o.mac_d2 = mac_d2
        if surrogate is not None:
            o.surrogate = surrogate._h
        o.graph = 1 if graph else 0
        h = ctypes.c_void_p()
        if interface_a is None:
            rc = lib().fmm_layered_plan(len(self.d), _ptr(self.d), _ptr(self.eps), self.n, _ptr(x),
                                        _ptr(y), _ptr(z), _ptr(layer), p, ctypes.byref(o),
                                        _stream_handle(stream), ctypes.byref(h))
        else:
            self.a = _host(interface_a, np.float64)
            if len(self.a) != len(self.eps):
                raise ValueError("interface_a needs one coefficient per layer")
            rc = lib().fmm_layered_plan_general(len(self.d), _ptr(self.d), _ptr(self.a), _ptr(self.eps),
                                                self.n, _ptr(x), _ptr(y), _ptr(z), _ptr(layer), p,
                                                ctypes.byref(o), _stream_handle(stream), ctypes.byref(h))
        check(rc)
        self._h = h
        self.p = p

    def eval(self, q, parts=FREE | REACTION, out=None, stream=None):
        """q: CUDA float64 tensor [n] or [nrhs, n] (user order) -> phi of the same shape."""
        import torch
        if not (q.is_cuda and q.dtype == torch.float64):
            raise ValueError("q must be a CUDA float64 tensor")
        q2 = q.reshape(-1, q.shape[-1]).contiguous()
        if q2.shape[1] != self.n:
            raise ValueError("q has the wrong length")
        if out is None:
            out = torch.empty_like(q2)
        rc = lib().fmm_layered_eval(self._h, q2.shape[0], ctypes.c_void_p(q2.data_ptr()), self.n,
                                    ctypes.c_void_p(out.data_ptr()), self.n, parts,
                                    _stream_handle(stream))
        check(rc)
        return out.reshape(q.shape)

    def solve(self, b, diag=None, x0=None, tol=1e-6, restart=30, max_iters=300, stream=None):
        """GMRES for (diag(diag) + G) x = b with G this plan's matvec
        (fmm_layered_solve).  b, diag, x0: CUDA float64 tensors [n] (user order);
        x0 None starts from zero.  Returns (x, info dict)."""
        import torch
        for name, t in (("b", b), ("diag", diag), ("x0", x0)):
            if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.numel() == self.n):
                raise ValueError(f"{name} must be a CUDA float64 tensor of length n")
        b = b.contiguous()
        x = torch.zeros_like(b) if x0 is None else x0.clone().contiguous()
        d = None if diag is None else diag.contiguous()
        o = SolveOpts(int(restart), int(max_iters), float(tol), 1 if x0 is None else 0, 0)
        info = SolveInfo()
        check(lib().fmm_layered_solve(self._h, None if d is None else ctypes.c_void_p(d.data_ptr()),
                                      ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                      ctypes.byref(o), _stream_handle(stream), ctypes.byref(info)))
        return x, {f: getattr(info, f) for f, _ in SolveInfo._fields_}

    def set_variants(self, m2l=-1, batch=-1, batch_min=-1):
        """Override the autotuner's choices (see fmm_layered_plan_set_variants)."""
        check(lib().fmm_layered_plan_set_variants(self._h, m2l, batch, batch_min))

    def stats(self) -> dict:
        s = Stats()
        check(lib().fmm_layered_plan_stats(self._h, ctypes.byref(s)))
        out = {f: getattr(s, f) for f, _ in Stats._fields_}
        out["m2l_variant_ms"] = list(out["m2l_variant_ms"])
        out["batch_variant_ms"] = list(out["batch_variant_ms"])
        out["m2l_eval_ms"] = list(out["m2l_eval_ms"])
        out["p2p_split_ms"] = list(out["p2p_split_ms"])
        return out

    def tree(self, t):
        lay = ctypes.c_int32()
        side = ctypes.c_int32()
        n = ctypes.c_int64()
        check(lib().fmm_layered_plan_tree(self._h, t, ctypes.byref(lay), ctypes.byref(side),
                                          ctypes.byref(n), None, None))
        keys = np.zeros(n.value, np.uint64)
        perm = np.zeros(n.value, np.int64)
        check(lib().fmm_layered_plan_tree(self._h, t, None, None, None, _ptr(keys), _ptr(perm)))
        return lay.value, side.value, keys, perm

    def lists(self, which):
        """Interaction-list table `which` (0 boxes, 1 M2L, 2 P2P free, 3 P2P reaction) as an
        int32 array (see fmm_layered_plan_lists)."""
        n = ctypes.c_int64()
        check(lib().fmm_layered_plan_lists(self._h, which, ctypes.byref(n), None))
        cols = 4 if which == 0 else 3
        out = np.zeros((n.value, cols), np.int32)
        check(lib().fmm_layered_plan_lists(self._h, which, ctypes.byref(n), _ptr(out)))
        return out

    def profile_begin(self, max_evals):
        check(lib().fmm_layered_profile_begin(self._h, max_evals))

    def profile_end(self):
        """Summed milliseconds per stage over the recorded evaluations, and their count."""
        ms = np.zeros(len(STAGES))
        n = ctypes.c_int64()
        check(lib().fmm_layered_profile_end(self._h, _ptr(ms), ctypes.byref(n)))
        return dict(zip(STAGES, ms)), n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().fmm_layered_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sommerfeld(d, eps, lt, ls, a, b, S, rho, z, nmax, stream=None):
    """S^N I_{N,M}(rho, z) for 0 <= M <= N <= nmax on the GPU; d=[] means sigma == 1."""
    d = _host(d, np.float64)
    eps = _host(eps, np.float64) if len(d) else np.ones(1)
    rho = _host(np.atleast_1d(rho), np.float64)
    z = _host(np.atleast_1d(z), np.float64)
    nc = (nmax + 1) * (nmax + 2) // 2
    out = np.zeros((len(rho), nc))
    check(lib().fmm_layered_sommerfeld(len(d), _ptr(d), _ptr(eps), lt, ls, a, b, float(S), len(rho),
                                       _ptr(rho), _ptr(z), nmax, _ptr(out), _stream_handle(stream)))
    return out


def sommerfeld_noalloc(d, eps, lt, ls, a, b, S, rho, z, nmax, out, stream=None):
    """fmm_layered_sommerfeld_noalloc: rho, z (CUDA float64 [npts]) -> out (CUDA float64
    [npts, (nmax+1)(nmax+2)/2]), asynchronous on the stream, allocating nothing."""
    import torch
    for name, t in (("rho", rho), ("z", z), ("out", out)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous CUDA float64 tensor")
    d = _host(d, np.float64)
    eps = _host(eps, np.float64) if len(d) else np.ones(1)
    check(lib().fmm_layered_sommerfeld_noalloc(len(d), _ptr(d), _ptr(eps), lt, ls, a, b, float(S), rho.numel(),
                                               ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                               nmax, ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def interp2d(npr, npz, rho_max, zeta_max, nodes, rho, zeta, stream=None):
    """The table form's interpolation on given node values [npr * npz, nout, 144]."""
    nodes = _host(nodes, np.float64)
    nout = nodes.shape[1]
    rho = _host(np.atleast_1d(rho), np.float64)
    zeta = _host(np.atleast_1d(zeta), np.float64)
    out = np.zeros((len(rho), nout))
    check(lib().fmm_layered_interp2d(npr, npz, float(rho_max), float(zeta_max), nout, _ptr(nodes), len(rho),
                                     _ptr(rho), _ptr(zeta), _ptr(out), _stream_handle(stream)))
    return out


def density(d, eps, lt, ls, a, b, k, stream=None):
    """sigma^{ab}_{lt,ls}(k) on the GPU for complex k (array)."""
    d = _host(d, np.float64)
    eps = _host(eps, np.float64)
    k = np.atleast_1d(np.asarray(k, np.complex128))
    kr = _host(k.real, np.float64)
    ki = _host(k.imag, np.float64)
    orr = np.zeros(len(k))
    oi = np.zeros(len(k))
    check(lib().fmm_layered_density(len(d), _ptr(d), _ptr(eps), lt, ls, a, b, len(k), _ptr(kr),
                                    _ptr(ki), _ptr(orr), _ptr(oi), _stream_handle(stream)))
    return orr + 1j * oi


def density_asymptotic(d, eps, lt, ls, a, b):
    """(sinf, zinf): sigma^{ab}_{lt,ls}(k) ~ sinf e^{-k zinf} as k -> infinity (host call)."""
    d = _host(d, np.float64)
    eps = _host(eps, np.float64)
    si = ctypes.c_double()
    zi = ctypes.c_double()
    check(lib().fmm_layered_density_asymptotic(len(d), _ptr(d), _ptr(eps), lt, ls, a, b,
                                               ctypes.byref(si), ctypes.byref(zi)))
    return si.value, zi.value


class Surrogate:
    """Learned form: fmm_layered_surrogate_* on a medium (or a plan's medium and domain).
    tables=True builds the table form instead (fmm_layered_tables_create*), which a plan
    takes the same way."""

    def __init__(self, d=None, eps=None, p=None, rho_max=None, zeta_max=None, seed=1, plan=None,
                 tables=False, stream=None):
        h = ctypes.c_void_p()
        if tables:
            if plan is not None:
                check(lib().fmm_layered_tables_create_for_plan(plan._h, _stream_handle(stream), ctypes.byref(h)))
                p = plan.p
            else:
                d = _host(d, np.float64)
                eps = _host(eps, np.float64)
                check(lib().fmm_layered_tables_create(len(d), _ptr(d), _ptr(eps), p, float(rho_max),
                                                      float(zeta_max), _stream_handle(stream), ctypes.byref(h)))
        elif plan is not None:
            check(lib().fmm_layered_surrogate_create_for_plan(plan._h, seed, ctypes.byref(h)))
            p = plan.p
        else:
            d = _host(d, np.float64)
            eps = _host(eps, np.float64)
            check(lib().fmm_layered_surrogate_create(len(d), _ptr(d), _ptr(eps), p, float(rho_max),
                                                     float(zeta_max), seed, ctypes.byref(h)))
        self._h = h
        self.nout = 4 * p + 1

    def table_info(self) -> dict:
        """Table form: panels per direction, device bytes, creation seconds."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        nb, sec = ctypes.c_int64(), ctypes.c_double()
        check(lib().fmm_layered_tables_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(nb),
                                            ctypes.byref(sec)))
        return {"npr": a.value, "npz": b.value, "bytes": nb.value, "seconds": sec.value}

    def train(self, nsamples=None, steps=None, batch=None, lr=None, seed=None, stream=None) -> dict:
        o = TrainOpts()
        lib().fmmlm_default_train_opts(ctypes.byref(o))
        for k, v in (("nsamples", nsamples), ("steps", steps), ("batch", batch), ("lr", lr),
                     ("seed", seed)):
            if v is not None:
                setattr(o, k, v)
        r = TrainReport()
        check(lib().fmm_layered_surrogate_train(self._h, ctypes.byref(o), _stream_handle(stream),
                                                ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in TrainReport._fields_}

    def params(self, set_to=None) -> np.ndarray:
        n = ctypes.c_int64()
        check(lib().fmm_layered_surrogate_params(self._h, None, None, ctypes.byref(n)))
        if set_to is not None:
            v = _host(set_to, np.float32)
            if v.size != n.value:
                raise ValueError("wrong parameter count")
            check(lib().fmm_layered_surrogate_params(self._h, None, _ptr(v), ctypes.byref(n)))
        out = np.zeros(n.value, np.float32)
        check(lib().fmm_layered_surrogate_params(self._h, _ptr(out), None, ctypes.byref(n)))
        return out

    def grad(self, comp, feat, target, stream=None):
        """(loss, gradient) of the mean squared error over one batch, on the GPU."""
        comp = _host(comp, np.int32)
        feat = _host(feat, np.float32)
        target = _host(target, np.float32)
        n = len(comp)
        g = np.zeros(self.params().size, np.float32)
        loss = ctypes.c_double()
        check(lib().fmm_layered_surrogate_grad(self._h, n, _ptr(comp), _ptr(feat), _ptr(target),
                                               ctypes.byref(loss), _ptr(g), _stream_handle(stream)))
        return loss.value, g

    def forward(self, comp, feat, stream=None):
        """Network outputs [n, nout] (FP32) for components comp [n] and features feat [n, 4]."""
        comp = _host(comp, np.int32)
        feat = _host(feat, np.float32)
        out = np.zeros((len(comp), self.nout), np.float32)
        check(lib().fmm_layered_surrogate_forward(self._h, len(comp), _ptr(comp), _ptr(feat), _ptr(out),
                                                  _stream_handle(stream)))
        return out

    def adam(self, grads, lr, stream=None):
        """Adam steps t = 1..len(grads) from zero moments with the given gradients [nsteps, nparams]
        and learning rates [nsteps]; updates the parameters in place and returns them after each
        step [nsteps, nparams]."""
        grads = _host(np.atleast_2d(grads), np.float32)
        lr = _host(np.broadcast_to(np.asarray(lr, np.float64), (grads.shape[0],)), np.float64)
        out = np.zeros_like(grads)
        check(lib().fmm_layered_surrogate_adam(self._h, grads.shape[0], _ptr(grads), _ptr(lr), _ptr(out),
                                               _stream_handle(stream)))
        return out

    def samples(self, n, seed=1, stream=None):
        """The training samples for seed: (comp, rho, zeta, feat [n, 4], target [n, nout])."""
        nout = self.nout
        comp = np.zeros(n, np.int32)
        rho = np.zeros(n)
        zeta = np.zeros(n)
        feat = np.zeros((n, 4), np.float32)
        target = np.zeros((n, nout), np.float32)
        check(lib().fmm_layered_surrogate_samples(self._h, n, seed, _ptr(comp), _ptr(rho), _ptr(zeta),
                                                  _ptr(feat), _ptr(target), _stream_handle(stream)))
        return comp, rho, zeta, feat, target

    def eval(self, lt, ls, a, b, S, rho, z, nmax, stream=None):
        """S^N I_{N,M} like sommerfeld(), through the network; also the served-by-network flags."""
        rho = _host(np.atleast_1d(rho), np.float64)
        z = _host(np.atleast_1d(z), np.float64)
        nc = (nmax + 1) * (nmax + 2) // 2
        out = np.zeros((len(rho), nc))
        used = np.zeros(len(rho), np.int32)
        check(lib().fmm_layered_surrogate_eval(self._h, lt, ls, a, b, float(S), len(rho), _ptr(rho),
                                               _ptr(z), nmax, _ptr(out), _ptr(used),
                                               _stream_handle(stream)))
        return out, used

    def close(self):
        if getattr(self, "_h", None):
            lib().fmm_layered_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
