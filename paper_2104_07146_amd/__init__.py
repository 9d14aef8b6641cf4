"""Python binding of the MI355X H-MLE library (libhmle.so, C ABI in include/hmle.h).

Argument marshalling only: every step of the log-likelihood evaluation runs in
the library's HIP kernels. PyTorch supplies device memory and the stream.
The library must be built (``python -m paper_2104_07146_amd.build``); there is
no fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhmle.so")

HMLE_OK, HMLE_E_INVALID, HMLE_E_NOMEM, HMLE_E_NOT_SPD, HMLE_E_STATE, HMLE_E_HIP, HMLE_E_NOCONV = range(7)
FP64, MIXED = 0, 1

FIT_STATE_BYTES = 320      # HMLE_FIT_STATE_BYTES of include/hmle.h

STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_NOT_SPD", 4: "E_STATE", 5: "E_HIP", 6: "E_NOCONV"}

EXPORTED = ["hmle_default_opts", "hmle_default_fit_opts", "hmle_build_tree", "hmle_build_tree_alloc",
            "hmle_build_batch_alloc", "hmle_assemble", "hmle_factor",
            "hmle_loglik", "hmle_fit", "hmle_fit_resumable", "hmle_fit_batch", "hmle_predict", "hmle_predict_var", "hmle_mloe_mmom", "hmle_matvec", "hmle_sample", "hmle_matern", "hmle_sizes", "hmle_export_tree",
            "hmle_export_blocks", "hmle_export_block", "hmle_stats", "hmle_assembly_info", "hmle_last_error", "hmle_destroy",
            "hmle_structure_host", "hmle_plan_stats", "hmle_profile", "hmle_build_batch", "hmle_assemble_batch",
            "hmle_factor_status", "hmle_loglik_batch", "hmle_eval_batch", "hmle_structure_batch_host",
            "hmle_mlp_param_count", "hmle_variogram", "hmle_variogram_noalloc", "hmle_mlp_create", "hmle_mlp_set_params", "hmle_mlp_get_params",
            "hmle_mlp_set_norm", "hmle_mlp_get_norm", "hmle_mlp_fit_norm", "hmle_mlp_forward", "hmle_mlp_grad",
            "hmle_mlp_train_step", "hmle_propose", "hmle_mlp_destroy", "hmle_autotune"]


class HmleError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class NotSPD(HmleError):
    pass


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


def torch_allocator():
    """An hmle_allocator backed by PyTorch's caching allocator on the current
    device (the returned object keeps the callbacks alive; keep it as long as
    any problem built with it)."""
    import torch
    dev = torch.cuda.current_device()

    def _alloc(nbytes, stream, user):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream))
        except Exception:
            return None

    def _free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    return a


class Theta(ctypes.Structure):
    _fields_ = [("sigma2", ctypes.c_double), ("range", ctypes.c_double), ("nu", ctypes.c_double),
                ("tau2", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("eta", ctypes.c_double), ("aca_tol", ctypes.c_double),
                ("max_rank", ctypes.c_int32), ("precision", ctypes.c_int32), ("pair_chunk", ctypes.c_int32),
                ("sketch_group", ctypes.c_int32), ("spd_margin", ctypes.c_double),
                ("seg_entries", ctypes.c_int32), ("gseg_rows", ctypes.c_int32), ("sum_kc", ctypes.c_int32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("opts", Opts), ("ms", ctypes.c_double)]


SCHEDULE_KEYS = ("pair_chunk", "sketch_group", "seg_entries", "gseg_rows", "sum_kc")


class FitOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("step", ctypes.c_double),
                ("use_backoff", ctypes.c_int32), ("report_every", ctypes.c_int32),
                ("profile_variance", ctypes.c_int32)]


class FitReport(ctypes.Structure):
    _fields_ = [("evals", ctypes.c_int32), ("iters", ctypes.c_int32), ("failed_evals", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("logL", ctypes.c_double), ("wall_s", ctypes.c_double)]


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libhmle.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2104_07146_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
        L.hmle_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.hmle_default_opts.restype = None
        L.hmle_default_fit_opts.argtypes = [ctypes.POINTER(FitOpts)]
        L.hmle_default_fit_opts.restype = None
        L.hmle_build_tree.argtypes = [vp, i64, i32, ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
        L.hmle_build_tree_alloc.argtypes = [vp, i64, i32, ctypes.POINTER(Opts), ctypes.POINTER(Allocator), vp,
                                            ctypes.POINTER(vp)]
        L.hmle_build_batch_alloc.argtypes = [vp, vp, i32, i32, ctypes.POINTER(Opts), ctypes.POINTER(Allocator), vp,
                                             ctypes.POINTER(vp)]
        L.hmle_assemble.argtypes = [vp, ctypes.POINTER(Theta)]
        L.hmle_factor.argtypes = [vp]
        L.hmle_loglik.argtypes = [vp, vp, dp]
        L.hmle_fit.argtypes = [vp, vp, ctypes.POINTER(Theta), ctypes.POINTER(FitOpts), ctypes.POINTER(Theta),
                               ctypes.POINTER(FitReport)]
        L.hmle_fit_resumable.argtypes = [vp, vp, ctypes.POINTER(Theta), ctypes.POINTER(FitOpts), vp, i64,
                                         ctypes.POINTER(Theta), ctypes.POINTER(FitReport)]
        L.hmle_fit_batch.argtypes = [vp, vp, ctypes.POINTER(Theta), ctypes.POINTER(FitOpts), ctypes.POINTER(Theta),
                                     ctypes.POINTER(FitReport), ctypes.POINTER(ctypes.c_int32)]
        L.hmle_sample.argtypes = [vp, vp, vp]
        L.hmle_matvec.argtypes = [vp, vp, vp]
        L.hmle_mloe_mmom.argtypes = [vp, vp, vp, ctypes.c_int64, i32, vp, vp, vp, dp]
        L.hmle_predict.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
        L.hmle_predict_var.argtypes = [vp, vp, ctypes.c_int64, vp]
        L.hmle_matern.argtypes = [vp, i64, ctypes.POINTER(Theta), i32, vp, vp]
        L.hmle_sizes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.hmle_export_tree.argtypes = [vp, vp, vp, vp, vp]
        L.hmle_export_blocks.argtypes = [vp, vp, vp]
        L.hmle_export_block.argtypes = [vp, i32, i64, vp, i64, ctypes.POINTER(ctypes.c_int32)]
        L.hmle_stats.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64)]
        L.hmle_assembly_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.hmle_structure_host.argtypes = [vp, i64, i32, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        L.hmle_plan_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.hmle_build_batch.argtypes = [vp, vp, i32, i32, ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
        L.hmle_assemble_batch.argtypes = [vp, vp]
        L.hmle_factor_status.argtypes = [vp, vp]
        L.hmle_loglik_batch.argtypes = [vp, vp, vp, vp]
        L.hmle_eval_batch.argtypes = [vp, vp, vp, vp, vp]
        L.hmle_structure_batch_host.argtypes = [vp, vp, i32, i32, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        fp = ctypes.POINTER(ctypes.c_float)
        L.hmle_mlp_param_count.argtypes = []
        L.hmle_mlp_param_count.restype = i64
        L.hmle_variogram.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp]
        L.hmle_variogram_noalloc.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, vp]
        L.hmle_mlp_create.argtypes = [vp, vp, ctypes.POINTER(vp)]
        L.hmle_mlp_set_params.argtypes = [vp, vp]
        L.hmle_mlp_get_params.argtypes = [vp, vp]
        L.hmle_mlp_set_norm.argtypes = [vp, vp]
        L.hmle_mlp_get_norm.argtypes = [vp, vp]
        L.hmle_mlp_fit_norm.argtypes = [vp, vp, vp, i64]
        L.hmle_mlp_forward.argtypes = [vp, vp, i32, vp]
        L.hmle_mlp_grad.argtypes = [vp, vp, vp, vp, i32, i64, vp, fp]
        L.hmle_mlp_train_step.argtypes = [vp, vp, vp, vp, i32, i64, ctypes.c_float, fp]
        L.hmle_propose.argtypes = [vp, vp, ctypes.POINTER(Theta)]
        L.hmle_autotune.argtypes = [vp, i64, i32, ctypes.POINTER(Opts), ctypes.POINTER(Theta), vp,
                                    ctypes.POINTER(Opts), ctypes.POINTER(TuneEntry), i32, ctypes.POINTER(i32)]
        L.hmle_mlp_destroy.argtypes = [vp]
        L.hmle_mlp_destroy.restype = None
        L.hmle_profile.argtypes = [vp, i32, dp]
        L.hmle_last_error.argtypes = [vp]
        L.hmle_last_error.restype = ctypes.c_char_p
        L.hmle_destroy.argtypes = [vp]
        L.hmle_destroy.restype = None
        for name in EXPORTED:
            getattr(L, name)                  # every declared symbol must be present
        _LIB = L
    return _LIB


def _check(status: int, handle=None):
    if status == HMLE_OK:
        return
    msg = lib().hmle_last_error(handle)
    msg = msg.decode() if msg else ""
    if status == HMLE_E_NOT_SPD:
        raise NotSPD(status, msg)
    raise HmleError(status, msg)


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream


def theta_struct(theta) -> Theta:
    s2, ell, nu, t2 = (float(v) for v in theta)
    return Theta(s2, ell, nu, t2)


def default_opts() -> Opts:
    o = Opts()
    lib().hmle_default_opts(ctypes.byref(o))
    return o


def make_opts(leaf_size=None, eta=None, aca_tol=None, max_rank=None, precision=None, pair_chunk=None,
              sketch_group=None, spd_margin=None, seg_entries=None, gseg_rows=None, sum_kc=None) -> Opts:
    o = default_opts()
    if seg_entries is not None:
        o.seg_entries = int(seg_entries)
    if gseg_rows is not None:
        o.gseg_rows = int(gseg_rows)
    if sum_kc is not None:
        o.sum_kc = int(sum_kc)
    if spd_margin is not None:
        o.spd_margin = float(spd_margin)
    if pair_chunk is not None:
        o.pair_chunk = int(pair_chunk)
    if sketch_group is not None:
        o.sketch_group = int(sketch_group)
    if leaf_size is not None:
        o.leaf_size = int(leaf_size)
    if eta is not None:
        o.eta = float(eta)
    if aca_tol is not None:
        o.aca_tol = float(aca_tol)
    if max_rank is not None:
        o.max_rank = int(max_rank)
    if precision is not None:
        o.precision = int(precision)
    return o


def autotune(pts, theta, **opts):
    """Coordinate search over the schedule options and the tile shape
    (SCHEDULE_KEYS) on this point set at theta (hmle_autotune); returns (best
    schedule dict, [(schedule dict, ms) in the order measured])."""
    import torch
    pts = pts.to(dtype=torch.float64).contiguous()
    base = make_opts(**opts)
    best = Opts()
    tried = (TuneEntry * 64)()
    nt = ctypes.c_int32()
    th = theta_struct(theta)
    _check(lib().hmle_autotune(_ptr(pts), pts.shape[0], pts.shape[1], ctypes.byref(base), ctypes.byref(th), _stream(),
                               ctypes.byref(best), tried, 64, ctypes.byref(nt)))
    sched = lambda o: {k: int(getattr(o, k)) for k in SCHEDULE_KEYS}
    return sched(best), [(sched(tried[i].opts), tried[i].ms) for i in range(min(nt.value, 64))]


TUNED_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "tuned.json")


def tune_key(n, dim, **opts) -> str:
    """Key of a tuned schedule: device architecture, precision, leaf size, rank
    cap, accuracy and the size class (n to the nearest power of two, dimension)."""
    import math
    import torch
    o = make_opts(**opts)
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    return (f"{arch}|prec{o.precision}|leaf{o.leaf_size}|rank{o.max_rank}|eps{o.aca_tol:.0e}"
            f"|n2^{round(math.log2(max(n, 1)))}|d{dim}")


def tuned_schedule(pts, theta, path=None, tune_if_missing=True, **opts):
    """The schedule options for this configuration from the JSON cache (default
    the package's data/tuned.json), measured with ``autotune`` and stored
    there when missing (tune_if_missing); None when missing and not tuned."""
    import json
    path = path or TUNED_FILE
    key = tune_key(int(pts.shape[0]), int(pts.shape[1]), **opts)
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    if key in cache:
        return {k: int(v) for k, v in cache[key]["schedule"].items() if k in SCHEDULE_KEYS}
    if not tune_if_missing:
        return None
    best, tried = autotune(pts, theta, **opts)
    cache[key] = {"schedule": best, "ms": min(ms for _, ms in tried), "candidates": len(tried)}
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return best


def matern(h, theta, precision: int = FP64):
    """Device Matern values (eq. 2, no nugget) at the distances of tensor h."""
    import torch
    out = torch.empty_like(h)
    th = theta_struct(theta)
    _check(lib().hmle_matern(_ptr(h), h.numel(), ctypes.byref(th), int(precision), _stream(), _ptr(out)))
    return out


@dataclass
class Fit:
    theta: tuple
    evals: int
    iters: int
    failed_evals: int
    converged: bool
    logL: float
    wall_s: float
    status: int


_PLAN_KEYS = ["pairs", "inner", "dense_entries", "lr_dims", "leaves", "rank_width", "col_solves", "lr_pairs",
              "grams", "gram_pairs", "steps", "problems", "lr_pairs_dd", "lr_pairs_dr", "lr_pairs_rd", "lr_pairs_rr"]


def _plan_stats(handle):
    s = (ctypes.c_int64 * 16)()
    _check(lib().hmle_plan_stats(handle, s), handle)
    return dict(zip(_PLAN_KEYS, list(s)))


def _offsets(sizes):
    import numpy as np
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.asarray(sizes, dtype=np.int64))
    return off


def _theta_array(thetas, count):
    arr = (Theta * count)()
    thetas = list(thetas)
    if len(thetas) != count:
        raise ValueError(f"expected {count} theta tuples, got {len(thetas)}")
    for q, t in enumerate(thetas):
        arr[q] = theta_struct(t)
    return arr


class _Handle:
    _h = None

    def close(self):
        if getattr(self, "_h", None):
            lib().hmle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def sizes(self):
        s = (ctypes.c_int64 * 6)()
        _check(lib().hmle_sizes(self._h, s), self._h)
        return dict(zip(["n", "dim", "n_nodes", "n_dense", "n_lowrank", "n_leaves"], list(s)))

    def export_tree(self):
        import numpy as np
        sz = self.sizes()
        perm = np.empty(sz["n"], dtype=np.int64)
        nodes = np.empty((sz["n_nodes"], 4), dtype=np.int64)
        bmin = np.empty((sz["n_nodes"], sz["dim"]))
        bmax = np.empty((sz["n_nodes"], sz["dim"]))
        _check(lib().hmle_export_tree(self._h, perm.ctypes.data, nodes.ctypes.data, bmin.ctypes.data,
                                      bmax.ctypes.data), self._h)
        return perm, nodes, bmin, bmax

    def export_blocks(self):
        import numpy as np
        sz = self.sizes()
        dense = np.empty((sz["n_dense"], 2), dtype=np.int64)
        lowrank = np.empty((sz["n_lowrank"], 2), dtype=np.int64)
        _check(lib().hmle_export_blocks(self._h, dense.ctypes.data, lowrank.ctypes.data), self._h)
        return dense, lowrank


class BatchStructure(_Handle):
    """Partition of a batch of host point sets (list of numpy (n_q, dim)
    arrays) without the GPU."""

    def __init__(self, pts_list, **opts):
        import numpy as np
        pts = np.ascontiguousarray(np.concatenate(pts_list, axis=0), dtype=np.float64)
        off = _offsets([len(a) for a in pts_list])
        self._opts = make_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().hmle_structure_batch_host(pts.ctypes.data, off.ctypes.data, len(pts_list), pts.shape[1],
                                               ctypes.byref(self._opts), ctypes.byref(h)))
        self._h = h
        self.offsets = off

    def plan_stats(self):
        return _plan_stats(self._h)


class Structure(_Handle):
    """Partition of a host point set (numpy (n, dim) float64) without the GPU:
    trees, blocks and plan statistics."""

    def __init__(self, pts, **opts):
        import numpy as np
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        n, dim = pts.shape
        self._opts = make_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().hmle_structure_host(pts.ctypes.data, n, dim, ctypes.byref(self._opts), ctypes.byref(h)))
        self._h = h

    def plan_stats(self):
        return _plan_stats(self._h)


class Problem(_Handle):
    """One point set: its trees and plan (built once), and the H-matrix
    assembled / factorised for the current theta."""

    def __init__(self, pts, allocator=None, **opts):
        """allocator: None (the library's hipMalloc), "torch" (PyTorch's caching
        allocator) or an Allocator structure."""
        import torch
        pts = pts.to(dtype=torch.float64).contiguous()
        n, dim = pts.shape
        self._opts = make_opts(**opts)
        h = ctypes.c_void_p()
        self._alloc = torch_allocator() if allocator == "torch" else allocator
        if self._alloc is None:
            _check(lib().hmle_build_tree(_ptr(pts), n, dim, ctypes.byref(self._opts), _stream(), ctypes.byref(h)))
        else:
            _check(lib().hmle_build_tree_alloc(_ptr(pts), n, dim, ctypes.byref(self._opts), ctypes.byref(self._alloc),
                                               _stream(), ctypes.byref(h)))
        self._h = h
        self.n, self.dim = int(n), int(dim)

    def assemble(self, theta):
        th = theta_struct(theta)
        _check(lib().hmle_assemble(self._h, ctypes.byref(th)), self._h)

    def factor(self):
        _check(lib().hmle_factor(self._h), self._h)

    def loglik(self, z):
        out = (ctypes.c_double * 3)()
        _check(lib().hmle_loglik(self._h, _ptr(z), out), self._h)
        return float(out[0]), float(out[1]), float(out[2])

    def eval(self, theta, z):
        """assemble + factor + loglik at theta."""
        self.assemble(theta)
        self.factor()
        return self.loglik(z)

    def sample(self, w):
        import torch
        z = torch.empty_like(w)
        _check(lib().hmle_sample(self._h, _ptr(w), _ptr(z)), self._h)
        return z

    def matvec(self, x):
        """C~ x with the assembled H-matrix (between assemble and factor)."""
        import torch
        y = torch.empty_like(x)
        _check(lib().hmle_matvec(self._h, _ptr(x), _ptr(y)), self._h)
        return y

    def predict(self, z1, pts2):
        """Kriging mean (eq. (4)) at the rows of pts2 (CUDA (m, dim) float64)
        from the training data z1, with the current factor."""
        import torch
        pts2 = pts2.to(dtype=torch.float64).contiguous()
        z2 = torch.empty(pts2.shape[0], dtype=torch.float64, device=pts2.device)
        _check(lib().hmle_predict(self._h, _ptr(z1), _ptr(pts2), int(pts2.shape[0]), _ptr(z2)), self._h)
        return z2

    def predict_var(self, pts2):
        """Kriging variance of the field at the rows of pts2 (CUDA (m, dim)
        float64) with the current factor."""
        import torch
        pts2 = pts2.to(dtype=torch.float64).contiguous()
        var = torch.empty(pts2.shape[0], dtype=torch.float64, device=pts2.device)
        _check(lib().hmle_predict_var(self._h, _ptr(pts2), int(pts2.shape[0]), _ptr(var)), self._h)
        return var

    def fit(self, z, start=None, max_iter=400, tol=1e-4, step=1.0, use_backoff=True, report_every=0,
            profile_variance=False) -> Fit:
        fo = FitOpts(int(max_iter), float(tol), float(step), 1 if use_backoff else 0, int(report_every),
                     1 if profile_variance else 0)
        th = Theta()
        rep = FitReport()
        st = theta_struct(start) if start is not None else None
        status = lib().hmle_fit(self._h, _ptr(z), ctypes.byref(st) if st is not None else None, ctypes.byref(fo),
                                ctypes.byref(th), ctypes.byref(rep))
        if status not in (HMLE_OK, HMLE_E_NOCONV):
            _check(status, self._h)
        return Fit((th.sigma2, th.range, th.nu, th.tau2), rep.evals, rep.iters, rep.failed_evals,
                   bool(rep.converged), rep.logL, rep.wall_s, status)

    def fit_resumable(self, z, state=None, start=None, max_iter=400, tol=1e-4, step=1.0, use_backoff=True,
                      report_every=0, profile_variance=False):
        """The fit of ``fit`` with a checkpoint: ``state`` None starts a new
        fit, the bytes returned by an earlier call continue it (start is then
        ignored). Returns (Fit, checkpoint bytes); a fit stopped by max_iter
        and continued with a larger max_iter equals the uninterrupted fit."""
        buf = ctypes.create_string_buffer(FIT_STATE_BYTES)
        if state is not None:
            if len(state) != FIT_STATE_BYTES:
                raise ValueError(f"a checkpoint has {FIT_STATE_BYTES} bytes")
            ctypes.memmove(buf, bytes(state), FIT_STATE_BYTES)
        fo = FitOpts(int(max_iter), float(tol), float(step), 1 if use_backoff else 0, int(report_every),
                     1 if profile_variance else 0)
        th = Theta()
        rep = FitReport()
        st = theta_struct(start) if start is not None else None
        status = lib().hmle_fit_resumable(self._h, _ptr(z), ctypes.byref(st) if st is not None else None,
                                          ctypes.byref(fo), buf, FIT_STATE_BYTES, ctypes.byref(th),
                                          ctypes.byref(rep))
        if status not in (HMLE_OK, HMLE_E_NOCONV):
            _check(status, self._h)
        fit = Fit((th.sigma2, th.range, th.nu, th.tau2), rep.evals, rep.iters, rep.failed_evals,
                  bool(rep.converged), rep.logL, rep.wall_s, status)
        return fit, buf.raw

    def export_block(self, kind: int, which: int, m: int, k: int):
        """kind 0: dense list index -> (m x k) array; kind 1: low-rank -> (U, V)."""
        import numpy as np
        cap = max(m * k, (m + k) * 64)
        buf = np.empty(cap)
        r = ctypes.c_int32()
        _check(lib().hmle_export_block(self._h, int(kind), int(which), buf.ctypes.data, cap, ctypes.byref(r)),
               self._h)
        if r.value < 0:
            return buf[:m * k].reshape(k, m).T.copy()
        rk = r.value
        U = buf[:m * rk].reshape(rk, m).T.copy()
        V = buf[m * rk:(m + k) * rk].reshape(rk, k).T.copy()
        return U, V

    def profile(self, enable=None):
        """Live timing of the dense-pair (k_dpairs), sketch-pass (k_rpass) and
        diagonal-leaf (k_potrf) kernels: enable True/False to (re)start/stop;
        returns {name: (ms, launches, flops)} so far."""
        out = (ctypes.c_double * 9)()
        flag = -1 if enable is None else (1 if enable else 0)
        _check(lib().hmle_profile(self._h, flag, out), self._h)
        return {"k_dpairs": (out[0], out[1], out[2]), "k_rpass": (out[3], out[4], out[5]),
                "k_potrf": (out[6], out[7], out[8])}

    def plan_stats(self):
        return _plan_stats(self._h)

    def assembly_info(self):
        """(last assemble reused the saved assembly, reuses so far)."""
        i = (ctypes.c_int64 * 2)()
        _check(lib().hmle_assembly_info(self._h, i), self._h)
        return bool(i[0]), int(i[1])

    def stats(self):
        t = (ctypes.c_double * 3)()
        c = (ctypes.c_int64 * 3)()
        _check(lib().hmle_stats(self._h, t, c), self._h)
        return {"assemble_ms": t[0], "factor_ms": t[1], "loglik_ms": t[2], "rank_sum": c[0], "rank_max": c[1],
                "cap_hits": c[2]}


class Batch(_Handle):
    """Many independent problems (each its own point set and theta) evaluated
    together: one plan over all of them, the factorisation stepping through
    the s-th leaf of every problem at once, and a captured graph replayed per
    evaluation (``eval``)."""

    def __init__(self, pts_list, allocator=None, **opts):
        import torch
        sizes = [int(a.shape[0]) for a in pts_list]
        pts = torch.cat([a.to(dtype=torch.float64) for a in pts_list], dim=0).contiguous()
        if not pts.is_cuda:
            raise ValueError("points must be CUDA tensors")
        off = _offsets(sizes)
        self._opts = make_opts(**opts)
        h = ctypes.c_void_p()
        self._alloc = torch_allocator() if allocator == "torch" else allocator
        if self._alloc is None:
            _check(lib().hmle_build_batch(_ptr(pts), off.ctypes.data, len(sizes), int(pts.shape[1]),
                                          ctypes.byref(self._opts), _stream(), ctypes.byref(h)))
        else:
            _check(lib().hmle_build_batch_alloc(_ptr(pts), off.ctypes.data, len(sizes), int(pts.shape[1]),
                                                ctypes.byref(self._opts), ctypes.byref(self._alloc), _stream(),
                                                ctypes.byref(h)))
        self._h = h
        self.count = len(sizes)
        self.sizes_ = sizes
        self.offsets = off
        self.n = int(off[-1])

    def _out(self):
        import numpy as np
        return np.empty((self.count, 3)), np.empty(self.count, dtype=np.int32)

    def assemble(self, thetas):
        arr = _theta_array(thetas, self.count)
        _check(lib().hmle_assemble_batch(self._h, arr), self._h)

    def factor(self):
        import numpy as np
        _check(lib().hmle_factor(self._h), self._h)
        st = np.empty(self.count, dtype=np.int32)
        _check(lib().hmle_factor_status(self._h, st.ctypes.data), self._h)
        return st

    def loglik(self, z):
        out, st = self._out()
        _check(lib().hmle_loglik_batch(self._h, _ptr(z), out.ctypes.data, st.ctypes.data), self._h)
        return out, st

    def eval(self, thetas, z):
        """Graph-replayed assemble + factor + loglik of every problem; returns
        (out (count, 3): logL, logdet, quad; status per problem)."""
        arr = _theta_array(thetas, self.count)
        out, st = self._out()
        _check(lib().hmle_eval_batch(self._h, arr, _ptr(z), out.ctypes.data, st.ctypes.data), self._h)
        return out, st

    def sample(self, w):
        import torch
        z = torch.empty_like(w)
        _check(lib().hmle_sample(self._h, _ptr(w), _ptr(z)), self._h)
        return z

    def matvec(self, x):
        """C~ x of the block-diagonal batch H-matrix (between assemble and factor)."""
        import torch
        y = torch.empty_like(x)
        _check(lib().hmle_matvec(self._h, _ptr(x), _ptr(y)), self._h)
        return y

    def fit(self, z, start=None, max_iter=400, tol=1e-4, step=1.0, use_backoff=True, report_every=0,
            profile_variance=False):
        """Nelder-Mead fit with theta candidates evaluated together; the batch
        must hold copies of one point set, z is the data of one copy. Returns
        (Fit, rounds): the Fit equals Problem.fit on one copy."""
        fo = FitOpts(int(max_iter), float(tol), float(step), 1 if use_backoff else 0, int(report_every),
                     1 if profile_variance else 0)
        th = Theta()
        rep = FitReport()
        rounds = ctypes.c_int32()
        st = theta_struct(start) if start is not None else None
        status = lib().hmle_fit_batch(self._h, _ptr(z), ctypes.byref(st) if st is not None else None,
                                      ctypes.byref(fo), ctypes.byref(th), ctypes.byref(rep), ctypes.byref(rounds))
        if status not in (HMLE_OK, HMLE_E_NOCONV):
            _check(status, self._h)
        return (Fit((th.sigma2, th.range, th.nu, th.tau2), rep.evals, rep.iters, rep.failed_evals, bool(rep.converged),
                    rep.logL, rep.wall_s, status), int(rounds.value))

    def split(self, v):
        """Per-problem views of a concatenated vector."""
        return [v[int(self.offsets[q]):int(self.offsets[q + 1])] for q in range(self.count)]

    def plan_stats(self):
        return _plan_stats(self._h)

    def stats(self):
        t = (ctypes.c_double * 3)()
        c = (ctypes.c_int64 * 3)()
        _check(lib().hmle_stats(self._h, t, c), self._h)
        return {"assemble_ms": t[0], "factor_ms": t[1], "loglik_ms": t[2], "rank_sum": c[0], "rank_max": c[1],
                "cap_hits": c[2]}


# ------------------------------------------------------- learned start -----
N_FEAT, N_OUT = 33, 4


def _fptr(t, dtype_name="float32"):
    import torch
    dt = {"float32": torch.float32, "int32": torch.int32}[dtype_name]
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype_name} CUDA tensor")
    return t.data_ptr()


def mloe_mmom(est, true, pts2, noisy=True):
    """MLOE and MMOM (eqs. (5), (6)) at the new points pts2 (m x dim float64
    CUDA) for problems factorised at the estimated (est) and the true (true)
    parameters; returns (mloe, mmom, e_ta, e_tt, e_aa) with the per-point
    expected squared errors as CUDA tensors."""
    import torch
    m = int(pts2.shape[0])
    e = [torch.empty(m, dtype=torch.float64, device=pts2.device) for _ in range(3)]
    out = (ctypes.c_double * 2)()
    _check(lib().hmle_mloe_mmom(est._h, true._h, _ptr(pts2), m, 1 if noisy else 0, _ptr(e[0]), _ptr(e[1]),
                                _ptr(e[2]), out), est._h)
    return out[0], out[1], e[0], e[1], e[2]


def variogram(pts, z, offsets=None, sel=None, sel_offsets=None, out=None, noalloc=False):
    """Variogram features (count x 33 float32 CUDA tensor) of fields stored one
    after another in pts (N x dim float64 CUDA) and z (N float64 CUDA);
    offsets (host int64, count+1) delimit the fields (default: one field);
    sel (int32 CUDA, local indices) / sel_offsets (host int64) pick the points used.
    out: optional preallocated count x 33 float32 CUDA tensor. noalloc: call
    hmle_variogram_noalloc (the library's fixed workspace, no device allocation)."""
    import numpy as np
    import torch
    n, dim = pts.shape
    off = np.asarray(offsets if offsets is not None else [0, n], dtype=np.int64)
    count = len(off) - 1
    if out is None:
        out = torch.empty((count, N_FEAT), dtype=torch.float32, device=pts.device)
    elif out.dtype != torch.float32 or not out.is_contiguous() or out.numel() < count * N_FEAT:
        raise ValueError("out must be a contiguous float32 tensor of count x 33 values")
    soff = None if sel is None else np.asarray(sel_offsets, dtype=np.int64)
    fn = lib().hmle_variogram_noalloc if noalloc else lib().hmle_variogram
    _check(fn(_ptr(pts), _ptr(z), off.ctypes.data, count, dim, None if sel is None else _fptr(sel, "int32"),
              None if soff is None else soff.ctypes.data, _stream(), _fptr(out)))
    return out


class Mlp:
    """The start-proposal network on the device (weights, Adam state,
    normalisation); every pass runs in the library's kernels."""

    def __init__(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != lib().hmle_mlp_param_count():
            raise ValueError("wrong parameter count")
        h = ctypes.c_void_p()
        _check(lib().hmle_mlp_create(p.ctypes.data, _stream(), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().hmle_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, status):
        _check(status, None)

    def params(self):
        import numpy as np
        p = np.empty(lib().hmle_mlp_param_count(), dtype=np.float32)
        self._chk(lib().hmle_mlp_get_params(self._h, p.ctypes.data))
        return p

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._chk(lib().hmle_mlp_set_params(self._h, p.ctypes.data))

    def norm(self):
        import numpy as np
        a = np.empty(2 * N_FEAT + 2 * N_OUT, dtype=np.float32)
        self._chk(lib().hmle_mlp_get_norm(self._h, a.ctypes.data))
        return a

    def set_norm(self, norm):
        import numpy as np
        a = np.ascontiguousarray(norm, dtype=np.float32)
        self._chk(lib().hmle_mlp_set_norm(self._h, a.ctypes.data))

    def fit_norm(self, x, lt):
        self._chk(lib().hmle_mlp_fit_norm(self._h, _fptr(x), _fptr(lt), int(x.shape[0])))

    def forward(self, x):
        """Predicted log(sigma2, range, nu, tau2) for raw features x (rows x 33)."""
        import torch
        y = torch.empty((x.shape[0], N_OUT), dtype=torch.float32, device=x.device)
        self._chk(lib().hmle_mlp_forward(self._h, _fptr(x), int(x.shape[0]), _fptr(y)))
        return y

    def grad(self, x, lt, idx=None, rows=None):
        import torch
        rows = int(idx.shape[0]) if idx is not None else int(x.shape[0]) if rows is None else rows
        g = torch.empty(lib().hmle_mlp_param_count(), dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        self._chk(lib().hmle_mlp_grad(self._h, _fptr(x), _fptr(lt), None if idx is None else _fptr(idx, "int32"),
                                      rows, int(x.shape[0]), _fptr(g), ctypes.byref(loss)))
        return g, float(loss.value)

    def train_step(self, x, lt, idx=None, lr=1e-3, want_loss=True):
        rows = int(idx.shape[0]) if idx is not None else int(x.shape[0])
        loss = ctypes.c_float()
        self._chk(lib().hmle_mlp_train_step(self._h, _fptr(x), _fptr(lt),
                                            None if idx is None else _fptr(idx, "int32"), rows, int(x.shape[0]),
                                            float(lr), ctypes.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None

    def propose(self, feat):
        th = Theta()
        self._chk(lib().hmle_propose(self._h, _fptr(feat), ctypes.byref(th)))
        return (th.sigma2, th.range, th.nu, th.tau2)
