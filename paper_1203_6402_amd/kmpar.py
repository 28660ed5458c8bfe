"""Python binding of libkmpar.so (the C ABI in include/kmpar.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  Importing this module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import functools
from types import SimpleNamespace
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkmpar.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")

_lib = ctypes.CDLL(LIB_PATH)

MAX_ROUNDS = 64
F32, BF16, FP8_E4M3 = 0, 1, 2
MODE_PLAIN_FP32, MODE_REFINED = 0, 1
OP_INIT, OP_COST, OP_ASSIGN, OP_LLOYD, OP_KMEANSPP, OP_ASSIGN_SHARDED = 0, 1, 2, 3, 4, 5
OK, E_INVAL, E_WORKSPACE, E_HIP, E_TOOFEW, E_OVERFLOW, E_NODEVICE = 0, -1, -2, -3, -4, -5, -6


class Stats(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_double * (MAX_ROUNDS + 1)),
                ("round_count", ctypes.c_int32 * (MAX_ROUNDS + 1)),
                ("n_candidates", ctypes.c_int32),
                ("n_centers", ctypes.c_int32),
                ("status", ctypes.c_int32),
                ("n_rescanned", ctypes.c_int32),
                ("flagged_draws", ctypes.c_int32),
                ("flagged_picks", ctypes.c_int32),
                ("flagged_argmins", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Trace(ctypes.Structure):
    _fields_ = [("cand_point", ctypes.c_void_p), ("cand_weight", ctypes.c_void_p),
                ("center_cand", ctypes.c_void_p), ("assign", ctypes.c_void_p),
                ("d2", ctypes.c_void_p)]


_vp, _i64, _i32, _u64, _dbl, _sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t)
_lib.kmpar_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]
_lib.kmpar_destroy.argtypes = [_vp]
_lib.kmpar_strerror.argtypes = [ctypes.c_int]
_lib.kmpar_strerror.restype = ctypes.c_char_p
_lib.kmpar_last_error.argtypes = [_vp]
_lib.kmpar_last_error.restype = ctypes.c_char_p
_lib.kmpar_sizeof_stats.restype = _sz
_lib.kmpar_max_candidates.argtypes = [_i64, _dbl, _i32, ctypes.POINTER(_i64)]
_lib.kmpar_workspace_size.argtypes = [_vp, ctypes.c_int, _i64, _i32, _i32, _dbl, _i32,
                                      ctypes.c_int, ctypes.POINTER(_sz)]
_lib.kmpar_init.argtypes = [_vp, _vp, _vp, ctypes.c_int, _i64, _i32, _i32, _dbl, _i32, _u64,
                            _vp, _vp, _sz, _vp, ctypes.POINTER(Trace), _vp]
_lib.kmpar_cost.argtypes = [_vp, _vp, _vp, ctypes.c_int, _i64, _i32, _vp, _i32, _vp, _vp, _sz, _vp]
_lib.kmpar_cost_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_int, _i64, _i32, _vp, _i32, _vp, _vp]
_lib.kmpar_assign.argtypes = [_vp, _vp, _vp, ctypes.c_int, _i64, _i32, _vp, _i32, _vp, _vp, _vp,
                              _sz, _vp]
_lib.lloyd_step.argtypes = [_vp, _vp, _vp, ctypes.c_int, _i64, _i32, _vp, _i32, _vp, _vp, _vp,
                            _sz, _vp]
_lib.kmpar_lloyd.argtypes = [_vp, _vp, _vp, ctypes.c_int, _i64, _i32, _vp, _i32, _i32, _vp, _vp,
                             _vp, _sz, _vp]
_lib.kmpar_kmeanspp.argtypes = [_vp, _vp, _vp, ctypes.c_int, _i64, _i32, _i32, _u64, _vp, _vp, _vp,
                                _vp, _sz, _vp, _vp]
_lib.kmpar_lloyd_until_stable.argtypes = [_vp, _vp, _vp, ctypes.c_int, _i64, _i32, _vp, _i32, _i32,
                                          ctypes.POINTER(_i32), _vp, _vp, _vp, _sz, _vp]
_lib.kmpar_assign_sharded.argtypes = [_vp, _vp, _vp, ctypes.c_int, _i64, _i32, _vp, _i32, _i32, _vp,
                                     _vp, _vp, _vp, _sz, _vp]
_lib.kmpar_workspace_size_batched.argtypes = [_vp, _vp, _i32, ctypes.c_int, ctypes.POINTER(_sz)]
_lib.kmpar_init_batched.argtypes = [_vp, _vp, _vp, _i32, ctypes.c_int, _u64, _vp, _sz, _vp, _vp]
_lib.kmpar_set_option.argtypes = [_vp, ctypes.c_int, _i64]
_lib.kmpar_batch_tiles.argtypes = [_vp, _vp, _vp, _vp, _i32, ctypes.POINTER(_i32)]
_lib.kmpar_profile_enable.argtypes = [_vp, ctypes.c_int]
_lib.kmpar_profile_read.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(_i64),
                                    ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]
assert _lib.kmpar_sizeof_stats() == ctypes.sizeof(Stats), "kmpar_stats layout mismatch"

EXPORTED = ["kmpar_create", "kmpar_destroy", "kmpar_strerror", "kmpar_last_error",
            "kmpar_sizeof_stats", "kmpar_max_candidates", "kmpar_workspace_size", "kmpar_init",
            "kmpar_cost", "kmpar_assign", "lloyd_step", "kmpar_lloyd", "kmpar_profile_enable",
            "kmpar_profile_read", "kmpar_workspace_size_batched", "kmpar_init_batched",
            "kmpar_set_option", "kmpar_batch_tiles", "kmpar_cost_noalloc", "kmpar_kmeanspp",
            "kmpar_lloyd_until_stable", "kmpar_assign_sharded"]
NOALLOC_SCRATCH_BYTES = 64 << 20
OPT_RECLUSTER_PATH = 0
OPT_BATCH_AUTOTUNE = 1
OPT_SAMPLING = 2
SAMPLING_BERNOULLI, SAMPLING_EXACT = 0, 1

# kmpar_instance (include/kmpar.h), 64 bytes.
INSTANCE_DTYPE = np.dtype([("X", "<u8"), ("row_scale", "<u8"), ("centers", "<u8"), ("stats", "<u8"),
                           ("n", "<i8"), ("d", "<i4"), ("k", "<i4"), ("ell", "<f8"),
                           ("rounds", "<i4"), ("reserved", "<i4")])
assert INSTANCE_DTYPE.itemsize == 64
SLOT_FOLD_DIRECT, SLOT_SCREEN, SLOT_RESCAN, SLOT_BATCH_FOLD = 0, 1, 2, 3


class KmparError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"kmpar status {status} ({_lib.kmpar_strerror(status).decode()}): {msg}")
        self.status = status


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _on_stream(method):
    """Runs a call's own tensor work (output allocation, zero fills, input
    conversions) on the stream the call is given, so that it is ordered
    before the library's kernels there rather than racing them from the
    current stream."""
    @functools.wraps(method)
    def wrapped(self, *args, **kwargs):
        stream = kwargs.get("stream")
        if stream is None:
            return method(self, *args, **kwargs)
        with torch.cuda.stream(stream):
            return method(self, *args, **kwargs)
    return wrapped


def dtype_code(X: torch.Tensor, row_scale) -> int:
    if X.dtype == torch.float32:
        return F32
    if X.dtype == torch.bfloat16:
        return BF16
    if X.dtype in (torch.uint8, getattr(torch, "float8_e4m3fn", None)):
        if row_scale is None:
            raise ValueError("FP8 input needs a per-row scale")
        return FP8_E4M3
    raise TypeError(f"unsupported X dtype {X.dtype}")


def max_candidates(n: int, ell: float, rounds: int) -> int:
    out = _i64(0)
    rc = _lib.kmpar_max_candidates(n, ell, rounds, ctypes.byref(out))
    if rc:
        raise KmparError(rc, "kmpar_max_candidates")
    return int(out.value)


@dataclass
class InitResult:
    centers: torch.Tensor
    stats: dict
    trace: dict | None


class Context:
    """One library context on one device; caches its workspace."""

    def __init__(self, device: int | None = 0, mode: int = MODE_PLAIN_FP32):
        h = _vp()
        dev = -1 if device is None else int(device)
        rc = _lib.kmpar_create(dev, mode, ctypes.byref(h))
        if rc:
            raise KmparError(rc, "kmpar_create")
        self._h = h
        self.device = dev
        self.mode = mode
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:  # _lib is gone at interpreter exit
            _lib.kmpar_destroy(h)
            self._h = None

    # -------------------------------------------------------------- helpers
    def _check(self, rc: int, what: str):
        if rc:
            raise KmparError(rc, f"{what}: {_lib.kmpar_last_error(self._h).decode()}")

    def workspace_size(self, op, n, d, k, ell=1.0, rounds=0, dtype=F32) -> int:
        out = _sz(0)
        self._check(_lib.kmpar_workspace_size(self._h, op, n, d, k, ell, rounds, dtype,
                                              ctypes.byref(out)), "kmpar_workspace_size")
        return int(out.value)

    def _workspace(self, nbytes: int, device) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes or self._ws.device != device:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self._ws

    @staticmethod
    def _x(X, row_scale):
        if not X.is_contiguous():
            raise ValueError("X must be contiguous row-major")
        if X.dim() != 2:
            raise ValueError("X must be 2-D")
        return dtype_code(X, row_scale)

    def set_option(self, opt: int, value: int):
        self._check(_lib.kmpar_set_option(self._h, opt, int(value)), "kmpar_set_option")

    def batch_tiles(self) -> list:
        """[(dtype code, padded row length, fold variant)] the batched tuner
        has chosen so far: 1, 2, 4 or 8 candidates per step, or 200 for rows
        split over two waves."""
        cnt = _i32(0)
        self._check(_lib.kmpar_batch_tiles(self._h, None, None, None, 0, ctypes.byref(cnt)),
                    "kmpar_batch_tiles")
        n = cnt.value
        a, b, c = (np.zeros(max(n, 1), np.int32) for _ in range(3))
        self._check(_lib.kmpar_batch_tiles(self._h, a.ctypes.data, b.ctypes.data, c.ctypes.data, n,
                                           ctypes.byref(cnt)), "kmpar_batch_tiles")
        return [(int(a[i]), int(b[i]), int(c[i])) for i in range(n)]

    def profile(self, on: bool = True):
        self._check(_lib.kmpar_profile_enable(self._h, 1 if on else 0), "kmpar_profile_enable")

    def profile_read(self, slot: int = SLOT_FOLD_DIRECT) -> dict:
        """Launch count, summed milliseconds and summed point-center pairs of
        the timed launches of one distance kernel (clears them)."""
        la, ms, pr = _i64(0), _dbl(0), _dbl(0)
        self._check(_lib.kmpar_profile_read(self._h, slot, ctypes.byref(la), ctypes.byref(ms),
                                            ctypes.byref(pr)), "kmpar_profile_read")
        return {"launches": int(la.value), "ms": float(ms.value), "pairs": float(pr.value)}

    # ----------------------------------------------------------------- calls
    @_on_stream
    def init(self, X: torch.Tensor, k: int, ell: float, rounds: int, seed: int = 0,
             row_scale: torch.Tensor | None = None, trace: bool = False,
             stream=None, check: bool = True, allow_toofew: bool = False) -> InitResult:
        """kmpar_init.  With check (the default) the call synchronises, reads
        the stats and raises KmparError for any device status other than OK;
        allow_toofew accepts KMPAR_E_TOOFEW (fewer than k distinct candidates:
        the |C| centers found are returned).  check=False returns at once with
        the raw stats record (the caller reads it after synchronising)."""
        dt = self._x(X, row_scale)
        n, d = X.shape
        ws = self._workspace(self.workspace_size(OP_INIT, n, d, k, ell, rounds, dt), X.device)
        centers = torch.empty(k, d, dtype=torch.float32, device=X.device)
        st = torch.zeros(ctypes.sizeof(Stats), dtype=torch.uint8, device=X.device)
        tr = None
        trp = None
        if trace:
            cap = max_candidates(n, ell, rounds)
            i32 = dict(dtype=torch.int32, device=X.device)
            tr = {"cand_point": torch.empty(cap, **i32), "cand_weight": torch.empty(cap, **i32),
                  "center_cand": torch.full((k,), -1, **i32), "assign": torch.empty(n, **i32),
                  "d2": torch.empty(n, dtype=torch.float32, device=X.device)}
            trp = Trace(*(tr[f].data_ptr() for f in ("cand_point", "cand_weight", "center_cand",
                                                     "assign", "d2")))
        rc = _lib.kmpar_init(self._h, X.data_ptr(), _ptr(row_scale), dt, n, d, k, float(ell),
                             rounds, seed, centers.data_ptr(), ws.data_ptr(), ws.numel(),
                             st.data_ptr(), ctypes.byref(trp) if trp is not None else None,
                             _stream(stream))
        self._check(rc, "kmpar_init")
        if not check:
            return InitResult(centers, {"_raw": st}, tr)
        stats = parse_stats(st, rounds)
        check_status(stats["status"], allow_toofew, "kmpar_init")
        if tr is not None:
            nc = stats["n_candidates"]
            tr["cand_point"] = tr["cand_point"][:nc]
            tr["cand_weight"] = tr["cand_weight"][:nc]
            tr["center_cand"] = tr["center_cand"][:stats["n_centers"]]
        return InitResult(centers[:stats["n_centers"]], stats, tr)

    @_on_stream
    def cost(self, X, C, row_scale=None, stream=None) -> torch.Tensor:
        dt = self._x(X, row_scale)
        n, d = X.shape
        C = C.contiguous().float()
        ws = self._workspace(self.workspace_size(OP_COST, n, d, C.shape[0], dtype=dt), X.device)
        phi = torch.empty(1, dtype=torch.float64, device=X.device)
        self._check(_lib.kmpar_cost(self._h, X.data_ptr(), _ptr(row_scale), dt, n, d,
                                    C.data_ptr(), C.shape[0], phi.data_ptr(), ws.data_ptr(),
                                    ws.numel(), _stream(stream)), "kmpar_cost")
        return phi

    @_on_stream
    def cost_noalloc(self, X, C, row_scale=None, stream=None) -> torch.Tensor:
        """kmpar_cost_noalloc: the cost in the library's fixed scratch (no
        workspace).  C must already be contiguous float32 on the device."""
        dt = self._x(X, row_scale)
        n, d = X.shape
        if C.dtype != torch.float32 or not C.is_contiguous():
            raise ValueError("C must be contiguous float32")
        phi = torch.empty(1, dtype=torch.float64, device=X.device)
        self._check(_lib.kmpar_cost_noalloc(self._h, X.data_ptr(), _ptr(row_scale), dt, n, d,
                                            C.data_ptr(), C.shape[0], phi.data_ptr(),
                                            _stream(stream)), "kmpar_cost_noalloc")
        return phi

    @_on_stream
    def assign_sharded(self, X, C, shards: int, row_scale=None, stream=None):
        """kmpar_assign_sharded: nearest of m (up to 2^24) centers with the
        centers cut into `shards` slices merged by a packed minimum.
        Returns (assign, d2, phi)."""
        dt = self._x(X, row_scale)
        n, d = X.shape
        C = C.contiguous().float()
        m = C.shape[0]
        ws = self._workspace(self.workspace_size(OP_ASSIGN_SHARDED, n, d, m, dtype=dt), X.device)
        a = torch.empty(n, dtype=torch.int32, device=X.device)
        d2 = torch.empty(n, dtype=torch.float32, device=X.device)
        phi = torch.empty(1, dtype=torch.float64, device=X.device)
        self._check(_lib.kmpar_assign_sharded(self._h, X.data_ptr(), _ptr(row_scale), dt, n, d,
                                              C.data_ptr(), m, int(shards), a.data_ptr(),
                                              d2.data_ptr(), phi.data_ptr(), ws.data_ptr(),
                                              ws.numel(), _stream(stream)), "kmpar_assign_sharded")
        return a, d2, phi

    @_on_stream
    def assign(self, X, C, row_scale=None, stream=None):
        dt = self._x(X, row_scale)
        n, d = X.shape
        C = C.contiguous().float()
        ws = self._workspace(self.workspace_size(OP_ASSIGN, n, d, C.shape[0], dtype=dt), X.device)
        a = torch.empty(n, dtype=torch.int32, device=X.device)
        d2 = torch.empty(n, dtype=torch.float32, device=X.device)
        self._check(_lib.kmpar_assign(self._h, X.data_ptr(), _ptr(row_scale), dt, n, d,
                                      C.data_ptr(), C.shape[0], a.data_ptr(), d2.data_ptr(),
                                      ws.data_ptr(), ws.numel(), _stream(stream)), "kmpar_assign")
        return a, d2

    @_on_stream
    def init_batched(self, Xs, ks, ells, rounds: int, seed: int = 0, row_scales=None,
                     stream=None, check: bool = True, trace: bool = False,
                     allow_toofew: bool = False):
        """kmpar_init_batched: instance i uses Philox inst = i.  Returns
        (list of k_i x d_i center tensors, list of stats dicts, list of traces
        or None).  With check, any instance whose status is not OK (TOOFEW
        allowed with allow_toofew) raises KmparError naming the instance."""
        b = _batched_impl(self, Xs, ks, ells, rounds, seed, row_scales, stream, trace)
        self._batch_keep = b                      # device tables live until the next call
        traces = b.traces
        if not check:
            views = [b.centers[b.offs[i]:b.offs[i] + int(ks[i]) * Xs[i].shape[1]]
                     .view(int(ks[i]), Xs[i].shape[1]) for i in range(len(Xs))]
            return views, b.stats, traces
        centers, st = _batched_results(b, ks, Xs, rounds)
        for i, s_ in enumerate(st):
            check_status(s_["status"], allow_toofew, f"kmpar_init_batched instance {i}")
        if traces is not None:
            for t, s_ in zip(traces, st):
                t["cand_point"] = t["cand_point"][:s_["n_candidates"]]
                t["cand_weight"] = t["cand_weight"][:s_["n_candidates"]]
                t["center_cand"] = t["center_cand"][:s_["n_centers"]]
        return centers, st, traces

    @_on_stream
    def lloyd_step(self, X, C, row_scale=None, want_assign=False, stream=None):
        """Updates C (k x d FP32, contiguous) in place; returns (assign|None, phi)."""
        dt = self._x(X, row_scale)
        n, d = X.shape
        if C.dtype != torch.float32 or not C.is_contiguous():
            raise ValueError("C must be contiguous float32")
        k = C.shape[0]
        ws = self._workspace(self.workspace_size(OP_LLOYD, n, d, k, dtype=dt), X.device)
        a = torch.empty(n, dtype=torch.int32, device=X.device) if want_assign else None
        phi = torch.empty(1, dtype=torch.float64, device=X.device)
        self._check(_lib.lloyd_step(self._h, X.data_ptr(), _ptr(row_scale), dt, n, d,
                                    C.data_ptr(), k, _ptr(a), phi.data_ptr(), ws.data_ptr(),
                                    ws.numel(), _stream(stream)), "lloyd_step")
        return a, phi

    @_on_stream
    def kmeanspp(self, X, k: int, seed: int = 0, row_scale=None, stream=None, check: bool = True,
                 allow_toofew: bool = False):
        """kmpar_kmeanspp: k-means++ on all of X.  Returns (centers k x d,
        picks [k] int32, phi [k]: cost after each pick, stats) -- with check
        the call synchronises and the outputs are cut to the centers made."""
        dt = self._x(X, row_scale)
        n, d = X.shape
        ws = self._workspace(self.workspace_size(OP_KMEANSPP, n, d, k, dtype=dt), X.device)
        centers = torch.empty(k, d, dtype=torch.float32, device=X.device)
        picks = torch.full((k,), -1, dtype=torch.int32, device=X.device)
        phi = torch.zeros(k, dtype=torch.float64, device=X.device)
        st = torch.zeros(ctypes.sizeof(Stats), dtype=torch.uint8, device=X.device)
        self._check(_lib.kmpar_kmeanspp(self._h, X.data_ptr(), _ptr(row_scale), dt, n, d, k, seed,
                                        centers.data_ptr(), picks.data_ptr(), phi.data_ptr(),
                                        ws.data_ptr(), ws.numel(), st.data_ptr(),
                                        _stream(stream)), "kmpar_kmeanspp")
        if not check:
            return centers, picks, phi, {"_raw": st}
        stats = parse_stats(st, 0)
        check_status(stats["status"], allow_toofew, "kmpar_kmeanspp")
        m = stats["n_centers"]
        return centers[:m], picks[:m], phi[:m], stats

    @_on_stream
    def lloyd_until_stable(self, X, C, max_iters: int, row_scale=None, want_assign=False,
                           stream=None):
        """kmpar_lloyd_until_stable: Lloyd until the assignment no longer
        changes (at most max_iters updates).  Updates C in place; returns
        (updates made, final assignment|None, phi[updates + 1]).  The call
        synchronises the stream once per iteration."""
        dt = self._x(X, row_scale)
        n, d = X.shape
        if C.dtype != torch.float32 or not C.is_contiguous():
            raise ValueError("C must be contiguous float32")
        k = C.shape[0]
        ws = self._workspace(self.workspace_size(OP_LLOYD, n, d, k, dtype=dt), X.device)
        a = torch.empty(n, dtype=torch.int32, device=X.device) if want_assign else None
        phi = torch.empty(int(max_iters) + 1, dtype=torch.float64, device=X.device)
        it = _i32(-1)
        self._check(_lib.kmpar_lloyd_until_stable(self._h, X.data_ptr(), _ptr(row_scale), dt, n, d,
                                                  C.data_ptr(), k, int(max_iters), ctypes.byref(it),
                                                  _ptr(a), phi.data_ptr(), ws.data_ptr(), ws.numel(),
                                                  _stream(stream)), "kmpar_lloyd_until_stable")
        return int(it.value), a, phi[:int(it.value) + 1]

    @_on_stream
    def lloyd(self, X, C, iters: int, row_scale=None, want_assign=False, stream=None):
        """kmpar_lloyd: `iters` Lloyd iterations in one call (X prepared once).
        Updates C in place; returns (last assignment|None, phi[iters])."""
        dt = self._x(X, row_scale)
        n, d = X.shape
        if C.dtype != torch.float32 or not C.is_contiguous():
            raise ValueError("C must be contiguous float32")
        k = C.shape[0]
        ws = self._workspace(self.workspace_size(OP_LLOYD, n, d, k, dtype=dt), X.device)
        a = torch.empty(n, dtype=torch.int32, device=X.device) if want_assign else None
        phi = torch.empty(max(1, int(iters)), dtype=torch.float64, device=X.device)
        self._check(_lib.kmpar_lloyd(self._h, X.data_ptr(), _ptr(row_scale), dt, n, d,
                                     C.data_ptr(), k, int(iters), _ptr(a), phi.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _stream(stream)), "kmpar_lloyd")
        return a, phi[:max(0, int(iters))]


class CapturedInit:
    """kmpar_init captured once into a HIP graph (torch.cuda.CUDAGraph) and
    replayed; every replay rewrites `centers` and the raw stats record."""

    def __init__(self, ctx, X, k, ell, rounds, seed, row_scale=None):
        ctx.init(X, k=k, ell=ell, rounds=rounds, seed=seed, row_scale=row_scale)  # sizes the workspace
        torch.cuda.synchronize()
        self.rounds = rounds
        self.graph = torch.cuda.CUDAGraph()
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            with torch.cuda.graph(self.graph, stream=self.stream):
                r = ctx.init(X, k=k, ell=ell, rounds=rounds, seed=seed, row_scale=row_scale,
                             stream=self.stream, check=False)
        self.centers = r.centers
        self.stats_raw = r.stats["_raw"]
        self._keep = (ctx, X, row_scale)

    def replay(self):
        self.graph.replay()

    def stats(self) -> dict:
        return parse_stats(self.stats_raw, self.rounds)


def _batched_impl(ctx, Xs, ks, ells, rounds, seed, row_scales, stream, trace=False, launch=True,
                  shared_ws=True):
    count = len(Xs)
    dev = Xs[0].device
    dt = ctx._x(Xs[0], row_scales[0] if row_scales else None)
    desc = np.zeros(count, dtype=INSTANCE_DTYPE)
    offs = np.zeros(count + 1, dtype=np.int64)
    for i, X in enumerate(Xs):      # each instance's centers start 16-byte aligned
        offs[i + 1] = offs[i] + (int(ks[i]) * X.shape[1] + 3) // 4 * 4
    centers = torch.empty(max(1, int(offs[-1])), dtype=torch.float32, device=dev)
    ssz = ctypes.sizeof(Stats)
    stats = torch.zeros(count * ssz, dtype=torch.uint8, device=dev)
    for i, X in enumerate(Xs):
        if ctx._x(X, row_scales[i] if row_scales else None) != dt:
            raise ValueError("all instances must share one dtype")
        desc[i]["X"] = X.data_ptr()
        desc[i]["row_scale"] = row_scales[i].data_ptr() if row_scales else 0
        desc[i]["centers"] = centers.data_ptr() + 4 * int(offs[i])
        desc[i]["stats"] = stats.data_ptr() + i * ssz
        desc[i]["n"], desc[i]["d"], desc[i]["k"] = X.shape[0], X.shape[1], int(ks[i])
        desc[i]["ell"], desc[i]["rounds"] = float(ells[i]), int(rounds)
    desc_dev = torch.from_numpy(desc.view(np.uint8).copy()).to(dev)
    traces, tr_dev = None, None
    if trace:
        traces = []
        tarr = np.zeros((count, 5), dtype=np.uint64)
        for i, X in enumerate(Xs):
            cap = max_candidates(X.shape[0], float(ells[i]), int(rounds))
            i32 = dict(dtype=torch.int32, device=dev)
            t = {"cand_point": torch.empty(cap, **i32), "cand_weight": torch.empty(cap, **i32),
                 "center_cand": torch.full((int(ks[i]),), -1, **i32),
                 "assign": torch.empty(X.shape[0], **i32),
                 "d2": torch.empty(X.shape[0], dtype=torch.float32, device=dev)}
            traces.append(t)
            tarr[i] = [t[f].data_ptr() for f in ("cand_point", "cand_weight", "center_cand",
                                                 "assign", "d2")]
        tr_dev = torch.from_numpy(tarr.view(np.uint8).reshape(-1).copy()).to(dev)
    out = _sz(0)
    ctx._check(_lib.kmpar_workspace_size_batched(ctx._h, desc.ctypes.data, count, dt,
                                                 ctypes.byref(out)), "kmpar_workspace_size_batched")
    ws = ctx._workspace(int(out.value), dev) if shared_ws else \
        torch.empty(max(int(out.value), 256), dtype=torch.uint8, device=dev)
    batch = SimpleNamespace(desc=desc, desc_dev=desc_dev, count=count, dt=dt, ws=ws, tr_dev=tr_dev,
                            centers=centers, offs=offs, stats=stats, traces=traces)
    if launch:
        _batched_launch(ctx, batch, seed, stream)
    return batch


def _batched_launch(ctx, b, seed, stream):
    ctx._check(_lib.kmpar_init_batched(ctx._h, b.desc.ctypes.data, b.desc_dev.data_ptr(), b.count,
                                       b.dt, seed, b.ws.data_ptr(), b.ws.numel(),
                                       b.tr_dev.data_ptr() if b.tr_dev is not None else None,
                                       _stream(stream)),
               "kmpar_init_batched")


def _batched_results(b, ks, Xs, rounds):
    """Center views and parsed stats of a finished batch."""
    views = [b.centers[b.offs[i]:b.offs[i] + int(ks[i]) * Xs[i].shape[1]].view(int(ks[i]),
                                                                                Xs[i].shape[1])
             for i in range(len(Xs))]
    ssz = ctypes.sizeof(Stats)
    raw = b.stats.cpu()
    st = [parse_stats(raw[i * ssz:(i + 1) * ssz], rounds) for i in range(len(Xs))]
    return [v[:s_["n_centers"]] for v, s_ in zip(views, st)], st


class CapturedBatch:
    """kmpar_init_batched captured once into a HIP graph (torch.cuda.CUDAGraph)
    and replayed.  The instance table, the outputs and a workspace of its own
    are made before the capture, so the graph holds only the library's
    launches; every replay rewrites the centers and the stats records."""

    def __init__(self, ctx, Xs, ks, ells, rounds, seed, row_scales=None):
        self.batch = _batched_impl(ctx, Xs, ks, ells, rounds, seed, row_scales, None,
                                   launch=True, shared_ws=False)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            with torch.cuda.graph(self.graph, stream=self.stream):
                _batched_launch(ctx, self.batch, seed, self.stream)
        self._keep = (ctx, list(Xs), row_scales)
        self._shape = (list(ks), rounds)

    def replay(self):
        self.graph.replay()

    def results(self):
        """(list of k_i x d_i center tensors, list of stats dicts)."""
        ks, rounds = self._shape
        return _batched_results(self.batch, ks, self._keep[1], rounds)


def check_status(status: int, allow_toofew: bool, what: str):
    """Raises KmparError for a device status other than OK (and TOOFEW when
    allowed)."""
    if status == OK or (allow_toofew and status == E_TOOFEW):
        return
    raise KmparError(status, f"{what}: device status")


def parse_stats(st: torch.Tensor, rounds: int) -> dict:
    raw = st.cpu().numpy().tobytes()
    s = Stats.from_buffer_copy(raw)
    return {"phi": [s.phi[i] for i in range(rounds + 1)],
            "round_count": [s.round_count[i] for i in range(rounds + 1)],
            "n_candidates": s.n_candidates, "n_centers": s.n_centers, "status": s.status,
            "n_rescanned": s.n_rescanned, "flagged_draws": s.flagged_draws,
            "flagged_picks": s.flagged_picks, "flagged_argmins": s.flagged_argmins}
