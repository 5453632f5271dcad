"""Thin Python binding of the C ABI in include/blest.h (argument marshalling only).

Every traversal step runs in libblest.so's HIP kernels; torch provides device
memory and streams. torch is imported before the library is loaded so that
both share one HIP runtime. Missing library => ImportError-style RuntimeError:
there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from enum import IntEnum

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libblest.so")


class Status(IntEnum):
    OK = 0
    INVALID_ARG = -1
    INVALID_GRAPH = -2
    OUT_OF_RANGE = -3
    OOM = -4
    HIP = -5
    OVERFLOW = -6
    UNSUPPORTED = -7
    TIMEOUT = -8
    NO_DEVICE = -9
    IO = -10


class Policy(IntEnum):
    HEURISTIC = 0
    BVSS = 1
    PUSH = 2
    BOTTOM_UP = 3
    LEARNED = 4
    RANDOM = 5


class Update(IntEnum):
    LAZY = 0
    EAGER = 1
    AUTO = 2


class Engine(IntEnum):
    BVSS = 0
    PUSH = 1
    BOTTOM_UP = 2


class Reorder(IntEnum):
    NONE = 0
    RCM = 1
    AUTO = 2
    JACCARD = 3


MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_NPARAMS = 12, 64, 3, 5187


class BlestError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = Status(status) if status in Status._value2member_map_ else status
        super().__init__(f"{getattr(self.status, 'name', status)}: {message}")


class CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("row_ptr", ctypes.POINTER(ctypes.c_int32)),
                ("col_idx", ctypes.POINTER(ctypes.c_int32))]


class Opts(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_int32), ("tau", ctypes.c_int32), ("reorder", ctypes.c_int32),
                ("policy", ctypes.c_int32), ("eta", ctypes.c_float), ("block_size", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("persistent", ctypes.c_int32), ("wide_slices", ctypes.c_int32),
                ("prefilter", ctypes.c_int32), ("async_", ctypes.c_int32), ("msbfs_width", ctypes.c_int32),
                ("random_seed", ctypes.c_uint64), ("device", ctypes.c_int32), ("single_block", ctypes.c_int32),
                ("panel", ctypes.c_int32), ("panel_log2_rows", ctypes.c_int32),
                ("stage2_count_first", ctypes.c_int32), ("msbfs_graph", ctypes.c_int32),
                ("jaccard_window", ctypes.c_int32), ("update_scheme", ctypes.c_int32),
                ("directed", ctypes.c_int32), ("ms_ablation", ctypes.c_int32), ("ms_mfma", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class GraphStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("sigma", ctypes.c_int32), ("tau", ctypes.c_int32),
                ("slice_bytes", ctypes.c_int32), ("reordered", ctypes.c_int32), ("n_slice_sets", ctypes.c_int64),
                ("n_vss", ctypes.c_int64), ("n_slices", ctypes.c_int64), ("bvss_bytes", ctypes.c_int64),
                ("csr_bytes", ctypes.c_int64), ("work_bytes", ctypes.c_int64), ("grid_blocks", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("device", ctypes.c_int32),
                ("panel_log2_rows", ctypes.c_int32), ("update_scheme", ctypes.c_int32),
                ("directed", ctypes.c_int32), ("ms_graph_captures", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("u_div", ctypes.c_double)]


class LevelStat(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("engine", ctypes.c_int32), ("frontier", ctypes.c_int64),
                ("queue", ctypes.c_int64), ("queue_slices", ctypes.c_int64), ("frontier_edges", ctypes.c_int64),
                ("unvisited", ctypes.c_int64), ("unvisited_edges", ctypes.c_int64), ("deg_ge_32", ctypes.c_int64),
                ("deg_ge_1024", ctypes.c_int64), ("t_step_us", ctypes.c_double), ("t_stage1_us", ctypes.c_double),
                ("t_engine_us", ctypes.c_double * 3),
                ("mlp_fallback", ctypes.c_int32), ("bvss_panel", ctypes.c_int32), ("work", ctypes.c_int64),
                ("t_count_us", ctypes.c_double)]


class MsLevelStat(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("level", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("mlp_fallback", ctypes.c_int32), ("width", ctypes.c_int32), ("live", ctypes.c_int32),
                ("new_pairs", ctypes.c_int64), ("queue", ctypes.c_int64), ("queue_slices", ctypes.c_int64),
                ("unvisited_pairs", ctypes.c_int64), ("t_engine_us", ctypes.c_double * 2),
                ("feat", ctypes.c_float * 12)]


# Every exported symbol of the C ABI: name -> (restype, argtypes).
_vp, _i32, _i64, _u64, _f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
_p32 = ctypes.POINTER(ctypes.c_int32)
_p64 = ctypes.POINTER(ctypes.c_int64)
_pu64 = ctypes.POINTER(ctypes.c_uint64)
_pf32 = ctypes.POINTER(ctypes.c_float)
SIGNATURES = {
    "blest_status_str": (ctypes.c_char_p, [_i32]),
    "blest_last_error": (ctypes.c_char_p, []),
    "blest_default_opts": (None, [ctypes.POINTER(Opts)]),
    "blest_build": (_i32, [ctypes.POINTER(CSR), ctypes.POINTER(Opts), ctypes.POINTER(_vp)]),
    "blest_free": (None, [_vp]),
    "blest_bfs": (_i32, [_vp, _i32, _vp, _vp]),
    "blest_bfs_probe": (_i32, [_vp, _i32, _vp, _vp]),
    "blest_msbfs": (_i32, [_vp, _p32, _i32, _vp, _vp]),
    "blest_msbfs_batched": (_i32, [_vp, _p32, _i32, _p32, _i32, _vp, _vp]),
    "blest_msbfs_noalloc": (_i32, [_vp, _p32, _i32, _vp, _vp]),
    "blest_closeness": (_i32, [_vp, _p32, _i64, _vp, _vp, _vp, _vp]),
    "blest_far": (_i32, [_vp, _p32, _i64, _vp, _vp]),
    "blest_msbfs_probe": (_i32, [_vp, _p32, _i32, _p32, _i32, _vp, _vp]),
    "blest_msbfs_last_levels": (_i32, [_vp, ctypes.POINTER(MsLevelStat), _i32, _p32]),
    "blest_set_ms_switch_model": (_i32, [_vp, _pf32, _i32, _pf32, _pf32]),
    "blest_sync": (_i32, [_vp, _vp]),
    "blest_set_policy": (_i32, [_vp, _i32, _f32, _u64]),
    "blest_graph_info": (_i32, [_vp, ctypes.POINTER(GraphStats)]),
    "blest_closeness_resumable": (_i32, [_vp, _p32, _i64, _vp, _vp, _vp, ctypes.c_char_p, _i64, _p64, _vp]),
    "blest_reorder_jaccard": (_i32, [ctypes.POINTER(CSR), _i32, _i32, _p32]),
    "blest_update_divergence": (_i32, [ctypes.POINTER(CSR), _i32, _i32, ctypes.POINTER(ctypes.c_double)]),
    "blest_last_level_stats": (_i32, [_vp, ctypes.POINTER(LevelStat), _i32, _p32]),
    "blest_last_level_features": (_i32, [_vp, _pf32, _i32, _p32]),
    "blest_export_bvss": (_i32, [_vp, _p64, _p64, _p64, _p32, _pu64, _p32]),
    "blest_set_switch_model": (_i32, [_vp, _pf32, _i32, _pf32, _pf32]),
    "blest_set_switch_confidence": (_i32, [_vp, _f32]),
    "blest_set_log_work": (_i32, [_vp, _i32]),
    "blest_mlp_forward": (_i32, [_vp, _vp, _i32, _vp, _vp]),
    "blest_mlp_loss_grad": (_i32, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    "blest_mlp_adam": (_i32, [_vp, _vp, _vp, _vp, _i32, _i32, _f32, _f32, _f32, _f32, _vp]),
    "blest_mlp_train": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _i32, _f32, _u64, _vp, _vp]),
}

_lib = None


def lib():
    """Loads libblest.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build(); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != 0:
        msg = lib().blest_last_error().decode(errors="replace")
        raise BlestError(status, msg)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().blest_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        key = "async_" if k == "async" else k
        if not hasattr(o, key):
            raise TypeError(f"unknown option {k}")
        setattr(o, key, int(v) if key not in ("eta",) else float(v))
    return o


# ---- functions with the C ABI's names --------------------------------------

def blest_build(row_ptr, col, opts: Opts | None = None):
    """Builds a device graph from a host CSR; returns an opaque handle."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    csr = CSR(rp.size - 1, int(rp[-1]) if rp.size else 0, rp.ctypes.data_as(_p32), cl.ctypes.data_as(_p32))
    h = ctypes.c_void_p()
    _check(lib().blest_build(ctypes.byref(csr), ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)))
    return h


def blest_closeness_resumable(h, srcs, sums, reach, cc, path: str, max_sources: int = 0, stream=None) -> int:
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    done = ctypes.c_int64(0)
    _check(lib().blest_closeness_resumable(h, s.ctypes.data_as(_p32) if s.size else None, s.size, _ptr(sums),
                                           _ptr(reach), _ptr(cc), os.fsencode(path), int(max_sources),
                                           ctypes.byref(done), _stream(stream)))
    return done.value


def blest_update_divergence(row_ptr, col, sigma: int = 8, tau: int = 128) -> float:
    """Update divergence U_div of the CSR's BVSS as given (host only)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    csr = CSR(rp.size - 1, int(rp[-1]) if rp.size else 0, rp.ctypes.data_as(_p32), cl.ctypes.data_as(_p32))
    out = ctypes.c_double()
    _check(lib().blest_update_divergence(ctypes.byref(csr), int(sigma), int(tau), ctypes.byref(out)))
    return float(out.value)


def blest_reorder_jaccard(row_ptr, col, sigma: int = 8, window: int = 1024) -> np.ndarray:
    """JaccardWithWindows on the host: the new id of every vertex (int32[n])."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    if cl.size == 0:
        cl = np.zeros(1, dtype=np.int32)
    n = rp.size - 1
    out = np.empty(max(n, 1), dtype=np.int32)
    csr = CSR(n, int(rp[-1]) if rp.size else 0, rp.ctypes.data_as(_p32), cl.ctypes.data_as(_p32))
    _check(lib().blest_reorder_jaccard(ctypes.byref(csr), int(sigma), int(window), out.ctypes.data_as(_p32)))
    return out[:n]


def blest_free(h):
    lib().blest_free(h)


def blest_bfs(h, src: int, levels: torch.Tensor, stream=None):
    _check(lib().blest_bfs(h, int(src), _ptr(levels), _stream(stream)))


def blest_bfs_probe(h, src: int, levels: torch.Tensor, stream=None):
    _check(lib().blest_bfs_probe(h, int(src), _ptr(levels), _stream(stream)))


def blest_msbfs(h, srcs, levels: torch.Tensor, stream=None):
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    _check(lib().blest_msbfs(h, s.ctypes.data_as(_p32) if s.size else None, s.size, _ptr(levels), _stream(stream)))


def blest_msbfs_noalloc(h, srcs, levels: torch.Tensor, stream=None):
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    _check(lib().blest_msbfs_noalloc(h, s.ctypes.data_as(_p32) if s.size else None, s.size, _ptr(levels),
                                     _stream(stream)))


def blest_msbfs_batched(h, srcs, widths, levels: torch.Tensor, stream=None):
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    _check(lib().blest_msbfs_batched(h, s.ctypes.data_as(_p32) if s.size else None, s.size, w.ctypes.data_as(_p32),
                                     w.size, _ptr(levels), _stream(stream)))


def blest_msbfs_probe(h, srcs, widths, levels: torch.Tensor, stream=None):
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    _check(lib().blest_msbfs_probe(h, s.ctypes.data_as(_p32) if s.size else None, s.size, w.ctypes.data_as(_p32),
                                   w.size, _ptr(levels), _stream(stream)))


def blest_closeness(h, srcs, sums, reach, cc, stream=None):
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    _check(lib().blest_closeness(h, s.ctypes.data_as(_p32) if s.size else None, s.size, _ptr(sums), _ptr(reach),
                                 _ptr(cc), _stream(stream)))


def blest_far(h, srcs, far, stream=None):
    s = np.ascontiguousarray(srcs, dtype=np.int32)
    _check(lib().blest_far(h, s.ctypes.data_as(_p32) if s.size else None, s.size, _ptr(far), _stream(stream)))


def blest_sync(h, stream=None):
    _check(lib().blest_sync(h, _stream(stream)))


def blest_set_policy(h, policy: int, eta: float = 10.0, seed: int = 1):
    _check(lib().blest_set_policy(h, int(policy), float(eta), int(seed)))


def blest_set_switch_model(h, params, mean, std):
    p = np.ascontiguousarray(params, dtype=np.float32)
    mu = np.ascontiguousarray(mean, dtype=np.float32)
    sd = np.ascontiguousarray(std, dtype=np.float32)
    _check(lib().blest_set_switch_model(h, p.ctypes.data_as(_pf32), p.size, mu.ctypes.data_as(_pf32),
                                        sd.ctypes.data_as(_pf32)))


def blest_set_ms_switch_model(h, params, mean, std):
    p = np.ascontiguousarray(params, dtype=np.float32)
    mu = np.ascontiguousarray(mean, dtype=np.float32)
    sd = np.ascontiguousarray(std, dtype=np.float32)
    _check(lib().blest_set_ms_switch_model(h, p.ctypes.data_as(_pf32), p.size, mu.ctypes.data_as(_pf32),
                                           sd.ctypes.data_as(_pf32)))


def blest_set_switch_confidence(h, min_prob: float):
    _check(lib().blest_set_switch_confidence(h, float(min_prob)))


def blest_set_log_work(h, on: bool):
    _check(lib().blest_set_log_work(h, int(bool(on))))


def blest_mlp_forward(params, x, logits, stream=None):
    _check(lib().blest_mlp_forward(_ptr(params), _ptr(x), x.shape[0], _ptr(logits), _stream(stream)))


def blest_mlp_loss_grad(params, x, y, w, loss, grad, stream=None):
    _check(lib().blest_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(y), _ptr(w), x.shape[0], _ptr(loss), _ptr(grad),
                                     _stream(stream)))


def blest_mlp_adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().blest_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), int(t), lr, beta1, beta2,
                                eps, _stream(stream)))


def blest_mlp_train(params, m, v, x, y, w, batch, steps, lr, seed, loss_log=None, stream=None):
    _check(lib().blest_mlp_train(_ptr(params), _ptr(m), _ptr(v), _ptr(x), _ptr(y), _ptr(w), x.shape[0], int(batch),
                                 int(steps), float(lr), int(seed), _ptr(loss_log), _stream(stream)))


# ---- convenience wrapper ---------------------------------------------------

# Graphs still open; closed by an exit handler while the HIP runtime is intact.
_live_graphs = weakref.WeakSet()


@atexit.register
def _close_live_graphs():
    for g in list(_live_graphs):
        try:
            g.close()
        except Exception:
            pass


class Graph:
    """A device-resident BVSS graph. Methods allocate outputs with torch.

    Call close() (or use the graph as a context manager) to release its device
    memory. Graphs left open are closed by an exit handler that runs before the
    interpreter finalises; a graph collected during finalisation is not freed
    (the process is ending and the HIP runtime may already be torn down)."""

    def __init__(self, row_ptr, col, autotune: bool = False, family: str | None = None, **opts):
        """autotune=True: options the autotuner cached for the closest graph of
        this family (autotune.graph_options) fill in every option not given."""
        self._h = None
        self.autotuned = None
        if autotune:
            from . import autotune as _at
            tuned, self.autotuned = _at.graph_options(row_ptr, col, family)
            opts = {**tuned, **opts}
        self.opts = default_opts(**opts)
        self._h = blest_build(row_ptr, col, self.opts)
        _live_graphs.add(self)
        st = GraphStats()
        _check(lib().blest_graph_info(self._h, ctypes.byref(st)))
        self.n = st.n
        self.m = st.m
        self.device = torch.device("cuda", st.device)

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            _live_graphs.discard(self)
            blest_free(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check reachable while module globals
        # (sys among them) are being torn down
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        st = GraphStats()
        _check(lib().blest_graph_info(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in GraphStats._fields_ if k != "reserved"}

    def set_policy(self, policy, eta: float = 10.0, seed: int = 1):
        blest_set_policy(self._h, int(policy), eta, seed)

    def bfs(self, src: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        blest_bfs(self._h, src, out, stream)
        return out

    def bfs_probe(self, src: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        blest_bfs_probe(self._h, src, out, stream)
        return out

    def msbfs(self, srcs, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        k = len(srcs)
        if out is None:
            out = torch.empty((k, self.n), dtype=torch.int16, device=self.device)
        blest_msbfs(self._h, srcs, out, stream)
        return out

    def msbfs_noalloc(self, srcs, out: torch.Tensor, stream=None) -> torch.Tensor:
        """blest_msbfs_noalloc: the caller passes the (k, n) int16 output."""
        blest_msbfs_noalloc(self._h, srcs, out, stream)
        return out

    def msbfs_batched(self, srcs, widths, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        k = len(srcs)
        if out is None:
            out = torch.empty((k, self.n), dtype=torch.int16, device=self.device)
        blest_msbfs_batched(self._h, srcs, widths, out, stream)
        return out

    def msbfs_probe(self, srcs, widths, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        k = len(srcs)
        if out is None:
            out = torch.empty((k, self.n), dtype=torch.int16, device=self.device)
        blest_msbfs_probe(self._h, srcs, widths, out, stream)
        return out

    def ms_level_stats(self, cap: int = 1 << 16) -> list:
        """Per-level records of the last multi-source call (dicts; 'feat' is a list)."""
        buf = (MsLevelStat * cap)()
        nr = ctypes.c_int32()
        _check(lib().blest_msbfs_last_levels(self._h, buf, cap, ctypes.byref(nr)))
        out = []
        for i in range(min(cap, nr.value)):
            r = buf[i]
            d = {k: getattr(r, k) for k, _ in MsLevelStat._fields_ if k not in ("reserved", "t_engine_us", "feat")}
            d["t_engine_us"] = list(r.t_engine_us)
            d["feat"] = list(r.feat)
            out.append(d)
        return out

    def set_ms_switch_model(self, params, mean, std, min_confidence: float | None = None):
        """Multi-source network; min_confidence (if given) applies to both networks."""
        blest_set_ms_switch_model(self._h, params, mean, std)
        if min_confidence is not None:
            blest_set_switch_confidence(self._h, min_confidence)

    def closeness(self, srcs, stream=None):
        k = len(srcs)
        sums = torch.empty(k, dtype=torch.int64, device=self.device)
        reach = torch.empty(k, dtype=torch.int64, device=self.device)
        cc = torch.empty(k, dtype=torch.float64, device=self.device)
        blest_closeness(self._h, srcs, sums, reach, cc, stream)
        return sums, reach, cc

    def closeness_resumable(self, srcs, path: str, max_sources: int = 0, stream=None):
        """Closeness with a checkpoint file (blest_closeness_resumable).
        Returns (sums, reach, cc, done); outputs are valid for the first done sources."""
        k = len(srcs)
        sums = torch.zeros(max(k, 1), dtype=torch.int64, device=self.device)
        reach = torch.zeros(max(k, 1), dtype=torch.int64, device=self.device)
        cc = torch.zeros(max(k, 1), dtype=torch.float64, device=self.device)
        done = blest_closeness_resumable(self._h, srcs, sums, reach, cc, path, max_sources, stream)
        return sums[:k], reach[:k], cc[:k], done

    def far(self, srcs, stream=None):
        """Per-target distance sums of Eq. 4: int64[n], input vertex ids."""
        out = torch.empty(self.n, dtype=torch.int64, device=self.device)
        blest_far(self._h, srcs, out, stream)
        return out

    def sync(self, stream=None):
        blest_sync(self._h, stream)

    def level_stats(self, cap: int = 1 << 16) -> list:
        buf = (LevelStat * cap)()
        nl = ctypes.c_int32()
        _check(lib().blest_last_level_stats(self._h, buf, cap, ctypes.byref(nl)))
        out = []
        for i in range(min(cap, nl.value)):
            r = buf[i]
            d = {k: getattr(r, k) for k, _ in LevelStat._fields_ if k not in ("reserved", "t_engine_us")}
            d["t_engine_us"] = list(r.t_engine_us)
            out.append(d)
        return out

    def level_features(self, cap: int = 1 << 16) -> np.ndarray:
        nl = ctypes.c_int32()
        _check(lib().blest_last_level_features(self._h, None, 0, ctypes.byref(nl)))
        k = min(cap, nl.value)
        feat = np.zeros((max(k, 1), MLP_IN), dtype=np.float32)
        _check(lib().blest_last_level_features(self._h, feat.ctypes.data_as(_pf32), k, ctypes.byref(nl)))
        return feat[:k]

    def export_bvss(self) -> dict:
        st = self.info()
        ns, nv, nsl, n = st["n_slice_sets"], st["n_vss"], st["n_slices"], st["n"]
        real_ptrs = np.zeros(ns + 1, np.int64)
        v2r = np.zeros(max(nv, 1), np.int64)
        slice_ptr = np.zeros(ns + 1, np.int64)
        rows = np.zeros(max(nsl, 1), np.int32)
        masks = np.zeros(max(nsl, 1), np.uint64)
        perm = np.zeros(n, np.int32)
        _check(lib().blest_export_bvss(self._h, real_ptrs.ctypes.data_as(_p64), v2r.ctypes.data_as(_p64),
                                       slice_ptr.ctypes.data_as(_p64), rows.ctypes.data_as(_p32),
                                       masks.ctypes.data_as(_pu64), perm.ctypes.data_as(_p32)))
        return {"real_ptrs": real_ptrs, "v2r": v2r[:nv], "slice_ptr": slice_ptr, "slice_row": rows[:nsl],
                "slice_mask": masks[:nsl], "perm": perm}

    def set_switch_model(self, params, mean, std, min_confidence: float | None = None):
        blest_set_switch_model(self._h, params, mean, std)
        if min_confidence is not None:
            blest_set_switch_confidence(self._h, min_confidence)

    def set_log_work(self, on: bool = True):
        blest_set_log_work(self._h, on)


def set_default_switch_model(params, mean, std):
    blest_set_switch_model(None, params, mean, std)
