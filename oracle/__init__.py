"""CPU oracle for BVSS BFS -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may import
this package. The GPU library never imports or links it, and the two share no
code: this side is plain C (oracle.c) plus plain numpy in float64.

Contents, each following the passage cited beside it:
  bfs            -- hop distances, -1 = unreachable (Background, Eq. 1 and the
                    level definition after it; "infinity" read as -1)
  msbfs16        -- repeated BFS, int16 levels (Multi-Source BFS, Alg. 5)
  closeness      -- per-source sums/reach/cc (Closeness Centrality, Eq. 4/5,
                    normalised per source as (reach-1)/sum)
  far            -- per-target sums of Eq. 4
  components     -- connected-component labels (reach(s) = size of s's
                    component, the reachable set of Eq. 4's sums)
  certificate    -- O(m) proof that a level array is the BFS distance
  certificate_directed -- the same along arcs of a directed graph
  bvss           -- BVSS slices, realPtrs, virtualToReal (Section BVSS)
  get_vi         -- the multi-source index remap (Multi-Source BFS)
  switch_replay  -- Eq. 3 decisions replayed from oracle levels
  update_divergence -- U_div of a BVSS (Section "Boosting Cache Locality")
  mlp            -- float64 MLP forward/backward/Adam (oracle/mlp.py)
  jaccard        -- JaccardWithWindows over Python sets (oracle/jaccard.py,
                    Section "Increasing Compression Ratio")
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import mlp  # noqa: F401  (float64 MLP oracle)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, ERR_ARG, ERR_OOM, ERR_OVERFLOW = 0, -1, -4, -6


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .build import build
        build()
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    p32 = ctypes.POINTER(ctypes.c_int32)
    p16 = ctypes.POINTER(ctypes.c_int16)
    p64 = ctypes.POINTER(ctypes.c_int64)
    pu64 = ctypes.POINTER(ctypes.c_uint64)
    pf64 = ctypes.POINTER(ctypes.c_double)
    lib.oracle_bfs.argtypes = [i64, p32, p32, i32, p32]
    lib.oracle_bfs.restype = i32
    lib.oracle_msbfs16.argtypes = [i64, p32, p32, p32, i64, p16, i32]
    lib.oracle_msbfs16.restype = i32
    lib.oracle_closeness.argtypes = [i64, p32, p32, p32, i64, p64, p64, pf64, i32]
    lib.oracle_closeness.restype = i32
    lib.oracle_far.argtypes = [i64, p32, p32, p32, i64, p64, i32]
    lib.oracle_certificate_directed.argtypes = [i64, p32, p32, i32, p32, p64]
    lib.oracle_certificate_directed.restype = i32
    lib.oracle_far.restype = i32
    lib.oracle_certificate.argtypes = [i64, p32, p32, i32, p32, p64]
    lib.oracle_certificate.restype = i32
    lib.oracle_bvss_count.argtypes = [i64, p32, p32, i32, i32, p64, p64]
    lib.oracle_bvss_count.restype = i32
    lib.oracle_bvss_fill.argtypes = [i64, p32, p32, i32, i32, p64, p64, p64, p32, pu64]
    lib.oracle_bvss_fill.restype = i32
    lib.oracle_components.argtypes = [i64, p32, p32, p32]
    lib.oracle_components.restype = i64
    _lib = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _csr(rp, col):
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.int32)
    return rp, col, rp.size - 1


def _threads(t):
    return t if t and t > 0 else max(1, min(os.cpu_count() or 1, 64))


def bfs(rp, col, src: int) -> np.ndarray:
    """int32 hop distances from src; -1 where unreachable."""
    rp, col, n = _csr(rp, col)
    lev = np.empty(n, dtype=np.int32)
    r = _load().oracle_bfs(n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), int(src), _ptr(lev, ctypes.c_int32))
    if r < 0:
        raise ValueError(f"oracle_bfs failed ({r})")
    return lev


def msbfs16(rp, col, srcs, threads: int = 0) -> np.ndarray:
    """int16 (k, n) source-major levels; raises OverflowError past 32767."""
    rp, col, n = _csr(rp, col)
    srcs = np.ascontiguousarray(srcs, dtype=np.int32)
    k = srcs.size
    out = np.empty((k, n), dtype=np.int16)
    if k == 0:
        return out
    r = _load().oracle_msbfs16(n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(srcs, ctypes.c_int32), k,
                               _ptr(out, ctypes.c_int16), _threads(threads))
    if r == ERR_OVERFLOW:
        raise OverflowError("a distance exceeds int16")
    if r < 0:
        raise ValueError(f"oracle_msbfs16 failed ({r})")
    return out


def closeness(rp, col, srcs, threads: int = 0):
    """(sums int64[k], reach int64[k], cc float64[k]) per source."""
    rp, col, n = _csr(rp, col)
    srcs = np.ascontiguousarray(srcs, dtype=np.int32)
    k = srcs.size
    sums = np.zeros(k, dtype=np.int64)
    reach = np.zeros(k, dtype=np.int64)
    cc = np.zeros(k, dtype=np.float64)
    if k == 0:
        return sums, reach, cc
    r = _load().oracle_closeness(n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(srcs, ctypes.c_int32), k,
                                 _ptr(sums, ctypes.c_int64), _ptr(reach, ctypes.c_int64), _ptr(cc, ctypes.c_double),
                                 _threads(threads))
    if r < 0:
        raise ValueError(f"oracle_closeness failed ({r})")
    return sums, reach, cc


def components(rp, col) -> np.ndarray:
    """Component label of every vertex, components numbered by smallest vertex."""
    rp, col, n = _csr(rp, col)
    lab = np.empty(n, dtype=np.int32)
    r = _load().oracle_components(n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(lab, ctypes.c_int32))
    if r < 0:
        raise ValueError(f"oracle_components failed ({r})")
    return lab


def far(rp, col, srcs, threads: int = 0) -> np.ndarray:
    """Per-target sums far[u] = sum_s d(s, u) over finite pairs (Eq. 4)."""
    rp, col, n = _csr(rp, col)
    srcs = np.ascontiguousarray(srcs, dtype=np.int32)
    out = np.zeros(n, dtype=np.int64)
    if srcs.size == 0:
        return out
    r = _load().oracle_far(n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(srcs, ctypes.c_int32), srcs.size,
                           _ptr(out, ctypes.c_int64), _threads(threads))
    if r < 0:
        raise ValueError(f"oracle_far failed ({r})")
    return out


CERT_REASONS = {0: "ok", 1: "bad source level", 2: "edge with one end unreached", 3: "edge spans >1 level",
                4: "reached vertex without parent"}


def certificate(rp, col, src: int, levels):
    """(code, vertex): code 0 iff levels are exactly the BFS distances from src."""
    rp, col, n = _csr(rp, col)
    lev = np.ascontiguousarray(levels, dtype=np.int32)
    if lev.size != n:
        raise ValueError("levels has the wrong length")
    where = np.zeros(1, dtype=np.int64)
    r = _load().oracle_certificate(n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), int(src),
                                   _ptr(lev, ctypes.c_int32), _ptr(where, ctypes.c_int64))
    if r < 0:
        raise ValueError(f"oracle_certificate failed ({r})")
    return int(r), int(where[0])


def certificate_directed(rp, col, src: int, levels):
    """(code, where) for a directed graph (rp/col hold out-arcs); code 0 iff
    levels are the hop distances from src along arcs (oracle.c documents the
    four conditions)."""
    rp, col, n = _csr(rp, col)
    lev = np.ascontiguousarray(levels, dtype=np.int32)
    where = np.zeros(1, np.int64)
    r = _load().oracle_certificate_directed(n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), int(src),
                                            _ptr(lev, ctypes.c_int32), _ptr(where, ctypes.c_int64))
    if r < 0:
        raise ValueError(f"oracle_certificate_directed failed ({r})")
    return int(r), int(where[0])


def bvss(rp, col, sigma: int = 8, tau: int = 128):
    """BVSS arrays as a dict: real_ptrs, v2r, slice_ptr, slice_row, slice_mask."""
    rp, col, n = _csr(rp, col)
    lib = _load()
    ns_, nv_ = np.zeros(1, np.int64), np.zeros(1, np.int64)
    r = lib.oracle_bvss_count(n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), sigma, tau,
                              _ptr(ns_, ctypes.c_int64), _ptr(nv_, ctypes.c_int64))
    if r < 0:
        raise ValueError(f"oracle_bvss_count failed ({r})")
    nsets = (n + sigma - 1) // sigma
    nsl, nv = int(ns_[0]), int(nv_[0])
    real_ptrs = np.zeros(nsets + 1, np.int64)
    v2r = np.zeros(max(nv, 1), np.int64)
    slice_ptr = np.zeros(nsets + 1, np.int64)
    rows = np.zeros(max(nsl, 1), np.int32)
    masks = np.zeros(max(nsl, 1), np.uint64)
    r = lib.oracle_bvss_fill(n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), sigma, tau,
                             _ptr(real_ptrs, ctypes.c_int64), _ptr(v2r, ctypes.c_int64), _ptr(slice_ptr, ctypes.c_int64),
                             _ptr(rows, ctypes.c_int32), _ptr(masks, ctypes.c_uint64))
    if r < 0:
        raise ValueError(f"oracle_bvss_fill failed ({r})")
    return {"real_ptrs": real_ptrs, "v2r": v2r[:nv], "slice_ptr": slice_ptr, "slice_row": rows[:nsl],
            "slice_mask": masks[:nsl], "n_slice_sets": nsets, "n_vss": nv, "n_slices": nsl}


def update_divergence(rp, col, sigma: int = 8, tau: int = 128, theta: int | None = None) -> float:
    """Update divergence U_div (Section "Boosting Cache Locality").

    Each VSS is read as the paper's matrix of tau / theta rows and theta
    columns (32 x 4 at tau = 128), slice j of the VSS in column j mod theta.
    Column divergence: standard deviation (population form) of the row ids of
    the column's slices with a nonzero mask; set divergence of a VSS: mean
    over its non-empty columns; U_div: mean over all N_v VSSs. Computed from
    the oracle's own BVSS, one VSS at a time."""
    theta = max(1, tau // 32) if theta is None else theta
    b = bvss(rp, col, sigma, tau)
    rows = b["slice_row"].astype(np.float64)
    masks = b["slice_mask"]
    sp, real_ptrs, v2r = b["slice_ptr"], b["real_ptrs"], b["v2r"]
    nv = int(b["n_vss"])
    if nv == 0:
        return 0.0
    total = 0.0
    for v in range(nv):
        s = int(v2r[v])
        first = int(sp[s]) + (v - int(real_ptrs[s])) * tau
        last = min(first + tau, int(sp[s + 1]))
        col_div = []
        for c in range(theta):
            idx = np.arange(first + c, last, theta)
            idx = idx[masks[idx] != 0]
            if idx.size:
                col_div.append(float(np.std(rows[idx])))
        total += float(np.mean(col_div))
    return total / nv


def get_vi(u, sigma: int, rho: int):
    """Multi-source vertex index remap: (u mod sigma) * rho + floor(u / sigma)."""
    u = np.asarray(u, dtype=np.int64)
    return (u % sigma) * rho + u // sigma


def level_counts(levels) -> np.ndarray:
    """cnt[l] = number of vertices at level l (unreached excluded)."""
    lev = np.asarray(levels)
    lev = lev[lev >= 0]
    if lev.size == 0:
        return np.zeros(0, dtype=np.int64)
    return np.bincount(lev.astype(np.int64)).astype(np.int64)


def switch_replay(levels, rp, real_ptrs, sigma: int, eta: float = 10.0):
    """Eq. 3 decisions replayed from exact levels.

    Before exploring from frontier level l (l = 0 .. max level), the queue holds
    every VSS of every slice set that contains a level-l vertex, so
    |Q_l| = sum of (real_ptrs[s+1] - real_ptrs[s]) over those slice sets, and
    #unvisited_l = n - #{v : level[v] <= l}. The step is bottom-up iff
    #unvisited_l < eta * |Q_l|. Returns a list of dicts, one per level.
    """
    lev = np.asarray(levels, dtype=np.int64)
    n = lev.size
    real_ptrs = np.asarray(real_ptrs, dtype=np.int64)
    nv_per_set = real_ptrs[1:] - real_ptrs[:-1]
    maxl = int(lev.max()) if (lev >= 0).any() else -1
    out = []
    visited = 0
    for l in range(maxl + 1):
        fr = np.nonzero(lev == l)[0]
        visited += fr.size
        sets = np.unique(fr // sigma)
        q = int(nv_per_set[sets].sum())
        unv = n - visited
        out.append({"level": l, "frontier": int(fr.size), "queue": q, "unvisited": int(unv),
                    "bottom_up": bool(unv < eta * q)})
    return out
