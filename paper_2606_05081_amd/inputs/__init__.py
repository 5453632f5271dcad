"""Seeded synthetic graph inputs (R-MAT, grid with deletions, Erdos-Renyi).

A module of its own: it manufactures inputs and holds none of the BFS
arithmetic. Both the GPU library's callers and the CPU oracle take their
graphs from here. Graphs are returned as (row_ptr int32[n+1], col int32[m])
numpy arrays of an undirected simple graph with sorted rows (the directed
generators: out-neighbour rows of a simple digraph).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgraphgen.so")

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    p32 = ctypes.POINTER(ctypes.c_int32)
    lib.gg_free.argtypes = [vp]
    lib.gg_n.argtypes = [vp]
    lib.gg_n.restype = i64
    lib.gg_m.argtypes = [vp]
    lib.gg_m.restype = i64
    lib.gg_row_ptr.argtypes = [vp]
    lib.gg_row_ptr.restype = p32
    lib.gg_col.argtypes = [vp]
    lib.gg_col.restype = p32
    lib.gg_rmat.argtypes = [i32, i32, f64, f64, f64, u64, i32, i32]
    lib.gg_rmat.restype = vp
    lib.gg_grid.argtypes = [i32, f64, u64, i32, i32]
    lib.gg_grid.restype = vp
    lib.gg_erdos_renyi.argtypes = [i64, i64, u64, i32]
    lib.gg_erdos_renyi.restype = vp
    lib.gg_from_pairs.argtypes = [i64, i64, p32, p32]
    lib.gg_from_pairs.restype = vp
    lib.gg_directed_from_pairs.argtypes = [i64, i64, p32, p32, i32]
    lib.gg_directed_from_pairs.restype = vp
    lib.gg_rmat_directed.argtypes = [i32, i32, f64, f64, f64, u64, i32, i32, i32]
    lib.gg_rmat_directed.restype = vp
    lib.gg_permute.argtypes = [i64, p32, p32, u64, p32, i32]
    lib.gg_permute.restype = vp
    lib.gg_sources.argtypes = [i64, p32, i64, u64, i32, i32, p32]
    lib.gg_sources.restype = i64
    _lib = lib
    return lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _take(h):
    lib = _load()
    if not h:
        raise MemoryError("graph generation failed (bad arguments or out of memory)")
    try:
        n, m = lib.gg_n(h), lib.gg_m(h)
        rp = np.ctypeslib.as_array(lib.gg_row_ptr(h), shape=(n + 1,)).copy()
        col = np.ctypeslib.as_array(lib.gg_col(h), shape=(max(m, 1),))[:m].copy()
    finally:
        lib.gg_free(h)
    return rp, col


def rmat(scale: int, edgefactor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, permute: bool = True, threads: int = 0):
    """R-MAT graph on 2**scale vertices from edgefactor * 2**scale samples."""
    return _take(_load().gg_rmat(scale, edgefactor, a, b, c, seed, int(permute), threads))


def grid(side: int, p_delete: float = 0.10, seed: int = 1, permute: bool = True, threads: int = 0):
    """side x side 4-neighbour grid, each edge deleted with probability p_delete."""
    return _take(_load().gg_grid(side, p_delete, seed, int(permute), threads))


def erdos_renyi(n: int, npairs: int, seed: int = 1, threads: int = 0):
    """npairs uniform random pairs on n vertices, symmetrised and deduplicated."""
    return _take(_load().gg_erdos_renyi(n, npairs, seed, threads))


def from_pairs(n: int, us, vs):
    """Canonical CSR of the undirected pairs (us[i], vs[i])."""
    us = np.ascontiguousarray(us, dtype=np.int32)
    vs = np.ascontiguousarray(vs, dtype=np.int32)
    if us.shape != vs.shape:
        raise ValueError("us and vs differ in length")
    return _take(_load().gg_from_pairs(n, us.size, _p32(us), _p32(vs)))


def directed_from_pairs(n: int, us, vs):
    """CSR of the arcs us[i] -> vs[i] (sorted rows, self loops and duplicates dropped)."""
    us = np.ascontiguousarray(us, dtype=np.int32)
    vs = np.ascontiguousarray(vs, dtype=np.int32)
    if us.shape != vs.shape:
        raise ValueError("us and vs differ in length")
    return _take(_load().gg_directed_from_pairs(n, us.size, _p32(us), _p32(vs), 1))


def rmat_directed(scale: int, seed: int, edgefactor: int = 16, permute: bool = True, threads: int = 0):
    """Directed R-MAT: the same samples as rmat_graph kept as arcs u -> v."""
    a, b, c = RMAT_ABC
    return _take(_load().gg_rmat_directed(scale, edgefactor, a, b, c, seed, int(permute), threads, 1))


def permute(row_ptr, col, seed: int, threads: int = 0):
    """Relabels a CSR by a seeded random permutation. Returns (rp, col, perm) with perm[old] = new."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n = row_ptr.size - 1
    perm = np.empty(n, dtype=np.int32)
    h = _load().gg_permute(n, _p32(row_ptr), _p32(col if col.size else np.zeros(1, np.int32)), seed, _p32(perm), threads)
    rp2, col2 = _take(h)
    return rp2, col2, perm


def sources(row_ptr, count: int, seed: int, nonzero_degree: bool = True, distinct: bool = True):
    """Seeded source vertices (int32). Raises if not enough eligible vertices."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    out = np.empty(max(count, 1), dtype=np.int32)
    got = _load().gg_sources(row_ptr.size - 1, _p32(row_ptr), count, seed, int(nonzero_degree), int(distinct), _p32(out))
    if got != count:
        raise ValueError("not enough eligible source vertices")
    return out[:count]


# Workload recipes: the graph shapes of the paper's workload classes
# (Kronecker/social, uniform random, road-like), with fixed seeds.
RMAT_ABC = (0.57, 0.19, 0.19)


def rmat_graph(scale: int, seed: int, edgefactor: int = 16):
    a, b, c = RMAT_ABC
    return rmat(scale, edgefactor, a, b, c, seed=seed, permute=True)


def grid_graph(side: int, seed: int):
    return grid(side, 0.10, seed=seed, permute=True)


def er_graph(log2n: int, seed: int, mean_degree: int = 16):
    n = 1 << log2n
    return erdos_renyi(n, n * mean_degree // 2, seed=seed)
