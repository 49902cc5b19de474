"""Seeded synthetic graph inputs shared by the CPU oracle and the GPU path.

Everything here builds inputs only (edge samples, symmetric CSR, priority
arrays); none of the colouring method's arithmetic lives in this module.
The heavy generators (uniform pairs, R-MAT, CSR assembly) are plain C in
``graphgen.c`` behind ctypes; the structured graphs are small numpy builders.

Input recipes follow the paper's test-graph section (R-MAT with parameters
(a, b, c, d), self-loops and duplicate edges removed) and the workloads the
colouring is measured on (uniform random graphs, R-MAT, stencil grids with
random extra edges, random geometric graphs).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import List, NamedTuple, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_SRC = os.path.join(_HERE, "graphgen.c")

_lib = None


def build() -> str:
    """Compile graphgen.c into libgraphgen.so (gcc, OpenMP)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.gg_hash_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, u64p]
    lib.gg_hash_u64.restype = None
    lib.gg_uniform_pairs.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, i32p, i32p]
    lib.gg_uniform_pairs.restype = None
    lib.gg_rmat_pairs.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_double, i32p, i32p]
    lib.gg_rmat_pairs.restype = None
    lib.gg_extra_pairs.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, i32p, i32p]
    lib.gg_extra_pairs.restype = None
    lib.gg_unit_points.argtypes = [ctypes.c_uint64, ctypes.c_int32, f64p, f64p]
    lib.gg_unit_points.restype = None
    lib.gg_rgg_pairs.argtypes = [ctypes.c_int32, f64p, f64p, ctypes.c_double, i32p, i32p, ctypes.c_int64]
    lib.gg_rgg_pairs.restype = ctypes.c_int64
    lib.gg_build_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, i32p]
    lib.gg_build_csr.restype = ctypes.c_int64
    lib.gg_num_threads.argtypes = []
    lib.gg_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class CSR(NamedTuple):
    """Symmetric CSR: rows sorted ascending, no self-loops, no duplicates."""
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col_idx: np.ndarray  # int32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def edges(self) -> int:
        """Undirected edge count m = nnz / 2."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def from_pairs(n: int, src: np.ndarray, dst: np.ndarray) -> CSR:
    """Symmetrise, drop self-loops, sort rows, merge duplicates."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = int(src.shape[0])
    if m and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("endpoint out of range")
    lib = _load()
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.empty(max(2 * m, 1), dtype=np.int32)
    nnz = lib.gg_build_csr(n, m, _p(src, ctypes.c_int32), _p(dst, ctypes.c_int32),
                           _p(row_ptr, ctypes.c_int32), _p(col, ctypes.c_int32))
    if nnz < 0:
        raise MemoryError("CSR assembly failed (nnz >= 2^31 or out of memory)")
    col_idx = col[:nnz].copy() if nnz < col.shape[0] // 2 else col[:nnz]
    return CSR(n, row_ptr, col_idx)


def hash_u64(seed: int, tag: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gg_hash_u64(seed, tag, count, _p(out, ctypes.c_uint64))
    return out


def uniform(n: int, m: int, seed: int) -> CSR:
    """m endpoint pairs drawn uniformly on [0, n); loops and duplicates removed
    after drawing (no resampling)."""
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _load().gg_uniform_pairs(seed, n, m, _p(src, ctypes.c_int32), _p(dst, ctypes.c_int32))
    return from_pairs(n, src, dst)


def rmat(scale: int, edge_factor: int, abcd: Sequence[float], seed: int) -> CSR:
    """R-MAT with edge_factor * 2^scale samples; quadrant bits most-significant
    first, no noise; symmetrised, deduplicated, self-loops removed."""
    a, b, c = float(abcd[0]), float(abcd[1]), float(abcd[2])
    n = 1 << scale
    m = edge_factor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _load().gg_rmat_pairs(seed, scale, m, a, b, c, _p(src, ctypes.c_int32), _p(dst, ctypes.c_int32))
    g = from_pairs(n, src, dst)
    del src, dst
    return g


def random_priority(n: int, seed: int) -> np.ndarray:
    """A seeded random permutation of [0, n) as uint32 priorities."""
    h = hash_u64(seed, 77, n)
    order = np.argsort(h, kind="stable")
    pri = np.empty(n, dtype=np.uint32)
    pri[order] = np.arange(n, dtype=np.uint32)
    return pri


def random_keys(n: int, seed: int, bits: int = 32) -> np.ndarray:
    """Seeded uint32 priorities with possible ties (top `bits` bits kept)."""
    h = hash_u64(seed, 78, n)
    return (h >> np.uint64(64 - bits)).astype(np.uint32)


# ---------------------------------------------------------------------------
# Structured graphs (small numpy builders)
# ---------------------------------------------------------------------------

def empty(n: int) -> CSR:
    return CSR(n, np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32))


def path(n: int) -> CSR:
    v = np.arange(n - 1, dtype=np.int32)
    return from_pairs(n, v, v + 1)


def cycle(n: int) -> CSR:
    v = np.arange(n, dtype=np.int32)
    return from_pairs(n, v, (v + 1) % n)


def complete(n: int) -> CSR:
    i, j = np.triu_indices(n, 1)
    return from_pairs(n, i.astype(np.int32), j.astype(np.int32))


def star(n: int, center: int = 0) -> CSR:
    leaves = np.array([v for v in range(n) if v != center], dtype=np.int32)
    return from_pairs(n, np.full(leaves.shape, center, dtype=np.int32), leaves)


def complete_bipartite(p: int, q: int) -> CSR:
    i, j = np.meshgrid(np.arange(p), np.arange(p, p + q), indexing="ij")
    return from_pairs(p + q, i.ravel().astype(np.int32), j.ravel().astype(np.int32))


def _stencil_offsets(dim: int, full: bool) -> List[Tuple[int, ...]]:
    """Half of the stencil's neighbour offsets (lexicographically positive)."""
    offs = []
    rng = [-1, 0, 1]
    import itertools
    for d in itertools.product(rng, repeat=dim):
        if all(x == 0 for x in d):
            continue
        if not full and sum(abs(x) for x in d) != 1:
            continue
        if d > tuple(0 for _ in d):
            offs.append(d)
    return offs


def grid(shape: Sequence[int], full: bool = False) -> CSR:
    """Row-major stencil grid: star stencil (2D 5-point, 3D 7-point) when
    full=False, box stencil (2D 9-point, 3D 27-point) when full=True."""
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    n = int(np.prod(shape))
    coords = np.indices(shape).reshape(dim, -1)
    ids = np.arange(n, dtype=np.int64)
    src_l, dst_l = [], []
    for d in _stencil_offsets(dim, full):
        nb = coords + np.array(d).reshape(dim, 1)
        ok = np.ones(n, dtype=bool)
        for k in range(dim):
            ok &= (nb[k] >= 0) & (nb[k] < shape[k])
        nid = np.ravel_multi_index(tuple(nb[:, ok]), shape)
        src_l.append(ids[ok])
        dst_l.append(nid)
    if src_l:
        src = np.concatenate(src_l).astype(np.int32)
        dst = np.concatenate(dst_l).astype(np.int32)
    else:
        src = dst = np.zeros(0, dtype=np.int32)
    return from_pairs(n, src, dst)


def grid_with_extra(shape: Sequence[int], full: bool, extra_frac: float, seed: int) -> CSR:
    """Stencil grid plus extra_frac * (its edge count) uniform random edges."""
    g = grid(shape, full)
    n = g.n
    m_extra = int(round(extra_frac * g.edges))
    src = np.repeat(np.arange(n, dtype=np.int32), np.diff(g.row_ptr))
    es = np.empty(m_extra, dtype=np.int32)
    ed = np.empty(m_extra, dtype=np.int32)
    if m_extra:
        _load().gg_extra_pairs(seed, n, m_extra, _p(es, ctypes.c_int32), _p(ed, ctypes.c_int32))
    return from_pairs(n, np.concatenate([src, es]), np.concatenate([g.col_idx, ed]))


def rgg(n: int, mean_degree: float, seed: int) -> CSR:
    """Random geometric graph: n uniform points in the unit square, edge when
    the distance is at most r = sqrt(k / (pi n))."""
    x = np.empty(n, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    lib = _load()
    lib.gg_unit_points(seed, n, _p(x, ctypes.c_double), _p(y, ctypes.c_double))
    r = math.sqrt(mean_degree / (math.pi * n))
    cap = int(n * mean_degree) + 1024
    while True:
        src = np.empty(cap, dtype=np.int32)
        dst = np.empty(cap, dtype=np.int32)
        cnt = lib.gg_rgg_pairs(n, _p(x, ctypes.c_double), _p(y, ctypes.c_double), r,
                               _p(src, ctypes.c_int32), _p(dst, ctypes.c_int32), cap)
        if cnt >= 0:
            break
        cap *= 2
    return from_pairs(n, src[:cnt], dst[:cnt])


# ---------------------------------------------------------------------------
# Batched workload: many small graphs of uneven size
# ---------------------------------------------------------------------------

BATCH_KINDS = ("grid2d5", "grid2d9", "grid3d7", "grid3d27", "rgg")


class BatchSpec(NamedTuple):
    kind: str
    n_target: int
    seed: int
    mean_degree: float


def batch_specs(count: int, seed: int, log2_lo: float = 8.0, log2_hi: float = 16.0) -> List[BatchSpec]:
    """Per-graph recipe: n log-uniform in [2^lo, 2^hi], kind uniform over the
    five families, RGG mean degree uniform in [6, 27]."""
    h = hash_u64(seed, 91, 4 * count)
    specs = []
    for i in range(count):
        u0 = float(h[4 * i] >> np.uint64(11)) / float(1 << 53)
        u1 = int(h[4 * i + 1] % np.uint64(len(BATCH_KINDS)))
        u2 = float(h[4 * i + 2] >> np.uint64(11)) / float(1 << 53)
        n_t = int(round(2.0 ** (log2_lo + (log2_hi - log2_lo) * u0)))
        specs.append(BatchSpec(BATCH_KINDS[u1], n_t, int(h[4 * i + 3] >> np.uint64(1)), 6.0 + 21.0 * u2))
    return specs


def batch_graph(spec: BatchSpec) -> CSR:
    kind, n_t = spec.kind, spec.n_target
    if kind == "rgg":
        return rgg(n_t, spec.mean_degree, spec.seed)
    dim = 2 if kind.startswith("grid2d") else 3
    full = kind in ("grid2d9", "grid3d27")
    side = max(2, int(round(n_t ** (1.0 / dim))))
    return grid_with_extra((side,) * dim, full, 0.05, spec.seed)


class Batch(NamedTuple):
    """Graphs concatenated: local ids per graph, offsets into the arrays."""
    graphs: List[CSR]
    vtx_off: np.ndarray   # int64[G+1]
    edge_off: np.ndarray  # int64[G+1]
    row_ptr: np.ndarray   # int32[V_total + G]: each graph's n+1 local offsets
    col_idx: np.ndarray   # int32[nnz_total]: local neighbour ids


def concat(graphs: Sequence[CSR]) -> Batch:
    G = len(graphs)
    vtx_off = np.zeros(G + 1, dtype=np.int64)
    edge_off = np.zeros(G + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx_off[i + 1] = vtx_off[i] + g.n
        edge_off[i + 1] = edge_off[i] + g.nnz
    row_ptr = np.concatenate([g.row_ptr for g in graphs]) if G else np.zeros(0, np.int32)
    col_idx = np.concatenate([g.col_idx for g in graphs]) if G else np.zeros(0, np.int32)
    return Batch(list(graphs), vtx_off, edge_off, row_ptr.astype(np.int32), col_idx.astype(np.int32))
