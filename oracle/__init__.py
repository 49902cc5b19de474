"""CPU oracle for the speculative distance-1 colouring -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It shares no code with the GPU library in
``paper_1205_3809_amd`` and never imports it.

Two layers:

* ``oracle.c`` (loaded through ctypes): serial greedy first-fit (Algorithm 1),
  the round-synchronous simulation of the iterative speculative colouring
  (Algorithm 2, snapshot reads, losers revoked), the dataflow colouring
  (Algorithm 3) read in rounds, the block Gauss-Seidel variant of
  Algorithm 2 (fixed id blocks coloured in order, seeing their own colours
  of the round), and smallest-last ordering.  Fast enough for full-size
  graphs.
* Pure-Python definitions below (``greedy_py``, ``spec_sim_py``,
  ``block_gs_py``, ``dataflow_py``) for small inputs, written straight from
  the set notation,
  plus brute-force tools (chromatic number, greedy over every ordering, the
  longest chain of preceding vertices) used to pin the oracle.

Readings of the paper that the oracle fixes (the paper leaves them open):
phase 1 reads the previous round's committed colours; losers are reset to 0;
ties of the priority break by vertex id; self-loops are ignored.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from typing import Dict, List, NamedTuple, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None


def build() -> str:
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC])
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
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.or_greedy.argtypes = [ctypes.c_int32, i32p, i32p, u32p, i32p]
    lib.or_greedy.restype = ctypes.c_int32
    lib.or_spec_sim.argtypes = [ctypes.c_int32, i32p, i32p, u32p, i32p, i32p, i64p,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.or_spec_sim.restype = ctypes.c_int32
    lib.or_smallest_last.argtypes = [ctypes.c_int32, i32p, i32p, i32p]
    lib.or_smallest_last.restype = ctypes.c_int32
    lib.or_dataflow.argtypes = [ctypes.c_int32, i32p, i32p, u32p, i32p, i32p]
    lib.or_dataflow.restype = ctypes.c_int32
    lib.or_block_gs.argtypes = [ctypes.c_int32, i32p, i32p, u32p, ctypes.c_int32, i32p, i64p,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.or_block_gs.restype = ctypes.c_int32
    lib.or_spec_tail.argtypes = [ctypes.c_int32, i32p, i32p, u32p, ctypes.c_int64, i32p, i64p, ctypes.c_int32]
    lib.or_spec_tail.restype = ctypes.c_int32
    lib.or_num_threads.argtypes = []
    lib.or_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a, ct):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ct))


def _csr_args(row_ptr, col_idx):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    return row_ptr, col_idx


def num_threads() -> int:
    return int(_load().or_num_threads())


def greedy(row_ptr, col_idx, key: Optional[np.ndarray] = None) -> np.ndarray:
    """Serial first-fit greedy (Algorithm 1) in ascending (key, id) order."""
    row_ptr, col_idx = _csr_args(row_ptr, col_idx)
    n = row_ptr.shape[0] - 1
    if key is not None:
        key = np.ascontiguousarray(key, dtype=np.uint32)
    color = np.zeros(max(n, 1), dtype=np.int32)
    _load().or_greedy(n, _p(row_ptr, ctypes.c_int32), _p(col_idx, ctypes.c_int32),
                      _p(key, ctypes.c_uint32), _p(color, ctypes.c_int32))
    return color[:n]


class SpecResult(NamedTuple):
    colors: np.ndarray       # int32[n], every entry >= 1
    rounds: int
    fixed_round: np.ndarray  # int32[n]: round in which the vertex kept its colour
    log: np.ndarray          # int64[rounds, 4]: (k, |U_k|, sum deg over U_k, |R_k|)


def spec_sim(row_ptr, col_idx, key: Optional[np.ndarray] = None, threads: int = 1,
             max_rounds: Optional[int] = None) -> SpecResult:
    """Round-synchronous iterative speculative colouring (Algorithm 2 with
    snapshot reads and revoked losers).  Raises if the round cap is hit."""
    row_ptr, col_idx = _csr_args(row_ptr, col_idx)
    n = row_ptr.shape[0] - 1
    if key is not None:
        key = np.ascontiguousarray(key, dtype=np.uint32)
    if max_rounds is None:
        max_rounds = max(n, 1)
    color = np.zeros(max(n, 1), dtype=np.int32)
    fixed = np.zeros(max(n, 1), dtype=np.int32)
    max_log = max(1, min(max_rounds, 1 << 20))
    log = np.zeros((max_log, 4), dtype=np.int64)
    k = _load().or_spec_sim(n, _p(row_ptr, ctypes.c_int32), _p(col_idx, ctypes.c_int32),
                            _p(key, ctypes.c_uint32), _p(color, ctypes.c_int32),
                            _p(fixed, ctypes.c_int32), _p(log, ctypes.c_int64),
                            max_log, max_rounds, threads)
    if k < 0:
        raise RuntimeError("spec_sim: round cap %d exceeded" % max_rounds)
    return SpecResult(color[:n], int(k), fixed[:n], log[:k].copy())


class TailResult(NamedTuple):
    colors: np.ndarray  # int32[n]
    rounds: int         # rounds of Algorithm 2 before the sequential finish
    tail: int           # vertices the sequential finish coloured


def spec_tail(row_ptr, col_idx, key: Optional[np.ndarray] = None, tail: int = 0,
              max_rounds: Optional[int] = None) -> TailResult:
    """Algorithm 2's rounds (as spec_sim) while more than `tail` vertices are
    uncoloured, then the rest coloured one at a time in ascending (key, id)
    order with first-fit (the sequential switch of section "Iterative and
    degree of concurrency").  tail = 0 is spec_sim; tail >= n is greedy."""
    row_ptr, col_idx = _csr_args(row_ptr, col_idx)
    n = row_ptr.shape[0] - 1
    if key is not None:
        key = np.ascontiguousarray(key, dtype=np.uint32)
    if max_rounds is None:
        max_rounds = max(n, 1)
    color = np.zeros(max(n, 1), dtype=np.int32)
    cnt = np.zeros(1, dtype=np.int64)
    k = _load().or_spec_tail(n, _p(row_ptr, ctypes.c_int32), _p(col_idx, ctypes.c_int32),
                             _p(key, ctypes.c_uint32), int(tail), _p(color, ctypes.c_int32),
                             _p(cnt, ctypes.c_int64), max_rounds)
    if k < 0:
        raise RuntimeError("spec_tail: round cap %d exceeded" % max_rounds)
    return TailResult(color[:n], int(k), int(cnt[0]))


class DataflowResult(NamedTuple):
    colors: np.ndarray    # int32[n]
    rounds: int
    round_of: np.ndarray  # int32[n]: round in which the vertex is coloured (1-based)


def dataflow(row_ptr, col_idx, key: Optional[np.ndarray] = None) -> DataflowResult:
    """Dataflow colouring (Algorithm 3) read in rounds: the colours and the
    round of every vertex (one more than the latest round among its
    preceding neighbours)."""
    row_ptr, col_idx = _csr_args(row_ptr, col_idx)
    n = row_ptr.shape[0] - 1
    if key is not None:
        key = np.ascontiguousarray(key, dtype=np.uint32)
    color = np.zeros(max(n, 1), dtype=np.int32)
    rnd = np.zeros(max(n, 1), dtype=np.int32)
    k = _load().or_dataflow(n, _p(row_ptr, ctypes.c_int32), _p(col_idx, ctypes.c_int32),
                            _p(key, ctypes.c_uint32), _p(color, ctypes.c_int32), _p(rnd, ctypes.c_int32))
    return DataflowResult(color[:n], int(k), rnd[:n])


class BlockResult(NamedTuple):
    colors: np.ndarray  # int32[n]
    rounds: int
    log: np.ndarray     # int64[rounds, 4]: (k, |U_k|, sum deg over U_k, losers)


def block_gs(row_ptr, col_idx, key: Optional[np.ndarray] = None, block: int = 64,
             max_rounds: Optional[int] = None, threads: int = 1) -> BlockResult:
    """Block Gauss-Seidel speculative colouring: Algorithm 2 in rounds where
    each block of `block` consecutive ids colours its worklist vertices in id
    order, seeing the block's own colours of the round; conflicts by (key,
    id) precedence as in Algorithm 2.  threads: OpenMP threads (0 = all);
    the result does not depend on it."""
    row_ptr, col_idx = _csr_args(row_ptr, col_idx)
    n = row_ptr.shape[0] - 1
    if key is not None:
        key = np.ascontiguousarray(key, dtype=np.uint32)
    if max_rounds is None:
        max_rounds = max(n, 1)
    color = np.zeros(max(n, 1), dtype=np.int32)
    max_log = max(1, min(max_rounds, 1 << 20))
    log = np.zeros((max_log, 4), dtype=np.int64)
    k = _load().or_block_gs(n, _p(row_ptr, ctypes.c_int32), _p(col_idx, ctypes.c_int32),
                            _p(key, ctypes.c_uint32), int(block), _p(color, ctypes.c_int32),
                            _p(log, ctypes.c_int64), max_log, max_rounds, int(threads))
    if k == -1:
        raise ValueError("block size must be at least 1")
    if k < 0:
        raise RuntimeError("block_gs: round cap %d exceeded" % max_rounds)
    return BlockResult(color[:n], int(k), log[:k].copy())


def smallest_last_rank(row_ptr, col_idx) -> Tuple[np.ndarray, int]:
    """Matula-Beck smallest-last order: rank[v] = position in the colouring
    order (0 first).  Returns (rank, degeneracy)."""
    row_ptr, col_idx = _csr_args(row_ptr, col_idx)
    n = row_ptr.shape[0] - 1
    rank = np.zeros(max(n, 1), dtype=np.int32)
    d = _load().or_smallest_last(n, _p(row_ptr, ctypes.c_int32), _p(col_idx, ctypes.c_int32),
                                 _p(rank, ctypes.c_int32))
    return rank[:n], int(d)


# ---------------------------------------------------------------------------
# Pure-Python definitions (small inputs)
# ---------------------------------------------------------------------------

def adjacency(row_ptr, col_idx) -> List[List[int]]:
    n = len(row_ptr) - 1
    return [[int(w) for w in col_idx[row_ptr[v]:row_ptr[v + 1]] if int(w) != v] for v in range(n)]


def _order_key(key, v):
    return (int(key[v]) if key is not None else v, v)


def first_fit(forbidden: set) -> int:
    """Smallest positive integer not in `forbidden`."""
    c = 1
    while c in forbidden:
        c += 1
    return c


def greedy_py(adj: List[List[int]], order: Optional[Sequence[int]] = None) -> List[int]:
    """Algorithm 1 over an explicit visit order (default 0..n-1)."""
    n = len(adj)
    color = [0] * n
    for v in (range(n) if order is None else order):
        color[v] = first_fit({color[w] for w in adj[v] if color[w] > 0})
    return color


def spec_sim_py(adj: List[List[int]], key=None, trace=None) -> Tuple[List[int], int, List[Tuple[int, int, int, int]]]:
    """The round-synchronous simulation, straight from its set definition.
    trace(k, U, tent, R, color) is called at the end of each round if given."""
    n = len(adj)
    color = [0] * n
    U = list(range(n))
    k = 0
    log = []
    while U:
        k += 1
        snap = list(color)
        tent = {v: first_fit({snap[w] for w in adj[v] if snap[w] > 0}) for v in U}
        for v in U:
            color[v] = tent[v]
        R = [v for v in U
             if any(color[w] == color[v] and _order_key(key, w) < _order_key(key, v) for w in adj[v])]
        for v in R:
            color[v] = 0
        log.append((k, len(U), sum(len(adj[v]) for v in U), len(R)))
        if trace is not None:
            trace(k, list(U), dict(tent), list(R), list(color))
        U = R
    return color, k, log


def spec_tail_py(adj: List[List[int]], key=None, tail: int = 0) -> Tuple[List[int], int]:
    """Set-notation definition of the iterative colouring with a sequential
    finish: rounds of Algorithm 2 (snapshot reads, losers revoked) while
    |U| > tail, then the vertices of U one at a time in ascending (key, id)
    order, each taking the smallest colour none of its neighbours holds."""
    n = len(adj)
    color = [0] * n
    U = list(range(n))
    k = 0
    while len(U) > tail:
        k += 1
        snap = list(color)
        tent = {v: first_fit({snap[w] for w in adj[v] if w != v}) for v in U}
        for v in U:
            color[v] = tent[v]
        R = [v for v in U if any(w != v and color[w] == color[v] and _order_key(key, w) < _order_key(key, v)
                                 for w in adj[v])]
        for v in R:
            color[v] = 0
        U = R
    for v in sorted(U, key=lambda x: _order_key(key, x)):
        color[v] = first_fit({color[w] for w in adj[v] if w != v})
    return color, k


def block_gs_py(adj: List[List[int]], key=None, block: int = 1) -> Tuple[List[int], int]:
    """The block Gauss-Seidel rounds from their set definition: in each
    round, block b = {v : v // block == b} takes its uncoloured vertices in
    id order, each choosing the smallest colour held neither by a coloured
    neighbour nor by a neighbour of the same block chosen earlier in the
    round; then every uncoloured vertex whose choice equals that of a
    preceding ((key, id) order) uncoloured neighbour gives it back.
    Returns (colours, rounds)."""
    n = len(adj)
    color = [0] * n
    k = 0
    while any(c == 0 for c in color):
        k += 1
        U = [v for v in range(n) if color[v] == 0]
        chosen = {}
        for v in U:  # ascending id: within a block, earlier choices are known
            seen = {color[w] for w in adj[v] if color[w] > 0}
            seen |= {chosen[w] for w in adj[v] if w in chosen and w // block == v // block}
            chosen[v] = first_fit(seen)
        keep = [v for v in U
                if not any(w in chosen and chosen[w] == chosen[v] and _order_key(key, w) < _order_key(key, v)
                           for w in adj[v] if w != v)]
        for v in keep:
            color[v] = chosen[v]
    return color, k


def dataflow_py(adj: List[List[int]], key=None) -> Tuple[List[int], int, List[int]]:
    """Algorithm 3 in rounds, from its description: each round colours, all
    at once, every uncoloured vertex whose preceding neighbours are all
    coloured, with the smallest colour none of them holds.  Returns
    (colours, rounds, round of each vertex)."""
    n = len(adj)
    color = [0] * n
    round_of = [0] * n
    k = 0
    while any(c == 0 for c in color):
        k += 1
        before = lambda v: [w for w in adj[v] if _order_key(key, w) < _order_key(key, v)]
        ready = [v for v in range(n) if color[v] == 0 and all(color[w] > 0 for w in before(v))]
        if not ready:
            raise RuntimeError("no vertex ready")  # precedence is a strict total order: cannot happen
        chosen = {v: first_fit({color[w] for w in before(v)}) for v in ready}
        for v in ready:
            color[v] = chosen[v]
            round_of[v] = k
    return color, k, round_of


def longest_chain(adj: List[List[int]], key=None) -> int:
    """Vertices on the longest path v1, v2, ... along which each vertex
    precedes the next, by enumerating every such path (tiny graphs only)."""
    best = 0

    def walk(v: int, length: int) -> None:
        nonlocal best
        best = max(best, length)
        for w in adj[v]:
            if _order_key(key, v) < _order_key(key, w):
                walk(w, length + 1)

    for v in range(len(adj)):
        walk(v, 1)
    return best


def is_proper(adj: List[List[int]], color: Sequence[int]) -> bool:
    return all(color[v] >= 1 for v in range(len(adj))) and all(
        color[v] != color[w] for v in range(len(adj)) for w in adj[v])


def chromatic_number(adj: List[List[int]]) -> int:
    """Smallest k admitting a proper k-colouring, by exhaustive backtracking."""
    n = len(adj)
    if n == 0:
        return 0

    def colorable(k: int) -> bool:
        col = [0] * n

        def go(v: int) -> bool:
            if v == n:
                return True
            used = {col[w] for w in adj[v] if w < v}
            # symmetry breaking: vertex v may open at most one new colour
            top = max(col[:v], default=0)
            for c in range(1, min(k, top + 1) + 1):
                if c not in used:
                    col[v] = c
                    if go(v + 1):
                        return True
            col[v] = 0
            return False

        return go(0)

    k = 1
    while not colorable(k):
        k += 1
    return k


def min_greedy_over_orders(adj: List[List[int]]) -> int:
    """Fewest colours Algorithm 1 uses over every visit order."""
    n = len(adj)
    best = n
    for perm in itertools.permutations(range(n)):
        best = min(best, max(greedy_py(adj, perm), default=0))
    return best


def edges_to_adj(n: int, edges: Sequence[Tuple[int, int]]) -> List[List[int]]:
    adj = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    return [sorted(a) for a in adj]


def adj_to_csr(adj: List[List[int]]) -> Tuple[np.ndarray, np.ndarray]:
    row_ptr = np.zeros(len(adj) + 1, dtype=np.int32)
    for v, a in enumerate(adj):
        row_ptr[v + 1] = row_ptr[v] + len(a)
    col = np.array([w for a in adj for w in a], dtype=np.int32)
    return row_ptr, col
