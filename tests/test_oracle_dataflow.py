"""Pins of the dataflow oracle (Algorithm 3 read in rounds).

The C routine computes each vertex's colour and round from its preceding
neighbours in one ordered visit.  It is checked against things other than
itself:
* a round-by-round simulation written from the algorithm's description
  (``dataflow_py``: each round colours every vertex whose preceding
  neighbours are all coloured);
* the serial greedy of Algorithm 1 in the same order, which the dataflow
  algorithm reproduces (each vertex waits for exactly the neighbours that
  the serial visit colours before it);
* brute force over every increasing path for the number of rounds;
* closed forms derived by hand (paths, complete graphs, stars, stencil
  grids), and invariants on R-MAT graphs.
"""
import itertools

import numpy as np
import pytest

import graphgen
import oracle


def _keyed(key):
    return None if key is None else np.asarray(key, dtype=np.uint32)


def _check_small(adj, key=None):
    rp, ci = oracle.adj_to_csr(adj)
    r = oracle.dataflow(rp, ci, _keyed(key))
    colors, rounds, round_of = oracle.dataflow_py(adj, key)
    assert list(r.colors) == colors
    assert r.rounds == rounds
    assert list(r.round_of) == round_of
    assert rounds == oracle.longest_chain(adj, key)
    n = len(adj)
    order = sorted(range(n), key=lambda v: ((int(key[v]) if key is not None else v), v))
    assert colors == oracle.greedy_py(adj, order)
    assert list(oracle.greedy(rp, ci, _keyed(key))) == colors
    if n:
        assert oracle.is_proper(adj, colors)


def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield oracle.edges_to_adj(n, [pairs[i] for i in range(len(pairs)) if mask >> i & 1])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_every_small_graph_natural_order(n):
    for adj in _all_graphs(n):
        _check_small(adj)


def test_every_order_of_small_graphs():
    """All graphs on 4 vertices under all 24 visit orders."""
    for adj in _all_graphs(4):
        for perm in itertools.permutations(range(4)):
            _check_small(adj, list(perm))


def test_random_graphs_with_tied_keys():
    """Keys drawn from a small range so that ties (broken by id) are common."""
    rng = np.random.default_rng(3809)
    for trial in range(150):
        n = int(rng.integers(2, 11))
        p = float(rng.uniform(0.1, 0.9))
        adj = oracle.edges_to_adj(n, [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p])
        key = None if trial % 3 == 0 else list(rng.integers(0, 3 if trial % 3 == 1 else 1 << 30, n))
        _check_small(adj, key)


def test_empty_and_isolated():
    r = oracle.dataflow(np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert r.rounds == 0 and r.colors.size == 0
    g = graphgen.empty(9)
    r = oracle.dataflow(g.row_ptr, g.col_idx)
    assert r.rounds == 1 and list(r.colors) == [1] * 9 and list(r.round_of) == [1] * 9


@pytest.mark.parametrize("n", [1, 2, 3, 10, 101])
def test_path(n):
    """P_n in natural order: vertex v waits for v-1, so it is coloured in
    round v+1 (n rounds); colours alternate.  With keys 0,1,0,1,... every
    even vertex is ready at once and the odd ones follow: 2 rounds."""
    g = graphgen.path(n)
    r = oracle.dataflow(g.row_ptr, g.col_idx)
    assert r.rounds == n
    assert list(r.round_of) == list(range(1, n + 1))
    assert list(r.colors) == [1 + v % 2 for v in range(n)]
    alt = (np.arange(n) % 2).astype(np.uint32)
    r = oracle.dataflow(g.row_ptr, g.col_idx, alt)
    assert r.rounds == min(n, 2)
    assert list(r.round_of) == [1 + v % 2 for v in range(n)]
    assert list(r.colors) == [1 + v % 2 for v in range(n)]


@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_complete_graph(n):
    """K_n: vertex v waits for all smaller ones: round v+1, colour v+1."""
    g = graphgen.complete(n)
    r = oracle.dataflow(g.row_ptr, g.col_idx)
    assert r.rounds == n
    assert list(r.colors) == list(range(1, n + 1))
    assert list(r.round_of) == list(range(1, n + 1))


@pytest.mark.parametrize("n", [2, 3, 50])
@pytest.mark.parametrize("center", ["first", "last"])
def test_star(n, center):
    """Centre first: it is the only round-1 vertex, the leaves follow with
    colour 2.  Centre last: every leaf takes colour 1 in round 1, the centre
    colour 2 in round 2."""
    c = 0 if center == "first" else n - 1
    g = graphgen.star(n, c)
    r = oracle.dataflow(g.row_ptr, g.col_idx)
    assert r.rounds == 2
    leaves = [v for v in range(n) if v != c]
    if center == "first":
        assert r.colors[c] == 1 and r.round_of[c] == 1
        assert all(r.colors[v] == 2 and r.round_of[v] == 2 for v in leaves)
    else:
        assert r.colors[c] == 2 and r.round_of[c] == 2
        assert all(r.colors[v] == 1 and r.round_of[v] == 1 for v in leaves)


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (6, 1), (5, 7), (12, 3)])
def test_grid_5_point(shape):
    """Row-major 5-point grid: (i, j) waits for (i-1, j) and (i, j-1), so
    its round is i + j + 1 (rows + cols - 1 rounds); the colours are the
    checkerboard 1 + (i + j) mod 2."""
    R, C = shape
    g = graphgen.grid(shape)
    r = oracle.dataflow(g.row_ptr, g.col_idx)
    i, j = np.divmod(np.arange(R * C), C)
    assert np.array_equal(r.round_of, i + j + 1)
    assert r.rounds == R + C - 1
    assert np.array_equal(r.colors, 1 + (i + j) % 2)


@pytest.mark.parametrize("shape", [(2, 2), (4, 6), (7, 3), (9, 9)])
def test_grid_9_point(shape):
    """Row-major 9-point grid: (i, j) also waits for (i-1, j+1), which is
    coloured in round 2(i-1) + (j+1) + 1, so round(i, j) = 2i + j + 1 and
    there are 2(rows - 1) + cols rounds."""
    R, C = shape
    g = graphgen.grid(shape, True)
    r = oracle.dataflow(g.row_ptr, g.col_idx)
    i, j = np.divmod(np.arange(R * C), C)
    assert np.array_equal(r.round_of, 2 * i + j + 1)
    assert r.rounds == 2 * (R - 1) + C


def test_self_loops_and_duplicates_are_harmless():
    rng = np.random.default_rng(7)
    g = graphgen.rmat(10, 8, (0.55, 0.1, 0.1), 4)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    loops = rng.choice(g.n, 100, replace=False)
    dup = rng.choice(g.nnz, 300, replace=False)
    s2 = np.concatenate([src, loops, src[dup]])
    d2 = np.concatenate([g.col_idx, loops, g.col_idx[dup]])
    order = np.lexsort((d2, s2))
    s2, d2 = s2[order], d2[order]
    rp = np.zeros(g.n + 1, np.int32)
    np.add.at(rp, s2 + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    ci = d2.astype(np.int32)
    key = graphgen.random_priority(g.n, 5)
    for k in (None, key):
        a, b = oracle.dataflow(g.row_ptr, g.col_idx, k), oracle.dataflow(rp, ci, k)
        assert np.array_equal(a.colors, b.colors) and np.array_equal(a.round_of, b.round_of)


@pytest.mark.parametrize("order", ["natural", "random"])
def test_rmat_invariants(order):
    """R-MAT scale 14: colours equal the serial greedy's; every preceding
    neighbour is coloured in an earlier round, and a vertex past round 1 has
    one coloured in the round just before (it waited for exactly that)."""
    g = graphgen.rmat(14, 16, (0.57, 0.19, 0.19), 2)
    key = None if order == "natural" else graphgen.random_priority(g.n, 9)
    r = oracle.dataflow(g.row_ptr, g.col_idx, key)
    assert np.array_equal(r.colors, oracle.greedy(g.row_ptr, g.col_idx, key))
    kk = np.arange(g.n, dtype=np.int64) if key is None else key.astype(np.int64)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    dst = g.col_idx.astype(np.int64)
    before = (kk[dst] < kk[src]) | ((kk[dst] == kk[src]) & (dst < src))
    assert np.all(r.round_of[dst[before]] < r.round_of[src[before]])
    latest = np.zeros(g.n, np.int64)
    np.maximum.at(latest, src[before], r.round_of[dst[before]])
    assert np.array_equal(r.round_of, latest + 1)
    assert r.rounds == r.round_of.max()
    assert np.all(r.colors[src[src != dst]] != r.colors[dst[src != dst]])
