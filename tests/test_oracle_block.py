"""Pins of the block Gauss-Seidel oracle (Algorithm 2 with fixed id blocks,
each coloured in id order and seeing its own colours of the round).

Checked against things other than itself:
* block size 1 is the round-synchronous simulation of Algorithm 2 (colours,
  rounds and per-round log);
* one block holding every vertex is the serial greedy (Algorithm 1) in id
  order, finished in one round, whatever the priority;
* a set-based Python version written from the definition, on every graph of
  up to 5 vertices and every priority order of 4 vertices;
* closed forms derived by hand for paths, and invariants on R-MAT graphs.
"""
import itertools

import numpy as np
import pytest

import graphgen
import oracle


def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield oracle.edges_to_adj(n, [pairs[i] for i in range(len(pairs)) if mask >> i & 1])


def _key(key):
    return None if key is None else np.asarray(key, dtype=np.uint32)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_every_small_graph_against_the_set_definition(n):
    for adj in _all_graphs(n):
        rp, ci = oracle.adj_to_csr(adj)
        for block in sorted({1, 2, 3, n}):
            r = oracle.block_gs(rp, ci, None, block)
            colors, rounds = oracle.block_gs_py(adj, None, block)
            assert list(r.colors) == colors and r.rounds == rounds, (adj, block)
            assert oracle.is_proper(adj, colors)


def test_every_priority_order_of_small_graphs():
    for adj in _all_graphs(4):
        rp, ci = oracle.adj_to_csr(adj)
        for perm in itertools.permutations(range(4)):
            for block in (1, 2, 3):
                r = oracle.block_gs(rp, ci, _key(perm), block)
                colors, rounds = oracle.block_gs_py(adj, list(perm), block)
                assert list(r.colors) == colors and r.rounds == rounds


@pytest.mark.parametrize("order", ["natural", "perm", "ties"])
def test_block_of_one_is_algorithm_2(order):
    g = graphgen.rmat(12, 8, (0.55, 0.1, 0.1), 4)
    key = {"natural": None, "perm": graphgen.random_priority(g.n, 3),
           "ties": graphgen.random_keys(g.n, 5, bits=3)}[order]
    a = oracle.block_gs(g.row_ptr, g.col_idx, key, 1)
    b = oracle.spec_sim(g.row_ptr, g.col_idx, key)
    assert np.array_equal(a.colors, b.colors)
    assert a.rounds == b.rounds
    assert np.array_equal(a.log, b.log)


@pytest.mark.parametrize("order", ["natural", "perm"])
def test_one_block_is_the_serial_greedy_in_one_round(order):
    g = graphgen.rmat(12, 8, (0.55, 0.1, 0.1), 6)
    key = None if order == "natural" else graphgen.random_priority(g.n, 1)
    for block in (g.n, g.n + 17, 1 << 30):
        r = oracle.block_gs(g.row_ptr, g.col_idx, key, block)
        assert r.rounds == 1
        assert np.array_equal(r.colors, oracle.greedy(g.row_ptr, g.col_idx, None))


@pytest.mark.parametrize("n", [2, 5, 12, 31])
@pytest.mark.parametrize("block", [2, 4, 6])
def test_path_even_blocks(n, block):
    """P_n in natural order with an even block size: each block alternates
    1, 2 from its first vertex (an even id), so neighbouring blocks meet as
    2 | 1 and nothing conflicts: one round, colour 1 + v mod 2."""
    g = graphgen.path(n)
    r = oracle.block_gs(g.row_ptr, g.col_idx, None, block)
    assert r.rounds == 1
    assert list(r.colors) == [1 + v % 2 for v in range(n)]


@pytest.mark.parametrize("n", [7, 10, 22])
@pytest.mark.parametrize("block", [3, 5])
def test_path_odd_blocks(n, block):
    """P_n in natural order with an odd block size B >= 3: in round 1 block j
    colours 1, 2, 1, ... from its first vertex jB; for j >= 1 that vertex
    meets the previous block's last vertex (colour 1, smaller id) and gives
    its colour back, while the rest of the block keeps 2, 1, 2, ...  Round 2
    gives each such vertex colour 3 (its neighbours hold 1 and 2), or 2 when
    it is the last vertex of the path (its one neighbour holds 1)."""
    g = graphgen.path(n)
    r = oracle.block_gs(g.row_ptr, g.col_idx, None, block)
    want = []
    for v in range(n):
        j, i = divmod(v, block)
        if j >= 1 and i == 0:
            want.append(3 if v + 1 < n else 2)
        else:
            want.append(1 + i % 2)
    assert list(r.colors) == want
    assert r.rounds == (2 if n > block else 1)
    assert r.log[0, 3] == (n - 1) // block


def test_empty_and_isolated():
    r = oracle.block_gs(np.zeros(1, np.int32), np.zeros(0, np.int32), None, 8)
    assert r.rounds == 0 and r.colors.size == 0
    g = graphgen.empty(10)
    r = oracle.block_gs(g.row_ptr, g.col_idx, None, 3)
    assert r.rounds == 1 and list(r.colors) == [1] * 10
    with pytest.raises(ValueError):
        oracle.block_gs(g.row_ptr, g.col_idx, None, 0)


@pytest.mark.parametrize("block", [2, 16, 64, 1024])
@pytest.mark.parametrize("order", ["natural", "perm"])
def test_rmat_invariants(block, order):
    """Proper colouring, colour <= degree + 1, fewer losers every round (the
    uncoloured vertex first in (key, id) order always keeps its colour), and
    rounds no more than Algorithm 2 needs with blocks of one."""
    g = graphgen.rmat(13, 16, (0.57, 0.19, 0.19), 2)
    key = None if order == "natural" else graphgen.random_priority(g.n, 7)
    r = oracle.block_gs(g.row_ptr, g.col_idx, key, block)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    dst = g.col_idx
    off = src != dst
    assert np.all(r.colors[src[off]] != r.colors[dst[off]])
    assert np.all((r.colors >= 1) & (r.colors <= g.degrees() + 1))
    assert np.all(r.log[:, 3] < r.log[:, 1])
    assert np.array_equal(r.log[1:, 1], r.log[:-1, 3])
    assert r.log[-1, 3] == 0
    assert r.rounds <= oracle.spec_sim(g.row_ptr, g.col_idx, key).rounds


def test_self_loops_and_duplicates_are_harmless():
    g = graphgen.rmat(10, 8, (0.55, 0.1, 0.1), 4)
    rng = np.random.default_rng(9)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    loops = rng.choice(g.n, 80, replace=False)
    s2 = np.concatenate([src, loops])
    d2 = np.concatenate([g.col_idx, loops])
    order = np.lexsort((d2, s2))
    rp = np.zeros(g.n + 1, np.int64)
    np.add.at(rp, s2[order] + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    ci = d2[order].astype(np.int32)
    for block in (1, 5, 64):
        a = oracle.block_gs(g.row_ptr, g.col_idx, None, block)
        b = oracle.block_gs(rp, ci, None, block)
        assert np.array_equal(a.colors, b.colors) and a.rounds == b.rounds


@pytest.mark.parametrize("block", [1, 5, 64, 1000])
@pytest.mark.parametrize("order", ["natural", "perm", "ties"])
def test_result_independent_of_threads(block, order):
    """Phase 1 runs the blocks on OpenMP threads and phase 2 the vertices:
    colours, rounds and the per-round log are those of one thread at every
    thread count."""
    g = graphgen.rmat(15, 8, (0.55, 0.1, 0.1), 5)
    key = {"natural": None, "perm": graphgen.random_priority(g.n, 6),
           "ties": graphgen.random_keys(g.n, 7, bits=3)}[order]
    ref = oracle.block_gs(g.row_ptr, g.col_idx, key, block, threads=1)
    for th in (2, 3, 8, 0):
        r = oracle.block_gs(g.row_ptr, g.col_idx, key, block, threads=th)
        assert np.array_equal(r.colors, ref.colors) and r.rounds == ref.rounds
        assert np.array_equal(r.log, ref.log)


def test_stamps_do_not_leak_between_rounds():
    """A vertex that lost keeps no forbidden colour from its earlier visit: on
    these graphs (random keys with ties, small blocks) the oracle equals the
    set definition, which rebuilds every forbidden set from scratch."""
    rng = np.random.default_rng(42)
    for _ in range(400):
        n = int(rng.integers(4, 22))
        p = rng.uniform(0.15, 0.6)
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
        adj = oracle.edges_to_adj(n, edges)
        rp, ci = oracle.adj_to_csr(adj)
        key = rng.integers(0, 3, n).astype(np.uint32)
        block = int(rng.integers(2, 7))
        r = oracle.block_gs(rp, ci, key, block=block, threads=2)
        c, k = oracle.block_gs_py(adj, key, block=block)
        assert list(r.colors) == list(c) and r.rounds == k
