"""Pins of the sequential-finish oracle (Algorithm 2's rounds while more than
`tail` vertices are uncoloured, then the rest coloured one at a time in
(key, id) order: the switch to a sequential computation that the section
"Iterative and degree of concurrency" suggests once conflicts are few).

Checked against things other than itself:
* tail = 0 is the round-synchronous simulation of Algorithm 2 (colours and
  rounds), tail >= n is the serial greedy (Algorithm 1) with no rounds;
* the rounds it runs are exactly Algorithm 2's rounds that start with more
  than `tail` vertices uncoloured, and every vertex those rounds fix keeps
  Algorithm 2's colour;
* a set-based Python version written from the definition, on every graph of
  up to 5 vertices under every tail, and on random graphs with tied keys;
* hand-worked cases (a path, a complete graph) and invariants on R-MAT.
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


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_every_small_graph_against_the_set_definition(n):
    for adj in _all_graphs(n):
        rp, ci = oracle.adj_to_csr(adj)
        for tail in range(n + 1):
            r = oracle.spec_tail(rp, ci, None, tail)
            colors, rounds = oracle.spec_tail_py(adj, None, tail)
            assert list(r.colors) == colors and r.rounds == rounds, (adj, tail)
            assert oracle.is_proper(adj, colors)


def test_random_graphs_with_tied_keys_against_the_set_definition():
    rng = np.random.default_rng(8)
    for _ in range(300):
        n = int(rng.integers(2, 18))
        p = rng.uniform(0.1, 0.7)
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
        adj = oracle.edges_to_adj(n, edges)
        rp, ci = oracle.adj_to_csr(adj)
        key = rng.integers(0, 4, n).astype(np.uint32)
        tail = int(rng.integers(0, n + 1))
        r = oracle.spec_tail(rp, ci, key, tail)
        colors, rounds = oracle.spec_tail_py(adj, list(key), tail)
        assert list(r.colors) == colors and r.rounds == rounds


@pytest.mark.parametrize("order", ["natural", "perm", "ties"])
def test_limits_are_algorithm_2_and_the_serial_greedy(order):
    g = graphgen.rmat(13, 8, (0.55, 0.1, 0.1), 2)
    key = {"natural": None, "perm": graphgen.random_priority(g.n, 3),
           "ties": graphgen.random_keys(g.n, 4, bits=3)}[order]
    a = oracle.spec_tail(g.row_ptr, g.col_idx, key, 0)
    b = oracle.spec_sim(g.row_ptr, g.col_idx, key)
    assert np.array_equal(a.colors, b.colors) and a.rounds == b.rounds and a.tail == 0
    for tail in (g.n, g.n + 5):
        c = oracle.spec_tail(g.row_ptr, g.col_idx, key, tail)
        assert np.array_equal(c.colors, oracle.greedy(g.row_ptr, g.col_idx, key))
        assert c.rounds == 0 and c.tail == g.n


@pytest.mark.parametrize("order", ["natural", "perm"])
@pytest.mark.parametrize("tail", [1, 7, 100, 1000])
def test_rounds_and_fixed_colours_are_algorithm_2s(order, tail):
    """The rounds run are those of Algorithm 2 that start with more than
    `tail` vertices uncoloured; the vertices they fix keep Algorithm 2's
    colours; the finish colours exactly the vertices left."""
    g = graphgen.rmat(14, 8, (0.55, 0.1, 0.1), 6)
    key = None if order == "natural" else graphgen.random_priority(g.n, 7)
    ref = oracle.spec_sim(g.row_ptr, g.col_idx, key)
    r = oracle.spec_tail(g.row_ptr, g.col_idx, key, tail)
    u = ref.log[:, 1]
    assert r.rounds == int(np.sum(u > tail))
    fixed = ref.fixed_round <= r.rounds
    assert np.array_equal(r.colors[fixed], ref.colors[fixed])
    assert r.tail == g.n - int(fixed.sum())
    deg = g.degrees()
    src = np.repeat(np.arange(g.n), deg)
    assert r.colors.min() >= 1 and np.all(r.colors <= deg + 1)
    assert not np.any(r.colors[src] == r.colors[g.col_idx])


def test_hand_worked_cases():
    """P_5 in natural order: round 1 keeps vertex 0 (colour 1), everyone else
    had colour 1 and a smaller neighbour with it; with tail 4 the finish then
    colours 1, 2, 3, 4 in turn: 2, 1, 2, 1.  K_4 with tail 2: two rounds fix
    vertices 0 and 1 (colours 1, 2), the finish gives 3 and 4."""
    r = oracle.spec_tail(*graphgen.path(5)[1:], None, 4)
    assert list(r.colors) == [1, 2, 1, 2, 1] and r.rounds == 1 and r.tail == 4
    r = oracle.spec_tail(*graphgen.complete(4)[1:], None, 2)
    assert list(r.colors) == [1, 2, 3, 4] and r.rounds == 2 and r.tail == 2
