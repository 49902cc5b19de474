"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Every assertion here compares the oracle with something other than itself:
brute force (chromatic number, greedy over every ordering), closed forms
derived by hand for paths, cycles, complete and complete bipartite graphs,
stars and bipartite grids, the bounds the paper states for first-fit
(Delta + 1, back degree + 1), invariants of the round-synchronous scheme, and
relabelling equivariance.
"""
import itertools
import math

import numpy as np
import pytest

import graphgen
import oracle


def csr_of(adj):
    return oracle.adj_to_csr(adj)


def run_both(adj, key=None):
    """C oracle results (O1 colours, O2 result) on an adjacency list."""
    rp, ci = csr_of(adj)
    k = None if key is None else np.asarray(key, dtype=np.uint32)
    return oracle.greedy(rp, ci, k), oracle.spec_sim(rp, ci, k)


def all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield oracle.edges_to_adj(n, [pairs[i] for i in range(len(pairs)) if mask >> i & 1])


# ---------------------------------------------------------------------------
# first-fit and brute force
# ---------------------------------------------------------------------------

def test_first_fit_definition():
    assert oracle.first_fit(set()) == 1
    assert oracle.first_fit({2, 3}) == 1
    assert oracle.first_fit({1, 2, 4}) == 3
    assert oracle.first_fit(set(range(1, 100))) == 100


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_small_graphs(n):
    """Every graph on n <= 5 vertices: greedy over all orders reaches exactly
    the chromatic number, no order does better, and both oracles (C and the
    set-notation definition) agree and colour properly."""
    for adj in all_graphs(n):
        chi = oracle.chromatic_number(adj)
        o1, o2 = run_both(adj)
        assert oracle.is_proper(adj, o1) and oracle.is_proper(adj, o2.colors)
        assert list(o1) == oracle.greedy_py(adj)
        c2, k2, _ = oracle.spec_sim_py(adj)
        assert list(o2.colors) == c2 and o2.rounds == k2
        assert max(o1) >= chi and max(o2.colors) >= chi
        assert oracle.min_greedy_over_orders(adj) == chi


def _random_adj(rng, n, p):
    return oracle.edges_to_adj(n, [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p])


def test_random_graphs_up_to_10_vertices():
    rng = np.random.default_rng(1205)
    for trial in range(120):
        n = int(rng.integers(6, 11))
        adj = _random_adj(rng, n, float(rng.uniform(0.15, 0.8)))
        chi = oracle.chromatic_number(adj)
        key = rng.permutation(n) if trial % 2 else None
        o1, o2 = run_both(adj, key)
        order = list(range(n)) if key is None else list(np.argsort(key, kind="stable"))
        assert list(o1) == oracle.greedy_py(adj, order)
        c2, k2, _ = oracle.spec_sim_py(adj, key)
        assert list(o2.colors) == c2 and o2.rounds == k2
        assert oracle.is_proper(adj, o1) and oracle.is_proper(adj, o2.colors)
        assert max(o1) >= chi and max(o2.colors) >= chi
        if n <= 7:
            assert oracle.min_greedy_over_orders(adj) == chi


# ---------------------------------------------------------------------------
# closed forms (derived by hand, natural order)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", list(range(1, 13)))
def test_complete_graph(n):
    """K_n: n colours; the round-synchronous scheme fixes exactly the
    smallest remaining vertex each round, so it takes n rounds."""
    g = graphgen.complete(n)
    o1 = oracle.greedy(g.row_ptr, g.col_idx)
    o2 = oracle.spec_sim(g.row_ptr, g.col_idx)
    assert o1.max() == n and o2.colors.max() == n and o2.rounds == n
    assert sorted(o2.colors) == list(range(1, n + 1))


@pytest.mark.parametrize("n", [2, 3, 5, 17, 64])
@pytest.mark.parametrize("center", ["first", "last"])
def test_star(n, center):
    """A star needs 2 colours in 2 rounds whether the centre has the smallest
    or the largest index."""
    c = 0 if center == "first" else n - 1
    g = graphgen.star(n, c)
    o1 = oracle.greedy(g.row_ptr, g.col_idx)
    o2 = oracle.spec_sim(g.row_ptr, g.col_idx)
    assert o1.max() == 2 and o2.colors.max() == 2 and o2.rounds == 2
    assert o2.colors[c] == (1 if center == "first" else 2)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 33, 64, 65, 200])
def test_path(n):
    """P_n in natural order: round 1 fixes vertex 0, every later round fixes
    the next two vertices, so rounds = 1 + ceil((n-1)/2); colours alternate."""
    g = graphgen.path(n)
    o2 = oracle.spec_sim(g.row_ptr, g.col_idx)
    assert o2.rounds == 1 + math.ceil((n - 1) / 2)
    assert list(o2.colors) == [1 + (v % 2) for v in range(n)]
    assert list(oracle.greedy(g.row_ptr, g.col_idx)) == [1 + (v % 2) for v in range(n)]


@pytest.mark.parametrize("n", [4, 6, 8, 10, 50, 128, 198])
def test_even_cycle(n):
    """Even C_n in natural order: 2 colours (alternating) in n/2 rounds.  The
    literal reading of Algorithm 2, in which losers keep their stale colour,
    would give 3 colours on C_4; this pins the revoke-losers reading."""
    g = graphgen.cycle(n)
    o2 = oracle.spec_sim(g.row_ptr, g.col_idx)
    assert o2.colors.max() == 2 and o2.rounds == n // 2
    assert list(o2.colors) == [1 + (v % 2) for v in range(n)]
    assert oracle.greedy(g.row_ptr, g.col_idx).max() == 2


@pytest.mark.parametrize("n", [3, 5, 7, 51])
def test_odd_cycle(n):
    g = graphgen.cycle(n)
    assert oracle.spec_sim(g.row_ptr, g.col_idx).colors.max() == 3
    assert oracle.greedy(g.row_ptr, g.col_idx).max() == 3


@pytest.mark.parametrize("p,q", [(1, 1), (1, 5), (3, 4), (10, 7)])
def test_complete_bipartite(p, q):
    """K_{p,q}, the p-side first: the p-side has no preceding neighbour and
    keeps colour 1 in round 1; the q-side takes colour 2 in round 2."""
    g = graphgen.complete_bipartite(p, q)
    o2 = oracle.spec_sim(g.row_ptr, g.col_idx)
    assert o2.rounds == 2
    assert list(o2.colors) == [1] * p + [2] * q


def test_empty_graph():
    g = graphgen.empty(10)
    o2 = oracle.spec_sim(g.row_ptr, g.col_idx)
    assert o2.rounds == 1 and list(o2.colors) == [1] * 10
    assert oracle.spec_sim(np.zeros(1, np.int32), np.zeros(0, np.int32)).rounds == 0


@pytest.mark.parametrize("shape", [(8, 8), (5, 13), (64, 64), (6, 7, 5), (12, 12, 12)])
def test_bipartite_grid_two_colours(shape):
    """Star-stencil grids are bipartite; in natural (row-major) order both
    schemes give the parity checkerboard colour 1 + (sum of coordinates mod 2)."""
    g = graphgen.grid(shape, full=False)
    o1 = oracle.greedy(g.row_ptr, g.col_idx)
    o2 = oracle.spec_sim(g.row_ptr, g.col_idx)
    parity = 1 + np.indices(shape).sum(axis=0).ravel() % 2
    assert np.array_equal(o1, parity)
    assert np.array_equal(o2.colors, parity)


# ---------------------------------------------------------------------------
# invariants on generated graphs
# ---------------------------------------------------------------------------

def _cases():
    yield "uniform", graphgen.uniform(3000, 12000, 7), None
    g = graphgen.rmat(12, 8, (0.45, 0.15, 0.15), 3)
    yield "rmat_g", g, None
    yield "rmat_g_perm", g, graphgen.random_priority(g.n, 4)
    g = graphgen.rmat(12, 8, (0.55, 0.1, 0.1), 5)
    yield "rmat_skew", g, None
    yield "rmat_skew_ties", g, graphgen.random_keys(g.n, 6, bits=3)


@pytest.mark.parametrize("name,g,key", list(_cases()), ids=lambda x: x if isinstance(x, str) else "")
def test_invariants(name, g, key):
    n = g.n
    deg = g.degrees()
    src = np.repeat(np.arange(n), deg)
    o1 = oracle.greedy(g.row_ptr, g.col_idx, key)
    o2 = oracle.spec_sim(g.row_ptr, g.col_idx, key, threads=4)
    kk = np.arange(n, dtype=np.int64) if key is None else key.astype(np.int64)
    before = (kk[g.col_idx] < kk[src]) | ((kk[g.col_idx] == kk[src]) & (g.col_idx < src))
    for col in (o1, o2.colors):
        assert col.min() >= 1
        assert not np.any(col[src] == col[g.col_idx]), "improper colouring"
        assert np.all(col <= deg + 1)
    # first-fit in the serial order: colour <= back degree + 1
    back = np.bincount(src[before], minlength=n)
    assert np.all(o1 <= back + 1)
    # a vertex fixed in round k has colour <= k, so colours <= rounds
    assert np.all(o2.colors <= o2.fixed_round)
    assert o2.colors.max() <= o2.rounds <= n
    # round 1: every vertex is tentatively 1; exactly those with a preceding
    # neighbour lose
    has_pred = np.bincount(src[before], minlength=n) > 0
    assert o2.log[0, 1] == n and o2.log[0, 2] == g.nnz and o2.log[0, 3] == has_pred.sum()
    assert np.array_equal(o2.fixed_round == 1, ~has_pred)
    assert np.all(o2.colors[~has_pred] == 1)
    # the worklist shrinks every round; the log chains
    assert np.all(np.diff(o2.log[:, 1]) < 0)
    assert np.array_equal(o2.log[1:, 1], o2.log[:-1, 3]) and o2.log[-1, 3] == 0
    # the oracle's answer does not depend on its thread count
    o2b = oracle.spec_sim(g.row_ptr, g.col_idx, key, threads=1)
    assert np.array_equal(o2.colors, o2b.colors) and np.array_equal(o2.log, o2b.log)


def test_round_invariants_traced():
    """Per-round facts of the scheme on random small graphs: the committed set
    is always properly coloured, the smallest-key worklist vertex always
    keeps its colour, and tentative colours never decrease."""
    rng = np.random.default_rng(42)
    for trial in range(40):
        n = int(rng.integers(5, 40))
        adj = _random_adj(rng, n, float(rng.uniform(0.05, 0.5)))
        key = rng.integers(0, 4, n) if trial % 2 else None
        last = {}

        def trace(k, U, tent, R, color):
            fixed = [v for v in range(n) if color[v] > 0]
            for v in fixed:
                assert all(color[w] != color[v] for w in adj[v] if color[w] > 0)
            kmin = min(U, key=lambda v: oracle._order_key(key, v))
            assert kmin not in R
            for v in U:
                assert tent[v] >= last.get(v, 0)
                last[v] = tent[v]

        oracle.spec_sim_py(adj, key, trace)


def test_relabelling_equivariance():
    """Relabelling vertices by a permutation, keys carried along (tie-free),
    permutes both colourings the same way."""
    g = graphgen.rmat(11, 8, (0.55, 0.1, 0.1), 9)
    n = g.n
    key = graphgen.random_priority(n, 10)
    pi = graphgen.random_priority(n, 11).astype(np.int64)  # new id of v
    src = np.repeat(np.arange(n), g.degrees())
    h = graphgen.from_pairs(n, pi[src].astype(np.int32), pi[g.col_idx].astype(np.int32))
    key2 = np.empty(n, np.uint32)
    key2[pi] = key
    a1, a2 = oracle.greedy(g.row_ptr, g.col_idx, key), oracle.spec_sim(g.row_ptr, g.col_idx, key)
    b1, b2 = oracle.greedy(h.row_ptr, h.col_idx, key2), oracle.spec_sim(h.row_ptr, h.col_idx, key2)
    assert np.array_equal(b1[pi], a1)
    assert np.array_equal(b2.colors[pi], a2.colors) and a2.rounds == b2.rounds
    # natural order is the special case key = id
    nat = oracle.spec_sim(g.row_ptr, g.col_idx)
    ident = oracle.spec_sim(g.row_ptr, g.col_idx, np.arange(n, dtype=np.uint32))
    assert np.array_equal(nat.colors, ident.colors)


# ---------------------------------------------------------------------------
# smallest-last ordering
# ---------------------------------------------------------------------------

def test_smallest_last_definition():
    """Each removal takes a vertex of minimum remaining degree, smallest id on
    ties; the degeneracy returned is the largest min-degree over all induced
    subgraphs (brute force on small graphs)."""
    rng = np.random.default_rng(5)
    for trial in range(60):
        n = int(rng.integers(1, 11))
        adj = _random_adj(rng, n, float(rng.uniform(0.1, 0.7)))
        rp, ci = csr_of(adj)
        rank, degen = oracle.smallest_last_rank(rp, ci)
        assert sorted(rank) == list(range(n))
        removal = sorted(range(n), key=lambda v: -rank[v])  # removed first = coloured last
        alive = set(range(n))
        for v in removal:
            d = {u: sum(1 for w in adj[u] if w in alive) for u in alive}
            m = min(d.values())
            assert d[v] == m and v == min(u for u in alive if d[u] == m)
            alive.remove(v)
        best = 0
        for r in range(1, n + 1):
            for sub in itertools.combinations(range(n), r):
                s = set(sub)
                best = max(best, min(sum(1 for w in adj[u] if w in s) for u in sub))
        assert degen == best
        col = oracle.greedy_py(adj, sorted(range(n), key=lambda v: rank[v]))
        assert max(col, default=0) <= degen + 1


# ---------------------------------------------------------------------------
# input generator pins
# ---------------------------------------------------------------------------

def test_uniform_generator_edge_count():
    """2^17 uniform pairs on 2^14 vertices: expected loops m/n = 8 and expected
    duplicate pairs about m^2 / (n (n-1)) = 64, so about 131,000 distinct edges
    (standard deviation under 10)."""
    g = graphgen.uniform(1 << 14, 1 << 17, 1)
    assert abs(g.edges - 131000) < 40
    assert np.all(np.diff(g.row_ptr) >= 0)
    assert np.all(g.col_idx[:-1][np.diff(np.repeat(np.arange(g.n), g.degrees())) == 0]
                  < g.col_idx[1:][np.diff(np.repeat(np.arange(g.n), g.degrees())) == 0])


def test_generator_symmetric_sorted_no_loops():
    g = graphgen.rmat(12, 8, (0.55, 0.15, 0.15), 2)
    src = np.repeat(np.arange(g.n), g.degrees())
    assert not np.any(src == g.col_idx)
    a = set(zip(src.tolist(), g.col_idx.tolist()))
    assert all((w, v) in a for v, w in a)
    same_row = src[1:] == src[:-1]
    assert np.all(g.col_idx[1:][same_row] > g.col_idx[:-1][same_row])


@pytest.mark.slow
def test_rmat_scale24_matches_paper_tables():
    """The generator reproduces the paper's scale-24 R-MAT statistics (edge
    count, degree variance, isolated share, max degree) and the serial greedy
    colour counts in shuffled order fall in the paper's range."""
    import json
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    gold = json.load(open(os.path.join(here, "golden", "paper_rmat_s24.json")))["graphs"]
    for name, row in gold.items():
        g = graphgen.rmat(24, 8, row["abcd"][:3], 11)
        d = g.degrees()
        assert abs(g.edges - row["edges"]) / row["edges"] < 1e-4, name
        assert abs(d.var() - row["variance"]) / row["variance"] < 5e-3, name
        assert abs(100.0 * (d == 0).mean() - row["isolated_pct"]) < 0.1, name
        assert abs(d.max() - row["max_degree"]) / row["max_degree"] < 0.12, name
        pri = graphgen.random_priority(g.n, 3)
        c = int(oracle.greedy(g.row_ptr, g.col_idx, pri).max())
        ref = row["serial_greedy_colors"]
        assert abs(c - ref) <= max(2, 0.15 * ref), (name, c, ref)
        del g
