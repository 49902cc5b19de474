"""The rule by which the device smallest-last peel removes many vertices per
step, written out in plain Python, against the oracle's one-at-a-time peel
(CPU only).

A step takes the m smallest ids c_0 < c_1 < ... of the least remaining degree
delta and removes the longest prefix that the one-at-a-time process would
remove in that order.  c_{q+1} follows c_q unless removing c_0..c_q drops a
remaining vertex below delta (other than c_{q+1}), or brings a vertex y down to
delta with y < c_{q+1} (for y > c_{q+1}: before the first later candidate
above y).  The device may look at fewer candidates than the bucket holds (a
chunk size) and may cut them where its pair stage overflows; the next step's
candidates may be carried over (the vertices left at delta - 1, or the
candidates not taken with the vertices that came down to delta).  The rule
must give the oracle's order for every such choice, which these tests draw at
random; on small graphs no step may remove more than a brute-force run of the
one-at-a-time process removes in candidate order from the same state.
"""
import random

import numpy as np
import pytest

import graphgen
import oracle


def longest_prefix(n, rp, ci, deg, rank, cand, limit):
    """Brute force: how many of cand[0..limit) the one-at-a-time process
    removes next, in that order, from this state."""
    deg = deg.copy()
    gone = rank >= 0
    for i in range(limit):
        alive = np.flatnonzero(~gone)
        nxt = min(alive, key=lambda u: (deg[u], u))
        if nxt != cand[i]:
            return i
        gone[nxt] = True
        for p in range(rp[nxt], rp[nxt + 1]):
            y = int(ci[p])
            if y != nxt and not gone[y]:
                deg[y] -= 1
    return limit


def peel_by_steps(n, rp, ci, rng, chunk=None, stage=None, carry=True, exact=False):
    deg = np.array([sum(1 for p in range(rp[v], rp[v + 1]) if ci[p] != v) for v in range(n)])
    rank = np.full(n, -1)
    removed, delta, steps = 0, 0, 0
    carried, carried_delta = None, None
    while removed < n:
        steps += 1
        alive = np.flatnonzero(rank < 0)
        least = int(deg[alive].min())
        assert least >= max(delta - 1, 0)  # the least degree falls by at most one per step
        bucket = sorted(int(v) for v in alive[deg[alive] == least])
        k = chunk or rng.randint(1, 40)
        if carried:
            assert carried_delta == least and carried == bucket[:len(carried)]
            cand = carried[:k]
        else:
            cand = bucket[:k]
        delta = least
        m = len(cand)
        pos = {c: i for i, c in enumerate(cand)}
        pairs = []
        for q, v in enumerate(cand):
            for p in range(rp[v], rp[v + 1]):
                y = int(ci[p])
                if y == v or rank[y] >= 0 or (y in pos and pos[y] <= q):
                    continue
                pairs.append((q, y, pos.get(y, -1), int(deg[y])))
        cap = stage or rng.randint(1, 60)
        rng.shuffle(pairs)
        cut = min([m] + [pr[0] for pr in pairs[cap:]])
        pairs = [pr for pr in pairs[:cap] if pr[0] < cut]
        hits = {}
        for q, y, _, _ in pairs:
            hits.setdefault(y, []).append(q)
        first_bad = None
        for q, y, py, dy in pairs:
            qs = hits[y]
            bad = None
            if py >= 0:
                if min(qs) == q and q + 1 != py:
                    bad = q + 1
            else:
                t0 = dy - delta
                if t0 <= 0:
                    if min(qs) == q:
                        bad = q + 1
                elif len(qs) >= t0:
                    r = sum(1 for x in qs if x < q)
                    if r + 1 == t0:
                        a = q + 1
                        while a < cut and cand[a] < y:
                            a += 1
                        if a < cut:
                            bad = a
                    elif r == t0:
                        bad = q + 1
            if bad is not None:
                first_bad = bad if first_bad is None else min(first_bad, bad)
        take = 1 if cut == 0 else max(1, min(cut, cut if first_bad is None else first_bad))
        if exact and cut > 0:
            # never more than the one-at-a-time process removes in this
            # order (it may stop early: a vertex dropping below delta ends the
            # step even when the next candidate dropped too and goes first)
            assert 1 <= take <= longest_prefix(n, rp, ci, deg, rank, cand, cut)
        for t in range(take):
            rank[cand[t]] = n - 1 - (removed + t)
        touched = set()
        for t in range(take):
            v = cand[t]
            for p in range(rp[v], rp[v + 1]):
                y = int(ci[p])
                if y != v and rank[y] < 0:
                    deg[y] -= 1
                    touched.add(y)
        removed += take
        carried = None
        if carry:
            low = sorted(y for y in touched if deg[y] == delta - 1)
            join = [y for y in touched if deg[y] == delta]
            left = int(np.sum((rank < 0) & (deg == delta)))
            if low:
                carried, carried_delta = low, delta - 1
            elif left > 0:
                rest = list(cand[take:m])
                limit = float("inf") if len(rest) + len(join) == left else cand[m - 1]
                nxt = sorted(rest + [y for y in join if y < limit])
                if nxt:
                    carried, carried_delta = nxt, delta
    return rank, steps


def _random_graph(rng, n, p, loops):
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    adj = oracle.edges_to_adj(n, edges)
    if loops:
        for v in rng.sample(range(n), max(1, n // 4)):
            adj[v] = sorted(set(adj[v]) | {v})
    return oracle.adj_to_csr(adj)


@pytest.mark.parametrize("carry", [False, True])
def test_random_graphs_random_chunks_and_cuts(carry):
    rng = random.Random(5)
    for trial in range(400):
        n = rng.randint(1, 26)
        rp, ci = _random_graph(rng, n, rng.uniform(0.02, 0.7), trial % 4 == 0)
        rank, _ = peel_by_steps(n, rp, ci, rng, carry=carry, exact=True)
        want, _ = oracle.smallest_last_rank(rp, ci)
        assert np.array_equal(rank, want), trial


@pytest.mark.parametrize("chunk,stage", [(1024, 2048), (64, 2048), (7, 5), (1, 1)])
def test_structured_graphs(chunk, stage):
    rng = random.Random(9)
    for g in [graphgen.rmat(9, 8, (0.57, 0.19, 0.19), 3), graphgen.grid((9, 11), True), graphgen.complete(30),
              graphgen.star(40, 7), graphgen.path(50), graphgen.complete_bipartite(6, 13)]:
        rank, steps = peel_by_steps(g.n, g.row_ptr, g.col_idx, rng, chunk, stage)
        want, _ = oracle.smallest_last_rank(g.row_ptr, g.col_idx)
        assert np.array_equal(rank, want)
        assert steps <= g.n


def test_one_candidate_a_step_is_the_plain_peel():
    """Chunks of one candidate: every step removes exactly the first, so the
    steps are the n removals of the one-at-a-time process."""
    rng = random.Random(2)
    g = graphgen.rmat(8, 8, (0.57, 0.19, 0.19), 1)
    rank, steps = peel_by_steps(g.n, g.row_ptr, g.col_idx, rng, chunk=1, stage=2048, carry=False)
    assert steps == g.n
    assert np.array_equal(rank, oracle.smallest_last_rank(g.row_ptr, g.col_idx)[0])
