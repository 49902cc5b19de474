"""The oracle's pins catch plausible mistakes.

Each mutant below is a copy of the round-synchronous definition with one
planted mistake (all on the CPU).  The same battery of pins the oracle passes
(brute force, closed forms, invariants) must reject every mutant.
"""
import math

import numpy as np

import graphgen
import oracle


def _adj(g):
    return oracle.adjacency(g.row_ptr, g.col_idx)


def _ok_key(key, v):
    return (int(key[v]) if key is not None else v, v)


def sim_reference(adj, key=None):
    c, k, _ = oracle.spec_sim_py(adj, key)
    return c, k


def sim_live_reads(adj, key=None):
    """Mistake: phase 1 sees tentative colours of this round (no snapshot)."""
    n = len(adj)
    color = [0] * n
    U = list(range(n))
    k = 0
    while U:
        k += 1
        for v in U:
            color[v] = oracle.first_fit({color[w] for w in adj[v] if color[w] > 0})
        R = [v for v in U if any(color[w] == color[v] and _ok_key(key, w) < _ok_key(key, v) for w in adj[v])]
        for v in R:
            color[v] = 0
        U = R
    return color, k


def sim_stale_losers(adj, key=None):
    """Mistake: losers keep their stale tentative colour (the literal text)."""
    n = len(adj)
    color = [0] * n
    U = list(range(n))
    k = 0
    while U and k < 10 * n + 10:
        k += 1
        snap = list(color)
        Uset = set(U)
        tent = {v: oracle.first_fit({snap[w] for w in adj[v] if snap[w] > 0 and w != v}) for v in U}
        for v in U:
            color[v] = tent[v]
        U = [v for v in U if any(color[w] == color[v] and _ok_key(key, w) < _ok_key(key, v) for w in adj[v])]
    return color, k


def sim_reversed_tiebreak(adj, key=None):
    """Mistake: the earlier vertex of a conflicting pair is re-queued."""
    n = len(adj)
    color = [0] * n
    U = list(range(n))
    k = 0
    while U:
        k += 1
        snap = list(color)
        tent = {v: oracle.first_fit({snap[w] for w in adj[v] if snap[w] > 0}) for v in U}
        for v in U:
            color[v] = tent[v]
        R = [v for v in U if any(color[w] == color[v] and _ok_key(key, w) > _ok_key(key, v) for w in adj[v])]
        for v in R:
            color[v] = 0
        U = R
    return color, k


def sim_both_lose(adj, key=None):
    """Mistake: both ends of a conflict are re-queued."""
    n = len(adj)
    color = [0] * n
    U = list(range(n))
    k = 0
    while U and k < 4 * n + 4:
        k += 1
        snap = list(color)
        tent = {v: oracle.first_fit({snap[w] for w in adj[v] if snap[w] > 0}) for v in U}
        for v in U:
            color[v] = tent[v]
        R = [v for v in U if any(color[w] == color[v] for w in adj[v])]
        for v in R:
            color[v] = 0
        U = R
    return color, k


def sim_off_by_one(adj, key=None):
    """Mistake: first-fit skips colour 1 once anything is forbidden."""
    def ff(forb):
        c = 2 if forb else 1
        while c in forb:
            c += 1
        return c
    n = len(adj)
    color = [0] * n
    U = list(range(n))
    k = 0
    while U:
        k += 1
        snap = list(color)
        tent = {v: ff({snap[w] for w in adj[v] if snap[w] > 0}) for v in U}
        for v in U:
            color[v] = tent[v]
        R = [v for v in U if any(color[w] == color[v] and _ok_key(key, w) < _ok_key(key, v) for w in adj[v])]
        for v in R:
            color[v] = 0
        U = R
    return color, k


def sim_ignore_key(adj, key=None):
    """Mistake: the priority array is ignored (index order always)."""
    return sim_reference(adj, None)


def battery(sim):
    """Names of the pins that `sim` violates."""
    failed = []
    for n in (4, 6, 10):
        c, k = sim(_adj(graphgen.cycle(n)))
        if max(c) != 2 or k != n // 2:
            failed.append("even_cycle_%d" % n)
    for n in (5, 9):
        c, k = sim(_adj(graphgen.path(n)))
        if c != [1 + v % 2 for v in range(n)] or k != 1 + math.ceil((n - 1) / 2):
            failed.append("path_%d" % n)
    for n in (3, 5):
        c, k = sim(_adj(graphgen.complete(n)))
        if sorted(c) != list(range(1, n + 1)) or k != n:
            failed.append("complete_%d" % n)
    c, k = sim(_adj(graphgen.complete_bipartite(3, 4)))
    if c != [1] * 3 + [2] * 4 or k != 2:
        failed.append("kpq")
    c, k = sim(_adj(graphgen.star(6, 5)))
    if max(c) != 2 or k != 2 or c[5] != 2:
        failed.append("star_last")
    rng = np.random.default_rng(3)
    for t in range(30):
        n = int(rng.integers(5, 12))
        adj = oracle.edges_to_adj(n, [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.4])
        key = list(rng.permutation(n))
        c, k = sim(adj, key)
        if not oracle.is_proper(adj, c) or max(c) > k:
            failed.append("proper_%d" % t)
        # the smallest-key vertex keeps colour 1 in round 1
        first = min(range(n), key=lambda v: key[v])
        if c[first] != 1:
            failed.append("min_key_%d" % t)
    return failed


def test_reference_passes_battery():
    assert battery(sim_reference) == []


def test_each_mutant_is_caught():
    for mut in (sim_live_reads, sim_stale_losers, sim_reversed_tiebreak, sim_both_lose,
                sim_off_by_one, sim_ignore_key):
        assert battery(mut), mut.__name__
