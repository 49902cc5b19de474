"""Pins of the learned-ordering oracle (CPU only): the hash against splitmix64's
published first output, features against closed forms and brute force, the
analytic gradient against central finite differences, BF16 rounding and the
order-preserving key map; and the library's host smallest-last routine
against the oracle's."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import learned as OL


def test_mix_matches_splitmix64_reference():
    # splitmix64 started from state 0 first returns mix(0 + GAMMA)
    assert OL.mix_int(OL.GAMMA) == 0xE220A8397B1DCDAF
    rng = np.random.default_rng(0)
    vals = rng.integers(0, 2 ** 63, 200, dtype=np.uint64)
    arr = OL.mix(vals)
    assert all(int(a) == OL.mix_int(int(v)) for a, v in zip(arr, vals))


def _adj(g):
    return oracle.adjacency(g.row_ptr, g.col_idx)


@pytest.mark.parametrize("n", [3, 4, 7, 12])
def test_features_complete_graph(n):
    g = graphgen.complete(n)
    F = OL.features(g.row_ptr, g.col_idx)
    d = n - 1
    assert np.allclose(F[:, 0], d) and np.allclose(F[:, 2:5], d)
    assert np.allclose(F[:, 1], np.log2(1 + d))
    assert np.allclose(F[:, 5], d * (d - 1))
    assert np.allclose(F[:, 6], d * (d - 1) / 2)  # every wedge closes
    assert np.allclose(F[:, 7], d)


def test_features_star_and_cycle():
    n = 9
    F = OL.features(*graphgen.star(n, 0)[1:])
    assert F[0, 0] == n - 1 and F[0, 2] == F[0, 4] == 1 and F[0, 5] == 0 and F[0, 6] == 0 and F[0, 7] == 1
    assert np.all(F[1:, 0] == 1) and np.all(F[1:, 3] == n - 1) and np.all(F[1:, 5] == n - 2)
    assert np.all(F[1:, 6] == 0) and np.all(F[1:, 7] == 1)
    C = OL.features(*graphgen.cycle(10)[1:])
    assert np.all(C[:, 0] == 2) and np.all(C[:, 6] == 0) and np.all(C[:, 7] == 2)
    T = OL.features(*graphgen.cycle(3)[1:])
    assert np.all(T[:, 6] == 1)  # the single wedge of a triangle vertex closes


def test_features_against_loops():
    g = graphgen.rmat(9, 8, (0.55, 0.15, 0.15), 3)
    adj = _adj(g)
    deg = [len(a) for a in adj]
    F = OL.features(g.row_ptr, g.col_idx, seed=11)
    eset = {(u, w) for u in range(g.n) for w in adj[u]}
    x = list(deg)
    for _ in range(OL.CORE_STEPS):
        x = [max([k for k in range(deg[v] + 1) if sum(1 for w in adj[v] if x[w] >= k) >= k], default=0)
             for v in range(g.n)]
    for v in range(g.n):
        nd = [deg[w] for w in adj[v]]
        d = deg[v]
        assert F[v, 7] == x[v]
        if d:
            assert F[v, 2] == min(nd) and F[v, 4] == max(nd) and np.isclose(F[v, 3], sum(nd) / d)
            assert F[v, 5] == sum(x - 1 for x in nd)
        if d >= 2:
            closed = 0
            for i in range(8):
                hh = OL.mix_int(11 * OL.GAMMA + OL.mix_int(8 * v + i + 1))
                a = (hh & 0xFFFFFFFF) % d
                b = (hh >> 32) % (d - 1)
                b += b >= a
                closed += (adj[v][a], adj[v][b]) in eset
            assert np.isclose(F[v, 6], closed / 8 * d * (d - 1) / 2)


def _coreness_by_peeling(adj):
    """Core numbers from their definition: repeatedly delete a vertex of
    least remaining degree; a vertex's core number is the largest such
    least degree seen up to its deletion."""
    n = len(adj)
    alive = set(range(n))
    deg = {v: len(set(adj[v]) - {v}) for v in range(n)}
    core = [0] * n
    k = 0
    while alive:
        v = min(alive, key=lambda u: (deg[u], u))
        k = max(k, deg[v])
        core[v] = k
        alive.remove(v)
        for w in set(adj[v]) - {v}:
            if w in alive:
                deg[w] -= 1
    return core


@pytest.mark.parametrize("n", [3, 4, 5, 9, 16])
def test_core_estimate_on_paths(n):
    """Path 0 - 1 - ... - (n-1): after k steps a vertex at distance j from the
    nearer end holds 1 if j <= k, else 2 (step 0 is the degrees; each step
    carries the ends' 1 one vertex inward, since an interior vertex keeps 2
    only while both neighbours hold 2)."""
    g = graphgen.path(n)
    for k in range(n + 1):
        h = OL.core_estimate(g.row_ptr, g.col_idx, k)
        want = [1 if min(v, n - 1 - v) <= k else 2 for v in range(n)]
        assert list(h) == want, (n, k)


def test_core_estimate_falls_to_the_coreness():
    """The H sequence never rises, stays at or above the core numbers at
    every step, and reaches them (Lu et al. 2016); n steps always suffice on
    these graphs.  Core numbers come from peeling, not from H."""
    rng = np.random.default_rng(3)
    graphs = [graphgen.rmat(9, 8, (0.57, 0.19, 0.19), 1), graphgen.star(12, 4), graphgen.complete(6),
              graphgen.grid((5, 7), True)]
    for _ in range(60):
        n = int(rng.integers(2, 24))
        p = rng.uniform(0.05, 0.6)
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
        rp, ci = oracle.adj_to_csr(oracle.edges_to_adj(n, edges))
        graphs.append((n, rp, ci))
    for g in graphs:
        n, rp, ci = (g.n, g.row_ptr, g.col_idx) if isinstance(g, graphgen.CSR) else g
        core = np.array(_coreness_by_peeling(oracle.adjacency(rp, ci)))
        prev = np.diff(np.asarray(rp, dtype=np.int64))
        for k in range(1, n + 2):
            h = OL.core_estimate(rp, ci, k)
            assert np.all(h <= prev) and np.all(h >= core), k
            prev = h
        assert np.array_equal(prev, core)


def test_core_estimate_on_a_clique_with_a_tail():
    """K_5 on vertices 0..4 with a path 4 - 5 - 6 - 7 hanging off vertex 4:
    the clique's core number is 4 and the tail's 1; the clique vertices hold
    4 from the first step on (four neighbours of degree >= 4), the tail's
    end 7 holds 1 from the start, vertex 6 drops to 1 at the first step (its
    neighbour 7 has degree 1) and vertex 5 at the second (its neighbour 6
    then holds 1)."""
    edges = [(i, j) for i in range(5) for j in range(i + 1, 5)] + [(4, 5), (5, 6), (6, 7)]
    rp, ci = oracle.adj_to_csr(oracle.edges_to_adj(8, edges))
    assert list(OL.core_estimate(rp, ci, 0)) == [4, 4, 4, 4, 5, 2, 2, 1]
    assert list(OL.core_estimate(rp, ci, 1)) == [4, 4, 4, 4, 4, 2, 1, 1]
    assert list(OL.core_estimate(rp, ci, 2)) == [4, 4, 4, 4, 4, 1, 1, 1]


def _random_model(seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.4, OL.NPARAM)
    return OL.params_from_vector(p), p


def test_gradient_matches_finite_differences():
    params, p = _random_model(1)
    rng = np.random.default_rng(2)
    X = rng.normal(0, 1, (37, OL.NF))
    t = rng.uniform(0, 1, 37)
    g, _ = OL.grad(X, t, params)
    h = 1e-6
    for j in list(range(0, OL.NPARAM, 97)) + [OL.B3, OL.W3 + 5, OL.B1 + 3, OL.B2 + 7]:
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        fd = (OL.loss(X, t, OL.params_from_vector(pp)) - OL.loss(X, t, OL.params_from_vector(pm))) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), (j, fd, g[j])


def test_gradient_descent_reduces_loss():
    rng = np.random.default_rng(4)
    p = rng.normal(0, 0.1, OL.NPARAM)
    params = OL.params_from_vector(p)
    X = rng.normal(0, 1, (200, OL.NF))
    t = np.tanh(X[:, 0]) * 0.5 + 0.5
    l0 = OL.loss(X, t, params)
    for _ in range(200):
        g, _ = OL.grad(X, t, OL.params_from_vector(p))
        p = p - 0.02 * g
    assert OL.loss(X, t, OL.params_from_vector(p)) < 0.5 * l0


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159, 0.0], dtype=np.float32)
    r = OL.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0  # halfway: ties to even
    assert r[2] == 1.0 + 2 ** -7        # above halfway rounds up
    assert r[3] == -2.5 and r[5] == 0.0
    assert abs(r[4] - 3.14159) < 2 ** -7 * 4


def test_keys_preserve_order():
    rng = np.random.default_rng(5)
    s = np.concatenate([rng.normal(0, 3, 500), [0.0, -0.0, 1e-30, -1e-30, 1e30, -1e30]]).astype(np.float32)
    k = OL.keys_from_scores(s).astype(np.int64)
    lt = s[:, None] < s[None, :]
    assert np.all(k[:, None] < k[None, :], where=lt)      # strictly ordered where the scores are
    eq = (s[:, None] == s[None, :]) & (np.signbit(s)[:, None] == np.signbit(s)[None, :])
    assert np.all(k[:, None] == k[None, :], where=eq)     # equal scores, equal keys (-0.0 below +0.0)


def test_library_host_smallest_last_matches_oracle():
    """The library's host smallest-last routine (the training targets) against
    the oracle's, on random and structured graphs."""
    from paper_1205_3809_amd import learned as L
    for g in [graphgen.rmat(12, 16, (0.57, 0.19, 0.19), 1), graphgen.uniform(3000, 15000, 2),
              graphgen.grid((20, 30), True), graphgen.complete(9), graphgen.star(50, 17), graphgen.empty(4)]:
        r, d = L.smallest_last_rank(g.row_ptr, g.col_idx)
        ro, do = oracle.smallest_last_rank(g.row_ptr, g.col_idx)
        assert np.array_equal(r, ro) and d == do


def test_adam_two_steps_by_hand():
    """Adam with beta1 = 1/2, beta2 = 3/4, lr = 1, eps = 0 from zero moments,
    worked out by hand: gradient 2 gives m = 1, v = 1, bias-corrected 2 and
    4, a step of 2 / 2 = 1; then gradient -2 gives m = 1/2 - 1 = -1/2,
    v = 3/4 + 1 = 7/4, corrected -1/2 / (3/4) = -2/3 and (7/4) / (7/16) = 4,
    a step of (-2/3) / 2 = -1/3."""
    w, m, v = OL.adam_step(np.array([5.0]), np.zeros(1), np.zeros(1), np.array([2.0]), 1, 1.0, 0.5, 0.75, 0.0)
    assert np.allclose([w[0], m[0], v[0]], [4.0, 1.0, 1.0], rtol=1e-15)
    w, m, v = OL.adam_step(w, m, v, np.array([-2.0]), 2, 1.0, 0.5, 0.75, 0.0)
    assert np.allclose([w[0], m[0], v[0]], [4.0 + 1.0 / 3.0, -0.5, 1.75], rtol=1e-15)


def test_adam_constant_gradient_moves_by_lr():
    """With a constant gradient g the bias-corrected moments are g and g^2 at
    every step, so each step moves every parameter by lr * g / (|g| + eps)
    (= lr * sign(g) for eps = 0), independent of the betas."""
    g = np.array([3.0, -0.25, 1e-3, -7.0])
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for step in range(1, 6):
        w, m, v = OL.adam_step(w, m, v, g, step, 0.01, 0.9, 0.999, 0.0)
        assert np.allclose(w, -0.01 * step * np.sign(g), rtol=1e-12, atol=1e-15)
    # zero gradient with zero moments: no move (0 / (0 + eps))
    w2, _, _ = OL.adam_step(np.ones(3), np.zeros(3), np.zeros(3), np.zeros(3), 1, 0.1, 0.9, 0.999, 1e-8)
    assert np.array_equal(w2, np.ones(3))


def test_normalisation_closed_forms():
    """Feature e - 1 (log1p = 1) on every vertex: mean 1, spread 0 (floored
    at 1e-6); features e^a - 1 and e^b - 1 on half the vertices each: mean
    (a + b) / 2, standard deviation |a - b| / 2."""
    n = 10
    F = np.zeros((n, OL.NF))
    F[:, 0] = np.e - 1.0
    F[:5, 1] = np.expm1(1.0)
    F[5:, 1] = np.expm1(3.0)
    F[:, 2] = 0.0
    norm = OL.norm_from_sums(OL.feature_sums(F), n)
    assert abs(norm[0] - 1.0) < 1e-12 and abs(norm[OL.NF] - 1e-6) < 1e-12
    assert abs(norm[1] - 2.0) < 1e-12 and abs(norm[OL.NF + 1] - 1.0) < 1e-9
    assert norm[2] == 0.0 and abs(norm[OL.NF + 2] - 1e-6) < 1e-12
    # sums over parts add up: the statistics of a union are the sums of the parts
    s = OL.feature_sums(F[:3]) + OL.feature_sums(F[3:])
    assert np.allclose(s, OL.feature_sums(F), rtol=1e-14)


def test_rank_target_closed_forms():
    """Position 0 maps to 0, position n - 1 to log(n) / log(n) = 1, and
    position sqrt(n) - 1 to 1/2; the map is strictly increasing."""
    n = 1024
    t = OL.rank_target(np.arange(n))
    assert t[0] == 0.0 and abs(t[n - 1] - 1.0) < 1e-15 and abs(t[31] - 0.5) < 1e-15
    assert np.all(np.diff(t) > 0)
    assert np.array_equal(OL.rank_target(np.zeros(1)), [0.0])
