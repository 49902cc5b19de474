"""Learned ordering on the GPU vs the FP64 CPU oracle: features, MLP forward
(within 1e-2 relative), gradients, key map; training reduces the loss, and
the trained ordering colours with no more colours than natural order."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from oracle import learned as OL

pytestmark = pytest.mark.gpu

TRAIN_ABCD = (0.57, 0.19, 0.19)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def hub_of_hubs(d=6000, top=9000, pool=10000):
    """Vertex 0 joined to 1..d; vertex i also joined to top // i vertices of a
    pool: neighbour degrees reach top + 1, so the hub's h-index search range
    (min(degree, max neighbour degree) = d > 4096) takes more than one
    histogram pass."""
    src = [np.zeros(d, np.int64)]
    dst = [np.arange(1, d + 1)]
    rng = np.random.default_rng(3)
    for i in range(1, d + 1):
        k = top // i
        src.append(np.full(k, i))
        dst.append(d + 1 + rng.choice(pool, k, replace=False))
    return graphgen.from_pairs(d + 1 + pool, np.concatenate(src), np.concatenate(dst))


def test_features_match_oracle():
    from paper_1205_3809_amd import learned as L
    for g in [graphgen.rmat(14, 16, TRAIN_ABCD, 5), graphgen.rmat(17, 16, TRAIN_ABCD, 9), hub_of_hubs(),
              graphgen.grid((30, 40), True), graphgen.complete(20), graphgen.complete(300),
              graphgen.star(5000, 3), graphgen.empty(7)]:
        got = L.features(dev(g.row_ptr), dev(g.col_idx), 123).cpu().numpy().astype(np.float64)
        ref = OL.features(g.row_ptr, g.col_idx, 123)
        assert got.shape == ref.shape
        for f in (0, 2, 4, 7):
            assert np.array_equal(got[:, f], ref[:, f]), f
        assert np.allclose(got, ref, rtol=2e-6, atol=1e-6)


def test_features_at_evaluation_scale():
    """All features of every vertex of the scale-22 evaluation graph (hubs
    above 160,000 neighbours): integer features exact, the others within
    2e-6 relative."""
    from paper_1205_3809_amd import learned as L
    g = graphgen.rmat(22, 16, TRAIN_ABCD, 1000)
    print("features rmat22: n=%d nnz=%d" % (g.n, g.nnz), flush=True)
    got = L.features(dev(g.row_ptr), dev(g.col_idx), 123).cpu().numpy().astype(np.float64)
    ref = OL.features(g.row_ptr, g.col_idx, 123)
    for f in (0, 2, 4, 7):
        assert np.array_equal(got[:, f], ref[:, f]), f
    assert np.allclose(got, ref, rtol=2e-6, atol=1e-6)


def _model_with_norm(g_feats_ref, seed=0):
    from paper_1205_3809_amd import learned as L
    m = L.MLP(seed=seed)
    lf = np.log1p(g_feats_ref)
    norm = np.r_[lf.mean(0), lf.std(0) + 1e-3].astype(np.float32)
    m.norm = dev(norm)
    return m


def test_forward_matches_oracle():
    from paper_1205_3809_amd import learned as L
    g = graphgen.rmat(15, 16, TRAIN_ABCD, 6)
    F = OL.features(g.row_ptr, g.col_idx)
    m = _model_with_norm(F, seed=3)
    got = m.scores(dev(F.astype(np.float32))).cpu().numpy().astype(np.float64)
    params = OL.unpack(m.master.cpu().numpy(), m.wbf.cpu().numpy().view(np.uint16))
    X = OL.normalise(F.astype(np.float32).astype(np.float64), m.norm.cpu().numpy())
    ref, _ = OL.forward(X, params)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-2)
    print("forward: max relative error %.3g over %d vertices" % (err.max(), err.size))
    assert err.max() < 1e-2, err.max()


def test_gradient_matches_oracle():
    from paper_1205_3809_amd import learned as L
    g = graphgen.rmat(13, 16, TRAIN_ABCD, 7)
    F = OL.features(g.row_ptr, g.col_idx).astype(np.float32)
    rank, _ = L.smallest_last_rank(g.row_ptr, g.col_idx)
    t = L.rank_target(rank)
    m = _model_with_norm(F.astype(np.float64), seed=4)
    rng = np.random.default_rng(0)
    idx = rng.choice(g.n, 5000, replace=False).astype(np.int32)
    gg = m.grad(dev(idx), dev(F), dev(t)).cpu().numpy().astype(np.float64)
    params = OL.unpack(m.master.cpu().numpy(), m.wbf.cpu().numpy().view(np.uint16))
    X = OL.normalise(F[idx].astype(np.float64), m.norm.cpu().numpy())
    ref, loss = OL.grad(X, t[idx].astype(np.float64), params)
    assert abs(gg[-1] - loss) <= 1e-4 * max(loss, 1e-3)
    assert np.linalg.norm(gg[:-1] - ref) <= 1e-3 * np.linalg.norm(ref)


def test_keys_match_oracle():
    from paper_1205_3809_amd import learned as L
    s = np.concatenate([np.random.default_rng(1).normal(0, 2, 10000), [0.0, -0.0, 3e38, -3e38]]).astype(np.float32)
    keys, bad = L.keys_from_scores(dev(s))
    assert int(bad.item()) == 0
    assert np.array_equal(keys.cpu().numpy().view(np.uint32), OL.keys_from_scores(s))
    _, bad = L.keys_from_scores(dev(np.array([1.0, np.nan], dtype=np.float32)))
    assert int(bad.item()) == 1


def test_training_and_gain():
    """Train on 16 R-MAT scale-14 graphs (edge factor 16, the training
    parameters); the loss falls, and on an unseen scale-16 graph the learned
    order colours (same speculative scheme, priority = learned keys) with at
    most the natural order's colours; the colouring matches the oracle run
    with the same keys."""
    from paper_1205_3809_amd import learned as L
    graphs = [graphgen.rmat(14, 16, TRAIN_ABCD, s) for s in range(16)]
    m = L.MLP(seed=0)
    rep = L.train(m, [(g.row_ptr, g.col_idx) for g in graphs], epochs=8, batch=16384, lr=3e-3)
    assert rep.losses[-1] < 0.6 * rep.losses[0] or rep.losses[-1] < 0.02, rep.losses
    ev = graphgen.rmat(16, 16, TRAIN_ABCD, 1000)
    rp, ci = dev(ev.row_ptr), dev(ev.col_idx)
    keys, bad = L.order_learned(m, rp, ci)
    assert int(bad.item()) == 0
    k = keys.cpu().numpy().view(np.uint32)
    ref = oracle.spec_sim(ev.row_ptr, ev.col_idx, k, threads=0)
    col, used, learned_c, natural_c = L.color_learned(m, rp, ci, fallback=True)
    assert learned_c == int(ref.colors.max())
    nat = oracle.spec_sim(ev.row_ptr, ev.col_idx, threads=0)
    assert natural_c == int(nat.colors.max())
    assert learned_c <= natural_c, (learned_c, natural_c)
    assert used
    assert np.array_equal(col.cpu().numpy(), ref.colors)
