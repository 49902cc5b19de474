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


def _check_blocks(got, ref, rel, floor, what):
    """Entry by entry, per parameter block: |got - ref| <= rel |ref| +
    floor * max |ref| over the block (so that a small block such as b3 or W3
    is judged on its own scale)."""
    for name, lo, hi in (("W1", OL.W1, OL.B1), ("b1", OL.B1, OL.W2), ("W2", OL.W2, OL.B2), ("b2", OL.B2, OL.W3),
                         ("W3", OL.W3, OL.B3), ("b3", OL.B3, OL.NPARAM)):
        g, r = got[lo:hi], ref[lo:hi]
        scale = np.abs(r).max()
        tol = rel * np.abs(r) + floor * scale
        bad = np.abs(g - r) > tol
        ratio = float((np.abs(g - r) / np.maximum(tol, 1e-300)).max())
        print("%s %s: max |err| / tol = %.3g (block scale %.3g)" % (what, name, ratio, scale))
        assert not bad.any(), (what, name, int(bad.sum()), np.flatnonzero(bad)[:5])


def test_gradient_matches_oracle():
    """Every gradient entry against the FP64 analytic gradient at the same
    BF16 weights (the GPU accumulates in FP32)."""
    from paper_1205_3809_amd import learned as L
    g = graphgen.rmat(13, 16, TRAIN_ABCD, 7)
    F = OL.features(g.row_ptr, g.col_idx).astype(np.float32)
    rank, _ = L.smallest_last_rank(g.row_ptr, g.col_idx)
    t = L.rank_targets(dev(rank)).cpu().numpy()
    m = _model_with_norm(F.astype(np.float64), seed=4)
    rng = np.random.default_rng(0)
    for size in (5000, 33, 1):
        idx = rng.choice(g.n, size, replace=False).astype(np.int32)
        gg = m.grad(dev(idx), dev(F), dev(t)).cpu().numpy().astype(np.float64)
        params = OL.unpack(m.master.cpu().numpy(), m.wbf.cpu().numpy().view(np.uint16))
        X = OL.normalise(F[idx].astype(np.float64), m.norm.cpu().numpy())
        ref, loss = OL.grad(X, t[idx].astype(np.float64), params)
        assert abs(gg[-1] - loss) <= 1e-4 * max(loss, 1e-3)
        _check_blocks(gg[:-1], ref, 2e-3, 2e-4, "grad batch %d" % size)


def test_adam_matches_oracle():
    """k_adam against one FP64 Adam step from the same FP32 state (moments
    not zero, step 3): master weights and moments within FP32 rounding of
    the step, BF16 copies the nearest-even rounding of the new masters."""
    from paper_1205_3809_amd import learned as L
    rng = np.random.default_rng(11)
    m = L.MLP(seed=2)
    w0 = m.master.cpu().numpy().astype(np.float64)
    mom = rng.normal(0, 0.05, OL.NPARAM).astype(np.float32)
    vel = rng.uniform(0, 0.01, OL.NPARAM).astype(np.float32)
    vel[:7] = 0.0  # zero second moment with a zero gradient below
    grad = rng.normal(0, 0.1, OL.NPARAM + 1).astype(np.float32)
    grad[:4] = 0.0
    m.mom = dev(mom)
    m.vel = dev(vel)
    m.step = 2
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-8
    m.adam(dev(grad), lr=lr, beta1=b1, beta2=b2, eps=eps)
    # the kernel receives the hyperparameters as FP32 values (1 - 0.999f is
    # 0.00099998713...): the oracle takes those same values
    lr, b1, b2, eps = (float(np.float32(x)) for x in (lr, b1, b2, eps))
    w_ref, m_ref, v_ref = OL.adam_step(w0, mom, vel, grad[:OL.NPARAM], 3, lr, b1, b2, eps)
    w = m.master.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(w - w_ref) <= 1e-6 * np.abs(w_ref) + 2e-5 * lr), np.abs(w - w_ref).max()
    # FP32 rounding of b1 m + (1 - b1) g: a few units in the last place of
    # the larger term (the sum itself may cancel); the second moment sums
    # non-negative terms, so it is relatively accurate
    ulp = 2.0 ** -23
    m_bound = 4 * ulp * (np.abs(b1 * mom.astype(np.float64)) + np.abs((1 - b1) * grad[:OL.NPARAM].astype(np.float64)))
    assert np.all(np.abs(m.mom.cpu().numpy() - m_ref) <= m_bound + 1e-30)
    assert np.allclose(m.vel.cpu().numpy(), v_ref, rtol=8 * ulp, atol=1e-30)
    assert np.array_equal(OL.bf16_bits_to_f64(m.wbf.cpu().numpy().view(np.uint16)),
                          OL.bf16_round(m.master.cpu().numpy()))


def test_feature_stats_and_norm_match_oracle():
    """Sums of log1p(feature) and their squares (FP64 on the device), split
    over two calls, and the normalisation computed from them on the device."""
    from paper_1205_3809_amd import learned as L
    g1 = graphgen.rmat(14, 16, TRAIN_ABCD, 2)
    g2 = graphgen.uniform(3000, 20000, 4)
    F1 = L.features(dev(g1.row_ptr), dev(g1.col_idx))
    F2 = L.features(dev(g2.row_ptr), dev(g2.col_idx))
    m = L.MLP(seed=0)
    m.fit_norm([F1, F2])
    acc = torch.zeros(16, dtype=torch.float64, device="cuda")
    for f in (F1, F2):
        assert L.B._lib.gcolor_feature_stats(f.shape[0], L._vp(f), L._vp(acc), L._stream()) == 0
    Fh = np.concatenate([F1.cpu().numpy(), F2.cpu().numpy()]).astype(np.float64)
    ref = OL.feature_sums(Fh)
    assert np.allclose(acc.cpu().numpy(), ref, rtol=1e-12, atol=1e-9)
    norm_ref = OL.norm_from_sums(ref, Fh.shape[0])
    assert np.allclose(m.norm.cpu().numpy(), norm_ref, rtol=1e-6, atol=1e-12)


def test_rank_targets_match_oracle():
    from paper_1205_3809_amd import learned as L
    for n in (1, 2, 1000, 65536):
        r = np.random.default_rng(n).permutation(n).astype(np.int32)
        got = L.rank_targets(dev(r)).cpu().numpy().astype(np.float64)
        ref = OL.rank_target(r)
        assert np.allclose(got, ref, rtol=2 ** -23, atol=1e-30), n


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


def test_order_learned_single_call():
    """gcolor_order_learned (features, forward and key map in one call, caller
    workspace) gives the keys of the three separate calls bit for bit;
    a NaN score sets the flag; a short workspace is refused."""
    from paper_1205_3809_amd import learned as L
    g = graphgen.rmat(15, 16, TRAIN_ABCD, 21)
    rp, ci = dev(g.row_ptr), dev(g.col_idx)
    m = L.MLP(seed=5)
    m.fit_norm([L.features(rp, ci)])
    keys, bad = L.order_learned(m, rp, ci)
    assert int(bad.item()) == 0
    k2, bad2 = L.keys_from_scores(m.scores(L.features(rp, ci)))
    assert int(bad2.item()) == 0
    assert torch.equal(keys, k2)
    # the keys colour as the oracle does with them
    ref = oracle.spec_sim(g.row_ptr, g.col_idx, keys.cpu().numpy().view(np.uint32), threads=0)
    col = L.B.color_graph(rp, ci, keys)
    assert np.array_equal(col.cpu().numpy(), ref.colors)
    n = g.n
    nb = int(L.B._lib.gcolor_order_learned_workspace_bytes(n))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = L.B._lib.gcolor_order_learned(n, L._vp(rp), L._vp(ci), 0x5EED, L._vp(m.master), L._vp(m.wbf), L._vp(m.norm),
                                       L._vp(out), L._vp(flag), L._vp(ws), nb - 1, L._stream())
    assert rc == -3  # GCOLOR_EWORKSPACE
    m.master[L.B3] = float("nan")
    rc = L.B._lib.gcolor_order_learned(n, L._vp(rp), L._vp(ci), 0x5EED, L._vp(m.master), L._vp(m.wbf), L._vp(m.norm),
                                       L._vp(out), L._vp(flag), L._vp(ws), nb, L._stream())
    assert rc == 0 and int(flag.item()) == 1


def test_learned_at_configured_scale():
    """The configured learned-ordering workload: train on 256 R-MAT scale-16
    edge-factor-16 graphs (0.57, 0.19, 0.19, 0.05) with exact smallest-last
    targets, then colour the unseen scale-22 graph (seed 1000) with the
    learned keys.  The colouring equals the oracle's with the same keys,
    vertex for vertex, and uses no more colours than natural order; the
    colour counts of largest-degree-first and exact smallest-last are
    reported beside it."""
    import time

    from paper_1205_3809_amd import learned as L
    t0 = time.time()
    train = [graphgen.rmat(16, 16, TRAIN_ABCD, s) for s in range(256)]
    m = L.MLP(seed=0)
    rep = L.train(m, [(g.row_ptr, g.col_idx) for g in train], epochs=4, batch=65536, lr=2e-3)
    del train
    print("trained in %.1fs (loss %.5f -> %.5f)" % (time.time() - t0, rep.losses[0], rep.losses[-1]), flush=True)
    ev = graphgen.rmat(22, 16, TRAIN_ABCD, 1000)
    rp, ci = dev(ev.row_ptr), dev(ev.col_idx)
    keys, bad = L.order_learned(m, rp, ci)
    assert int(bad.item()) == 0
    col, st = L.B.color_graph_ex(rp, ci, keys, stats=True)
    k = keys.cpu().numpy().view(np.uint32)
    t0 = time.time()
    ref = oracle.spec_sim(ev.row_ptr, ev.col_idx, k, threads=0)
    print("oracle with learned keys: %.1fs, %d rounds" % (time.time() - t0, ref.rounds), flush=True)
    got = col.cpu().numpy()
    assert np.array_equal(got, ref.colors), int((got != ref.colors).sum())
    assert st.rounds == ref.rounds
    src = np.repeat(np.arange(ev.n), np.diff(ev.row_ptr))
    assert got.min() >= 1 and not np.any(got[src] == got[ev.col_idx])
    nat, st_nat = L.B.color_graph_ex(rp, ci, None, stats=True)
    deg = np.diff(ev.row_ptr.astype(np.int64))
    lf = np.empty(ev.n, dtype=np.int32)
    lf[np.lexsort((np.arange(ev.n), -deg))] = np.arange(ev.n, dtype=np.int32)
    _, st_lf = L.B.color_graph_ex(rp, ci, dev(lf), stats=True)
    rank, _ = L.smallest_last_rank(ev.row_ptr, ev.col_idx)
    _, st_sl = L.B.color_graph_ex(rp, ci, dev(rank), stats=True)
    print("colours: natural %d, learned %d, largest-degree-first %d, exact smallest-last %d"
          % (st_nat.num_colors, st.num_colors, st_lf.num_colors, st_sl.num_colors), flush=True)
    assert st.num_colors <= st_nat.num_colors
