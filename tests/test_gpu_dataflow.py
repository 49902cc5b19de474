"""Dataflow engine (GCOLOR_DATAFLOW) vs the CPU oracle, through the C ABI.

Each case compares colors_out element by element with the oracle's dataflow
colouring (which equals the serial greedy in (priority, id) order), the
round count with the oracle's, and the per-round log with the oracle's
rounds: the vertices coloured in round k are exactly those the oracle puts
in round k (counted, with their degree sum), and the edge work over all
rounds is nnz.  Also: self-loops and repeated pairs for every engine.
"""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu

DATAFLOW = 8


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gpu_color(g, key=None, flags=DATAFLOW):
    import paper_1205_3809_amd as gc
    rp, ci = dev(g.row_ptr), dev(g.col_idx)
    pr = None if key is None else dev(np.ascontiguousarray(key, dtype=np.uint32).view(np.int32))
    col, st = gc.color_graph_ex(rp, ci, pr, flags=flags, stats=True, max_log=1 << 16)
    torch.cuda.synchronize()
    return col.cpu().numpy(), st


def check(g, key=None, label=""):
    print("case %s n=%d nnz=%d key=%s" % (label, g.n, g.nnz, None if key is None else "set"), flush=True)
    ref = oracle.dataflow(g.row_ptr, g.col_idx, key)
    col, st = gpu_color(g, key)
    mism = np.flatnonzero(col != ref.colors)
    assert mism.size == 0, "%s: %d mismatches, first at %s" % (label, mism.size, mism[:5])
    assert st.rounds == ref.rounds
    assert st.num_colors == (int(ref.colors.max()) if g.n else 0)
    assert st.edge_work == g.nnz
    if ref.rounds <= 1 << 16:
        deg = g.degrees()
        per_round = np.bincount(ref.round_of, minlength=ref.rounds + 1)[1:]
        deg_round = np.bincount(ref.round_of, weights=deg, minlength=ref.rounds + 1)[1:].astype(np.int64)
        got = np.array([[k, u, e] for k, u, e in st.round_log], dtype=np.int64).reshape(-1, 3)
        assert np.array_equal(got[:, 0], np.arange(1, ref.rounds + 1))
        assert np.array_equal(got[:, 1], per_round)
        assert np.array_equal(got[:, 2], deg_round)
        assert [d[0] for d in st.detail] == list(per_round)
    return col, st


def test_equals_serial_greedy():
    g = graphgen.rmat(13, 16, (0.57, 0.19, 0.19), 3)
    for key in (None, graphgen.random_priority(g.n, 4)):
        col, _ = check(g, key, "rmat13")
        assert np.array_equal(col, oracle.greedy(g.row_ptr, g.col_idx, key))


@pytest.mark.parametrize("n", [1, 7, 1000])
def test_empty_graph(n):
    col, st = check(graphgen.empty(n), label="empty")
    assert st.rounds == 1 and np.all(col == 1)


@pytest.mark.parametrize("n", [1, 2, 3, 65, 1000, 5000])
def test_paths(n):
    """Natural order: one vertex per round (n rounds); alternating keys: 2."""
    g = graphgen.path(n)
    _, st = check(g, label="path")
    assert st.rounds == n
    check(g, (np.arange(n) % 2).astype(np.uint32), label="path-alt")


@pytest.mark.parametrize("n", [1, 2, 65, 130, 300])
def test_complete_graphs(n):
    col, st = check(graphgen.complete(n), label="complete")
    assert st.rounds == n and list(col) == list(range(1, n + 1))


@pytest.mark.parametrize("n,order", [(600, "natural"), (2100, "natural"), (2100, "perm")])
def test_complete_long_rows(n, order):
    """Rows in the workgroup tier; colours above 255 go through colors_out."""
    g = graphgen.complete(n)
    key = None if order == "natural" else graphgen.random_priority(n, 3)
    col, st = check(g, key, label="complete-%s" % order)
    assert st.num_colors == n


@pytest.mark.parametrize("n,center", [(3000, 0), (3000, 2999), (70000, 123)])
def test_star_hubs(n, center):
    check(graphgen.star(n, center), label="star")


@pytest.mark.parametrize("shape,full", [((64, 64), False), ((37, 41), True), ((16, 16, 16), False),
                                        ((9, 10, 11), True)])
def test_grids(shape, full):
    check(graphgen.grid(shape, full), label="grid%s" % (shape,))


def test_grid_with_extra_edges_and_rgg():
    check(graphgen.grid_with_extra((120, 130), True, 0.05, 3), label="grid+extra")
    check(graphgen.rgg(20000, 12.0, 4), label="rgg")


@pytest.mark.parametrize("order", ["natural", "perm", "ties3", "ties12", "allsame"])
def test_rmat_priorities(order):
    g = graphgen.rmat(14, 8, (0.55, 0.1, 0.1), 3)
    if order == "natural":
        key = None
    elif order == "perm":
        key = graphgen.random_priority(g.n, 8)
    elif order == "allsame":
        key = np.full(g.n, 7, dtype=np.uint32)
    else:
        key = graphgen.random_keys(g.n, 9, bits=int(order[4:]))
    check(g, key, label="rmat14-" + order)


def test_unsorted_rows_with_priority():
    g = graphgen.rmat(12, 8, (0.55, 0.1, 0.1), 5)
    rng = np.random.default_rng(0)
    col = g.col_idx.copy()
    for v in range(g.n):
        s, e = g.row_ptr[v], g.row_ptr[v + 1]
        col[s:e] = rng.permutation(col[s:e])
    key = graphgen.random_priority(g.n, 1)
    got, _ = gpu_color(graphgen.CSR(g.n, g.row_ptr, col), key)
    assert np.array_equal(got, oracle.dataflow(g.row_ptr, g.col_idx, key).colors)


def with_loops_and_repeats(g, seed):
    """g plus self-loops on a tenth of the vertices and a fifth of its edges
    listed a second (some a third) time, in both rows; rows sorted."""
    rng = np.random.default_rng(seed)
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    dst = g.col_idx.astype(np.int64)
    up = np.flatnonzero(src < dst)
    rep = rng.choice(up, up.size // 5, replace=False)
    rep3 = rep[: rep.size // 4]
    loops = rng.choice(g.n, g.n // 10, replace=False)
    s2 = np.concatenate([src, src[rep], dst[rep], src[rep3], dst[rep3], loops])
    d2 = np.concatenate([dst, dst[rep], src[rep], dst[rep3], src[rep3], loops])
    order = np.lexsort((d2, s2))
    s2, d2 = s2[order], d2[order]
    rp = np.zeros(g.n + 1, np.int64)
    np.add.at(rp, s2 + 1, 1)
    return graphgen.CSR(g.n, np.cumsum(rp).astype(np.int32), d2.astype(np.int32))


@pytest.mark.parametrize("flags,name", [(0, "incremental"), (4, "plain"), (DATAFLOW, "dataflow")])
def test_self_loops_and_repeated_pairs(flags, name):
    """Every engine colours the graph with loops and repeated pairs exactly
    as the graph without them."""
    g = graphgen.rmat(13, 8, (0.55, 0.1, 0.1), 6)
    h = with_loops_and_repeats(g, 1)
    assert h.nnz > g.nnz
    for key in (None, graphgen.random_priority(g.n, 2)):
        if flags == DATAFLOW:
            ref = oracle.dataflow(g.row_ptr, g.col_idx, key).colors
        else:
            ref = oracle.spec_sim(g.row_ptr, g.col_idx, key, threads=0).colors
        print("case loops+repeats engine=%s key=%s" % (name, key is not None), flush=True)
        got, _ = gpu_color(h, key, flags=flags)
        assert np.array_equal(got, ref), name


def test_result_independent_of_tuning():
    import paper_1205_3809_amd as gc
    g = graphgen.rmat(15, 8, (0.55, 0.1, 0.1), 6)
    key = graphgen.random_priority(g.n, 2)
    ref = oracle.dataflow(g.row_ptr, g.col_idx, key).colors
    old, bpc = gc.get_tuning()
    try:
        for bins, b in [([0, 0, 0, 0], 2), ([1, 2, 3, 4], 1), ([64, 64, 64, 64], 16), ([1000000] * 4, 3)]:
            gc.set_tuning(bins, b)
            got, _ = gpu_color(g, key)
            assert np.array_equal(got, ref), (bins, b)
    finally:
        gc.set_tuning(old, bpc)


def test_flag_combination_rejected():
    import paper_1205_3809_amd as gc
    g = graphgen.path(10)
    with pytest.raises(gc.GColorError) as e:
        gpu_color(g, flags=DATAFLOW | 4)
    assert e.value.code == -1


@pytest.mark.parametrize("order", ["natural", "perm"])
def test_rmat_scale24(order):
    """The benchmark graph (R-MAT scale 24, edge factor 8, (0.55, 0.1, 0.1,
    0.25), seed 11): every colour, the round count and the per-round log."""
    g = graphgen.rmat(24, 8, (0.55, 0.1, 0.1), 11)
    key = None if order == "natural" else graphgen.random_priority(g.n, 12)
    check(g, key, label="rmat24-" + order)
