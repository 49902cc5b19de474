"""GPU colouring vs the CPU oracle, bit for bit, through the C ABI.

Every case compares colors_out element by element with the oracle's
round-synchronous simulation on the same seeded input, checks the round count,
the colour count and the per-round worklist/edge-work log, and validates the
colouring independently (adjacent vertices differ, colour <= degree + 1).
"""
import functools

import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gpu_color(g, key=None, workspace=None, **kw):
    import paper_1205_3809_amd as gc
    rp, ci = dev(g.row_ptr), dev(g.col_idx)
    pr = None if key is None else dev(np.ascontiguousarray(key, dtype=np.uint32).view(np.int32))
    col, st = gc.color_graph_ex(rp, ci, pr, workspace=workspace, stats=True, max_log=1 << 16, **kw)
    torch.cuda.synchronize()
    return col.cpu().numpy(), st


def valid(g, col):
    src = np.repeat(np.arange(g.n), g.degrees())
    return col.min(initial=1) >= 1 and not np.any(col[src] == col[g.col_idx]) and np.all(col <= g.degrees() + 1)


# both engines compute the same function: the default incremental one and
# the plain one that rescans every worklist row each round
ENGINES = (("incremental", 0), ("plain", 4))


def check(g, key=None, label="", engines=ENGINES):
    ref = oracle.spec_sim(g.row_ptr, g.col_idx, key, threads=0)
    out = None
    for name, flags in engines:
        print("case %s engine=%s n=%d nnz=%d key=%s" % (label, name, g.n, g.nnz,
                                                         None if key is None else key.dtype), flush=True)
        col, st = gpu_color(g, key, flags=flags)
        assert col.shape == ref.colors.shape
        mism = np.flatnonzero(col != ref.colors)
        assert mism.size == 0, "%s: %d mismatches, first at %s" % (name, mism.size, mism[:5])
        assert valid(g, col)
        assert st.rounds == ref.rounds, name
        assert st.num_colors == (int(ref.colors.max()) if g.n else 0)
        assert st.edge_work == int(ref.log[:, 2].sum()), name
        got = np.array([[k, u, e] for k, u, e in st.round_log], dtype=np.int64).reshape(-1, 3)
        assert np.array_equal(got, ref.log[:, :3]), name
        committed = np.array([d[0] for d in st.detail], dtype=np.int64)
        assert np.array_equal(committed, ref.log[:, 1] - ref.log[:, 3]), name
        out = (col, st) if out is None else out
    return out


# ---------------------------------------------------------------------------
# structured graphs and closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 300, 1001])
def test_empty_graph(n):
    col, st = check(graphgen.empty(n), label="empty")
    assert st.rounds == 1 and np.all(col == 1)


@pytest.mark.parametrize("n", [2, 3, 4, 63, 64, 65, 257, 1000])
def test_paths_and_cycles(n):
    check(graphgen.path(n), label="path")
    if n >= 3:
        check(graphgen.cycle(n), label="cycle")


@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65, 66, 129, 130, 200, 300])
def test_complete_graphs_many_windows(n):
    """K_n needs n colours: more than one 64-colour window from n = 64 on."""
    col, st = check(graphgen.complete(n), label="complete")
    assert st.num_colors == n and st.rounds == n


@pytest.mark.parametrize("n,order", [(600, "natural"), (600, "perm"), (2100, "natural"), (2100, "perm"),
                                     (4300, "natural"), (4300, "perm")])
def test_complete_long_rows(n, order):
    """K_n with rows beyond the register cache of the wave tier (600) and the
    workgroup tier (2100), and with more than 64 + 4096 colours (4300).
    Closed form: the vertex of rank r in (key, id) order gets colour r + 1, in
    n rounds; the oracle is not needed."""
    import paper_1205_3809_amd as gc
    g = graphgen.complete(n)
    key = None if order == "natural" else graphgen.random_priority(n, 17)
    engines = ENGINES if n <= 2100 else ENGINES[:1]
    for name, flags in engines:
        print("case complete-long n=%d order=%s engine=%s" % (n, order, name), flush=True)
        col, st = gpu_color(g, key, flags=flags)
        rank = np.arange(n) if key is None else np.argsort(np.argsort(key.astype(np.int64), kind="stable"))
        assert np.array_equal(col, rank + 1), name
        assert st.rounds == n and st.num_colors == n, name


def clique_plus_hub(m, leaves):
    """Clique on 0..m-1, leaves m..m+leaves-1, and a hub (the last id) joined
    to every clique vertex and every leaf: the hub's long row stays dirty
    while the clique commits one colour per round."""
    hub = m + leaves
    iu, ju = np.triu_indices(m, 1)
    src = np.concatenate([iu, np.full(m + leaves, hub)])
    dst = np.concatenate([ju, np.arange(m + leaves)])
    return graphgen.from_pairs(hub + 1, src, dst)


@pytest.mark.parametrize("m,leaves", [(70, 600), (300, 600), (300, 3000), (130, 9000), (200, 40000)])
def test_long_dirty_rows(m, leaves):
    """Long rows that stay dirty for many rounds (wave and workgroup tiers,
    colours past the first 64-colour window), against the oracle.  Past
    round 127 the state words widen: to 16 bits, and to 32 bits for the hub
    of degree 40200."""
    col, st = check(clique_plus_hub(m, leaves), label="clique+hub")
    assert col[-1] == m + 1


def clique_in_sparse(m, n, pairs, seed):
    """A clique on 0..m-1 beside a sparse uniform graph on m..n-1: the
    clique commits one vertex a round, so every round its remaining
    vertices are dirty with up to m-2 dirty preceding neighbours."""
    iu, ju = np.triu_indices(m, 1)
    rng = np.random.default_rng(seed)
    a = rng.integers(m, n, pairs)
    b = rng.integers(m, n, pairs)
    return graphgen.from_pairs(n, np.concatenate([iu, a]), np.concatenate([ju, b]))


@pytest.mark.parametrize("blocks_a", [0, 16])
def test_pair_lists_long_and_overflowing(blocks_a):
    """The dirty-vertex kernel's pair lists (each dirty vertex's dirty
    preceding neighbours, written per wavefront region) and both fallbacks to
    the commit kernel's row rescan: lists longer than 127 (the clique's later
    vertices, rows of 299 entries held in registers) and regions that fill up
    (16 workgroups per CU give 16,384 wavefronts, regions of 36 entries for
    600,000 vertices).  Colours, rounds and log equal the oracle's."""
    import paper_1205_3809_amd as gc
    g = clique_in_sparse(300, 600_000, 2_400_000, 5)
    old = gc.get_kernel_blocks()
    try:
        gc.set_kernel_blocks(blocks_a, old[1])
        col, st = check(g, label="clique+sparse blocks_a=%d" % blocks_a, engines=ENGINES[:1])
    finally:
        gc.set_kernel_blocks(*old)
    assert st.rounds >= 300 and col[:300].max() == 300


def dirty_model(g, key=None):
    """Per round: number and degree sum of the worklist vertices whose
    tentative colour differs from the previous round's (the vertices the
    incremental engine must revisit), from the set-notation simulation."""
    adj = oracle.adjacency(g.row_ptr, g.col_idx)
    deg = g.degrees()
    prev, out = {}, []

    def trace(k, U, tent, R, color):
        moved = [v for v in U if k > 1 and tent[v] != prev[v]]
        out.append((len(moved), int(sum(deg[v] for v in moved))))
        prev.update(tent)

    oracle.spec_sim_py(adj, None if key is None else [int(x) for x in key], trace=trace)
    return out


@pytest.mark.parametrize("case", ["rmat12", "rmat12-perm", "clique+hub"])
def test_dirty_statistics(case):
    """The incremental engine's per-round dirty count and dirty degree sum
    (heavy rows included: R-MAT scale 12 with the training skew has rows above
    512, the hub row has 670) equal the model's."""
    g = clique_plus_hub(70, 600) if case == "clique+hub" else rmat(12, 16, (0.57, 0.19, 0.19), 4)
    key = graphgen.random_priority(g.n, 3) if case.endswith("perm") else None
    col, st = gpu_color(g, key)
    want = dirty_model(g, key)
    got = [(int(d[1]), int(d[2])) for d in st.detail]
    assert got == want
    # entries read: the whole row, except rows above 512 entries once part of
    # them has committed
    assert all(d[3] <= d[2] for d in st.detail)
    if g.degrees().max() <= 512:
        assert all(d[3] == d[2] for d in st.detail)
    else:
        assert sum(d[3] for d in st.detail) < sum(d[2] for d in st.detail)


@pytest.mark.parametrize("n,center", [(3000, 0), (3000, 2999), (20000, 0), (20000, 19999), (32767, 5), (32768, 5), (70000, 123)])
def test_star_hubs(n, center):
    """A centre of degree up to 70k runs on the workgroup-per-vertex bin."""
    check(graphgen.star(n, center), label="star")


@pytest.mark.parametrize("shape,full", [((64, 64), False), ((37, 41), True), ((16, 16, 16), False),
                                        ((9, 10, 11), True)])
def test_grids(shape, full):
    col, st = check(graphgen.grid(shape, full), label="grid")
    if not full:
        assert st.num_colors == 2


def test_grid_with_extra_edges_and_rgg():
    check(graphgen.grid_with_extra((90, 90), False, 0.05, 1), label="grid+extra")
    check(graphgen.rgg(20000, 15.0, 2), label="rgg")


# ---------------------------------------------------------------------------
# random graphs, several orders
# ---------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def rmat(scale, ef, abc, seed):
    return graphgen.rmat(scale, ef, abc, seed)


def test_uniform_config():
    """2^14 vertices, 2^17 uniform pairs, natural order."""
    check(graphgen.uniform(1 << 14, 1 << 17, 1), label="uniform")


@pytest.mark.parametrize("abc", [(0.25, 0.25, 0.25), (0.45, 0.15, 0.15), (0.55, 0.1, 0.1), (0.55, 0.15, 0.15)])
def test_rmat_small_natural(abc):
    check(rmat(14, 8, abc, 3), label="rmat14")


@pytest.mark.parametrize("order", ["perm", "ties3", "ties12", "allsame"])
def test_rmat_small_priorities(order):
    g = rmat(14, 8, (0.55, 0.1, 0.1), 3)
    if order == "perm":
        key = graphgen.random_priority(g.n, 8)
    elif order == "allsame":
        key = np.full(g.n, 7, dtype=np.uint32)
    else:
        key = graphgen.random_keys(g.n, 9, bits=int(order[4:]))
    check(g, key, label="rmat14-" + order)


def test_priority_identity_equals_natural():
    g = rmat(14, 8, (0.45, 0.15, 0.15), 4)
    a, _ = gpu_color(g)
    b, _ = gpu_color(g, np.arange(g.n, dtype=np.uint32))
    assert np.array_equal(a, b)


def test_unsorted_rows_with_priority():
    """With a priority array the rows may come in any order."""
    g = rmat(12, 8, (0.55, 0.1, 0.1), 5)
    rng = np.random.default_rng(0)
    col = g.col_idx.copy()
    for v in range(g.n):
        s, e = g.row_ptr[v], g.row_ptr[v + 1]
        col[s:e] = rng.permutation(col[s:e])
    h = graphgen.CSR(g.n, g.row_ptr, col)
    key = graphgen.random_priority(g.n, 1)
    ref = oracle.spec_sim(g.row_ptr, g.col_idx, key)
    got, _ = gpu_color(h, key)
    assert np.array_equal(got, ref.colors)


# ---------------------------------------------------------------------------
# launch-shape independence, determinism, workspace handling, streams
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("engine", [0, 4], ids=["incremental", "plain"])
def test_result_independent_of_tuning(engine):
    import paper_1205_3809_amd as gc
    g = rmat(15, 8, (0.55, 0.1, 0.1), 6)
    key = graphgen.random_priority(g.n, 2)
    ref = oracle.spec_sim(g.row_ptr, g.col_idx, key, threads=0).colors
    refn = oracle.spec_sim(g.row_ptr, g.col_idx, None, threads=0).colors
    old, bpc = gc.get_tuning()
    kold = gc.get_kernel_blocks()
    try:
        for bins, b, kb in [([0, 0, 0, 0], 2, (0, 0)), ([1, 2, 3, 4], 1, (1, 3)),
                            ([64, 64, 64, 64], 16, (0, 0)), ([2, 8, 64, 256], 8, (12, 0)),
                            ([1000000] * 4, 3, (0, 16))]:
            gc.set_tuning(bins, b)
            gc.set_kernel_blocks(*kb)
            got, _ = gpu_color(g, key, flags=engine)
            assert np.array_equal(got, ref), (bins, b, kb)
            got, _ = gpu_color(g, None, flags=engine)
            assert np.array_equal(got, refn), (bins, b, kb)
    finally:
        gc.set_tuning(old, bpc)
        gc.set_kernel_blocks(*kold)


def test_repeatable():
    g = rmat(16, 8, (0.55, 0.1, 0.1), 7)
    runs = [gpu_color(g)[0] for _ in range(3)] + [gpu_color(g, flags=4)[0] for _ in range(2)]
    assert all(np.array_equal(runs[0], r) for r in runs[1:])


def test_caller_workspace_and_shrinking_inputs():
    import paper_1205_3809_amd as gc
    big = rmat(14, 8, (0.45, 0.15, 0.15), 1)
    small = graphgen.uniform(5000, 20000, 3)
    ws = torch.empty(gc.workspace_bytes(big.n, big.nnz), dtype=torch.uint8, device="cuda")
    for g in (big, small, big):
        got, _ = gpu_color(g, workspace=ws)
        assert np.array_equal(got, oracle.spec_sim(g.row_ptr, g.col_idx).colors)
    with pytest.raises(gc.GColorError) as e:
        gpu_color(big, workspace=ws[:1000])
    assert e.value.code == -3


def test_plain_entry_point_on_side_stream():
    import paper_1205_3809_amd as gc
    g = graphgen.uniform(1 << 14, 1 << 17, 5)
    s = torch.cuda.Stream()
    rp, ci = dev(g.row_ptr), dev(g.col_idx)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        out = gc.color_graph(rp, ci)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.spec_sim(g.row_ptr, g.col_idx).colors)


# ---------------------------------------------------------------------------
# validation of malformed input (host-forced error paths)
# ---------------------------------------------------------------------------

def _validate(rp, ci, key=None):
    import paper_1205_3809_amd as gc
    with pytest.raises(gc.GColorError) as e:
        gc.color_graph_ex(dev(rp), dev(ci), None if key is None else dev(key), flags=gc.FLAG_VALIDATE)
    return e.value.code


def test_validate_rejects_malformed_csr():
    g = graphgen.cycle(10)
    rp, ci = g.row_ptr.copy(), g.col_idx.copy()
    bad = ci.copy(); bad[3] = 10
    assert _validate(rp, bad) == -2           # neighbour id out of range
    bad = ci.copy(); bad[0], bad[1] = bad[1], bad[0]
    assert _validate(rp, bad) == -2           # unsorted row
    bad = ci.copy(); bad[2] = 5
    assert _validate(rp, bad) == -2           # asymmetric
    badr = rp.copy(); badr[4] = badr[6]
    assert _validate(badr, ci) == -2          # row_ptr not monotone
    import paper_1205_3809_amd as gc
    out, _ = gc.color_graph_ex(dev(rp), dev(ci), flags=gc.FLAG_VALIDATE)
    assert np.array_equal(out.cpu().numpy(), oracle.spec_sim(rp, ci).colors)


@pytest.mark.parametrize("flags,name", [(0, "incremental"), (4, "plain"), (8, "dataflow")])
def test_round_cap_forced_from_the_host(flags, name):
    """A cap below the rounds a colouring needs returns GCOLOR_EROUNDS (-5)
    for every engine; a cap equal to them, or above, colours as without a
    cap.  The graphs need 1, a few tens and 151 to 300 rounds (the
    incremental engine widens its state words after round 127; caps of 127
    and 128 stop it on either side of that step)."""
    import paper_1205_3809_amd as gc
    cases = [graphgen.empty(50), rmat(12, 8, (0.55, 0.1, 0.1), 3), graphgen.path(300)]
    assert gc.get_round_cap() == 0
    try:
        for g in cases:
            print("case round-cap engine=%s n=%d" % (name, g.n), flush=True)
            ref, st = gpu_color(g, flags=flags)
            need = st.rounds
            assert need >= 1
            for cap in sorted(c for c in {1, 127, 128, need - 1, need, need + 1} if 1 <= c <= need + 1):
                gc.set_round_cap(cap)
                if cap < need:
                    with pytest.raises(gc.GColorError) as e:
                        gpu_color(g, flags=flags)
                    assert e.value.code == -5, (name, g.n, cap, need)
                else:
                    got, st2 = gpu_color(g, flags=flags)
                    assert np.array_equal(got, ref) and st2.rounds == need, (name, g.n, cap)
                gc.set_round_cap(0)
    finally:
        gc.set_round_cap(0)
    # the library works as before after an aborted call
    g = cases[1]
    got, _ = gpu_color(g, flags=flags)
    if flags == 8:
        ref = oracle.dataflow(g.row_ptr, g.col_idx).colors
    else:
        ref = oracle.spec_sim(g.row_ptr, g.col_idx, None, threads=0).colors
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------------------
# full-size workloads
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("abc", [(0.25, 0.25, 0.25), (0.45, 0.15, 0.15)])
def test_rmat_scale20_natural(abc):
    """R-MAT scale 20, edge factor 8, ER-like and skewed parameters."""
    check(rmat(20, 8, abc, 11), label="rmat20")


@pytest.mark.parametrize("order", ["natural", "ties8"])
def test_skewed_scale22_in_its_bench_configuration(order):
    """The learned-ordering evaluation graph (R-MAT scale 22, edge factor 16,
    (0.57, 0.19, 0.19, 0.05), seed 1000) coloured with the launch parameters
    the bench applies to it (tuning table entry learned22-eval), in natural
    order and with 8-bit keys (many ties, like quantised learned scores)."""
    import paper_1205_3809_amd as gc
    from paper_1205_3809_amd import autotune
    g = rmat(22, 16, (0.57, 0.19, 0.19), 1000)
    key = None if order == "natural" else graphgen.random_keys(g.n, 77, bits=8)
    old, bpc = gc.get_tuning()
    kold = gc.get_kernel_blocks()
    try:
        entry = autotune.apply(autotune.TABLE, "learned22-eval", "gfx950")
        assert entry is not None
        check(g, key, label="rmat22-skewed-" + order, engines=(("incremental", 0),))
    finally:
        gc.set_tuning(old, bpc)
        gc.set_kernel_blocks(*kold)


@pytest.mark.parametrize("order", ["natural", "perm"])
def test_rmat_scale24(order):
    """R-MAT scale 24, edge factor 8, (0.55, 0.1, 0.1, 0.25): the full
    benchmark workload, compared on every vertex."""
    g = rmat(24, 8, (0.55, 0.1, 0.1), 11)
    key = None if order == "natural" else graphgen.random_priority(g.n, 12)
    check(g, key, label="rmat24-" + order)
