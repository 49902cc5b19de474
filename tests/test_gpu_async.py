"""The stream-ordered entry point color_graph_async (a round budget, no host
synchronisation, no allocation) against the oracle: same colours, rounds,
colour count and edge work as the round-synchronous simulation; statuses for
a short budget and a malformed CSR written on the device; and the call
captured in a HIP graph and replayed, each replay checked."""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu

OK, ECSR, EROUNDS = 0, -2, -5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def keyt(key):
    return None if key is None else dev(np.ascontiguousarray(key, dtype=np.uint32).view(np.int32))


def run_async(g, key=None, budget=None, validate=False, ws=None, stream=None):
    import paper_1205_3809_amd as gc
    if ws is None:
        ws = torch.empty(max(gc.workspace_bytes(g.n, g.nnz), 1), dtype=torch.uint8, device="cuda")
    if budget is None:
        budget = g.n + 1
    col, st = gc.color_graph_async(dev(g.row_ptr), dev(g.col_idx), g.nnz, ws, budget, keyt(key),
                                   validate=validate, stream=stream)
    torch.cuda.synchronize()
    return col.cpu().numpy(), gc.stats_from_device(st)


def check(g, key=None, budget=None, label=""):
    print("case %s n=%d nnz=%d key=%s" % (label, g.n, g.nnz, key is not None), flush=True)
    ref = oracle.spec_sim(g.row_ptr, g.col_idx, key, threads=0)
    col, (rounds, colours, ework, status) = run_async(g, key, budget)
    assert status == OK
    assert np.array_equal(col, ref.colors), int((col != ref.colors).sum())
    assert rounds == ref.rounds
    assert colours == (int(ref.colors.max()) if g.n else 0)
    assert ework == int(ref.log[:, 2].sum())
    return ref


@pytest.mark.parametrize("order", ["natural", "perm", "ties"])
def test_matches_oracle(order):
    g = graphgen.rmat(16, 8, (0.55, 0.1, 0.1), 4)
    key = {"natural": None, "perm": graphgen.random_priority(g.n, 5),
           "ties": graphgen.random_keys(g.n, 6, bits=3)}[order]
    check(g, key, budget=400, label="rmat16-" + order)


def test_more_than_127_rounds():
    """K_200 needs exactly 200 rounds (one vertex kept per round), so the
    state widens before round 128; a 300-vertex path needs 151."""
    check(graphgen.complete(200), None, budget=260, label="K200")
    check(graphgen.path(300), None, budget=300, label="P300")
    g = graphgen.grid((40, 40), True)
    check(g, None, budget=200, label="grid40-9pt")


def test_round_budget():
    """A budget one short of the rounds needed reports GCOLOR_EROUNDS on the
    device; the exact budget succeeds."""
    g = graphgen.complete(150)
    ref = oracle.spec_sim(g.row_ptr, g.col_idx)
    assert ref.rounds == 150
    _, st = run_async(g, None, budget=149)
    assert st[3] == EROUNDS and st[0] == 0
    col, st = run_async(g, None, budget=150)
    assert st[3] == OK and st[0] == 150 and np.array_equal(col, ref.colors)
    g = graphgen.rmat(12, 8, (0.55, 0.1, 0.1), 2)
    ref = oracle.spec_sim(g.row_ptr, g.col_idx)
    _, st = run_async(g, None, budget=ref.rounds - 1)
    assert st[3] == EROUNDS
    col, st = run_async(g, None, budget=ref.rounds)
    assert st[3] == OK and np.array_equal(col, ref.colors)


def test_validation_on_the_device():
    """With validation, a malformed CSR (an asymmetric pair, an id out of
    range, decreasing row offsets) is reported as GCOLOR_ECSR in the device
    stats, and a well-formed one colours normally."""
    g = graphgen.rmat(10, 8, (0.55, 0.1, 0.1), 1)
    col, st = run_async(g, None, budget=200, validate=True)
    assert st[3] == OK and np.array_equal(col, oracle.spec_sim(g.row_ptr, g.col_idx).colors)
    rp = g.row_ptr.copy()
    ci = g.col_idx.copy()
    # asymmetric: the reverse entry of (v, w) redirected to another vertex
    v = int(np.argmax(np.diff(rp)))
    w = int(ci[rp[v]])
    ci_asym = ci.copy()
    pos = rp[w] + int(np.searchsorted(ci[rp[w]:rp[w + 1]], v))
    ci_asym[pos] = (v + 1) % g.n if (v + 1) % g.n != w else (v + 2) % g.n
    ci_range = ci.copy()
    ci_range[3] = g.n + 5  # an id out of range
    rp_dec = rp.copy()
    rp_dec[5] = rp_dec[7] + 1  # decreasing offsets
    for label, r, c in (("asymmetric", rp, ci_asym), ("id out of range", rp, ci_range),
                        ("decreasing offsets", rp_dec, ci)):
        print("malformed CSR: %s" % label, flush=True)
        _, st = run_async(graphgen.CSR(g.n, r, c), None, budget=50, validate=True)
        assert st[3] == ECSR, label


def test_empty_graph():
    col, st = run_async(graphgen.empty(0), None, budget=1)
    assert col.size == 0 and st == (0, 0, 0, OK)


def test_host_argument_errors():
    import paper_1205_3809_amd as gc
    g = graphgen.rmat(8, 8, (0.55, 0.1, 0.1), 1)
    ws = torch.empty(gc.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    with pytest.raises(gc.GColorError) as e:
        gc.color_graph_async(dev(g.row_ptr), dev(g.col_idx), g.nnz, ws, 0)
    assert e.value.code == -1
    with pytest.raises(gc.GColorError) as e:
        gc.color_graph_async(dev(g.row_ptr), dev(g.col_idx), g.nnz, ws[:100], 10)
    assert e.value.code == -3


def test_on_a_side_stream():
    """Enqueued on a non-default stream, the call waits for nothing on the
    host; the colours are ready once that stream is synchronised."""
    g = graphgen.rmat(15, 8, (0.55, 0.1, 0.1), 9)
    ref = oracle.spec_sim(g.row_ptr, g.col_idx)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    col, st = run_async(g, None, budget=300, stream=s)
    assert st[3] == OK and np.array_equal(col, ref.colors)


@pytest.mark.parametrize("order", ["natural", "perm"])
def test_hip_graph_capture_and_replays(order):
    """The whole colouring captured once into a HIP graph and replayed three
    times, with eager work and synchronisations between the replays (the
    outputs are overwritten with -1 first): every replay gives the oracle's
    colours and statistics."""
    import paper_1205_3809_amd as gc
    g = graphgen.rmat(17, 8, (0.55, 0.1, 0.1), 13)
    key = None if order == "natural" else graphgen.random_priority(g.n, 14)
    ref = oracle.spec_sim(g.row_ptr, g.col_idx, key, threads=0)
    rp, ci, pr = dev(g.row_ptr), dev(g.col_idx), keyt(key)
    ws = torch.empty(gc.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    stats = torch.zeros(6, dtype=torch.int32, device="cuda")
    budget = ref.rounds + 40
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside the capture
        gc.color_graph_async(rp, ci, g.nnz, ws, budget, pr, out, stats)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gc.color_graph_async(rp, ci, g.nnz, ws, budget, pr, out, stats)
    for rep in range(3):
        out.fill_(-1)
        stats.fill_(-1)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        col = out.cpu().numpy()
        rounds, colours, ework, status = gc.stats_from_device(stats)
        print("replay %d: status %d rounds %d" % (rep, status, rounds), flush=True)
        assert status == OK and rounds == ref.rounds and colours == int(ref.colors.max())
        assert ework == int(ref.log[:, 2].sum())
        assert np.array_equal(col, ref.colors), int((col != ref.colors).sum())
        del junk
