"""Batched colouring on the GPU vs the CPU oracle, graph by graph.

A batch must colour every graph exactly as the oracle's round-synchronous
simulation colours it alone (bit-exact colours and round counts); the call is
asynchronous and is also checked under HIP-graph capture with replays.
"""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run_batch(graphs, keys=None, capture=False):
    import paper_1205_3809_amd as gc
    b = graphgen.concat(graphs)
    V, nnz, G = int(b.vtx_off[-1]), int(b.edge_off[-1]), len(graphs)
    vo, eo, rp, ci = dev(b.vtx_off), dev(b.edge_off), dev(b.row_ptr), dev(b.col_idx)
    pr = None
    if keys is not None:
        pr = dev(np.concatenate(keys).astype(np.uint32).view(np.int32))
    out = torch.full((V,), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(gc.batch_workspace_bytes(G, V, nnz), dtype=torch.uint8, device="cuda")
    ticks = torch.zeros(2 * G, dtype=torch.int64, device="cuda")
    rounds = torch.zeros(G, dtype=torch.int32, device="cuda")
    if not capture:
        gc.color_graph_batch(vo, eo, rp, ci, V, nnz, pr, out, ws, ticks, rounds)
        torch.cuda.synchronize()
        return b, [out.cpu().numpy()], rounds.cpu().numpy(), ticks.cpu().numpy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside the capture
        gc.color_graph_batch(vo, eo, rp, ci, V, nnz, pr, out, ws, ticks, rounds)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gc.color_graph_batch(vo, eo, rp, ci, V, nnz, pr, out, ws, ticks, rounds)
    outs = []
    for rep in range(3):
        out.fill_(-7)            # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy().copy())
    return b, outs, rounds.cpu().numpy(), ticks.cpu().numpy()


def check_batch(graphs, keys=None, capture=False):
    b, outs, rounds, ticks = run_batch(graphs, keys, capture)
    for out in outs:
        for i, g in enumerate(graphs):
            lo, hi = b.vtx_off[i], b.vtx_off[i + 1]
            ref = oracle.spec_sim(g.row_ptr, g.col_idx, None if keys is None else keys[i])
            got = out[lo:hi]
            assert np.array_equal(got, ref.colors), "graph %d (n=%d): %d mismatches" % (
                i, g.n, int((got != ref.colors).sum()))
            assert rounds[i] == ref.rounds, (i, rounds[i], ref.rounds)
    # start <= end for every graph
    t = ticks.reshape(-1, 2)
    assert np.all(t[:, 1] >= t[:, 0])


def mixed_graphs(seed, count=40, lo=4.0, hi=10.0):
    specs = graphgen.batch_specs(count, seed, lo, hi)
    gs = [graphgen.batch_graph(s) for s in specs]
    # structural edge cases in the same batch
    # (K_127: degree 126 and colour 127, the largest that keeps its state in
    # LDS; K_128 and the star take the global-memory path)
    gs += [graphgen.empty(1), graphgen.empty(0), graphgen.empty(5), graphgen.complete(70),
           graphgen.complete(127), graphgen.complete(128),
           graphgen.star(3000, 0), graphgen.path(130), graphgen.cycle(64),
           graphgen.rmat(10, 8, (0.55, 0.1, 0.1), 4), graphgen.uniform(700, 3000, 2)]
    return gs


def test_batch_matches_oracle():
    check_batch(mixed_graphs(5))


def test_batch_with_priorities():
    gs = mixed_graphs(6, count=20)
    keys = [graphgen.random_keys(g.n, 100 + i, bits=(32 if i % 2 else 4)) for i, g in enumerate(gs)]
    check_batch(gs, keys)


def test_batch_single_and_large_graph():
    check_batch([graphgen.grid((200, 200), True)])
    check_batch([graphgen.rmat(15, 8, (0.55, 0.1, 0.1), 3), graphgen.empty(3)])


@pytest.mark.parametrize("count", [8192, 8193])
def test_batch_at_and_past_the_sort_limit(count):
    """Up to 8192 graphs are processed largest first (sorted in LDS), more
    in index order; either way every graph is coloured as alone."""
    specs = graphgen.batch_specs(count, 40 + count, 3.0, 7.0)
    graphs = [graphgen.batch_graph(s) for s in specs]
    graphs[count // 2] = graphgen.grid((40, 40), True)  # one large graph in the middle
    graphs[-1] = graphgen.empty(0)
    print("batch of %d graphs" % count, flush=True)
    check_batch(graphs)


def test_batch_graph_capture_replays():
    check_batch(mixed_graphs(7, count=24), capture=True)


def test_batch_full_size_every_graph():
    """The full batched workload: 4096 graphs, n log-uniform in [2^8, 2^16],
    stencil grids with 5% extra edges and random geometric graphs, in one
    launch.  Every graph's colours and round count equal the oracle's run on
    that graph alone (the oracle runs graph by graph on the host threads);
    every colouring is also proper and within degree + 1."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1))
    specs = graphgen.batch_specs(4096, 2026)
    with ThreadPoolExecutor(workers) as ex:
        graphs = list(ex.map(graphgen.batch_graph, specs))
    print("batch generated: %d graphs" % len(graphs), flush=True)
    b, outs, rounds, _ = run_batch(graphs)
    out = outs[0]
    print("batch coloured", flush=True)

    def compare(i):
        g = graphs[i]
        c = out[b.vtx_off[i]:b.vtx_off[i + 1]]
        ref = oracle.spec_sim(g.row_ptr, g.col_idx)
        src = np.repeat(np.arange(g.n), g.degrees())
        ok = (np.array_equal(c, ref.colors) and int(rounds[i]) == ref.rounds and c.min(initial=1) >= 1
              and not np.any(c[src] == c[g.col_idx]) and bool(np.all(c <= g.degrees() + 1)))
        return i, ok

    order = np.argsort([-g.nnz for g in graphs], kind="stable")  # largest first: even finish
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(compare, order))
    bad = [i for i, ok in results if not ok]
    print("compared %d graphs with the oracle, %d differ" % (len(results), len(bad)), flush=True)
    assert len(results) == 4096 and not bad, bad[:10]


def test_batch_tuning_does_not_change_colours():
    """Every batch launch setting (256 or 1024 threads, LDS capacity, LDS path
    off) gives the oracle's colours."""
    import paper_1205_3809_amd as gc
    gs = mixed_graphs(9, count=24) + [graphgen.grid((90, 90), True)]
    old = gc.get_batch_tuning()
    try:
        for t in [(256, 8, 65536), (1024, 8, 65536), (256, 1, 1024), (1024, 64, 65536), (256, 8, 0),
                  (1024, 8, 0), (0, 2, 16384)]:
            print("batch tuning", t, flush=True)
            gc.set_batch_tuning(*t)
            check_batch(gs)
    finally:
        gc.set_batch_tuning(*old)


def test_autotuner_searches_keep_colours():
    """The autotuner's searches run, return their best setting, and check on
    every trial that the colours do not change (they raise otherwise)."""
    import torch
    import paper_1205_3809_amd as gc
    from paper_1205_3809_amd import autotune
    s_old, b_old = gc.get_tuning(), gc.get_batch_tuning()
    try:
        g = graphgen.rmat(14, 8, (0.55, 0.1, 0.1), 3)
        rp, ci = dev(g.row_ptr), dev(g.col_idx)
        e = autotune.tune_single(rp, ci, reps=1, passes=1)
        assert e["kind"] == "single" and len(e["trials"]) > 5 and e["ms"] <= e["start_ms"]
        b = graphgen.concat(mixed_graphs(11, count=16))
        V, E = int(b.vtx_off[-1]), int(b.edge_off[-1])
        e = autotune.tune_batch(dev(b.vtx_off), dev(b.edge_off), dev(b.row_ptr), dev(b.col_idx), V, E, reps=1)
        assert e["kind"] == "batch" and e["ms"] <= e["start_ms"]
    finally:
        gc.set_tuning(*s_old)
        gc.set_batch_tuning(*b_old)
