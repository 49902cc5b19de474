"""Exact smallest-last order on the GPU (gcolor_smallest_last) against the
oracle's peel, rank for rank: every graph of up to 5 vertices, random graphs
full of ties and self-loops, structured graphs whose steps stress the LDS
stage (a clique larger than the stage: one removal a step, streamed), and
R-MAT graphs at the training scale and at the evaluation scale of the
learned ordering."""
import itertools

import numpy as np
import pytest
import torch

import graphgen
import oracle
import paper_1205_3809_amd as gc

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def check(rp, ci, label):
    rank, d = gc.smallest_last(dev(rp), dev(ci))
    ro, do = oracle.smallest_last_rank(rp, ci)
    got = rank.cpu().numpy()
    assert np.array_equal(got, ro), (label, int((got != ro).sum()))
    assert d == do, (label, d, do)
    return got


def test_every_graph_up_to_five_vertices():
    for n in range(1, 6):
        pairs = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(pairs)):
            adj = oracle.edges_to_adj(n, [pairs[i] for i in range(len(pairs)) if mask >> i & 1])
            rp, ci = oracle.adj_to_csr(adj)
            check(rp, ci, (n, mask))


def test_random_graphs_with_ties_and_self_loops():
    rng = np.random.default_rng(11)
    for trial in range(300):
        n = int(rng.integers(2, 200))
        p = rng.uniform(0.01, 0.5)
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
        adj = oracle.edges_to_adj(n, edges)
        if trial % 3 == 0:
            for v in rng.choice(n, max(1, n // 5), replace=False):
                adj[v] = sorted(set(adj[v]) | {int(v)})
        rp, ci = oracle.adj_to_csr(adj)
        check(rp, ci, trial)


@pytest.mark.parametrize("name", ["empty", "path", "star", "complete300", "complete2100", "grid9", "grid3d27",
                                  "bipartite", "rgg"])
def test_structured(name):
    g = {"empty": lambda: graphgen.empty(7), "path": lambda: graphgen.path(5000),
         "star": lambda: graphgen.star(5000, 1234), "complete300": lambda: graphgen.complete(300),
         # 2099 remaining neighbours per vertex: more than the 2048 pairs the
         # stage holds, so every step removes one vertex from its streamed row
         "complete2100": lambda: graphgen.complete(2100),
         "grid9": lambda: graphgen.grid((60, 70), True), "grid3d27": lambda: graphgen.grid((12, 13, 14), True),
         "bipartite": lambda: graphgen.complete_bipartite(40, 700), "rgg": lambda: graphgen.rgg(20000, 12, 3)}[name]()
    print("smallest-last %s: n=%d nnz=%d" % (name, g.n, g.nnz), flush=True)
    check(g.row_ptr, g.col_idx, name)


def test_rmat_training_scale():
    for seed in (0, 1, 2):
        g = graphgen.rmat(16, 16, (0.57, 0.19, 0.19), seed)
        print("smallest-last rmat16 seed %d" % seed, flush=True)
        check(g.row_ptr, g.col_idx, seed)
    g = graphgen.uniform(1 << 16, 1 << 19, 4)
    check(g.row_ptr, g.col_idx, "uniform")


def test_rmat_evaluation_scale():
    """The learned ordering's evaluation graph (R-MAT scale 22, edge factor 16,
    seed 1000): every rank equals the oracle's, and colouring with the ranks as
    priorities equals the oracle's colouring with them."""
    g = graphgen.rmat(22, 16, (0.57, 0.19, 0.19), 1000)
    print("smallest-last rmat22: n=%d nnz=%d" % (g.n, g.nnz), flush=True)
    rank = check(g.row_ptr, g.col_idx, "rmat22")
    assert sorted(rank.tolist()) == list(range(g.n))


def test_malformed_csr_is_refused():
    rp = np.array([0, 2, 3, 4], np.int32)
    ci = np.array([1, 7, 0, 0], np.int32)  # 7 is outside [0, 3)
    with pytest.raises(gc.GColorError) as e:
        gc.smallest_last(dev(rp), dev(ci))
    assert e.value.code == -2
    # entries but no col_idx (an empty tensor passes a NULL pointer)
    none = torch.empty(0, dtype=torch.int32, device="cuda")
    assert none.data_ptr() == 0
    with pytest.raises(gc.GColorError) as e:
        gc.smallest_last(dev(rp), none)
    assert e.value.code == -2
    # no entries at all: col_idx may be NULL
    rank, d = gc.smallest_last(dev(np.zeros(4, np.int32)), none)
    assert rank.cpu().tolist() == [2, 1, 0] and d == 0
