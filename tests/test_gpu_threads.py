"""Calls that use the library's cached per-device workspace from several host
threads at once, each on its own stream: every colouring equals the oracle's
(the library serialises such calls on their device instead of sharing the
buffer)."""
import threading

import numpy as np
import pytest
import torch

import graphgen
import oracle
import paper_1205_3809_amd as gc

pytestmark = pytest.mark.gpu


def test_concurrent_calls_on_the_library_workspace():
    graphs = [graphgen.rmat(14, 8, (0.55, 0.1, 0.1), s) for s in range(4)] + \
             [graphgen.uniform(20000, 90000, 7), graphgen.grid((90, 110), True)]
    want = [oracle.spec_sim(g.row_ptr, g.col_idx, threads=0).colors for g in graphs]
    want_blk = [oracle.block_gs(g.row_ptr, g.col_idx, None, 16, threads=0).colors for g in graphs]
    dev = [(torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col_idx).cuda()) for g in graphs]
    errors = []

    def work(t):
        s = torch.cuda.Stream()
        try:
            with torch.cuda.stream(s):
                for rep in range(6):
                    i = (t + rep) % len(graphs)
                    rp, ci = dev[i]
                    col = gc.color_graph(rp, ci, stream=s)
                    blk, _ = gc.color_graph_blocks(rp, ci, None, 16, stream=s)
                    s.synchronize()
                    if not np.array_equal(col.cpu().numpy(), want[i]):
                        errors.append(("color_graph", t, i))
                    if not np.array_equal(blk.cpu().numpy(), want_blk[i]):
                        errors.append(("color_graph_blocks", t, i))
        except Exception as e:  # reported below
            errors.append(("raised", t, repr(e)))

    ts = [threading.Thread(target=work, args=(t,)) for t in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
