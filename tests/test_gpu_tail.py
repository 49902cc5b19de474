"""The sequential finish (GCOLOR_SERIAL_TAIL) against its oracle: Algorithm
2's rounds while more than T vertices are uncoloured, then the rest one at
a time in (priority, id) order.  Colours, rounds and the size of the finish
equal the oracle's vertex for vertex, for several T, orders and graphs."""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run_tail(g, key, tail):
    import paper_1205_3809_amd as gc
    old = gc.get_serial_tail()
    try:
        gc.set_serial_tail(tail)
        pr = None if key is None else dev(np.ascontiguousarray(key, dtype=np.uint32).view(np.int32))
        col, st = gc.color_graph_ex(dev(g.row_ptr), dev(g.col_idx), pr, flags=gc.FLAG_SERIAL_TAIL, stats=True)
        torch.cuda.synchronize()
        return col.cpu().numpy(), st
    finally:
        gc.set_serial_tail(old)


def check(g, key, tail, label):
    print("case %s n=%d nnz=%d tail=%d key=%s" % (label, g.n, g.nnz, tail, key is not None), flush=True)
    ref = oracle.spec_tail(g.row_ptr, g.col_idx, key, tail)
    col, st = run_tail(g, key, tail)
    mism = np.flatnonzero(col != ref.colors)
    assert mism.size == 0, "%d mismatches, first at %s" % (mism.size, mism[:5])
    assert st.rounds == ref.rounds and st.serial_tail == ref.tail
    assert st.num_colors == (int(ref.colors.max()) if g.n else 0)


@pytest.mark.parametrize("tail", [1, 7, 100, 1024, 8192])
@pytest.mark.parametrize("order", ["natural", "perm", "ties"])
def test_rmat(tail, order):
    g = graphgen.rmat(16, 8, (0.55, 0.1, 0.1), 3)
    key = {"natural": None, "perm": graphgen.random_priority(g.n, 4),
           "ties": graphgen.random_keys(g.n, 5, bits=3)}[order]
    check(g, key, tail, "rmat16-" + order)


def test_whole_graph_in_the_finish_is_the_serial_greedy():
    """n <= T: no round, every vertex in the finish: the serial greedy."""
    for g in (graphgen.rmat(12, 8, (0.55, 0.1, 0.1), 2), graphgen.complete(60), graphgen.path(100),
              graphgen.empty(5)):
        key = graphgen.random_priority(g.n, 9)
        col, st = run_tail(g, key, 8192)
        assert np.array_equal(col, oracle.greedy(g.row_ptr, g.col_idx, key))
        assert st.rounds == 0 and st.serial_tail == g.n


def test_grids_and_long_rounds():
    """Meshes in natural order need many rounds; K_300 needs 300, so the
    finish also starts after the state words have widened."""
    check(graphgen.grid((120, 120), True), None, 50, "grid120-9pt")
    check(graphgen.complete(300), None, 20, "K300")


def test_rmat_scale24_natural():
    g = graphgen.rmat(24, 8, (0.55, 0.1, 0.1), 11)
    check(g, None, 1024, "rmat24-natural")


def test_flag_combinations_and_range():
    import paper_1205_3809_amd as gc
    g = graphgen.rmat(8, 8, (0.55, 0.1, 0.1), 1)
    for bad in (gc.FLAG_PLAIN, gc.FLAG_DATAFLOW):
        with pytest.raises(gc.GColorError) as e:
            gc.color_graph_ex(dev(g.row_ptr), dev(g.col_idx), None, flags=gc.FLAG_SERIAL_TAIL | bad)
        assert e.value.code == -1
