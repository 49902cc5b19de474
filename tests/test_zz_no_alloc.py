"""The allocation-free entry point color_graph_async_noalloc (its workspace is
a fixed device array of the library, for callers that cannot allocate)
against color_graph_async with a caller workspace: the same colours and
device statistics on two calls in a row, the second on a smaller graph (the
array keeps the first call's contents), and a clear error for a graph whose
workspace does not fit."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def lib():
    import paper_1205_3809_amd as gc
    L = gc.raw_library()
    L.color_graph_async_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                                            ctypes.c_void_p, ctypes.c_void_p]
    L.color_graph_async_noalloc.restype = ctypes.c_int
    L.gcolor_noalloc_max_bytes.argtypes = []
    L.gcolor_noalloc_max_bytes.restype = ctypes.c_size_t
    return L


def stream():
    return ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))


def both(g, key, budget):
    """(colours, stats words) from the allocation-free call and from
    color_graph_async with its own workspace, same inputs."""
    import paper_1205_3809_amd as gc
    L = lib()
    rp, ci = dev(g.row_ptr), dev(g.col_idx)
    pr = None if key is None else dev(np.ascontiguousarray(key, dtype=np.uint32).view(np.int32))
    out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    st = torch.full((6,), -7, dtype=torch.int32, device="cuda")
    rc = L.color_graph_async_noalloc(g.n, g.nnz, vp(rp), vp(ci), vp(pr), vp(out), budget, 0, vp(st), stream())
    assert rc == 0, rc
    ws = torch.empty(gc.workspace_bytes(g.n, g.nnz), dtype=torch.uint8, device="cuda")
    ref, rst = gc.color_graph_async(rp, ci, g.nnz, ws, budget, pr)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st.cpu().numpy(), ref.cpu().numpy(), rst.cpu().numpy()


def test_two_calls_second_smaller():
    big = graphgen.rmat(15, 8, (0.55, 0.1, 0.1), 21)
    small = graphgen.rmat(11, 8, (0.55, 0.1, 0.1), 22)
    for g, key in ((big, None), (small, graphgen.random_priority(small.n, 23))):
        print("no-alloc case n=%d nnz=%d key=%s" % (g.n, g.nnz, key is not None), flush=True)
        col, st, ref, rst = both(g, key, 300)
        assert np.array_equal(col, ref) and np.array_equal(st, rst)
        assert st[4] == 0  # status OK
        assert np.array_equal(col, oracle.spec_sim(g.row_ptr, g.col_idx, key).colors)


def test_too_large_is_refused_before_any_work():
    import paper_1205_3809_amd as gc
    L = lib()
    cap = int(L.gcolor_noalloc_max_bytes())
    assert cap == 64 << 20
    n, nnz = 1 << 22, 1 << 25
    assert gc.workspace_bytes(n, nnz) > cap
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the size check fails first
    assert L.color_graph_async_noalloc(n, nnz, fake, fake, None, fake, 10, 0, fake, stream()) == -6
