"""ctypes binding of libgcolor.so (argument marshalling only).

Every function here takes torch tensors that live on a HIP device, passes
their raw device pointers and torch's current stream to the C ABI declared in
``include/gcolor.h``, and turns negative return codes into ``GColorError``.
No step of the colouring runs in Python.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, NamedTuple, Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgcolor.so")

FLAG_VALIDATE = 1
FLAG_STATS = 2
FLAG_PLAIN = 4
FLAG_DATAFLOW = 8  # dataflow colouring (Algorithm 3): the serial greedy's result
FLAG_SERIAL_TAIL = 16  # rounds, then the last vertices one at a time (a different colouring)


class GColorError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, strerror(code) if _lib else "?", code))


class _Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("num_colors", ctypes.c_int32),
                ("edge_work", ctypes.c_int64), ("status", ctypes.c_int32), ("serial_tail", ctypes.c_int32)]


class _Round(ctypes.Structure):
    _fields_ = [("round", ctypes.c_int64), ("worklist", ctypes.c_int64), ("edge_work", ctypes.c_int64),
                ("committed", ctypes.c_int64), ("dirty", ctypes.c_int64), ("dirty_edges", ctypes.c_int64),
                ("scanned", ctypes.c_int64)]


class Stats(NamedTuple):
    rounds: int
    num_colors: int
    edge_work: int
    round_log: List[Tuple[int, int, int]]  # (k, |U_k|, E_k)
    # per round: (committed, dirty, dirty degree sum, row entries the dirty pass read)
    detail: List[Tuple[int, int, int, int]]
    serial_tail: int = 0  # vertices the sequential finish coloured (FLAG_SERIAL_TAIL)


def library_path() -> str:
    return _SO


def _load():
    if not os.path.exists(_SO):
        raise ImportError(
            "libgcolor.so is not built (%s); run `python -m paper_1205_3809_amd.build` "
            "or __graft_entry__.build()" % _SO)
    lib = ctypes.CDLL(_SO)
    vp = ctypes.c_void_p
    lib.gcolor_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64]
    lib.gcolor_workspace_bytes.restype = ctypes.c_size_t
    lib.color_graph.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
    lib.color_graph.restype = ctypes.c_int
    lib.color_graph_ex.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_uint32,
                                   ctypes.POINTER(_Stats), ctypes.POINTER(_Round), ctypes.c_int32, vp]
    lib.color_graph_ex.restype = ctypes.c_int
    lib.color_graph_async.argtypes = [ctypes.c_int32, ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_size_t,
                                      ctypes.c_int32, ctypes.c_uint32, vp, vp]
    lib.color_graph_async.restype = ctypes.c_int
    lib.gcolor_strerror.argtypes = [ctypes.c_int]
    lib.gcolor_strerror.restype = ctypes.c_char_p
    lib.gcolor_version.argtypes = []
    lib.gcolor_version.restype = ctypes.c_char_p
    lib.gcolor_set_tuning.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    lib.gcolor_set_tuning.restype = ctypes.c_int
    lib.gcolor_get_tuning.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.gcolor_set_batch_tuning.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.gcolor_set_kernel_blocks.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.gcolor_set_kernel_blocks.restype = ctypes.c_int
    lib.gcolor_get_kernel_blocks.argtypes = [ctypes.POINTER(ctypes.c_int32)] * 2
    lib.gcolor_blocks_workspace_bytes.argtypes = [ctypes.c_int32]
    lib.gcolor_blocks_workspace_bytes.restype = ctypes.c_size_t
    lib.color_graph_blocks.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp, ctypes.c_size_t,
                                       ctypes.POINTER(_Stats), vp]
    lib.color_graph_blocks.restype = ctypes.c_int
    lib.gcolor_set_serial_tail.argtypes = [ctypes.c_int32]
    lib.gcolor_set_serial_tail.restype = ctypes.c_int
    lib.gcolor_get_serial_tail.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.gcolor_get_serial_tail.restype = ctypes.c_int
    lib.gcolor_set_round_cap.argtypes = [ctypes.c_int32]
    lib.gcolor_set_round_cap.restype = ctypes.c_int
    lib.gcolor_get_round_cap.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.gcolor_get_round_cap.restype = ctypes.c_int
    lib.gcolor_set_batch_tuning.restype = ctypes.c_int
    lib.gcolor_get_batch_tuning.argtypes = [ctypes.POINTER(ctypes.c_int32)] * 3
    lib.gcolor_get_tuning.restype = ctypes.c_int
    lib.gcolor_profile.argtypes = [ctypes.c_int32]
    lib.gcolor_profile.restype = ctypes.c_int
    lib.gcolor_profile_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64)]
    lib.gcolor_profile_read.restype = ctypes.c_int
    lib.gcolor_batch_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64]
    lib.gcolor_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.color_graph_batch.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp, vp, vp,
                                      vp, ctypes.c_size_t, vp, vp, vp]
    lib.color_graph_batch.restype = ctypes.c_int
    lib.gcolor_wall_clock_khz.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.gcolor_wall_clock_khz.restype = ctypes.c_int
    lib.gcolor_features_workspace_bytes.argtypes = [ctypes.c_int32]
    lib.gcolor_features_workspace_bytes.restype = ctypes.c_size_t
    lib.gcolor_features.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_uint64, vp, vp, ctypes.c_size_t, vp]
    lib.gcolor_feature_stats.argtypes = [ctypes.c_int64, vp, vp, vp]
    lib.gcolor_feature_norm.argtypes = [ctypes.c_int64, vp, vp, vp]
    lib.gcolor_rank_targets.argtypes = [ctypes.c_int32, vp, vp, vp]
    lib.gcolor_order_learned_workspace_bytes.argtypes = [ctypes.c_int32]
    lib.gcolor_order_learned_workspace_bytes.restype = ctypes.c_size_t
    lib.gcolor_order_learned.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_uint64, vp, vp, vp, vp, vp, vp,
                                         ctypes.c_size_t, vp]
    lib.gcolor_mlp_forward.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    lib.gcolor_mlp_partial_floats.argtypes = [ctypes.c_int32]
    lib.gcolor_mlp_partial_floats.restype = ctypes.c_size_t
    lib.gcolor_mlp_grad.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.gcolor_mlp_adam.argtypes = [vp, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_int32, vp]
    lib.gcolor_mlp_refresh_bf16.argtypes = [vp, vp, vp]
    lib.gcolor_scores_to_keys.argtypes = [ctypes.c_int64, vp, vp, vp, vp]
    lib.gcolor_smallest_last_host.argtypes = [ctypes.c_int32, vp, vp, vp, vp]
    lib.gcolor_smallest_last.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
    for f in ("gcolor_features", "gcolor_feature_stats", "gcolor_feature_norm", "gcolor_rank_targets",
              "gcolor_order_learned", "gcolor_mlp_forward", "gcolor_mlp_grad", "gcolor_mlp_adam",
              "gcolor_mlp_refresh_bf16", "gcolor_scores_to_keys", "gcolor_smallest_last_host",
              "gcolor_smallest_last"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


_lib = _load()


def strerror(code: int) -> str:
    return _lib.gcolor_strerror(int(code)).decode()


def version() -> str:
    return _lib.gcolor_version().decode()


def workspace_bytes(n: int, nnz: int) -> int:
    return int(_lib.gcolor_workspace_bytes(int(n), int(nnz)))


def _dev_ptr(t: Optional[torch.Tensor], name: str, dtypes, n: Optional[int] = None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be on a HIP device (got %s)" % (name, t.device))
    if t.dtype not in dtypes:
        raise TypeError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


_I32 = (torch.int32,)
_KEY = (torch.int32, torch.uint32) if hasattr(torch, "uint32") else (torch.int32,)


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def color_graph_ex(row_ptr: torch.Tensor, col_idx: torch.Tensor, priority: Optional[torch.Tensor] = None,
                   colors_out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                   flags: int = 0, stats: bool = False, max_log: int = 0, stream=None):
    """Colour a symmetric CSR graph on its device.  Returns (colors, Stats or None).

    priority (int32/uint32, bit pattern taken as uint32) sets the precedence
    (priority, id); None means the vertex index alone (rows must be sorted).
    """
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr must have n+1 entries")
    rp = _dev_ptr(row_ptr, "row_ptr", _I32)
    ci = _dev_ptr(col_idx, "col_idx", _I32)
    pr = _dev_ptr(priority, "priority", _KEY, n)
    if colors_out is None:
        colors_out = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    co = _dev_ptr(colors_out, "colors_out", _I32, n)
    ws = None
    ws_bytes = 0
    if workspace is not None:
        ws = _dev_ptr(workspace, "workspace", (torch.uint8, torch.int8, torch.int32, torch.int64))
        ws_bytes = workspace.numel() * workspace.element_size()
    st = _Stats()
    want = stats or max_log > 0
    if want:
        flags |= FLAG_STATS
    logbuf = (_Round * max(max_log, 1))() if max_log > 0 else None
    with torch.cuda.device(row_ptr.device):
        rc = _lib.color_graph_ex(n, rp, ci, pr, co, ws, ws_bytes, flags,
                                 ctypes.byref(st) if want else None,
                                 logbuf if logbuf is not None else None, max_log, _stream_handle(stream))
    if rc != 0:
        raise GColorError(rc, "color_graph_ex")
    if not want:
        return colors_out, None
    log = []
    detail = []
    if logbuf is not None:
        for i in range(min(st.rounds, max_log)):
            log.append((int(logbuf[i].round), int(logbuf[i].worklist), int(logbuf[i].edge_work)))
            detail.append((int(logbuf[i].committed), int(logbuf[i].dirty), int(logbuf[i].dirty_edges),
                           int(logbuf[i].scanned)))
    return colors_out, Stats(int(st.rounds), int(st.num_colors), int(st.edge_work), log, detail,
                             int(st.serial_tail))


STATS_DTYPE_WORDS = 6  # gcolor_stats_t as int32 words: rounds, colours, edge work (2), status, serial tail


def color_graph_async(row_ptr: torch.Tensor, col_idx: torch.Tensor, nnz: int, workspace: torch.Tensor,
                      max_rounds: int, priority: Optional[torch.Tensor] = None,
                      colors_out: Optional[torch.Tensor] = None, stats_out: Optional[torch.Tensor] = None,
                      validate: bool = False, stream=None):
    """Stream-ordered colouring with a round budget: nothing is read back and
    nothing allocated by the library, so the call can be captured in a HIP
    graph.  stats_out: int32[6] device tensor receiving gcolor_stats_t (see
    stats_from_device).  Returns (colors_out, stats_out)."""
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr must have n+1 entries")
    rp = _dev_ptr(row_ptr, "row_ptr", _I32)
    ci = _dev_ptr(col_idx, "col_idx", _I32)
    pr = _dev_ptr(priority, "priority", _KEY, n)
    if colors_out is None:
        colors_out = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    co = _dev_ptr(colors_out, "colors_out", _I32, n)
    if stats_out is None:
        stats_out = torch.zeros(STATS_DTYPE_WORDS, dtype=torch.int32, device=row_ptr.device)
    so = _dev_ptr(stats_out, "stats_out", _I32, STATS_DTYPE_WORDS)
    ws = _dev_ptr(workspace, "workspace", (torch.uint8, torch.int8, torch.int32, torch.int64))
    ws_bytes = workspace.numel() * workspace.element_size()
    with torch.cuda.device(row_ptr.device):
        rc = _lib.color_graph_async(n, int(nnz), rp, ci, pr, co, ws, ws_bytes, int(max_rounds),
                                    FLAG_VALIDATE if validate else 0, so, _stream_handle(stream))
    if rc != 0:
        raise GColorError(rc, "color_graph_async")
    return colors_out, stats_out


def stats_from_device(stats_out: torch.Tensor):
    """(rounds, num_colors, edge_work, status) from a stats tensor that
    color_graph_async filled (synchronises with its stream)."""
    w = stats_out.cpu().numpy()
    edge = int(w[2].astype("uint32")) | (int(w[3]) << 32)
    return int(w[0]), int(w[1]), edge, int(w[4])


def blocks_workspace_bytes(n: int) -> int:
    return int(_lib.gcolor_blocks_workspace_bytes(int(n)))


def color_graph_blocks(row_ptr: torch.Tensor, col_idx: torch.Tensor, priority: Optional[torch.Tensor] = None,
                       block_size: int = 64, colors_out: Optional[torch.Tensor] = None,
                       workspace: Optional[torch.Tensor] = None, stream=None):
    """Block Gauss-Seidel colouring (fixed id blocks of block_size vertices
    coloured in order within each round).  Returns (colors, Stats); the
    Stats carry no per-round log."""
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr must have n+1 entries")
    rp = _dev_ptr(row_ptr, "row_ptr", _I32)
    ci = _dev_ptr(col_idx, "col_idx", _I32)
    pr = _dev_ptr(priority, "priority", _KEY, n)
    if colors_out is None:
        colors_out = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    co = _dev_ptr(colors_out, "colors_out", _I32, n)
    ws, ws_bytes = None, 0
    if workspace is not None:
        ws = _dev_ptr(workspace, "workspace", (torch.uint8, torch.int8, torch.int32, torch.int64))
        ws_bytes = workspace.numel() * workspace.element_size()
    st = _Stats()
    with torch.cuda.device(row_ptr.device):
        rc = _lib.color_graph_blocks(n, rp, ci, pr, int(block_size), co, ws, ws_bytes, ctypes.byref(st),
                                     _stream_handle(stream))
    if rc != 0:
        raise GColorError(rc, "color_graph_blocks")
    return colors_out, Stats(int(st.rounds), int(st.num_colors), int(st.edge_work), [], [])


def color_graph(row_ptr: torch.Tensor, col_idx: torch.Tensor, priority: Optional[torch.Tensor] = None,
                colors_out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Colour with the library's own cached workspace; returns colors_out."""
    n = row_ptr.numel() - 1
    rp = _dev_ptr(row_ptr, "row_ptr", _I32)
    ci = _dev_ptr(col_idx, "col_idx", _I32)
    pr = _dev_ptr(priority, "priority", _KEY, n)
    if colors_out is None:
        colors_out = torch.empty(max(n, 0), dtype=torch.int32, device=row_ptr.device)
    co = _dev_ptr(colors_out, "colors_out", _I32, n)
    with torch.cuda.device(row_ptr.device):
        rc = _lib.color_graph(n, rp, ci, pr, co, _stream_handle(stream))
    if rc != 0:
        raise GColorError(rc, "color_graph")
    return colors_out


def smallest_last(row_ptr: torch.Tensor, col_idx: torch.Tensor, rank_out: Optional[torch.Tensor] = None,
                  stream=None):
    """Exact smallest-last order on the device: returns (rank, degeneracy),
    rank[v] = v's position in the colouring order (int32, on the device)."""
    n = row_ptr.numel() - 1
    rp = _dev_ptr(row_ptr, "row_ptr", _I32)
    ci = _dev_ptr(col_idx, "col_idx", _I32)
    if rank_out is None:
        rank_out = torch.empty(max(n, 0), dtype=torch.int32, device=row_ptr.device)
    ro = _dev_ptr(rank_out, "rank_out", _I32, n)
    deg = ctypes.c_int32()
    with torch.cuda.device(row_ptr.device):
        rc = _lib.gcolor_smallest_last(n, rp, ci, ro, ctypes.byref(deg), _stream_handle(stream))
    if rc != 0:
        raise GColorError(rc, "gcolor_smallest_last")
    return rank_out, int(deg.value)


def set_tuning(bin_limits=None, blocks_per_cu: int = 0) -> None:
    """Degree-bin limits (4 non-decreasing ints) and blocks per CU of the
    phase grids; affects speed only, never the colouring."""
    arr = None
    if bin_limits is not None:
        if len(bin_limits) != 4:
            raise ValueError("bin_limits needs 4 entries")
        arr = (ctypes.c_int32 * 4)(*[int(x) for x in bin_limits])
    rc = _lib.gcolor_set_tuning(arr, int(blocks_per_cu))
    if rc != 0:
        raise GColorError(rc, "gcolor_set_tuning")


def get_tuning():
    arr = (ctypes.c_int32 * 4)()
    bpc = ctypes.c_int32()
    _lib.gcolor_get_tuning(arr, ctypes.byref(bpc))
    return list(arr), int(bpc.value)


def set_kernel_blocks(blocks_a: int = 0, blocks_c: int = 0) -> None:
    """Blocks per CU of the two round kernels of the incremental engine
    (0: the common blocks_per_cu of set_tuning); speed only."""
    rc = _lib.gcolor_set_kernel_blocks(int(blocks_a), int(blocks_c))
    if rc != 0:
        raise GColorError(rc, "gcolor_set_kernel_blocks")


def get_kernel_blocks():
    v = [ctypes.c_int32() for _ in range(2)]
    _lib.gcolor_get_kernel_blocks(*[ctypes.byref(x) for x in v])
    return tuple(int(x.value) for x in v)


def set_round_cap(max_rounds: int = 0) -> None:
    """Most rounds a later colouring may take (0: the default, n + 64);
    a colouring that needs more raises GColorError with code -5."""
    rc = _lib.gcolor_set_round_cap(int(max_rounds))
    if rc != 0:
        raise GColorError(rc, "gcolor_set_round_cap")


def set_serial_tail(max_vertices: int) -> None:
    """Vertices left to the sequential finish of FLAG_SERIAL_TAIL (1..8192)."""
    rc = _lib.gcolor_set_serial_tail(int(max_vertices))
    if rc != 0:
        raise GColorError(rc, "gcolor_set_serial_tail")


def get_serial_tail() -> int:
    v = ctypes.c_int32()
    _lib.gcolor_get_serial_tail(ctypes.byref(v))
    return int(v.value)


def get_round_cap() -> int:
    v = ctypes.c_int32()
    _lib.gcolor_get_round_cap(ctypes.byref(v))
    return int(v.value)


def set_batch_tuning(block_threads: int = 0, lds_factor: int = 8, lds_max_vertices: int = 65536) -> None:
    """Threads per workgroup (0 = automatic, 256, 1024) and the LDS path's
    vertex capacity (lds_factor x mean graph size, capped at lds_max_vertices;
    0 disables it) of color_graph_batch; speed only, never the colouring."""
    rc = _lib.gcolor_set_batch_tuning(int(block_threads), int(lds_factor), int(lds_max_vertices))
    if rc != 0:
        raise GColorError(rc, "gcolor_set_batch_tuning")


def get_batch_tuning():
    v = [ctypes.c_int32() for _ in range(3)]
    _lib.gcolor_get_batch_tuning(*[ctypes.byref(x) for x in v])
    return tuple(int(x.value) for x in v)


PROF_PHASE1 = 0   # plain engine: tentative colouring
PROF_PHASE2 = 1   # plain engine: conflict detection + compaction
PROF_INC_A = 2    # incremental: tentative colours of dirty vertices
PROF_LISTS = 3    # incremental: dirty lists of the next round, in vertex order
PROF_INC_C = 4    # incremental: commit + push
PROF_FLOW = 5     # dataflow: one round


def profile(enable: bool) -> None:
    """Turn per-launch HIP-event timing of the phase kernels on (totals cleared) or off."""
    _lib.gcolor_profile(1 if enable else 0)


def profile_read(kernel: int):
    """(total milliseconds, launches) recorded for kernel PROF_PHASE1 / PROF_PHASE2."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    rc = _lib.gcolor_profile_read(int(kernel), ctypes.byref(ms), ctypes.byref(n))
    if rc != 0:
        raise GColorError(rc, "gcolor_profile_read")
    return float(ms.value), int(n.value)


def raw_library():
    """The loaded ctypes library (for ABI-level tests)."""
    return _lib


def batch_workspace_bytes(num_graphs: int, total_vertices: int, total_nnz: int) -> int:
    return int(_lib.gcolor_batch_workspace_bytes(int(num_graphs), int(total_vertices), int(total_nnz)))


def wall_clock_khz() -> int:
    khz = ctypes.c_int32()
    rc = _lib.gcolor_wall_clock_khz(ctypes.byref(khz))
    if rc != 0:
        raise GColorError(rc, "gcolor_wall_clock_khz")
    return int(khz.value)


def color_graph_batch(vtx_off: torch.Tensor, edge_off: torch.Tensor, row_ptr: torch.Tensor, col_idx: torch.Tensor,
                      total_vertices: int, total_nnz: int, priority: Optional[torch.Tensor] = None,
                      colors_out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                      ticks: Optional[torch.Tensor] = None, rounds: Optional[torch.Tensor] = None, stream=None):
    """Colour G independent graphs in one launch (asynchronous, capturable).

    vtx_off/edge_off: int64[G+1]; row_ptr: int32[V+G] (each graph's local
    offsets, concatenated); col_idx: int32[nnz] local ids.  total_vertices and
    total_nnz are V and nnz (passed in so that nothing is read back).
    Returns colors_out (int32[V]).
    """
    G = vtx_off.numel() - 1
    if G < 0:
        raise ValueError("vtx_off must have G+1 entries")
    i64 = (torch.int64,)
    vo = _dev_ptr(vtx_off, "vtx_off", i64, G + 1)
    eo = _dev_ptr(edge_off, "edge_off", i64, G + 1)
    rp = _dev_ptr(row_ptr, "row_ptr", _I32, int(total_vertices) + G)
    ci = _dev_ptr(col_idx, "col_idx", _I32)
    pr = _dev_ptr(priority, "priority", _KEY, int(total_vertices))
    if colors_out is None:
        colors_out = torch.empty(int(total_vertices), dtype=torch.int32, device=row_ptr.device)
    co = _dev_ptr(colors_out, "colors_out", _I32, int(total_vertices))
    if workspace is None:
        workspace = torch.empty(batch_workspace_bytes(G, total_vertices, total_nnz), dtype=torch.uint8,
                                device=row_ptr.device)
    ws = _dev_ptr(workspace, "workspace", (torch.uint8, torch.int8, torch.int32, torch.int64))
    tk = _dev_ptr(ticks, "ticks", i64, 2 * G)
    rd = _dev_ptr(rounds, "rounds", _I32, G)
    with torch.cuda.device(row_ptr.device):
        rc = _lib.color_graph_batch(G, int(total_vertices), int(total_nnz), vo, eo, rp, ci, pr, co, ws,
                                    workspace.numel() * workspace.element_size(), tk, rd, _stream_handle(stream))
    if rc != 0:
        raise GColorError(rc, "color_graph_batch")
    return colors_out
