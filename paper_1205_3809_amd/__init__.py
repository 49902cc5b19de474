"""MI355X-native speculative iterative graph colouring.

The colouring itself runs in ``libgcolor.so`` (hand-written HIP for gfx950,
C ABI in ``include/gcolor.h``); this package only marshals torch tensors into
that ABI.  There is no CPU fallback: if the library is missing, importing the
binding raises.
"""
from ._binding import (  # noqa: F401
    GColorError,
    Stats,
    blocks_workspace_bytes,
    color_graph,
    color_graph_blocks,
    color_graph_ex,
    color_graph_async,
    stats_from_device,
    library_path,
    strerror,
    version,
    workspace_bytes,
    FLAG_VALIDATE,
    FLAG_STATS,
    FLAG_PLAIN,
    FLAG_DATAFLOW,
    FLAG_SERIAL_TAIL,
    PROF_PHASE1,
    PROF_PHASE2,
    PROF_INC_A,
    PROF_LISTS,
    PROF_INC_C,
    PROF_FLOW,
    get_tuning,
    get_batch_tuning,
    set_batch_tuning,
    get_kernel_blocks,
    set_kernel_blocks,
    get_round_cap,
    get_serial_tail,
    set_serial_tail,
    set_round_cap,
    profile,
    profile_read,
    raw_library,
    set_tuning,
    smallest_last,
    batch_workspace_bytes,
    color_graph_batch,
    wall_clock_khz,
)

from . import autotune  # noqa: E402,F401

# A tuning table chosen by the autotuner can be applied at import:
# GCOLOR_TUNING=<table.json>:<config name>.
import os as _os

if _os.environ.get("GCOLOR_TUNING"):
    from .autotune import apply_from_env as _apply_from_env

    _apply_from_env(_os.environ["GCOLOR_TUNING"])
