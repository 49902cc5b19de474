"""Autotuner for the library's launch parameters.

The parameters change speed only: the colouring is a function of the graph
and the priority alone, and every candidate's colours are compared with the
colours of the starting setting (a mismatch raises).

* Single graph (color_graph): the four degree-bin limits (one lane, 4 lanes,
  16 lanes and one wavefront per vertex; a workgroup above the last), the
  blocks per CU of the round grids and of the two round kernels, by coordinate
  descent from the current setting: each coordinate tries all its candidate
  values and takes the fastest when it beats the current setting by more than
  the noise margin.
* Batch (color_graph_batch): threads per workgroup (256 or 1024) and the LDS
  path's vertex capacity (a factor of the batch's mean graph size, capped),
  by exhaustive search over a small grid that includes the LDS path switched
  off.

Results form a JSON table keyed by device architecture, then configuration
name; apply() loads an entry into the library, and so does the environment
variable GCOLOR_TUNING=<table.json>:<name> when the package is imported.
"""
from __future__ import annotations

import json
import os
from typing import Callable, Dict, Optional

import torch

from . import _binding as B

BIN_CANDIDATES = ([2, 4, 8, 16], [16, 32, 64], [64, 128, 256], [256, 384, 512, 768, 1024, 2048, 4096])
BPC_CANDIDATES = [1, 2, 3, 4, 5, 6, 8, 12, 16]
KERNEL_BLOCK_CANDIDATES = [0, 2, 3, 4, 6, 8, 12]  # per round kernel; 0 = blocks_per_cu
BATCH_BLOCKS = [256, 1024]
BATCH_FACTORS = [2, 4, 8, 16]
BATCH_CAPS = [16384, 32768, 65536]
MARGIN = 0.995  # a candidate must be at least 0.5% faster (repeated trials agree within 0.2%)


def arch() -> str:
    """gfx name of the current device (e.g. 'gfx950')."""
    name = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    return name.split(":")[0]


def _time_ms(fn: Callable[[], torch.Tensor], reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune_single(row_ptr: torch.Tensor, col_idx: torch.Tensor, priority: Optional[torch.Tensor] = None,
                reps: int = 3, passes: int = 2, log: Optional[Callable[[str], None]] = None,
                flags: int = 0) -> Dict:
    """Coordinate descent over (bin limits, blocks per CU) for color_graph_ex
    with these flags (engine choice) on this graph.  Leaves the best setting
    applied and returns it with the timings of every trial."""
    out = torch.empty(row_ptr.numel() - 1, dtype=torch.int32, device=row_ptr.device)
    bins0, bpc0 = B.get_tuning()
    cur = list(bins0) + [bpc0] + list(B.get_kernel_blocks())

    def setup(setting):
        B.set_tuning(setting[:4], setting[4])
        B.set_kernel_blocks(*setting[5:7])

    def run(setting):
        setup(setting)
        return B.color_graph_ex(row_ptr, col_idx, priority, out, flags=flags)

    run(cur)
    torch.cuda.synchronize()
    ref = out.clone()

    def measure(trial):
        t = _time_ms(lambda: run(trial), reps)
        if not torch.equal(out, ref):
            setup(cur)
            raise RuntimeError("colours changed under tuning %s" % trial)
        if log:
            log("tune_single %s: %.3f ms" % (trial, t))
        return t

    cur, best_t, t0, trials = coordinate_descent(cur, SINGLE_CANDIDATES, measure, passes)
    setup(cur)
    return {"kind": "single", "bin_limits": cur[:4], "blocks_per_cu": cur[4], "kernel_blocks": cur[5:7],
            "ms": round(best_t, 4), "start_ms": round(t0, 4), "trials": trials}


SINGLE_CANDIDATES = list(BIN_CANDIDATES) + [BPC_CANDIDATES, KERNEL_BLOCK_CANDIDATES, KERNEL_BLOCK_CANDIDATES]


def coordinate_descent(start, candidates, measure, passes=2, margin=MARGIN):
    """Coordinate descent over the settings (one list of candidate values per
    coordinate; the first four, the bin limits, must stay non-decreasing):
    each coordinate tries all its values with the others fixed and takes the
    fastest of them when it beats the current setting by the noise margin;
    up to `passes` sweeps, stopping after one that changes nothing.  Returns
    (setting, its time, the starting time, every trial)."""
    cur = list(start)
    t0 = measure(cur)
    best_t, trials = t0, [{"setting": list(cur), "ms": round(t0, 4)}]
    for _ in range(passes):
        changed = False
        for i, values in enumerate(candidates):
            pick, pick_t = None, float("inf")
            for v in values:
                trial = list(cur)
                trial[i] = v
                if trial == cur or any(trial[j] > trial[j + 1] for j in range(3)):
                    continue
                t = measure(trial)
                trials.append({"setting": trial, "ms": round(t, 4)})
                if t < pick_t:
                    pick, pick_t = trial, t
            if pick is not None and pick_t < best_t * margin:
                best_t, cur, changed = pick_t, pick, True
        if not changed:
            break
    return cur, best_t, t0, trials


def tune_batch(vtx_off: torch.Tensor, edge_off: torch.Tensor, row_ptr: torch.Tensor, col_idx: torch.Tensor,
               total_vertices: int, total_nnz: int, priority: Optional[torch.Tensor] = None, reps: int = 3,
               log: Optional[Callable[[str], None]] = None) -> Dict:
    """Exhaustive search over (threads per workgroup, LDS capacity factor,
    LDS cap) for color_graph_batch on this batch, plus the LDS path off.
    Leaves the best setting applied and returns it with every trial."""
    G = vtx_off.numel() - 1
    out = torch.empty(int(total_vertices), dtype=torch.int32, device=row_ptr.device)
    ws = torch.empty(B.batch_workspace_bytes(G, total_vertices, total_nnz), dtype=torch.uint8,
                     device=row_ptr.device)
    start = B.get_batch_tuning()

    def run(setting):
        B.set_batch_tuning(*setting)
        return B.color_graph_batch(vtx_off, edge_off, row_ptr, col_idx, total_vertices, total_nnz, priority,
                                   colors_out=out, workspace=ws)

    run(start)
    torch.cuda.synchronize()
    ref = out.clone()
    settings = [(bt, f, cap) for bt in BATCH_BLOCKS for f in BATCH_FACTORS for cap in BATCH_CAPS]
    settings += [(256, 8, 0), (1024, 8, 0)]
    best, best_t, trials = tuple(start), _time_ms(lambda: run(start), reps), []
    t0 = best_t
    trials.append({"setting": list(start), "ms": round(t0, 4)})
    for s in settings:
        t = _time_ms(lambda: run(s), reps)
        if not torch.equal(out, ref):
            B.set_batch_tuning(*best)
            raise RuntimeError("colours changed under batch tuning %s" % (s,))
        trials.append({"setting": list(s), "ms": round(t, 4)})
        if log:
            log("tune_batch %s: %.3f ms" % (s, t))
        if t < best_t * MARGIN:
            best, best_t = s, t
    B.set_batch_tuning(*best)
    return {"kind": "batch", "block_threads": best[0], "lds_factor": best[1], "lds_max_vertices": best[2],
            "ms": round(best_t, 4), "start_ms": round(t0, 4), "trials": trials}


def load_table(path: str) -> Dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(path: str, name: str, entry: Dict, arch_name: Optional[str] = None) -> None:
    """Store entry under table[arch][name] (other entries are kept)."""
    table = load_table(path)
    table.setdefault(arch_name or arch(), {})[name] = entry
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")


def apply(table, name: str, arch_name: Optional[str] = None) -> Optional[Dict]:
    """Load table[arch][name] into the library; returns the entry, or None
    when the table has none for this device and name."""
    if isinstance(table, str):
        table = load_table(table)
    entry = table.get(arch_name or arch(), {}).get(name)
    if entry is None:
        return None
    if entry["kind"] == "single":
        B.set_tuning(entry["bin_limits"], entry["blocks_per_cu"])
        kb = list(entry.get("kernel_blocks", (0, 0)))
        if len(kb) == 3:  # older entries: (dirty kernel, unused, commit kernel)
            kb = [kb[0], kb[2]]
        B.set_kernel_blocks(*kb)
    elif entry["kind"] == "batch":
        B.set_batch_tuning(entry["block_threads"], entry["lds_factor"], entry["lds_max_vertices"])
    else:
        raise ValueError("unknown tuning entry kind %r" % entry["kind"])
    return entry


def apply_from_env(spec: str) -> Optional[Dict]:
    """spec = '<table.json>:<name>' (the value of GCOLOR_TUNING)."""
    path, sep, name = spec.rpartition(":")
    if not sep or not path or not name:
        raise ValueError("GCOLOR_TUNING must be <table.json>:<config name>, got %r" % spec)
    return apply(path, name)


TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
