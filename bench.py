#!/usr/bin/env python3
"""Benchmark: speculative iterative colouring of R-MAT scale 24 on one MI355X.

A step is one full colouring (every round, to an empty worklist) of a graph
already resident in HBM, through the C ABI.  Prints one JSON line with
edges coloured per second, the roofline of the dominant kernel, the CPU
oracle's throughput on the same workload, and the colour counts of the GPU
result and of serial greedy.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--order natural|perm] [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s

WORKLOADS = {
    # name: (kind, params)
    "rmat24": ("rmat", dict(scale=24, edge_factor=8, abcd=(0.55, 0.1, 0.1, 0.25), seed=11)),
    "rmat20-er": ("rmat", dict(scale=20, edge_factor=8, abcd=(0.25, 0.25, 0.25, 0.25), seed=11)),
    "rmat20-g": ("rmat", dict(scale=20, edge_factor=8, abcd=(0.45, 0.15, 0.15, 0.25), seed=11)),
    "uniform14": ("uniform", dict(n=1 << 14, samples=1 << 17, seed=1)),
    # 4096 graphs, n log-uniform in [2^8, 2^16]: 2D 5/9-point and 3D 7/27-point
    # stencil grids with 5% extra random edges, random geometric graphs with
    # mean degree 6..27; natural order; one persistent launch per step
    "batch4096": ("batch", dict(count=4096, seed=2026, log2_lo=8, log2_hi=16)),
    # learned ordering: train on 256 R-MAT scale-16 edge-factor-16 graphs
    # (0.57, 0.19, 0.19, 0.05), seeds 0..255; evaluate on scale 22, seed 1000
    "learned22": ("learned", dict(train_graphs=256, train_scale=16, eval_scale=22, edge_factor=16,
                                  abcd=(0.57, 0.19, 0.19, 0.05), eval_seed=1000, epochs=4, batch=65536)),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_graph(name):
    import graphgen
    kind, p = WORKLOADS[name]
    if kind == "rmat":
        return graphgen.rmat(p["scale"], p["edge_factor"], p["abcd"][:3], p["seed"])
    return graphgen.uniform(p["n"], p["samples"], p["seed"])


def apply_tuning(args, name, search):
    """Launch parameters for this workload: searched and stored with
    --autotune, else read from the package's tuning table (library defaults
    with --no-tuning or when the table has no entry).  Returns what was used."""
    from paper_1205_3809_amd import autotune
    import paper_1205_3809_amd as gc

    if args.autotune:
        entry = search()
        autotune.save(autotune.TABLE, name, entry)
        log("autotune %s: %s (%.3f ms, from %.3f ms)" % (name, {k: v for k, v in entry.items()
                                                              if k not in ("trials", "ms", "start_ms")},
                                                       entry["ms"], entry["start_ms"]))
    elif not args.no_tuning:
        entry = autotune.apply(autotune.TABLE, name)
    else:
        entry = None
    if entry is None:
        return {"source": "library defaults", "single": gc.get_tuning(), "batch": list(gc.get_batch_tuning())}
    return {"source": "autotuner table", **{k: v for k, v in entry.items() if k not in ("trials",)}}


def kernel_source(workload):
    """The source file of the kernels a workload's stored counter traffic
    describes: the batch kernel, or the single-graph kernels."""
    return "batch.hip" if WORKLOADS.get(workload, ("",))[0] == "batch" else "gcolor.hip"


def code_digest(text):
    """Digest of HIP source text without its comments and with whitespace
    runs folded: comment edits leave it unchanged, code edits do not."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = re.sub(r"\s+", " ", text).strip()
    return hashlib.sha256(text.encode()).hexdigest()


def kernel_source_digest(workload="rmat24"):
    """Code digest of the kernel source a workload's counter traffic was
    taken on (stored with the traffic; the traffic is used only while the
    current source has the same digest)."""
    return code_digest(open(os.path.join(ROOT, "paper_1205_3809_amd", "csrc", kernel_source(workload))).read())


def load_traffic_file(workload, order):
    """The stored rocprofv3 counter traffic of this workload, if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, order))
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_sha256") != kernel_source_digest(workload):
        return None
    return d


def load_traffic(workload, order, kernel, launches):
    """Bytes per launch of one kernel between L2 and the memory fabric,
    measured by rocprofv3 counters, if they were taken on the current kernel
    sources; else None."""
    d = load_traffic_file(workload, order)
    k = (d or {}).get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("l2_fabric_bytes_per_launch")


# rocprofv3 --pmc passes of the traffic measurement (at most 4 TCC counters
# each): read requests by size, write requests by size, L2 hits and misses
TRAFFIC_PASSES = (
    ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_sum"),
    ("TCC_EA0_WRREQ_64B_sum", "TCC_EA0_WRREQ_sum", "TCC_BUBBLE_sum"),
    ("TCC_HIT_sum", "TCC_MISS_sum"),
)


def derive_traffic(csv_paths, workload, order, out_path=None):
    """Write profiles/traffic_<workload>_<order>.json from the rocprofv3
    --pmc runs of TRAFFIC_PASSES (each run: this script with --steps 1
    --warmup 0 --copy-calibration).  Read bytes are summed by request size
    (32, 64 and 128 bytes), write bytes likewise (64-byte requests and the
    rest at 32); both are counted where the L2 meets the memory fabric, so
    reads the Infinity Cache serves are included (the counters cannot tell
    them apart).  The 1 GiB device copy of the calibration checks the byte
    arithmetic: it must read and write 1 GiB."""
    import csv
    import re

    tot, disp = {}, {}        # (kernel, counter) -> sum over dispatches, dispatches
    lib, calls = {}, {}       # counter -> sum over every library kernel; colourings
    copy = {}

    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            cn, name, val = r["Counter_Name"], r["Kernel_Name"], float(r["Counter_Value"])
            if "copyBuffer" in name and int(r["Grid_Size"]) == 131072:
                copy[cn] = val  # the 1 GiB calibration copy
                continue
            if re.search(r"::k_\w+", name):
                lib[cn] = lib.get(cn, 0.0) + val
                calls[cn] = calls.get(cn, 0) + ("k_zero_ctl" in name)
            m = re.search(r"k_(inc_[ac]|phase[12]|flow|batch)\b", name)
            if m:
                key = (m.group(1), cn)
                tot[key] = tot.get(key, 0.0) + val
                disp[key] = disp.get(key, 0) + 1

    def rd_bytes(get):
        return 32 * get("TCC_EA0_RDREQ_32B_sum") + 64 * get("TCC_EA0_RDREQ_64B_sum") + \
            128 * get("TCC_EA0_RDREQ_128B_sum")

    def wr_bytes(get):
        w64 = get("TCC_EA0_WRREQ_64B_sum")
        return 64 * w64 + 32 * (get("TCC_EA0_WRREQ_sum") - w64)

    def fetch_size(get):
        # rocprofv3's derived FETCH_SIZE expression (bytes), for comparison
        b, rq, r32 = get("TCC_BUBBLE_sum"), get("TCC_EA0_RDREQ_sum"), get("TCC_EA0_RDREQ_32B_sum")
        return 128 * b + 64 * (rq - b - r32) + 32 * r32

    out = {"kernel_source_sha256": kernel_source_digest(workload), "workload": workload, "order": order,
           "method": "read bytes = 32 x TCC_EA0_RDREQ_32B + 64 x TCC_EA0_RDREQ_64B + 128 x TCC_EA0_RDREQ_128B; "
                     "write bytes = 64 x TCC_EA0_WRREQ_64B + 32 x (TCC_EA0_WRREQ - TCC_EA0_WRREQ_64B); "
                     "counted between L2 and the memory fabric (Infinity Cache hits included)",
           "passes": [list(p) for p in TRAFFIC_PASSES], "kernels": {}}
    if copy:
        g = lambda c: copy.get(c, 0.0)
        out["copy_check"] = {"true_bytes": 1 << 30, "read_bytes": rd_bytes(g), "write_bytes": wr_bytes(g),
                             "fetch_size_formula_bytes": fetch_size(g),
                             "read_requests": {c: g(c) for c in TRAFFIC_PASSES[0]}}
    ncol = max(calls.get("TCC_EA0_RDREQ_sum", 0), 1)
    gl = lambda c: lib.get(c, 0.0) / max(calls.get(c, 0), 1)
    rd, wr = rd_bytes(gl), wr_bytes(gl)
    out["per_colouring"] = {"colourings_counted": ncol, "read_bytes": rd, "write_bytes": wr,
                            "l2_fabric_bytes": rd + wr}
    for k in sorted({k for k, _ in tot}):
        g = lambda c: tot.get((k, c), 0.0) / max(disp.get((k, c), 0), 1)
        rdk, wrk = rd_bytes(g), wr_bytes(g)
        hit, miss = g("TCC_HIT_sum"), g("TCC_MISS_sum")
        out["kernels"][k] = {
            "launches_counted": disp.get((k, "TCC_EA0_RDREQ_sum"), 0),
            "read_bytes_per_launch": rdk, "write_bytes_per_launch": wrk,
            "l2_fabric_bytes_per_launch": rdk + wrk,
            "fetch_size_formula_bytes_per_launch": fetch_size(g),
            "read_requests_per_launch": {c.replace("TCC_EA0_RDREQ_", "").replace("_sum", ""): g(c)
                                         for c in TRAFFIC_PASSES[0]},
            "l2_hit_rate": hit / (hit + miss) if hit + miss else None}
    path = out_path or os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, order))
    json.dump(out, open(path, "w"), indent=1, sort_keys=True)
    print(path)
    return out


def bench_blocks(args):
    """The block Gauss-Seidel variant (color_graph_blocks) on a single-graph
    workload: K timed colourings; the roofline is priced over the whole call
    (the entry point records no per-kernel events)."""
    import numpy as np
    import torch

    import graphgen
    import paper_1205_3809_amd as gc

    if not torch.cuda.is_available():
        print("bench.py: no HIP device visible", file=sys.stderr)
        sys.exit(1)
    g = make_graph(args.workload)
    key = graphgen.random_priority(g.n, 12) if args.order == "perm" else None
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    pr = None if key is None else torch.from_numpy(key.view(np.int32)).to(dev)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    ws = torch.empty(gc.blocks_workspace_bytes(g.n), dtype=torch.uint8, device=dev)
    B = args.block_size
    _, st = gc.color_graph_blocks(rp, ci, pr, block_size=B, colors_out=out, workspace=ws)
    torch.cuda.synchronize()
    log("blocks B=%d: rounds=%d colours=%d edge_work=%.2f x nnz" % (B, st.rounds, st.num_colors,
                                                                   st.edge_work / max(g.nnz, 1)))

    def step():
        gc.color_graph_blocks(rp, ci, pr, block_size=B, colors_out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = 1000.0 * wall / args.steps
    ev_ms = ev0.elapsed_time(ev1) / args.steps
    log("timed %d steps: %.3f ms/step (wall), %.3f ms/step (events)" % (args.steps, ms_per_step, ev_ms))
    # roofline over the whole call against the input's floor: read every row
    # once (4 B per entry) and write every colour (plus the row_ptr, 4 B per
    # vertex).  The plain two-pass method's bytes (8 B per entry of an
    # uncoloured row in each pass, 24 B per vertex and round, one colour
    # write) are reported beside it as an effective rate only: the kernels
    # move less than that.
    bmin = 4 * g.nnz + 8 * g.n
    plain = 16 * st.edge_work + 24 * g.n * st.rounds + 4 * g.n
    achieved = bmin / (ev_ms / 1e3) / 1e9
    roofline = {"kernel": "whole call (k_blk_first + k_blk_check)", "bound": "hbm",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "bytes_model": "lower bound: 4 B per row entry + 8 B per vertex",
                "algorithmic_bytes_per_step": int(bmin),
                "effective": {"plain_method_bytes": int(plain),
                              "plain_method_GBps": round(plain / (ev_ms / 1e3) / 1e9, 1),
                              "plain_method_frac": round(plain / (ev_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}}
    # the block oracle (every host thread) on the same workload: baseline
    # and parity; the serial greedy for the colour count
    cpu = None
    parity = None
    greedy_colors = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        ref = oracle.block_gs(g.row_ptr, g.col_idx, key, B, threads=0)
        dt = time.perf_counter() - t
        parity = bool(np.array_equal(ref.colors, out.cpu().numpy())) and ref.rounds == st.rounds
        cpu = {"value": round(g.edges / dt, 1), "unit": "edges/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "the full workload (%.1f s)" % dt}
        greedy_colors = int(oracle.greedy(g.row_ptr, g.col_idx, key).max())
        log("block oracle %.1fs parity=%s; serial greedy %d colours" % (dt, parity, greedy_colors))

    p = WORKLOADS[args.workload][1]
    config = {"workload": "%s-%s" % (args.workload, args.order), "engine": "blocks", "block_size": B,
              "n": g.n, "nnz": g.nnz, "edges": g.edges}
    config.update({k: v for k, v in p.items()})
    res = {
        "metric": "edges colored/sec + % HBM peak at R-MAT s24; colors vs serial greedy",
        "value": round(g.edges / (ms_per_step / 1e3), 1), "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic", "config": config, "colors": int(st.num_colors), "serial_greedy_colors": greedy_colors,
        "rounds": int(st.rounds), "edge_work_over_nnz": round(st.edge_work / max(g.nnz, 1), 3),
        "parity_vs_oracle": parity, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--derive-traffic":
        # --derive-traffic WORKLOAD ORDER CSV [CSV ...] (one per pass of TRAFFIC_PASSES)
        derive_traffic(sys.argv[4:], sys.argv[2], sys.argv[3])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS))
    ap.add_argument("--order", default="natural", choices=["natural", "perm"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event-timed pass")
    ap.add_argument("--engine", default="incremental", choices=["incremental", "plain", "dataflow", "blocks"],
                    help="dataflow: the dataflow algorithm in rounds (a different colouring: the serial "
                         "greedy's); blocks: the block Gauss-Seidel variant (a different colouring)")
    ap.add_argument("--block-size", type=int, default=64, help="vertices per block of --engine blocks")
    ap.add_argument("--serial-tail", type=int, default=0,
                    help="incremental engine with the sequential finish: rounds while more than this many "
                         "vertices are uncoloured, then one at a time (a different colouring; 0 = off)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--autotune", action="store_true",
                    help="search the launch parameters for this workload, store them in the package's "
                         "tuning table, then measure with them")
    ap.add_argument("--no-tuning", action="store_true", help="ignore the tuning table (library defaults)")
    args = ap.parse_args()

    if WORKLOADS[args.workload][0] == "batch" and args.gpus == 1:
        return bench_batch(args)
    if WORKLOADS[args.workload][0] == "learned" and args.gpus == 1:
        return bench_learned(args)
    if args.engine == "blocks" and args.gpus == 1:
        return bench_blocks(args)
    if args.gpus != 1:
        print("bench.py: the colouring runs on one GPU (got --gpus %d); sharding the method across "
              "GPUs is not built." % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_1205_3809_amd as gc

    if not torch.cuda.is_available():
        print("bench.py: no HIP device visible", file=sys.stderr)
        sys.exit(1)

    t0 = time.time()
    g = make_graph(args.workload)
    key = graphgen.random_priority(g.n, 12) if args.order == "perm" else None
    log("graph %s n=%d nnz=%d edges=%d built in %.1fs" % (args.workload, g.n, g.nnz, g.edges, time.time() - t0))

    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    pr = None if key is None else torch.from_numpy(key.view(np.int32)).to(dev)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    flags = {"plain": gc.FLAG_PLAIN, "dataflow": gc.FLAG_DATAFLOW}.get(args.engine, 0)
    if args.serial_tail:
        if args.engine != "incremental":
            print("bench.py: --serial-tail applies to the incremental engine", file=sys.stderr)
            sys.exit(2)
        gc.set_serial_tail(args.serial_tail)
        flags |= gc.FLAG_SERIAL_TAIL
    tuning = apply_tuning(args, "%s-%s%s" % (args.workload, args.order,
                                             "-dataflow" if args.engine == "dataflow" else ""),
                          lambda: gc.autotune.tune_single(rp, ci, pr, log=log, flags=flags))

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst

    # one run with statistics: rounds, colours, per-round worklist and edge work
    _, st = gc.color_graph_ex(rp, ci, pr, out, flags=flags, stats=True, max_log=1 << 16)
    torch.cuda.synchronize()
    gpu_colors = out.cpu().numpy()
    log("rounds=%d colours=%d edge_work=%.2f x nnz" % (st.rounds, st.num_colors, st.edge_work / max(g.nnz, 1)))

    def step():
        if flags:
            gc.color_graph_ex(rp, ci, pr, out, flags=flags)
        else:
            gc.color_graph(rp, ci, pr, out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K full colourings
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = 1000.0 * wall / args.steps
    log("timed %d steps: %.3f ms/step (wall), %.3f ms/step (events)"
        % (args.steps, ms_per_step, ev0.elapsed_time(ev1) / args.steps))
    edges_per_s = g.edges / (ms_per_step / 1000.0)

    # per-kernel durations: HIP events around every launch, same steps again
    roofline = None
    kern = {}
    if not args.no_profile:
        gc.profile(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        if args.engine == "plain":
            kinds = (("phase1", gc.PROF_PHASE1), ("phase2", gc.PROF_PHASE2))
        elif args.engine == "dataflow":
            kinds = (("flow", gc.PROF_FLOW),)
        else:
            kinds = (("inc_a", gc.PROF_INC_A), ("inc_c", gc.PROF_INC_C))
        for name, kid in kinds:
            ms, nl = gc.profile_read(kid)
            kern[name] = dict(total_ms=ms / args.steps, launches=nl // args.steps,
                              avg_us=1000.0 * ms / max(nl, 1))
        gc.profile(False)
        # algorithmic bytes per kernel over one colouring (per-unit figures:
        # bytes every correct implementation of the kernel must move)
        U = [u for _, u, _ in st.round_log]
        E = [e for _, _, e in st.round_log]
        C = [d[0] for d in st.detail]
        D = [d[1] for d in st.detail]
        DE = [d[2] for d in st.detail]
        if args.engine == "plain":
            # phase 1: neighbour id + its colour (8 B) per row entry; list entry,
            # row_ptr pair and tentative write (16 B) per worklist vertex
            algo = {"phase1": sum(8 * e + 16 * u for u, e in zip(U, E))}
        elif args.engine == "dataflow":
            # per vertex (once): list entry, row_ptr pair, split, colour and
            # colour-byte writes, its append to a list (25 B); per preceding
            # entry: neighbour id + its colour byte (5 B); per later entry:
            # neighbour id + a read-modify-write of its counter (12 B); each
            # undirected edge is one preceding and one later entry
            algo = {"flow": 25 * g.n + 17 * (g.nnz // 2)}
        else:
            # state words: 1 byte in rounds 1..127, then 2 (4 when the largest
            # degree + 1 exceeds 32767)
            wide = 2 if int(g.degrees().max()) + 1 <= 32767 else 4
            sw = [1 if r + 1 <= 127 else wide for r in range(len(C))]
            SC = [d[3] for d in st.detail]
            # inc_a: list entry, row_ptr pair, split, state read/write, counter
            #        (24 B) per dirty vertex; neighbour id + its state word per
            #        row entry read (rows above 512 entries: their active part)
            # inc_c: list entry, state, counter, row_ptr pair, split, colour and
            #        state writes (28 B) per committed vertex; neighbour id + its
            #        state word per later entry (nnz/2 entries per colouring)
            sw_c = sum(c * w for c, w in zip(C, sw)) / max(sum(C), 1)  # state bytes, commit-weighted
            algo = {"inc_a": sum(24 * d + (4 + w) * sc for d, sc, w in zip(D, SC, sw)),
                    "inc_c": 28 * sum(C) + (4 + sw_c) * g.nnz / 2}
        dom = max(algo, key=lambda k: kern[k]["total_ms"])  # kernels with a per-unit byte model
        launches = kern[dom]["launches"]
        achieved = (algo[dom] / max(launches, 1)) / (kern[dom]["avg_us"] * 1e-6) / 1e9
        traffic = load_traffic(args.workload, args.order, dom, launches)
        if traffic is not None:
            traffic = {"l2_fabric_bytes_per_launch": round(traffic), "algorithmic_bytes_per_launch":
                       round(algo[dom] / max(launches, 1)),
                       "GB_per_s": round(traffic / (kern[dom]["avg_us"] * 1e-6) / 1e9, 1),
                       "counted": "between L2 and the memory fabric, Infinity Cache hits included"}
        roofline = {
            "kernel": dom,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_step": {k: int(v) for k, v in algo.items()},
            "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in kern.items()},
        }
        # the method's own byte counts: the plain rounds (16 B per worklist row
        # entry, 32 B per worklist vertex) and the floor (read the CSR once,
        # write the colours), over the whole step
        b_plain = sum(16 * e + 32 * u for u, e in zip(U, E))
        b_min = 4 * g.nnz + 8 * g.n
        step_s = ms_per_step / 1e3
        whole = (load_traffic_file(args.workload, args.order) or {}).get("per_colouring")
        if whole:
            # counter bytes of every library kernel of one colouring over the
            # step time: traffic between L2 and the fabric, an upper bound of
            # the HBM share (Infinity Cache hits are counted too)
            roofline["whole_call_traffic"] = {
                "l2_fabric_bytes": int(whole["l2_fabric_bytes"]),
                "GBps": round(whole["l2_fabric_bytes"] / step_s / 1e9, 1),
                "frac_upper_bound": round(whole["l2_fabric_bytes"] / step_s / 1e9 / HBM_PEAK_GBS, 4)}
        roofline["effective"] = {
            "plain_method_bytes": int(b_plain), "plain_method_GBps": round(b_plain / step_s / 1e9, 1),
            "plain_method_frac": round(b_plain / step_s / 1e9 / HBM_PEAK_GBS, 4),
            "floor_bytes": int(b_min), "floor_GBps": round(b_min / step_s / 1e9, 1)}
        if args.engine == "incremental":
            # the gather ceiling of this graph: one byte gathered per row entry
            # through the graph's own col_idx (torch indexing of an n-byte
            # array), against the row entries k_inc_a reads per second
            st8 = torch.zeros(g.n, dtype=torch.uint8, device=dev)
            st8[ci]
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                st8[ci]
            e1.record()
            torch.cuda.synchronize()
            probe = g.nnz / (e0.elapsed_time(e1) / 5 / 1e3)
            scanned = sum(d[3] for d in st.detail)
            krate = scanned / (kern["inc_a"]["total_ms"] / 1e3)
            roofline["gather"] = {
                "kernel": "inc_a", "entries_per_s": round(krate / 1e9, 2), "probe_entries_per_s": round(probe / 1e9, 2),
                "unit": "G entries/s", "frac": round(krate / probe, 3),
                "probe": "torch indexing of an n-byte array by the graph's col_idx (one byte per row entry)"}
            del st8
        log("kernels: %s" % json.dumps(roofline["kernels"]))

    # CPU oracle on the same workload, and serial greedy for the colour count
    cpu = None
    parity = None
    greedy_colors = None
    if not args.no_cpu_baseline and args.engine == "dataflow":
        # the dataflow oracle is one ordered visit on one core
        import oracle
        t = time.perf_counter()
        ref = oracle.dataflow(g.row_ptr, g.col_idx, key)
        dt = time.perf_counter() - t
        parity = bool(np.array_equal(ref.colors, gpu_colors)) and ref.rounds == st.rounds
        greedy_colors = int(ref.colors.max())
        cpu = {"value": round(g.edges / dt, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "the full workload (%.1f s)" % dt}
        log("dataflow oracle %.1fs parity=%s rounds=%d" % (dt, parity, ref.rounds))
    elif not args.no_cpu_baseline and args.serial_tail:
        import oracle
        t = time.perf_counter()
        ref = oracle.spec_tail(g.row_ptr, g.col_idx, key, args.serial_tail)
        dt = time.perf_counter() - t
        parity = bool(np.array_equal(ref.colors, gpu_colors)) and ref.rounds == st.rounds
        greedy_colors = int(oracle.greedy(g.row_ptr, g.col_idx, key).max())
        cpu = {"value": round(g.edges / dt, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "the full workload (%.1f s)" % dt}
        log("sequential-finish oracle %.1fs parity=%s rounds=%d finished one at a time=%d"
            % (dt, parity, ref.rounds, ref.tail))
    elif not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        ref = oracle.spec_sim(g.row_ptr, g.col_idx, key, threads=0)
        dt = time.perf_counter() - t
        parity = bool(np.array_equal(ref.colors, gpu_colors))
        cpu = {"value": round(g.edges / dt, 1), "unit": "edges/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": "the full workload: every vertex and every round (%.1f s)" % dt}
        t = time.perf_counter()
        greedy_colors = int(oracle.greedy(g.row_ptr, g.col_idx, key).max())
        log("oracle %.1fs parity=%s; serial greedy %d colours (%.1fs)"
            % (dt, parity, greedy_colors, time.perf_counter() - t))

    p = WORKLOADS[args.workload][1]
    config = {"workload": "%s-%s" % (args.workload, args.order), "engine": args.engine,
              "n": g.n, "nnz": g.nnz, "edges": g.edges, "tuning": tuning}
    if args.serial_tail:
        config["serial_tail"] = args.serial_tail
    config.update({k: v for k, v in p.items()})
    res = {
        "metric": "edges colored/sec + % HBM peak at R-MAT s24; colors vs serial greedy",
        "value": round(edges_per_s, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": config,
        "colors": int(st.num_colors),
        "serial_greedy_colors": greedy_colors,
        "rounds": int(st.rounds),
        "edge_work_over_nnz": round(st.edge_work / max(g.nnz, 1), 3),
        "parity_vs_oracle": parity,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def bench_batch(args):
    """Batched workload: one step = one replay of a HIP graph holding the
    persistent batch launch over all graphs (inputs resident in HBM)."""
    import numpy as np
    import torch

    import graphgen
    import paper_1205_3809_amd as gc

    p = WORKLOADS[args.workload][1]
    t0 = time.time()
    specs = graphgen.batch_specs(p["count"], p["seed"], p["log2_lo"], p["log2_hi"])
    graphs = [graphgen.batch_graph(sp) for sp in specs]
    b = graphgen.concat(graphs)
    G, V, nnz = len(graphs), int(b.vtx_off[-1]), int(b.edge_off[-1])
    edges = nnz // 2
    log("batch of %d graphs: V=%d nnz=%d built in %.1fs" % (G, V, nnz, time.time() - t0))
    dev = torch.device("cuda:0")
    vo, eo = torch.from_numpy(b.vtx_off).to(dev), torch.from_numpy(b.edge_off).to(dev)
    rp, ci = torch.from_numpy(b.row_ptr).to(dev), torch.from_numpy(b.col_idx).to(dev)
    out = torch.empty(V, dtype=torch.int32, device=dev)
    ws = torch.empty(gc.batch_workspace_bytes(G, V, nnz), dtype=torch.uint8, device=dev)
    ticks = torch.zeros(2 * G, dtype=torch.int64, device=dev)
    rounds = torch.zeros(G, dtype=torch.int32, device=dev)
    tuning = apply_tuning(args, args.workload,
                          lambda: gc.autotune.tune_batch(vo, eo, rp, ci, V, nnz, log=log))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gc.color_graph_batch(vo, eo, rp, ci, V, nnz, None, out, ws, ticks, rounds)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gc.color_graph_batch(vo, eo, rp, ci, V, nnz, None, out, ws, ticks, rounds)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    # the replays run on the current stream; HIP events on it time the launches
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        graph.replay()
    ev1.record()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - w0) / args.steps
    kms = ev0.elapsed_time(ev1) / args.steps
    khz = gc.wall_clock_khz()
    t = ticks.cpu().numpy().reshape(-1, 2).astype(np.float64)
    service_ms = (t[:, 1] - t[:, 0]) / khz
    done_ms = (t[:, 1] - t[:, 0].min()) / khz
    rnd = rounds.cpu().numpy()
    colors = out.cpu().numpy()
    log("batch step %.3f ms; rounds max %d; service p50 %.3f p99 %.3f ms; completion p50 %.3f p99 %.3f ms"
        % (ms, rnd.max(), np.percentile(service_ms, 50), np.percentile(service_ms, 99),
           np.percentile(done_ms, 50), np.percentile(done_ms, 99)))
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(1)
        sample = rng.choice(G, 256, replace=False)
        sedges, tcpu, ok = 0, 0.0, True
        for i in sample:
            g = graphs[i]
            t1 = time.perf_counter()
            ref = oracle.spec_sim(g.row_ptr, g.col_idx)
            tcpu += time.perf_counter() - t1
            sedges += g.edges
            ok &= bool(np.array_equal(ref.colors, colors[b.vtx_off[i]:b.vtx_off[i + 1]]))
        cpu = {"value": round(sedges / tcpu, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": "256 random graphs of the batch, one core, %.1f s" % tcpu, "parity_on_sample": ok}
    bmin = 4 * nnz + 8 * V  # read every row once, write every colour
    traffic = load_traffic(args.workload, "natural", "batch", 1)
    if traffic is not None:
        traffic = {"l2_fabric_bytes_per_launch": round(traffic), "algorithmic_bytes_per_launch": bmin,
                   "GB_per_s": round(traffic / (kms / 1000.0) / 1e9, 1),
                   "counted": "between L2 and the memory fabric, Infinity Cache hits included"}
    res = {
        "metric": "edges colored/sec, batched small graphs (one persistent launch)",
        "value": round(edges / (ms / 1000.0), 1), "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "graphs": G, "vertices": V, "nnz": nnz, "edges": edges,
                   "tuning": tuning},
        "per_graph_ms": {"service_p50": round(float(np.percentile(service_ms, 50)), 4),
                         "service_p99": round(float(np.percentile(service_ms, 99)), 4),
                         "completion_p50": round(float(np.percentile(done_ms, 50)), 4),
                         "completion_p99": round(float(np.percentile(done_ms, 99)), 4)},
        "rounds_max": int(rnd.max()), "rounds_mean": round(float(rnd.mean()), 2),
        "roofline": {"kernel": "k_batch", "bound": "hbm", "achieved": round(bmin / (kms / 1000.0) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(bmin / (kms / 1000.0) / 1e9 / HBM_PEAK_GBS, 4),
                     "launch_ms_events": round(kms, 4), "traffic": traffic,
                     "bytes_model": "lower bound: 4 B per row entry + 8 B per vertex"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def bench_learned(args):
    """Learned ordering vs natural order vs exact smallest-last on the
    evaluation graph; every timed path starts from the graph resident in HBM
    and ends with the colours in HBM."""
    import numpy as np
    import torch

    import graphgen
    import paper_1205_3809_amd as gc
    from paper_1205_3809_amd import learned as L

    p = WORKLOADS[args.workload][1]
    dev = torch.device("cuda:0")
    t0 = time.time()
    train = [graphgen.rmat(p["train_scale"], p["edge_factor"], p["abcd"][:3], s) for s in range(p["train_graphs"])]
    log("%d training graphs built in %.1fs" % (len(train), time.time() - t0))
    model = L.MLP(seed=0)
    t0 = time.time()
    rep = L.train(model, [(g.row_ptr, g.col_idx) for g in train], epochs=p["epochs"], batch=p["batch"], lr=2e-3,
                  log=log)
    train_s = time.time() - t0
    del train
    ev = graphgen.rmat(p["eval_scale"], p["edge_factor"], p["abcd"][:3], p["eval_seed"])
    log("eval graph n=%d nnz=%d" % (ev.n, ev.nnz))
    rp = torch.from_numpy(ev.row_ptr).to(dev)
    ci = torch.from_numpy(ev.col_idx).to(dev)
    out = torch.empty(ev.n, dtype=torch.int32, device=dev)
    # launch parameters for colouring the evaluation graph, searched with the
    # trained model's keys (the order whose end-to-end time is the metric)
    tuning = apply_tuning(args, "%s-eval" % args.workload,
                          lambda: gc.autotune.tune_single(rp, ci, L.order_learned(model, rp, ci)[0], log=log))

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        w = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - w) * 1000.0 / reps, r

    def natural():
        return gc.color_graph_ex(rp, ci, None, out, stats=True)[1].num_colors

    def learned():
        keys, _ = L.order_learned(model, rp, ci)
        return gc.color_graph_ex(rp, ci, keys, out, stats=True)[1].num_colors

    def learned_fb():
        return L.color_learned(model, rp, ci, fallback=True)

    def ordering_only():
        return L.order_learned(model, rp, ci)[0]

    def learned_flow():
        keys, _ = L.order_learned(model, rp, ci)
        return gc.color_graph_ex(rp, ci, keys, out, flags=gc.FLAG_DATAFLOW, stats=True)[1]

    reps = max(1, args.steps)
    t_nat, c_nat = timed(natural, reps)
    t_order, _ = timed(ordering_only, reps)
    t_learn, c_learn = timed(learned, reps)
    t_fb, fb = timed(learned_fb, reps)
    # the dataflow engine with the same learned keys: the serial greedy's
    # colouring in the learned order
    t_lflow, st_lflow = timed(learned_flow, reps)
    # exact smallest-last: the library's host routine (the order is a
    # sequential peel), keys to the device, same colouring
    w = time.perf_counter()
    rank, degen = L.smallest_last_rank(ev.row_ptr, ev.col_idx)
    t_sl_order = (time.perf_counter() - w) * 1000.0
    slk = torch.from_numpy(rank.astype(np.int32)).to(dev)
    # the same order on the device (one workgroup walks the removals)
    t_sl_gpu, (gpu_rank, gpu_degen) = timed(lambda: gc.smallest_last(rp, ci), 1)
    sl_gpu_equal = bool(torch.equal(gpu_rank, slk)) and gpu_degen == degen
    log("device smallest-last %.1f ms, equal to the host order: %s" % (t_sl_gpu, sl_gpu_equal))
    t_sl_col, c_sl = timed(lambda: gc.color_graph_ex(rp, ci, slk, out, stats=True)[1].num_colors, reps)
    t_sl_flow, st_sl_flow = timed(lambda: gc.color_graph_ex(rp, ci, slk, out, flags=gc.FLAG_DATAFLOW,
                                                            stats=True)[1], reps)
    # reference order: largest degree first (ties by id), keys built here on
    # the host; the colouring is timed alone
    deg = np.diff(ev.row_ptr.astype(np.int64))
    lf_order = np.lexsort((np.arange(ev.n), -deg))
    lf_key = np.empty(ev.n, dtype=np.int32)
    lf_key[lf_order] = np.arange(ev.n, dtype=np.int32)
    lfk = torch.from_numpy(lf_key).to(dev)
    t_lf_col, c_lf = timed(lambda: gc.color_graph_ex(rp, ci, lfk, out, stats=True)[1].num_colors, reps)
    res = {
        "metric": "learned ordering: colours and end-to-end ms vs natural order and exact smallest-last",
        "value": round(t_learn, 3), "unit": "ms", "higher_is_better": False, "n_gpus": 1, "steps": reps,
        "dtype": "int32 colouring; bf16 weights, fp32 accumulation", "data": "synthetic",
        "config": {"workload": args.workload, "eval_n": ev.n, "eval_nnz": ev.nnz, **{k: v for k, v in p.items()},
                   "tuning": tuning},
        "colours": {"natural": c_nat, "learned": c_learn, "learned_with_fallback": int(min(fb[2], fb[3])),
                    "exact_smallest_last": c_sl, "degeneracy_plus_1": degen + 1,
                    "largest_degree_first": c_lf,
                    "learned_dataflow": int(st_lflow.num_colors),
                    "exact_smallest_last_dataflow": int(st_sl_flow.num_colors)},
        "ms": {"natural": round(t_nat, 3), "learned": round(t_learn, 3), "learned_with_fallback": round(t_fb, 3),
               "learned_ordering_only": round(t_order, 3),
               "largest_degree_first_colouring": round(t_lf_col, 3),
               "learned_dataflow": round(t_lflow, 3),
               "exact_smallest_last_order_host": round(t_sl_order, 1),
               "exact_smallest_last_total": round(t_sl_order + t_sl_col, 1),
               "exact_smallest_last_order_gpu": round(t_sl_gpu, 1),
               "exact_smallest_last_total_gpu": round(t_sl_gpu + t_sl_col, 1),
               "exact_smallest_last_dataflow_colouring": round(t_sl_flow, 3)},
        "dataflow_rounds": {"learned": int(st_lflow.rounds), "exact_smallest_last": int(st_sl_flow.rounds)},
        "smallest_last_gpu_equals_host": sl_gpu_equal,
        "training": {"seconds": round(train_s, 2), "vertices": rep.vertices, "final_minibatch_loss":
                     round(rep.losses[-1], 6)},
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
