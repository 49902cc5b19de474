"""Host-side pieces of the benchmark: the counter-to-bytes derivation that
fills the roofline's traffic figures, the flag values the binding passes
through the C ABI, and the refusal of multi-GPU runs.  CPU only."""
import csv
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, grid, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": value})


def test_derive_traffic_sums_request_sizes_per_launch(tmp_path):
    """Read bytes are 32, 64 and 128 bytes per request of each size, write
    bytes 64 per 64-byte request and 32 per other request; per-kernel figures
    are per launch; the per-colouring figure sums every library kernel and
    divides by the colourings (k_zero_ctl launches); the calibration copy is
    reported apart (here 2^23 requests of 128 bytes: exactly 1 GiB)."""
    a = "void (anonymous namespace)::k_inc_a<signed char>((anonymous namespace)::Args, int)"
    c = "void (anonymous namespace)::k_inc_c<signed char>((anonymous namespace)::Args, int)"
    z = "(anonymous namespace)::k_zero_ctl((anonymous namespace)::Ctl*)"
    copy = "__amd_rocclr_copyBuffer"
    R32, R64, R128, RQ = bench.TRAFFIC_PASSES[0]
    W64, WQ, BUB = bench.TRAFFIC_PASSES[1]
    HIT, MISS = bench.TRAFFIC_PASSES[2]
    rows_r, rows_w, rows_h = [], [], []
    for rep in range(2):  # two colourings
        rows_r += [(z, 1, R32, 0), (z, 1, R64, 0), (z, 1, R128, 0), (z, 1, RQ, 0)]
        for kern, r32, r64, r128 in ((a, 10, 20, 5), (a, 30, 0, 15), (c, 4, 4, 4)):
            rows_r += [(kern, 4096, R32, r32), (kern, 4096, R64, r64), (kern, 4096, R128, r128),
                       (kern, 4096, RQ, r32 + r64 + r128)]
        rows_w += [(z, 1, W64, 0), (z, 1, WQ, 0), (z, 1, BUB, 0)]
        for kern, w64, wq in ((a, 3, 5), (a, 1, 1), (c, 2, 2)):
            rows_w += [(kern, 4096, W64, w64), (kern, 4096, WQ, wq), (kern, 4096, BUB, 0)]
        rows_h += [(z, 1, HIT, 0), (z, 1, MISS, 0), (a, 4096, HIT, 3), (a, 4096, MISS, 1), (a, 4096, HIT, 3),
                   (a, 4096, MISS, 1), (c, 4096, HIT, 1), (c, 4096, MISS, 1)]
    rows_r += [(copy, 131072, R32, 0), (copy, 131072, R64, 0), (copy, 131072, R128, 1 << 23),
               (copy, 131072, RQ, 1 << 23)]
    rows_w += [(copy, 131072, W64, 1 << 24), (copy, 131072, WQ, 1 << 24), (copy, 131072, BUB, 1 << 23)]
    paths = []
    for name, rows in (("r", rows_r), ("w", rows_w), ("h", rows_h)):
        paths.append(str(tmp_path / (name + ".csv")))
        write_csv(paths[-1], rows)
    out = bench.derive_traffic(paths, "w", "o", out_path=str(tmp_path / "t.json"))
    ka, kc = out["kernels"]["inc_a"], out["kernels"]["inc_c"]
    assert ka["launches_counted"] == 4 and kc["launches_counted"] == 2
    # inc_a: requests (10, 20, 5) and (30, 0, 15), averaged per launch
    assert abs(ka["read_bytes_per_launch"] - (32 * 20 + 64 * 10 + 128 * 10)) < 1e-9
    # writes (64 x 3 + 32 x 2) and (64 x 1), averaged
    assert abs(ka["write_bytes_per_launch"] - (192 + 64 + 64) / 2) < 1e-9
    assert abs(kc["l2_fabric_bytes_per_launch"] - (4 * (32 + 64 + 128) + 2 * 64)) < 1e-9
    assert abs(ka["l2_hit_rate"] - 0.75) < 1e-12 and abs(kc["l2_hit_rate"] - 0.5) < 1e-12
    pc = out["per_colouring"]
    assert pc["colourings_counted"] == 2
    per_col_read = (32 * 40 + 64 * 20 + 128 * 20) + 4 * (32 + 64 + 128)
    assert abs(pc["read_bytes"] - per_col_read) < 1e-9
    assert out["copy_check"]["read_bytes"] == 1 << 30 and out["copy_check"]["write_bytes"] == 1 << 30
    assert out["copy_check"]["fetch_size_formula_bytes"] == 1 << 30


def test_binding_flags_match_the_header():
    import paper_1205_3809_amd as gc
    text = open(os.path.join(ROOT, "include", "gcolor.h")).read()
    for name, value in (("GCOLOR_VALIDATE", gc.FLAG_VALIDATE), ("GCOLOR_STATS", gc.FLAG_STATS),
                        ("GCOLOR_PLAIN", gc.FLAG_PLAIN), ("GCOLOR_DATAFLOW", gc.FLAG_DATAFLOW),
                        ("GCOLOR_SERIAL_TAIL", gc.FLAG_SERIAL_TAIL)):
        m = re.search(r"\b%s\s*=\s*1u\s*<<\s*(\d+)" % name, text)
        assert m, name
        assert value == 1 << int(m.group(1)), name


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
