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


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, grid, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": value})


def test_derive_traffic_scales_by_the_copy_and_averages_per_launch(tmp_path):
    """The 1 GiB calibration copy reads 1 GiB and writes 1 GiB; a counter
    that reports half of it for the read is scaled by 2.  Per-kernel figures
    are per launch; the per-colouring figure sums every library kernel and
    divides by the colourings (k_zero_ctl launches)."""
    a = "void (anonymous namespace)::k_inc_a<signed char>((anonymous namespace)::Args, int)"
    c = "void (anonymous namespace)::k_inc_c<signed char>((anonymous namespace)::Args, int)"
    z = "(anonymous namespace)::k_zero_ctl((anonymous namespace)::Ctl*)"
    seed = "void (anonymous namespace)::k_inc_seed<signed char>((anonymous namespace)::Args, int)"
    copy = "__amd_rocclr_copyBuffer"
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    # KiB values; the copy's FETCH_SIZE reads half its true 1 GiB
    write_csv(fetch, "FETCH_SIZE", [(copy, 131072, 524288), (z, 1, 0), (seed, 4096, 1000), (a, 4096, 100),
                                    (a, 4096, 300), (c, 4096, 50), (z, 1, 0), (seed, 4096, 1000), (a, 4096, 200),
                                    (c, 4096, 150), (copy, 64, 7)])
    write_csv(write, "WRITE_SIZE", [(copy, 131072, 1048576), (z, 1, 0), (seed, 4096, 10), (a, 4096, 30),
                                    (a, 4096, 30), (c, 4096, 20), (z, 1, 0), (seed, 4096, 10), (a, 4096, 30),
                                    (c, 4096, 40), (copy, 64, 7)])
    out = bench.derive_traffic(str(fetch), str(write), "w", "o", None, out_path=str(tmp_path / "t.json"))
    assert abs(out["scale"]["FETCH_SIZE"] - 2.0) < 1e-12 and abs(out["scale"]["WRITE_SIZE"] - 1.0) < 1e-12
    ka, kc = out["kernels"]["inc_a"], out["kernels"]["inc_c"]
    assert ka["launches_counted"] == 3 and kc["launches_counted"] == 2
    assert abs(ka["read_bytes_per_launch"] - 200 * 1024 * 2) < 1e-6      # (100+300+200)/3 KiB, x2
    assert abs(ka["write_bytes_per_launch"] - 30 * 1024) < 1e-6
    assert abs(kc["hbm_bytes_per_launch"] - (100 * 1024 * 2 + 30 * 1024)) < 1e-6
    pc = out["per_colouring"]
    assert pc["colourings_counted"] == 2
    # every library kernel (seed, inc_a, inc_c, zero_ctl) of both colourings, halved; copies excluded
    assert abs(pc["read_bytes"] - (2000 + 600 + 200) / 2 * 1024 * 2) < 1e-6
    assert abs(pc["write_bytes"] - (20 + 90 + 60) / 2 * 1024) < 1e-6


def test_binding_flags_match_the_header():
    import paper_1205_3809_amd as gc
    text = open(os.path.join(ROOT, "include", "gcolor.h")).read()
    for name, value in (("GCOLOR_VALIDATE", gc.FLAG_VALIDATE), ("GCOLOR_STATS", gc.FLAG_STATS),
                        ("GCOLOR_PLAIN", gc.FLAG_PLAIN), ("GCOLOR_DATAFLOW", gc.FLAG_DATAFLOW)):
        m = re.search(r"\b%s\s*=\s*1u\s*<<\s*(\d+)" % name, text)
        assert m, name
        assert value == 1 << int(m.group(1)), name


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
