"""The benchmark's host-side pieces, without a GPU: the refusal of more
than one GPU, the kernel naming that ties the live roofline to the committed
counter summary, and the algorithmic byte and flop counts of the headline
workload."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_counts_of_the_headline_workload():
    N, Ms = 512 * 512, 512
    # per node 2 offsets + cell word + weight + sample (float32), plus the grid
    assert bench.spread_algorithmic_bytes(N, Ms, 2, "f32") == N * 28 + Ms * Ms * 8 == 9437184
    assert bench.spread_flops(N, 6, 2) == 4 * 144 * N == 150994944


def test_kernel_names_follow_the_tuning():
    t = {"tile_edge": 16, "spread_mode": 3, "spread_threads": 256, "spread_planes": 2}
    assert bench.spread_kernel_name(t) == "spread_group_kernel<float, 2, 6, 256, 16, true, 1>"
    assert bench.spread_kernel_name(dict(t, spread_mode=4, spread_planes=1)) == \
        "spread_group_kernel<float, 2, 6, 256, 16, false, 2>"
    assert bench.spread_kernel_name(dict(t, spread_mode=1, tile_edge=32)) == \
        "spread_group_kernel<float, 2, 6, 256, 0, true, 0>"
    assert bench.spread_kernel_name(dict(t, spread_mode=2)) == "spread_rows_kernel<float, 6, 16, 1>"
    assert bench.spread_kernel_name(dict(t, spread_mode=5)) == "spread_reg_kernel<6, 4>"
    assert bench.spread_kernel_name(dict(t, spread_mode=7)) == "spread_mma_kernel<float, 6, 4>"
    assert bench.spread_kernel_name(dict(t, spread_mode=5, spread_threads=512)) == \
        "spread_reg_kernel<6, 8>"


def test_traffic_record_is_tied_to_the_sources():
    """The counter summary under profiles/ is reported as the kernel's HBM
    traffic only while the spreading sources are the ones it was taken on
    (sha256 recorded with it) and the kernel name matches."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "spread_traffic_polar512.json")))
    kernel = rec["kernel"].replace("nfft::", "")
    if rec["source_sha256"] == bench.spread_source_sha():
        assert bench.traffic_record(kernel) == rec["bytes_per_launch"] > 0
    else:
        assert bench.traffic_record(kernel) is None
    assert bench.traffic_record(kernel + "x") is None
