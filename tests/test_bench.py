"""Host-side checks of bench.py's contract (no GPU): the flag for more than one
GPU is refused with a message, and the HBM traffic it reports is tied to the
current text of the FP32 pair kernel."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pair_kernel_hash_finds_the_kernel_text():
    h = bench.pair_kernel_hash()
    assert h is not None and len(h) == 16


def test_traffic_is_reported_only_for_the_profiled_kernel_text():
    for name in ("p2p_f32_uniform_cube_N100k_hbm_counters.json", "p2p_f32_clustered_N1M_hbm_counters.json"):
        path = os.path.join(ROOT, "profiles", name)
        t = bench.measured_traffic("fp32", name)
        if not os.path.exists(path):
            assert t is None
            continue
        rec = json.load(open(path))
        if rec["source_sha256_16"] == bench.pair_kernel_hash():
            assert t == rec["traffic_bytes"]
        else:
            assert t is None
        assert bench.measured_traffic("fp64", name) is None
