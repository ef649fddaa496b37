"""CPU checks of the benchmark driver's contract: more than one GPU is refused
with a message, and the roofline helpers read the committed profiles only
when they were taken on the current kernel source."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_traffic_matches_the_current_kernel_source():
    """The committed counter summary names the benchmarked kernel and its
    source hash; traffic is reported for that kernel and withheld for any
    other."""
    with open(os.path.join(ROOT, "profiles", "step_kernel_L1x64_pmc.json")) as fh:
        d = json.load(fh)
    kernel = d["kernel"].removeprefix("pdmi::")
    assert kernel in bench.SHAPE_KERNELS
    if d["kernel_source_hash"] == bench.kernel_source_hash():
        t = bench.traffic_from_profiles(kernel)
        assert t == d["hbm_bytes_per_launch"] and t > 0
    other = [k for k in bench.SHAPE_KERNELS if k != kernel][0]
    assert bench.traffic_from_profiles(other) is None


def test_roofline_constants():
    """HBM bound at the chip's 8 TB/s with 7.8 algorithmic bytes per unique
    bond-update; the FP32 vector rate (256 CUs x 4 SIMDs x 32 lanes x FMA x
    2.4 GHz) is kept as a labelled extra."""
    assert bench.PEAK_HBM_GBPS == 8000.0
    assert bench.ALG_BYTES_PER_BOND_UPDATE_F32 == 7.8
    assert abs(bench.PEAK_TFLOPS_F32 - 157.2864) < 1e-9


def test_bench_line_is_strict_json():
    """Non-finite values (a rounding-negative variance's root, an empty
    maximum) become null, so the line parses as strict JSON."""
    import json
    import math
    import bench
    line = {"a": float("nan"), "b": [1.0, float("inf"), {"c": -float("inf")}], "d": 2, "e": "x", "f": (3.0,)}
    out = json.dumps(bench.finite_json(line), allow_nan=False)
    assert json.loads(out) == {"a": None, "b": [1.0, None, {"c": None}], "d": 2, "e": "x", "f": [3.0]}
    assert math.isfinite(bench.finite_json(1.5))
