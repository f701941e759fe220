"""The benchmark's contract on the CPU: it refuses more than one GPU, and
the committed rocprofv3 traffic figures belong to the current fit kernels
(their source hash matches), so the headline line carries measured bytes."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stdout + r.stderr


def test_traffic_figures_match_the_kernel_sources():
    import json

    import bench
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert t["source_sha"] == bench.kernel_sources_sha()
    launch = {"block": 128, "waves_per_simd": 3, "tracks_per_lane": 1, "persistent": False}
    for ts, tc in (("float", "double"), ("float", "float")):
        name = bench.fit_kernel_name(ts, "float", tc, launch)
        assert name in t["kernels"]
        assert bench.measured_traffic(name) > 0
    assert bench.measured_traffic("fit_layer_kernel<float, float, 256, false>") > 0
