"""Host-side checks of the benchmark script: the one-GPU contract and the
kernel-source hash that keys the stored PMC traffic figures (no GPU)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_stored_traffic_figures_cover_the_cgs_classes():
    """The PMC summary carries every class that can be the dominant one, with
    traffic close to the algorithmic bytes (the passes read the basis once)."""
    tr = json.load(open(os.path.join(ROOT, "profiles", "traffic_workload2.json")))
    assert set(tr["kernels"]) >= {"cgs_proj", "cgs_updproj", "cgs_updnorm"}
    assert 1.9 < tr["fetch_scale"] < 2.1 and abs(tr["write_scale"] - 1.0) < 0.05
    for cls, d in tr["kernels"].items():
        assert 0.9 < d["traffic_over_alg"] < 1.2, (cls, d)
        assert d["bytes_per_launch"] == d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"] or \
            abs(d["bytes_per_launch"] - d["fetch_bytes_per_launch"] - d["write_bytes_per_launch"]) <= 2


def test_kernel_source_hash_is_stable_and_keys_the_stored_figures():
    """bench.py reports the stored traffic only for the kernel sources it was
    measured on (null otherwise)."""
    import pytest
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 16
    tr = json.load(open(os.path.join(ROOT, "profiles", "traffic_workload2.json")))
    if tr["source_hash"] != h:
        pytest.skip("stored PMC traffic figures predate the current kernel sources (bench reports null)")
