"""Host-side checks of bench.py (no GPU): the single-GPU contract and the keying of the
committed HBM counter records on the kernel source, the device header and the capacity."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_records_are_used_only_for_their_sources_and_capacity():
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
        rec = json.load(f)
    assert {"elem_kernel", "factor_kernel", "subst_kernel"} <= set(rec)
    for k, v in rec.items():
        cap = v["contact_capacity"]
        current = bench.traffic_key(k, cap) == v["key_sha256"]
        assert bench.measured_traffic(k, cap) == (v["bytes_per_launch"] if current else None)
        assert bench.measured_traffic(k, cap + 1) is None
        assert bench.traffic_key(k, cap) != bench.traffic_key(k, 2 * cap)
        assert v["bytes_per_launch"] > 0 and v["fetch_scale"] > 0 and v["write_scale"] > 0
