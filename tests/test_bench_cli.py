"""Command-line contract of bench.py that needs no GPU."""
import json
import os
import subprocess
import sys

from conftest import ROOT


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2",
                        "--steps", "1", "--warmup", "0"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_matches_its_source():
    """The committed HBM-counter record names the kernel source it was taken from; the
    benchmark reports its traffic only while that source is unchanged."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert os.path.exists(os.path.join(ROOT, rec["source"]))
    assert os.path.exists(os.path.join(ROOT, rec["summary"]))
    cal = rec["calibration"]
    assert cal["fetch_scale"] == 2.0 and cal["write_scale"] == 0.999
    sys.path.insert(0, ROOT)
    import hashlib
    import bench
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    same = hashlib.sha256(src).hexdigest()[:16] == rec["source_sha256_prefix"]
    assert rec["kernels"]
    for name, k in rec["kernels"].items():
        # the calibrated bytes are the counters times the copy-probe factors
        want = (k["fetch_kib"] * cal["fetch_scale"] + k["write_kib"] * cal["write_scale"]) * 1024
        assert abs(k["hbm_bytes_per_launch"] - want) <= 1e5
        assert bench.measured_traffic(name) == (k["hbm_bytes_per_launch"] if same else None)
    assert bench.measured_traffic("k_not_a_kernel") is None
