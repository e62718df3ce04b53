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


def test_algorithmic_bytes_per_sweep():
    """The roofline's algorithmic bytes: joint FP64 sweep 40 B per slot (incoming Lt and m,
    coefficient, outgoing Lt and m) plus the reverse index, 16 B per row (diagonal, b);
    mean-only FP64 24 B + reverse per slot, 8 B per row; FP32 12 B + reverse, 4 B per row.
    At the 2048^2 benchmark operator (16,769,024 directed slots, 4,194,304 rows) a joint
    pass is 804,945,920 B with 4-byte reverse indices (the tiled launch) and 771,407,872 B
    with 2-byte deltas (the one-sweep kernel)."""
    sys.path.insert(0, ROOT)
    import bench
    slots, n = 16769024, 4194304
    assert bench.sweep_bytes_joint64(slots, n, 4) == 804945920
    assert bench.sweep_bytes_joint64(slots, n, 2) == 771407872
    assert bench.sweep_bytes_mean64(1, 0, 2) == 26 and bench.sweep_bytes_mean64(0, 1) == 8
    assert bench.sweep_bytes_mean32(1, 0, 2) == 14 and bench.sweep_bytes_mean32(0, 1) == 4
    # the fraction the benchmark line reports: one pass per launch over the launch's time
    t_launch = 162.83e-6
    frac = bench.sweep_bytes_joint64(slots, n, 4) / t_launch / 1e9 / bench.HBM_PEAK_GBS
    assert abs(frac - 0.618) < 1e-3 and bench.HBM_PEAK_GBS == 8000.0
