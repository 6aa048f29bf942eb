"""The benchmark script's host-side contract (no GPU): it refuses more than
one GPU with a JSON message, its roofline arithmetic follows the stage
records, and the committed HBM-traffic records name the kernels it reports."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_roofline_from_stage_records():
    import bench
    prof = {"toeapply32": {"ms": 6.0, "count": 3, "bytes": 3 * 160e6}}
    r = bench.roofline(prof, "toeapply32")
    assert abs(r["avg_launch_us"] - 2000.0) < 1e-9
    assert abs(r["bytes_per_launch"] - 160e6) < 1e-3
    assert abs(r["achieved"] - 160e6 / 2e-3 / 1e9) < 1e-9   # GB/s
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12


def test_traffic_records_match_reported_kernels():
    """Every committed traffic record names the kernel the benchmark reports
    for its stage (a stage without a record reports traffic null)."""
    import bench
    for stage, (kernel, src) in bench.ROOFLINE_KERNELS.items():
        assert os.path.exists(os.path.join(ROOT, "paper_1004_5076_amd", "csrc", src))
        p = os.path.join(ROOT, "profiles", "traffic_%s_two_channel.json" % stage)
        if not os.path.exists(p):
            assert bench.measured_ratio(stage) is None
            continue
        d = json.load(open(p))
        assert d["kernel"] == kernel
        assert d["ratio"] > 0.9          # measured bytes cannot fall far below the algorithmic ones
        assert os.path.exists(os.path.join(ROOT, "paper_1004_5076_amd", "csrc", src))
