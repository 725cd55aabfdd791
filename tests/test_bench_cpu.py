"""Host-side checks of bench.py that need no GPU: the one-GPU refusal and the
roofline bookkeeping (algorithmic bytes, the counter-calibration record)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_traffic_record_is_tied_to_the_kernel_sources():
    """the committed counter record names the source hash it was taken on;
    bench.py reports its bytes only while that hash is the current one"""
    with open(os.path.join(ROOT, "profiles", "k_stage_traffic.json")) as f:
        rec = json.load(f)["disc512_p4_fp64"]
    assert rec["hbm_bytes_per_launch"] > 0
    # FETCH_SIZE prices 128-byte read requests as 64 bytes, and the request
    # counters see 5/6 of a plain copy's reads: the copy-calibrated factor is
    # about 2.4 for reads and 1 for writes.  The read bytes from FETCH_SIZE and
    # from the request-size counters, each calibrated on the copy, must agree.
    assert 1.0 < rec["fetch_factor"] < 3.0 and 0.9 < rec["write_factor"] < 1.1
    assert abs(rec["direct_read_bytes_per_launch"] / rec["read_bytes_per_launch"] - 1) < 0.01
    assert rec["hbm_bytes_per_launch"] == rec["read_bytes_per_launch"] + rec["written_bytes_per_launch"]
    cur = bench.kernel_source_hash()
    got = bench.measured_traffic("disc512_p4_fp64")
    assert got == (rec["hbm_bytes_per_launch"] if rec["kernel_source_sha256_16"] == cur else None)


def test_count_model_is_positive_and_grows_with_order():
    f = [bench.flop_per_element_stage(n, 3) for n in (2, 3, 4, 5)]
    assert all(a < b for a, b in zip(f, f[1:]))
    # the sum-factorised volume part dominates at order 5: 2 (7 n^3 nvar - n^3) FLOP
    assert f[-1] > 2 * (7 * 125 * 3 - 125)


def test_one_thread_oracle_child_reports_a_rate():
    """the single-thread oracle timing runs as a child process (OMP_NUM_THREADS=1)
    and prints one JSON line with its DOF-stage rate"""
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-child", "8", "3", "1"],
                       capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["value"] > 0 and rec["seconds"] > 0
