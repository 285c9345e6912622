"""Host checks of the benchmark script's contract (no GPU)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_record_is_tied_to_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2608_29082_amd import pmc_summary as P
    assert bench.kernel_sources_sha256() == P.kernel_sources_sha256()
    with open(os.path.join(ROOT, "profiles", bench.TRAFFIC_FILES[("conv", 0)])) as fh:
        rec = json.load(fh)
    got = bench.counter_traffic("conv", 0)
    if rec["kernel_sources_sha256"] == bench.kernel_sources_sha256():
        assert got == rec["bytes_per_dispatch"]
    else:
        assert got is None          # stale counters are never reported
    assert bench.counter_traffic("hop", 3) is None
