"""CPU checks of bench.py's command-line contract that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_records_match_their_sources():
    """The committed HBM traffic summaries are the ones bench.py reports:
    each names the hash of the kernel sources it was measured on."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.measured_traffic("plain-large") is not None
    rec = bench.traffic_record(bench.TM_TRAFFIC_FILE, bench.TM_SOURCES)
    assert rec is not None and int(rec["fetch_bytes_per_product"]) > 0
