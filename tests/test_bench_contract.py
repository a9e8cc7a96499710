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


def test_traffic_records_are_used_only_for_their_sources():
    """Each committed HBM traffic summary names the hash of the kernel
    sources it was measured on; bench.py reports its bytes only while the
    sources still hash to that value (null once a kernel has changed)."""
    sys.path.insert(0, ROOT)
    import bench
    for path, sources in bench.TRAFFIC_RECORDS:
        if not os.path.exists(path):
            continue
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        assert len(fields.get("kernel_source_sha256", "")) == 64, path
        rec = bench.traffic_record(path, sources)
        current = fields["kernel_source_sha256"] == bench.kernel_source_hash(sources)
        assert (rec is not None) == current, path
        if rec is not None:
            assert all(int(rec[k]) > 0 for k in rec if k.endswith("_bytes_per_launch")
                       or k.endswith("_bytes_per_product")), path
