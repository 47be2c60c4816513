"""Host checks of the benchmark's command-line contract (no GPU): more than one GPU is
refused before anything touches a device, and the committed ray-sampling counter summary
parses into the fields the benchmark reads from it."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_summary_has_the_fields_the_benchmark_reads():
    sys.path.insert(0, ROOT)
    import bench
    fields = {}
    for line in open(bench.TRAFFIC_FILE):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    assert int(fields["traffic_bytes_per_launch"]) > 0
    assert len(fields["source_sha256"]) == 64
    csrc = os.path.join(ROOT, "paper_2210_06160_amd", "csrc")
    assert all(os.path.exists(os.path.join(csrc, f)) for f in bench.TRAFFIC_SOURCES)
