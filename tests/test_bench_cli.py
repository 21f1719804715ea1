"""bench.py's command-line contract on the CPU: more than one GPU is refused with a
message, and the stage-kernel source hash (which gates the committed traffic counters)
is printed on request."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_source_hash_matches_the_counter_file_format():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--source-hash"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 0
    h = r.stdout.strip()
    assert len(h) == 16 and all(ch in "0123456789abcdef" for ch in h)
    with open(os.path.join(ROOT, "profiles", "k_bssn_stage_lds_256cubed_traffic.txt")) as f:
        assert f"source_hash: {h}" in f.read(), "the committed counters are for other stage-kernel sources"
