"""bench.py's command-line contract on the CPU: more than one GPU is refused with a
message, and the stage-kernel source hash, printed on request, gates the committed
traffic counters."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_source_hash_gates_the_committed_counters(tmp_path, monkeypatch):
    """--source-hash prints the 16-hex-digit hash of the stage-kernel sources; the committed
    FETCH/WRITE counters are used for roofline.traffic only while their recorded hash, workload
    and grid equal the current ones (otherwise traffic is reported as null)."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--source-hash"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 0
    h = r.stdout.strip()
    assert len(h) == 16 and all(ch in "0123456789abcdef" for ch in h)
    sys.path.insert(0, ROOT)
    import bench
    assert bench.stage_source_hash() == h
    body = ("source_hash: {h}\nconfig: lds:16x4x4:blocked\npoints: 4096\nfetch_kib_per_dispatch: 100\n"
            "write_kib_per_dispatch: 50\nfetch_scale: 2.0\nwrite_scale: 1.0\nfp64_flop_per_point: 4789\n")
    f = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    f.write_text(body.format(h=h))
    assert bench.measured_traffic("lds:16x4x4:blocked", 4096) == (100 * 2.0 + 50) * 1024
    assert bench.measured_counters("lds:16x4x4:blocked", 4096) == ((100 * 2.0 + 50) * 1024, 4789.0)
    assert bench.measured_traffic("lds:16x4x4:blocked", 8192) is None  # another grid
    assert bench.measured_traffic("lds:16x8x2:blocked", 4096) is None  # another configuration
    f.write_text(body.format(h="0" * 16))
    assert bench.measured_traffic("lds:16x4x4:blocked", 4096) is None  # counters of other sources
    assert bench.measured_counters("lds:16x4x4:blocked", 4096) == (None, None)
