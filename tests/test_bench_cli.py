"""bench.py's command line on the CPU: more than one GPU is refused with a
message and exit status 2 before anything touches a device; the workload's
algorithmic bytes per launch are the stated 6.4508 GB."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_of_the_bench_workload():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1005_2314_amd import inputs
    out_b, state_b = bench.workload_bytes(inputs.batched_f32(), 4)
    # 2^30 binary32 outputs; each of 65536 streams reads and writes its pool of
    # 4096 binary32 values and its 64-byte header
    assert out_b == 4 * 2**30
    assert state_b == 65536 * 2 * (4096 * 4 + 64)
    assert out_b + state_b == 6450839552


def test_traffic_is_reported_only_for_the_profiled_sources(monkeypatch, tmp_path):
    # the committed HBM-traffic profile matches the kernel sources as they are;
    # a changed source makes the bench report no traffic rather than a stale one
    sys.path.insert(0, ROOT)
    import bench
    t = bench.measured_traffic()
    assert t is not None and abs(t / 6450839552 - 1) < 0.01
    changed = tmp_path / "wn_device.hpp"
    changed.write_bytes(open(bench.FILL_SOURCES[0], "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(bench, "FILL_SOURCES", [str(changed)] + bench.FILL_SOURCES[1:])
    assert bench.measured_traffic() is None
