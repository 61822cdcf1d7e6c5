"""Host logic of bench.py (no GPU): a multi-GPU request exits with a message,
and measured HBM traffic is reported only while the hashed kernel sources
match the ones the counters were taken with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_traffic_only_for_matching_sources(tmp_path):
    import bench
    good = tmp_path / "good.md"
    good.write_text(f"- round_bytes: `123`\n- source_hash: `{bench.kernel_source_hash()}`\n")
    stale = tmp_path / "stale.md"
    stale.write_text("- round_bytes: `123`\n- source_hash: `0000000000000000`\n")
    assert bench.measured_traffic(str(good), "round_bytes") == 123
    assert bench.measured_traffic(str(stale), "round_bytes") is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), "round_bytes") is None
