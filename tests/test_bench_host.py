"""Host logic of bench.py (no GPU): a multi-GPU request exits with a message,
the roofline is taken for the phase whose single kernel takes the longest,
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


def test_dominant_phase_by_single_kernel_time():
    import bench
    # per-kernel times of an R-MAT 26 round: the hub path is the longest as a
    # path (27.8 ms) but its longest kernel (11.7 ms) is shorter than the
    # small tiles' one
    phases = {"lane": 2.09, "tile": 20.5, "block": 8.49, "hub": 27.8, "accept": 3.98}
    hubs = {"hub_whole": 11.7, "hub_pieces": 8.4, "hub_reduce": 7.6}
    assert bench.dominant_phase(phases, hubs) == "tile"
    # one hub kernel longer than every tile kernel: the hub path is reported
    assert bench.dominant_phase(phases, dict(hubs, hub_reduce=25.0)) == "hub"
    # acceptance is never the dominant kernel, and hub kernels without a hub
    # phase are ignored
    assert bench.dominant_phase({"lane": 1.0, "accept": 9.0}, {"hub_whole": 5.0}) == "lane"
    assert bench.dominant_phase({"accept": 9.0}, {}) is None
