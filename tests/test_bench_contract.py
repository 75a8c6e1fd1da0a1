"""Host-side pieces of bench.py: graph length, algorithmic byte counts, the
one-GPU guard, and the traffic record lookup (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("steps,g", [(1500, 15), (1000, 10), (16, 16), (17, 1), (1, 1), (48, 16), (20, 10)])
def test_graph_len_divides_the_timed_steps(steps, g):
    assert bench.graph_len(steps) == g
    assert steps % bench.graph_len(steps) == 0


def test_byte_counts_follow_the_per_agent_budget():
    n = 4096
    # step: state read 76 + 8 + 16, state write 76 + 8, actions 8, outputs 6
    assert bench.STEP_BYTES_PER_AGENT == 198
    assert bench.step_bytes(n) == 198 * n
    assert bench.step_bytes(n, road=12345.0) == 198 * n + 12345.0
    # observation: the 1 KB row, plus the network and the actions when fused
    assert bench.obs_bytes(n, False) == 1024 * n
    assert bench.obs_bytes(n, True) == 1024 * n + 132098 * 2 + 8 * n
    assert bench.obs_bytes(n, False, road=7.0) == 1024 * n + 7.0
    assert bench.CONTROL_STEP_BYTES_PER_AGENT == 1222


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_needs_matching_source_and_size():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0
    name, k = next(iter(rec["launches"].items()))
    # a different workload size never takes the recorded counters
    assert bench.recorded_traffic(k["kernel"], name, k["agents"] + 1) is None
    assert bench.recorded_traffic(k["kernel"], "no such launch", k["agents"]) is None
    v = bench.recorded_traffic(k["kernel"], name, k["agents"])
    from paper_2605_08528_amd.profile_summary import kernel_source_hash
    if k["source_hash"] == kernel_source_hash(k["kernel"]):
        assert v == pytest.approx((k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]) * 1024)
    else:
        assert v is None
