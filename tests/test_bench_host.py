"""bench.py's host-side contract (no GPU): one GPU only, per-workload defaults,
and the traffic lookup keyed by the kernel sources' digest."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("workload,steps", [("spheres512", 20), ("spheres512_cutoff", 20),
                                            ("spheres512_reinit", 20), ("torus1024_f16s", 50),
                                            ("batch256", 10)])
def test_default_steps_cover_the_whole_run(workload, steps, monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", workload])
    a = bench.parse()
    assert a.steps == steps and a.gpus == 1 and a.warmup == 2 and a.snapshot_every == 0


def test_traffic_lookup_is_keyed_by_the_source_digest():
    step = bench.kernel_source_digest()
    gather = bench.kernel_source_digest(bench.GATHER_KERNEL_SOURCES)
    batch = bench.kernel_source_digest(bench.BATCH_KERNEL_SOURCES)
    dense = bench.kernel_source_digest(bench.DENSE_KERNEL_SOURCES)
    assert len({step, gather, batch, dense}) == 4 and len(step) == 16
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    for key, v in rec.items():
        want = (gather if key.startswith("gather/") else batch if "batch" in key else
                step if key.startswith("brick") else dense)
        kernel, workload = key.split("/", 1)
        got = bench.measured_traffic(kernel, workload, want)
        # an entry taken on other sources reads as unmeasured, never as stale bytes
        assert got == (v["bytes_per_launch"] if v["source_digest"] == want else None)
        assert bench.measured_traffic(kernel, workload, "0" * 16) is None
