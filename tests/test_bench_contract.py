"""CPU checks of the benchmark's contract: it measures one GPU only and says
so when asked for more (before touching a device), and the memory-counter
traffic it reports still belongs to the roofline kernel's current source."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, env=e, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_a_distributed_launch_is_refused():
    r = _run([], env={"WORLD_SIZE": "2"})
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_counter_traffic_matches_the_current_kernel():
    # the committed counters were taken on the kernel as it is: its source
    # region still hashes as recorded, so the bench reports them
    for workload in ("64cube_timesteps", "128cube_planar_front"):
        t = bench.counter_traffic(workload)
        assert t is not None and t > 0, workload
    assert bench.counter_traffic("no_such_workload") is None
