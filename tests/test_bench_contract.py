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


def test_counter_traffic_is_reported_only_for_the_current_kernel():
    # counters are reported only for the kernel they were taken on, and only
    # while its source region hashes as it did then; otherwise None
    import hashlib
    import json

    with open(os.path.join(ROOT, "profiles", "roofline_traffic.json")) as f:
        data = json.load(f)
    with open(os.path.join(ROOT, data["source_file"])) as f:
        text = f.read()
    for workload, e in data["workloads"].items():
        begin, end = e["source_region"]
        current = begin in text and end in text and hashlib.sha256(
            text[text.index(begin):text.index(end)].encode()).hexdigest() == e["source_sha256"]
        for kernel in e["kernels"]:
            t = bench.counter_traffic(workload, kernel)
            assert (t is not None and t > 0) if current else t is None, (workload, kernel)
        assert bench.counter_traffic(workload, "k_no_such_kernel") is None
    assert bench.counter_traffic("no_such_workload", "k_csr<2, 16, double>") is None
