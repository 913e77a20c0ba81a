"""bench.py's command line on the CPU: more than one GPU is refused with a
message before any GPU work."""
import os
import subprocess
import sys

from tests.conftest import ROOT


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_mixed_workload_problem_list():
    sys.path.insert(0, ROOT)
    import bench
    import paper_1508_02748_amd as R
    unit = bench.WORKLOADS["c3mix"][0]
    probs = bench.problems(3, R, unit)
    assert len(probs) == 3 * 6
    assert sorted({p.seed for p in probs}) == list(range(18))
    assert [p.L for p in probs[:6]] == [32, 8, 12, 16, 24, 32]
    assert [p.n_windows for p in probs[:6]] == [16, 2, 4, 8, 12, 16]
    assert {p.interval for p in probs} == {10_000}
    # one-problem workloads keep seed = replica index
    assert [p.seed for p in bench.problems(4, R, bench.C2)] == [0, 1, 2, 3]


def test_launch_key_of_measured_and_unknown_shapes():
    """The traffic and VALU-busy tables are keyed by launch shape: grids that give every tile of
    walkers its own workgroup are the same launch; a shape left to the library has no key."""
    sys.path.insert(0, ROOT)
    import bench
    k = ("c4", 256, 3, 256, 4, 0)
    assert k in bench.TRAFFIC_BYTES
    assert bench.launch_key("c4", 256, 3, 65536, 256, 4, 0) == k
    assert bench.launch_key("c4", 256, 3, 65536, 256, 8, 0) == k     # same launch: 256 tiles, 256 slots
    assert bench.launch_key("c4", 256, 3, 65536, 256, 2, 0) not in bench.TRAFFIC_BYTES
    assert bench.launch_key("c4", 256, 3, 65536, 0, 0, 0) is None      # --no-autotune, library's choice
