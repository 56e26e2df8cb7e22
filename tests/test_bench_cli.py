"""bench.py command line, on the CPU: the one-GPU rule and the argument
surface (no GPU work is started by these calls)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=env)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="2")
    r = _run(env=env)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_unknown_workload_is_rejected():
    r = _run("--workload", "d2q9_riemann")
    assert r.returncode == 2
    assert "invalid choice" in r.stderr


def test_step_workloads_exist():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1309_1656_amd import synthetic
    for name, storages in bench.STEP_WORKLOADS.items():
        assert name in synthetic.WORKLOADS
        assert set(storages) <= set(bench.STORAGE_NAMES)
    assert "d3q19_128" in bench.STEP_WORKLOADS


def test_cpu_leg_runs_in_a_spawned_child():
    """The CPU oracle leg runs in a spawned child process: bench.py must import there without side effects
    (no GPU use at import), and its functions must reach the child by reference."""
    import concurrent.futures
    import multiprocessing
    sys.path.insert(0, ROOT)
    import bench
    with concurrent.futures.ProcessPoolExecutor(max_workers=1, mp_context=multiprocessing.get_context("spawn")) as ex:
        assert ex.submit(bench._cpu_model).result(timeout=120) == bench._cpu_model()


def test_fewer_than_three_steps_are_refused():
    r = _run("--steps", "2")
    assert r.returncode == 2
    assert "at least 3" in r.stderr
