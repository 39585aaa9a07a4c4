"""bench.py on the CPU: the module imports, the help text lists the modes,
and a multi-GPU request exits with a message (single-GPU build)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_help_lists_modes():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--workload", "--dtype", "--gram", "--cpu-sample", "--ordering", "--generic"):
        assert opt in r.stdout


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_module_helpers():
    sys.path.insert(0, ROOT)
    import bench
    assert len(bench.kernel_source_hash()) == 64
    assert "logical CPUs" in bench.host_cpu()
