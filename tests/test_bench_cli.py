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


def test_committed_traffic_record_is_consistent():
    """profiles/traffic.json: the bytes per launch are the two counters times
    their copy-kernel scales, and the write counter is exactly one store of
    Y_{k+1} over the padded rows (16 nm: 53,417,472 rows x 256 FP32 vectors)."""
    import json
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["d16nm:f32:256"]
    total = rec["fetch_kib"] * 1024 * rec["fetch_scale"] + rec["write_kib"] * 1024 * rec["write_scale"]
    assert abs(total - rec["bytes_per_launch"]) < 1e-6 * total
    assert rec["write_kib"] * 1024 == 53_417_472 * 256 * 4
    assert 1.9 < rec["fetch_scale"] < 2.1 and rec["write_scale"] == 1.0
    assert len(rec["source_sha256"]) == 64
