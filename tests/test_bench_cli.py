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


def test_algorithmic_bytes_per_launch():
    """16 nm, 256 FP32 vectors, degree 16: 49,925,477 points x 256 x 4 B x (2 + 3 x 15) / 16
    = 150,175,834,816 B per launch; a degree-1 pass only reads Y_0 and writes Y_1."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.alg_bytes_per_launch(49_925_477, 256, 4, 16) == 150_175_834_816
    assert bench.alg_bytes_per_launch(1000, 8, 8, 1) == 1000 * 8 * 8 * 2
    # FP64 doubles the bytes; a long pass tends to three block passes per launch
    assert bench.alg_bytes_per_launch(10, 4, 8, 3) == 2 * bench.alg_bytes_per_launch(10, 4, 4, 3)
    assert abs(bench.alg_bytes_per_launch(1, 1, 1, 10 ** 6) - 3) < 1e-5
