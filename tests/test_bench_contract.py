"""Host-side parts of bench.py: the one-GPU guard and the tie between the
committed HBM counter record and the query kernel's code (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_kernel_hash_ignores_comments_and_blank_space_only():
    code = "__global__ void k(float* x) {\n  x[0] = 1.f;  // store\n}\n"
    same = "// header comment\n__global__   void k(float* x) {\n\n    x[0] = 1.f;\n}\n"
    changed = "__global__ void k(float* x) {\n  x[1] = 1.f;  // store\n}\n"
    assert bench.kernel_source_hash(code) == bench.kernel_source_hash(same)
    assert bench.kernel_source_hash(code) != bench.kernel_source_hash(changed)


def test_kernel_hash_covers_every_kernel_source():
    texts = []
    for path in bench.KERNEL_SRCS:
        assert os.path.isfile(path), path
        with open(path) as f:
            texts.append(f.read())
    full = bench.kernel_source_hash()
    assert full == bench.kernel_source_hash("\n".join(texts))
    # a code line appended to any one of the files changes the hash
    for i in range(len(texts)):
        edited = list(texts)
        edited[i] += "\nstatic int probe_line;\n"
        assert bench.kernel_source_hash("\n".join(edited)) != full


def test_traffic_record_only_serves_its_own_launch():
    # whatever the record holds, it never answers for another launch size or precision
    assert bench.measured_traffic(128 * 16384 + 64, "bf16x2_f16") is None
    assert bench.measured_traffic(128 * 16384, "not-a-precision") is None
