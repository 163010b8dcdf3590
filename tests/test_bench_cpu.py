"""Host-side checks of bench.py: the one-GPU contract and the per-launch
update count behind its roofline figure."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("T,H", [(64, 6), (64, 8), (32, 2), (1, 4), (7, 3), (5, 1)])
def test_launch_updates_sum_to_the_run(T, H):
    b = load_bench()
    per = b.launch_lups(10, 20, 30, T, H)
    assert len(per) == (T - 1) // H + 2
    assert sum(per) == pytest.approx(10 * 20 * 30 * T)


def test_kernel_source_hash_ignores_comments_only():
    import bench as b
    code = "int a = 1;  // one\n\n// a comment line\nint b = 2;\n"
    assert b._code_only(code) == "int a = 1;\nint b = 2;"
    assert b._code_only(code) != b._code_only(code.replace("2", "3"))


def test_kernel_source_hash_is_stable():
    b = load_bench()
    assert b.kernel_source_hash() == b.kernel_source_hash()
    assert len(b.kernel_source_hash()) == 16
