"""The benchmark's host-side contract (CPU): one GPU only, argument checks,
and the counter summary is used only when taken on the current kernel
sources."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, HERE)
import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(HERE, "bench.py"), *args], capture_output=True, text=True,
                          timeout=60)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("n", ["0", "12"])
def test_calculating_solve_count_is_checked(n):
    r = _run("--eig-calc", n)
    assert r.returncode == 2 and "--eig-calc" in r.stderr


def test_counter_summary_needs_current_sources(tmp_path):
    good = tmp_path / "good.txt"
    good.write_text(f"kernel_sources_sha256 {bench.kernel_source_hash()}\ntraffic stencil_f16 123\nvalu stencil_f16 45\n")
    assert bench.read_counter("traffic", "stencil_f16", str(good))[0] == 123.0
    assert bench.read_counter("valu", "stencil_f16", str(good))[0] == 45.0
    assert bench.read_counter("traffic", "shift_update_f16", str(good))[0] is None
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_sources_sha256 0000000000000000\ntraffic stencil_f16 123\n")
    v, note = bench.read_counter("traffic", "stencil_f16", str(stale))
    assert v is None and "changed" in note
    assert bench.read_counter("traffic", "stencil_f16", str(tmp_path / "missing.txt"))[0] is None
