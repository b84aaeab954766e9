"""Host-side checks of the library's own index arithmetic, run on the CPU.

``tests/native/panel_layout_check.hip`` includes the library's panel-layout
header and runs the very functions the layout-building kernels call (count,
offsets, scatter: one row or one chunk each) on the host, over CSR matrices
whose rows list their columns in random order, and checks the launch shape of
the panel-ordered product (grid within the partial slots of a reduction,
every row block covered once) for up to 1e8 rows.  It is built host-side with
hipcc; no kernel is launched.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(shutil.which(HIPCC) is None, reason="hipcc not installed")
def test_panel_layout_any_column_order_and_launch_shape(tmp_path):
    exe = tmp_path / "panel_layout_check"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17",
                           "-I", os.path.join(ROOT, "paper_2507_02470_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "native", "panel_layout_check.hip"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-3000:]


@pytest.mark.skipif(shutil.which(HIPCC) is None, reason="hipcc not installed")
def test_split_layout_any_column_order(tmp_path):
    """``tests/native/split_layout_check.hip``: the column-split layout's count
    and scatter steps (the functions its build kernels call) on the host,
    checked segment by segment for sorted, shuffled and repeated columns."""
    exe = tmp_path / "split_layout_check"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17",
                           "-I", os.path.join(ROOT, "paper_2507_02470_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "native", "split_layout_check.hip"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-3000:]
