"""The kernels' index arithmetic, compiled for the host and run on the CPU
(no GPU): cell decomposition and periodic neighbours on every lattice size
the library accepts (8^3 to 1024^3, with the last nodes of a 1024^3 plane),
the AA slot mapping of the in-place step (each slot read and written once
per step; two steps stream every population by its velocity, on both
lattices), the XCD block renumbering and the launch tables' segment search.
The program includes the library's own device header (tests/c/index_check.hip)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_index_arithmetic_on_the_host(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "index_check")
    src = os.path.join(ROOT, "tests", "c", "index_check.hip")
    subprocess.run([hipcc, "-std=c++17", "-O1", "--offload-host-only", "-x", "hip", "-I",
                    os.path.join(ROOT, "include"), "-o", exe, src], check=True, capture_output=True, text=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stderr[-3000:]
    assert "index arithmetic ok" in p.stdout
