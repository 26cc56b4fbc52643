"""Host code under the address and undefined-behaviour sanitizers (CPU):
the oracle's C entry points on small inputs, and the library's host side
(argument checks, sizing, parameter map, host-only statistics) driven
through its C header. No GPU is touched: the library part runs only calls
that return before any device work."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_23786_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_oracle_is_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    b = _run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", *SAN, "-o", exe,
              os.path.join(ROOT, "tests", "c", "oracle_sanitize.cpp"), os.path.join(ROOT, "oracle", "lbm_oracle.cpp")])
    assert b.returncode == 0, b.stderr[-2000:]
    r = _run([exe], env=ENV)
    assert r.returncode == 0 and "ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])


def test_library_host_side_is_clean_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc")
    clang = "/opt/rocm/llvm/bin/clang"
    objs = [os.path.join(CSRC, f + ".o") for f in ("step_d3q27_f32", "step_d3q27_f64", "step_d3q19_f32",
                                                     "step_d3q19_f64", "kernels", "observables")]
    if hipcc is None or not os.path.exists(clang) or not all(os.path.exists(o) for o in objs):
        pytest.skip("hipcc, the ROCm clang or the built kernel objects are missing")
    host = [a for f in SAN for a in ("-Xarch_host", f)]
    api = str(tmp_path / "api_san.o")
    b = _run([hipcc, "--offload-host-only", *host, "-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"),
              "-c", os.path.join(CSRC, "api.hip"), "-o", api])
    assert b.returncode == 0, b.stderr[-2000:]
    chk = str(tmp_path / "abi_check.o")
    b = _run([clang, "-std=c99", "-O1", "-g", *SAN, "-I", os.path.join(ROOT, "include"), "-c",
              os.path.join(ROOT, "tests", "c", "abi_host_check.c"), "-o", chk])
    assert b.returncode == 0, b.stderr[-2000:]
    exe = str(tmp_path / "abi_check_san")
    b = _run([hipcc, "--hip-link", *SAN, "-o", exe, chk, api, *objs])
    assert b.returncode == 0, b.stderr[-2000:]
    r = _run([exe], env=ENV)
    assert r.returncode == 0 and "ok" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
