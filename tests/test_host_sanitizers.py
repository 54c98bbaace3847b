"""The host set-up under sanitizers (CPU only): tests/sanitize_setup.cpp,
built with g++ against the library's host sources, runs the hierarchy
construction, the explicit row sets and the quadrature exports on geometries
covering every curve kind and boundary condition.  AddressSanitizer and
UndefinedBehaviorSanitizer (all cases, leaks included) and ThreadSanitizer
(smaller grids, 4 set-up threads) must report nothing."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2504_00724_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "sanitize_setup.cpp"), os.path.join(CSRC, "setup.cpp"),
           os.path.join(CSRC, "quadrature.cpp")]


def _build_and_run(tmp_path, flags, args, env_extra):
    if shutil.which("g++") is None:
        pytest.skip("no C++ compiler")
    exe = str(tmp_path / "san")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", "-I",
                    os.path.join(ROOT, "include"), "-I", CSRC] + flags + SOURCES + ["-o", exe], check=True)
    env = dict(os.environ, **env_extra)
    res = subprocess.run([exe] + args, capture_output=True, text=True, env=env, timeout=600)
    print(res.stdout[-2000:])
    assert res.returncode == 0, res.stderr[-4000:]
    assert "checked" in res.stdout
    assert "runtime error" not in res.stderr and "Sanitizer" not in res.stderr, res.stderr[-4000:]


@pytest.mark.slow
def test_host_setup_under_address_and_undefined_sanitizers(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"], [],
                   {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"})


@pytest.mark.slow
def test_host_setup_under_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"], ["small"], {"TSAN_OPTIONS": "halt_on_error=1"})
