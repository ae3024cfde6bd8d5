"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): host-only builds of

* tests/sanitize_host_check.cpp with csrc/abi.cpp: every validation path of
  the C ABI that runs before device work (valid, invalid and extreme
  configurations, null handles and arguments), kernel launchers stubbed;
* tests/layout_check.cpp: the step kernel's addressing helpers over every
  tile, thread and population of ragged grids.

The sanitizers instrument host code only (each -fsanitize= is given to the
host pass with -Xarch_host; --offload-host-only builds no device code). Any
report aborts the program and fails the test.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2112_08479_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def _build_and_run(sources, extra, expect):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "check")
        cmd = [hipcc, "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17", *SAN,
               "-I", CSRC, "-I", os.path.join(ROOT, "include"), "-o", exe, *sources, *extra]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        print(r.stdout[-2000:], r.stderr[-4000:])
        assert r.returncode == 0 and expect in r.stdout, r.stderr[-4000:]


@pytest.mark.timeout(900)
def test_abi_host_paths_under_sanitizers():
    _build_and_run([os.path.join(HERE, "sanitize_host_check.cpp"), os.path.join(CSRC, "abi.cpp")],
                   ["-L/opt/rocm/lib", "-lamdhip64"], "sanitize ok")


@pytest.mark.timeout(900)
def test_layout_check_under_sanitizers():
    _build_and_run([os.path.join(HERE, "layout_check.cpp")], [], "fails 0")
