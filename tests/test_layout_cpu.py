"""Host check of the step kernel's x-blocked gather addressing (no GPU).

The per-lane offsets (TileLanes), the block-uniform segments (pull_segment,
bounce_segment) and the x-wall selection (x_wall) of csrc/lattice.h are
host-and-device functions. tests/layout_check.cpp runs them for every tile,
thread and population of the launch geometry, on ragged grids (nx from 1 to
1024, ny and nz from 1 to 4) for all three models, and checks that every load
and store index lies inside the buffer, that the value a node finally pulls
(after the x-wall fix-up) is the element the reference pull (pull_ptr) names,
and that the stores hit every (population, node) slot exactly once.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2112_08479_amd", "csrc")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.timeout(300)
def test_x_blocked_gather_addressing():
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "layout_check")
        r = subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O1", "-std=c++17",
                            "-I", CSRC, "-o", exe, os.path.join(HERE, "layout_check.cpp")],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        r = subprocess.run([exe], capture_output=True, text=True, timeout=240)
        print(r.stdout[-2000:])
        assert r.returncode == 0 and "fails 0" in r.stdout
