"""The 3D work lists (host code of the HIP library, built here for the CPU
host): every tile-chunk with a general plane is in exactly one of the three
general launches, with the absorber axes and design code it needs, and the
plain launch's box covers every plain tile-plane; the two-step super-chunks
keep to plain background with three nodes to spare and store every node the
per-step launches read from them.  The 256^3 geometry, a small one, one
without absorber and one with ragged tiles and chunks."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = {
    "c3": [256, 256, 256, 16, 6, 64, 64, 112, 128, 128, 32, 126, 126, 126, 4, 4, 4],
    "small": [48, 48, 48, 8, 4, 20, 20, 20, 10, 10, 6, 24, 24, 22, 2, 2, 2],
    "no_absorber": [40, 40, 40, 0, 4, 14, 14, 14, 10, 10, 8, 18, 18, 18, 2, 2, 2],
    "ragged": [100, 72, 50, 10, 5, 30, 20, 18, 37, 29, 13, 45, 31, 23, 3, 2, 2],
    # the GPU parity cases: design chunks next to the absorber / away from it
    "medium3d": [80, 80, 80, 6, 3, 30, 30, 35, 20, 20, 10, 39, 39, 39, 2, 2, 2],
    "medium3d_interior": [80, 80, 80, 6, 3, 34, 30, 35, 20, 20, 10, 43, 39, 39, 2, 2, 2],
}
# absorber axes compiled into the design launch (0: none, 7: all)
AXD = {"c3": 0, "medium3d": 7, "medium3d_interior": 0}


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("plan3d") / "plan3d_check")
    src = os.path.join(ROOT, "tests", "plan3d_check.hip")
    cmd = ["hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2203_01462_amd", "csrc"), src, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return out


@pytest.mark.parametrize("case", sorted(CASES))
def test_plan3d_lists(exe, case):
    r = subprocess.run([exe] + [str(v) for v in CASES[case]], capture_output=True, text=True, timeout=60)
    print(case, r.stdout.strip())
    assert r.returncode == 0, r.stdout + r.stderr
    fields = r.stdout.split()
    general = int(fields[fields.index("general") + 1])
    assert general > 0
    if case in AXD:
        assert int(fields[fields.index("axD") + 1]) == AXD[case]
    assert int(fields[fields.index("super-bad") + 1]) == 0
    if case == "c3":
        # about a third of the 256^3 grid advances two steps per pass
        assert int(fields[fields.index("super-nodes") + 1]) > 0.3 * 256 ** 3
