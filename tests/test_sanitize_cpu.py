"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (oracle/fdtd2d.c, fdtd3d.c) linked into tests/sanitize_driver.c
  with -fsanitize=address,undefined: the small 2D and 3D problems with every
  feature on (absorber with stretching, plane wave, Drude design with
  artificial damping, gap), with the full history and checkpointed, must run
  without a report and give the normal oracle build's F and gradient.
* The host planner of the 3D work lists (the HIP library's host code, built
  for the CPU through tests/plan3d_check.hip) with the sanitizers on its host
  pass only, on its test geometries.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import fdtd_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    out = str(tmp_path_factory.mktemp("san") / "sanitize_driver")
    srcs = [os.path.join(ROOT, "tests", "sanitize_driver.c"), os.path.join(ROOT, "oracle", "fdtd2d.c"),
            os.path.join(ROOT, "oracle", "fdtd3d.c")]
    cmd = ["gcc", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99", "-D_DEFAULT_SOURCE",
           *SAN, *srcs, "-o", out, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    return out


def problem_text(oracle_mod, w, rho, ckpt):
    cfg, _ = oracle_mod.make_cfg(w)
    vals = []
    for name, _ in cfg._fields_:
        if name == "freqs_hz":
            continue
        v = getattr(cfg, name)
        vals += [str(x) for x in v] if hasattr(v, "__len__") else [repr(float(v)) if isinstance(v, float) else str(v)]
    vals.append(str(ckpt))
    vals += [repr(float(x)) for x in np.asarray(rho).ravel()]
    return " ".join(vals) + "\n"


@pytest.mark.parametrize("dims,ckpt", [(2, 0), (2, 97), (3, 0), (3, 64)])
def test_oracle_under_sanitizers(driver, oracle_mod, dims, ckpt):
    w = (W.tiny2d(n_steps=300, pml_kappa_max=2.0, pml_alpha_max=0.03) if dims == 2 else
         W.tiny3d(n_steps=200, pml_kappa_max=2.0, pml_alpha_max=0.03))
    rho = W.seeded_rho(w, 1)
    r = subprocess.run([driver], input=problem_text(oracle_mod, w, rho, ckpt), capture_output=True, text=True,
                       timeout=600, env=ENV)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    out = np.array([float(x) for x in r.stdout.split()])
    o = oracle_mod.Oracle(w)
    F, g = o.run(rho)
    o.close()
    assert abs(out[0] - F) <= 1e-13 * abs(F)
    assert np.allclose(out[1:], g.ravel(), rtol=1e-12, atol=1e-12 * np.abs(g).max())


def test_planner_under_sanitizers(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    from test_plan3d_cpu import CASES
    out = str(tmp_path / "plan3d_check_san")
    src = os.path.join(ROOT, "tests", "plan3d_check.hip")
    # the sanitizers apply to the host pass only
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    cmd = ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", *host_san,
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2203_01462_amd", "csrc"), src,
           "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    for case, args in sorted(CASES.items()):
        r = subprocess.run([out] + [str(v) for v in args], capture_output=True, text=True, timeout=120, env=ENV)
        assert r.returncode == 0, (case, r.stdout + r.stderr[-4000:])
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, (case, r.stderr[-4000:])
