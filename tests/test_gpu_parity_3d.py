"""GPU parity of the 3D HIP path against the 3D CPU oracle (same seeded inputs).

Bars as in 2D: FP64 <= 1e-11 relative L2 on the gap DFT, objective and
gradient; FP32 <= 1e-4 (DFT, objective) and <= 1e-3 (gradient)."""
import numpy as np
import pytest

import fdtd_workloads as W
from test_gpu_parity_2d import compare, gpu, say  # noqa: F401

pytestmark = pytest.mark.gpu

VARIANTS3 = [
    dict(),
    dict(sigma_max=0.0, gamma_mult=1.0),
    dict(objective="time_energy"),
    dict(pml_kappa_max=2.0, pml_alpha_max=0.05, weights="unit", source="sinc_hann"),
    # ragged: odd sizes, partial 32 x 8 x 2 blocks on every axis
    dict(n=(27, 29, 31), design_lo=(9, 10, 12), design_n=(7, 9, 5), gap_lo=(11, 12, 13), gap_n=(3, 2, 3)),
]


@pytest.mark.parametrize("over", VARIANTS3)
def test_tiny3d_fp64(gpu, oracle_mod, over):
    w = W.tiny3d(**over)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 0), 1e-11, 1e-11, "tiny3d fp64")


@pytest.mark.parametrize("over", VARIANTS3[:2])
def test_tiny3d_fp32(gpu, oracle_mod, over):
    w = W.tiny3d(precision=32, **over)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 0), 1e-4, 1e-3, "tiny3d fp32")


def test_medium3d_fp64(gpu, oracle_mod):
    w = W.medium3d()
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 1), 1e-11, 1e-11, "medium3d fp64")


@pytest.mark.parametrize("prec", [64, 32])
def test_medium3d_interior_design(gpu, oracle_mod, prec):
    """The design box inside one column of tiles that reaches no absorber:
    its tile-chunks take the general variant with the absorber code compiled
    out (the C3 layout; the other 3D cases put design chunks next to the
    absorber)."""
    w = W.medium3d(precision=prec, design_lo=(34, 30, 35), gap_lo=(43, 39, 39))
    tol = (1e-11, 1e-11) if prec == 64 else (1e-4, 1e-3)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 4), tol[0], tol[1], f"medium3d interior design fp{prec}")


@pytest.mark.parametrize("kind", ["smooth", "binary"])
def test_medium3d_fp32(gpu, oracle_mod, kind):
    w = W.medium3d(precision=32, sigma_max=5e5)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 2, kind), 1e-4, 1e-3, f"medium3d fp32 {kind}")


def test_c3_full_directional_derivative(gpu):
    """Full 256^3 x 8000-step FP32 workload: the adjoint gradient predicts the
    change of F along a random smooth direction; F and dF/drho are finite."""
    w = W.c3()
    rho = W.seeded_rho(w, 0).astype(np.float32)
    say("[parity] C3 full 256^3 x 8000 fp32: forward+adjoint+gradient")
    g = gpu.FDTD(w)
    F, grad = g.run(rho)
    assert np.isfinite(F) and F > 0 and np.all(np.isfinite(grad))
    d = W.box_smooth(np.random.default_rng(7).standard_normal(rho.shape)).astype(np.float32)
    h = 0.02
    rp = np.clip(rho + h * d, 0, 1)
    rm = np.clip(rho - h * d, 0, 1)
    g.set_density(rp); Fp = g.forward()
    g.set_density(rm); Fm = g.forward()
    g.close()
    pred = float(np.dot(grad.astype(np.float64).ravel(), (rp - rm).astype(np.float64).ravel()))
    say(f"   F={F:.6e}  dF fd={Fp - Fm:.6e} adjoint={pred:.6e}")
    assert abs((Fp - Fm) - pred) <= 0.02 * abs(Fp - Fm)
