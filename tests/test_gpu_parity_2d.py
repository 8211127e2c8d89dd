"""GPU parity of the 2D TMz HIP path against the CPU oracle (same seeded inputs).

Bars: FP64 build <= 1e-11 relative L2 on the gap DFT, the objective and the
gradient; FP32 build <= 1e-4 on the DFT/objective and <= 1e-3 on the gradient.
Every call goes through the C ABI (paper_2203_01462_amd.FDTD)."""
import sys

import numpy as np
import pytest

import fdtd_workloads as W

pytestmark = pytest.mark.gpu


def max_rel(a, b):
    """max |a - b| over max |b| (complex arrays by modulus)."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import paper_2203_01462_amd as P
    P.load_library()
    return P


def compare(gpu, oracle_mod, w, rho, tol_f, tol_g, label=""):
    say(f"[parity] {label} {w['name']} n={w['n']} N={w['n_steps']} prec={w['precision']}")
    o = oracle_mod.Oracle(W.with_(w, precision=64))
    Fo, go = o.run(rho)
    dfo = o.dft()
    g = gpu.FDTD(w)
    Fg, gg = g.run(rho.astype(g.dtype))
    dfg = g.dft()
    g.close()
    eF = abs(Fg - Fo) / abs(Fo)
    eD = rel_l2(dfg, dfo)
    eG = rel_l2(gg, go)
    # a localised error (a few cells near the gap) could hide under the
    # whole-array norm: the largest single deviation, against the largest value
    mD = max_rel(dfg, dfo)
    mG = max_rel(gg, go)
    say(f"   F {Fg:.12e} vs {Fo:.12e}  relF={eF:.2e} relDFT={eD:.2e} relGrad={eG:.2e} "
        f"maxDFT={mD:.2e} maxGrad={mG:.2e}")
    assert Fo > 0
    assert eF <= tol_f and eD <= tol_f, (eF, eD)
    assert eG <= tol_g, eG
    assert mD <= 10 * tol_f and mG <= 10 * tol_g, (mD, mG)
    return Fg, gg


VARIANTS = [
    dict(),
    dict(sigma_max=0.0, gamma_mult=1.0),
    dict(objective="time_energy"),
    dict(weights="unit"),
    dict(pml_kappa_max=3.0, pml_alpha_max=0.05, source="sinc_hann"),
    dict(eps_inf=4.469, gap_n=(1, 1, 1)),
    # ragged: grid and boxes not multiples of the 64x16 tile
    dict(n=(77, 53, 1), design_lo=(20, 18, 0), design_n=(37, 17, 1), gap_lo=(31, 24, 0), gap_n=(3, 2, 1)),
]


@pytest.mark.parametrize("over", VARIANTS)
def test_tiny_fp64(gpu, oracle_mod, over):
    w = W.tiny2d(**over)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 0), 1e-11, 1e-11, "tiny fp64")


@pytest.mark.parametrize("over", VARIANTS[:3])
def test_tiny_fp32(gpu, oracle_mod, over):
    w = W.tiny2d(precision=32, **over)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 0), 1e-4, 1e-3, "tiny fp32")


@pytest.mark.parametrize("seed,kind", [(0, "smooth"), (1, "smooth"), (2, "smooth"), (0, "half"), (0, "binary")])
def test_c1_fp64(gpu, oracle_mod, seed, kind):
    w = W.c1()
    compare(gpu, oracle_mod, w, W.seeded_rho(w, seed, kind), 1e-11, 1e-11, f"C1 seed={seed} {kind}")


def test_c1_in_fp32(gpu, oracle_mod):
    w = W.with_(W.c1(), precision=32)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 0), 1e-4, 1e-3, "C1 fp32")


@pytest.mark.parametrize("gmult", [1.0, 16.0])
def test_medium_fp32_c2_physics(gpu, oracle_mod, gmult):
    """512^2 grid with the 2048^2 workload's dx, CPML, gap and band, FP32,
    3600 steps (the pulse reaches the gap), damping multipliers 1 and 16."""
    w = W.medium2d(gamma_mult=gmult)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 0), 1e-4, 1e-3, f"medium fp32 gamma x{gmult}")


def test_medium_fp64(gpu, oracle_mod):
    w = W.medium2d(precision=64, sigma_max=5e5)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 1), 1e-11, 1e-11, "medium fp64")


def test_c2_full_directional_derivative(gpu):
    """Full 2048^2 x 20000-step workload in FP64: the adjoint gradient predicts
    the change of F along a random smooth direction (central difference of
    two more full solves) to 1e-3 (observed ~8e-5)."""
    w = W.with_(W.c2(), precision=64)
    rho = W.seeded_rho(w, 0)
    say("[parity] C2 full 2048^2 x 20000 fp64: forward+adjoint+gradient")
    g = gpu.FDTD(w)
    F, grad = g.run(rho)
    assert np.isfinite(F) and F > 0 and np.all(np.isfinite(grad))
    d = W.box_smooth(np.random.default_rng(7).standard_normal(rho.shape))
    h = 0.02
    rp = np.clip(rho + h * d, 0, 1)
    rm = np.clip(rho - h * d, 0, 1)
    g.set_density(rp); Fp = g.forward()
    g.set_density(rm); Fm = g.forward()
    g.close()
    pred = float(np.dot(grad.ravel(), (rp - rm).ravel()))
    say(f"   F={F:.9e}  dF fd={Fp - Fm:.9e} adjoint={pred:.9e}")
    assert abs((Fp - Fm) - pred) <= 1e-3 * abs(Fp - Fm)


@pytest.mark.xfail(reason="FP32 storage limit at this gap depth (see test_gpu_fullsize.C2_FP32_LIMIT)",
                   strict=False)
def test_c2_full_fp32_against_fp64(gpu):
    """The FP32 build at the full 2048^2 x 20000-step size against the FP64
    build, at the FP32 bars 1e-4 (F) and 1e-3 (gradient).  Measured:
    1.5e-4 and 2.5e-2 -- the gap field is below FP32's resolution of the
    background field; FP32 parity on the 512^2 grids is ~1e-6 / ~2e-4."""
    w = W.c2()
    rho = W.seeded_rho(w, 0)
    say("[parity] C2 full 2048^2 x 20000: fp32 vs fp64")
    res = {}
    for prec in (32, 64):
        g = gpu.FDTD(W.with_(w, precision=prec))
        res[prec] = g.run(rho.astype(g.dtype))
        g.close()
    (F32, g32), (F64, g64) = res[32], res[64]
    eF = abs(F32 - F64) / F64
    eG = rel_l2(g32, g64)
    say(f"   F32={F32:.9e} F64={F64:.9e} relF={eF:.2e} relGrad={eG:.2e}")
    assert eF <= 1e-4 and eG <= 1e-3

def test_call_order_and_validation(gpu):
    w = W.tiny2d()
    g = gpu.FDTD(w)
    with pytest.raises(gpu.FDTDError) as e:
        g.forward()
    assert e.value.name == "ESTATE"
    rho = W.seeded_rho(w, 0)
    bad = rho.copy(); bad[1, 1] = np.nan
    with pytest.raises(gpu.FDTDError) as e:
        g.set_density(bad)
    assert e.value.name == "EINVAL"
    g.set_density(rho)
    with pytest.raises(gpu.FDTDError) as e:
        g.adjoint()
    assert e.value.name == "ESTATE"
    g.forward()
    with pytest.raises(gpu.FDTDError) as e:
        g.gradient()
    assert e.value.name == "ESTATE"
    g.adjoint()
    g.gradient()
    g.set_density(rho)  # a new density invalidates the solves
    with pytest.raises(gpu.FDTDError) as e:
        g.adjoint()
    assert e.value.name == "ESTATE"
    with pytest.raises(gpu.FDTDError) as e:
        gpu.FDTD(W.tiny2d(design_lo=(3, 3, 0)))
    assert e.value.name == "EINVAL"
    g.close()


def test_device_pointers_and_determinism(gpu, oracle_mod):
    """Density and gradient passed as torch device tensors on the library's
    stream give the same result as host arrays, bit for bit, twice."""
    import torch
    w = W.tiny2d(precision=32)
    rho = W.seeded_rho(w, 3).astype(np.float32)
    s = torch.cuda.Stream()
    g = gpu.FDTD(w, stream=s.cuda_stream)
    F1, g1 = g.run(rho)
    with torch.cuda.stream(s):
        rd = torch.from_numpy(rho).to("cuda")
        out = torch.empty_like(rd)
    s.synchronize()
    g.set_density(rd)
    F2 = g.forward()
    g.adjoint()
    g.gradient(out)
    s.synchronize()
    g2 = out.cpu().numpy()
    g.close()
    assert F1 == F2
    assert np.array_equal(g1, g2)
