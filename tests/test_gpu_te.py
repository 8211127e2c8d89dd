"""The 2D TEz HIP path (E in the plane: the paper's plasmonic 2D case,
Sec. 4.1) against the TEz CPU oracle on the same seeded inputs, through the C
ABI: objective, gap DFT and per-edge gradient at the stated bars (FP64 1e-11;
FP32 1e-4 on F and the DFT, 1e-3 on the gradient), the cavity closed form and
free evolution through the state hooks, the paper's per-edge layout, and
validation."""
import numpy as np
import pytest

import fdtd_workloads as W
from test_gpu_parity_2d import compare, gpu, rel_l2, say  # noqa: F401

pytestmark = pytest.mark.gpu

C0 = 299792458.0

VARIANTS = [
    dict(),
    dict(sigma_max=0.0, gamma_mult=1.0),
    dict(objective="time_energy"),
    dict(pml_kappa_max=3.0, pml_alpha_max=0.05, source="sinc_hann"),
    dict(eps_inf=4.469, weights="unit"),
    # ragged: grid and boxes not multiples of the 64 x 4 workgroup tile
    dict(n=(77, 53, 1), design_lo=(20, 18, 0), design_n=(37, 17, 1), gap_lo=(31, 24, 0), gap_n=(3, 2, 1)),
]


@pytest.mark.parametrize("over", VARIANTS)
def test_tiny_te_fp64(gpu, oracle_mod, over):
    w = W.tiny_te(**over)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 0), 1e-11, 1e-11, "TEz fp64")


@pytest.mark.parametrize("over", VARIANTS[:4])
def test_tiny_te_fp32(gpu, oracle_mod, over):
    w = W.tiny_te(precision=32, **over)
    compare(gpu, oracle_mod, w, W.seeded_rho(w, 1), 1e-4, 1e-3, "TEz fp32")


@pytest.mark.parametrize("prec,tol", [(64, (1e-11, 1e-11)), (32, (1e-4, 1e-3))])
def test_medium_te(gpu, oracle_mod, prec, tol):
    """384^2 with the 2048^2 workload's physics, a 96^2 design box (18,624
    design edges), 2400 steps: several workgroup tiles and the ragged tail."""
    w = W.medium_te(precision=prec)
    _, g = compare(gpu, oracle_mod, w, W.seeded_rho(w, 2), tol[0], tol[1], f"TEz medium fp{prec}")
    assert g.shape == (W.te_edges(w["design_n"])[1],)


def test_papers_layout_counts(gpu):
    """The paper's 2D case at 0.5 nm: a 200 x 200-cell design box around a
    20 x 20-cell gap takes 80,400 edge densities, of which the 840 gap edges
    carry no gradient, leaving 79,560 design variables (Sec. 4.1)."""
    w = W.tiny_te(n=(240, 240, 1), n_steps=900, design_lo=(20, 20, 0), design_n=(200, 200, 1),
                  gap_lo=(110, 110, 0), gap_n=(20, 20, 1), precision=64)
    g = gpu.FDTD(w)
    assert g.nd == 80400 and g.ng == 840
    F, grad = g.run(W.seeded_rho(w, 0))
    g.close()
    assert F > 0 and grad.shape == (80400,)
    # the gap's edges in the density layout: E_x rows 90..110 x cols 90..109,
    # E_y rows 90..109 x cols 90..110 (design-local)
    gapm = np.zeros(80400, bool)
    ex = gapm[:200 * 201].reshape(201, 200)
    ey = gapm[200 * 201:].reshape(200, 201)
    ex[90:111, 90:110] = True
    ey[90:110, 90:111] = True
    assert gapm.sum() == 840
    nz = np.count_nonzero(grad)
    say(f"[te] layout: F {F:.4e}, {nz} non-zero gradient entries of {grad.size}")
    assert np.all(grad[gapm] == 0) and nz > 0.99 * 79560
    with pytest.raises(Exception):
        g2 = gpu.FDTD(w)
        try:
            g2.set_density(np.zeros(79560))
        finally:
            g2.close()


def hz_mode(nx, ny, m, l):
    x = (np.arange(nx) + 0.5) / (nx - 1)
    y = (np.arange(ny) + 0.5) / (ny - 1)
    h = np.outer(np.cos(l * np.pi * y), np.cos(m * np.pi * x))
    h[-1, :] = 0.0
    h[:, -1] = 0.0
    return h


@pytest.mark.parametrize("prec,tol", [(64, 1e-11), (32, 2e-4)])
def test_te_cavity_closed_form(gpu, prec, tol):
    """Source-free PEC cavity on the GPU kernels: H_z^{-1/2} a cavity mode,
    E^0 = 0; after N steps H_z^{N-1/2} = H_z^{-1/2} cos((N-1/2) w dt)/cos(w dt/2)
    with sin^2(w dt/2) = (v dt)^2 ktilde^2 / 4."""
    nx, ny, m, l = 40, 36, 3, 2
    w = W.tiny_te(n=(nx, ny, 1), pml_cells=0, tfsf_margin=0, source="none", design_lo=(4, 4, 0),
                  design_n=(8, 8, 1), gap_lo=(20, 20, 0), gap_n=(2, 2, 1), omega_p=0.0, eps_inf=2.25,
                  sigma_max=0.0, weights="unit", n_steps=600, precision=prec)
    g = gpu.FDTD(w)
    st = np.zeros(g.state_shape())
    H0 = hz_mode(nx, ny, m, l)
    st[2, 0] = H0
    g.set_state(st)
    g.set_density(np.full(g.dshape, 0.4, dtype=g.dtype))
    g.forward()
    out = g.get_state()
    g.close()
    dt = w["courant"] * w["dx"] / C0
    v = C0 / np.sqrt(w["eps_s"])
    k2 = 4.0 / w["dx"] ** 2 * (np.sin(m * np.pi / (2 * (nx - 1))) ** 2 + np.sin(l * np.pi / (2 * (ny - 1))) ** 2)
    th = 2 * np.arcsin(v * dt * np.sqrt(k2) / 2)
    N = w["n_steps"]
    want = H0 * np.cos((N - 0.5) * th) / np.cos(th / 2)
    err = np.abs(out[2, 0] - want).max() / np.abs(H0).max()
    say(f"[te] cavity fp{prec}: max error {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("prec", [64, 32])
def test_te_free_evolution_matches_oracle(gpu, oracle_mod, prec):
    """A seeded random state in a closed lossy Drude box (no absorber, no
    source) evolved by the GPU and by the oracle."""
    nx, ny = 50, 46
    w = W.tiny_te(n=(nx, ny, 1), pml_cells=0, tfsf_margin=0, source="none", design_lo=(10, 9, 0),
                  design_n=(20, 18, 1), gap_lo=(18, 16, 0), gap_n=(3, 3, 1), weights="unit", n_steps=300,
                  precision=prec)
    rng = np.random.default_rng(11)
    rho = W.seeded_rho(w, 4)
    st = np.zeros((5, 1, ny, nx))
    for f in range(3):
        st[f, 0] = W.box_smooth(rng.standard_normal((ny, nx))) * (1.0 if f < 2 else 1 / 377)
    st[3, 0] = rng.standard_normal((ny, nx)) * 1e3
    st[4, 0] = rng.standard_normal((ny, nx)) * 1e3
    g = gpu.FDTD(w)
    g.set_state(st)
    g.set_density(rho.astype(g.dtype))
    g.forward()
    got = g.get_state()
    g.close()
    o = oracle_mod.Oracle(W.with_(w, precision=64))
    o.set_density(rho)
    # the oracle keeps every slot of the arrays; give it what the GPU keeps:
    # the E/H nodes the update writes and J on the Drude edges
    ex, ey, hz, jx, jy = [st[f, 0].copy() for f in range(5)]
    ex[0, :] = ex[-1, :] = 0; ex[:, -1] = 0
    ey[:, 0] = ey[:, -1] = 0; ey[-1, :] = 0
    hz[-1, :] = 0; hz[:, -1] = 0
    dnx, dny = w["design_n"][:2]
    d0x, d0y = w["design_lo"][:2]
    gx0, gy0 = w["gap_lo"][:2]
    gnx, gny = w["gap_n"][:2]
    mx = np.zeros((ny, nx), bool); mx[d0y:d0y + dny + 1, d0x:d0x + dnx] = True
    mx[gy0:gy0 + gny + 1, gx0:gx0 + gnx] = False
    my = np.zeros((ny, nx), bool); my[d0y:d0y + dny, d0x:d0x + dnx + 1] = True
    my[gy0:gy0 + gny, gx0:gx0 + gnx + 1] = False
    jx = np.where(mx, jx, 0.0)
    jy = np.where(my, jy, 0.0)
    if prec == 32:
        ex, ey, hz, jx, jy = [a.astype(np.float32).astype(np.float64) for a in (ex, ey, hz, jx, jy)]
        o.set_density(rho.astype(np.float32).astype(np.float64))
    o.set_state(ex, ey, hz, jx, jy)
    o.step_free(w["n_steps"])
    want = o.get_state()
    errs = [rel_l2(got[f, 0], want[f]) for f in range(5)]
    say(f"[te] free evolution fp{prec}: " + " ".join(f"{e:.1e}" for e in errs))
    tol = 1e-11 if prec == 64 else 1e-4
    assert max(errs) <= tol


def test_te_validation(gpu):
    w = W.tiny_te()
    with pytest.raises(gpu.FDTDError, match="checkpoint"):
        gpu.FDTD(w, ckpt_every=100)
    with pytest.raises(gpu.FDTDError):
        gpu.FDTD(W.with_(w, pol_axis="y"))
    # TEz boxes include their upper edge line: a design box reaching the
    # total-field box's last node is rejected
    P, m = w["pml_cells"], w["tfsf_margin"]
    ib = w["n"][0] - 1 - P - m
    with pytest.raises(gpu.FDTDError, match="total-field"):
        gpu.FDTD(W.with_(w, design_lo=(ib - 12, 16, 0), design_n=(12, 12, 1)))
    with pytest.raises(gpu.FDTDError, match="TMz"):
        gpu.Batch([w])
