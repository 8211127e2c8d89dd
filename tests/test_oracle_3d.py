"""Pins of the 3D CPU oracle: Yee cavity dispersion for each polarization, the
discrete Drude dispersion of eqs. (4)-(5)/(10), exact plane-wave injection,
the whole-run adjoint dot-product identity (absorber transpose included),
Parseval between the DFT objective and eq. (24), and finite differences."""
import numpy as np
import pytest

import fdtd_workloads as W
from test_oracle_2d import C0, drude_char_poly

pytestmark = []


def cavity3(n=(14, 12, 10), **over):
    nx, ny, nz = n
    w = W.tiny3d(n=n, pml_cells=0, tfsf_margin=0, source="none", design_lo=(0, 0, 0), design_n=n,
                 gap_lo=(0, 0, 0), gap_n=(0, 0, 0), weights="unit")
    w.update(over)
    return w


def mode_field(n, comp, m1, m2):
    """Single-component cavity mode: the component is uniform along its own
    axis and a product of sines (zero on the walls it is tangential to) along
    the two others."""
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    crd = [i, j, k]
    axes = [a for a in range(3) if a != comp]
    f = np.sin(m1 * np.pi * crd[axes[0]] / (n[axes[0]] - 1)) * np.sin(m2 * np.pi * crd[axes[1]] / (n[axes[1]] - 1))
    k2 = 4.0 * (np.sin(m1 * np.pi / (2 * (n[axes[0]] - 1))) ** 2 + np.sin(m2 * np.pi / (2 * (n[axes[1]] - 1))) ** 2)
    return f, k2


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_yee_cavity_dispersion_each_polarization(oracle_mod, comp):
    n = (14, 12, 10)
    w = cavity3(n, omega_p=0.0)
    o = oracle_mod.Oracle(w)
    o.set_density(np.zeros(o.dshape))
    f, k2 = mode_field(n, comp, 2, 1)
    z = np.zeros(o.shape)
    E = [z, z, z]
    E[comp] = f
    o.set_state(E, [z, z, z], [z, z, z])
    dt = o.info()["dt"]
    v = C0 / np.sqrt(w["eps_s"])
    th = 2 * np.arcsin(v * dt * np.sqrt(k2) / w["dx"] / 2)
    worst = 0.0
    nstep = 0
    # E_c lives at half positions along its own axis: index n-1 is no edge
    phys = [slice(None)] * 3
    phys[2 - comp] = slice(0, n[comp] - 1)
    phys = tuple(phys)
    for chunk in (1, 9, 190, 800):
        o.step_free(chunk)
        nstep += chunk
        Ec = o.get_state()[0][comp]
        pred = f * np.cos((nstep + 0.5) * th) / np.cos(th / 2)
        worst = max(worst, np.abs(Ec - pred)[phys].max())
        others = [o.get_state()[0][c] for c in range(3) if c != comp]
        assert max(np.abs(x).max() for x in others) < 1e-12
    assert worst < 1e-10, worst


@pytest.mark.parametrize("rho,sigma_max,gmult", [(1.0, 0.0, 1.0), (0.5, 5e5, 4.0)])
def test_drude_cavity_characteristic_polynomial_3d(oracle_mod, rho, sigma_max, gmult):
    n = (12, 12, 10)
    w = cavity3(n, sigma_max=sigma_max, gamma_mult=gmult, eps_inf=4.469)
    o = oracle_mod.Oracle(w)
    o.set_density(np.full(o.dshape, rho))
    f, k2 = mode_field(n, 2, 1, 2)
    z = np.zeros(o.shape)
    o.set_state([z, z, f], [z, z, z], [z, z, z])
    dt = o.info()["dt"]
    psi = w["omega_p"] ** 2
    psi_i = w["psi_s_ratio"] * psi + rho * (1 - w["psi_s_ratio"]) * psi
    eps_i = w["eps_s"] + rho * (w["eps_inf"] - w["eps_s"])
    c = drude_char_poly(dt, eps_i, psi_i, gmult * w["gamma_p"], rho * (1 - rho) * sigma_max, k2 / w["dx"] ** 2)
    e = [f[3, 4, 5]]
    for _ in range(300):
        o.step_free(1)
        e.append(o.get_state()[0][2][3, 4, 5])
    e = np.array(e)
    res = max(abs(sum(c[k] * e[t + k] for k in range(4))) / sum(abs(c[k] * e[t + k]) for k in range(4))
              for t in range(len(e) - 3))
    assert res < 1e-10, res


def test_tfsf_no_scatterer_is_exact_3d(oracle_mod):
    w = W.tiny3d(psi_s_ratio=0.0, sigma_max=0.0, n_steps=600)
    o = oracle_mod.Oracle(w)
    o.set_density(np.zeros(o.dshape))
    o.forward()
    lo0, hi0, lo1, hi1, lo2, hi2 = o.info()["tf_box"]
    E, H, _ = o.get_state()
    peak = max(np.abs(o.incident_column(k)).max() for k in range(lo2, hi2 + 1))
    assert peak > 0.1
    inc = np.array([o.incident_column(k)[-1] for k in range(lo2, hi2 + 1)])
    # E_x in the total-field box (x half-positions lo0+1/2 .. hi0-1/2) equals the line
    tf = E[0][lo2:hi2 + 1, lo1:hi1 + 1, lo0:hi0]
    assert np.abs(tf - inc[:, None, None]).max() < 1e-12 * peak
    sf = E[0].copy()
    sf[lo2:hi2 + 1, lo1:hi1 + 1, lo0:hi0] = 0
    assert np.abs(sf).max() < 1e-12 * peak
    assert np.abs(E[1]).max() < 1e-12 * peak and np.abs(E[2]).max() < 1e-12 * peak


@pytest.mark.parametrize("kappa,alpha", [(1.0, 0.0), (3.0, 0.05)])
def test_adjoint_dot_product_whole_run_3d(oracle_mod, kappa, alpha):
    w = W.tiny3d(n_steps=30, pml_kappa_max=kappa, pml_alpha_max=alpha)
    o = oracle_mod.Oracle(w)
    o.set_density(W.seeded_rho(w, 2))
    rng = np.random.default_rng(5)
    shape = (w["n_steps"], 3) + o.shape
    q = rng.standard_normal(shape)
    s = rng.standard_normal(shape)
    E = o.forward_ext(q)
    Es = o.adjoint_ext(s)
    lhs, rhs = np.sum(s * E), np.sum(q * Es)
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum((s * E) ** 2)) * np.sqrt(s.size), (lhs, rhs)


@pytest.mark.parametrize("over", [dict(), dict(sigma_max=0.0, gamma_mult=1.0), dict(objective="time_energy"),
                                  dict(pml_kappa_max=2.0, pml_alpha_max=0.05, weights="unit")])
def test_gradient_matches_central_differences_3d(oracle_mod, over):
    w = W.tiny3d(**over)
    o = oracle_mod.Oracle(w)
    rho = W.seeded_rho(w, 0)
    F, g = o.run(rho)
    h = 1e-4
    for idx in [(0, 0, 0), (5, 7, 1), (1, 2, 6), (4, 0, 7)]:
        rp = rho.copy(); rp[idx] += h
        rm = rho.copy(); rm[idx] -= h
        o.set_density(rp); Fp = o.forward()
        o.set_density(rm); Fm = o.forward()
        fd = (Fp - Fm) / (2 * h)
        assert abs(g[idx] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (idx, g[idx], fd)
    assert np.all(g[2:4, 3:5, 3:5] == 0.0)  # gap cells


def test_parseval_dft_vs_time_energy_3d(oracle_mod):
    w = W.tiny3d(n_steps=300, weights="unit")
    dt = oracle_mod.Oracle(w).info()["dt"]
    N = w["n_steps"]
    rho = W.seeded_rho(w, 1)
    Fd, gd = oracle_mod.Oracle(W.with_(w, freqs_hz=[k / (N * dt) for k in range(N)])).run(rho)
    Fe, ge = oracle_mod.Oracle(W.with_(w, objective="time_energy")).run(rho)
    fac = 2 * N * dt / (w["eps_g"] * w["dx"] ** 3)
    assert abs(Fd - fac * Fe) < 1e-12 * abs(Fd)
    assert np.abs(gd - fac * ge).max() < 1e-10 * np.abs(gd).max()


def test_cpml_reflection_3d(oracle_mod):
    """Gap probe in the standard tiny domain versus the same probe in a domain
    enlarged by 24 cells on every side (no reflection can return in time)."""
    N = 260
    base = W.tiny3d(n_steps=N, sigma_max=0.0, gamma_mult=1.0)
    o = oracle_mod.Oracle(base)
    o.set_density(np.ones(o.dshape))
    o.forward()
    small = o.gap_series()[:, 0, 0]
    e = 24
    nx, ny, nz = base["n"]
    big = W.with_(base, n=(nx + 2 * e, ny + 2 * e, nz + 2 * e), tfsf_margin=2 + e,
                  design_lo=tuple(v + e for v in base["design_lo"]), gap_lo=tuple(v + e for v in base["gap_lo"]))
    ob = oracle_mod.Oracle(big)
    ob.set_density(np.ones(ob.dshape))
    ob.forward()
    ref = ob.gap_series()[:, 0, 0]
    err = np.abs(small - ref).max() / np.abs(ref).max()
    assert err < 1e-2, err
