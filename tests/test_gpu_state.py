"""Physics pins of the HIP update itself, through the test-only state hooks of
the C ABI (fdtd_set_state / fdtd_get_state) with the plane wave off
(FDTD_SRC_NONE), and the in-solve watchdog.

* Yee closed form: a source-free PEC cavity mode evolves as
  E^n = E^0 cos((n + 1/2) w dt) / cos(w dt / 2) with the discrete dispersion
  relation sin^2(w dt / 2) = (v dt)^2 ktilde^2 / 4 (Sec. 3.2 discretization of
  eqs. (10a-c) without dispersion), in 2D and for two polarizations in 3D.
* Discrete energy identity of the trapezoidal Drude update (PEC box, lossy
  Drude design region, random state): U^{n+1} - U^n = -dt sum[sigma Ebar^2 +
  gamma Jbar^2 / (eps0 psi)] (eqs. (10a-c) with eqs. (4)-(5)).
* Parity with the oracle of a free evolution with absorber, lossy Drude
  design and random initial state (FP64 to 1e-11, FP32 to 1e-4).
* Watchdog: a non-finite or runaway field stops the solve with EUNSTABLE.
"""
import numpy as np
import pytest

import fdtd_workloads as W
from test_gpu_parity_2d import gpu, say  # noqa: F401

pytestmark = pytest.mark.gpu

C0 = 299792458.0
MU0 = 4e-7 * np.pi
EPS0 = 1.0 / (MU0 * C0 * C0)


def cavity2d(nx=24, ny=20, **over):
    """PEC box, no absorber, no plane wave, design box filling the interior."""
    w = W.tiny2d(n=(nx, ny, 1), pml_cells=0, tfsf_margin=0, source="none",
                 design_lo=(1, 1, 0), design_n=(nx - 2, ny - 2, 1),
                 gap_lo=(3, 3, 0), gap_n=(1, 1, 1), weights="unit")
    w.update(over)
    return w


def evolve(gpu, w, state, rho, steps):
    """The state after `steps` steps from `state` (one forward solve)."""
    g = gpu.FDTD(W.with_(w, n_steps=steps))
    g.set_density(np.asarray(rho, dtype=g.dtype))
    g.set_state(state)
    g.forward()
    out = g.get_state()
    g.close()
    return out


def sin_mode(n_a, m):
    return np.sin(m * np.pi * np.arange(n_a) / (n_a - 1))


@pytest.mark.parametrize("prec,tol", [(64, 1e-11), (32, 2e-4)])
def test_cavity_closed_form_2d(gpu, prec, tol):
    nx, ny, m, l = 24, 20, 2, 3
    w = cavity2d(nx, ny, omega_p=0.0, precision=prec)  # psi = 0: the design box is plain eps_s
    st = np.zeros((4, 1, ny, nx))
    E0 = np.outer(sin_mode(ny, l), sin_mode(nx, m))
    st[0, 0] = E0
    dt = w["courant"] * w["dx"] / C0
    v = C0 / np.sqrt(w["eps_s"])
    kt2 = 4.0 / w["dx"] ** 2 * (np.sin(m * np.pi / (2 * (nx - 1))) ** 2 + np.sin(l * np.pi / (2 * (ny - 1))) ** 2)
    th = 2 * np.arcsin(v * dt * np.sqrt(kt2) / 2)
    rho = np.zeros((ny - 2, nx - 2))
    worst = 0.0
    for n in (1, 10, 1000, 4000):
        E = evolve(gpu, w, st, rho, n)[0, 0]
        pred = E0 * np.cos((n + 0.5) * th) / np.cos(th / 2)
        worst = max(worst, np.abs(E - pred).max())
    say(f"[state] 2D cavity closed form fp{prec}: max |E - closed form| = {worst:.2e}")
    assert worst < tol


@pytest.mark.parametrize("pol", ["z", "x"])
def test_cavity_closed_form_3d(gpu, pol):
    """TM modes uniform along the field direction: E_z(i, j) (pol z) or E_x(j, k) (pol x)."""
    nx, ny, nz = 14, 12, 10
    w = W.tiny3d(n=(nx, ny, nz), pml_cells=0, tfsf_margin=0, source="none", omega_p=0.0, weights="unit",
                 design_lo=(1, 1, 1), design_n=(nx - 2, ny - 2, nz - 2), gap_lo=(3, 3, 3), gap_n=(1, 1, 1))
    st = np.zeros((9, nz, ny, nx))
    if pol == "z":
        m, l = 2, 1
        E0 = np.outer(sin_mode(ny, l), sin_mode(nx, m))[None, :, :] * np.ones((nz, 1, 1))
        E0[nz - 1] = 0.0  # E_z lives at k + 1/2, k <= nz - 2
        st[2] = E0
        kt2 = 4.0 / w["dx"] ** 2 * (np.sin(m * np.pi / (2 * (nx - 1))) ** 2 + np.sin(l * np.pi / (2 * (ny - 1))) ** 2)
        comp = 2
    else:
        l, p = 1, 2
        E0 = np.outer(sin_mode(nz, p), sin_mode(ny, l))[:, :, None] * np.ones((1, 1, nx))
        E0[:, :, nx - 1] = 0.0  # E_x lives at i + 1/2, i <= nx - 2
        st[0] = E0
        kt2 = 4.0 / w["dx"] ** 2 * (np.sin(l * np.pi / (2 * (ny - 1))) ** 2 + np.sin(p * np.pi / (2 * (nz - 1))) ** 2)
        comp = 0
    dt = w["courant"] * w["dx"] / C0
    th = 2 * np.arcsin(C0 / np.sqrt(w["eps_s"]) * dt * np.sqrt(kt2) / 2)
    rho = np.zeros((nz - 2, ny - 2, nx - 2))
    worst = 0.0
    for n in (1, 7, 600):
        out = evolve(gpu, w, st, rho, n)
        pred = E0 * np.cos((n + 0.5) * th) / np.cos(th / 2)
        worst = max(worst, np.abs(out[comp] - pred).max())
        # the other components stay at round-off (tile-planes next to the walls
        # and interior ones are updated by different kernels)
        others = [c for c in range(3) if c != comp]
        assert np.abs(out[others]).max() < 1e-14
    say(f"[state] 3D cavity closed form pol {pol}: max |E - closed form| = {worst:.2e}")
    assert worst < 1e-11


def written_mask(shape):
    """Slots of the state the update writes: E and H off the PEC walls (Yee
    staggering: E_c spans nodes 0..n-2 along c and 1..n-2 across it, H_c the
    opposite).  The test zeroes the others so both sides start alike."""
    nf, nz, ny, nx = shape
    m = np.zeros(shape, bool)
    if nf == 4:  # E_z, H_x, H_y, J_z
        m[0, 0, 1:ny - 1, 1:nx - 1] = True
        m[1, 0, 0:ny - 1, 1:nx - 1] = True
        m[2, 0, 1:ny - 1, 0:nx - 1] = True
        m[3] = True
        return m
    n3 = (nx, ny, nz)
    for f in range(6):
        c, isE = f % 3, f < 3
        sl = []
        for d in (2, 1, 0):  # array axes z, y, x
            lo = 0 if (d == c) == isE else 1
            sl.append(slice(lo, n3[d] - 1))
        m[(f, *sl)] = True
    m[6:] = True
    return m


def random_state(shape, rng, design_mask, jscale=1e3):
    """Smooth random E and H (H scaled by the wave impedance) and random J on
    the Drude edges, zero on the slots the update never writes."""
    nf = shape[0]
    st = np.zeros(shape)
    ne = 1 if nf == 4 else 3
    for f in range(2 * ne):
        a = rng.standard_normal(shape[1:])
        a = W.box_smooth(a[0] if nf == 4 else a)
        st[f] = (a if nf != 4 else a[None]) / (377.0 if f >= ne else 1.0)
    for c in range(ne):
        st[2 * ne + c] = np.where(design_mask, rng.standard_normal(shape[1:]) * jscale, 0.0)
    return np.where(written_mask(shape), st, 0.0)


def test_energy_identity_2d(gpu):
    """PEC box, lossy Drude design region (sigma_max = 5e5 S/m, m_gamma = 16),
    random state: U^{n+1} - U^n = -D^n to 1e-12 of U, and U never grows."""
    nx, ny = 26, 22
    w = W.tiny2d(n=(nx, ny, 1), pml_cells=0, tfsf_margin=0, source="none", weights="unit",
                 design_lo=(6, 5, 0), design_n=(12, 10, 1), gap_lo=(2, 2, 0), gap_n=(1, 1, 1),
                 sigma_max=5e5, gamma_mult=16.0)
    rng = np.random.default_rng(3)
    rho = rng.random((10, 12))
    dmask = np.zeros((1, ny, nx), bool)
    dmask[0, 5:15, 6:18] = True
    st = random_state((4, 1, ny, nx), rng, dmask)
    # the update never writes E on the walls nor the H slots past the last row / column
    g = gpu.FDTD(W.with_(w, n_steps=1))
    g.set_density(rho)
    states = [st]
    for _ in range(40):
        g.set_state(states[-1])
        g.forward()
        states.append(g.get_state())
    g.close()
    psi = w["omega_p"] ** 2
    m = dmask[0]
    psi_i = np.ones((ny, nx)); eps_r = np.full((ny, nx), w["eps_s"]); sig = np.zeros((ny, nx))
    psi_i[m] = (w["psi_s_ratio"] * psi + rho * (1 - w["psi_s_ratio"]) * psi).ravel()
    eps_r[m] = (w["eps_s"] + rho * (w["eps_inf"] - w["eps_s"])).ravel()
    sig[m] = (rho * (1 - rho) * w["sigma_max"]).ravel()
    gam = w["gamma_mult"] * w["gamma_p"]
    dt = w["courant"] * w["dx"] / C0

    def U(n):
        E, Jn = states[n][0, 0], states[n][3, 0]
        Hm, Hp = states[n][1:3, 0], states[n + 1][1:3, 0]
        return (0.5 * np.sum(EPS0 * eps_r * E ** 2) + 0.5 * MU0 * np.sum(Hm * Hp)
                + np.sum(np.where(m, Jn ** 2 / (2 * EPS0 * psi_i), 0.0)))

    Us = [U(n) for n in range(len(states) - 1)]
    worst = 0.0
    for n in range(len(Us) - 1):
        Eb = 0.5 * (states[n + 1][0, 0] + states[n][0, 0])
        Jb = 0.5 * (states[n + 1][3, 0] + states[n][3, 0])
        D = dt * np.sum(sig * Eb ** 2 + np.where(m, gam * Jb ** 2 / (EPS0 * psi_i), 0.0))
        worst = max(worst, abs(Us[n + 1] - Us[n] + D) / Us[0])
        assert Us[n + 1] <= Us[n] * (1 + 1e-14)
    say(f"[state] 2D energy identity: worst residual {worst:.2e} of U; U fell by {1 - Us[-1] / Us[0]:.3e}")
    assert worst < 1e-12
    assert Us[-1] < Us[0]


@pytest.mark.parametrize("dims,prec", [(2, 64), (2, 32), (3, 64), (3, 32)])
def test_free_evolution_matches_oracle(gpu, oracle_mod, dims, prec):
    """Random initial state, absorber on (kappa/alpha stretched), lossy Drude
    design, no plane wave: the HIP state after N steps equals the oracle's."""
    if dims == 2:
        w = W.tiny2d(source="none", weights="unit", tfsf_margin=0, pml_kappa_max=2.0, pml_alpha_max=0.03,
                     n_steps=300, precision=prec)
    else:
        w = W.tiny3d(source="none", weights="unit", tfsf_margin=0, pml_kappa_max=2.0, pml_alpha_max=0.03,
                     n_steps=200, precision=prec)
    nx, ny, nz = w["n"]
    rng = np.random.default_rng(11)
    rho = W.seeded_rho(w, 5)
    shape = (4, 1, ny, nx) if dims == 2 else (9, nz, ny, nx)
    dmask = np.zeros(shape[1:], bool)
    lo, dn = w["design_lo"], w["design_n"]
    if dims == 2:
        dmask[0, lo[1]:lo[1] + dn[1], lo[0]:lo[0] + dn[0]] = True
        glo, gn = w["gap_lo"], w["gap_n"]
        dmask[0, glo[1]:glo[1] + gn[1], glo[0]:glo[0] + gn[0]] = False
    else:
        dmask[lo[2]:lo[2] + dn[2], lo[1]:lo[1] + dn[1], lo[0]:lo[0] + dn[0]] = True
        glo, gn = w["gap_lo"], w["gap_n"]
        dmask[glo[2]:glo[2] + gn[2], glo[1]:glo[1] + gn[1], glo[0]:glo[0] + gn[0]] = False
    st = random_state(shape, rng, dmask)
    g = gpu.FDTD(w)
    g.set_density(rho.astype(g.dtype))
    g.set_state(st)
    g.forward()
    out = g.get_state()
    g.close()
    o = oracle_mod.Oracle(W.with_(w, precision=64))
    o.set_density(rho)
    if dims == 2:
        o.set_state(st[0, 0], st[1, 0], st[2, 0], st[3, 0])
    else:
        o.set_state(list(st[0:3]), list(st[3:6]), list(st[6:9]))
    o.step_free(w["n_steps"])
    ref = o.get_state()
    ref = np.stack([ref[0], ref[1], ref[2], ref[3]])[:, None] if dims == 2 else np.stack([*ref[0], *ref[1], *ref[2]])
    o.close()
    ne = 1 if dims == 2 else 3
    errE = np.linalg.norm(out[:ne] - ref[:ne]) / np.linalg.norm(ref[:ne])
    errH = np.linalg.norm(out[ne:2 * ne] - ref[ne:2 * ne]) / np.linalg.norm(ref[ne:2 * ne])
    errJ = np.linalg.norm(out[2 * ne:] - ref[2 * ne:]) / np.linalg.norm(ref[2 * ne:])
    say(f"[state] free evolution {dims}D fp{prec} N={w['n_steps']}: rel E {errE:.2e} H {errH:.2e} J {errJ:.2e}")
    tol = 1e-11 if prec == 64 else 1e-4
    assert errE < tol and errH < tol and errJ < tol


def test_watchdog_stops_a_nonfinite_solve(gpu):
    w = cavity2d(n_steps=5000)
    nx, ny, _ = w["n"]
    st = np.zeros((4, 1, ny, nx))
    st[0, 0] = np.outer(sin_mode(ny, 1), sin_mode(nx, 1))
    st[0, 0, 7, 9] = np.nan
    g = gpu.FDTD(w)
    g.set_density(np.full((ny - 2, nx - 2), 0.5))
    g.set_state(st)
    with pytest.raises(gpu.FDTDError) as e:
        g.forward()
    assert e.value.name == "EUNSTABLE" and "after step 1024" in str(e.value), str(e.value)
    with pytest.raises(gpu.FDTDError) as e2:  # no valid forward: no adjoint, no state
        g.adjoint()
    assert e2.value.name == "ESTATE"
    with pytest.raises(gpu.FDTDError) as e3:
        g.get_state()
    assert e3.value.name == "ESTATE"
    g.set_state(None)  # cleared: a zero start stays zero
    F = g.forward()
    assert F == 0.0 and np.all(g.get_state() == 0.0)
    g.close()


@pytest.mark.parametrize("prec", [64, 32])
def test_watchdog_runaway_field_with_plane_wave(gpu, prec):
    # a closed box (no absorber) keeps the field from leaving before the first check
    w = W.tiny2d(n_steps=3000, precision=prec, pml_cells=0, tfsf_margin=3)
    nx, ny, _ = w["n"]
    st = np.zeros((4, 1, ny, nx))
    st[0, 0, 20, 20] = 1e14  # 1e14 times the incident amplitude
    g = gpu.FDTD(w)
    g.set_density(W.seeded_rho(w, 0).astype(g.dtype))
    g.set_state(st)
    with pytest.raises(gpu.FDTDError) as e:
        g.forward()
    assert e.value.name == "EUNSTABLE" and "after step 1024" in str(e.value), str(e.value)
    g.set_state(None)
    F = g.forward()  # the same context solves normally again
    assert np.isfinite(F) and F > 0
    g.close()


def test_state_hooks_call_order_and_validation(gpu):
    w = W.tiny2d()
    g = gpu.FDTD(w)
    with pytest.raises(gpu.FDTDError) as e:
        g.get_state()
    assert e.value.name == "ESTATE"
    rho = W.seeded_rho(w, 0)
    g.set_density(rho)
    g.forward()
    s1 = g.get_state()
    assert s1.shape == g.state_shape() and np.any(s1 != 0)
    g.adjoint()
    with pytest.raises(gpu.FDTDError) as e:
        g.get_state()
    assert e.value.name == "ESTATE"
    with pytest.raises(gpu.FDTDError) as e:
        g.set_state(np.zeros(7))
    assert e.value.name == "EINVAL"
    g.close()
    # boxes next to the absorber need the plane wave off; axes other than the defaults are refused
    with pytest.raises(gpu.FDTDError) as e:
        gpu.FDTD(W.tiny2d(design_lo=(7, 7, 0)))
    assert e.value.name == "EINVAL"
    gpu.FDTD(W.tiny2d(design_lo=(7, 7, 0), source="none")).close()
    with pytest.raises(gpu.FDTDError) as e:  # 2D: E along z (TMz) or x (TEz)
        gpu.FDTD(W.tiny2d(pol_axis="y"))
    assert e.value.name == "EINVAL"
    gpu.FDTD(W.tiny2d(pol_axis="z", prop_axis="y")).close()
    with pytest.raises(gpu.FDTDError) as e:
        gpu.FDTD(W.tiny3d(prop_axis="y"))
    assert e.value.name == "EINVAL"
