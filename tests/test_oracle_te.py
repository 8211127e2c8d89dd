"""Pins of the 2D TEz CPU oracle (E in the plane, H along z: the paper's
plasmonic 2D polarization, Sec. 4.1) against what the physics and the
mathematics fix: the Yee cavity dispersion closed form, the Drude cavity
frequency, the discrete energy identity, exact plane-wave injection, the
adjoint dot-product identity, central finite differences of the oracle's own
forward solve, and the per-edge design layout of the paper's 2D case."""
import numpy as np
import pytest

import fdtd_workloads as W

C0 = 299792458.0
MU0 = 4e-7 * np.pi
EPS0 = 1.0 / (MU0 * C0 * C0)


def cavity_te(nx=24, ny=20, **over):
    """PEC box, no absorber, no excitation, design box filling the interior."""
    w = W.tiny_te(n=(nx, ny, 1), pml_cells=0, tfsf_margin=0, source="none",
                  design_lo=(1, 1, 0), design_n=(nx - 3, ny - 3, 1),
                  gap_lo=(0, 0, 0), gap_n=(0, 0, 0), weights="unit")
    w.update(over)
    return w


def hz_mode(nx, ny, m, l):
    """cos(m pi x / a) cos(l pi y / b) at the H_z positions ((i+1/2) dx, (j+1/2) dx)."""
    x = (np.arange(nx) + 0.5) / (nx - 1)
    y = (np.arange(ny) + 0.5) / (ny - 1)
    h = np.outer(np.cos(l * np.pi * y), np.cos(m * np.pi * x))
    h[-1, :] = 0.0
    h[:, -1] = 0.0
    return h


def ktilde2(nx, ny, m, l, dx):
    return 4.0 / dx ** 2 * (np.sin(m * np.pi / (2 * (nx - 1))) ** 2 + np.sin(l * np.pi / (2 * (ny - 1))) ** 2)


def test_layout_of_the_papers_2d_case(oracle_mod):
    """The paper's 2D TM case: a 100 nm design box at 0.5 nm (200 x 200
    cells) around a 10 nm observation box (20 x 20 cells) holds 79,560 design
    edges outside the observation box (Sec. 4.1); the 200 nm box with the
    same gap holds 319,960 (Sec. 4.1).  The oracle's layout counts them."""
    for side, free in ((200, 79560), (400, 319960)):
        n = side + 40
        lo = 20
        g0 = lo + (side - 20) // 2
        w = W.tiny_te(n=(n, n, 1), n_steps=1, pml_cells=6, tfsf_margin=4, design_lo=(lo, lo, 0),
                      design_n=(side, side, 1), gap_lo=(g0, g0, 0), gap_n=(20, 20, 1))
        o = oracle_mod.Oracle(w)
        assert o.nd - o.ng == free == W.te_edges((side, side), (20, 20))[2]
        o.close()


def test_yee_cavity_dispersion_closed_form(oracle_mod):
    """Source-free PEC cavity, H_z^{-1/2} a cavity mode and E^0 = 0:
    H_z^{n-1/2} = H_z^{-1/2} cos((n-1/2) w dt)/cos(w dt/2) with the Yee
    relation sin^2(w dt/2) = (v dt)^2 ktilde^2 / 4."""
    nx, ny, m, l = 24, 20, 2, 3
    w = cavity_te(nx, ny, omega_p=0.0, eps_inf=2.25, sigma_max=0.0)
    o = oracle_mod.Oracle(w)
    o.set_density(np.full(o.dshape, 0.3))
    H0 = hz_mode(nx, ny, m, l)
    z = np.zeros_like(H0)
    o.set_state(z, z, H0, z, z)
    dt = o.info()["dt"]
    v = C0 / np.sqrt(w["eps_s"])
    th = 2 * np.arcsin(v * dt * np.sqrt(ktilde2(nx, ny, m, l, w["dx"])) / 2)
    for n in (1, 7, 200, 2000):
        o.set_state(z, z, H0, z, z)
        o.step_free(n)
        Ex, Ey, Hz, _, _ = o.get_state()
        want = H0 * np.cos((n - 0.5) * th) / np.cos(th / 2)
        assert np.abs(Hz - want).max() < 1e-12 * np.abs(H0).max() * max(1, n / 100), n
        # PEC: tangential E stays zero on the walls
        assert np.all(Ex[0] == 0) and np.all(Ex[-1] == 0) and np.all(Ey[:, 0] == 0) and np.all(Ey[:, -1] == 0)
    # a plausible slip (a grading factor in the wrong place, a swapped
    # difference) would not keep this mode's shape: check E_y's shape too
    o.set_state(z, z, H0, z, z)
    o.step_free(1)
    Ex, Ey, _, _, _ = o.get_state()
    xi = np.arange(nx) / (nx - 1)
    yh = (np.arange(ny) + 0.5) / (ny - 1)
    shape_y = np.outer(np.cos(l * np.pi * yh), np.sin(m * np.pi * xi))
    shape_y[-1, :] = 0
    r = Ey[:-1, 1:-1] / shape_y[:-1, 1:-1]
    assert np.ptp(r[np.abs(shape_y[:-1, 1:-1]) > 0.2]) < 1e-12 * np.abs(r).max()


def test_lossless_drude_cavity_frequency(oracle_mod):
    """gamma = sigma = 0 with every edge metal: H_z^{n-1/2} is a pure
    sinusoid at sin^2(w dt/2) = (psi + c0^2 k^2)/(4 eps_inf/dt^2 + psi), the
    discrete form of eps_inf w^2 = psi + c0^2 k^2 (eq. (1) with gamma = 0)."""
    nx, ny, m, l = 18, 16, 2, 1
    w = cavity_te(nx, ny, gamma_mult=0.0, sigma_max=0.0, design_lo=(0, 0, 0), design_n=(nx - 1, ny - 1, 1),
                  pml_cells=0)
    o = oracle_mod.Oracle(w)
    o.set_density(np.ones(o.dshape))
    # E^0 = the discrete curl of a cavity mode of H_z (H = J = 0), which
    # leaves the static current mode of the lossless ADE unexcited
    H0 = hz_mode(nx, ny, m, l)
    Ex0 = np.zeros_like(H0)
    Ey0 = np.zeros_like(H0)
    Ex0[1:-1, :-1] = H0[1:-1, :-1] - H0[:-2, :-1]
    Ey0[:-1, 1:-1] = -(H0[:-1, 1:-1] - H0[:-1, :-2])
    z = np.zeros_like(H0)
    o.set_state(Ex0, Ey0, z, z, z)
    dt = o.info()["dt"]
    psi = w["omega_p"] ** 2
    s = (psi + C0 ** 2 * ktilde2(nx, ny, m, l, w["dx"])) / (4 * w["eps_inf"] / dt ** 2 + psi)
    cth = 1 - 2 * s
    e = [Ey0[5, 4]]
    for _ in range(300):
        o.step_free(1)
        e.append(o.get_state()[1][5, 4])
    e = np.array(e)
    assert np.abs(e).max() > 0
    r = e[2:] - 2 * cth * e[1:-1] + e[:-2]
    assert np.abs(r).max() < 1e-11 * np.abs(e).max()


def test_energy_identity_lossy_drude(oracle_mod):
    """PEC box, no absorber, no source: U^{n+1} - U^n = -dt sum[sigma Ebar^2 +
    gamma Jbar^2/(eps0 psi)] exactly over the E_x and E_y edges, with U^n =
    1/2 sum eps0 eps E^2 + 1/2 sum mu0 H_z^{n-1/2} H_z^{n+1/2} + sum
    J^2/(2 eps0 psi); U never grows."""
    nx, ny = 26, 22
    w = W.tiny_te(n=(nx, ny, 1), pml_cells=0, tfsf_margin=0, source="none",
                  design_lo=(6, 5, 0), design_n=(12, 10, 1), gap_lo=(2, 2, 0), gap_n=(1, 1, 1),
                  sigma_max=5e5, gamma_mult=16.0, weights="unit")
    o = oracle_mod.Oracle(w)
    rng = np.random.default_rng(3)
    rho = rng.random(o.dshape)
    o.set_density(rho)
    dt = o.info()["dt"]
    dnx, dny = 12, 10
    ndx = dnx * (dny + 1)
    masks, rhos = [], []
    for comp, (rows, cols) in enumerate(((dny + 1, dnx), (dny, dnx + 1))):
        m = np.zeros((ny, nx), bool)
        m[5:5 + rows, 6:6 + cols] = True
        masks.append(m)
        r = np.zeros((ny, nx))
        r[m] = rho[:ndx] if comp == 0 else rho[ndx:]
        rhos.append(r)
    psi = w["omega_p"] ** 2
    gam = w["gamma_mult"] * w["gamma_p"]

    def mat(comp):
        m, r = masks[comp], rhos[comp]
        eps = np.where(m, w["eps_s"] + r * (w["eps_inf"] - w["eps_s"]), w["eps_s"])
        ps = np.where(m, w["psi_s_ratio"] * psi + r * (1 - w["psi_s_ratio"]) * psi, 1.0)
        sg = np.where(m, r * (1 - r) * w["sigma_max"], 0.0)
        return eps, ps, sg

    Ex = W.box_smooth(rng.standard_normal((ny, nx)))
    Ey = W.box_smooth(rng.standard_normal((ny, nx)))
    Ex[0, :] = Ex[-1, :] = 0; Ex[:, -1] = 0
    Ey[:, 0] = Ey[:, -1] = 0; Ey[-1, :] = 0
    Hz = W.box_smooth(rng.standard_normal((ny, nx))) / 377
    Hz[-1, :] = 0; Hz[:, -1] = 0
    Jx = np.where(masks[0], rng.standard_normal((ny, nx)) * 1e3, 0.0)
    Jy = np.where(masks[1], rng.standard_normal((ny, nx)) * 1e3, 0.0)
    o.set_state(Ex, Ey, Hz, Jx, Jy)
    states = [(Ex, Ey, Hz, Jx, Jy)]
    for _ in range(60):
        o.step_free(1)
        states.append(tuple(o.get_state()))
    M = [mat(0), mat(1)]

    def U(n):
        s, sp = states[n], states[n + 1]
        u = 0.5 * MU0 * np.sum(s[2] * sp[2])
        for c in range(2):
            eps, ps, _ = M[c]
            u += 0.5 * np.sum(EPS0 * eps * s[c] ** 2) + np.sum(np.where(masks[c], s[3 + c] ** 2 / (2 * EPS0 * ps), 0))
        return u

    Us = [U(n) for n in range(len(states) - 1)]
    for n in range(len(Us) - 1):
        loss = 0.0
        for c in range(2):
            _, ps, sg = M[c]
            Eb = 0.5 * (states[n + 1][c] + states[n][c])
            Jb = 0.5 * (states[n + 1][3 + c] + states[n][3 + c])
            loss += dt * np.sum(sg * Eb ** 2 + np.where(masks[c], gam * Jb ** 2 / (EPS0 * ps), 0))
        assert abs((Us[n + 1] - Us[n]) + loss) <= 1e-11 * Us[0], (n, Us[n + 1] - Us[n], -loss)
        assert Us[n + 1] <= Us[n] * (1 + 1e-14)
    assert Us[-1] < Us[0]


def test_tfsf_no_scatterer_is_exact(oracle_mod):
    """Design = background (rho = 0, psi_s = 0): outside the total-field box
    the field stays at round-off, and inside it is a plane wave (E_x uniform
    along x, E_y zero)."""
    w = W.tiny_te(psi_s_ratio=0.0, sigma_max=0.0, n_steps=700)
    o = oracle_mod.Oracle(w)
    o.set_density(np.zeros(o.dshape))
    o.forward()
    ia, ib, ja, jb = o.info()["tf_box"][:4]
    Ex, Ey, Hz, _, _ = o.get_state()
    tf = Ex[ja:jb + 1, ia:ib]
    peak = np.abs(tf).max()
    assert peak > 0.1
    assert np.abs(tf - tf[:, :1]).max() < 1e-12 * peak
    assert np.abs(Ey).max() < 1e-12 * peak
    sf = Ex.copy()
    sf[ja:jb + 1, ia:ib] = 0
    assert np.abs(sf).max() < 1e-12 * peak
    hz = Hz.copy()
    hz[ja:jb, ia:ib] = 0
    assert np.abs(hz).max() < 1e-12 * peak / 377


@pytest.mark.parametrize("kappa,alpha", [(1.0, 0.0), (3.0, 0.05)])
def test_adjoint_dot_product_whole_run(oracle_mod, kappa, alpha):
    """<s, L q> = <L^T s, q> for random sources in both E equations: the
    Drude ADE on E_x and E_y edges, the absorber transpose (stretched and
    frequency-shifted grading) and the time-index bookkeeping."""
    w = W.tiny_te(n_steps=70, pml_kappa_max=kappa, pml_alpha_max=alpha)
    o = oracle_mod.Oracle(w)
    o.set_density(W.seeded_rho(w, 2))
    rng = np.random.default_rng(5)
    shape = (w["n_steps"], 2) + o.shape
    q = rng.standard_normal(shape)
    s = rng.standard_normal(shape)
    E = o.forward_ext(q)
    Es = o.adjoint_ext(s)
    lhs = np.sum(s * E)
    rhs = np.sum(q * Es)
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum((s * E) ** 2)) * np.sqrt(s.size), (lhs, rhs)


@pytest.mark.parametrize("over", [dict(), dict(sigma_max=0.0, gamma_mult=1.0), dict(objective="time_energy"),
                                  dict(pml_kappa_max=2.0, pml_alpha_max=0.05, source="sinc_hann")])
def test_gradient_matches_central_differences(oracle_mod, over):
    w = W.tiny_te(**over)
    o = oracle_mod.Oracle(w)
    rho = W.seeded_rho(w, 0)
    F, g = o.run(rho)
    ndx = o.ndx
    # E_x edges and E_y edges, inside and on the design box's boundary lines
    picks = [0, 5, 40, ndx - 1, ndx, ndx + 7, ndx + 60, o.nd - 1]
    h = 1e-4
    for d in picks:
        rp = rho.copy(); rp[d] += h
        rm = rho.copy(); rm[d] -= h
        o.set_density(rp); Fp = o.forward()
        o.set_density(rm); Fm = o.forward()
        fd = (Fp - Fm) / (2 * h)
        assert abs(g[d] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (d, g[d], fd)
    # gap edges (gap box 2 x 2 cells at design-local (5, 5)) carry no gradient
    dnx = w["design_n"][0]
    for (i, j) in [(5, 5), (6, 7)]:
        assert g[j * dnx + i] == 0.0
    assert g[ndx + 5 * (dnx + 1) + 7] == 0.0
    assert np.abs(g).max() > 0
