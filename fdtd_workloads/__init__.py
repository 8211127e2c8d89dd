"""Seeded synthetic inputs shared by the oracle tests, the HIP parity tests and bench.py.

This module holds no arithmetic of the method: only the problem descriptions
(grid sizes, spacings, material constants, box positions, band edges) and the
seeded density generator.  Every derived quantity (time step, absorber
profiles, incident-field tables, DFT phasors, weights, update coefficients) is
computed separately by each implementation.

Workloads follow the problem statement of the paper (Sec. 2, eqs. (1)-(5)):
a Yee grid, a per-cell density rho in [0,1] on a design box that interpolates
between the background dielectric and a Drude metal, a gap region where the
field is observed, a plane-wave pulse and an objective on the DFT of the gap
field over a band.  The paper's own geometries need its optimized designs; the
densities here are seeded box-smoothed uniform noise of the same shape.
"""
from __future__ import annotations

import copy

import numpy as np

# Drude and dielectric constants of the synthetic workloads.
DRUDE = dict(eps_inf=1.0, omega_p=1.37e16, gamma_p=4.08e13)
# The paper's silver fit over 350-1000 nm (Sec. 2): eps_inf, omega_p, gamma_p.
SILVER_PAPER = dict(eps_inf=4.469, omega_p=1.426e16, gamma_p=4.571e13)

_COMMON = dict(
    courant=0.5,
    pml_order=3.0,
    pml_sigma_scale=1.0,
    pml_kappa_max=1.0,
    pml_alpha_max=0.0,
    eps_s=2.25,
    eps_g=2.25,
    gamma_mult=1.0,
    sigma_max=0.0,
    psi_s_ratio=0.01,
    source="gauss",
    t0_over_tau=4.0,
    amplitude=1.0,
    objective="dft",
    weights="enhancement",
    freqs_hz=None,
    periodic_x=False,
    **DRUDE,
)


def _centered(n, m):
    return (n - m) // 2


def c1():
    """2D TMz FP64 200x200, dx=5 nm, 20-cell CPML, 60x60 design, point gap, 2000 steps, K=8."""
    w = dict(_COMMON)
    w.update(name="tmz2d_200_fp64", dims=2, precision=64, n=(200, 200, 1), dx=5e-9,
             n_steps=2000, pml_cells=20, tfsf_margin=5,
             design_lo=(70, 70, 0), design_n=(60, 60, 1),
             gap_lo=(100, 100, 0), gap_n=(1, 1, 1),
             lambda_lo=500e-9, lambda_hi=1000e-9, n_freq=8)
    return w


def c2(gamma_mult=1.0):
    """2D TMz FP32 2048x2048, dx=2 nm, 32-cell CPML, 512x512 design, 5x5 gap, 20000 steps, K=16."""
    w = dict(_COMMON)
    w.update(name="tmz2d_2048_fp32", dims=2, precision=32, n=(2048, 2048, 1), dx=2e-9,
             n_steps=20000, pml_cells=32, tfsf_margin=8,
             design_lo=(768, 768, 0), design_n=(512, 512, 1),
             gap_lo=(1022, 1022, 0), gap_n=(5, 5, 1),
             lambda_lo=500e-9, lambda_hi=1000e-9, n_freq=16, gamma_mult=gamma_mult)
    return w


def c3():
    """3D FP32 256^3, dx=2 nm, 16-cell CPML, 128x128x32 slab, 4^3 gap, x-pol along +z, 8000 steps, K=16."""
    w = dict(_COMMON)
    w.update(name="yee3d_256_fp32", dims=3, precision=32, n=(256, 256, 256), dx=2e-9,
             n_steps=8000, pml_cells=16, tfsf_margin=6,
             design_lo=(64, 64, 112), design_n=(128, 128, 32),
             gap_lo=(126, 126, 126), gap_n=(4, 4, 4),
             lambda_lo=600e-9, lambda_hi=900e-9, n_freq=16)
    return w


def medium2d(**over):
    """512x512 2D TMz FP32 with the 2048^2 workload's physics (dx = 2 nm,
    32-cell CPML, 5x5 gap, K = 16) and a 96x96 design box, run long enough
    for the pulse to reach the gap; sized for the oracle to finish in seconds."""
    w = dict(_COMMON)
    w.update(name="tmz2d_512_fp32", dims=2, precision=32, n=(512, 512, 1), dx=2e-9,
             n_steps=3600, pml_cells=32, tfsf_margin=8, t0_over_tau=3.0,
             design_lo=(208, 120, 0), design_n=(96, 96, 1),
             gap_lo=(254, 166, 0), gap_n=(5, 5, 1),
             lambda_lo=500e-9, lambda_hi=1000e-9, n_freq=16)
    w.update(over)
    return w


def medium3d(**over):
    """80^3 3D case large enough to hold plain-background blocks as well as
    absorber, injection, design and gap blocks; sized for the oracle."""
    w = dict(_COMMON)
    w.update(name="yee3d_80", dims=3, precision=64, n=(80, 80, 80), dx=5e-9,
             n_steps=900, pml_cells=6, tfsf_margin=3, t0_over_tau=3.0,
             design_lo=(30, 30, 35), design_n=(20, 20, 10),
             gap_lo=(39, 39, 39), gap_n=(2, 2, 2),
             lambda_lo=600e-9, lambda_hi=900e-9, n_freq=8)
    w.update(over)
    return w


def tiny2d(**over):
    """Small 2D TMz case exercising every feature: CPML, plane wave, Drude design, gap."""
    w = dict(_COMMON)
    w.update(name="tmz2d_tiny", dims=2, precision=64, n=(40, 44, 1), dx=5e-9,
             n_steps=1100, pml_cells=6, tfsf_margin=2, t0_over_tau=3.0,
             design_lo=(14, 16, 0), design_n=(12, 12, 1),
             gap_lo=(19, 21, 0), gap_n=(2, 2, 1),
             lambda_lo=500e-9, lambda_hi=1000e-9, n_freq=4,
             sigma_max=5e5, gamma_mult=4.0)
    w.update(over)
    return w


def tiny3d(**over):
    """Small 3D case exercising every feature."""
    w = dict(_COMMON)
    w.update(name="yee3d_tiny", dims=3, precision=64, n=(24, 24, 28), dx=5e-9,
             n_steps=900, pml_cells=5, tfsf_margin=2, t0_over_tau=3.0,
             design_lo=(8, 8, 11), design_n=(8, 8, 6),
             gap_lo=(11, 11, 13), gap_n=(2, 2, 2),
             lambda_lo=500e-9, lambda_hi=1000e-9, n_freq=4,
             sigma_max=5e5, gamma_mult=4.0)
    w.update(over)
    return w


def tiny_te(**over):
    """Small 2D TEz case (E in the plane, along x; H along z; plane wave along
    +y), the paper's plasmonic 2D polarization, with every feature: CPML,
    plane wave, Drude design edges, gap."""
    w = tiny2d(name="te2d_tiny", pol_axis="x")
    w.update(over)
    return w


def medium_te(**over):
    """384x384 TEz FP32 case with the 2048^2 workload's physics (dx = 2 nm,
    16-cell CPML, K = 16) and a 96x96 design box around a 6x6 gap, run long
    enough for the pulse to reach the gap; sized for the oracle."""
    w = dict(_COMMON)
    w.update(name="te2d_384_fp32", dims=2, precision=32, n=(384, 384, 1), dx=2e-9,
             n_steps=2400, pml_cells=16, tfsf_margin=6, t0_over_tau=3.0,
             design_lo=(144, 144, 0), design_n=(96, 96, 1),
             gap_lo=(189, 189, 0), gap_n=(6, 6, 1),
             lambda_lo=500e-9, lambda_hi=1000e-9, n_freq=16, pol_axis="x")
    w.update(over)
    return w


def te_edges(design_n, gap_n=(0, 0)):
    """Edge counts of the TEz design layout: a box of nx x ny cells holds
    nx (ny + 1) E_x edges and (nx + 1) ny E_y edges, both boundary lines
    included; returns (E_x edges, all edges, edges that are not in a gap box
    of gap_n cells lying inside it)."""
    nx, ny = design_n[0], design_n[1]
    gx, gy = gap_n[0], gap_n[1]
    ndx = nx * (ny + 1)
    nd = ndx + (nx + 1) * ny
    ng = gx * (gy + 1) + (gx + 1) * gy if gx > 0 and gy > 0 else 0
    return ndx, nd, nd - ng


def is_te(w):
    return w["dims"] == 2 and w.get("pol_axis") == "x"


def instance2d(side, gamma_mult, lambda_lo, lambda_hi, n_steps, precision=32, n_freq=8, name=None):
    """One square 2D TMz instance with the 2048^2 workload's physics (dx = 2 nm,
    eps_s = 2.25, Drude metal), scaled to its side: 16-cell CPML, a centred
    design box of side/4 and a 3x3 gap at its centre."""
    w = dict(_COMMON)
    m = max(side // 4, 8)
    lo = _centered(side, m)
    g = lo + m // 2 - 1
    w.update(name=name or f"tmz2d_{side}_b", dims=2, precision=precision, n=(side, side, 1), dx=2e-9,
             n_steps=n_steps, pml_cells=16, tfsf_margin=6, t0_over_tau=3.0,
             design_lo=(lo, lo, 0), design_n=(m, m, 1), gap_lo=(g, g, 0), gap_n=(3, 3, 1),
             lambda_lo=lambda_lo, lambda_hi=lambda_hi, n_freq=n_freq, gamma_mult=gamma_mult)
    return w


def c4(count=64, n_steps=5000, seed=0, sides=(128, 256, 512, 1024)):
    """Batched uneven 2D FP32: `count` TMz instances with sides drawn from
    `sides`, collision-rate multipliers uniform in [1, 16] and an 8-frequency
    band of at least 100 nm inside 500-1000 nm, `n_steps` steps each."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        side = int(rng.choice(sides))
        gm = float(rng.uniform(1.0, 16.0))
        a = float(rng.uniform(500e-9, 900e-9))
        b = float(rng.uniform(a + 100e-9, 1000e-9))
        out.append(instance2d(side, gm, a, b, n_steps, name=f"tmz2d_{side}_b{k}"))
    return out


def c5(n_steps=5000):
    """Surrogate workload: one 512x512 TMz FP32 instance with the 2048^2
    workload's physics (m_gamma = 1, 500-1000 nm band, 8 frequencies) and a
    128x128 design box, the size the surrogate network maps."""
    return instance2d(512, 1.0, 500e-9, 1000e-9, n_steps, name="tmz2d_512_c5")


def _logistic(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def random_designs(count, shape, seed):
    """`count` seeded design-variable maps in [0, 1] of `shape` (float32), a
    mix of the kinds an optimizer visits: near-uniform fields with weak
    structure, smooth fields of random correlation length (2-24 cells) and
    contrast, and sharpened, nearly binary ones.  Gaussian smoothing of white
    noise in the Fourier domain, then a logistic map of random slope and
    offset; one generator draws every number."""
    rng = np.random.default_rng(seed)
    ny, nx = shape
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    k2 = ky * ky + kx * kx
    out = np.empty((count, ny, nx), np.float32)
    for i in range(count):
        ell = rng.uniform(2.0, 24.0)
        noise = rng.standard_normal((ny, nx))
        f = np.real(np.fft.ifft2(np.fft.fft2(noise) * np.exp(-2.0 * (np.pi * ell) ** 2 * k2)))
        f -= f.mean()
        f /= max(f.std(), 1e-12)
        kind = rng.random()
        if kind < 0.3:      # near-uniform start region
            x = 0.5 + rng.uniform(0.0, 0.25) * np.tanh(f) + rng.uniform(-0.2, 0.2)
        elif kind < 0.75:   # smooth, intermediate contrast
            x = _logistic(rng.uniform(0.5, 3.0) * f + rng.uniform(-1.5, 1.5))
        else:               # nearly binary
            x = _logistic(rng.uniform(6.0, 30.0) * f + rng.uniform(-3.0, 3.0))
        out[i] = np.clip(x, 0.0, 1.0)
    return out


def te2048():
    """2D TEz FP32 2048x2048 with the 2048^2 TMz workload's physics and boxes
    (512x512-cell design box: 525,312 design edges; 5x5-cell gap: 60 gap
    edges), 20000 steps: the in-plane polarization at the benchmark size."""
    w = c2()
    w.update(name="te2d_2048_fp32", pol_axis="x")
    return w


PRESETS = {"c1": c1, "c2": c2, "c3": c3, "medium2d": medium2d, "medium3d": medium3d, "tiny2d": tiny2d,
           "tiny3d": tiny3d, "c5": c5, "te": te2048, "tiny_te": tiny_te, "medium_te": medium_te}


def with_(w, **over):
    """Copy of workload ``w`` with fields replaced."""
    x = copy.deepcopy(w)
    x.update(over)
    return x


def design_shape(w):
    """Array shape of the density over the design box: [z][y][x] in 3D, [y][x] in 2D
    TMz; in 2D TEz one value per design edge (E_x edges, then E_y edges)."""
    nx, ny, nz = w["design_n"]
    if is_te(w):
        return (te_edges(w["design_n"])[1],)
    return (nz, ny, nx) if w["dims"] == 3 else (ny, nx)


def box_smooth(a):
    """Mean over a 3-wide box along every axis with edge-replicate padding."""
    p = np.pad(a, 1, mode="edge")
    out = np.zeros_like(a)
    if a.ndim == 2:
        for dy in range(3):
            for dx in range(3):
                out += p[dy:dy + a.shape[0], dx:dx + a.shape[1]]
        return out / 9.0
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += p[dz:dz + a.shape[0], dy:dy + a.shape[1], dx:dx + a.shape[2]]
    return out / 27.0


def seeded_rho(w, seed, kind="smooth"):
    """Seeded density over the design box, float64.

    kind: "smooth"  U[0,1) from ``numpy.random.default_rng(seed)``, box-smoothed, clipped;
          "half"    rho = 0.5 everywhere (the paper's initial design);
          "binary"  the smooth field thresholded at 0.5;
          "zero"/"one" constant fields.
    """
    shape = design_shape(w)
    if is_te(w) and kind in ("smooth", "binary"):
        # the E_x block ([ny+1][nx]) and the E_y block ([ny][nx+1]), each drawn
        # and smoothed as a 2D field
        nx, ny, _ = w["design_n"]
        rng = np.random.default_rng(seed)
        bx = np.clip(box_smooth(rng.random((ny + 1, nx))), 0.0, 1.0)
        by = np.clip(box_smooth(rng.random((ny, nx + 1))), 0.0, 1.0)
        r = np.concatenate([bx.ravel(), by.ravel()])
        return (r >= 0.5).astype(np.float64) if kind == "binary" else r
    if kind == "half":
        return np.full(shape, 0.5)
    if kind == "zero":
        return np.zeros(shape)
    if kind == "one":
        return np.ones(shape)
    r = np.random.default_rng(seed).random(shape)
    r = np.clip(box_smooth(r), 0.0, 1.0)
    if kind == "binary":
        return (r >= 0.5).astype(np.float64)
    if kind != "smooth":
        raise ValueError(f"unknown density kind {kind!r}")
    return r


def cell_updates(w, include_adjoint=True):
    """Cells x steps (x2 with the adjoint solve): the unit of the throughput metric."""
    nx, ny, nz = w["n"]
    cells = nx * ny * (nz if w["dims"] == 3 else 1)
    return cells * w["n_steps"] * (2 if include_adjoint else 1)
