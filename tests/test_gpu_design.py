"""The design-update loop (paper_2203_01462_amd.design, include/fdtd_design.h)
on the GPU: the filter and its transpose against the CPU reference, the
transpose identity, one MMA step against a NumPy transcription of the same
formulas, GCMMA on a convex problem with a known minimizer, the statistics,
and a short optimization of a small 2D antenna (objective non-decreasing
within each continuation level, as GCMMA's conservative approximations
guarantee)."""
import numpy as np
import pytest

import fdtd_workloads as W
from oracle import filter as OF
from test_gpu_parity_2d import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    from paper_2203_01462_amd import design
    return torch, design


@pytest.mark.parametrize("shape,alpha", [((40, 33), 0.3), ((40, 33), 8.0), ((7, 12, 10), 0.05)])
def test_filter_matches_reference(D, shape, alpha):
    torch, design = D
    x = 0.05 + 0.9 * np.random.default_rng(1).random(shape)
    g = np.random.default_rng(2).random(shape) - 0.5
    f = design.Filter(shape, 2.5, torch.float64)
    y = f.apply(torch.tensor(x, device="cuda"), alpha).cpu().numpy()
    gt = f.transpose(torch.tensor(g, device="cuda")).cpu().numpy()
    yr, xs = OF.open_close(x, 2.5, alpha)
    gr = OF.open_close_transpose(xs, g, 2.5, alpha)
    assert np.abs(y - yr).max() <= 1e-12
    assert np.linalg.norm(gt - gr) <= 1e-12 * np.linalg.norm(gr)
    f.close()


def test_filter_fp32_close_to_fp64(D):
    torch, design = D
    shape = (64, 48)
    x = np.random.default_rng(3).random(shape)
    f32 = design.Filter(shape, 2.5, torch.float32)
    y32 = f32.apply(torch.tensor(x, dtype=torch.float32, device="cuda"), 0.1).cpu().numpy()
    yr, _ = OF.open_close(x, 2.5, 0.1)
    assert np.abs(y32 - yr).max() <= 1e-5


def mma_step_ref(x, xo1, xo2, Lo, Uo, df, f0, k, rho, move=0.5, s0=0.5, inc=1.2, dec=0.7):
    """One MMA step (Svanberg), box constraints [0, 1] only."""
    if k < 2:
        L, U = x - s0, x + s0
    else:
        s = (x - xo1) * (xo1 - xo2)
        g = np.where(s < 0, dec, np.where(s > 0, inc, 1.0))
        L = x - g * (xo1 - Lo)
        U = x + g * (Uo - xo1)
        L = np.minimum(np.maximum(L, x - 10), x - 0.01)
        U = np.maximum(np.minimum(U, x + 10), x + 0.01)
    lo = np.maximum(np.maximum(0.0, L + 0.1 * (x - L)), x - move)
    hi = np.minimum(np.minimum(1.0, U - 0.1 * (U - x)), x + move)
    gp, gm = np.maximum(df, 0), np.maximum(-df, 0)
    p = (U - x) ** 2 * (1.001 * gp + 0.001 * gm + rho)
    q = (x - L) ** 2 * (0.001 * gp + 1.001 * gm + rho)
    xs = np.clip((np.sqrt(p) * L + np.sqrt(q) * U) / (np.sqrt(p) + np.sqrt(q)), lo, hi)
    approx = f0 - np.sum(p / (U - x) + q / (x - L)) + np.sum(p / (U - xs) + q / (xs - L))
    dist = np.sum((U - L) * (xs - x) ** 2 / ((U - xs) * (xs - L)))
    return xs, approx, dist, L, U


def test_mma_steps_match_reference(D):
    torch, design = D
    n = 1000
    rng = np.random.default_rng(4)
    m = design.MMA(n, torch.float64)
    x = rng.random(n)
    xo1 = xo2 = Lo = Uo = None
    hist = []
    for k in range(4):
        df = rng.standard_normal(n)
        f0 = float(rng.standard_normal())
        rho0 = m.begin(torch.tensor(x, device="cuda"), f0, torch.tensor(df, device="cuda"))
        assert abs(rho0 - max(1e-6, 0.1 * np.abs(df).sum() / n)) <= 1e-12 * rho0
        xn = torch.empty(n, dtype=torch.float64, device="cuda")
        a, d = m.solve(rho0, xn)
        xs, ar, dr, L, U = mma_step_ref(x, xo1, xo2, Lo, Uo, df, f0, k, rho0)
        assert np.abs(xn.cpu().numpy() - xs).max() <= 1e-12
        assert abs(a - ar) <= 1e-10 * max(1, abs(ar)) and abs(d - dr) <= 1e-10 * max(1, abs(dr))
        m.accept(xn)
        xo2, xo1, x, Lo, Uo = xo1, x, xs, L, U
    m.close()


def test_gcmma_converges_on_a_convex_problem(D):
    """min sum_j (x_j - c_j)^4 + (x_j - c_j)^2 over [0,1]: minimizer clip(c, 0, 1)."""
    torch, design = D
    n = 500
    c = np.random.default_rng(5).random(n) * 1.6 - 0.3
    f = lambda x: float(np.sum((x - c) ** 4 + (x - c) ** 2))
    df = lambda x: 4 * (x - c) ** 3 + 2 * (x - c)
    m = design.MMA(n, torch.float64)
    x = np.full(n, 0.5)
    prev = f(x)
    for it in range(60):
        rho = m.begin(torch.tensor(x, device="cuda"), f(x), torch.tensor(df(x), device="cuda"))
        xn = torch.empty(n, dtype=torch.float64, device="cuda")
        for inner in range(20):
            a, d = m.solve(rho, xn)
            fn = f(xn.cpu().numpy())
            if fn <= a + 1e-14:
                break
            rho = min(1.1 * (rho + (fn - a) / d), 10 * rho)
        m.accept(xn)
        x = xn.cpu().numpy()
        assert f(x) <= prev + 1e-12   # conservative approximations: monotone
        prev = f(x)
    assert np.abs(x - np.clip(c, 0, 1)).max() < 1e-4
    m.close()


def test_design_stats(D):
    torch, design = D
    x = np.random.default_rng(6).random(777)
    g = np.random.default_rng(7).standard_normal(777)
    z, k = design.stats(torch.tensor(x, device="cuda"), torch.tensor(g, device="cuda"))
    assert abs(z - 4 * np.dot(x, 1 - x) / x.size) <= 1e-13
    assert abs(k - np.linalg.norm(x - np.clip(x - g, 0, 1))) <= 1e-12 * max(1, k)


def test_optimize_small_antenna(D):
    torch, design = D
    w = W.instance2d(96, 1.0, 600e-9, 800e-9, 700, precision=64, n_freq=4, name="opt2d")
    w = W.with_(w, sigma_max=5e5)
    levels = []
    res = design.optimize(w, max_iter=40, zeta_min=0.001, alphas=(8.0, 0.5, 0.1), gamma_levels=(4.0, 1.0),
                          level_min_iters=6, max_inner=40, callback=levels.append)
    h = res["history"]
    say(f"[design] {len(h)} records, F {h[0]['F']:.4e} -> {h[-1]['F']:.4e}, zeta {h[0]['zeta']:.3f} -> "
        f"{h[-1]['zeta']:.3f}, levels {sorted(set(r['level'] for r in h))}, thresholded F {res['F_final']:.4e}")
    for a, b in zip(h, h[1:]):
        if a["level"] == b["level"] and a.get("conservative"):
            assert b["F"] >= a["F"] * (1 - 1e-12), (a, b)
    assert sum(1 for r in h if r.get("conservative")) >= len([r for r in h if "inner" in r]) - 1
    assert h[-1]["F"] > h[0]["F"]
    rb = res["rho_binary"].cpu().numpy()
    assert set(np.unique(rb)) <= {0.0, 1.0}
    assert np.isfinite(res["F_final"]) and res["F_final"] > 0


def test_optimize_fixed_gap_metal_and_planar_tie(D):
    """The paper's 3D setting (Sec. 4.3): the metal boxes next to the gap
    held fixed and the design uniform along the slab's thin axis (z here):
    every iterate's density is 1 on the fixed cells and constant along z,
    the variables live on the (y, x) plane, and F rises."""
    torch, design = D
    w = W.tiny3d()
    fixed = design.gap_guard_mask(w)
    assert fixed.sum() == 2 * 2 * 2 * 2
    seen = []
    res = design.optimize(w, max_iter=8, zeta_min=0.0, alphas=(4.0,), gamma_levels=(4.0,), max_inner=20,
                          fixed=fixed, tie_axis=0, callback=seen.append)
    h = res["history"]
    say(f"[design] fixed + tied: F {h[0]['F']:.4e} -> {h[-1]['F']:.4e} over {len(h)} records")
    assert res["variables"].shape == (w["design_n"][1], w["design_n"][0])
    rf = res["rho_filtered"].cpu().numpy()
    assert np.all(rf[fixed] == 1.0)
    # off the fixed cells every column (y, x) holds one value along z
    free = np.where(fixed, np.nan, rf)
    assert np.nanmax(free, axis=0).tolist() == np.nanmin(free, axis=0).tolist()
    x = res["x"].cpu().numpy()
    assert np.array_equal(x, np.broadcast_to(x[:1], x.shape))
    assert h[-1]["F"] > h[0]["F"]
