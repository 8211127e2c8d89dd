"""Two-step blocking of the 2D background against the per-step update.

A single 2D context advances the plain background two steps per pass and the
other tiles one step per launch; a one-instance batch (same tile depth) runs
the per-step kernel everywhere.  The two-step pass uses the per-step
expressions, so in FP64 the objective and the gradient agree to the last
bit -- with an odd step
count (a final single step) and with checkpoint intervals that put pairs and
single steps at every segment edge and into the re-run segments.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def super_tiles(w):
    """Number of 64 x 16 super-tiles whose reach (three nodes) holds only the
    background: the blocked path is exercised only where this is positive."""
    nx, ny, _ = w["n"]
    P, m = w["pml_cells"], w["tfsf_margin"]
    ia, ib, ja, jb = P + m, nx - 1 - P - m, P + m, ny - 1 - P - m
    d0, dn, g0, gn = w["design_lo"], w["design_n"], w["gap_lo"], w["gap_n"]

    def meets(a0, a1, b0, bn):
        return bn > 0 and a1 >= b0 and a0 <= b0 + bn - 1

    count = 0
    for sy in range(ny // 16):
        for tx in range((nx + 63) // 64):
            x0, x1, y0, y1 = tx * 64 - 3, tx * 64 + 66, sy * 16 - 3, sy * 16 + 18
            ok = tx * 64 + 64 <= nx and x0 >= P + 2 and x1 <= nx - 3 - P and y0 >= P + 2 and y1 <= ny - 3 - P
            ok = ok and not any(x0 <= v <= x1 for v in (ia - 1, ia, ib, ib + 1))
            ok = ok and not any(y0 <= v <= y1 for v in (ja - 1, ja, jb, jb + 1))
            ok = ok and not (meets(x0, x1, d0[0], dn[0]) and meets(y0, y1, d0[1], dn[1]))
            ok = ok and not (meets(x0, x1, g0[0], gn[0]) and meets(y0, y1, g0[1], gn[1]))
            count += ok
    return count


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_01462_amd as P
    return P


@pytest.mark.parametrize("n_steps", [1201, 1200])
def test_blocked_schedule_bit_identical_to_per_step(gpu, n_steps):
    import fdtd_workloads as W
    w = W.with_(W.medium2d(precision=64), n_steps=n_steps)
    assert super_tiles(w) > 100
    rho = W.seeded_rho(w, 3)
    # two rows per thread, the single context's per-step variant (the row
    # variants form the FP64 sensitivity sums in different orders), one step
    # per launch
    b = gpu.Batch([w], rows=2, depth=1)
    b.set_density(0, rho)
    F_ref = float(b.forward()[0])
    b.adjoint()
    g_ref = b.gradient(0)
    b.close()
    for K in (0, 7, 50, n_steps - 1):
        g = gpu.FDTD(w, ckpt_every=K)
        F, grad = g.run(rho)
        g.close()
        print(f"[blocking] N={n_steps} K={K}: F {F:.17e} vs {F_ref:.17e}", flush=True)
        assert F == F_ref, (K, F, F_ref)
        assert np.array_equal(grad, g_ref), K


def test_blocked_schedule_bit_identical_full_size(gpu):
    """The 2048^2 workload's grid and physics in FP64, 6001 steps (the pulse
    peak reaches the gap; an odd count ends on a single step): the single
    context's blocked schedule, with its super-tile and rest lists in XCD order
    at this size, against the one-instance per-step batch, to the last bit;
    also with checkpoints every 1000 steps (segment re-runs beside the
    adjoint sweep)."""
    import fdtd_workloads as W
    w = W.with_(W.c2(), precision=64, n_steps=6001)
    assert super_tiles(w) > 3000
    rho = W.seeded_rho(w, 0)
    print("[blocking] 2048^2 fp64 x 6001: per-step batch reference", flush=True)
    b = gpu.Batch([w], rows=2, depth=1)
    b.set_density(0, rho)
    F_ref = float(b.forward()[0])
    b.adjoint()
    g_ref = b.gradient(0)
    b.close()
    assert F_ref > 0 and np.abs(g_ref).max() > 0
    for K in (0, 1000):
        g = gpu.FDTD(w, ckpt_every=K)
        F, grad = g.run(rho)
        g.close()
        print(f"[blocking] 2048^2 K={K}: F {F:.17e} vs {F_ref:.17e}", flush=True)
        assert F == F_ref, (K, F, F_ref)
        assert np.array_equal(grad, g_ref), K


def solve_3d(gpu, w, rho, K, blocking):
    """Forward (objective, gap DFT, final state) and adjoint (gradient) of one
    3D context created with the two-step pass on or off."""
    import os
    old = os.environ.get("FDTD_TEMPORAL_BLOCKING")
    os.environ["FDTD_TEMPORAL_BLOCKING"] = "1" if blocking else "0"
    try:
        g = gpu.FDTD(w, ckpt_every=K)
    finally:
        if old is None:
            del os.environ["FDTD_TEMPORAL_BLOCKING"]
        else:
            os.environ["FDTD_TEMPORAL_BLOCKING"] = old
    g.set_density(rho.astype(g.dtype))
    F = g.forward()
    d = g.dft()
    st = g.get_state()
    g.adjoint()
    grad = g.gradient()
    g.close()
    return F, d, st, grad


@pytest.mark.parametrize("n_steps,K", [(1201, 0), (1200, 0), (1201, 300), (1200, 7)])
def test_3d_two_step_bit_identical_to_per_step(gpu, n_steps, K):
    """The 256^3 workload's grid in FP32 with the 3D two-step pass switched
    on (765 super-chunks of 60 x 16 x 8 nodes, 35% of the nodes, advance two
    steps per pass, on a stream of their own beside the first per-step
    update): objective, gap DFT, the whole final state and the gradient equal
    those of the per-step schedule (the 3D default) to the last bit -- odd
    and even step counts, with and without checkpoint segments (segment
    edges at odd steps, re-runs on the second state)."""
    import fdtd_workloads as W
    w = W.with_(W.c3(), n_steps=n_steps)
    rho = W.seeded_rho(w, 1)
    print(f"[blocking3d] 256^3 fp32 N={n_steps} K={K}: per-step reference", flush=True)
    F0, d0, s0, g0 = solve_3d(gpu, w, rho, K, False)
    print(f"[blocking3d] 256^3 fp32 N={n_steps} K={K}: two-step", flush=True)
    F1, d1, s1, g1 = solve_3d(gpu, w, rho, K, True)
    print(f"   F {F1:.9e} vs {F0:.9e}; max|state| {np.abs(s0).max():.3e}", flush=True)
    assert F0 > 0 and np.abs(g0).max() > 0 and np.abs(s0).max() > 0
    assert F1 == F0
    assert np.array_equal(d1, d0)
    assert np.array_equal(s1, s0)
    assert np.array_equal(g1, g0)
