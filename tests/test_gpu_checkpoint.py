"""Checkpointed adjoint (ckpt_every = K > 0): full-state snapshots every K
steps and segment re-runs in the adjoint give the same objective and the same
gradient, bit for bit, as the stored full history (the kernels are
deterministic and the re-run repeats the forward's arithmetic exactly), for
ragged last segments, K = 1, K >= N, both precisions and both dimensions,
with the re-runs overlapping the adjoint on a second stream (two history
buffers) and without (a budget for one).  Calls go through the C ABI."""
import numpy as np
import pytest

import fdtd_workloads as W
from test_gpu_parity_2d import gpu, say  # noqa: F401

pytestmark = pytest.mark.gpu


def run(gpu, w, rho, K):
    g = gpu.FDTD(w, ckpt_every=K)
    F, grad = g.run(rho.astype(g.dtype))
    dft = g.dft()
    g.close()
    return F, grad, dft


def check_same(gpu, w, Ks, seed=0):
    rho = W.seeded_rho(w, seed)
    F0, g0, d0 = run(gpu, w, rho, 0)
    assert np.any(g0 != 0)
    for K in Ks:
        F, g, d = run(gpu, w, rho, K)
        say(f"[ckpt] {w['name']} prec={w['precision']} N={w['n_steps']} K={K}: F {F:.15e} vs {F0:.15e}, "
            f"max|dg|={np.abs(g - g0).max():.3e}")
        assert F == F0
        assert np.array_equal(d, d0)
        assert np.array_equal(g, g0)


@pytest.mark.parametrize("prec", [64, 32])
def test_tiny2d_checkpoint_bit_identical(gpu, prec):
    w = W.tiny2d(precision=prec)
    N = w["n_steps"]
    check_same(gpu, w, [1, 7, 250, N - 1, N, N + 5])


def test_tiny2d_checkpoint_variants(gpu):
    for over in (dict(objective="time_energy"), dict(pml_kappa_max=3.0, pml_alpha_max=0.05)):
        check_same(gpu, W.tiny2d(**over), [97])


@pytest.mark.parametrize("prec", [64, 32])
def test_tiny3d_checkpoint_bit_identical(gpu, prec):
    w = W.tiny3d(precision=prec)
    check_same(gpu, w, [1, 64, w["n_steps"] - 1])


def test_medium3d_checkpoint_bit_identical(gpu):
    check_same(gpu, W.medium3d(precision=32), [128])


def test_medium2d_checkpoint_bit_identical(gpu):
    check_same(gpu, W.medium2d(), [500])


def test_checkpoints_fit_where_the_full_history_does_not(gpu):
    # a long run: 4000 steps of design-edge history (36.9 MB) against seven
    # snapshots of the whole state (2.08 MB each) plus 500 steps of history
    # (4.6 MB); budget 27.6 MB
    w = W.tiny3d(n_steps=4000)
    nd = int(np.prod(w["design_n"]))
    full = w["n_steps"] * 3 * nd * 8
    with pytest.raises(gpu.FDTDError) as e:
        gpu.FDTD(w, history_budget_bytes=3 * full // 4)
    assert e.value.name == "ENOMEM"
    g = gpu.FDTD(w, history_budget_bytes=3 * full // 4, ckpt_every=500)
    F, grad = g.run(W.seeded_rho(w, 0))
    g.close()
    assert np.isfinite(F) and np.all(np.isfinite(grad))


@pytest.mark.parametrize("dims", [2, 3])
def test_checkpoint_with_one_history_buffer(gpu, dims):
    """A budget that holds one K-step history but not two (two K-step
    segments; the history dominates the one snapshot): the re-run stays on
    the context stream instead of overlapping the adjoint.  Still bit for bit
    the stored-history result."""
    w = W.tiny2d(n_steps=4400) if dims == 2 else W.tiny3d(n_steps=3600)
    K = w["n_steps"] // 2
    hist = K * (1 if dims == 2 else 3) * int(np.prod(w["design_n"])) * 8
    rho = W.seeded_rho(w, 0)
    F0, g0, d0 = run(gpu, w, rho, 0)
    g = gpu.FDTD(w, ckpt_every=K, history_budget_bytes=int(1.4 * hist))
    F, grad = g.run(rho.astype(g.dtype))
    d = g.dft()
    g.close()
    say(f"[ckpt] one history buffer, {dims}D, K={K}: F {F:.15e} vs {F0:.15e}")
    assert F == F0 and np.array_equal(grad, g0) and np.array_equal(d, d0)


def test_c3_checkpoint_every_500_matches_stored_history(gpu):
    """The 256^3 x 8000-step FP32 workload with a checkpoint every 500 steps."""
    w = W.c3()
    rho = W.seeded_rho(w, 0).astype(np.float32)
    say("[ckpt] C3 full: stored history")
    F0, g0, d0 = run(gpu, w, rho, 0)
    say("[ckpt] C3 full: checkpoint every 500")
    F, g, d = run(gpu, w, rho, 500)
    say(f"   F {F:.9e} vs {F0:.9e}, max|dg|={np.abs(g - g0).max():.3e}")
    assert F == F0 and np.array_equal(g, g0) and np.array_equal(d, d0)


def test_medium2d_checkpoint_after_recycled_memory(gpu):
    """Regression: every buffer the checkpointed re-runs read before writing
    (the wall nodes of all three field copies of the two-step schedule) is
    cleared at create.  A first context fills its device memory with non-zero
    fields and is destroyed, so the next context's allocations are likely to
    reuse that memory; the checkpointed result must still equal the stored
    history bit for bit."""
    w = W.medium2d(precision=64)
    rho = W.seeded_rho(w, 0)
    F0, g0, d0 = run(gpu, w, rho, 0)
    for _ in range(2):
        dirty = gpu.FDTD(w, ckpt_every=500)
        dirty.run(rho)  # fields, absorber memories and re-run copies all non-zero
        dirty.close()
        F, g, d = run(gpu, w, rho, 500)
        say(f"[ckpt] recycled memory: F {F:.15e} vs {F0:.15e}")
        assert F == F0 and np.array_equal(g, g0) and np.array_equal(d, d0)
