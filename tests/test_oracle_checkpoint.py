"""The oracle's segment checkpointing (snapshots every K steps, segments
re-run in the adjoint on a second state) reproduces the stored-history
oracle bit for bit: the re-runs repeat the forward's arithmetic in the same
order, and the compact snapshots hold every non-zero value of the state.
This lets the oracle solve the full-size workloads, whose design-edge
history (eq. (25) reads E^n of every step) would not fit in host memory."""
import numpy as np
import pytest

import fdtd_workloads as W


def run(oracle_mod, w, rho, K):
    o = oracle_mod.Oracle(w, ckpt_every=K)
    F, g = o.run(rho)
    d = o.dft()
    o.close()
    return F, g, d


@pytest.mark.parametrize("over", [dict(), dict(objective="time_energy"),
                                  dict(pml_kappa_max=3.0, pml_alpha_max=0.05)])
def test_checkpoint_2d_bit_identical(oracle_mod, over):
    w = W.tiny2d(n_steps=400, **over)
    rho = W.seeded_rho(w, 1)
    F0, g0, d0 = run(oracle_mod, w, rho, 0)
    assert np.any(g0 != 0)
    for K in (1, 7, 100, 399, 400, 1000):
        F, g, d = run(oracle_mod, w, rho, K)
        assert F == F0 and np.array_equal(g, g0) and np.array_equal(d, d0), K


def test_checkpoint_3d_bit_identical(oracle_mod):
    w = W.tiny3d(n_steps=300, pml_kappa_max=2.0, pml_alpha_max=0.02)
    rho = W.seeded_rho(w, 2)
    F0, g0, d0 = run(oracle_mod, w, rho, 0)
    assert np.any(g0 != 0)
    for K in (1, 64, 299):
        F, g, d = run(oracle_mod, w, rho, K)
        assert F == F0 and np.array_equal(g, g0) and np.array_equal(d, d0), K


def test_checkpoint_repeated_solves(oracle_mod):
    """Two densities in turn on one checkpointed instance: every solve starts
    from zero state and fresh snapshots."""
    w = W.tiny2d(n_steps=300)
    ra, rb = W.seeded_rho(w, 0), W.seeded_rho(w, 0, "binary")
    o = oracle_mod.Oracle(w, ckpt_every=70)
    Fa, ga = o.run(ra)
    Fb, gb = o.run(rb)
    Fa2, ga2 = o.run(ra)
    o.close()
    Fa0, ga0, _ = run(oracle_mod, w, ra, 0)
    Fb0, gb0, _ = run(oracle_mod, w, rb, 0)
    assert Fa == Fa0 == Fa2 and Fb == Fb0
    assert np.array_equal(ga, ga0) and np.array_equal(ga2, ga0) and np.array_equal(gb, gb0)
