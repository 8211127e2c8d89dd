"""Host-side pieces of the surrogate: the seeded design generator, the U-Net
layer plan and the workspace query of the weight-gradient kernels (no GPU)."""
import numpy as np
import pytest

import fdtd_workloads as W


def test_random_designs_seeded_and_in_range():
    a = W.random_designs(24, (32, 48), seed=7)
    b = W.random_designs(24, (32, 48), seed=7)
    c = W.random_designs(24, (32, 48), seed=8)
    assert a.shape == (24, 32, 48) and a.dtype == np.float32
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.0 and a.max() <= 1.0
    # a mix of kinds: some nearly uniform designs and some nearly binary ones
    spread = a.reshape(24, -1).std(axis=1)
    binary = ((a < 0.05) | (a > 0.95)).reshape(24, -1).mean(axis=1)
    assert spread.min() < 0.15 and binary.max() > 0.8


def test_c5_workload_shape():
    w = W.c5()
    assert w["n"] == (512, 512, 1) and w["design_n"] == (128, 128, 1)
    assert w["precision"] == 32 and w["dims"] == 2
    lo, n = w["design_lo"], w["design_n"]
    g = w["gap_lo"]
    assert lo[0] <= g[0] < lo[0] + n[0] and lo[1] <= g[1] < lo[1] + n[1]


def test_layer_plan():
    nn = pytest.importorskip("paper_2203_01462_amd.nn")
    plan = nn.layer_plan((32, 64, 128, 256))
    assert len(plan) == 15
    # encoder
    assert plan[:8] == [(1, 32, 0), (32, 32, 0), (32, 64, 1), (64, 64, 1), (64, 128, 2), (128, 128, 2),
                        (128, 256, 3), (256, 256, 3)]
    # decoder: concatenation of the upsampled level below and the skip
    assert plan[8:14] == [(384, 128, 2), (128, 128, 2), (192, 64, 1), (64, 64, 1), (96, 32, 0), (32, 32, 0)]
    assert plan[14] == (32, 1, 0)
    weights = sum(ci * co * 9 + co for ci, co, _ in plan) + 256 + 1
    assert weights == 1_946_818  # summed by hand per layer: 1.95 M parameters


def test_wgrad_workspace_query():
    fdtd = pytest.importorskip("paper_2203_01462_amd.fdtd")
    try:
        L = fdtd.load_library()
    except ImportError:
        pytest.skip("library not built")
    for n, cin, cout, h, w in [(32, 32, 32, 128, 128), (1, 1, 32, 128, 128), (3, 5, 70, 13, 11),
                               (32, 256, 256, 16, 16)]:
        need = L.fdtd_nn_wgrad_work(n, cin, cout, h, w)
        assert need >= cout * cin * 9 + cout
    assert L.fdtd_nn_wgrad_work(0, 1, 1, 4, 4) == 0
    assert L.fdtd_nn_mse_work(1000) == 4 and L.fdtd_nn_mse_work(0) == 0
