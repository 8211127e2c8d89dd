"""Host-side helpers of the design loop: the mask of the metal held fixed
next to the gap (Sec. 4.1, 4.3)."""
import numpy as np
import pytest

import fdtd_workloads as W

design = pytest.importorskip("paper_2203_01462_amd.design")


@pytest.mark.parametrize("wl,axis", [("tiny3d", None), ("tiny3d", 1), ("c5", None), ("c5", 1)])
def test_gap_guard_mask_boxes(wl, axis):
    w = W.tiny3d() if wl == "tiny3d" else W.c5(100)
    m = design.gap_guard_mask(w, axis)
    d0, dn, g0, gn = w["design_lo"], w["design_n"], w["gap_lo"], w["gap_n"]
    dims = w["dims"]
    a = 0 if axis is None else axis
    assert m.shape == ((dn[2], dn[1], dn[0]) if dims == 3 else (dn[1], dn[0]))
    # two boxes of the gap's size, one on each side along the axis, off the gap
    assert m.sum() == 2 * int(np.prod([gn[k] for k in range(dims)]))
    idx = np.argwhere(m)[:, ::-1]  # (x, y[, z]) in design coordinates
    gl = np.array([g0[k] - d0[k] for k in range(dims)])
    gh = gl + np.array([gn[k] for k in range(dims)])
    inside = np.all((idx >= gl) & (idx < gh), axis=1)
    assert not inside.any()
    for k in range(dims):
        if k == a:
            side = (idx[:, k] < gl[k]) | (idx[:, k] >= gh[k])
            assert side.all()
            assert idx[:, k].min() == gl[k] - gn[k] and idx[:, k].max() == gh[k] + gn[k] - 1
        else:
            assert idx[:, k].min() == gl[k] and idx[:, k].max() == gh[k] - 1
