"""Pins of the CPU filter reference (oracle/filter.py): the linear limit
against an independent correlation, constants, erosion/dilation ordering and
the binary-density limit against min/max morphology, and the transpose
against central differences of the forward through the dot-product identity."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import filter as OF


def rng_field(shape, seed):
    return np.random.default_rng(seed).random(shape)


def cone_kernel(radius, three_d):
    R = int(np.ceil(radius))
    Rz = R if three_d else 0
    K = np.zeros((2 * Rz + 1, 2 * R + 1, 2 * R + 1))
    for dz in range(-Rz, Rz + 1):
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                K[dz + Rz, dy + R, dx + R] = max(0.0, radius - np.sqrt(dx * dx + dy * dy + dz * dz))
    return K


def linear_filter(x, radius):
    x3 = x.reshape((1,) + x.shape) if x.ndim == 2 else x
    K = cone_kernel(radius, x3.shape[0] > 1)
    num = ndimage.correlate(x3, K, mode="constant", cval=0.0)
    den = ndimage.correlate(np.ones_like(x3), K, mode="constant", cval=0.0)
    return (num / den).reshape(x.shape)


@pytest.mark.parametrize("shape", [(9, 11), (5, 6, 7)])
def test_large_alpha_is_the_linear_cone_filter(shape):
    x = rng_field(shape, 1)
    for dual in (False, True):
        y = OF.stage(x, 2.5, 1e7, dual)
        assert np.abs(y - linear_filter(x, 2.5)).max() < 1e-6
    y, _ = OF.open_close(x, 2.5, 1e7)
    ref = x
    for _ in range(4):
        ref = linear_filter(ref, 2.5)
    assert np.abs(y - ref).max() < 1e-6


def test_constants_are_kept_and_stages_are_ordered():
    x = rng_field((12, 10), 2)
    for c in (0.0, 0.3, 1.0):
        y, _ = OF.open_close(np.full((6, 7), c), 2.5, 0.05)
        assert np.abs(y - c).max() < 1e-12
    for a in (1.0, 0.1, 0.01):
        e = OF.stage(x, 2.5, a, False)
        d = OF.stage(x, 2.5, a, True)
        lin = linear_filter(x, 2.5)
        assert np.all(e <= lin + 1e-12) and np.all(lin <= d + 1e-12)


def test_small_alpha_approaches_min_max_morphology():
    x = (rng_field((14, 13), 3) > 0.5).astype(float)
    K = cone_kernel(2.5, False)[0] > 0
    e = OF.stage(x, 2.5, 1e-9, False)
    d = OF.stage(x, 2.5, 1e-9, True)
    assert np.abs(e - ndimage.minimum_filter(x, footprint=K, mode="nearest")).max() < 1e-6
    assert np.abs(d - ndimage.maximum_filter(x, footprint=K, mode="nearest")).max() < 1e-6


@pytest.mark.parametrize("shape,alpha", [((8, 9), 0.3), ((8, 9), 0.02), ((4, 5, 6), 0.1)])
def test_transpose_matches_central_differences(shape, alpha):
    x = 0.05 + 0.9 * rng_field(shape, 4)
    v = rng_field(shape, 5) - 0.5
    g = rng_field(shape, 6) - 0.5
    y, xs = OF.open_close(x, 2.5, alpha)
    h = 1e-6
    yp, _ = OF.open_close(x + h * v, 2.5, alpha)
    ym, _ = OF.open_close(x - h * v, 2.5, alpha)
    lhs = np.sum(g * (yp - ym) / (2 * h))
    rhs = np.sum(v * OF.open_close_transpose(xs, g, 2.5, alpha))
    assert abs(lhs - rhs) <= 1e-7 * max(1.0, abs(lhs))
