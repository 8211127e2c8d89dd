"""Open-close density filter (paper, Methods, eq. (26)) and the transpose of
its Jacobian (eq. (27)): plain FP64 numpy, test infrastructure only.

The paper names the filter -- a cascade of four fW-mean filters forming an
open-close operator, size 5 dx, one nonlinearity parameter -- without its
formula.  Reading taken here: each stage is the weighted f-mean
    e_i = f^-1( sum_j w_ij f(u_j) / sum_j w_ij ),   f(u) = 1/(u + alpha),
with cone weights w_ij = max(0, r - |x_i - x_j|) over the cells of the design
box (r = 2.5 cells for size 5 dx).  The erosion E uses u = x (small values
dominate as alpha -> 0); the dilation is its dual D(x) = 1 - E(1 - x).
Open = D(E(.)), close = E(D(.)); open-close = close(open(.)) = E D D E.
Large alpha turns every stage into the linear cone filter.
"""
import numpy as np


def offsets(radius, three_d):
    R = int(np.ceil(radius))
    Rz = R if three_d else 0
    out = []
    for dz in range(-Rz, Rz + 1):
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                w = radius - np.sqrt(dx * dx + dy * dy + dz * dz)
                if w > 0:
                    out.append((dz, dy, dx, w))
    return out


def _as3(x):
    x = np.asarray(x, dtype=np.float64)
    return x.reshape((1,) + x.shape) if x.ndim == 2 else x


def shifted(a, dz, dy, dx):
    """b[k, j, i] = a[k+dz, j+dy, i+dx] inside the box, 0 outside."""
    nz, ny, nx = a.shape
    b = np.zeros_like(a)
    zs, ys, xs = slice(max(0, -dz), min(nz, nz - dz)), slice(max(0, -dy), min(ny, ny - dy)), slice(max(0, -dx), min(nx, nx - dx))
    zt, yt, xt = slice(max(0, dz), min(nz, nz + dz)), slice(max(0, dy), min(ny, ny + dy)), slice(max(0, dx), min(nx, nx + dx))
    b[zs, ys, xs] = a[zt, yt, xt]
    return b


def weight_sums(shape3, radius):
    W = np.zeros(shape3)
    one = np.ones(shape3)
    for dz, dy, dx, w in offsets(radius, shape3[0] > 1):
        W += w * shifted(one, dz, dy, dx)
    return W


def stage(x, radius, alpha, dual):
    """One fW-mean stage (erosion, or dilation when dual)."""
    x3 = _as3(x)
    u = 1.0 - x3 if dual else x3
    fu = 1.0 / (u + alpha)
    s = np.zeros_like(x3)
    for dz, dy, dx, w in offsets(radius, x3.shape[0] > 1):
        s += w * shifted(fu, dz, dy, dx)
    e = 1.0 / (s / weight_sums(x3.shape, radius)) - alpha
    y = 1.0 - e if dual else e
    return y.reshape(np.shape(x))


DUALS = (False, True, True, False)   # erode, dilate, dilate, erode


def open_close(x, radius, alpha):
    """Filtered density and the inputs of the four stages."""
    xs = [np.asarray(x, dtype=np.float64)]
    for d in DUALS:
        xs.append(stage(xs[-1], radius, alpha, d))
    return xs[-1], xs


def stage_transpose(x, y, g, radius, alpha, dual):
    """J^T g for one stage with input x and output y:
    J_ij = (w_ij / W_i) f'(u_j) / f'(e_i) = (w_ij / W_i) (e_i + alpha)^2 / (u_j + alpha)^2."""
    x3, y3, g3 = _as3(x), _as3(y), _as3(g)
    u = 1.0 - x3 if dual else x3
    e = 1.0 - y3 if dual else y3
    h = g3 * (e + alpha) ** 2 / weight_sums(x3.shape, radius)
    s = np.zeros_like(x3)
    for dz, dy, dx, w in offsets(radius, x3.shape[0] > 1):
        s += w * shifted(h, dz, dy, dx)
    return (s / (u + alpha) ** 2).reshape(np.shape(x))


def open_close_transpose(xs, g, radius, alpha):
    """d(.)/drho from d(.)/drho_f through the cascade (reverse order)."""
    for k in (3, 2, 1, 0):
        g = stage_transpose(xs[k], xs[k + 1], g, radius, alpha, DUALS[k])
    return g
