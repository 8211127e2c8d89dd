"""The design-update loop around the FDTD hot path (paper, Methods: eqs.
(26)-(28) and the optimization flowchart).

Per iteration: filter the design variables (open-close cascade of four
fW-mean filters, eq. (26)), run the forward and adjoint FDTD solves on the
filtered density, map dF/drho_f back through the filter (eq. (27)), and update
rho with the globally convergent method of moving asymptotes (GCMMA) for
"maximize F subject to 0 <= rho <= 1" (eq. (28)).  Continuation: levels of
(filter nonlinearity, damping); a level ends once at least 12 iterations have
run and the first-order optimality norm has fallen by 70% from its value at
the 12th; the run ends when the non-discreteness zeta of the filtered density
drops below zeta_min or after max_iter iterations, and the design is then
thresholded at 0.5 and evaluated without the artificial damping.

Every per-element operation runs in the HIP library (fdtd.h, fdtd_design.h);
this module holds the scalar control flow and moves device pointers.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from .fdtd import FDTD, FDTDError, load_library


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _check(rc):
    if rc:
        raise FDTDError(rc, load_library().fdtd_design_last_error().decode())


def _stream():
    """torch's current stream.  Objects of this module, FDTD contexts and torch
    work are ordered only when they share one stream; torch's default stream
    has handle 0, which the library reads as "create a private stream", so
    callers mixing them run inside ``torch.cuda.stream(<non-default stream>)``
    (``optimize`` does)."""
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Filter:
    """Open-close fW-mean filter over a design box shape (z, y, x) or (y, x)."""

    def __init__(self, shape, radius=2.5, dtype=torch.float64):
        L = load_library()
        n = (C.c_int32 * 3)(*(list(reversed(shape)) + [1] * (3 - len(shape))))
        h = C.c_void_p()
        self.prec = 32 if dtype == torch.float32 else 64
        _check(L.fdtd_filter_create(n, float(radius), self.prec, _stream(), C.byref(h)))
        self.h, self.shape, self.dtype = h, tuple(shape), dtype

    def apply(self, rho, alpha, out=None):
        out = torch.empty_like(rho) if out is None else out
        _check(load_library().fdtd_filter_apply(self.h, _ptr(rho), _ptr(out), float(alpha)))
        return out

    def transpose(self, g_f, out=None):
        out = torch.empty_like(g_f) if out is None else out
        _check(load_library().fdtd_filter_transpose(self.h, _ptr(g_f), _ptr(out)))
        return out

    def close(self):
        if getattr(self, "h", None) and load_library is not None:
            load_library().fdtd_filter_destroy(self.h)
            self.h = None

    __del__ = close


class MMA:
    """Method of moving asymptotes for min f0(x), xmin <= x <= xmax (no other
    constraints), with the conservative inner loop of its globally
    convergent variant driven by the caller."""

    def __init__(self, n, dtype=torch.float64, xmin=0.0, xmax=1.0, move=0.5, asyinit=0.5, asyincr=1.2,
                 asydecr=0.7):
        h = C.c_void_p()
        prec = 32 if dtype == torch.float32 else 64
        _check(load_library().fdtd_mma_create(int(n), prec, xmin, xmax, move, asyinit, asyincr, asydecr, _stream(),
                                              C.byref(h)))
        self.h = h

    def begin(self, x, f0, df0):
        r = C.c_double()
        _check(load_library().fdtd_mma_begin(self.h, _ptr(x), float(f0), _ptr(df0), C.byref(r)))
        return r.value

    def solve(self, rho, xnew):
        a, d = C.c_double(), C.c_double()
        _check(load_library().fdtd_mma_solve(self.h, float(rho), _ptr(xnew), C.byref(a), C.byref(d)))
        return a.value, d.value

    def accept(self, xnew):
        _check(load_library().fdtd_mma_accept(self.h, _ptr(xnew)))

    def close(self):
        if getattr(self, "h", None) and load_library is not None:
            load_library().fdtd_mma_destroy(self.h)
            self.h = None

    __del__ = close


def stats(x, g=None, xmin=0.0, xmax=1.0):
    """(zeta, ||x - clamp(x - g)||): non-discreteness and first-order optimality."""
    out = (C.c_double * 2)()
    prec = 32 if x.dtype == torch.float32 else 64
    _check(load_library().fdtd_design_stats(x.numel(), prec, _ptr(x), _ptr(g) if g is not None else None, xmin, xmax,
                                            _stream(), out))
    return out[0], out[1]


def gap_guard_mask(w, axis=None):
    """Design-box mask (True = held at metal) of the two boxes of the gap's
    size next to the gap on either side along `axis` (index into (x, y, z);
    default: the polarization axis in 3D (x), x in 2D), clipped to the design
    box (Sec. 4.1, 4.3: the regions on either side of the gap, of its size,
    held at the metal)."""
    d0, dn, g0, gn = w["design_lo"], w["design_n"], w["gap_lo"], w["gap_n"]
    dims = w["dims"]
    axis = 0 if axis is None else axis
    shape = (dn[2], dn[1], dn[0]) if dims == 3 else (dn[1], dn[0])
    m = np.zeros(shape, dtype=bool)
    for side in (-1, 1):
        lo = [g0[a] - d0[a] for a in range(3)]
        lo[axis] += side * gn[axis]
        hi = [lo[a] + gn[a] for a in range(3)]
        lo = [max(lo[a], 0) for a in range(3)]
        hi = [min(hi[a], dn[a]) for a in range(3)]
        if any(hi[a] <= lo[a] for a in range(dims)):
            continue
        if dims == 3:
            m[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = True
        else:
            m[lo[1]:hi[1], lo[0]:hi[0]] = True
    return m


def optimize(w, rho0=0.5, max_iter=600, zeta_min=0.005, alphas=(64.0, 1.0, 0.3, 0.1, 0.05),
             gamma_levels=(16.0, 4.0, 1.0), sigma_levels=None, radius=2.5, level_min_iters=12, kkt_drop=0.7,
             max_inner=40, ckpt_every=0, threshold=0.5, callback=None, fixed=None, tie_axis=None):
    """Maximize the objective of workload `w` over the design density.

    `fixed`: boolean mask of the design box (array order) whose cells are
    held at metal (the filtered density is 1 there and their sensitivities
    are dropped; see gap_guard_mask).  `tie_axis`: an axis of the design
    array (3D: 0 = z) along which the design is uniform (a planar structure,
    Sec. 4.3): the variables live on the other axes, the filter acts there,
    the density is the extrusion of the filtered variables, and the gradient
    of a filtered variable is the sum of its cells' gradients.

    Level i uses filter nonlinearity alphas[min(i, .)] and damping
    gamma_levels[min(i, .)] (collision-rate multiplier) and, if given,
    sigma_levels[min(i, .)] (artificial conductivity peak, eq. (5c)).
    Each outer iteration raises the GCMMA curvature weight until the
    approximation is conservative at the trial point (at most max_inner
    forward solves); a trial that is still not conservative is accepted only
    if it does not lower F, else the level ends there.
    Returns a dict with the final variables, the filtered and thresholded
    densities, the thresholded design's objective without artificial damping,
    and the per-iteration history."""
    dev = torch.device("cuda", torch.cuda.current_device())
    caller = torch.cuda.current_stream()
    work = torch.cuda.Stream()   # every object and tensor op of the loop runs here
    work.wait_stream(caller)
    with torch.cuda.stream(work):
        res = _optimize(w, rho0, max_iter, zeta_min, alphas, gamma_levels, sigma_levels, radius, level_min_iters,
                        kkt_drop, max_inner, ckpt_every, threshold, callback, dev, fixed, tie_axis)
    caller.wait_stream(work)
    return res


def _optimize(w, rho0, max_iter, zeta_min, alphas, gamma_levels, sigma_levels, radius, level_min_iters, kkt_drop,
              max_inner, ckpt_every, threshold, callback, dev, fixed=None, tie_axis=None):
    dtype = torch.float32 if w["precision"] == 32 else torch.float64
    nlev = max(len(alphas), len(gamma_levels), len(sigma_levels or [0]))

    def level_params(i):
        i = min(i, nlev - 1)
        a = alphas[min(i, len(alphas) - 1)]
        g = gamma_levels[min(i, len(gamma_levels) - 1)]
        s = sigma_levels[min(i, len(sigma_levels) - 1)] if sigma_levels else w["sigma_max"]
        return a, g, s

    stream = torch.cuda.current_stream().cuda_stream
    solvers = {}

    def solver(g, s):
        key = (g, s)
        if key not in solvers:
            ww = dict(w)
            ww.update(gamma_mult=g, sigma_max=s)
            solvers[key] = FDTD(ww, stream=stream, ckpt_every=ckpt_every)
        return solvers[key]

    dnx, dny, dnz = w["design_n"]
    shape = (dnz, dny, dnx) if w["dims"] == 3 else (dny, dnx)
    if tie_axis is not None and not 0 <= tie_axis < len(shape):
        raise ValueError(f"tie_axis {tie_axis} outside the design array's {len(shape)} axes")
    vshape = shape if tie_axis is None else tuple(n for a, n in enumerate(shape) if a != tie_axis)
    if np.isscalar(rho0):
        x = torch.full(vshape, float(rho0), dtype=dtype, device=dev)
    else:
        x = torch.as_tensor(rho0, dtype=dtype, device=dev)
        x = (x.reshape(shape).mean(dim=tie_axis) if tie_axis is not None else x.reshape(shape)).contiguous()
    fmask = None
    if fixed is not None:
        fmask = torch.as_tensor(np.asarray(fixed, dtype=bool), device=dev).reshape(shape)
    filt = Filter(vshape, radius, dtype)
    mma = MMA(x.numel(), dtype)
    rt = torch.empty(shape, dtype=dtype, device=dev)   # the density over the design box
    gt = torch.empty_like(rt)
    rv = torch.empty_like(x)                          # filtered variables and their gradient (tied)
    gv = torch.empty_like(x)
    df0 = torch.empty_like(x)
    xnew = torch.empty_like(x)

    def extrude(v, out):
        out.copy_(v.unsqueeze(tie_axis).expand(shape))
        return out
    history = []
    level, it_level, kkt_ref = 0, 0, None
    F_ref = None
    alpha, g_mult, s_max = level_params(0)
    sol = solver(g_mult, s_max)

    def density(xv, a):
        if tie_axis is None:
            filt.apply(xv, a, out=rt)
        else:
            extrude(filt.apply(xv, a, out=rv), rt)
        if fmask is not None:
            rt.masked_fill_(fmask, 1.0)
        return rt

    def sensitivity():
        """dF/d(variables) from dF/drho_f in gt (eq. (27); fixed cells drop out)."""
        if fmask is not None:
            gt.masked_fill_(fmask, 0.0)
        if tie_axis is None:
            filt.transpose(gt, out=df0)
        else:
            torch.sum(gt, dim=tie_axis, out=gv)
            filt.transpose(gv, out=df0)

    def evaluate(xv, grad):
        sol.set_density(density(xv, alpha))
        F = sol.forward()
        if grad:
            sol.adjoint()
            sol.gradient(out=gt)
            sensitivity()
        return F

    F = evaluate(x, True)
    it = 0
    while True:
        if F_ref is None:
            F_ref = abs(F) if F != 0 else 1.0
        df0.mul_(-1.0 / F_ref)             # minimize f0 = -F / F_ref
        f0 = -F / F_ref
        zeta, _ = stats(rt)
        _, kkt = stats(x, df0)
        history.append(dict(iter=it, level=level, alpha=alpha, gamma_mult=g_mult, sigma_max=s_max, F=F, zeta=zeta,
                            kkt=kkt))
        if callback:
            callback(history[-1])
        if zeta < zeta_min or it >= max_iter:
            break
        it_level += 1
        if it_level == level_min_iters:
            kkt_ref = kkt
        if level < nlev - 1 and it_level > level_min_iters and kkt <= (1.0 - kkt_drop) * kkt_ref:
            level += 1
            it_level, kkt_ref = 0, None
            alpha, g_mult, s_max = level_params(level)
            sol = solver(g_mult, s_max)
            F = evaluate(x, True)
            continue
        # one GCMMA outer iteration: raise the curvature weight until the
        # approximation is conservative at the trial point
        rho_m = mma.begin(x, f0, df0)
        conservative = False
        for inner in range(max_inner):
            approx, dist = mma.solve(rho_m, xnew)
            Fn = evaluate(xnew, False)
            f0n = -Fn / F_ref
            if f0n <= approx + 1e-12 * max(1.0, abs(approx)):
                conservative = True
                break
            rho_m = min(1.1 * (rho_m + (f0n - approx) / max(dist, 1e-300)), 10.0 * rho_m)
        history[-1]["inner"] = inner + 1
        history[-1]["conservative"] = conservative
        if not conservative and f0n > f0:
            # no acceptable step at this level: move on (or stop at the last)
            if level == nlev - 1:
                break
            level += 1
            it_level, kkt_ref = 0, None
            alpha, g_mult, s_max = level_params(level)
            sol = solver(g_mult, s_max)
            F = evaluate(x, True)
            continue
        mma.accept(xnew)
        x.copy_(xnew)
        # the forward at x is in the solver: adjoint and gradient only
        sol.adjoint()
        sol.gradient(out=gt)
        sensitivity()
        F = Fn
        it += 1
    rho_f = density(x, alpha).clone()
    rho_b = (rho_f >= threshold).to(dtype)
    final = solver(1.0, 0.0)
    final.set_density(rho_b)
    F_final = final.forward()
    for s in solvers.values():
        s.close()
    filt.close()
    mma.close()
    xs = x if tie_axis is None else extrude(x, torch.empty_like(rt))
    return dict(x=xs, variables=x, rho_filtered=rho_f, rho_binary=rho_b, F_final=F_final, iterations=it, zeta=zeta,
                history=history)
