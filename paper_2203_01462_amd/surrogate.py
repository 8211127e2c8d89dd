"""Surrogate-guided design on the 512x512 TMz workload (128x128 design box).

Pipeline (all device work in the HIP library: FDTD solves, filter, MMA,
network layers; this module moves tensors and holds the control flow):

1. ``generate``: seeded synthetic design variables -> open-close filter ->
   batched forward + adjoint FDTD solves (one batch of identical instances,
   fdtd_batch_*) -> triples (rho_f, log F, dlogF/drho_f).  The network works
   in log space: F spans orders of magnitude across designs, and the
   log-derivative S/F has a far more uniform scale than S itself.
2. ``train``: the U-Net (nn.UNet) regresses normalized log F and the
   normalized log-derivative map with Adam on random minibatches.
3. ``guided``: from the current design, ``inner`` MMA steps are taken on the
   surrogate alone (its gradient corrected by the difference between the
   exact and the predicted gradient at the last FDTD-checked design), then one
   forward + adjoint FDTD solve checks the proposal.  A proposal that raises F
   is accepted; otherwise one exact GCMMA step is taken from the checked
   design.  Every checked design is added to the training set and the network
   is tuned on it for a few steps.
4. ``plain``: the design loop alone (design.optimize with damping
   continuation and the grayness stop) as the reference; ``compare`` reports
   the wall-clock time both take to reach within 1% of the plain optimizer's
   converged objective, and the offline cost (data and training) with the
   number of designs over which it pays back.
"""
from __future__ import annotations

import argparse
import copy
import json
import math
import time

import numpy as np
import torch

import fdtd_workloads as W

from . import design
from .fdtd import FDTD, Batch
from .nn import UNet


class Dataset:
    """Training triples on the device: rho [N][s][s] (filtered densities),
    logF [N], G [N][s][s] = dlogF/drho_f; normalization constants."""

    def __init__(self, side, cap, device):
        self.rho = torch.empty(cap, side, side, device=device)
        self.logF = torch.empty(cap, device=device)
        self.G = torch.empty(cap, side, side, device=device)
        self.n = 0
        self.mu, self.sd, self.gsd = 0.0, 1.0, 1.0

    def add(self, rho, F, g):
        """rho, g: device [s][s] FP32 (g = dF/drho_f); F: host float."""
        i = self.n
        if i >= self.rho.shape[0]:
            raise RuntimeError("dataset capacity exceeded")
        self.rho[i].copy_(rho)
        self.logF[i] = math.log(F)
        self.G[i].copy_(g / F)
        self.n += 1

    def set_norms(self):
        lf = self.logF[:self.n]
        self.mu = float(lf.mean())
        self.sd = float(lf.std().clamp_min(1e-6))
        self.gsd = float(self.G[:self.n].pow(2).mean().sqrt().clamp_min(1e-30))

    def batch(self, idx):
        return (self.rho[idx].contiguous(), ((self.logF[idx] - self.mu) / self.sd).contiguous(),
                (self.G[idx] / self.gsd).contiguous())


def _stream_handle():
    return torch.cuda.current_stream().cuda_stream


def generate(w, count, alpha=1.0, radius=2.5, seed=0, batch=64, data=None, log=None):
    """Solve forward + adjoint for `count` seeded designs; returns a Dataset.
    Runs on torch's current stream (must not be the default stream)."""
    shape = W.design_shape(w)
    side = shape[0]
    dev = torch.device("cuda", torch.cuda.current_device())
    data = Dataset(side, count, dev) if data is None else data
    filt = design.Filter(shape, radius, torch.float32)
    nb = min(batch, count)
    B = Batch([w] * nb, stream=_stream_handle())
    x = torch.empty(nb, *shape, device=dev)
    rf = torch.empty(nb, *shape, device=dev)
    g = torch.empty(nb, *shape, device=dev)
    done, chunk = 0, 0
    t0 = time.perf_counter()
    while done < count:
        m = min(nb, count - done)
        x.copy_(torch.from_numpy(W.random_designs(nb, shape, seed * 100003 + chunk)))
        for k in range(nb):
            filt.apply(x[k], alpha, out=rf[k])
            B.set_density(k, rf[k])
        F = B.forward()
        B.adjoint()
        for k in range(m):
            if not (np.isfinite(F[k]) and F[k] > 0.0):
                raise RuntimeError(f"non-positive objective {F[k]} for design {done + k}")
            B.gradient(k, out=g[k])
            data.add(rf[k], float(F[k]), g[k])
        done += m
        chunk += 1
        if log:
            log(f"generate: {done}/{count} triples, {time.perf_counter() - t0:.1f} s")
    B.close()
    filt.close()
    torch.cuda.synchronize()
    return data


def view(net, batch):
    """A U-Net sharing `net`'s parameters with buffers for another batch size."""
    v = copy.copy(net)
    v.batch = batch
    v._alloc(batch)
    return v


def train(net, data, steps, lr=1e-3, lr_min=1e-5, wF=1.0, wS=1.0, seed=0, val=None, log=None, log_every=200):
    """Adam on random minibatches of data[:n] (val: index tensor held out);
    cosine learning-rate decay from lr to lr_min."""
    gen = torch.Generator(device=net.dev).manual_seed(seed)
    n = data.n
    pool = torch.arange(n, device=net.dev)
    if val is not None:
        mask = torch.ones(n, dtype=torch.bool, device=net.dev)
        mask[val] = False
        pool = pool[mask]
    hist = []
    t0 = time.perf_counter()
    for it in range(steps):
        idx = pool[torch.randint(0, pool.numel(), (net.batch,), generator=gen, device=net.dev)]
        rho, lf, G = data.batch(idx)
        net.forward(rho)
        dF, dS = net.loss_grad(lf, G, wF, wS)
        net.backward(dF, dS)
        cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * it / max(steps, 1)))
        net.step(cur)
        if log and (it % log_every == 0 or it == steps - 1):
            l = net.loss.cpu()
            lF = float(l[0]) / net.batch
            lS = float(l[1]) / (net.batch * net.side * net.side)
            hist.append(dict(step=it, lossF=lF, lossS=lS, t=time.perf_counter() - t0))
            log(f"train: step {it} lossF {lF:.4f} lossS {lS:.4f} lr {cur:.2e} {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    return hist


def evaluate_net(net, data, idx):
    """Held-out metrics: RMSE of normalized log F, R^2 of log F, mean cosine
    similarity between predicted and exact log-derivative maps."""
    v = view(net, 1)
    errs, lfs, coss = [], [], []
    for i in idx.tolist():
        rho, lf, G = data.batch(torch.tensor([i], device=net.dev))
        Fh, Sh = v.forward(rho)
        errs.append(float(Fh[0]) - float(lf[0]))
        lfs.append(float(lf[0]))
        a, b = Sh.reshape(-1).double(), G.reshape(-1).double()
        coss.append(float(a @ b / (a.norm() * b.norm() + 1e-30)))
    errs, lfs = np.array(errs), np.array(lfs)
    r2 = 1.0 - (errs ** 2).sum() / max(((lfs - lfs.mean()) ** 2).sum(), 1e-30)
    return dict(rmse_logF_norm=float(np.sqrt((errs ** 2).mean())), r2_logF=float(r2),
                grad_cos_mean=float(np.mean(coss)), grad_cos_median=float(np.median(coss)), n=len(idx))


class _Exact:
    """Forward + adjoint FDTD on the filtered density of x."""

    def __init__(self, w, alpha, radius):
        shape = W.design_shape(w)
        self.sol = FDTD(w, stream=_stream_handle())
        self.filt = design.Filter(shape, radius, torch.float32)
        self.alpha = alpha
        dev = torch.device("cuda", torch.cuda.current_device())
        self.rf = torch.empty(shape, device=dev)
        self.gt = torch.empty(shape, device=dev)
        self.gx = torch.empty(shape, device=dev)
        self.solves = 0

    def __call__(self, x, grad=True):
        self.filt.apply(x, self.alpha, out=self.rf)
        self.sol.set_density(self.rf)
        F = self.sol.forward()
        self.solves += 1
        if grad:
            self.sol.adjoint()
            self.sol.gradient(out=self.gt)
            self.filt.transpose(self.gt, out=self.gx)
            self.solves += 1
        return F

    def gradient_only(self):
        """Adjoint and gradient for the density of the last forward solve."""
        self.sol.adjoint()
        self.sol.gradient(out=self.gt)
        self.filt.transpose(self.gt, out=self.gx)
        self.solves += 1

    def close(self):
        self.sol.close()
        self.filt.close()


class _ExactBatch:
    """Forward + adjoint FDTD of several candidate designs in one batched
    solve (fdtd_batch_*: the instance replicated, graph replay)."""

    def __init__(self, w, alpha, radius, count):
        shape = W.design_shape(w)
        self.b = Batch([w] * count, stream=_stream_handle())
        self.filt = design.Filter(shape, radius, torch.float32)
        self.alpha = alpha
        dev = torch.device("cuda", torch.cuda.current_device())
        self.rf = [torch.empty(shape, device=dev) for _ in range(count)]
        self.gt = [torch.empty(shape, device=dev) for _ in range(count)]
        self.gx = [torch.empty(shape, device=dev) for _ in range(count)]
        self.solves = 0

    def __call__(self, xs):
        for k, x in enumerate(xs):
            self.filt.apply(x, self.alpha, out=self.rf[k])
            self.b.set_density(k, self.rf[k])
        F = self.b.forward()
        self.b.adjoint()
        for k in range(len(xs)):
            self.b.gradient(k, out=self.gt[k])
            self.filt.transpose(self.gt[k], out=self.gx[k])
        self.solves += 2 * len(xs)
        return [float(f) for f in F]

    def close(self):
        self.b.close()
        self.filt.close()


def plain(w, alpha=1.0, radius=2.5, max_iter=600, max_inner=40, gamma_levels=None, zeta_min=0.005, log=None,
          log_every=10):
    """The design loop alone: damping continuation over `gamma_levels`
    (collision-rate multipliers, the last one the workload's own; None: the
    workload's only) at filter nonlinearity `alpha`, stopped at grayness
    zeta < zeta_min or max_iter iterations.  Returns [(t, F, level)] per outer
    iteration (F at that level's damping) and design.optimize's result."""
    trace = []
    levels = tuple(gamma_levels) if gamma_levels else (w["gamma_mult"],)
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def cb(h):
        trace.append((time.perf_counter() - t0, h["F"], h["level"]))
        if log and (h["iter"] % log_every == 0 or len(trace) == 1):
            log(f"plain: iteration {h['iter']} level {h['level']} F {h['F']:.6g} zeta {h['zeta']:.4f} "
                f"inner {h.get('inner', 0)} t {trace[-1][0]:.2f} s")

    res = design.optimize(w, alphas=(alpha,), gamma_levels=levels, max_iter=max_iter, zeta_min=zeta_min,
                          radius=radius, max_inner=max_inner, callback=cb)
    torch.cuda.synchronize()
    res["seconds"] = time.perf_counter() - t0
    res["levels"] = levels
    return trace, res


def guided(w, net, data, alpha=1.0, radius=2.5, checks=30, inner=4, move=0.2, tune_steps=2, tune_batch=8,
           tune_lr=2e-4, max_inner=40, target=None, log=None):
    """Surrogate-guided loop; returns [(t, F of the current design)] per FDTD
    check and counters.  Stops after `checks` checks, or once F reaches
    `target`.

    A proposal: `inner` MMA steps (move limit `move`) on the surrogate, whose
    log F and log-derivative are shifted by the exact-minus-predicted
    difference at the current design (so its first step is the exact MMA
    step); the iterate with the best shifted prediction is checked.  With a
    tuple of move limits, one proposal per limit is made and all of them are
    checked in one batched FDTD solve; the best is accepted if it raises F,
    and every checked design joins the training set."""
    moves = tuple(move) if isinstance(move, (tuple, list)) else (move,)
    if inner < 1 or not moves:
        raise ValueError("guided: need inner >= 1 and at least one move limit")
    shape = W.design_shape(w)
    dev = net.dev
    nd = int(np.prod(shape))
    net1 = view(net, 1)
    tnet = view(net, tune_batch) if tune_steps else None
    tgen = torch.Generator(device=dev).manual_seed(1234)
    if tnet is not None:
        tnet.t = net.t
    ex = _Exact(w, alpha, radius)
    exb = _ExactBatch(w, alpha, radius, len(moves)) if len(moves) > 1 else None
    mma = design.MMA(nd, torch.float32)
    x = torch.full(shape, 0.5, device=dev)
    xs = torch.empty_like(x)
    xbest = torch.empty_like(x)
    xnew = torch.empty_like(x)
    rs = torch.empty_like(x)
    gs = torch.empty_like(x)
    filt = design.Filter(shape, radius, torch.float32)
    trace = []
    clock = dict(surrogate=0.0, check=0.0, fallback=0.0, tune=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = ex(x)
    gx = ex.gx.clone()
    rf = ex.rf.clone()
    gt = ex.gt.clone()
    trace.append((time.perf_counter() - t0, F))
    stats = dict(accepted=0, fallback=0, checks=0, best_step=[])

    def predict(xv):
        filt.apply(xv, alpha, out=rs)
        Fh, Sh = net1.forward(rs.reshape(1, *shape))
        return float(Fh[0]) * data.sd + data.mu, Sh[0] * data.gsd

    def propose(mv, lf0, S0, dlf, corr):
        """The best shifted-prediction iterate of `inner` surrogate MMA steps
        from x with move limit mv (into a new tensor) and its step index."""
        xs.copy_(x)
        ms = design.MMA(nd, torch.float32, move=mv)
        best, kbest, out = -math.inf, 0, torch.empty_like(x)
        for k in range(inner + 1):
            lf, S = predict(xs) if k else (lf0, S0)
            val = lf + dlf
            if k and val > best:
                best, kbest = val, k
                out.copy_(xs)
            if k == inner:
                break
            torch.add(S, corr, out=gs)
            filt.transpose(gs, out=xnew)              # dlogF/dx
            xnew.neg_()
            r0 = ms.begin(xs, -val, xnew)
            ms.solve(r0, xnew)
            ms.accept(xnew)
            xs.copy_(xnew)
        ms.close()
        return out, kbest

    while stats["checks"] < checks and not (target is not None and F >= target):
        ta = time.perf_counter()
        lf0, S0 = predict(x)
        dlf = math.log(F) - lf0          # value shift
        corr = gt / F - S0               # log-derivative shift
        cands = [propose(mv, lf0, S0, dlf, corr) for mv in moves]
        tb = time.perf_counter()
        clock["surrogate"] += tb - ta
        if exb is None:
            xbest.copy_(cands[0][0])
            kbest = cands[0][1]
            Fs = ex(xbest)
            data.add(ex.rf, Fs, ex.gt)
            new_gx, new_rf, new_gt = ex.gx, ex.rf, ex.gt
        else:
            Fl = exb([c[0] for c in cands])
            for k in range(len(moves)):
                data.add(exb.rf[k], Fl[k], exb.gt[k])
            kb = int(np.argmax(Fl))
            xbest.copy_(cands[kb][0])
            kbest = cands[kb][1]
            Fs = Fl[kb]
            new_gx, new_rf, new_gt = exb.gx[kb], exb.rf[kb], exb.gt[kb]
        stats["best_step"].append(kbest)
        stats["checks"] += 1
        tc = time.perf_counter()
        clock["check"] += tc - tb
        if Fs > F:
            stats["accepted"] += 1
            # record the step in the exact MMA's iterate history (its
            # asymptotes adapt to the sequence of accepted designs)
            mma.begin(x, -1.0, gx * (-1.0 / F))
            mma.accept(xbest)
            x.copy_(xbest)
            F = Fs
            gx.copy_(new_gx)
            rf.copy_(new_rf)
            gt.copy_(new_gt)
        else:
            # one exact GCMMA step from x (as in the plain loop)
            stats["fallback"] += 1
            rho_m = mma.begin(x, -1.0, gx * (-1.0 / F))
            Fn = None
            for _ in range(max_inner):
                approx, dist = mma.solve(rho_m, xnew)
                Fn = ex(xnew, grad=False)
                f0n = -Fn / F
                if f0n <= approx + 1e-12 * max(1.0, abs(approx)):
                    break
                rho_m = min(1.1 * (rho_m + (f0n - approx) / max(dist, 1e-300)), 10.0 * rho_m)
            if Fn is not None and Fn > F:
                mma.accept(xnew)
                x.copy_(xnew)
                F = Fn
                ex.gradient_only()  # the forward solve at xnew is still in the context
                gx.copy_(ex.gx)
                rf.copy_(ex.rf)
                gt.copy_(ex.gt)
                data.add(ex.rf, F, ex.gt)
        td = time.perf_counter()
        clock["fallback"] += td - tc
        if tnet is not None:
            _tune(tnet, data, tune_steps, tune_lr, tgen)
        clock["tune"] += time.perf_counter() - td
        trace.append((time.perf_counter() - t0, F))
        if log:
            log(f"guided: check {stats['checks']} F {F:.6g} proposal {Fs:.6g} (step {kbest}) "
                f"t {trace[-1][0]:.2f} s")
    torch.cuda.synchronize()
    stats["solves"] = ex.solves + (exb.solves if exb is not None else 0)
    stats["clock"] = clock
    ex.close()
    if exb is not None:
        exb.close()
    mma.close()
    filt.close()
    return trace, stats


def _tune(net, data, steps, lr, gen=None):
    """A few Adam steps on minibatches holding the newest triple (`net` is a
    view sharing the trained parameters and Adam state; `gen` a seeded
    generator, so runs repeat)."""
    n = data.n
    for _ in range(steps):
        idx = torch.randint(0, n, (net.batch,), device=net.dev, generator=gen)
        idx[0] = n - 1
        rho, lf, G = data.batch(idx)
        net.forward(rho)
        dF, dS = net.loss_grad(lf, G)
        net.backward(dF, dS)
        net.step(lr)


def time_to(trace, target):
    for t, F in trace:
        if F >= target:
            return t
    return None


def _from_first(trace):
    """Times relative to the first point (the evaluation of the start design),
    so that context set-up is not counted for either loop."""
    t0 = trace[0][0]
    return [(r[0] - t0,) + tuple(r[1:]) for r in trace]


def compare(samples=20000, train_steps=8000, batch=32, alpha=1.0, checks=200, inner=10, seed=1, n_steps=5000,
            w=None, settings=((0.2, 2),), gamma_levels=(16.0, 4.0, 1.0), zeta_min=0.005, plain_max_iter=600,
            log=print):
    """Plain optimizer vs surrogate-guided loop from the same start design.

    Offline: `samples` triples from seeded random designs (batched solves),
    `train_steps` Adam steps.  Reference: the plain optimizer with damping
    continuation over `gamma_levels` and the grayness stop (zeta < zeta_min
    or `plain_max_iter` iterations); its converged objective F* is its final
    design's F at the workload's physics, and the target is 0.99 F*.  The
    plain time to target is the first iterate of its last level at or above
    the target.  One guided run per (move limit, tuning steps[, inner steps])
    in `settings`, each stopped at the target or after `checks` checks."""
    w = W.c5(n_steps) if w is None else w
    out = dict(workload=w["name"], samples=samples, train_steps=train_steps, batch=batch, alpha=alpha,
               inner=inner, n_steps=n_steps, seed=seed, gamma_levels=list(gamma_levels), zeta_min=zeta_min,
               plain_max_iter=plain_max_iter)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t = time.perf_counter()
        widest = max(len(st[0]) if isinstance(st[0], (tuple, list)) else 1 for st in settings)
        data = Dataset(W.design_shape(w)[0], samples + (widest + 3) * checks + 8, torch.device("cuda"))
        generate(w, samples, alpha=alpha, seed=seed, data=data, log=log)
        out["generate_s"] = time.perf_counter() - t
        data.set_norms()
        nval = max(samples // 20, 1)
        val = torch.arange(samples - nval, samples, device="cuda")
        net = UNet(W.design_shape(w)[0], batch, seed=seed, stream=None)
        t = time.perf_counter()
        out["train_hist"] = train(net, data, train_steps, val=val, log=log, seed=seed)
        out["train_s"] = time.perf_counter() - t
        out["offline_s"] = out["generate_s"] + out["train_s"]
        out["val"] = evaluate_net(net, data, val)
        log(f"validation: {out['val']}")
        ptrace, pres = plain(w, alpha=alpha, max_iter=plain_max_iter, gamma_levels=gamma_levels,
                             zeta_min=zeta_min, log=log)
        ptrace = _from_first(ptrace)
        ex = _Exact(w, alpha, 2.5)
        Fconv = ex(pres["x"], grad=False)
        ex.close()
        target = 0.99 * Fconv
        last = len(pres["levels"]) - 1
        hit = [t for t, F, lv in ptrace if lv == last and F >= target]
        out.update(plain_trace=ptrace, plain_converged_F=Fconv, target=target, plain_iterations=pres["iterations"],
                   plain_zeta=pres["zeta"], plain_seconds=ptrace[-1][0],
                   plain_reached_last_level=any(lv == last for _, _, lv in ptrace),
                   plain_time_to_target=hit[0] if hit else ptrace[-1][0],
                   plain_iters_to_target=next((i for i, (_, F, lv) in enumerate(ptrace) if lv == last and F >= target),
                                              len(ptrace) - 1))
        log(f"plain: converged F {Fconv:.6g} after {pres['iterations']} iterations, zeta {pres['zeta']:.4f}, "
            f"{out['plain_seconds']:.2f} s; time to 99%: {out['plain_time_to_target']:.2f} s")
        # every setting starts from the same trained network and dataset
        saved = (net.p.clone(), net.m.clone(), net.v.clone(), net.t, data.n)
        runs = []
        for st in settings:
            mv, tune = st[0], st[1]
            inn = st[2] if len(st) > 2 else inner
            net.p.copy_(saved[0])
            net.m.copy_(saved[1])
            net.v.copy_(saved[2])
            net.t, data.n = saved[3], saved[4]
            net.load(net.p)
            gtrace, gstats = guided(w, net, data, alpha=alpha, checks=checks, inner=inn, move=mv, tune_steps=tune,
                                    target=target, log=log)
            gtrace = _from_first(gtrace)
            tt = time_to(gtrace, target)
            hitg = [i for i, (_, F) in enumerate(gtrace) if F >= target]
            saved_s = out["plain_time_to_target"] - tt if tt is not None else None
            runs.append(dict(move=mv, tune_steps=tune, inner=inn, trace=gtrace, stats=gstats, time_to_target=tt,
                             checks_to_target=hitg[0] if hitg else None, best=max(F for _, F in gtrace),
                             speedup=out["plain_time_to_target"] / tt if tt else None,
                             designs_to_amortize=math.ceil(out["offline_s"] / saved_s) if saved_s and saved_s > 0
                             else None))
            log(f"guided move {mv} tune {tune} inner {inn}: time to target {tt}, "
                f"plain {out['plain_time_to_target']:.2f} s, best F {runs[-1]['best']:.6g}")
    torch.cuda.synchronize()
    out["guided"] = runs
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--samples", type=int, default=20000)
    ap.add_argument("--train-steps", type=int, default=8000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--alpha", type=float, default=1.0)
    ap.add_argument("--checks", type=int, default=200)
    ap.add_argument("--inner", type=int, default=10)
    ap.add_argument("--n-steps", type=int, default=5000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--gamma-levels", default="16,4,1",
                    help="damping continuation of the plain optimizer (collision-rate multipliers)")
    ap.add_argument("--zeta-min", type=float, default=0.005)
    ap.add_argument("--plain-max-iter", type=int, default=600)
    ap.add_argument("--settings", default="0.2:2",
                    help="comma-separated move:tune_steps[:inner] settings; move may be m1/m2/... (one proposal "
                         "per move limit, checked together in one batched solve)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    settings = []
    for item in a.settings.split(","):
        f = item.split(":")
        mv = tuple(float(m) for m in f[0].split("/"))
        settings.append((mv if len(mv) > 1 else mv[0], int(f[1])) + ((int(f[2]),) if len(f) > 2 else ()))
    res = compare(a.samples, a.train_steps, a.batch, a.alpha, a.checks, a.inner, a.seed, a.n_steps,
                  settings=settings, gamma_levels=tuple(float(g) for g in a.gamma_levels.split(",")),
                  zeta_min=a.zeta_min, plain_max_iter=a.plain_max_iter, log=lambda m: print(m, flush=True))
    summary = {k: v for k, v in res.items() if not k.endswith("_trace") and k not in ("train_hist", "guided")}
    summary["guided"] = [{k: v for k, v in r.items() if k != "trace"} for r in res["guided"]]
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
