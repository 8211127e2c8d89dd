"""Batches of uneven 2D instances (fdtd_batch_*): every instance of a batch
gives the objective, gap DFT and gradient of a single context with the same
config and tile depth, bit for bit, whether the step sequence runs eagerly or
is replayed from the captured graph (several replays with eager work between
them), at temporal-block depth 1 (every tile depth) and 2 (the blocked
schedule, odd and even step counts) and with the autotuned depths.  Calls go
through the C ABI."""
import numpy as np
import pytest

import fdtd_workloads as W
from test_gpu_parity_2d import gpu, say  # noqa: F401

pytestmark = pytest.mark.gpu


def uneven(n_steps, precision=32, sides=(64, 96, 128, 160), count=6, seed=1):
    rng = np.random.default_rng(seed)
    ws = []
    for k in range(count):
        side = int(sides[k % len(sides)])
        gm = float(rng.uniform(1, 16))
        a = float(rng.uniform(500e-9, 850e-9))
        ws.append(W.instance2d(side, gm, a, a + 150e-9, n_steps, precision=precision, n_freq=4, name=f"b{k}"))
    return ws


def singles(gpu, ws, rhos):
    out = []
    for w, r in zip(ws, rhos):
        g = gpu.FDTD(w)
        out.append(g.run(r.astype(g.dtype)))
        g.close()
    return out


def run_batch(gpu, ws, rhos, rows, use_graph, repeats=1, depth=0):
    b = gpu.Batch(ws, rows=rows, use_graph=use_graph, depth=depth)
    for k, r in enumerate(rhos):
        b.set_density(k, r.astype(b.dtype))
    res = []
    for _ in range(repeats):
        F = b.forward()
        b.adjoint()
        res.append((F, [b.gradient(k) for k in range(len(ws))]))
        # eager work on the same device between graph replays
        g = gpu.FDTD(ws[0])
        g.run(rhos[0].astype(g.dtype))
        g.close()
    info = [b.info(k) for k in range(len(ws))]
    b.close()
    return res, [i["rows"] for i in info], [i["depth"] for i in info]


def has_super_tiles(w):
    from test_gpu_blocking import super_tiles
    return super_tiles(w) > 0


@pytest.mark.parametrize("prec,depth,n_steps", [(64, 1, 400), (64, 2, 400), (64, 2, 401), (32, 1, 400),
                                                (32, 2, 401)])
def test_batch_matches_single_contexts(gpu, prec, depth, n_steps):
    """FP64: every instance bit-identical to its single context.  FP32: the
    batched kernels are separately compiled code, so single-ulp rounding may
    differ (observed 7.5e-10 on F); bars 1e-6 on F, 1e-5 on the gradient.
    Graph replays (three, with eager work between them) are bit-identical
    to the eager batch in both precisions.  At depth 2 the instances with
    plain-background super-tiles (sides 160 and up) take the blocked schedule
    and the small ones per-step launches inside it."""
    ws = uneven(n_steps, precision=prec, sides=(64, 160, 256, 384))
    rhos = [W.seeded_rho(w, k) for k, w in enumerate(ws)]
    ref = singles(gpu, ws, rhos)
    (eager,), d0, b0 = run_batch(gpu, ws, rhos, 2, False, depth=depth)
    graph, d1, b1 = run_batch(gpu, ws, rhos, 2, True, repeats=3, depth=depth)
    assert d0 == d1 == [2] * len(ws)
    expect = [2 if depth == 2 and has_super_tiles(w) else 1 for w in ws]
    assert b0 == b1 == expect, (b0, b1, expect)
    F, grads = eager
    for k in range(len(ws)):
        if prec == 64:
            assert F[k] == ref[k][0], (k, F[k], ref[k][0])
            assert np.array_equal(grads[k], ref[k][1]), k
        else:
            assert abs(F[k] - ref[k][0]) <= 1e-6 * abs(ref[k][0]), (k, F[k], ref[k][0])
            assert np.linalg.norm(grads[k] - ref[k][1]) <= 1e-5 * np.linalg.norm(ref[k][1]), k
    for Fg, gg in graph:
        assert np.array_equal(Fg, F)
        for k in range(len(ws)):
            assert np.array_equal(gg[k], grads[k])
    say(f"[batch] prec={prec} depth={depth} N={n_steps}: {len(ws)} instances match single contexts; "
        f"3 graph replays identical")


def test_batch_tile_depths_agree(gpu):
    ws = uneven(300, precision=64, count=4)
    rhos = [W.seeded_rho(w, k) for k, w in enumerate(ws)]
    out = {}
    for rows in (1, 2, 4):
        res, depths, _ = run_batch(gpu, ws, rhos, rows, True, depth=1)
        assert depths == [rows] * len(ws)
        out[rows] = res[0]
    for rows in (1, 4):
        for k in range(len(ws)):
            assert abs(out[rows][0][k] - out[2][0][k]) <= 1e-13 * abs(out[2][0][k])
            g1, g2 = out[rows][1][k], out[2][1][k]
            assert np.linalg.norm(g1 - g2) <= 1e-12 * np.linalg.norm(g2)


def test_batch_autotuned_depths(gpu):
    ws = uneven(300, precision=32, sides=(128, 512), count=4)
    rhos = [W.seeded_rho(w, k) for k, w in enumerate(ws)]
    res, depths, blocks = run_batch(gpu, ws, rhos, 0, True)
    say(f"[batch] autotuned tile depths {depths}, temporal-block depths {blocks}")
    assert all(d in (1, 2, 4) for d in depths) and all(d in (1, 2) for d in blocks)
    # one choice per grid size (tuned on the batch)
    assert depths[0] == depths[2] and depths[1] == depths[3]
    assert blocks[0] == blocks[2] == 1 and blocks[1] == blocks[3]  # 128^2 has no super-tiles
    if 2 in blocks:
        assert depths == [2] * len(ws)
    F, grads = res[0]
    assert np.all(np.isfinite(F)) and all(np.all(np.isfinite(g)) for g in grads)


def test_batch_validation(gpu):
    ws = uneven(100, count=2)
    with pytest.raises(gpu.FDTDError) as e:
        gpu.Batch([ws[0], W.with_(ws[1], n_steps=50)])
    assert e.value.name == "EINVAL"
    with pytest.raises(gpu.FDTDError):
        gpu.Batch([ws[0], W.tiny3d(precision=32)])
    for opts in (dict(depth=3), dict(depth=-1), dict(depth=2, rows=4), dict(depth=2, rows=1)):
        with pytest.raises(gpu.FDTDError) as e:
            gpu.Batch(ws, **opts)
        assert e.value.name == "EINVAL", opts
    b = gpu.Batch(ws)
    with pytest.raises(gpu.FDTDError) as e:
        b.forward()
    assert e.value.name == "ESTATE"
    b.close()


def test_c4_batch_shape(gpu):
    """The batched uneven workload: 64 instances with sides in {128, 256, 512,
    1024}, own damping and band, autotuned depths, graph replay; sampled
    instances against single contexts with the same depth (300 steps)."""
    ws = W.c4(n_steps=300)
    rhos = [W.seeded_rho(w, k) for k, w in enumerate(ws)]
    b = gpu.Batch(ws, rows=0, use_graph=True)
    for k, r in enumerate(rhos):
        b.set_density(k, r.astype(np.float32))
    F = b.forward()
    b.adjoint()
    info = [b.info(k) for k in range(len(ws))]
    say(f"[batch] C4 shape: 64 instances, tile depths {sorted(set(i['rows'] for i in info))}, "
        f"temporal-block depths by side {sorted(set((w['n'][0], i['depth']) for w, i in zip(ws, info)))}, "
        f"fwd {info[0]['forward_ms']:.1f} ms adj {info[0]['adjoint_ms']:.1f} ms for 300 steps")
    for k in (0, 17, 40, 63):
        g = gpu.FDTD(ws[k])
        g.set_density(rhos[k].astype(np.float32))
        Fk = g.forward()
        g.adjoint()
        gk = g.gradient()
        g.close()
        gb = b.gradient(k)
        assert abs(F[k] - Fk) <= 1e-5 * abs(Fk), (k, F[k], Fk)
        assert np.linalg.norm(gb - gk) <= 1e-4 * np.linalg.norm(gk), k
    b.close()


def oracle_runs(oracle_mod, ws, rhos):
    out = []
    for w, r in zip(ws, rhos):
        o = oracle_mod.Oracle(W.with_(w, precision=64))
        out.append(o.run(r))
        o.close()
    return out


def check_against_oracle(F, grads, ref, prec, label):
    tol_f, tol_g = (1e-11, 1e-11) if prec == 64 else (1e-4, 1e-3)
    for k, (Fo, go) in enumerate(ref):
        eF = abs(F[k] - Fo) / abs(Fo)
        eG = np.linalg.norm(grads[k] - go) / np.linalg.norm(go)
        eM = np.abs(grads[k] - go).max() / np.abs(go).max()
        say(f"[batch-oracle] {label} instance {k}: relF={eF:.2e} relGrad={eG:.2e} maxabs={eM:.2e}")
        assert eF <= tol_f and eG <= tol_g and eM <= 10 * tol_g, (k, eF, eG, eM)


@pytest.mark.parametrize("prec,depth,n_steps", [(64, 1, 400), (64, 2, 401), (32, 1, 400), (32, 2, 400)])
def test_batch_against_oracle(gpu, oracle_mod, prec, depth, n_steps):
    """Every instance of an uneven batch (sides 64-384, own damping and band)
    against the FP64 oracle on the same seeded inputs, at temporal-block depth
    1 and 2: FP64 to 1e-11, FP32 to 1e-4 on F and 1e-3 on the gradient (rel
    L2), max |error| within 10x the gradient bar of the largest entry."""
    ws = uneven(n_steps, precision=prec, sides=(64, 160, 256, 384))
    rhos = [W.seeded_rho(w, k) for k, w in enumerate(ws)]
    (res,), _, dep = run_batch(gpu, ws, rhos, 2, True, depth=depth)
    if depth == 2:
        assert any(d == 2 for d in dep)
    check_against_oracle(res[0], res[1], oracle_runs(oracle_mod, ws, rhos), prec, f"fp{prec} depth {depth}")


@pytest.mark.parametrize("prec", [64, 32])
def test_c4_batch_sampled_against_oracle(gpu, oracle_mod, prec):
    """The 64-instance uneven workload (sides 128-1024) batched with the tuned
    depths, 1500 steps (long enough for the pulse to reach the gap of every
    side); one instance of each side against the oracle."""
    ws = [W.with_(w, precision=prec) for w in W.c4(n_steps=1500)]
    rhos = [W.seeded_rho(w, k) for k, w in enumerate(ws)]
    b = gpu.Batch(ws, rows=0, use_graph=True, depth=0)
    for k, r in enumerate(rhos):
        b.set_density(k, r.astype(b.dtype))
    F = b.forward()
    b.adjoint()
    pick, seen = [], set()
    for k, w in enumerate(ws):
        if w["n"][0] not in seen:
            seen.add(w["n"][0])
            pick.append(k)
    grads = [b.gradient(k) for k in pick]
    depths = [b.info(k)["depth"] for k in pick]
    b.close()
    say(f"[batch-oracle] C4 sample: instances {pick}, sides {[ws[k]['n'][0] for k in pick]}, depths {depths}")
    ref = oracle_runs(oracle_mod, [ws[k] for k in pick], [rhos[k] for k in pick])
    check_against_oracle([F[k] for k in pick], grads, ref, prec, f"C4 fp{prec}")
