"""Surrogate pipeline on a small TMz instance (128x128 grid, 32x32 design box).

The training triples produced through the batched solver must be the triples a
single FDTD context gives for the same filtered density; the guided loop must
only ever keep FDTD-checked improvements.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import fdtd_workloads as W
    from paper_2203_01462_amd import FDTD, surrogate
    return W, FDTD, surrogate


def small(W):
    return W.instance2d(128, 1.0, 500e-9, 1000e-9, 1500, name="tmz2d_128_s")


def test_generated_triples_match_single_context(mods):
    W, FDTD, S = mods
    w = small(W)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        data = S.generate(w, 6, alpha=1.0, seed=5, batch=4)
        torch.cuda.synchronize()
        assert data.n == 6
        sol = FDTD(w)
        for i in (0, 3, 5):
            rho = data.rho[i].cpu().numpy()
            F, g = sol.run(rho)
            assert abs(np.log(F) - float(data.logF[i])) <= 1e-5
            G = data.G[i].cpu().numpy().astype(np.float64)
            ref = g / F
            assert np.linalg.norm(G - ref) <= 1e-4 * np.linalg.norm(ref)
        sol.close()


def test_compare_runs_and_keeps_improvements(mods):
    W, FDTD, S = mods
    w = small(W)
    res = S.compare(samples=64, train_steps=40, batch=4, plain_iters=3, checks=3, inner=3, w=w,
                    settings=((0.1, 2), (0.2, 0), ((0.1, 0.2, 0.3), 2)), log=lambda m: None)
    assert len(res["guided"]) == 3
    for run in res["guided"]:
        g = [F for _, F in run["trace"]]
        assert all(b >= a for a, b in zip(g, g[1:])), g
        st = run["stats"]
        assert st["checks"] == 3 and st["accepted"] + st["fallback"] == 3
        assert run["trace"][0][0] == 0.0
        # both loops start from the same design and physics
        assert abs(res["plain_trace"][0][1] - g[0]) <= 1e-5 * abs(g[0])
    # every run checks a surrogate iterate, never the unmoved design
    assert res["guided"][0]["stats"]["best_step"][0] >= 1
    # three proposals per check, solved together: 3 forward + 3 adjoint per check
    # beside the start design's solves and any fallback steps
    assert res["guided"][2]["stats"]["solves"] >= 2 + 6 * 3
    assert res["plain_trace"][0][0] == 0.0
    assert np.isfinite(res["val"]["grad_cos_mean"])
