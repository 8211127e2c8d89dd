"""Write the full-size expected values of the 2D 2048^2 x 20000-step and 3D
256^3 x 8000-step workloads (seed-0 densities) with the CPU oracle alone.

The oracle runs in FP64 with segment checkpointing (a snapshot every 500
steps; each segment re-run in the adjoint), which gives the same results as
its stored history (tests/test_oracle_checkpoint.py) within bounded host
memory.  Each file holds the objective F, the gap DFT [K][gap cell][component]
and dF/drho over the design box (eq. (27), filter = identity), plus the
workload description it was computed for.

    python tests/golden/make_fullsize.py c2      # ~15 min on 8 cores
    python tests/golden/make_fullsize.py c3      # ~2 h on 8 cores, ~30 GB of host memory
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import fdtd_workloads as W  # noqa: E402
import oracle  # noqa: E402

CASES = {"c2": lambda: W.c2(gamma_mult=1.0), "c3": W.c3}
CKPT = 500


def path(name):
    return os.path.join(HERE, f"fullsize_{name}_seed0.npz")


def make(name):
    w = W.with_(CASES[name](), precision=64)
    rho = W.seeded_rho(w, 0)
    t0 = time.time()
    o = oracle.Oracle(w, ckpt_every=CKPT)
    o.set_density(rho)
    F = o.forward()
    t1 = time.time()
    print(f"{name}: forward F = {F:.17e} ({t1 - t0:.0f} s)", flush=True)
    d = o.dft()
    o.adjoint()
    g = o.gradient()
    t2 = time.time()
    print(f"{name}: adjoint + gradient ({t2 - t1:.0f} s), |g| = {np.linalg.norm(g):.6e}", flush=True)
    o.close()
    meta = dict(workload={k: v for k, v in w.items() if k != "freqs_hz"}, seed=0, density="smooth",
                ckpt_every=CKPT, threads=oracle.num_threads(), seconds=round(t2 - t0, 1))
    np.savez_compressed(path(name), F=np.float64(F), dft=d, grad=g, meta=json.dumps(meta))
    print(f"{name}: wrote {path(name)}", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c2", "c3"]:
        make(n)
