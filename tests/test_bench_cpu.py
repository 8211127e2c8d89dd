"""bench.py's roofline numerator: the algorithmic bytes per time step, checked
against the per-cell model written out by hand (each array read once and
written once per step; FP32): 2D 24 B per cell (E_z, H_x, H_y) + 8 B per
absorber-memory pair over the CPML strips + design-edge bytes; 3D 48 B per
cell + 8 B per memory pair (4 pairs per slab direction) + design-edge bytes.
Also the one-GPU contract of the command line, and that the counter-measured
traffic records belong to the sources as they stand."""
import os
import subprocess
import sys

import fdtd_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_c2_bytes_per_step():
    w = W.c2()
    n, P, d = 2048, 32, 512 * 512
    fields = n * n * 3 * 2 * 4
    strips = 2 * (2 * P) * (n + n) * 2 * 4           # two memory arrays per strip, x and y strips
    fwd = fields + strips + d * (4 + 4 * 2 + 4)      # rho; J read + write; history write
    adj = fields + strips + d * (4 + 4 * 2 + 4 + 16)  # ... history read; FP64 sum read + write
    assert bench.algorithmic_bytes(w, False) == fwd == 109051904
    assert bench.algorithmic_bytes(w, True) == adj == 113246208


def test_c3_bytes_per_step():
    w = W.c3()
    n, P = 256, 16
    d = 128 * 128 * 32
    fields = n ** 3 * 6 * 2 * 4
    slabs = 4 * (2 * P) * (3 * n * n) * 2 * 4        # four memory pairs per slab direction, three directions
    fwd = fields + slabs + d * (4 + 3 * (2 * 4 + 4))
    adj = fields + slabs + d * (4 + 3 * (2 * 4 + 4 + 16))
    assert bench.algorithmic_bytes(w, False) == fwd
    assert bench.algorithmic_bytes(w, True) == adj
    # the figures the 3D bench line and its profile quote
    assert round(fwd / 1e6, 1) == 1027.6 and round(adj / 1e6, 1) == 1052.8


def test_measured_traffic_records_match_sources_and_profiles():
    """Every counter-measured traffic record was taken on the kernel sources
    as they stand (so bench.py reports it rather than null), and the profile
    summary it cites names the same source hash."""
    for name, rec in bench.MEASURED_TRAFFIC.items():
        assert bench.sources_sha(rec["sources"]) == rec["sha256_16"], name
        with open(os.path.join(ROOT, rec["profile"])) as f:
            assert rec["sha256_16"] in f.read(), name
        assert 0 < rec["fwd"] and 0 < rec["adj"], name


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
