"""CPU oracle for the Drude-FDTD forward/adjoint/sensitivity path (FP64, plain C).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The product path (the HIP library and
its binding) never imports this package, and this package imports nothing
from the product path.

The C sources (``fdtd2d.c``: 2D TMz; ``fdtd2d_te.c``: 2D TEz, E in the
plane; ``fdtd3d.c``) state which passage of the paper each step follows.  ``build()`` compiles them into ``liboracle_fdtd.so`` with
gcc, ``-O2 -ffp-contract=off``, OpenMP over the outer spatial loop.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_fdtd.so")
SOURCES = ["fdtd2d.c", "fdtd2d_te.c", "fdtd3d.c"]

C0 = 299792458.0

SRC_KIND = {"gauss": 0, "sinc_hann": 1, "none": 2}
OBJ_KIND = {"dft": 0, "time_energy": 1}
W_KIND = {"enhancement": 0, "unit": 1}
ERRORS = {1: "EINVAL", 2: "ESTATE", 3: "ENOMEM", 5: "EUNSTABLE"}


def build(verbose=False):
    """Compile the oracle with gcc (always rebuilds)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99",
           "-D_DEFAULT_SOURCE", "-Wall", "-shared", "-fPIC", "-o", LIB_PATH + ".tmp", *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Cfg(C.Structure):
    _fields_ = [
        ("dims", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("n_steps", C.c_int32), ("pml_cells", C.c_int32), ("tfsf_margin", C.c_int32),
        ("periodic_x", C.c_int32),
        ("design_lo", C.c_int32 * 3), ("design_n", C.c_int32 * 3),
        ("gap_lo", C.c_int32 * 3), ("gap_n", C.c_int32 * 3),
        ("source_kind", C.c_int32), ("objective_kind", C.c_int32), ("weight_kind", C.c_int32),
        ("n_freq", C.c_int32),
        ("dx", C.c_double), ("courant", C.c_double),
        ("pml_order", C.c_double), ("pml_sigma_scale", C.c_double),
        ("pml_kappa_max", C.c_double), ("pml_alpha_max", C.c_double),
        ("eps_s", C.c_double), ("eps_g", C.c_double), ("eps_inf", C.c_double),
        ("omega_p", C.c_double), ("gamma_p", C.c_double), ("gamma_mult", C.c_double),
        ("sigma_max", C.c_double), ("psi_s_ratio", C.c_double),
        ("f_lo", C.c_double), ("f_hi", C.c_double), ("t0_over_tau", C.c_double),
        ("amplitude", C.c_double),
        ("freqs_hz", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        for pre in ("or2d", "orte", "or3d"):
            if not hasattr(L, pre + "_create"):
                continue
            getattr(L, pre + "_create").argtypes = [C.POINTER(_Cfg), C.POINTER(P)]
            getattr(L, pre + "_destroy").argtypes = [P]
            getattr(L, pre + "_destroy").restype = None
            getattr(L, pre + "_last_error").argtypes = [P]
            getattr(L, pre + "_last_error").restype = C.c_char_p
            getattr(L, pre + "_set_density").argtypes = [P, dp]
            getattr(L, pre + "_forward").argtypes = [P, dp]
            getattr(L, pre + "_adjoint").argtypes = [P]
            getattr(L, pre + "_gradient").argtypes = [P, dp, dp, dp, dp]
            getattr(L, pre + "_get_dft").argtypes = [P, dp]
            getattr(L, pre + "_get_gap_series").argtypes = [P, dp]
            getattr(L, pre + "_info").argtypes = [P, dp, dp, dp, C.POINTER(C.c_int32)]
            getattr(L, pre + "_info").restype = None
            getattr(L, pre + "_forward_ext").argtypes = [P, dp, dp]
            getattr(L, pre + "_adjoint_ext").argtypes = [P, dp, dp]
            getattr(L, pre + "_step_free").argtypes = [P, C.c_int]
            if pre != "orte":
                getattr(L, pre + "_incident_column").argtypes = [P, C.c_int, dp]
                getattr(L, pre + "_set_checkpoint").argtypes = [P, C.c_int]
        dpa = C.POINTER(dp)
        L.or3d_set_state.argtypes = [P, dpa, dpa, dpa]
        L.or3d_get_state.argtypes = [P, dpa, dpa, dpa]
        L.or2d_set_state.argtypes = [P, dp, dp, dp, dp]
        L.or2d_get_state.argtypes = [P, dp, dp, dp, dp]
        L.orte_set_state.argtypes = [P, dp, dp, dp, dp, dp]
        L.orte_get_state.argtypes = [P, dp, dp, dp, dp, dp]
        L.orte_sizes.argtypes = [P, C.POINTER(C.c_int32)]
        L.orte_sizes.restype = None
        L.or2d_num_threads.restype = C.c_int
        _lib = L
    return _lib


def num_threads():
    return lib().or2d_num_threads()


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def band_hz(w):
    """Band edges in Hz from the workload's wavelength band."""
    return C0 / w["lambda_hi"], C0 / w["lambda_lo"]


def make_cfg(w):
    """Translate a workload dict into the oracle's own C struct."""
    c = _Cfg()
    c.dims = w["dims"]
    c.nx, c.ny, c.nz = w["n"]
    c.n_steps = w["n_steps"]
    c.pml_cells = w["pml_cells"]
    c.tfsf_margin = w["tfsf_margin"]
    c.periodic_x = 1 if w.get("periodic_x") else 0
    for k in range(3):
        c.design_lo[k] = w["design_lo"][k]
        c.design_n[k] = w["design_n"][k]
        c.gap_lo[k] = w["gap_lo"][k]
        c.gap_n[k] = w["gap_n"][k]
    c.source_kind = SRC_KIND[w["source"]]
    c.objective_kind = OBJ_KIND[w["objective"]]
    c.weight_kind = W_KIND[w["weights"]]
    c.dx = w["dx"]
    c.courant = w["courant"]
    for k in ("pml_order", "pml_sigma_scale", "pml_kappa_max", "pml_alpha_max", "eps_s", "eps_g",
              "eps_inf", "omega_p", "gamma_p", "gamma_mult", "sigma_max", "psi_s_ratio",
              "t0_over_tau", "amplitude"):
        setattr(c, k, float(w[k]))
    c.f_lo, c.f_hi = band_hz(w)
    keep = None
    if w.get("freqs_hz") is not None:
        keep = np.ascontiguousarray(np.asarray(w["freqs_hz"], dtype=np.float64))
        c.n_freq = len(keep)
        c.freqs_hz = _dp(keep)
    else:
        c.n_freq = w["n_freq"]
        c.freqs_hz = C.POINTER(C.c_double)()
    return c, keep


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


def is_te(w):
    """2D with E in the plane (E along x): the TEz oracle."""
    return w["dims"] == 2 and w.get("pol_axis") == "x"


class Oracle:
    """One problem instance of the CPU oracle (2D TMz, 2D TEz or 3D)."""

    def __init__(self, w, ckpt_every=0):
        """ckpt_every = K > 0 keeps K steps of design-edge history plus a
        snapshot of the state every K steps; the adjoint re-runs each segment
        (same results as the full history, bounded host memory; TMz and 3D)."""
        self.w = dict(w)
        self.dims = w["dims"]
        self.te = is_te(w)
        self.pre = "orte" if self.te else "or2d" if self.dims == 2 else "or3d"
        L = lib()
        cfg, keep = make_cfg(w)
        h = C.c_void_p()
        rc = getattr(L, self.pre + "_create")(C.byref(cfg), C.byref(h))
        if rc:
            raise OracleError(rc, getattr(L, self.pre + "_last_error")(None).decode())
        self.h = h
        self.K = cfg.n_freq
        nx, ny, nz = w["n"]
        self.shape = (nz, ny, nx) if self.dims == 3 else (ny, nx)
        gx, gy, gz = w["gap_n"]
        self.ng = gx * gy * (gz if self.dims == 3 else 1)
        self.ncomp = 3 if self.dims == 3 else 1
        dnx, dny, dnz = w["design_n"]
        self.dshape = (dnz, dny, dnx) if self.dims == 3 else (dny, dnx)
        self.N = w["n_steps"]
        if self.te:
            # per-edge layout: the design box's E_x edges, then its E_y edges
            sz = (C.c_int32 * 4)()
            L.orte_sizes(self.h, sz)
            self.nd, self.ndx, self.ng, self.ngx = tuple(sz)
            self.dshape = (self.nd,)
            if ckpt_every:
                raise OracleError(1, "checkpointing is not built for the TEz oracle")
        elif ckpt_every:
            self._check(self._fn("set_checkpoint")(self.h, int(ckpt_every)))

    def _fn(self, name):
        return getattr(lib(), self.pre + "_" + name)

    def _check(self, rc):
        if rc:
            msg = self._fn("last_error")(self.h).decode()
            raise OracleError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            self._fn("destroy")(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        dt = C.c_double()
        f = np.zeros(self.K)
        wts = np.zeros(self.K)
        box = (C.c_int32 * 6)()
        self._fn("info")(self.h, C.byref(dt), _dp(f), _dp(wts), box)
        return dict(dt=dt.value, freqs=f, weights=wts, tf_box=tuple(box))

    def set_density(self, rho):
        r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64).reshape(self.dshape))
        self._check(self._fn("set_density")(self.h, _dp(r)))

    def forward(self):
        F = C.c_double()
        self._check(self._fn("forward")(self.h, C.byref(F)))
        return F.value

    def adjoint(self):
        self._check(self._fn("adjoint")(self.h))

    def gradient(self, partials=False):
        g = np.zeros(self.dshape)
        if not partials:
            self._check(self._fn("gradient")(self.h, _dp(g), None, None, None))
            return g
        fe, fp, fs = np.zeros(self.dshape), np.zeros(self.dshape), np.zeros(self.dshape)
        self._check(self._fn("gradient")(self.h, _dp(g), _dp(fe), _dp(fp), _dp(fs)))
        return g, dict(eps_inf=fe, psi=fp, sigma=fs)

    def dft(self):
        """Gap DFT as complex array [K][gap cell][component]."""
        out = np.zeros(self.K * self.ng * self.ncomp * 2)
        self._check(self._fn("get_dft")(self.h, _dp(out)))
        out = out.reshape(self.K, self.ng, self.ncomp, 2)
        return out[..., 0] + 1j * out[..., 1]

    def gap_series(self):
        out = np.zeros((self.N + 1) * self.ng * self.ncomp)
        self._check(self._fn("get_gap_series")(self.h, _dp(out)))
        return out.reshape(self.N + 1, self.ng, self.ncomp)

    def incident_column(self, j):
        out = np.zeros(self.N + 1)
        self._check(self._fn("incident_column")(self.h, int(j), _dp(out)))
        return out

    def run(self, rho):
        """forward + adjoint + gradient; returns (F, dF/drho)."""
        self.set_density(rho)
        F = self.forward()
        self.adjoint()
        return F, self.gradient()

    # -- test hooks ------------------------------------------------------
    def forward_ext(self, q):
        """q: [N][ny][nx] (2D) or [N][3][nz][ny][nx] (3D) extra source in the curl bracket."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros_like(q)
        self._check(self._fn("forward_ext")(self.h, _dp(q), _dp(out)))
        return out

    def adjoint_ext(self, s):
        s = np.ascontiguousarray(s, dtype=np.float64)
        out = np.zeros_like(s)
        self._check(self._fn("adjoint_ext")(self.h, _dp(s), _dp(out)))
        return out

    def set_state(self, *fields):
        """2D TMz: (Ez, Hx, Hy, J).  2D TEz: (Ex, Ey, Hz, Jx, Jy).  3D: (E[3],
        H[3], J[3]) lists of arrays."""
        if self.te:
            arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape) for a in fields]
            self._check(lib().orte_set_state(self.h, *[_dp(a) for a in arrs]))
            return
        if self.dims == 2:
            arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape) for a in fields]
            self._check(lib().or2d_set_state(self.h, *[_dp(a) for a in arrs]))
            return
        self._keep = []
        ptrs = []
        for group in fields:
            arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape) for a in group]
            self._keep += arrs
            ptrs.append((C.POINTER(C.c_double) * 3)(*[_dp(a) for a in arrs]))
        self._check(lib().or3d_set_state(self.h, *ptrs))

    def get_state(self):
        if self.te:
            arrs = [np.zeros(self.shape) for _ in range(5)]
            self._check(lib().orte_get_state(self.h, *[_dp(a) for a in arrs]))
            return arrs
        if self.dims == 2:
            arrs = [np.zeros(self.shape) for _ in range(4)]
            self._check(lib().or2d_get_state(self.h, *[_dp(a) for a in arrs]))
            return arrs
        groups = [[np.zeros(self.shape) for _ in range(3)] for _ in range(3)]
        ptrs = [(C.POINTER(C.c_double) * 3)(*[_dp(a) for a in g]) for g in groups]
        self._check(lib().or3d_get_state(self.h, *ptrs))
        return groups

    def step_free(self, k):
        self._check(self._fn("step_free")(self.h, int(k)))
