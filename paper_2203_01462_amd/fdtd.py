"""ctypes binding of the C ABI in ``include/fdtd.h`` (argument marshalling only).

Every step of a solve runs in the HIP library: this module translates a
workload description into ``fdtd_config``, passes host arrays or torch device
pointers through, and raises on non-zero status codes.  There is no fallback:
if the library is missing or no HIP device is usable, construction raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd_hip.so")
ABI_VERSION = 5
C0 = 299792458.0

STATUS = {0: "OK", 1: "EINVAL", 2: "ESTATE", 3: "ENOMEM", 4: "EDEVICE", 5: "EUNSTABLE"}
SRC = {"gauss": 0, "sinc_hann": 1, "none": 2}
AXIS = {None: -1, "x": 0, "y": 1, "z": 2}
OBJ = {"dft": 0, "time_energy": 1}
WTS = {"enhancement": 0, "unit": 1}


class FDTDError(RuntimeError):
    def __init__(self, code, msg):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"{self.name}: {msg}")


class Config(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("dims", C.c_int32), ("precision", C.c_int32),
        ("n", C.c_int32 * 3), ("n_steps", C.c_int32), ("pml_cells", C.c_int32),
        ("tfsf_margin", C.c_int32), ("pol_axis", C.c_int32), ("prop_axis", C.c_int32),
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
        ("history_budget_bytes", C.c_int64),
        ("ckpt_every", C.c_int32),
        ("stream", C.c_void_p),
    ]


class Timing(C.Structure):
    _fields_ = [("forward_ms", C.c_double), ("adjoint_ms", C.c_double),
                ("forward_launches", C.c_int64), ("adjoint_launches", C.c_int64),
                ("cells", C.c_int64), ("design_cells", C.c_int64)]


class BatchOptions(C.Structure):
    _fields_ = [("rows", C.c_int32), ("use_graph", C.c_int32), ("depth", C.c_int32)]


# Every symbol the header declares (checked by the CPU tests).
EXPORTS = ["fdtd_abi_version", "fdtd_create", "fdtd_set_density", "fdtd_forward", "fdtd_adjoint",
           "fdtd_gradient", "fdtd_get_dft", "fdtd_set_state", "fdtd_get_state", "fdtd_get_timing",
           "fdtd_destroy", "fdtd_last_error",
           "fdtd_batch_create", "fdtd_batch_set_density", "fdtd_batch_forward", "fdtd_batch_adjoint",
           "fdtd_batch_gradient", "fdtd_batch_info", "fdtd_batch_depth", "fdtd_batch_destroy", "fdtd_batch_last_error",
           # include/fdtd_design.h
           "fdtd_filter_create", "fdtd_filter_apply", "fdtd_filter_transpose", "fdtd_filter_destroy",
           "fdtd_mma_create", "fdtd_mma_begin", "fdtd_mma_solve", "fdtd_mma_accept", "fdtd_mma_destroy",
           "fdtd_design_stats", "fdtd_design_last_error",
           # include/fdtd_nn.h
           "fdtd_nn_conv3x3", "fdtd_nn_conv3x3_dgrad", "fdtd_nn_conv3x3_dgrad_relu", "fdtd_nn_rot_weights",
           "fdtd_nn_wgrad_work",
           "fdtd_nn_conv3x3_wgrad", "fdtd_nn_conv3x3_wgrad_noalloc",
           "fdtd_nn_relu_bf16", "fdtd_nn_relu_bf16_backward", "fdtd_nn_to_bf16", "fdtd_nn_from_bf16",
           "fdtd_nn_pool2", "fdtd_nn_pool2_backward", "fdtd_nn_up2", "fdtd_nn_up2_backward", "fdtd_nn_adam",
           "fdtd_nn_axpy", "fdtd_nn_gap_linear", "fdtd_nn_gap_linear_backward", "fdtd_nn_mse_work", "fdtd_nn_mse",
           "fdtd_nn_last_error"]

_lib = None


def load_library(path=LIB_PATH):
    """Load libfdtd_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is missing: run __graft_entry__.build() first")
    # torch provides device memory and streams; importing it first makes the
    # library bind to the HIP runtime torch has already loaded (same SONAME),
    # so one process never holds two HIP runtimes.
    import torch  # noqa: F401
    L = C.CDLL(path)
    P = C.c_void_p
    L.fdtd_abi_version.restype = C.c_int32
    L.fdtd_create.argtypes = [C.POINTER(Config), C.POINTER(P)]
    L.fdtd_set_density.argtypes = [P, P, C.c_int64, C.c_int32]
    L.fdtd_forward.argtypes = [P, C.POINTER(C.c_double)]
    L.fdtd_adjoint.argtypes = [P]
    L.fdtd_gradient.argtypes = [P, P, C.c_int64, C.c_int32]
    L.fdtd_get_dft.argtypes = [P, C.POINTER(C.c_double), C.c_int64]
    L.fdtd_set_state.argtypes = [P, C.POINTER(C.c_double), C.c_int64]
    L.fdtd_get_state.argtypes = [P, C.POINTER(C.c_double), C.c_int64]
    L.fdtd_get_timing.argtypes = [P, C.POINTER(Timing)]
    L.fdtd_destroy.argtypes = [P]
    L.fdtd_last_error.argtypes = [P]
    L.fdtd_last_error.restype = C.c_char_p
    L.fdtd_batch_create.argtypes = [C.POINTER(Config), C.c_int32, C.POINTER(BatchOptions), C.POINTER(P)]
    L.fdtd_batch_set_density.argtypes = [P, C.c_int32, P, C.c_int64, C.c_int32]
    L.fdtd_batch_forward.argtypes = [P, C.POINTER(C.c_double)]
    L.fdtd_batch_adjoint.argtypes = [P]
    L.fdtd_batch_gradient.argtypes = [P, C.c_int32, P, C.c_int64, C.c_int32]
    L.fdtd_batch_info.argtypes = [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.fdtd_batch_depth.argtypes = [P, C.c_int32, C.POINTER(C.c_int32)]
    L.fdtd_batch_destroy.argtypes = [P]
    L.fdtd_batch_last_error.argtypes = [P]
    L.fdtd_batch_last_error.restype = C.c_char_p
    D = C.c_double
    L.fdtd_filter_create.argtypes = [C.POINTER(C.c_int32), D, C.c_int32, P, C.POINTER(P)]
    L.fdtd_filter_apply.argtypes = [P, P, P, D]
    L.fdtd_filter_transpose.argtypes = [P, P, P]
    L.fdtd_filter_destroy.argtypes = [P]
    L.fdtd_mma_create.argtypes = [C.c_int64, C.c_int32, D, D, D, D, D, D, P, C.POINTER(P)]
    L.fdtd_mma_begin.argtypes = [P, P, D, P, C.POINTER(D)]
    L.fdtd_mma_solve.argtypes = [P, D, P, C.POINTER(D), C.POINTER(D)]
    L.fdtd_mma_accept.argtypes = [P, P]
    L.fdtd_mma_destroy.argtypes = [P]
    L.fdtd_design_stats.argtypes = [C.c_int64, C.c_int32, P, P, D, D, P, C.POINTER(D)]
    L.fdtd_design_last_error.argtypes = []
    L.fdtd_design_last_error.restype = C.c_char_p
    for fn in ("fdtd_filter_create", "fdtd_filter_apply", "fdtd_filter_transpose", "fdtd_filter_destroy",
               "fdtd_mma_create", "fdtd_mma_begin", "fdtd_mma_solve", "fdtd_mma_accept", "fdtd_mma_destroy",
               "fdtd_design_stats"):
        getattr(L, fn).restype = C.c_int
    I32, I64, F = C.c_int32, C.c_int64, C.c_float
    nn = {
        "fdtd_nn_conv3x3": [I32, I32, I32, I32, I32, P, P, P, P, P, P],
        "fdtd_nn_conv3x3_dgrad": [I32, I32, I32, I32, I32, P, P, P, P, P],
        "fdtd_nn_conv3x3_dgrad_relu": [I32, I32, I32, I32, I32, P, P, P, P, P, P],
        "fdtd_nn_rot_weights": [I32, P, P, P, P, P, P],
        "fdtd_nn_conv3x3_wgrad": [I32, I32, I32, I32, I32, P, P, P, P, P, P],
        "fdtd_nn_conv3x3_wgrad_noalloc": [I32, I32, I32, I32, I32, P, P, P, P, P],
        "fdtd_nn_relu_bf16": [I64, P, P, P],
        "fdtd_nn_relu_bf16_backward": [I64, P, P, P, P],
        "fdtd_nn_to_bf16": [I64, P, P, P],
        "fdtd_nn_from_bf16": [I64, P, P, P],
        "fdtd_nn_pool2": [I64, I32, I32, P, P, P],
        "fdtd_nn_pool2_backward": [I64, I32, I32, P, P, P],
        "fdtd_nn_up2": [I64, I32, I32, P, P, P],
        "fdtd_nn_up2_backward": [I64, I32, I32, P, P, P],
        "fdtd_nn_adam": [I64, P, P, P, P, P, F, F, F, F, I32, P],
        "fdtd_nn_axpy": [I64, F, P, P, P],
        "fdtd_nn_gap_linear": [I32, I32, I32, P, P, P, P, P],
        "fdtd_nn_gap_linear_backward": [I32, I32, I32, P, P, P, P, P, P, P],
        "fdtd_nn_mse": [I64, P, P, F, P, P, P, P],
    }
    for fn, a in nn.items():
        getattr(L, fn).argtypes = a
        getattr(L, fn).restype = C.c_int
    L.fdtd_nn_wgrad_work.argtypes = [I32, I32, I32, I32, I32]
    L.fdtd_nn_wgrad_work.restype = I64
    L.fdtd_nn_mse_work.argtypes = [I64]
    L.fdtd_nn_mse_work.restype = I64
    L.fdtd_nn_last_error.argtypes = []
    L.fdtd_nn_last_error.restype = C.c_char_p
    for fn in ("fdtd_create", "fdtd_set_density", "fdtd_forward", "fdtd_adjoint", "fdtd_gradient",
               "fdtd_get_dft", "fdtd_set_state", "fdtd_get_state", "fdtd_get_timing", "fdtd_destroy",
               "fdtd_batch_create", "fdtd_batch_set_density",
               "fdtd_batch_forward", "fdtd_batch_adjoint", "fdtd_batch_gradient", "fdtd_batch_info",
               "fdtd_batch_depth", "fdtd_batch_destroy"):
        getattr(L, fn).restype = C.c_int
    if L.fdtd_abi_version() != ABI_VERSION:
        raise ImportError("libfdtd_hip.so ABI version mismatch")
    _lib = L
    return L


def make_config(w, stream=None, history_budget_bytes=0, ckpt_every=None):
    """Translate a workload dict into fdtd_config (pure marshalling).
    ``ckpt_every`` (or the workload's "ckpt_every"): 0 stores the whole forward
    history, K > 0 checkpoints every K steps."""
    c = Config()
    c.abi_version = ABI_VERSION
    c.dims = w["dims"]
    c.precision = w["precision"]
    for k in range(3):
        c.n[k] = w["n"][k]
        c.design_lo[k] = w["design_lo"][k]
        c.design_n[k] = w["design_n"][k]
        c.gap_lo[k] = w["gap_lo"][k]
        c.gap_n[k] = w["gap_n"][k]
    c.n_steps = w["n_steps"]
    c.pml_cells = w["pml_cells"]
    c.tfsf_margin = w["tfsf_margin"]
    c.pol_axis = AXIS[w.get("pol_axis")]
    c.prop_axis = AXIS[w.get("prop_axis")]
    c.source_kind = SRC[w["source"]]
    c.objective_kind = OBJ[w["objective"]]
    c.weight_kind = WTS[w["weights"]]
    c.dx = w["dx"]
    c.courant = w["courant"]
    for k in ("pml_order", "pml_sigma_scale", "pml_kappa_max", "pml_alpha_max", "eps_s", "eps_g",
              "eps_inf", "omega_p", "gamma_p", "gamma_mult", "sigma_max", "psi_s_ratio",
              "t0_over_tau", "amplitude"):
        setattr(c, k, float(w[k]))
    c.f_lo = C0 / w["lambda_hi"]
    c.f_hi = C0 / w["lambda_lo"]
    keep = None
    if w.get("freqs_hz") is not None:
        keep = np.ascontiguousarray(np.asarray(w["freqs_hz"], dtype=np.float64))
        c.n_freq = len(keep)
        c.freqs_hz = keep.ctypes.data_as(C.POINTER(C.c_double))
    else:
        c.n_freq = w["n_freq"]
        c.freqs_hz = C.POINTER(C.c_double)()
    c.history_budget_bytes = int(history_budget_bytes)
    c.ckpt_every = int(w.get("ckpt_every", 0) if ckpt_every is None else ckpt_every)
    c.stream = stream
    return c, keep


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class FDTD:
    """One problem instance on the GPU (a context of the HIP library)."""

    def __init__(self, w, stream=None, history_budget_bytes=0, ckpt_every=None):
        L = load_library()
        self.w = dict(w)
        self.dims = w["dims"]
        self.dtype = np.float32 if w["precision"] == 32 else np.float64
        cfg, keep = make_config(w, stream, history_budget_bytes, ckpt_every)
        self.ckpt_every = cfg.ckpt_every
        h = C.c_void_p()
        rc = L.fdtd_create(C.byref(cfg), C.byref(h))
        if rc:
            raise FDTDError(rc, L.fdtd_last_error(None).decode())
        self.h = h
        self.K = cfg.n_freq
        dnx, dny, dnz = w["design_n"]
        gx, gy, gz = w["gap_n"]
        # 2D TEz (E along x): one density per design edge, the box's E_x edges
        # ([dny+1][dnx]) then its E_y edges ([dny][dnx+1]); the gap's edges
        # are its monitors
        self.te = self.dims == 2 and w.get("pol_axis") == "x"
        if self.te:
            self.dshape = (dnx * (dny + 1) + (dnx + 1) * dny,)
            self.ng = gx * (gy + 1) + (gx + 1) * gy if gx > 0 and gy > 0 else 0
        else:
            self.dshape = (dnz, dny, dnx) if self.dims == 3 else (dny, dnx)
            self.ng = gx * gy * (gz if self.dims == 3 else 1)
        self.nd = int(np.prod(self.dshape))
        self.ncomp = 3 if self.dims == 3 else 1

    def _check(self, rc):
        if rc:
            raise FDTDError(rc, load_library().fdtd_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            load_library().fdtd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_density(self, rho):
        """rho: numpy array (host copy) or torch device tensor of the context dtype."""
        L = load_library()
        if _is_torch(rho) and rho.is_cuda:
            if not rho.is_contiguous() or rho.numel() != self.nd:
                raise ValueError("device density must be contiguous with one value per design cell")
            self._check(L.fdtd_set_density(self.h, C.c_void_p(rho.data_ptr()), rho.numel(), 1))
            return
        r = np.ascontiguousarray(np.asarray(rho, dtype=self.dtype).reshape(-1))
        self._check(L.fdtd_set_density(self.h, r.ctypes.data_as(C.c_void_p), r.size, 0))

    def forward(self):
        F = C.c_double()
        self._check(load_library().fdtd_forward(self.h, C.byref(F)))
        return F.value

    def adjoint(self):
        self._check(load_library().fdtd_adjoint(self.h))

    def gradient(self, out=None):
        """dF/drho per design cell: into ``out`` (torch device tensor) or a new numpy array."""
        L = load_library()
        if out is not None and _is_torch(out) and out.is_cuda:
            self._check(L.fdtd_gradient(self.h, C.c_void_p(out.data_ptr()), out.numel(), 1))
            return out
        g = np.zeros(self.nd, dtype=self.dtype)
        self._check(L.fdtd_gradient(self.h, g.ctypes.data_as(C.c_void_p), g.size, 0))
        return g.reshape(self.dshape)

    def run(self, rho):
        self.set_density(rho)
        F = self.forward()
        self.adjoint()
        return F, self.gradient()

    def dft(self):
        n = self.K * self.ng * self.ncomp * 2
        out = np.zeros(n)
        self._check(load_library().fdtd_get_dft(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), n))
        out = out.reshape(self.K, self.ng, self.ncomp, 2)
        return out[..., 0] + 1j * out[..., 1]

    def state_shape(self):
        """(fields, nz, ny, nx) of the test-only state arrays: 2D TMz E_z, H_x,
        H_y, J_z; 2D TEz E_x, E_y, H_z, J_x, J_y (nz = 1); 3D E_x, E_y, E_z,
        H_x, H_y, H_z, J_x, J_y, J_z."""
        nx, ny, nz = self.w["n"]
        if self.dims == 2:
            return (5 if self.te else 4, 1, ny, nx)
        return (9, nz, ny, nx)

    def set_state(self, state):
        """Test only: initial state (E^0, H^{-1/2}, J^0) of the following forward
        solves, array of state_shape() (or None to clear)."""
        L = load_library()
        if state is None:
            self._check(L.fdtd_set_state(self.h, None, 0))
            return
        a = np.ascontiguousarray(np.asarray(state, dtype=np.float64).reshape(-1))
        self._keep_state = a
        self._check(L.fdtd_set_state(self.h, a.ctypes.data_as(C.POINTER(C.c_double)), a.size))

    def get_state(self):
        """Test only: state after the last forward solve, array of state_shape()."""
        out = np.zeros(self.state_shape())
        self._check(load_library().fdtd_get_state(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        return out

    def timing(self):
        t = Timing()
        self._check(load_library().fdtd_get_timing(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Timing._fields_}


class Batch:
    """Uneven 2D instances advanced together (fdtd_batch_*): one launch per
    tile depth per time step (depth 1) or the two-step blocked schedule
    (depth 2), the step sequences replayed from HIP graphs.  rows = 0 and
    depth = 0 tune on the batch at creation."""

    def __init__(self, ws, stream=None, rows=0, use_graph=True, depth=0):
        L = load_library()
        self.ws = [dict(w) for w in ws]
        cfgs = (Config * len(ws))()
        keep = []
        for k, w in enumerate(ws):
            c, kp = make_config(w, stream if k == 0 else None)
            cfgs[k] = c
            keep.append(kp)
        opt = BatchOptions(int(rows), 1 if use_graph else 0, int(depth))
        h = C.c_void_p()
        rc = L.fdtd_batch_create(cfgs, len(ws), C.byref(opt), C.byref(h))
        if rc:
            raise FDTDError(rc, L.fdtd_batch_last_error(None).decode())
        self.h = h
        self.count = len(ws)
        self.dtype = np.float32 if ws[0]["precision"] == 32 else np.float64
        self.dshape = [(w["design_n"][1], w["design_n"][0]) for w in ws]

    def _check(self, rc):
        if rc:
            raise FDTDError(rc, load_library().fdtd_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            load_library().fdtd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_density(self, k, rho):
        L = load_library()
        if _is_torch(rho) and rho.is_cuda:
            self._check(L.fdtd_batch_set_density(self.h, k, C.c_void_p(rho.data_ptr()), rho.numel(), 1))
            return
        r = np.ascontiguousarray(np.asarray(rho, dtype=self.dtype).reshape(-1))
        self._check(L.fdtd_batch_set_density(self.h, k, r.ctypes.data_as(C.c_void_p), r.size, 0))

    def forward(self):
        F = (C.c_double * self.count)()
        self._check(load_library().fdtd_batch_forward(self.h, F))
        return np.array(F[:])

    def adjoint(self):
        self._check(load_library().fdtd_batch_adjoint(self.h))

    def gradient(self, k, out=None):
        L = load_library()
        if out is not None and _is_torch(out) and out.is_cuda:
            self._check(L.fdtd_batch_gradient(self.h, k, C.c_void_p(out.data_ptr()), out.numel(), 1))
            return out
        n = int(np.prod(self.dshape[k]))
        g = np.zeros(n, dtype=self.dtype)
        self._check(L.fdtd_batch_gradient(self.h, k, g.ctypes.data_as(C.c_void_p), n, 0))
        return g.reshape(self.dshape[k])

    def info(self, k):
        r = C.c_int32()
        f = C.c_double()
        a = C.c_double()
        self._check(load_library().fdtd_batch_info(self.h, k, C.byref(r), C.byref(f), C.byref(a)))
        d = C.c_int32()
        self._check(load_library().fdtd_batch_depth(self.h, k, C.byref(d)))
        return {"rows": r.value, "depth": d.value, "forward_ms": f.value, "adjoint_ms": a.value}
