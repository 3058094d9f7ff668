"""ctypes binding of liblbmve.so (the C ABI of include/lbmve.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of the library.  PyTorch provides the device workspace (a uint8 tensor) and
the stream (torch's current stream).  If the library has not been built the
import of this module succeeds but every constructor raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBMVE_LIB", os.path.join(_HERE, "liblbmve.so"))

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EUNSUP, LBM_ENAN, LBM_EFENE = 0, -1, -2, -3, -4, -5, -6
PRECISION = {"fp64": 0, "fp32": 1, "fp16s": 2}
FIELD = {"f": 0, "C": 1, "rho": 2, "u": 3}
FIELD_COMPONENTS = {"f": 38, "C": 6, "rho": 2, "u": 3}


class LbmError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("u_wall", ctypes.c_double),
        ("radius", ctypes.c_double),
        ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("cz", ctypes.c_double),
        ("rho_major", ctypes.c_double), ("rho_minor", ctypes.c_double),
        ("G", ctypes.c_double),
        ("tau", ctypes.c_double * 2),
        ("tau_P", ctypes.c_double * 2),
        ("eta_P", ctypes.c_double * 2),
        ("L2", ctypes.c_double * 2),
        ("chi_lo", ctypes.c_double), ("chi_hi", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("init_noise", ctypes.c_double),
        ("tau_minus", ctypes.c_double * 2),
    ]


class LbmObs(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("mass", ctypes.c_double * 2),
        ("weight", ctypes.c_double),
        ("centroid", ctypes.c_double * 3),
        ("inertia", ctypes.c_double * 3),
        ("D", ctypes.c_double),
        ("theta_deg", ctypes.c_double),
        ("Lp", ctypes.c_double),
        ("umax", ctypes.c_double),
        ("trC_max", ctypes.c_double),
        ("n_components", ctypes.c_int32),
        ("piece_nodes", ctypes.c_int32 * 4),
        ("status", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return dict(step=int(self.step), mass=(self.mass[0], self.mass[1]),
                    weight=self.weight, centroid=tuple(self.centroid),
                    inertia=tuple(self.inertia), D=self.D,
                    theta_deg=self.theta_deg, Lp=self.Lp, umax=self.umax,
                    trC_max=self.trC_max, n_components=int(self.n_components),
                    piece_nodes=[int(v) for v in self.piece_nodes], status=int(self.status))


class LbmLaunch(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("bz", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("grouped", ctypes.c_int32)]


_lib = None

_SIGNATURES = {
    "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lbm_validate": (ctypes.c_int, [ctypes.POINTER(LbmParams)]),
    "lbm_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(LbmParams), ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_init": (ctypes.c_int, [ctypes.POINTER(LbmParams), ctypes.c_void_p, ctypes.c_size_t,
                                ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "lbm_observe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(LbmObs)]),
    "lbm_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t]),
    "lbm_import": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t]),
    "lbm_destroy": (None, [ctypes.c_void_p]),
    "lbm_get_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(LbmLaunch)]),
    "lbm_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(LbmLaunch)]),
    "lbm_step_profiled": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "lbm_steps_done": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "lbm_batch_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(LbmParams), ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_batch_init": (ctypes.c_int, [ctypes.POINTER(LbmParams), ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "lbm_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_batch_observe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(LbmObs)]),
    "lbm_batch_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_size_t]),
    "lbm_batch_import": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_size_t]),
    "lbm_batch_nruns": (ctypes.c_int32, [ctypes.c_void_p]),
    "lbm_batch_state_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "lbm_batch_save_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_size_t]),
    "lbm_batch_load_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_size_t]),
    "sg_param_count": (ctypes.c_int32, []),
    "sg_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "sg_init": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p)]),
    "sg_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sg_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sg_get_working_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sg_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "sg_gradient": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "sg_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]),
    "sg_gradient_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "sg_destroy": (None, [ctypes.c_void_p]),
}

SG_NOALLOC_MAX_ROWS = 1024


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1411_2181_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().lbm_strerror(code).decode()
    except RuntimeError:
        return "library not loaded"


def _check(code: int, what: str):
    if code != LBM_OK:
        raise LbmError(code, what)


def make_params(d: dict, precision: str = "fp64") -> LbmParams:
    """Pack a parameter dictionary (names of lbm_params) into the C struct."""
    p = LbmParams()
    p.nx, p.ny, p.nz = int(d["nx"]), int(d["ny"]), int(d["nz"])
    p.precision = PRECISION[precision]
    p.u_wall = float(d["u_wall"])
    p.radius = float(d["radius"])
    p.cx, p.cy, p.cz = float(d.get("cx", -1.0)), float(d.get("cy", -1.0)), float(d.get("cz", -1.0))
    p.rho_major, p.rho_minor = float(d["rho_major"]), float(d["rho_minor"])
    p.G = float(d["G"])
    for name in ("tau", "tau_P", "eta_P", "L2"):
        v = d[name]
        arr = getattr(p, name)
        arr[0], arr[1] = float(v[0]), float(v[1])
    p.chi_lo = float(d.get("chi_lo", 0.0))
    p.chi_hi = float(d.get("chi_hi", 0.0))
    p.seed = int(d.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    p.init_noise = float(d.get("init_noise", 0.0))
    tm = d.get("tau_minus") or (0.0, 0.0)
    p.tau_minus[0], p.tau_minus[1] = float(tm[0]), float(tm[1])
    return p


def validate(d: dict, precision: str = "fp64") -> int:
    p = make_params(d, precision)
    return lib().lbm_validate(ctypes.byref(p))


def _stream_ptr(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Batch:
    """Independent runs of one precision advanced together (one run = a
    batch of one).  Holds its device workspace as a torch uint8 tensor."""

    def __init__(self, runs: Sequence[dict], precision: str = "fp64", device="cuda:0",
                 stream=None):
        import torch
        L = lib()
        self.nruns = len(runs)
        self.dicts = [dict(r) for r in runs]
        self.precision = precision
        arr = (LbmParams * self.nruns)(*[make_params(r, precision) for r in runs])
        self._arr = arr
        nbytes = ctypes.c_size_t()
        _check(L.lbm_batch_workspace_bytes(arr, self.nruns, ctypes.byref(nbytes)), "workspace size")
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.lbm_batch_init(arr, self.nruns, ctypes.c_void_p(self.workspace.data_ptr()),
                                    nbytes.value, ctypes.c_void_p(_stream_ptr(self.stream)),
                                    ctypes.byref(ctx)), "init")
        self._ctx = ctx

    # ------------------------------------------------------------------
    def _c(self):
        if self._ctx is None or not self._ctx.value:
            raise RuntimeError("context destroyed")
        return self._ctx

    def step(self, steps):
        """Advance every run by ``steps`` (int) or run r by steps[r]."""
        if np.isscalar(steps):
            steps = [int(steps)] * self.nruns
        if len(steps) != self.nruns:
            raise ValueError(f"{len(steps)} step counts for {self.nruns} runs")
        a = (ctypes.c_int32 * self.nruns)(*[int(s) for s in steps])
        _check(lib().lbm_batch_step(self._c(), a), "step")

    def observe(self, components: bool = False, check: bool = False) -> list:
        out = (LbmObs * self.nruns)()
        code = lib().lbm_batch_observe(self._c(), int(components), out)
        if code in (LBM_EINVAL, LBM_EHIP) or (check and code != LBM_OK):
            raise LbmError(code, "observe")
        return [o.as_dict() for o in out]

    def export(self, field: str, run: int = 0) -> np.ndarray:
        d = self.dicts[run]
        shape = (d["nz"], d["ny"], d["nx"])
        n = FIELD_COMPONENTS[field] * int(np.prod(shape))
        buf = np.empty(n, dtype=np.float64)
        _check(lib().lbm_batch_export(self._c(), run, FIELD[field], buf.ctypes.data, n), f"export {field}")
        if field == "f":
            return buf.reshape((2, 19) + shape)
        return buf.reshape((FIELD_COMPONENTS[field],) + shape)

    def import_(self, field: str, values: np.ndarray, run: int = 0):
        v = np.ascontiguousarray(values, dtype=np.float64).ravel()
        _check(lib().lbm_batch_import(self._c(), run, FIELD[field], v.ctypes.data, v.size), f"import {field}")

    def save_state(self, run: int = 0) -> bytes:
        """Raw state of one run (populations as stored, densities, C, step
        count) for a bit-exact restart."""
        n = ctypes.c_size_t()
        _check(lib().lbm_batch_state_bytes(self._c(), run, ctypes.byref(n)), "state_bytes")
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().lbm_batch_save_state(self._c(), run, buf, n.value), "save_state")
        return buf.raw

    def load_state(self, blob: bytes, run: int = 0):
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _check(lib().lbm_batch_load_state(self._c(), run, buf, len(blob)), "load_state")

    def step_profiled(self, nsteps: int) -> float:
        """Eager steps with HIP events around each step kernel; returns the
        summed kernel durations in milliseconds."""
        ms = ctypes.c_double()
        _check(lib().lbm_step_profiled(self._c(), int(nsteps), ctypes.byref(ms)), "step_profiled")
        return float(ms.value)

    def steps_done(self, run: int = 0) -> int:
        v = ctypes.c_int64()
        _check(lib().lbm_steps_done(self._c(), run, ctypes.byref(v)), "steps_done")
        return int(v.value)

    @property
    def launch(self) -> dict:
        l = LbmLaunch()
        _check(lib().lbm_get_launch(self._c(), ctypes.byref(l)), "get_launch")
        return dict(bx=l.bx, by=l.by, bz=l.bz, persistent=l.persistent, grouped=l.grouped)

    def set_launch(self, bx=32, by=8, bz=0, persistent=0, grouped=0):
        l = LbmLaunch(bx, by, bz, persistent, grouped)
        _check(lib().lbm_set_launch(self._c(), ctypes.byref(l)), "set_launch")

    def close(self):
        if self._ctx is not None and self._ctx.value:
            lib().lbm_destroy(self._ctx)
        self._ctx = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Solver(Batch):
    """A single run."""

    def __init__(self, params: dict, precision: str = "fp64", device="cuda:0", stream=None):
        super().__init__([params], precision, device, stream)

    def observe(self, components: bool = False, check: bool = False) -> dict:
        return super().observe(components, check)[0]


class Network:
    """The surrogate network's device state (sg_* calls).  Inputs and targets
    are float32 torch tensors on the context's device."""

    def __init__(self, batch_max: int, device="cuda:0", stream=None):
        import torch
        L = lib()
        self.batch_max = int(batch_max)
        self.n_params = int(L.sg_param_count())
        nbytes = ctypes.c_size_t()
        _check(L.sg_workspace_bytes(self.batch_max, ctypes.byref(nbytes)), "sg workspace")
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        _check(L.sg_init(self.batch_max, ctypes.c_void_p(self.workspace.data_ptr()), nbytes.value,
                         ctypes.c_void_p(_stream_ptr(self.stream)), ctypes.byref(ctx)), "sg init")
        self._ctx = ctx

    def set_params(self, p: np.ndarray):
        v = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().sg_set_params(self._ctx, v.ctypes.data, v.size), "sg set_params")

    def params(self, working: bool = False) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        fn = lib().sg_get_working_params if working else lib().sg_get_params
        _check(fn(self._ctx, out.ctypes.data, out.size), "sg get_params")
        return out

    def forward(self, x):
        import torch
        z = torch.empty((x.shape[0], 3), dtype=torch.float32, device=self.device)
        _check(lib().sg_forward(self._ctx, ctypes.c_void_p(x.data_ptr()), int(x.shape[0]),
                                ctypes.c_void_p(z.data_ptr())), "sg forward")
        return z

    def gradient(self, x, t, m):
        g = np.empty(self.n_params, dtype=np.float32)
        loss = ctypes.c_float()
        _check(lib().sg_gradient(self._ctx, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                 ctypes.c_void_p(m.data_ptr()), int(x.shape[0]), g.ctypes.data,
                                 ctypes.byref(loss)), "sg gradient")
        return g, float(loss.value)

    def gradient_noalloc(self, x, t, m, grad, loss):
        """The same gradient into caller-owned device tensors grad (float32,
        n_params) and loss (float32, 1), with the library's fixed scratch
        array; asynchronous, allocates nothing."""
        _check(lib().sg_gradient_noalloc(self._ctx, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                                         int(x.shape[0]), ctypes.c_void_p(grad.data_ptr()),
                                         ctypes.c_void_p(loss.data_ptr())), "sg gradient_noalloc")

    def train_step(self, x, t, m, lr: float) -> float:
        loss = ctypes.c_float()
        _check(lib().sg_train_step(self._ctx, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                   ctypes.c_void_p(m.data_ptr()), int(x.shape[0]), float(lr),
                                   ctypes.byref(loss)), "sg train_step")
        return float(loss.value)

    def close(self):
        if self._ctx is not None and self._ctx.value:
            lib().sg_destroy(self._ctx)
        self._ctx = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
