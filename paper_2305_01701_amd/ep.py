"""Python binding of libep.so (ctypes; argument marshalling only).

Functions carry the C names (ep_init, ep_load_step, ep_sweep, ep_residual,
ep_fields, ...).  `Solver` is a thin convenience wrapper: it asks the library
for the workspace size, allocates that many bytes on the GPU with PyTorch,
passes the current torch stream, and converts fields to numpy arrays.  Every
step of the solve runs in the library's HIP kernels; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libep.so")

EP_OK, EP_EINVAL, EP_ENOMEM, EP_EDEVICE, EP_ENOTCONV, EP_EDIVERGED = 0, -1, -2, -3, -4, -5
EP_FP64, EP_FP32_FIELDS = 0, 1
EP_SWEEP_AUTO, EP_SWEEP_FUSED, EP_SWEEP_UNFUSED = 0, 1, 2
EP_GET, EP_SET = 0, 1

FIELDS = [
    "vx", "vy", "vz", "p", "txx", "tyy", "tzz", "txy", "txz", "tyz",
    "p_old", "txx_old", "tyy_old", "tzz_old", "txy_old", "txz_old", "tyz_old",
    "ux", "uy", "uz", "exx", "eyy", "ezz", "exy", "exz", "eyz",
    "eps_p", "cohesion", "lambda_dot", "tau_ii", "yield", "lambda_frozen",
]
FIELD_ID = {n: i for i, n in enumerate(FIELDS)}

# every symbol include/ep.h declares
SYMBOLS = ["ep_abi_version", "ep_workspace_size", "ep_init", "ep_load_step", "ep_sweep",
           "ep_residual", "ep_residual_noalloc", "ep_fields", "ep_field_shape", "ep_destroy", "ep_last_error",
           "ep_enable_timing", "ep_sweep_timing", "ep_step_history", "ep_set_guess", "ep_set_guess_device", "ep_objective_update", "ep_set_strain_rate", "ep_set_shear_modulus",
           "ep_batch_workspace_size", "ep_batch_init", "ep_batch_tune", "ep_batch_tile_shape",
           "ep_batch_load_step", "ep_batch_model", "ep_batch_enable_timing", "ep_batch_timing",
           "ep_batch_destroy", "ep_batch_last_error",
           "ep_net_workspace_size", "ep_net_init", "ep_net_param_count", "ep_net_params", "ep_net_sample",
           "ep_net_record", "ep_net_observe", "ep_net_reset", "ep_net_forward", "ep_net_gradient", "ep_net_train",
           "ep_net_predict", "ep_net_destroy", "ep_net_last_error"]


class ep_params(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
        ("bulk", C.c_double), ("shear", C.c_double), ("visc", C.c_double),
        ("phi_deg", C.c_double), ("psi_deg", C.c_double), ("dt", C.c_double),
        ("erate", C.c_double * 3), ("tol", C.c_double),
        ("max_iter", C.c_int), ("n_check", C.c_int),
        ("re", C.c_double), ("r", C.c_double), ("cfl", C.c_double),
        ("precision", C.c_int), ("sweep", C.c_int), ("fp32_switch", C.c_double),
        ("fp32_stall", C.c_int), ("freeze_iter", C.c_int), ("guess_accept", C.c_double),
        ("objective", C.c_int), ("eta_vp", C.c_double), ("pt_blend", C.c_double),
        ("pt_blend_late", C.c_double),
    ]


class ep_step_stats(C.Structure):
    _fields_ = [
        ("status", C.c_int), ("iters", C.c_int), ("iters_fp32", C.c_int),
        ("r_ref", C.c_double), ("ref", C.c_double), ("resid", C.c_double), ("eps_rel", C.c_double),
        ("sxx_centre", C.c_double), ("sxx_left", C.c_double), ("sxx_right", C.c_double),
        ("n_yield", C.c_longlong), ("max_violation", C.c_double), ("seconds", C.c_double),
        ("fp32_exit", C.c_double), ("frozen_at", C.c_int), ("guess_used", C.c_int),
        ("r_guess", C.c_double), ("cert", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ep_net_config(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("base", C.c_int),
                ("max_samples", C.c_int), ("scale", C.c_float * 4), ("seed", C.c_int)]


class ep_residual_info(C.Structure):
    _fields_ = [("resid", C.c_double), ("momentum", C.c_double), ("physical", C.c_double),
                ("vmax", C.c_double), ("continuity", C.c_double), ("eps_rel", C.c_double)]


_lib = None


def lib():
    """Load libep.so; raises if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2305_01701_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.ep_abi_version.restype = C.c_int
        L.ep_workspace_size.argtypes = [C.POINTER(ep_params), C.POINTER(C.c_size_t)]
        L.ep_init.argtypes = [C.POINTER(ep_params), C.POINTER(C.c_double), C.POINTER(C.c_double), vp, C.c_size_t, vp,
                              C.POINTER(vp)]
        L.ep_load_step.argtypes = [vp, C.POINTER(ep_step_stats)]
        L.ep_sweep.argtypes = [vp, C.c_int, C.POINTER(C.c_double)]
        L.ep_residual.argtypes = [vp, C.POINTER(ep_residual_info)]
        L.ep_residual_noalloc.argtypes = [vp, C.POINTER(ep_residual_info)]
        L.ep_fields.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_size_t]
        L.ep_field_shape.restype = C.c_long
        L.ep_field_shape.argtypes = [vp, C.c_int, C.POINTER(C.c_int)]
        L.ep_destroy.argtypes = [vp]
        L.ep_destroy.restype = None
        L.ep_last_error.restype = C.c_char_p
        L.ep_last_error.argtypes = [vp]
        L.ep_enable_timing.argtypes = [vp, C.c_int]
        L.ep_sweep_timing.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_long)]
        L.ep_step_history.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_int]
        L.ep_set_guess.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ep_set_guess_device.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp]
        L.ep_objective_update.argtypes = [vp]
        L.ep_set_strain_rate.argtypes = [vp, C.POINTER(C.c_double)]
        L.ep_set_shear_modulus.argtypes = [vp, C.POINTER(C.c_double)]
        L.ep_batch_workspace_size.argtypes = [C.c_int, C.POINTER(ep_params), C.POINTER(C.c_size_t)]
        L.ep_batch_init.argtypes = [C.c_int, C.POINTER(ep_params), C.POINTER(C.POINTER(C.c_double)), vp,
                                    C.c_size_t, vp, C.POINTER(vp)]
        L.ep_batch_tune.argtypes = [vp, C.c_int]
        L.ep_batch_tile_shape.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.ep_batch_load_step.argtypes = [vp, C.POINTER(ep_step_stats)]
        L.ep_batch_model.restype = vp
        L.ep_batch_model.argtypes = [vp, C.c_int]
        L.ep_batch_enable_timing.argtypes = [vp, C.c_int]
        L.ep_batch_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_long)]
        L.ep_batch_destroy.argtypes = [vp]
        L.ep_batch_destroy.restype = None
        L.ep_batch_last_error.restype = C.c_char_p
        L.ep_batch_last_error.argtypes = [vp]
        fp, dp, ip = C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.ep_net_workspace_size.argtypes = [C.POINTER(ep_net_config), C.POINTER(C.c_size_t)]
        L.ep_net_init.argtypes = [C.POINTER(ep_net_config), vp, C.c_size_t, vp, C.POINTER(vp)]
        L.ep_net_param_count.restype = C.c_long
        L.ep_net_param_count.argtypes = [vp]
        L.ep_net_params.argtypes = [vp, C.c_int, fp, C.c_size_t]
        L.ep_net_sample.argtypes = [vp, C.c_int, C.c_int, fp, fp]
        L.ep_net_record.argtypes = [vp, vp, C.c_int]
        L.ep_net_observe.argtypes = [vp, vp, C.c_int]
        L.ep_net_reset.argtypes = [vp]
        L.ep_net_forward.argtypes = [vp, C.c_int, fp]
        L.ep_net_gradient.argtypes = [vp, C.c_int, dp, fp]
        L.ep_net_train.argtypes = [vp, ip, C.c_int, C.c_int, C.c_float, fp]
        L.ep_net_predict.argtypes = [vp, vp]
        L.ep_net_destroy.argtypes = [vp]
        L.ep_net_destroy.restype = None
        L.ep_net_last_error.restype = C.c_char_p
        L.ep_net_last_error.argtypes = [vp]
        _lib = L
    return _lib


# ---- thin C-named wrappers ---------------------------------------------------
def ep_abi_version() -> int:
    return lib().ep_abi_version()


def ep_workspace_size(p: ep_params) -> int:
    n = C.c_size_t(0)
    rc = lib().ep_workspace_size(C.byref(p), C.byref(n))
    if rc != EP_OK:
        raise ValueError(f"ep_workspace_size: {rc}")
    return n.value


def ep_init(p: ep_params, cohesion: Optional[np.ndarray], d_workspace: int, ws_bytes: int, stream: int,
            shear: Optional[np.ndarray] = None):
    h = C.c_void_p()
    coh = None if cohesion is None else np.ascontiguousarray(cohesion, dtype=np.float64)
    cp = None if coh is None else coh.ctypes.data_as(C.POINTER(C.c_double))
    sh = None if shear is None else np.ascontiguousarray(shear, dtype=np.float64)
    sp = None if sh is None else sh.ctypes.data_as(C.POINTER(C.c_double))
    rc = lib().ep_init(C.byref(p), cp, sp, C.c_void_p(d_workspace), ws_bytes, C.c_void_p(stream), C.byref(h))
    return rc, h


def ep_load_step(h) -> tuple:
    st = ep_step_stats()
    rc = lib().ep_load_step(h, C.byref(st))
    return rc, st.as_dict()


def ep_sweep(h, n: int) -> tuple:
    r = C.c_double(0)
    rc = lib().ep_sweep(h, n, C.byref(r))
    return rc, r.value


def ep_residual(h) -> tuple:
    r = ep_residual_info()
    rc = lib().ep_residual(h, C.byref(r))
    return rc, {k: getattr(r, k) for k, _ in r._fields_}


def ep_residual_noalloc(h) -> tuple:
    r = ep_residual_info()
    rc = lib().ep_residual_noalloc(h, C.byref(r))
    return rc, {k: getattr(r, k) for k, _ in r._fields_}


def ep_field_shape(h, field: int) -> tuple:
    shp = (C.c_int * 3)()
    n = lib().ep_field_shape(h, field, shp)
    return n, tuple(shp)


def ep_fields(h, field: int, direction: int, host: np.ndarray) -> int:
    assert host.dtype == np.float64 and host.flags.c_contiguous
    return lib().ep_fields(h, field, direction, host.ctypes.data_as(C.POINTER(C.c_double)), host.size)


def ep_destroy(h) -> None:
    lib().ep_destroy(h)


def ep_last_error(h) -> str:
    return lib().ep_last_error(h).decode()


def _params_array(params):
    arr = (ep_params * len(params))()
    for i, p in enumerate(params):
        arr[i] = p
    return arr


def ep_batch_workspace_size(params) -> int:
    n = C.c_size_t(0)
    rc = lib().ep_batch_workspace_size(len(params), _params_array(params), C.byref(n))
    if rc != EP_OK:
        raise ValueError(f"ep_batch_workspace_size: {rc}")
    return n.value


def ep_batch_init(params, cohesions, d_workspace: int, ws_bytes: int, stream: int):
    n = len(params)
    keep = [None if c is None else np.ascontiguousarray(c, dtype=np.float64) for c in cohesions]
    ptrs = (C.POINTER(C.c_double) * n)()
    for i, c in enumerate(keep):
        ptrs[i] = C.POINTER(C.c_double)() if c is None else c.ctypes.data_as(C.POINTER(C.c_double))
    b = C.c_void_p()
    rc = lib().ep_batch_init(n, _params_array(params), ptrs, C.c_void_p(d_workspace), ws_bytes,
                             C.c_void_p(stream), C.byref(b))
    return rc, b


def ep_batch_load_step(b, n: int) -> tuple:
    st = (ep_step_stats * n)()
    rc = lib().ep_batch_load_step(b, st)
    return rc, [s.as_dict() for s in st]


def ep_batch_tune(b, reps: int) -> int:
    return lib().ep_batch_tune(b, reps)


def ep_batch_tile_shape(b, i: int) -> tuple:
    tx, ty = C.c_int(0), C.c_int(0)
    rc = lib().ep_batch_tile_shape(b, i, C.byref(tx), C.byref(ty))
    return rc, (tx.value, ty.value)


def ep_batch_model(b, i: int):
    return C.c_void_p(lib().ep_batch_model(b, i))


def ep_batch_destroy(b) -> None:
    lib().ep_batch_destroy(b)


def ep_batch_last_error(b) -> str:
    return lib().ep_batch_last_error(b).decode()


# ---- convenience -----------------------------------------------------------
def ep_step_history(h, cap: int = 1 << 20) -> tuple:
    r = np.zeros(cap, dtype=np.float64)
    pr = np.zeros(cap, dtype=np.int32)
    n = lib().ep_step_history(h, r.ctypes.data_as(C.POINTER(C.c_double)),
                              pr.ctypes.data_as(C.POINTER(C.c_int)), cap)
    n = min(n, cap)
    return r[:n].copy(), pr[:n].copy()


def params_from_model(m, precision: int = EP_FP64, sweep: int = EP_SWEEP_AUTO,
                      fp32_switch: float = 0.0, fp32_stall: int = 0, guess_accept: float = 0.0) -> ep_params:
    p = ep_params()
    p.ndim, p.nx, p.ny = m.ndim, m.nx, m.ny
    p.nz = m.nz if m.ndim == 3 else 1
    p.lx, p.ly, p.lz = m.lx, m.ly, m.lz
    p.bulk, p.shear, p.visc = m.bulk, m.shear, m.visc
    p.phi_deg, p.psi_deg, p.dt = m.phi_deg, m.psi_deg, m.dt
    for q in range(3):
        p.erate[q] = m.erate[q]
    p.tol, p.max_iter, p.n_check = m.tol, m.max_iter, m.n_check
    p.re, p.r, p.cfl = m.re, m.r, m.cfl
    p.precision, p.sweep, p.fp32_switch, p.fp32_stall = precision, sweep, fp32_switch, fp32_stall
    p.freeze_iter = m.freeze_iter
    p.guess_accept = guess_accept
    p.objective = getattr(m, "objective", 0)
    p.eta_vp = getattr(m, "eta_vp", 0.0)
    p.pt_blend = getattr(m, "pt_blend", 0.25)
    p.pt_blend_late = getattr(m, "pt_blend_late", 0.75)
    return p


class EpError(RuntimeError):
    pass


class ModelView:
    """Field access and diagnostics of one solver handle."""

    def __init__(self, h):
        self.h = h

    def _check(self, rc, what):
        if rc not in (EP_OK,):
            raise EpError(f"{what} failed with {rc}: {ep_last_error(self.h)}")

    def sweep(self, n: int = 1) -> float:
        rc, r = ep_sweep(self.h, n)
        self._check(rc, "ep_sweep")
        return r

    def history(self) -> tuple:
        """(normalised residual, precision) at each check of the last increment."""
        return ep_step_history(self.h)

    def residual(self) -> dict:
        rc, r = ep_residual(self.h)
        self._check(rc, "ep_residual")
        return r

    def size(self, name: str) -> int:
        return ep_field_shape(self.h, FIELD_ID[name])[0]

    def get(self, name: str) -> np.ndarray:
        n = self.size(name)
        out = np.zeros(max(n, 0), dtype=np.float64)
        if n > 0:
            self._check(ep_fields(self.h, FIELD_ID[name], EP_GET, out), f"get {name}")
        return out

    def set(self, name: str, values) -> None:
        a = np.ascontiguousarray(values, dtype=np.float64).ravel()
        self._check(ep_fields(self.h, FIELD_ID[name], EP_SET, a), f"set {name}")

    def fields(self, names=None) -> Dict[str, np.ndarray]:
        names = names or [n for n in FIELDS if self.size(n) > 0]
        return {n: self.get(n) for n in names}

    def set_guess(self, vx, vy, vz=None) -> None:
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (vx, vy)]
        arrs.append(None if vz is None else np.ascontiguousarray(vz, dtype=np.float64))
        ptr = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))
        self._check(lib().ep_set_guess(self.h, ptr(arrs[0]), ptr(arrs[1]), ptr(arrs[2])), "ep_set_guess")

    GUESS_KIND = {"velocity": 0, "change": 1, "zero": 2}

    def set_guess_device(self, kind: str, vx=None, vy=None, vz=None) -> None:
        """Starting guess from device tensors (float64 or float32, contiguous,
        at the face-velocity shapes); kind "velocity", "change" or "zero"."""
        import torch
        ts = [t for t in (vx, vy, vz) if t is not None]
        dtype = 1 if ts and ts[0].dtype == torch.float32 else 0
        for t in ts:
            if not t.is_contiguous() or t.dtype != ts[0].dtype or t.dtype not in (torch.float32, torch.float64):
                raise ValueError("guess tensors must be contiguous float32 or float64 tensors of one dtype")
        ptr = lambda t: None if t is None else t.data_ptr()
        self._check(lib().ep_set_guess_device(self.h, self.GUESS_KIND[kind], dtype, ptr(vx), ptr(vy), ptr(vz)),
                    "ep_set_guess_device")

    def set_strain_rate(self, erate) -> None:
        """Background strain rate of the next increments (loading schedule)."""
        arr = (C.c_double * 3)(*[float(x) for x in erate])
        self._check(lib().ep_set_strain_rate(self.h, arr), "ep_set_strain_rate")

    def set_shear_modulus(self, shear) -> None:
        """Per-cell shear modulus (x fastest, each in (0, shear])."""
        arr = np.ascontiguousarray(shear, dtype=np.float64).ravel()
        if arr.size != self.model.n_cells:
            raise ValueError("set_shear_modulus: one value per cell expected")
        self._check(lib().ep_set_shear_modulus(self.h, arr.ctypes.data_as(C.POINTER(C.c_double))),
                    "ep_set_shear_modulus")

    def objective_update(self) -> None:
        """Objective (Jaumann) update of the current stresses with the current
        velocities, in place (what load_step applies first when the model's
        objective flag is set)."""
        self._check(lib().ep_objective_update(self.h), "ep_objective_update")


class Solver(ModelView):
    """One model on the GPU (device memory from torch, work on its stream)."""

    def __init__(self, model, cohesion: Optional[np.ndarray] = None, precision: int = EP_FP64,
                 sweep: int = EP_SWEEP_AUTO, fp32_switch: float = 0.0, fp32_stall: int = 0,
                 guess_accept: float = 0.0, device: str = "cuda:0", stream=None,
                 shear: Optional[np.ndarray] = None):
        import torch
        if not torch.cuda.is_available():
            raise EpError("no GPU visible: the solver runs only on the device")
        self.model = model
        self.params = params_from_model(model, precision, sweep, fp32_switch, fp32_stall, guess_accept)
        self.ws_bytes = ep_workspace_size(self.params)
        self.torch = torch
        self.device = torch.device(device)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        base = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if cohesion is None:
            from ep_workloads import cohesion_field
            cohesion = cohesion_field(model)
        with torch.cuda.device(self.device):
            rc, h = ep_init(self.params, cohesion, base, self.ws_bytes, self.stream.cuda_stream, shear)
        if rc != EP_OK:
            raise EpError(f"ep_init failed with {rc}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            ep_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_step(self) -> dict:
        rc, st = ep_load_step(self.h)
        if rc not in (EP_OK, EP_ENOTCONV, EP_EDIVERGED):
            self._check(rc, "ep_load_step")
        return st

    def enable_timing(self, on: bool = True) -> None:
        self._check(lib().ep_enable_timing(self.h, 1 if on else 0), "ep_enable_timing")

    def sweep_timing(self, precision: int) -> tuple:
        ms, n = C.c_double(0), C.c_long(0)
        self._check(lib().ep_sweep_timing(self.h, precision, C.byref(ms), C.byref(n)), "ep_sweep_timing")
        return ms.value, n.value


class Batch:
    """Many independent 2D models solved together (one workspace from torch)."""

    def __init__(self, models, cohesions=None, precision: int = EP_FP32_FIELDS, device: str = "cuda:0",
                 stream=None):
        import torch
        if not torch.cuda.is_available():
            raise EpError("no GPU visible: the solver runs only on the device")
        self.models = list(models)
        self.n = len(self.models)
        self.params = [params_from_model(m, precision) for m in self.models]
        self.ws_bytes = ep_batch_workspace_size(self.params)
        self.device = torch.device(device)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if cohesions is None:
            from ep_workloads import cohesion_field
            cohesions = [cohesion_field(m) for m in self.models]
        with torch.cuda.device(self.device):
            rc, b = ep_batch_init(self.params, cohesions, base, self.ws_bytes, self.stream.cuda_stream)
        if rc != EP_OK:
            raise EpError(f"ep_batch_init failed with {rc}")
        self.b = b

    def close(self):
        if getattr(self, "b", None):
            ep_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != EP_OK:
            raise EpError(f"{what} failed with {rc}: {ep_batch_last_error(self.b)}")

    def tune(self, reps: int = 5) -> list:
        self._check(ep_batch_tune(self.b, reps), "ep_batch_tune")
        return self.tile_shapes()

    def tile_shapes(self) -> list:
        out = []
        for i in range(self.n):
            rc, t = ep_batch_tile_shape(self.b, i)
            self._check(rc, "ep_batch_tile_shape")
            out.append(t)
        return out

    def load_step(self) -> list:
        rc, st = ep_batch_load_step(self.b, self.n)
        if rc not in (EP_OK, EP_ENOTCONV, EP_EDIVERGED):
            self._check(rc, "ep_batch_load_step")
        return st

    def model(self, i: int) -> ModelView:
        if not 0 <= i < self.n:
            raise IndexError(i)
        return ModelView(ep_batch_model(self.b, i))

    def enable_timing(self, on: bool = True) -> None:
        self._check(lib().ep_batch_enable_timing(self.b, 1 if on else 0), "ep_batch_enable_timing")

    def timing(self) -> dict:
        ms, c32, c64, n = C.c_double(0), C.c_double(0), C.c_double(0), C.c_long(0)
        self._check(lib().ep_batch_timing(self.b, C.byref(ms), C.byref(c32), C.byref(c64), C.byref(n)),
                    "ep_batch_timing")
        return {"ms": ms.value, "cell_sweeps32": c32.value, "cell_sweeps64": c64.value, "replays": n.value}


def _fptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_float))


class Net:
    """The warm-start network of one 3D grid (workspace from torch)."""

    def __init__(self, nx, ny, nz, base=32, max_samples=8, scale=(1e-3, 1e-4, 1e-5, 1e-5), seed=0,
                 device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise EpError("no GPU visible: the network runs only on the device")
        c = ep_net_config()
        c.nx, c.ny, c.nz, c.base, c.max_samples, c.seed = nx, ny, nz, base, max_samples, seed
        for q in range(4):
            c.scale[q] = scale[q]
        self.cfg = c
        n = C.c_size_t(0)
        if lib().ep_net_workspace_size(C.byref(c), C.byref(n)) != EP_OK:
            raise ValueError("invalid network configuration")
        self.ws_bytes = n.value
        self.device = torch.device(device)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = lib().ep_net_init(C.byref(c), C.c_void_p(base_ptr), self.ws_bytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != EP_OK:
            raise EpError(f"ep_net_init failed with {rc}")
        self.h = h
        r4 = lambda v: (v + 3) // 4 * 4
        self.dims = (r4(nz), r4(ny), r4(nx))
        self.nvox = int(np.prod(self.dims))

    def close(self):
        if getattr(self, "h", None):
            lib().ep_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != EP_OK:
            raise EpError(f"{what} failed with {rc}: {lib().ep_net_last_error(self.h).decode()}")

    @property
    def param_count(self) -> int:
        return lib().ep_net_param_count(self.h)

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.param_count, dtype=np.float32)
        self._check(lib().ep_net_params(self.h, EP_GET, _fptr(out), out.size), "ep_net_params")
        return out

    def set_params(self, w) -> None:
        a = np.ascontiguousarray(w, dtype=np.float32)
        self._check(lib().ep_net_params(self.h, EP_SET, _fptr(a), a.size), "ep_net_params")

    def set_sample(self, slot, x=None, t=None) -> None:
        xa = None if x is None else np.ascontiguousarray(x, dtype=np.float32)
        ta = None if t is None else np.ascontiguousarray(t, dtype=np.float32)
        self._check(lib().ep_net_sample(self.h, slot, EP_SET, _fptr(xa), _fptr(ta)), "ep_net_sample")

    def get_sample(self, slot):
        x = np.zeros(self.dims + (16,), dtype=np.float32)
        t = np.zeros(self.dims + (4,), dtype=np.float32)
        self._check(lib().ep_net_sample(self.h, slot, EP_GET, _fptr(x), _fptr(t)), "ep_net_sample")
        return x, t

    def record(self, solver, slot) -> None:
        self._check(lib().ep_net_record(self.h, solver.h, slot), "ep_net_record")

    def observe(self, solver, slot=-1) -> None:
        self._check(lib().ep_net_observe(self.h, solver.h, slot), "ep_net_observe")

    def reset(self) -> None:
        self._check(lib().ep_net_reset(self.h), "ep_net_reset")

    def forward(self, slot) -> np.ndarray:
        y = np.zeros(self.dims + (16,), dtype=np.float32)
        self._check(lib().ep_net_forward(self.h, slot, _fptr(y)), "ep_net_forward")
        return y

    def gradient(self, slot):
        loss = C.c_double(0)
        g = np.zeros(self.param_count, dtype=np.float32)
        self._check(lib().ep_net_gradient(self.h, slot, C.byref(loss), _fptr(g)), "ep_net_gradient")
        return loss.value, g

    def train(self, slots, steps, lr=1e-3) -> np.ndarray:
        s = np.ascontiguousarray(slots, dtype=np.int32)
        losses = np.zeros(steps, dtype=np.float32)
        self._check(lib().ep_net_train(self.h, s.ctypes.data_as(C.POINTER(C.c_int)), s.size, steps, lr,
                                       _fptr(losses)), "ep_net_train")
        return losses

    def predict(self, solver) -> None:
        self._check(lib().ep_net_predict(self.h, solver.h), "ep_net_predict")
