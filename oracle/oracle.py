"""ctypes wrapper around the C oracle (oracle/liborc.so).

Test infrastructure only.  Field names match ep_workloads.field_shapes plus
the accumulators ("ux", "exx", "eps_p", ...); arrays are FP64, x fastest, at
each field's own staggered shape.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

FIELDS = [
    "vx", "vy", "vz", "p", "txx", "tyy", "tzz", "txy", "txz", "tyz",
    "p_old", "txx_old", "tyy_old", "tzz_old", "txy_old", "txz_old", "tyz_old",
    "ux", "uy", "uz", "exx", "eyy", "ezz", "exy", "exz", "eyz",
    "eps_p", "cohesion", "lambda_dot", "tau_ii", "yield", "lambda_frozen",
]
FIELD_ID = {n: i for i, n in enumerate(FIELDS)}


class OrcParams(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
        ("bulk", C.c_double), ("shear", C.c_double), ("visc", C.c_double),
        ("phi_deg", C.c_double), ("psi_deg", C.c_double), ("dt", C.c_double),
        ("erate", C.c_double * 3), ("tol", C.c_double),
        ("max_iter", C.c_int), ("n_check", C.c_int),
        ("re", C.c_double), ("r", C.c_double), ("cfl", C.c_double),
        ("freeze_iter", C.c_int), ("objective", C.c_int), ("eta_vp", C.c_double),
        ("pt_blend", C.c_double), ("pt_blend_late", C.c_double), ("progress", C.c_int),
    ]


class OrcStats(C.Structure):
    _fields_ = [
        ("status", C.c_int), ("iters", C.c_int),
        ("r_ref", C.c_double), ("ref", C.c_double), ("resid", C.c_double), ("cert", C.c_double),
        ("eps_rel", C.c_double), ("sxx_centre", C.c_double), ("sxx_left", C.c_double),
        ("sxx_right", C.c_double), ("n_yield", C.c_longlong), ("max_violation", C.c_double),
        ("frozen_at", C.c_int),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcParams), C.POINTER(C.c_double)]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_field_size.restype = C.c_long
        L.orc_field_size.argtypes = [C.c_void_p, C.c_int]
        L.orc_get.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double)]
        L.orc_set.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_double)]
        L.orc_sweep.restype = C.c_double
        L.orc_sweep.argtypes = [C.c_void_p, C.c_int]
        L.orc_load_step.argtypes = [C.c_void_p, C.POINTER(OrcStats)]
        L.orc_scalars.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        L.orc_history.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_int]
        L.orc_history_len.argtypes = [C.c_void_p]
        L.orc_objective_update.argtypes = [C.c_void_p]
        L.orc_set_strain_rate.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        L.orc_set_shear_modulus.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
        L.orc_set_shear_modulus.restype = C.c_int
        L.orc_threads.restype = C.c_int
        _lib = L
    return _lib


def params_from_model(m, progress: int = 0) -> OrcParams:
    p = OrcParams()
    p.ndim, p.nx, p.ny = m.ndim, m.nx, m.ny
    p.nz = m.nz if m.ndim == 3 else 1
    p.lx, p.ly, p.lz = m.lx, m.ly, m.lz
    p.bulk, p.shear, p.visc = m.bulk, m.shear, m.visc
    p.phi_deg, p.psi_deg, p.dt = m.phi_deg, m.psi_deg, m.dt
    for q in range(3):
        p.erate[q] = m.erate[q]
    p.tol, p.max_iter, p.n_check = m.tol, m.max_iter, m.n_check
    p.re, p.r, p.cfl = m.re, m.r, m.cfl
    p.freeze_iter = m.freeze_iter
    p.objective = m.objective
    p.eta_vp = m.eta_vp
    p.pt_blend = m.pt_blend
    p.pt_blend_late = m.pt_blend_late
    p.progress = progress
    return p


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """One model held by the C oracle."""

    def __init__(self, model, cohesion: Optional[np.ndarray] = None, progress: int = 0):
        self.model = model
        self._p = params_from_model(model, progress)
        if cohesion is None:
            from ep_workloads import cohesion_field
            cohesion = cohesion_field(model)
        self._coh = np.ascontiguousarray(cohesion, dtype=np.float64)
        h = lib().orc_create(C.byref(self._p), _dptr(self._coh))
        if not h:
            raise ValueError("oracle rejected the parameters")
        self._h = h
        self._hist = None

    def close(self):
        if self._h:
            lib().orc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self, name: str) -> np.ndarray:
        fid = FIELD_ID[name]
        n = lib().orc_field_size(self._h, fid)
        out = np.zeros(max(n, 0), dtype=np.float64)
        if n > 0:
            lib().orc_get(self._h, fid, _dptr(out))
        return out

    def set(self, name: str, values: np.ndarray) -> None:
        fid = FIELD_ID[name]
        n = lib().orc_field_size(self._h, fid)
        a = np.ascontiguousarray(values, dtype=np.float64).ravel()
        if a.size != n:
            raise ValueError(f"{name}: expected {n} values, got {a.size}")
        lib().orc_set(self._h, fid, _dptr(a))

    def fields(self, names=None) -> Dict[str, np.ndarray]:
        names = names or [n for n in FIELDS if lib().orc_field_size(self._h, FIELD_ID[n]) > 0]
        return {n: self.get(n) for n in names}

    def set_strain_rate(self, erate) -> None:
        """Background strain rate of the next increments."""
        lib().orc_set_strain_rate(self._h, (C.c_double * 3)(*[float(x) for x in erate]))

    def set_shear_modulus(self, G) -> None:
        """Per-cell shear modulus (x fastest, every value in (0, shear])."""
        a = np.ascontiguousarray(G, dtype=np.float64).ravel()
        if a.size != self.model.n_cells:
            raise ValueError("set_shear_modulus: one value per cell expected")
        if lib().orc_set_shear_modulus(self._h, _dptr(a)) != 0:
            raise ValueError("set_shear_modulus: 0 < G <= shear")

    def objective_update(self) -> None:
        """Objective (Jaumann) update of the current stresses with the current
        velocities over one increment (what load_step applies first when the
        model's objective flag is set)."""
        lib().orc_objective_update(self._h)

    def sweep(self, physical: bool = False) -> float:
        return lib().orc_sweep(self._h, 1 if physical else 0)

    def evaluate(self) -> float:
        """One PT evaluation of the current state without committing it."""
        return lib().orc_sweep(self._h, 2)

    def load_step(self) -> dict:
        st = OrcStats()
        lib().orc_load_step(self._h, C.byref(st))
        return st.as_dict()

    def record_history(self, cap: int = 100000) -> None:
        self._hist = np.zeros(cap, dtype=np.float64)
        lib().orc_history(self._h, _dptr(self._hist), cap)

    def history(self) -> np.ndarray:
        n = lib().orc_history_len(self._h)
        return self._hist[:n].copy() if self._hist is not None else np.zeros(0)

    def scalars(self) -> dict:
        out = (C.c_double * 8)()
        lib().orc_scalars(self._h, out)
        keys = ["gdtau", "kdtau", "dtrho", "eta", "A", "B", "h", "L"]
        return dict(zip(keys, list(out)))

    @staticmethod
    def threads() -> int:
        return lib().orc_threads()


def run(model, steps: Optional[int] = None, cohesion=None) -> tuple:
    """Run `steps` increments; returns (oracle, list of per-step stats)."""
    o = Oracle(model, cohesion)
    stats = []
    for _ in range(model.steps if steps is None else steps):
        st = o.load_step()
        stats.append(st)
        if st["status"] != 0:
            break
    return o, stats
