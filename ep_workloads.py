"""Seeded synthetic workloads for the per-increment elasto-plastic solve.

This module only builds inputs: model parameters, per-cell cohesion fields and
seeded random states.  It holds none of the method's arithmetic and is the one
module that both the HIP path (through its binding) and the CPU oracle read.

Workloads follow the paper's model configuration (Section "Model
Configuration and Boundary conditions"): pure-shear loading v_x = a x,
v_y = -a y (and v_z = 0 in 3D) with a = 1, nondimensional scales L_x = 1,
G_0 = 1 (Tables of independent scales and dimensionless parameters), friction
angle 30 degrees, dilation 0.  The heterogeneity is a weak inclusion in
cohesion (c = 0.5 c0 inside a circle / sphere), a synthetic stand-in for the
paper's Gaussian cohesion field.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np


@dataclass
class Model:
    """One model: grid, material, loading and solver controls."""

    ndim: int = 2
    nx: int = 63
    ny: int = 63
    nz: int = 1
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    bulk: float = 2.0            # K
    shear: float = 1.0           # G
    visc: float = math.inf       # mu_s (inf = elasto-plastic)
    phi_deg: float = 30.0        # friction angle
    psi_deg: float = 0.0         # dilation angle (0 <= psi <= phi)
    dt: float = 1e-4             # load increment (time; a = 1 so also strain)
    erate: Tuple[float, float, float] = (1.0, -1.0, 0.0)
    tol: float = 1e-8
    max_iter: int = 200000
    n_check: int = 0             # 0 -> default chosen by the solver
    re: float = 0.0              # 0 -> 3 sqrt(10) pi / 2
    r: float = 0.5               # Ktilde / Gtilde
    cfl: float = 0.0             # 0 -> 0.9 / sqrt(ndim)
    freeze_iter: int = 0         # 0: off; else freeze the plastic multiplier after this many iterations
    objective: int = 0           # 1: objective (Jaumann) stress update at the start of every increment
    eta_vp: float = 0.0          # consistency regularisation viscosity of the return (0: perfect plasticity)
    pt_blend: float = 0.25       # weight of the pseudo-time trial in the centre plastic multiplier (path only) ...
    pt_blend_late: float = 0.75  # ... and after the first check at or after 16 max(nx, ny, nz) iterations
    # weak inclusion in cohesion
    c0: float = 1.75e-3
    incl_radius: float = 0.1
    incl_centre: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    incl_factor: float = 0.5
    steps: int = 10
    name: str = ""

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * (self.nz if self.ndim == 3 else 1)

    def with_(self, **kw) -> "Model":
        return replace(self, **kw)


def cohesion_field(m: Model) -> np.ndarray:
    """Per-cell cohesion, x fastest: c0 outside the inclusion, factor*c0 in it.

    A cell is inside when its centre lies strictly within incl_radius of the
    inclusion centre; the domain is centred at the origin.
    """
    dx = m.lx / m.nx
    dy = m.ly / m.ny
    xc = -0.5 * m.lx + (np.arange(m.nx) + 0.5) * dx
    yc = -0.5 * m.ly + (np.arange(m.ny) + 0.5) * dy
    if m.ndim == 2:
        X, Y = np.meshgrid(xc, yc, indexing="xy")          # shape (ny, nx)
        d2 = (X - m.incl_centre[0]) ** 2 + (Y - m.incl_centre[1]) ** 2
    else:
        dz = m.lz / m.nz
        zc = -0.5 * m.lz + (np.arange(m.nz) + 0.5) * dz
        Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")   # shape (nz, ny, nx)
        d2 = ((X - m.incl_centre[0]) ** 2 + (Y - m.incl_centre[1]) ** 2
              + (Z - m.incl_centre[2]) ** 2)
    c = np.full(d2.shape, m.c0, dtype=np.float64)
    c[d2 < m.incl_radius ** 2] = m.incl_factor * m.c0
    return np.ascontiguousarray(c.ravel())


# --------------------------------------------------------------------------
# The five workloads (small 2D case, 2D production, 3D production, batched 2D,
# large 3D).  Sizes and physical values follow the workload definitions; where
# a value is not given (3D cohesion, 3D increment for the large case) the 3D
# production values are reused.
# --------------------------------------------------------------------------

def e2_symmetry(increments: int, nx: int = 383, ny: int = 191, total_strain: float = 2e-3,
                tol: float = 1e-11) -> Model:
    """The symmetry study (section "Symmetry versus non-symmetry"): 2D pure
    shear of a 2:1 domain with uniform cohesion 2e-3, G = 1, the elastic limit
    (Deborah number 1e6: mu_s = 1e6), no objective update; the only
    perturbation is a central pressure anomaly p = c0/2 (pressure_anomaly).  The same
    total strain is applied in `increments` equal increments (7 and 180 in the
    paper).  The total strain and the anomaly radius are not given; 2e-3 takes
    the model through the first yield (about 8e-4) and the stress drop."""
    return Model(ndim=2, nx=nx, ny=ny, lx=2.0, ly=1.0, visc=1e6, c0=2e-3, incl_factor=1.0,
                 dt=total_strain / increments, tol=tol, n_check=100, steps=increments,
                 name=f"e2-{nx}x{ny}-{increments}")


def gaussian_cohesion(m: Model, rise: float = 0.2, width: float = 0.2, wall: float = 0.05,
                      wall_factor: float = 2.0, centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Per-cell cohesion of the heterogeneous setups (section on the initial
    conditions and heterogeneities), x fastest: c0 at the centre of the model,
    rising as a Gaussian towards the walls,
        c = c0 (1 + rise (1 - exp(-r^2 / (width L)^2))),
    with a jump to wall_factor c0 in the cells whose centre lies within
    wall L of a wall (L the smallest extent).  The paper gives the end values
    (2e-3 at the centre, 4e-3 at the walls) but not the width, the rise of the
    Gaussian part or the jump's distance; these defaults are readings.  An
    off-centre `centre` moves the Gaussian (not the wall band) and breaks the
    mirror symmetry of the setup."""
    L = min(m.lx, m.ly, m.lz if m.ndim == 3 else m.ly)
    axes = [-0.5 * e + (np.arange(n) + 0.5) * (e / n) for e, n in ((m.lx, m.nx), (m.ly, m.ny), (m.lz, m.nz))]
    if m.ndim == 2:
        Y, X = np.meshgrid(axes[1], axes[0], indexing="ij")
        r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2
        dwall = np.minimum(0.5 * m.lx - np.abs(X), 0.5 * m.ly - np.abs(Y))
    else:
        Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2
        dwall = np.minimum(np.minimum(0.5 * m.lx - np.abs(X), 0.5 * m.ly - np.abs(Y)), 0.5 * m.lz - np.abs(Z))
    c = m.c0 * (1.0 + rise * (1.0 - np.exp(-r2 / (width * L) ** 2)))
    c[dwall < wall * L] = wall_factor * m.c0
    return np.ascontiguousarray(c.ravel())


def gaussian_shear(m: Model, low: float = 1.0, high: float = 1.2, width: float = 0.2,
                   centre=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Per-cell shear modulus of the heterogeneous setups (x fastest): `low`
    at the centre rising as a Gaussian to `high` towards the walls,
        G = high - (high - low) exp(-r^2 / (width L)^2);
    the end values are the paper's (1 and 1.2), the width a reading."""
    ext = [(m.lx, m.nx), (m.ly, m.ny)] + ([(m.lz, m.nz)] if m.ndim == 3 else [])
    L = min(e for e, _ in ext)
    ax = [-0.5 * e + (np.arange(n) + 0.5) * (e / n) for e, n in ext]
    grids = np.meshgrid(*ax[::-1], indexing="ij")[::-1]          # x, y(, z), each (.., ny, nx)
    r2 = sum((g - c) ** 2 for g, c in zip(grids, centre))
    return np.ascontiguousarray((high - (high - low) * np.exp(-r2 / (width * L) ** 2)).ravel())


def c1_small_2d() -> Model:
    return Model(ndim=2, nx=63, ny=63, tol=1e-8, steps=10, name="2d-63x63-fp64")


def c2_2d(seed: int = 0, visc: float = math.inf) -> Model:
    rng = np.random.Generator(np.random.PCG64(seed))
    off = rng.uniform(-0.1, 0.1, size=2)
    return Model(ndim=2, nx=1023, ny=1023, tol=1e-6, steps=50, visc=visc, freeze_iter=16 * 1023,
                 incl_centre=(float(off[0]), float(off[1]), 0.0),
                 name=f"2d-1023x1023-seed{seed}" + ("-vp" if math.isfinite(visc) else "-ep"))


def c3_3d(n: int = 255, bulk: float = 2.0) -> Model:
    # more than 10^6 cells: frozen plasticity after 16 nx iterations (the
    # accelerated-PT section applies it to every run of that size)
    return Model(ndim=3, nx=n, ny=n, nz=n, dt=5e-5, tol=1e-6, steps=40, bulk=bulk,
                 freeze_iter=16 * n if n ** 3 > 10 ** 6 else 0, name=f"3d-{n}^3-K{bulk:g}")


def c5_3d() -> Model:
    # more than 10^6 cells: frozen plasticity after 16 nx iterations
    return Model(ndim=3, nx=511, ny=511, nz=511, dt=5e-5, tol=1e-6, steps=100, freeze_iter=16 * 511,
                 name="3d-511^3")


def c4_batch(seed: int = 0, n_models: int = 256,
             sizes=(127, 255, 383, 511)) -> List[Model]:
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(n_models):
        n = int(rng.choice(np.asarray(sizes)))
        phi = float(rng.uniform(20.0, 40.0))
        c0 = float(rng.uniform(1e-3, 3e-3))
        rad = float(rng.uniform(0.05, 0.15))
        lo, hi = -0.5 + rad + 0.05, 0.5 - rad - 0.05
        cx, cy = (float(v) for v in rng.uniform(lo, hi, size=2))
        out.append(Model(ndim=2, nx=n, ny=n, phi_deg=phi, c0=c0, incl_radius=rad,
                         incl_centre=(cx, cy, 0.0), dt=1e-4, tol=1e-6, steps=20, freeze_iter=16 * n,
                         name=f"batch{b}-{n}"))
    return out


# --------------------------------------------------------------------------
# Random states for single-sweep parity (every field filled, walls included).
# --------------------------------------------------------------------------

def field_shapes(m: Model) -> dict:
    """Staggered shapes (x fastest, listed as (nx_, ny_[, nz_]))."""
    nx, ny, nz = m.nx, m.ny, m.nz
    if m.ndim == 2:
        return {
            "vx": (nx + 1, ny), "vy": (nx, ny + 1),
            "p": (nx, ny), "txx": (nx, ny), "tyy": (nx, ny), "txy": (nx + 1, ny + 1),
        }
    return {
        "vx": (nx + 1, ny, nz), "vy": (nx, ny + 1, nz), "vz": (nx, ny, nz + 1),
        "p": (nx, ny, nz), "txx": (nx, ny, nz), "tyy": (nx, ny, nz),
        "txy": (nx + 1, ny + 1, nz), "txz": (nx + 1, ny, nz + 1),
        "tyz": (nx, ny + 1, nz + 1),
    }


def random_state(m: Model, seed: int, amp_v: float = 1e-3, amp_s: float = 1e-3) -> dict:
    """A seeded, smooth-plus-noise state.

    Velocities are the background field plus a perturbation of relative size
    amp_v; stresses (current and previous-increment copies) are random with
    amplitude amp_s.  Values are raw inputs only: walls are not made
    consistent here, the solver's own boundary handling decides that.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {}
    shapes = field_shapes(m)
    for name, shp in shapes.items():
        n = int(np.prod(shp))
        if name.startswith("v"):
            out[name] = rng.standard_normal(n) * amp_v
        else:
            out[name] = rng.standard_normal(n) * amp_s
            out[name + "_old"] = rng.standard_normal(n) * amp_s
    # the deviatoric stress is trace-free: fill tzz consistently in 3D
    if m.ndim == 3:
        out["tzz"] = -(out["txx"] + out["tyy"])
        out["tzz_old"] = -(out["txx_old"] + out["tyy_old"])
    return out


def background_velocity(m: Model) -> dict:
    """v = erate * x at every face, domain centred at the origin."""
    nx, ny, nz = m.nx, m.ny, m.nz
    dx, dy = m.lx / nx, m.ly / ny
    xf = -0.5 * m.lx + np.arange(nx + 1) * dx
    yf = -0.5 * m.ly + np.arange(ny + 1) * dy
    if m.ndim == 2:
        vx = np.tile(m.erate[0] * xf, ny)
        vy = np.repeat(m.erate[1] * yf, nx)
        return {"vx": vx, "vy": vy}
    dz = m.lz / nz
    zf = -0.5 * m.lz + np.arange(nz + 1) * dz
    vx = np.tile(m.erate[0] * xf, ny * nz)
    vy = np.tile(np.repeat(m.erate[1] * yf, nx), nz)
    vz = np.repeat(m.erate[2] * zf, nx * ny)
    return {"vx": vx, "vy": vy, "vz": vz}


def pressure_anomaly(m: Model, amplitude: float, radius: float) -> np.ndarray:
    """Initial pressure: amplitude inside a centred circle / sphere, else 0.

    Stand-in for the circular pressure anomaly of the symmetry study.
    """
    mm = replace(m, c0=0.0, incl_factor=1.0)
    inside = cohesion_field(replace(mm, c0=1.0, incl_factor=2.0, incl_radius=radius,
                                    incl_centre=(0.0, 0.0, 0.0))) > 1.5
    return np.where(inside, amplitude, 0.0)
