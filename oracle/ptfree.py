"""The increment's equations with the pseudo-time terms removed, and a direct
nonlinear solve of them.

TEST INFRASTRUCTURE ONLY: an independent pin for the oracle (oracle/ep_oracle.c
iterates in pseudo-time; this module writes the equations that iteration is
meant to solve and solves them by Newton-type root finding).  It shares no
code with the oracle or with the GPU library.

For one load increment with the previous state p^, tau^ (backward Euler in
physical time; sections on the governing equations, the rheology and the
return mapping), given the face velocities v:

    pressure    p = p^ - K dt div v (+ lambda_dot C K dt, dilatancy)
    trial       S = tau^ / (G dt) + 2 e'(v),  Dp = 1/(G dt) + 1/mu_s
    centres     J2 of S with each shear component averaged from its four
                shear points (2D vertices, 3D edges); Lambda from the radial
                return of S against Y = max(0, A p + B c) (+ eta_vp lambda_dot),
                sqrt(J2) = (Dp + Lambda) tauII;  tau = S / (Dp + Lambda)
    shear pts   Lambda averaged from the four adjacent centres,
                tau = S / (Dp_point + Lambda), zero on the walls (free slip)
    momentum    R = div(tau) - grad p at every interior face

A per-cell G gives each centre its own 1/(G dt); a shear point takes the
mean of its four cells.  Walls keep the background normal velocity.  Arrays
use the natural (z, y, x) shapes of numpy; fields passed in or out are flat,
x fastest (the oracle's layout).
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np


def _dp(ndim: int, deg: float):
    s, c = math.sin(math.radians(deg)), math.cos(math.radians(deg))
    if ndim == 2:
        return s, c
    d = math.sqrt(3.0) * (3.0 - s)
    return 6.0 * s / d, 6.0 * c / d


def _plastic(sq, Dp, p_tr, c, A, B, C, k, vp):
    """Plastic rate of yielding centres (arrays): lambda_dot solves
    Dp (max(0, A p + B c) + vp lambda_dot) + lambda_dot = sq, p = p_tr + lambda_dot C k."""
    ld = (sq - Dp * (A * p_tr + B * c)) / (1.0 + Dp * A * C * k + Dp * vp)
    apex = A * (p_tr + ld * C * k) + B * c < 0.0
    ld = np.where(apex, sq / (1.0 + Dp * vp), ld)
    p = p_tr + ld * C * k
    tii = np.maximum(0.0, A * p + B * c) + vp * ld
    with np.errstate(divide="ignore"):
        lam = np.where(tii > 0.0, ld / np.where(tii > 0.0, tii, 1.0), np.inf)
    return lam, p


class Increment:
    """The equations of one increment of a model (see the module docstring).

    model: an ep_workloads.Model; state: dict with the flat previous-state
    arrays 'p_old', 'txx_old', 'tyy_old', ('tzz_old' in 3D), 'txy_old' (3D:
    'txz_old', 'tyz_old'), 'cohesion', optional 'shear' (per-cell G)."""

    def __init__(self, model, state: Dict[str, np.ndarray]):
        m = model
        self.m = m
        self.nd = m.ndim
        nx, ny = m.nx, m.ny
        nz = m.nz if m.ndim == 3 else 1
        self.n = (nx, ny, nz)
        self.h = (m.lx / nx, m.ly / ny, m.lz / nz if m.ndim == 3 else 1.0)
        self.A, self.B = _dp(m.ndim, m.phi_deg)
        self.C = _dp(m.ndim, m.psi_deg)[0]
        self.vp = m.eta_vp
        self.kdt = m.bulk * m.dt
        imu = 0.0 if math.isinf(m.visc) else 1.0 / m.visc
        G = state.get("shear")
        G = np.full(nx * ny * nz, m.shear) if G is None else np.asarray(G, dtype=np.float64)
        self.igd = self._cells(1.0 / (G * m.dt))
        self.imu = imu
        self.c = self._cells(state["cohesion"])
        self.p_old = self._cells(state["p_old"])
        if self.nd == 2:
            self.old = {k: self._cells(state[k + "_old"]) for k in ("txx", "tyy")}
            self.old["txy"] = np.asarray(state["txy_old"], dtype=np.float64).reshape(ny + 1, nx + 1)
        else:
            self.old = {k: self._cells(state[k + "_old"]) for k in ("txx", "tyy", "tzz")}
            self.old["txy"] = np.asarray(state["txy_old"], dtype=np.float64).reshape(nz, ny + 1, nx + 1)
            self.old["txz"] = np.asarray(state["txz_old"], dtype=np.float64).reshape(nz + 1, ny, nx + 1)
            self.old["tyz"] = np.asarray(state["tyz_old"], dtype=np.float64).reshape(nz + 1, ny + 1, nx)
        self.er = m.erate

    def _cells(self, a):
        nx, ny, nz = self.n
        a = np.asarray(a, dtype=np.float64)
        return a.reshape(ny, nx) if self.nd == 2 else a.reshape(nz, ny, nx)

    # ------------------------------------------------------------ velocities
    def shapes(self):
        nx, ny, nz = self.n
        if self.nd == 2:
            return {"vx": (ny, nx + 1), "vy": (ny + 1, nx)}
        return {"vx": (nz, ny, nx + 1), "vy": (nz, ny + 1, nx), "vz": (nz + 1, ny, nx)}

    def with_walls(self, v: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
        """Velocity arrays (natural shapes) with the wall normal velocities set."""
        m = self.m
        out = {k: np.array(a, dtype=np.float64).reshape(self.shapes()[k]) for k, a in v.items()}
        out["vx"][..., 0] = -self.er[0] * 0.5 * m.lx
        out["vx"][..., -1] = self.er[0] * 0.5 * m.lx
        if self.nd == 2:
            out["vy"][0, :] = -self.er[1] * 0.5 * m.ly
            out["vy"][-1, :] = self.er[1] * 0.5 * m.ly
        else:
            out["vy"][:, 0, :] = -self.er[1] * 0.5 * m.ly
            out["vy"][:, -1, :] = self.er[1] * 0.5 * m.ly
            out["vz"][0] = -self.er[2] * 0.5 * m.lz
            out["vz"][-1] = self.er[2] * 0.5 * m.lz
        return out

    def interior_mask(self):
        """Boolean masks (natural shapes) of the unknown (interior) faces."""
        out = {}
        for k, shp in self.shapes().items():
            msk = np.ones(shp, dtype=bool)
            ax = {"vx": -1, "vy": -2, "vz": -3}[k]
            sl = [slice(None)] * len(shp)
            sl[ax] = 0
            msk[tuple(sl)] = False
            sl[ax] = -1
            msk[tuple(sl)] = False
            out[k] = msk
        return out

    # --------------------------------------------------------------- stresses
    def stresses(self, v):
        """Pressure and deviatoric stresses of the velocities v (natural
        shapes, walls set); also the centre Lambda."""
        return self._stress2(v) if self.nd == 2 else self._stress3(v)

    def _centre(self, nS2, sh2, p_tr):
        Dp = self.igd + self.imu
        Y = np.maximum(0.0, self.A * p_tr + self.B * self.c)
        sq = np.sqrt(nS2 + sh2)
        yl = sq / Dp > Y
        lam = np.zeros_like(sq)
        p = p_tr.copy()
        if yl.any():
            lp, pp = _plastic(sq[yl], Dp[yl], p_tr[yl], self.c[yl], self.A, self.B, self.C, self.kdt, self.vp)
            lam[yl] = lp
            p[yl] = pp
        return lam, p, Dp

    def _stress2(self, v):
        (dx, dy, _), (nx, ny, _) = self.h, self.n
        vx, vy = v["vx"], v["vy"]
        exx = (vx[:, 1:] - vx[:, :-1]) / dx
        eyy = (vy[1:, :] - vy[:-1, :]) / dy
        div = exx + eyy
        p_tr = self.p_old - self.kdt * div
        Sxx = self.old["txx"] * self.igd + 2.0 * (exx - div / 3.0)
        Syy = self.old["tyy"] * self.igd + 2.0 * (eyy - div / 3.0)
        # vertices (ny+1, nx+1): interior ones only
        igv = np.zeros((ny + 1, nx + 1))
        igv[1:-1, 1:-1] = 0.25 * (self.igd[:-1, :-1] + self.igd[:-1, 1:] + self.igd[1:, :-1] + self.igd[1:, 1:])
        Sxy = np.zeros((ny + 1, nx + 1))
        exy = 0.5 * ((vx[1:, 1:-1] - vx[:-1, 1:-1]) / dy + (vy[1:-1, 1:] - vy[1:-1, :-1]) / dx)
        Sxy[1:-1, 1:-1] = self.old["txy"][1:-1, 1:-1] * igv[1:-1, 1:-1] + 2.0 * exy
        Sb = 0.25 * (Sxy[:-1, :-1] + Sxy[:-1, 1:] + Sxy[1:, :-1] + Sxy[1:, 1:])
        lam, p, Dp = self._centre(0.5 * (Sxx ** 2 + Syy ** 2), Sb ** 2, p_tr)
        txx, tyy = Sxx / (Dp + lam), Syy / (Dp + lam)
        txy = np.zeros_like(Sxy)
        lv = 0.25 * (lam[:-1, :-1] + lam[:-1, 1:] + lam[1:, :-1] + lam[1:, 1:])
        txy[1:-1, 1:-1] = Sxy[1:-1, 1:-1] / (igv[1:-1, 1:-1] + self.imu + lv)
        return {"p": p, "txx": txx, "tyy": tyy, "txy": txy, "lam": lam}

    def _stress3(self, v):
        (dx, dy, dz), (nx, ny, nz) = self.h, self.n
        vx, vy, vz = v["vx"], v["vy"], v["vz"]
        exx = (vx[:, :, 1:] - vx[:, :, :-1]) / dx
        eyy = (vy[:, 1:, :] - vy[:, :-1, :]) / dy
        ezz = (vz[1:] - vz[:-1]) / dz
        div = exx + eyy + ezz
        p_tr = self.p_old - self.kdt * div
        S = {a: self.old["t" + a] * self.igd + 2.0 * (e - div / 3.0)
             for a, e in (("xx", exx), ("yy", eyy), ("zz", ezz))}
        g = self.igd
        # xy edges (nz, ny+1, nx+1): interior in x and y
        ig_xy = np.zeros((nz, ny + 1, nx + 1))
        ig_xy[:, 1:-1, 1:-1] = 0.25 * (g[:, :-1, :-1] + g[:, :-1, 1:] + g[:, 1:, :-1] + g[:, 1:, 1:])
        Sxy = np.zeros((nz, ny + 1, nx + 1))
        Sxy[:, 1:-1, 1:-1] = self.old["txy"][:, 1:-1, 1:-1] * ig_xy[:, 1:-1, 1:-1] + (
            (vx[:, 1:, 1:-1] - vx[:, :-1, 1:-1]) / dy + (vy[:, 1:-1, 1:] - vy[:, 1:-1, :-1]) / dx)
        # xz edges (nz+1, ny, nx+1): interior in x and z
        ig_xz = np.zeros((nz + 1, ny, nx + 1))
        ig_xz[1:-1, :, 1:-1] = 0.25 * (g[:-1, :, :-1] + g[:-1, :, 1:] + g[1:, :, :-1] + g[1:, :, 1:])
        Sxz = np.zeros((nz + 1, ny, nx + 1))
        Sxz[1:-1, :, 1:-1] = self.old["txz"][1:-1, :, 1:-1] * ig_xz[1:-1, :, 1:-1] + (
            (vx[1:, :, 1:-1] - vx[:-1, :, 1:-1]) / dz + (vz[1:-1, :, 1:] - vz[1:-1, :, :-1]) / dx)
        # yz edges (nz+1, ny+1, nx): interior in y and z
        ig_yz = np.zeros((nz + 1, ny + 1, nx))
        ig_yz[1:-1, 1:-1, :] = 0.25 * (g[:-1, :-1, :] + g[:-1, 1:, :] + g[1:, :-1, :] + g[1:, 1:, :])
        Syz = np.zeros((nz + 1, ny + 1, nx))
        Syz[1:-1, 1:-1, :] = self.old["tyz"][1:-1, 1:-1, :] * ig_yz[1:-1, 1:-1, :] + (
            (vy[1:, 1:-1, :] - vy[:-1, 1:-1, :]) / dz + (vz[1:-1, 1:, :] - vz[1:-1, :-1, :]) / dy)
        bxy = 0.25 * (Sxy[:, :-1, :-1] + Sxy[:, :-1, 1:] + Sxy[:, 1:, :-1] + Sxy[:, 1:, 1:])
        bxz = 0.25 * (Sxz[:-1, :, :-1] + Sxz[:-1, :, 1:] + Sxz[1:, :, :-1] + Sxz[1:, :, 1:])
        byz = 0.25 * (Syz[:-1, :-1, :] + Syz[:-1, 1:, :] + Syz[1:, :-1, :] + Syz[1:, 1:, :])
        nS2 = 0.5 * (S["xx"] ** 2 + S["yy"] ** 2 + S["zz"] ** 2)
        lam, p, Dp = self._centre(nS2, bxy ** 2 + bxz ** 2 + byz ** 2, p_tr)
        out = {"p": p, "lam": lam}
        for a in ("xx", "yy", "zz"):
            out["t" + a] = S[a] / (Dp + lam)
        L = lam
        txy = np.zeros_like(Sxy)
        lv = 0.25 * (L[:, :-1, :-1] + L[:, :-1, 1:] + L[:, 1:, :-1] + L[:, 1:, 1:])
        txy[:, 1:-1, 1:-1] = Sxy[:, 1:-1, 1:-1] / (ig_xy[:, 1:-1, 1:-1] + self.imu + lv)
        txz = np.zeros_like(Sxz)
        lv = 0.25 * (L[:-1, :, :-1] + L[:-1, :, 1:] + L[1:, :, :-1] + L[1:, :, 1:])
        txz[1:-1, :, 1:-1] = Sxz[1:-1, :, 1:-1] / (ig_xz[1:-1, :, 1:-1] + self.imu + lv)
        tyz = np.zeros_like(Syz)
        lv = 0.25 * (L[:-1, :-1, :] + L[:-1, 1:, :] + L[1:, :-1, :] + L[1:, 1:, :])
        tyz[1:-1, 1:-1, :] = Syz[1:-1, 1:-1, :] / (ig_yz[1:-1, 1:-1, :] + self.imu + lv)
        out.update(txy=txy, txz=txz, tyz=tyz)
        return out

    # --------------------------------------------------------------- residual
    def residual(self, v):
        """Momentum residual at the interior faces (dict of natural-shape
        arrays over the interior faces)."""
        s = self.stresses(v)
        dx, dy, dz = self.h
        if self.nd == 2:
            sxx, syy, txy = s["txx"] - s["p"], s["tyy"] - s["p"], s["txy"]
            rx = (sxx[:, 1:] - sxx[:, :-1]) / dx + (txy[1:, 1:-1] - txy[:-1, 1:-1]) / dy
            ry = (syy[1:, :] - syy[:-1, :]) / dy + (txy[1:-1, 1:] - txy[1:-1, :-1]) / dx
            return {"vx": rx, "vy": ry}
        sxx, syy, szz = s["txx"] - s["p"], s["tyy"] - s["p"], s["tzz"] - s["p"]
        txy, txz, tyz = s["txy"], s["txz"], s["tyz"]
        rx = ((sxx[:, :, 1:] - sxx[:, :, :-1]) / dx + (txy[:, 1:, 1:-1] - txy[:, :-1, 1:-1]) / dy
              + (txz[1:, :, 1:-1] - txz[:-1, :, 1:-1]) / dz)
        ry = ((txy[:, 1:-1, 1:] - txy[:, 1:-1, :-1]) / dx + (syy[:, 1:, :] - syy[:, :-1, :]) / dy
              + (tyz[1:, 1:-1, :] - tyz[:-1, 1:-1, :]) / dz)
        rz = ((txz[1:-1, :, 1:] - txz[1:-1, :, :-1]) / dx + (tyz[1:-1, 1:, :] - tyz[1:-1, :-1, :]) / dy
              + (szz[1:] - szz[:-1]) / dz)
        return {"vx": rx, "vy": ry, "vz": rz}

    def residual_max(self, v) -> float:
        return max(float(np.abs(r).max()) for r in self.residual(v).values())

    # ----------------------------------------------------------- direct solve
    def solve(self, v0, xtol: float = 1e-14):
        """Root of the momentum residual over the interior face velocities,
        by scipy's MINPACK hybrid method (finite-difference Jacobian), from
        the velocities v0 (flat, x fastest, the oracle's layout).  Returns the
        velocities (flat) and the scipy result."""
        from scipy.optimize import root

        shp = self.shapes()
        base = self.with_walls({k: np.asarray(v0[k], dtype=np.float64).reshape(shp[k]) for k in shp})
        msk = self.interior_mask()
        keys = list(shp)
        x0 = np.concatenate([base[k][msk[k]] for k in keys])
        scale = max(abs(e) for e in self.er) * max(self.m.lx, self.m.ly)

        def unpack(x):
            v = {k: base[k].copy() for k in keys}
            o = 0
            for k in keys:
                n = int(msk[k].sum())
                v[k][msk[k]] = x[o:o + n] * scale
                o += n
            return v

        def fun(x):
            r = self.residual(unpack(x))
            return np.concatenate([r[k].ravel() for k in keys])

        res = root(fun, x0 / scale, method="hybr", options={"xtol": xtol, "maxfev": 200000})
        v = unpack(res.x)
        return {k: v[k].ravel() for k in keys}, res


def previous_state(o) -> Dict[str, np.ndarray]:
    """The increment-start arrays held by an oracle object after a load step
    (its p^, tau^, cohesion)."""
    names = ["p_old", "txx_old", "tyy_old", "txy_old", "cohesion"]
    if o.model.ndim == 3:
        names += ["tzz_old", "txz_old", "tyz_old"]
    return {k: o.get(k) for k in names}
