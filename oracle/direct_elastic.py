"""Direct solve of one elastic load increment on the staggered grid.

TEST INFRASTRUCTURE ONLY: an independent pin for the oracle's discretisation
(stencils, deviatoric projection, boundary conditions).  When no cell yields,
the increment's discrete problem is linear in the face velocities:

    momentum      d_j (tau_ij - p delta_ij) = 0 at interior faces
    pressure      p   = p^ - K dt div v
    deviator      tau = tau^ + 2 G dt (sym grad v - div v / 3 I)   (mu_s = inf)
    walls         normal velocity = background value; shear stress = 0 on
                  wall vertices / edges (free slip)

(summary of the governing equations, backward Euler in physical time with
the pseudo-time terms at their fixed point).  It is assembled here as a
sparse matrix from Kronecker products of 1D difference matrices and solved
with a sparse LU; the PT oracle must reach the same solution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _fwd(n: int, h: float) -> sp.csr_matrix:
    """(n) x (n+1): (u[i+1]-u[i])/h."""
    return sp.diags([-np.ones(n), np.ones(n)], [0, 1], shape=(n, n + 1), format="csr") / h


def _back_interior(n: int, h: float) -> sp.csr_matrix:
    """(n+1) x n: row i = (u[i]-u[i-1])/h for 1<=i<=n-1, zero rows at i=0, n."""
    rows, cols, vals = [], [], []
    for i in range(1, n):
        rows += [i, i]
        cols += [i, i - 1]
        vals += [1.0 / h, -1.0 / h]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, n))


def _op(mats, in_shape):
    """Tensor-product operator on an x-fastest field.

    mats: per-axis matrix or None (identity of that axis's input length)."""
    full = None
    for ax in range(len(in_shape)):       # build kron(A_last, ..., A_0)
        m = mats[ax] if mats[ax] is not None else sp.identity(in_shape[ax], format="csr")
        full = m if full is None else sp.kron(m, full, format="csr")
    return full


def _mask(shape, walls):
    """Diagonal 0/1 matrix zeroing entries whose index hits a wall.

    walls: list of (axis, n) meaning index 0 or n on that axis is a wall."""
    grids = np.meshgrid(*[np.arange(s) for s in reversed(shape)], indexing="ij")
    idx = list(reversed(grids))           # idx[ax] has x-fastest flattening
    keep = np.ones(grids[0].shape, dtype=bool)
    for ax, n in walls:
        keep &= (idx[ax] != 0) & (idx[ax] != n)
    return sp.diags(keep.ravel().astype(np.float64))


def solve(m, old: dict, cohesion=None, lam=None, shear_field=None) -> dict:
    """Solve one elastic increment.

    m: ep_workloads.Model (visc must be inf); old: dict with p_old, txx_old,
    tyy_old, (tzz_old,) txy_old, (txz_old, tyz_old) as flat x-fastest arrays.
    Returns the face velocities and the stresses of the solution.

    lam (2D only): a fixed plastic multiplier Lambda per cell (frozen
    plasticity).  The deviator then satisfies tau (1/(G dt) + Lambda) =
    tau^/(G dt) + 2 (sym grad v - div v / 3 I), with Lambda at a vertex the
    mean of its four cells -- still linear in v.

    shear_field (2D only): a shear modulus per cell; the compliance 1/(G dt) of a vertex
    is the mean of its four cells' compliances."""
    assert np.isinf(m.visc)
    nx, ny = m.nx, m.ny
    dx, dy = m.lx / nx, m.ly / ny
    K, G, dt = m.bulk, m.shear, m.dt
    ex, ey = m.erate[0], m.erate[1]
    if m.ndim == 2:
        sh = {"vx": (nx + 1, ny), "vy": (nx, ny + 1), "c": (nx, ny), "xy": (nx + 1, ny + 1)}
        Dx_vx = _op([_fwd(nx, dx), None], sh["vx"])             # vx -> cells
        Dy_vy = _op([None, _fwd(ny, dy)], sh["vy"])             # vy -> cells
        Gy_vx = _op([None, _back_interior(ny, dy)], sh["vx"])   # vx -> vertices
        Gx_vy = _op([_back_interior(nx, dx), None], sh["vy"])   # vy -> vertices
        mxy = _mask(sh["xy"], [(0, nx), (1, ny)])
        nvx, nvy = nx * 0 + (nx + 1) * ny, nx * (ny + 1)
        Z = lambda r, c: sp.csr_matrix((r, c))
        nc = nx * ny
        # strain-rate operators acting on v = [vx; vy]
        div = sp.hstack([Dx_vx, Dy_vy])
        exx = sp.hstack([Dx_vx, Z(nc, nvy)]) - div / 3.0
        eyy = sp.hstack([Z(nc, nvx), Dy_vy]) - div / 3.0
        exy = mxy @ (0.5 * sp.hstack([Gy_vx, Gx_vy]))
        # stresses = const + L v; compliance factor c = 1 / (1/(G dt) + Lambda)
        if shear_field is None:
            igc = np.full(nc, 1.0 / (m.shear * dt))
        else:
            igc = 1.0 / (np.asarray(shear_field, dtype=np.float64).ravel() * dt)
        I2 = igc.reshape(ny, nx)
        igv = np.full((ny + 1, nx + 1), 1.0 / (m.shear * dt))      # wall vertices carry no stress
        igv[1:ny, 1:nx] = 0.25 * (I2[:-1, :-1] + I2[:-1, 1:] + I2[1:, :-1] + I2[1:, 1:])
        igv = igv.ravel()
        lc = np.zeros(nc) if lam is None else np.asarray(lam, dtype=np.float64)
        L2 = lc.reshape(ny, nx)
        lv = np.zeros((ny + 1, nx + 1))
        lv[1:ny, 1:nx] = 0.25 * (L2[:-1, :-1] + L2[:-1, 1:] + L2[1:, :-1] + L2[1:, 1:])
        cc = sp.diags(1.0 / (igc + lc))
        cv = sp.diags(1.0 / (igv + lv.ravel()))
        P_L, P_0 = -K * dt * div, old["p_old"]
        Txx_L, Txx_0 = cc @ (2 * exx), cc @ (igc * old["txx_old"])
        Tyy_L, Tyy_0 = cc @ (2 * eyy), cc @ (igc * old["tyy_old"])
        Txy_L, Txy_0 = cv @ (2 * exy), cv @ (mxy @ (igv * old["txy_old"]))
        # momentum operators
        Gx_c = _op([_back_interior(nx, dx), None], sh["c"])     # cells -> x-faces
        Dy_xy = _op([None, _fwd(ny, dy)], sh["xy"])             # vertices -> x-faces
        Gy_c = _op([None, _back_interior(ny, dy)], sh["c"])     # cells -> y-faces
        Dx_xy = _op([_fwd(nx, dx), None], sh["xy"])             # vertices -> y-faces
        Mx_L = Gx_c @ (Txx_L - P_L) + Dy_xy @ Txy_L
        Mx_0 = Gx_c @ (Txx_0 - P_0) + Dy_xy @ Txy_0
        My_L = Gy_c @ (Tyy_L - P_L) + Dx_xy @ Txy_L
        My_0 = Gy_c @ (Tyy_0 - P_0) + Dx_xy @ Txy_0
        # rows: interior faces -> momentum; wall faces -> Dirichlet
        ivx = np.arange(nvx)
        wall_x = (ivx % (nx + 1) == 0) | (ivx % (nx + 1) == nx)
        ivy = np.arange(nvy)
        wall_y = (ivy // nx == 0) | (ivy // nx == ny)
        xf = -0.5 * m.lx + (ivx % (nx + 1)) * dx
        yf = -0.5 * m.ly + (ivy // nx) * dy
        A = sp.vstack([Mx_L, My_L]).tolil()
        b = -np.concatenate([Mx_0, My_0])
        wall = np.concatenate([wall_x, wall_y])
        bc = np.concatenate([ex * xf, ey * yf])
        for r in np.nonzero(wall)[0]:
            A.rows[r] = [r]
            A.data[r] = [1.0]
            b[r] = bc[r]
        v = spla.spsolve(A.tocsc(), b)
        return {
            "vx": v[:nvx], "vy": v[nvx:],
            "p": P_0 + P_L @ v, "txx": Txx_0 + Txx_L @ v, "tyy": Tyy_0 + Tyy_L @ v,
            "txy": Txy_0 + Txy_L @ v,
        }

    assert lam is None, "frozen Lambda: 2D only"
    nz = m.nz
    dz = m.lz / nz
    ez = m.erate[2]
    sh = {"vx": (nx + 1, ny, nz), "vy": (nx, ny + 1, nz), "vz": (nx, ny, nz + 1),
          "c": (nx, ny, nz), "xy": (nx + 1, ny + 1, nz), "xz": (nx + 1, ny, nz + 1),
          "yz": (nx, ny + 1, nz + 1)}
    n = {k: int(np.prod(v)) for k, v in sh.items()}
    Z = lambda r, c: sp.csr_matrix((r, c))
    Dx_vx = _op([_fwd(nx, dx), None, None], sh["vx"])
    Dy_vy = _op([None, _fwd(ny, dy), None], sh["vy"])
    Dz_vz = _op([None, None, _fwd(nz, dz)], sh["vz"])
    nc = n["c"]
    div = sp.hstack([Dx_vx, Dy_vy, Dz_vz])
    exx = sp.hstack([Dx_vx, Z(nc, n["vy"]), Z(nc, n["vz"])]) - div / 3.0
    eyy = sp.hstack([Z(nc, n["vx"]), Dy_vy, Z(nc, n["vz"])]) - div / 3.0
    ezz = sp.hstack([Z(nc, n["vx"]), Z(nc, n["vy"]), Dz_vz]) - div / 3.0
    mxy = _mask(sh["xy"], [(0, nx), (1, ny)])
    mxz = _mask(sh["xz"], [(0, nx), (2, nz)])
    myz = _mask(sh["yz"], [(1, ny), (2, nz)])
    exy = mxy @ (0.5 * sp.hstack([_op([None, _back_interior(ny, dy), None], sh["vx"]),
                                  _op([_back_interior(nx, dx), None, None], sh["vy"]),
                                  Z(n["xy"], n["vz"])]))
    exz = mxz @ (0.5 * sp.hstack([_op([None, None, _back_interior(nz, dz)], sh["vx"]),
                                  Z(n["xz"], n["vy"]),
                                  _op([_back_interior(nx, dx), None, None], sh["vz"])]))
    eyz = myz @ (0.5 * sp.hstack([Z(n["yz"], n["vx"]),
                                  _op([None, None, _back_interior(nz, dz)], sh["vy"]),
                                  _op([None, _back_interior(ny, dy), None], sh["vz"])]))
    P_L, P_0 = -K * dt * div, old["p_old"]
    S = {"xx": (2 * G * dt * exx, old["txx_old"]), "yy": (2 * G * dt * eyy, old["tyy_old"]),
         "zz": (2 * G * dt * ezz, old["tzz_old"]),
         "xy": (2 * G * dt * exy, mxy @ old["txy_old"]),
         "xz": (2 * G * dt * exz, mxz @ old["txz_old"]),
         "yz": (2 * G * dt * eyz, myz @ old["tyz_old"])}
    gx_c = _op([_back_interior(nx, dx), None, None], sh["c"])
    gy_c = _op([None, _back_interior(ny, dy), None], sh["c"])
    gz_c = _op([None, None, _back_interior(nz, dz)], sh["c"])
    dy_xy = _op([None, _fwd(ny, dy), None], sh["xy"])
    dx_xy = _op([_fwd(nx, dx), None, None], sh["xy"])
    dz_xz = _op([None, None, _fwd(nz, dz)], sh["xz"])
    dx_xz = _op([_fwd(nx, dx), None, None], sh["xz"])
    dz_yz = _op([None, None, _fwd(nz, dz)], sh["yz"])
    dy_yz = _op([None, _fwd(ny, dy), None], sh["yz"])

    def lin(i):  # i = 0: operator part, 1: constant part
        sxx = S["xx"][i] - (P_L if i == 0 else P_0)
        syy = S["yy"][i] - (P_L if i == 0 else P_0)
        szz = S["zz"][i] - (P_L if i == 0 else P_0)
        mx = gx_c @ sxx + dy_xy @ S["xy"][i] + dz_xz @ S["xz"][i]
        my = dx_xy @ S["xy"][i] + gy_c @ syy + dz_yz @ S["yz"][i]
        mz = dx_xz @ S["xz"][i] + dy_yz @ S["yz"][i] + gz_c @ szz
        return mx, my, mz

    mxL, myL, mzL = lin(0)
    mx0, my0, mz0 = lin(1)
    A = sp.vstack([mxL, myL, mzL]).tolil()
    b = -np.concatenate([mx0, my0, mz0])
    ivx = np.arange(n["vx"]); ix = ivx % (nx + 1)
    ivy = np.arange(n["vy"]); jy = (ivy // nx) % (ny + 1)
    ivz = np.arange(n["vz"]); kz = ivz // (nx * ny)
    wall = np.concatenate([(ix == 0) | (ix == nx), (jy == 0) | (jy == ny), (kz == 0) | (kz == nz)])
    bc = np.concatenate([ex * (-0.5 * m.lx + ix * dx), ey * (-0.5 * m.ly + jy * dy),
                         ez * (-0.5 * m.lz + kz * dz)])
    for r in np.nonzero(wall)[0]:
        A.rows[r] = [r]
        A.data[r] = [1.0]
        b[r] = bc[r]
    v = spla.spsolve(A.tocsc(), b)
    o1, o2 = n["vx"], n["vx"] + n["vy"]
    out = {"vx": v[:o1], "vy": v[o1:o2], "vz": v[o2:], "p": P_0 + P_L @ v}
    for k in ("xx", "yy", "zz", "xy", "xz", "yz"):
        out["t" + k] = S[k][1] + S[k][0] @ v
    return out
