"""Pins of the oracle's objective (Jaumann) stress update (paper: Jaumann rate
of stress, equations j1-j14, and the appendix on the objective stress terms).

Each check is against something other than the oracle's own formulas:
  - a rigid rotation of a homogeneous stress: the stress must co-rotate, so the
    update divided by dt equals the time derivative of Q(t) tau Q(t)^T with
    Q = expm(W t) (central difference of the exact rotation); in 3D about a
    general axis and with all six components set, so every term of every
    component (and its sign) is exercised;
  - uniform translation of linear fields: first-order upwind transport is
    exact for a linear profile (away from the inflow edge);
  - pure shear (no vorticity) and zero velocity leave a homogeneous state
    unchanged; the update keeps the stress deviator trace-free.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from ep_workloads import Model
from oracle.oracle import Oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def coords(m):
    """Face, centre and node coordinates of the centred domain."""
    dx, dy = m.lx / m.nx, m.ly / m.ny
    xn = -m.lx / 2 + dx * np.arange(m.nx + 1)
    yn = -m.ly / 2 + dy * np.arange(m.ny + 1)
    xc, yc = xn[:-1] + dx / 2, yn[:-1] + dy / 2
    if m.ndim == 2:
        return xn, yn, xc, yc
    dz = m.lz / m.nz
    zn = -m.lz / 2 + dz * np.arange(m.nz + 1)
    return xn, yn, zn, xc, yc, xn[:-1] + dx / 2, zn[:-1] + dz / 2


def grid(*axes):
    """Arrays over the given 1D axes, x fastest (index order z, y, x)."""
    g = np.meshgrid(*axes[::-1], indexing="ij")
    return g[::-1]


def set_velocity(o, m, fx, fy, fz=None):
    if m.ndim == 2:
        xn, yn, xc, yc = coords(m)
        X, Y = grid(xn, yc)
        o.set("vx", fx(X, Y, 0 * X))
        X, Y = grid(xc, yn)
        o.set("vy", fy(X, Y, 0 * X))
        return
    xn, yn, zn, xc, yc, _, zc = coords(m)
    X, Y, Z = grid(xn, yc, zc)
    o.set("vx", fx(X, Y, Z))
    X, Y, Z = grid(xc, yn, zc)
    o.set("vy", fy(X, Y, Z))
    X, Y, Z = grid(xc, yc, zn)
    o.set("vz", fz(X, Y, Z))


def rot_rate(W, tau, h=1e-4):
    """d/dt of expm(W t) tau expm(W t)^T at t = 0 (central difference of the
    exact rotation; error O(h^2 |W|^3 |tau|))."""
    qp, qm = expm(W * h), expm(-W * h)
    return (qp @ tau @ qp.T - qm @ tau @ qm.T) / (2 * h)


def test_rigid_rotation_2d_corotates_the_stress():
    m = Model(ndim=2, nx=12, ny=10, dt=1e-3)
    om = 0.7
    o = Oracle(m)
    set_velocity(o, m, lambda x, y, z: -om * y, lambda x, y, z: om * x)
    sxx, syy, sxy = 0.3, -0.1, 0.25
    nc, nv = m.nx * m.ny, (m.nx + 1) * (m.ny + 1)
    o.set("txx", np.full(nc, sxx))
    o.set("tyy", np.full(nc, syy))
    o.set("txy", np.full(nv, sxy))
    o.set("p", np.full(nc, 0.4))
    o.objective_update()
    # spin of v = omega x r: W = [[0, -om], [om, 0]]
    W = np.array([[0.0, -om], [om, 0.0]])
    rate = rot_rate(W, np.array([[sxx, sxy], [sxy, syy]]))
    txx = o.get("txx").reshape(m.ny, m.nx)[1:-1, 1:-1]
    tyy = o.get("tyy").reshape(m.ny, m.nx)[1:-1, 1:-1]
    txy = o.get("txy").reshape(m.ny + 1, m.nx + 1)[1:-1, 1:-1]
    np.testing.assert_allclose((txx - sxx) / m.dt, rate[0, 0], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose((tyy - syy) / m.dt, rate[1, 1], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose((txy - sxy) / m.dt, rate[0, 1], rtol=1e-6, atol=1e-9)
    assert np.allclose(o.get("p"), 0.4, rtol=0, atol=1e-15)    # a scalar does not rotate
    o.close()


@pytest.mark.parametrize("axis", [(0.0, 0.0, 1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.3, -0.5, 0.8)],
                         ids=["z", "x", "y", "general"])
def test_rigid_rotation_3d_corotates_the_stress(axis):
    m = Model(ndim=3, nx=8, ny=7, nz=9, dt=1e-3)
    Om = 0.9 * np.array(axis) / np.linalg.norm(axis)
    ox, oy, oz = Om
    o = Oracle(m)
    # v = Omega x r
    set_velocity(o, m, lambda x, y, z: oy * z - oz * y, lambda x, y, z: oz * x - ox * z,
                 lambda x, y, z: ox * y - oy * x)
    tau = np.array([[0.3, 0.21, -0.13], [0.21, -0.1, 0.17], [-0.13, 0.17, -0.2]])
    nc = m.nx * m.ny * m.nz
    sizes = {"txy": (m.nx + 1) * (m.ny + 1) * m.nz, "txz": (m.nx + 1) * m.ny * (m.nz + 1),
             "tyz": m.nx * (m.ny + 1) * (m.nz + 1)}
    o.set("txx", np.full(nc, tau[0, 0]))
    o.set("tyy", np.full(nc, tau[1, 1]))
    o.set("tzz", np.full(nc, tau[2, 2]))
    o.set("txy", np.full(sizes["txy"], tau[0, 1]))
    o.set("txz", np.full(sizes["txz"], tau[0, 2]))
    o.set("tyz", np.full(sizes["tyz"], tau[1, 2]))
    o.objective_update()
    W = np.array([[0.0, -oz, oy], [oz, 0.0, -ox], [-oy, ox, 0.0]])   # grad v, antisymmetric
    rate = rot_rate(W, tau)
    nx, ny, nz = m.nx, m.ny, m.nz
    inner = (slice(2, -2), slice(2, -2), slice(2, -2))
    got = {
        "txx": o.get("txx").reshape(nz, ny, nx)[inner], "tyy": o.get("tyy").reshape(nz, ny, nx)[inner],
        "tzz": o.get("tzz").reshape(nz, ny, nx)[inner],
        "txy": o.get("txy").reshape(nz, ny + 1, nx + 1)[inner],
        "txz": o.get("txz").reshape(nz + 1, ny, nx + 1)[inner],
        "tyz": o.get("tyz").reshape(nz + 1, ny + 1, nx)[inner],
    }
    for name, (a, b) in {"txx": (0, 0), "tyy": (1, 1), "tzz": (2, 2), "txy": (0, 1), "txz": (0, 2),
                         "tyz": (1, 2)}.items():
        np.testing.assert_allclose((got[name] - tau[a, b]) / m.dt, rate[a, b], rtol=1e-6, atol=1e-9,
                                   err_msg=name)
    o.close()


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("sign", [1.0, -1.0], ids=["pos", "neg"])
def test_uniform_translation_transports_linear_fields_exactly(ndim, sign):
    m = Model(ndim=ndim, nx=10, ny=9, nz=8, dt=2e-3)
    U, V, Wz = sign * 0.6, sign * -0.4, sign * 0.5
    o = Oracle(m)
    set_velocity(o, m, lambda x, y, z: U + 0 * x, lambda x, y, z: V + 0 * x, lambda x, y, z: Wz + 0 * x)
    if ndim == 2:
        xn, yn, xc, yc = coords(m)
        X, Y = grid(xc, yc)
        Z = 0 * X
    else:
        xn, yn, zn, xc, yc, _, zc = coords(m)
        X, Y, Z = grid(xc, yc, zc)
    a, b, c = 0.7, -0.3, 0.45
    f = 0.1 + a * X + b * Y + c * Z
    o.set("p", f)
    o.set("txx", 2 * f)
    o.objective_update()
    drift = U * a + V * b + (Wz * c if ndim == 3 else 0.0)
    sl = tuple([slice(1, -1)] * ndim)
    got_p = o.get("p").reshape(f.shape)[sl]
    got_t = o.get("txx").reshape(f.shape)[sl]
    np.testing.assert_allclose(got_p, f[sl] - m.dt * drift, rtol=0, atol=1e-13)
    np.testing.assert_allclose(got_t, 2 * f[sl] - 2 * m.dt * drift, rtol=0, atol=1e-13)
    o.close()


def test_xy_shear_point_transport_2d():
    """Interior vertices carry tau_xy with the vertex-averaged velocity."""
    m = Model(ndim=2, nx=10, ny=9, dt=2e-3)
    U, V = 0.5, 0.3
    o = Oracle(m)
    set_velocity(o, m, lambda x, y, z: U + 0 * x, lambda x, y, z: V + 0 * x)
    xn, yn, xc, yc = coords(m)
    X, Y = grid(xn, yn)
    f = 0.2 + 0.6 * X - 0.8 * Y
    o.set("txy", f)
    o.objective_update()
    got = o.get("txy").reshape(f.shape)
    inner = (slice(2, -1), slice(2, -1))
    np.testing.assert_allclose(got[inner], f[inner] - m.dt * (U * 0.6 + V * -0.8), rtol=0, atol=1e-13)
    # wall vertices keep their values (free-slip walls carry no shear stress)
    assert np.array_equal(got[0, :], f[0, :]) and np.array_equal(got[:, -1], f[:, -1])
    o.close()


@pytest.mark.parametrize("ndim", [2, 3])
def test_pure_shear_and_rest_leave_homogeneous_state(ndim):
    m = Model(ndim=ndim, nx=9, ny=8, nz=7, dt=1e-3)
    for vel in ("rest", "pure shear"):
        o = Oracle(m)
        if vel == "pure shear":
            set_velocity(o, m, lambda x, y, z: 1.0 * x, lambda x, y, z: -1.0 * y, lambda x, y, z: 0 * z)
        before = {}
        for k in (["p", "txx", "tyy", "txy"] + (["tzz", "txz", "tyz"] if ndim == 3 else [])):
            n = o.get(k).size
            val = {"p": 0.3, "txx": 0.2, "tyy": -0.15, "tzz": -0.05, "txy": 0.1, "txz": -0.07, "tyz": 0.04}[k]
            o.set(k, np.full(n, val))
            before[k] = val
        o.objective_update()
        for k, val in before.items():
            assert np.allclose(o.get(k), val, rtol=0, atol=1e-15), (vel, k)
        o.close()


def test_update_keeps_the_3d_deviator_trace_free():
    m = Model(ndim=3, nx=7, ny=6, nz=8, dt=1e-3)
    r = np.random.Generator(np.random.PCG64(11))
    o = Oracle(m)
    for k in ("vx", "vy", "vz", "txy", "txz", "tyz", "p"):
        o.set(k, r.standard_normal(o.get(k).size))
    txx = r.standard_normal(o.get("txx").size)
    tyy = r.standard_normal(txx.size)
    o.set("txx", txx)
    o.set("tyy", tyy)
    o.set("tzz", -(txx + tyy))
    o.objective_update()
    tr = o.get("txx") + o.get("tyy") + o.get("tzz")
    assert np.abs(tr).max() < 1e-13
    o.close()


def test_load_step_applies_the_update_to_the_carried_stresses():
    """With the objective flag, an increment starts from the updated stresses:
    the increment-start copies equal one update of the previous state."""
    m = Model(ndim=2, nx=15, ny=13, dt=1e-4, tol=1e-8, steps=3, objective=1, incl_radius=0.2)
    a, b = Oracle(m), Oracle(m.with_(objective=0))
    for _ in range(2):
        a.load_step()
    names = ["vx", "vy", "p", "txx", "tyy", "txy"]
    st = a.fields(names)
    for k in names:
        b.set(k, st[k])
    b.objective_update()
    a.load_step()
    for k in ("p", "txx", "tyy", "txy"):
        np.testing.assert_allclose(a.get(k + "_old"), b.get(k), rtol=0, atol=1e-15, err_msg=k)
    a.close()
    b.close()


def test_rigid_rotation_of_linear_fields_2d_matches_the_continuum_rate():
    """Linear stress fields under a rigid rotation: the 4-point means and the
    upwind differences are exact for linear fields, so at interior points the
    update divided by dt equals tau^R - v.grad tau of the continuum fields."""
    m = Model(ndim=2, nx=14, ny=12, dt=1e-3)
    om = 0.6
    o = Oracle(m)
    set_velocity(o, m, lambda x, y, z: -om * y, lambda x, y, z: om * x)
    xn, yn, xc, yc = coords(m)
    XC, YC = grid(xc, yc)
    XN, YN = grid(xn, yn)
    fxx = lambda x, y: 0.3 + 0.2 * x - 0.1 * y
    fyy = lambda x, y: -0.2 + 0.05 * x + 0.15 * y
    fxy = lambda x, y: 0.1 - 0.3 * x + 0.25 * y
    o.set("txx", fxx(XC, YC))
    o.set("tyy", fyy(XC, YC))
    o.set("txy", fxy(XN, YN))
    o.set("p", 0.5 + 0.4 * XC - 0.2 * YC)
    o.objective_update()
    w = -om                                      # w_xy = (dvx/dy - dvy/dx) / 2
    vx, vy = -om * YC, om * XC
    inner = (slice(1, -1), slice(1, -1))
    rxx = 2 * fxy(XC, YC) * w - (vx * 0.2 + vy * -0.1)
    ryy = -2 * fxy(XC, YC) * w - (vx * 0.05 + vy * 0.15)
    rp = -(vx * 0.4 + vy * -0.2)
    got = lambda k, shape: o.get(k).reshape(shape)
    np.testing.assert_allclose(((got("txx", XC.shape) - fxx(XC, YC)) / m.dt)[inner], rxx[inner], rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(((got("tyy", XC.shape) - fyy(XC, YC)) / m.dt)[inner], ryy[inner], rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(((got("p", XC.shape) - (0.5 + 0.4 * XC - 0.2 * YC)) / m.dt)[inner], rp[inner],
                               rtol=1e-7, atol=1e-9)
    vxn, vyn = -om * YN, om * XN
    rxy = w * (fyy(XN, YN) - fxx(XN, YN)) - (vxn * -0.3 + vyn * 0.25)
    vin = (slice(2, -2), slice(2, -2))
    np.testing.assert_allclose(((got("txy", XN.shape) - fxy(XN, YN)) / m.dt)[vin], rxy[vin], rtol=1e-7, atol=1e-9)
    o.close()


def test_rigid_rotation_of_linear_fields_3d_matches_the_continuum_rate():
    m = Model(ndim=3, nx=10, ny=9, nz=11, dt=1e-3)
    Om = np.array([0.3, -0.5, 0.7])
    ox, oy, oz = Om
    o = Oracle(m)
    set_velocity(o, m, lambda x, y, z: oy * z - oz * y, lambda x, y, z: oz * x - ox * z,
                 lambda x, y, z: ox * y - oy * x)
    xn, yn, zn, xc, yc, _, zc = coords(m)
    r = np.random.Generator(np.random.PCG64(5))
    coef = {k: r.uniform(-0.3, 0.3, 4) for k in ("txx", "tyy", "txy", "txz", "tyz", "p")}
    lin = lambda k, X, Y, Z: coef[k][0] + coef[k][1] * X + coef[k][2] * Y + coef[k][3] * Z
    loc = {"c": (xc, yc, zc), "txy": (xn, yn, zc), "txz": (xn, yc, zn), "tyz": (xc, yn, zn)}
    G = {k: grid(*v) for k, v in loc.items()}
    for k in ("txx", "tyy", "p"):
        o.set(k, lin(k, *G["c"]))
    o.set("tzz", -(lin("txx", *G["c"]) + lin("tyy", *G["c"])))
    for k in ("txy", "txz", "tyz"):
        o.set(k, lin(k, *G[k]))
    o.objective_update()
    W = np.array([[0.0, -oz, oy], [oz, 0.0, -ox], [-oy, ox, 0.0]])   # w_ab = (dv_a/dx_b - dv_b/dx_a)/2

    def expected(name, X, Y, Z):
        tau = np.zeros(X.shape + (3, 3))
        tau[..., 0, 0], tau[..., 1, 1] = lin("txx", X, Y, Z), lin("tyy", X, Y, Z)
        tau[..., 2, 2] = -(tau[..., 0, 0] + tau[..., 1, 1])
        for (a, b), k in {(0, 1): "txy", (0, 2): "txz", (1, 2): "tyz"}.items():
            tau[..., a, b] = tau[..., b, a] = lin(k, X, Y, Z)
        rot = W @ tau - tau @ W                 # tau^R = w tau - tau w
        v = np.stack([oy * Z - oz * Y, oz * X - ox * Z, ox * Y - oy * X], -1)
        idx = {"txx": (0, 0), "tyy": (1, 1), "tzz": (2, 2), "txy": (0, 1), "txz": (0, 2), "tyz": (1, 2)}
        if name == "p":
            grad = coef["p"][1:]
            return -(v @ grad)
        a, b = idx[name]
        grad = coef[name][1:] if name != "tzz" else -(coef["txx"][1:] + coef["tyy"][1:])
        return rot[..., a, b] - v @ grad

    inner = (slice(2, -2), slice(2, -2), slice(2, -2))
    for name, where in [("txx", "c"), ("tyy", "c"), ("tzz", "c"), ("p", "c"), ("txy", "txy"), ("txz", "txz"),
                        ("tyz", "tyz")]:
        X, Y, Z = G[where]
        before = (lin(name, X, Y, Z) if name != "tzz" else -(lin("txx", X, Y, Z) + lin("tyy", X, Y, Z)))
        got = (o.get(name).reshape(X.shape) - before) / m.dt
        np.testing.assert_allclose(got[inner], expected(name, X, Y, Z)[inner], rtol=1e-7, atol=1e-9,
                                   err_msg=name)
    o.close()


def _checkerboard(shape, amp):
    """Face velocities alternating in sign along every axis: their means at
    centres and shear points vanish exactly (no advection), their
    differences do not (vorticity at every shear point)."""
    return amp * (-1.0) ** np.indices(shape).sum(axis=0)


@pytest.mark.parametrize("ndim", [2, 3])
def test_rotation_terms_preserve_j2_in_nonhomogeneous_states(ndim):
    """The co-rotational terms Wτ - τW do no work on the stress:
    τ : (Wτ - τW) = 0 pointwise for any symmetric τ and antisymmetric W.  On
    the staggered grid the centre terms (4-point means of shear products) and
    the shear-point terms (vorticity times 4-point means of centre stresses,
    and in 3D products of means of the other shear components) pair up so
    that the grid sum of τ : τ^R vanishes exactly for any stress field, not
    only homogeneous or linear ones.  Random non-homogeneous stresses with a
    checkerboard velocity field (vorticity everywhere, zero advection): the
    sum over centres and (twice) over shear points cancels to rounding while
    each part is of the size of the terms; a dropped term, a wrong sign or a
    mean taken over other points breaks the cancellation."""
    from fieldtools import shapes
    if ndim == 2:
        m = Model(ndim=2, nx=13, ny=11, lx=1.3, dt=1e-3, objective=1)
    else:
        m = Model(ndim=3, nx=9, ny=8, nz=7, ly=0.9, lz=0.8, dt=1e-3, objective=1)
    sh = shapes(m)
    r = np.random.Generator(np.random.PCG64(11))
    shear = ["txy"] + (["txz", "tyz"] if ndim == 3 else [])
    tau = {k: r.standard_normal(sh[k]) * 1e-3 for k in ["txx", "tyy"] + shear}
    p = r.standard_normal(sh["p"]) * 1e-3
    vel = {"vx": _checkerboard(sh["vx"], 0.7), "vy": _checkerboard(sh["vy"], -0.4)}
    if ndim == 3:
        vel["vz"] = _checkerboard(sh["vz"], 0.3)
    o = Oracle(m)
    for k, v in list(tau.items()) + list(vel.items()) + [("p", p)]:
        o.set(k, v.ravel())
    cent = ["txx", "tyy"] + (["tzz"] if ndim == 3 else [])
    t0 = {k: o.get(k).reshape(sh[k]) for k in cent + shear}
    o.objective_update()
    rate = {k: (o.get(k).reshape(sh[k]) - t0[k]) / m.dt for k in cent + shear}
    assert np.array_equal(o.get("p").reshape(sh["p"]), p)          # no advection
    c = sum((t0[k] * rate[k]).sum() for k in cent)
    s = 2.0 * sum((t0[k] * rate[k]).sum() for k in shear)
    size = sum(np.abs(t0[k] * rate[k]).sum() for k in cent) + 2.0 * sum(np.abs(t0[k] * rate[k]).sum() for k in shear)
    assert abs(c) > 1e-3 * size and abs(s) > 1e-3 * size       # both parts work ...
    assert abs(c + s) <= 1e-13 * size, (c, s, size)              # ... and cancel
    o.close()
