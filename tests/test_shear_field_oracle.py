"""Pins of the oracle's per-cell shear modulus (2D; the heterogeneous setups'
G field, section on the initial conditions and heterogeneities).

- Bilayer: two halves of different G under pure shear (free-slip walls, no
  yielding) have an exact piecewise-homogeneous solution: each half is
  uniformly strained, sigma_xx is continuous across the interface, the
  vertical strain rate is that of the walls and the horizontal rates average
  to that of the walls.  With a_k = K + 4 G_k / 3, b_k = K - 2 G_k / 3 and
  the wall rates (1, -1), the left rate is x1 = (2 a2 + b1 - b2)/(a1 + a2),
  the right one 2 - x1; stresses follow from Hooke's law in plane strain.
- A Gaussian G field (elastic): every converged increment equals the sparse
  direct solve of the discrete increment equations with the same field,
  under two reference moduli (which set only the pseudo-time steps).
- A field equal to the reference modulus reproduces the uniform run bit for
  bit; a G above the reference or a 3D model is rejected."""
import numpy as np
import pytest

from ep_workloads import Model
from oracle import direct_elastic
from oracle.oracle import Oracle


def test_bilayer_is_piecewise_homogeneous():
    G1, G2, K, n = 0.8, 1.0, 2.0, 4
    m = Model(ndim=2, nx=20, ny=9, lx=1.0, ly=1.0, bulk=K, shear=G2, c0=10.0, dt=1e-4, tol=1e-12, n_check=10,
              steps=n)
    G = np.where(np.arange(m.nx) < m.nx // 2, G1, G2)[None, :].repeat(m.ny, 0)
    o = Oracle(m)
    o.set_shear_modulus(G)
    for _ in range(n):
        assert o.load_step()["status"] == 0
    a1, b1, a2, b2 = K + 4 * G1 / 3, K - 2 * G1 / 3, K + 4 * G2 / 3, K - 2 * G2 / 3
    x1 = (2 * a2 + b1 - b2) / (a1 + a2)
    e = n * m.dt
    for half, (Gk, rate) in enumerate(((G1, x1), (G2, 2 - x1))):
        exx, eyy = rate * e, -e
        vol = exx + eyy
        cols = slice(0, m.nx // 2) if half == 0 else slice(m.nx // 2, m.nx)
        for name, want in (("p", -K * vol), ("txx", 2 * Gk * (exx - vol / 3)), ("tyy", 2 * Gk * (eyy - vol / 3))):
            got = o.get(name).reshape(m.ny, m.nx)[:, cols]
            np.testing.assert_allclose(got, want, rtol=1e-8, atol=1e-12 * e, err_msg=(name, half))
    sxx = (-o.get("p") + o.get("txx")).reshape(m.ny, m.nx)
    assert np.ptp(sxx) <= 1e-8 * np.abs(sxx).max()               # sigma_xx continuous
    assert abs(x1 - 1.0) > 0.02                                  # the layers do strain differently
    o.close()


def gaussian_G(m, centre=(0.07, -0.05)):
    """G = 1 at (near) the centre rising to 1.2 towards the walls (the
    heterogeneous setups' shear modulus), off-centre so no symmetry helps."""
    xc = -0.5 * m.lx + (np.arange(m.nx) + 0.5) * (m.lx / m.nx)
    yc = -0.5 * m.ly + (np.arange(m.ny) + 0.5) * (m.ly / m.ny)
    X, Y = np.meshgrid(xc, yc)
    return (1.2 - 0.2 * np.exp(-((X - centre[0]) ** 2 + (Y - centre[1]) ** 2) / 0.2 ** 2)).ravel()


def test_heterogeneous_elastic_increments_match_the_direct_solve():
    """Gaussian G, elastic: every converged increment equals the sparse direct
    solve of the discrete increment equations with the same G (shear stresses
    are non-zero, so the vertex compliance matters), and the reference
    modulus, which sets only the pseudo-time steps, does not move it."""
    m = Model(ndim=2, nx=29, ny=23, lx=1.2, shear=1.2, c0=10.0, dt=1e-4, tol=1e-12, n_check=10, steps=3)
    G = gaussian_G(m)
    a, b = Oracle(m), Oracle(m.with_(shear=1.5))
    a.set_shear_modulus(G)
    b.set_shear_modulus(G)
    for _ in range(m.steps):
        old = {k: a.get(k) for k in ("p", "txx", "tyy", "txy")}
        assert a.load_step()["status"] == 0 and b.load_step()["status"] == 0
        ref = direct_elastic.solve(m, {k + "_old": v for k, v in old.items()}, shear_field=G)
        for k in ("vx", "vy", "p", "txx", "tyy", "txy"):
            sc = np.abs(ref[k]).max()
            assert np.abs(a.get(k) - ref[k]).max() <= 1e-8 * sc, k
            assert np.abs(b.get(k) - ref[k]).max() <= 1e-8 * sc, k
    assert np.abs(a.get("txy")).max() > 1e-3 * np.abs(a.get("txx")).max()
    # the same increments with uniform G = 1.2 differ: the field is in effect
    u = direct_elastic.solve(m, {k + "_old": v for k, v in old.items()})
    assert np.abs(u["txy"] - a.get("txy")).max() > 1e-2 * np.abs(a.get("txy")).max()
    a.close()
    b.close()


def test_field_equal_to_the_reference_is_the_uniform_run_and_bad_fields_are_rejected():
    m = Model(ndim=2, nx=23, ny=19, dt=2e-4, tol=1e-9, n_check=10, incl_radius=0.2, steps=5)
    a, b = Oracle(m), Oracle(m)
    b.set_shear_modulus(np.full(m.nx * m.ny, m.shear))
    for _ in range(m.steps):
        assert a.load_step()["iters"] == b.load_step()["iters"]
    for k in ("vx", "vy", "p", "txx", "tyy", "txy"):
        assert np.array_equal(a.get(k), b.get(k)), k
    with pytest.raises(ValueError):
        b.set_shear_modulus(np.full(m.nx * m.ny, 1.01 * m.shear))
    with pytest.raises(ValueError):
        b.set_shear_modulus(np.zeros(m.nx * m.ny))
    a.close()
    b.close()


@pytest.mark.parametrize("plane", ["xy", "xz", "yz"])
def test_3d_field_invariant_along_one_axis_reduces_to_2d(plane):
    """A 3D model whose G field does not vary along one axis, loaded by pure
    shear in the other two (no strain rate along the invariant axis), has the
    plane-strain solution of the 2D model in that plane with the same G
    field: each edge type's compliance (xy edges for a z-invariant field, xz
    for y-invariant, yz for x-invariant) must reproduce the 2D vertex
    compliance, pinned above by the direct solve."""
    n2 = (13, 11)
    axes = {"xy": (0, 1, 2), "xz": (0, 2, 1), "yz": (1, 2, 0)}[plane]   # 2D x, 2D y, invariant axis
    m2 = Model(ndim=2, nx=n2[0], ny=n2[1], lx=1.2, ly=1.0, shear=1.2, c0=10.0, dt=1e-4, tol=1e-12, n_check=10,
               steps=3)
    G2 = gaussian_G(m2).reshape(n2[1], n2[0])
    n3 = [0, 0, 0]
    ext = [0.0, 0.0, 0.0]
    n3[axes[0]], n3[axes[1]], n3[axes[2]] = n2[0], n2[1], 4
    ext[axes[0]], ext[axes[1]], ext[axes[2]] = 1.2, 1.0, 0.7
    er = [0.0, 0.0, 0.0]
    er[axes[0]], er[axes[1]] = 1.0, -1.0
    m3 = Model(ndim=3, nx=n3[0], ny=n3[1], nz=n3[2], lx=ext[0], ly=ext[1], lz=ext[2], shear=1.2, c0=10.0,
               dt=1e-4, erate=tuple(er), tol=1e-12, n_check=10, steps=3)
    # G3 indexed (z, y, x); the 2D field (y2, x2) broadcast along the invariant axis
    z, y, x = np.meshgrid(np.arange(n3[2]), np.arange(n3[1]), np.arange(n3[0]), indexing="ij")
    pos = (x, y, z)
    G3 = G2[pos[axes[1]], pos[axes[0]]]
    o2, o3 = Oracle(m2), Oracle(m3)
    o2.set_shear_modulus(G2.ravel())
    o3.set_shear_modulus(G3.ravel())
    for _ in range(3):
        assert o2.load_step()["status"] == 0 and o3.load_step()["status"] == 0
    names3 = {"xy": ("txx", "tyy", "txy"), "xz": ("txx", "tzz", "txz"), "yz": ("tyy", "tzz", "tyz")}[plane]
    shapes3 = {"txy": (n3[2], n3[1] + 1, n3[0] + 1), "txz": (n3[2] + 1, n3[1], n3[0] + 1),
               "tyz": (n3[2] + 1, n3[1] + 1, n3[0])}
    for k2, k3 in zip(("p", "txx", "tyy", "txy"), ("p",) + names3):
        a2 = o2.get(k2)
        shape3 = shapes3.get(k3, (n3[2], n3[1], n3[0]))
        a3 = o3.get(k3).reshape(shape3)
        # move the 2D axes to (y2, x2) and take an interior slice along the invariant axis
        order = [2 - axes[1], 2 - axes[0], 2 - axes[2]]
        a3 = np.transpose(a3, order)
        sl = a3[..., 1] if a3.shape[2] > 1 else a3[..., 0]
        sc = np.abs(a2).max()
        assert sl.shape == (a2.size // sl.shape[1], sl.shape[1])
        assert np.abs(sl.ravel() - a2).max() <= 1e-8 * sc, (plane, k3)
    assert np.abs(o2.get("txy")).max() > 1e-3 * np.abs(o2.get("txx")).max()
    o2.close()
    o3.close()
