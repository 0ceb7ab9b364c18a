"""Pins for the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each expected value comes from
a closed form, a constant the paper prints, a textbook result, a different
algorithm (direct sparse solve), or an exact discrete identity.
"""
import math

import numpy as np
import pytest

from ep_workloads import Model, cohesion_field, c1_small_2d, pressure_anomaly, random_state
from oracle.oracle import Oracle
from oracle import direct_elastic
from fieldtools import field_errors, mirror

RE_OPT = 3.0 * math.sqrt(10.0) * math.pi / 2.0


def homog(ndim=2, n=(7, 5, 4), **kw):
    base = dict(ndim=ndim, nx=n[0], ny=n[1], nz=n[2] if ndim == 3 else 1,
                incl_factor=1.0, tol=1e-12, n_check=10, max_iter=200000)
    base.update(kw)
    return Model(**base)


def tau_ii_2d(f):
    """Centre tauII with the vertex shear averaged to centres (2D J2 as printed)."""
    return np.sqrt(0.5 * (f["txx"] ** 2 + f["tyy"] ** 2))


# --------------------------------------------------------------- constants
def test_drucker_prager_constants_30deg():
    """2D: A = sin30 = 1/2, B = cos30; 3D: B = 6cos30/(sqrt3 * 2.5) = 1.2, A = 1.2/sqrt3
    (Plasticity section, A and B for 2D and 3D)."""
    s2 = Oracle(homog(2)).scalars()
    assert s2["A"] == pytest.approx(0.5, rel=1e-15)
    assert s2["B"] == pytest.approx(math.sqrt(3.0) / 2.0, rel=1e-15)
    s3 = Oracle(homog(3)).scalars()
    assert s3["B"] == pytest.approx(1.2, rel=1e-15)
    assert s3["A"] == pytest.approx(1.2 / math.sqrt(3.0), rel=1e-15)


@pytest.mark.parametrize("ndim", [2, 3])
def test_pt_parameters_satisfy_their_definitions(ndim):
    """rho~, G~, K~ from the PT equations: K~/G~ = r, the numerical Reynolds number
    rho~ Vp L / eta equals 3 sqrt(10) pi / 2 (optimal value), and Vp dtau / h is the
    Courant number 0.9/sqrt(ndim)."""
    m = homog(ndim, dt=2e-4, visc=5e-3)
    s = Oracle(m).scalars()
    eta = 1.0 / (1.0 / (m.shear * m.dt) + 1.0 / m.visc)
    assert s["eta"] == pytest.approx(eta, rel=1e-14)
    assert s["kdtau"] / s["gdtau"] == pytest.approx(0.5, rel=1e-14)
    vp_dtau = math.sqrt((s["kdtau"] + 4.0 / 3.0 * s["gdtau"]) * s["dtrho"])   # Vp * dtau
    assert vp_dtau / s["h"] == pytest.approx(0.9 / math.sqrt(ndim), rel=1e-13)
    re = vp_dtau * s["L"] / (eta * s["dtrho"])                                   # rho~ Vp L / eta
    assert re == pytest.approx(RE_OPT, rel=1e-13)
    assert RE_OPT == pytest.approx(14.901882, rel=1e-6)


# ----------------------------------------------------- homogeneous elastic
@pytest.mark.parametrize("ndim", [2, 3])
def test_pure_shear_elastic_closed_form(ndim):
    """Homogeneous pure shear (v_x = a x, v_y = -a y [, v_z = 0]): tau_xx = 2 G a t,
    tau_yy = -2 G a t, p = 0, no shear stress, v stays the background field."""
    m = homog(ndim, c0=1.0)
    o = Oracle(m)
    v0 = {k: o.get(k) for k in (("vx", "vy") if ndim == 2 else ("vx", "vy", "vz"))}
    for n in range(1, 6):
        st = o.load_step()
        assert st["status"] == 0
        f = o.fields()
        t = n * m.dt
        np.testing.assert_allclose(f["txx"], 2 * m.shear * t, rtol=1e-11)
        np.testing.assert_allclose(f["tyy"], -2 * m.shear * t, rtol=1e-11)
        assert np.abs(f["p"]).max() < 1e-15
        assert np.abs(f["txy"]).max() < 1e-15
        if ndim == 3:
            assert np.abs(f["tzz"]).max() < 1e-15
            assert np.abs(f["txz"]).max() < 1e-15 and np.abs(f["tyz"]).max() < 1e-15
        for k, v in v0.items():
            np.testing.assert_allclose(f[k], v, rtol=0, atol=1e-15)
        # accumulated strain of the background field
        np.testing.assert_allclose(f["exx"], t, rtol=1e-12)


def test_isotropic_compression_2d_plane_strain():
    """erate = diag(-1, -1): dtheta = -2 t, p = -K dtheta = 2 K t; with the 1/3
    deviatoric projection in plane strain tau_xx = tau_yy = 2 G (-1 + 2/3) t."""
    m = homog(2, c0=1.0, erate=(-1.0, -1.0, 0.0))
    o = Oracle(m)
    for n in range(1, 4):
        assert o.load_step()["status"] == 0
        f = o.fields()
        t = n * m.dt
        np.testing.assert_allclose(f["p"], 2 * m.bulk * t, rtol=1e-10)
        np.testing.assert_allclose(f["txx"], -2.0 / 3.0 * m.shear * t, rtol=1e-10)
        np.testing.assert_allclose(f["tyy"], -2.0 / 3.0 * m.shear * t, rtol=1e-10)


def test_isotropic_compression_3d():
    """erate = diag(-1,-1,-1): p = 3 K t and the deviator stays zero."""
    m = homog(3, c0=1.0, erate=(-1.0, -1.0, -1.0))
    o = Oracle(m)
    for n in range(1, 4):
        assert o.load_step()["status"] == 0
        f = o.fields()
        np.testing.assert_allclose(f["p"], 3 * m.bulk * n * m.dt, rtol=1e-10)
        for k in ("txx", "tyy", "tzz", "txy", "txz", "tyz"):
            assert np.abs(f[k]).max() < 1e-13


def test_maxwell_relaxation_closed_form():
    """Visco-elastic limit: backward Euler of (1/2G) dtau/dt + tau/(2 mu_s) = e'
    gives tau_n = 2 mu_s e' (1 - q^n), q = 1/(1 + G dt/mu_s); the continuous Maxwell
    solution 2 mu_s e' (1 - exp(-G t/mu_s)) is matched to first order in dt."""
    m = homog(2, c0=1.0, visc=1e-3, dt=1e-4)
    o = Oracle(m)
    q = 1.0 / (1.0 + m.shear * m.dt / m.visc)
    for n in range(1, 8):
        assert o.load_step()["status"] == 0
        f = o.fields()
        exact_disc = 2 * m.visc * 1.0 * (1 - q ** n)
        np.testing.assert_allclose(f["txx"], exact_disc, rtol=1e-10)
        cont = 2 * m.visc * (1 - math.exp(-m.shear * n * m.dt / m.visc))
        assert abs(f["txx"][0] - cont) <= 0.6 * (m.shear * m.dt / m.visc) * cont


# ----------------------------------------------------- homogeneous plastic
@pytest.mark.parametrize("ndim", [2, 3])
def test_pure_shear_yields_at_b_c(ndim):
    """Radial return under pure shear (p = 0): tauII grows as 2 G t until it reaches
    the Drucker-Prager bound B c and then stays there (2D B = cos30, 3D B = 1.2)."""
    c = 4.7e-4            # keeps 2 G t away from an exact tie with B c
    B = math.cos(math.radians(30)) if ndim == 2 else 1.2
    m = homog(ndim, c0=c)
    o = Oracle(m)
    for n in range(1, 7):
        st = o.load_step()
        assert st["status"] == 0
        f = o.fields()
        expect = min(2 * m.shear * n * m.dt, B * c)
        np.testing.assert_allclose(np.abs(f["txx"]), expect, rtol=1e-10)
        np.testing.assert_allclose(f["tyy"], -f["txx"], rtol=1e-12)
        assert np.abs(f["p"]).max() < 1e-15
        if 2 * m.shear * n * m.dt > B * c:
            assert st["n_yield"] == m.n_cells
            # plastic rate: the elastic trial overshoot per step (|S| - Y/eta)
            np.testing.assert_allclose(f["tau_ii"], B * c, rtol=1e-12)


def test_compression_and_shear_yields_at_a_p_plus_b_c():
    """erate = (0.5, -1.5): p = K t grows, the deviator direction is fixed, and after
    yield tauII = A p + B c exactly (non-dilatant flow leaves p elastic)."""
    c = 5e-4
    m = homog(2, c0=c, erate=(0.5, -1.5, 0.0))
    A, B = 0.5, math.cos(math.radians(30))
    edev = np.array([0.5 + 1.0 / 3.0, -1.5 + 1.0 / 3.0])
    edev_ii = math.sqrt(0.5 * (edev ** 2).sum())
    o = Oracle(m)
    yielded = False
    for n in range(1, 10):
        assert o.load_step()["status"] == 0
        f = o.fields()
        t = n * m.dt
        np.testing.assert_allclose(f["p"], m.bulk * t, rtol=1e-10)
        tii = tau_ii_2d(f)
        expect = min(2 * m.shear * t * edev_ii, A * m.bulk * t + B * c)
        yielded |= 2 * m.shear * t * edev_ii > A * m.bulk * t + B * c
        np.testing.assert_allclose(tii, expect, rtol=1e-10)
        np.testing.assert_allclose(f["txx"] / f["tyy"], edev[0] / edev[1], rtol=1e-10)
    assert yielded


def test_apex_isotropic_extension_carries_no_shear():
    """Isotropic extension drives A p + B c below zero: the yield bound is clamped
    at 0 and the returned deviator vanishes (apex of the cone)."""
    m = homog(2, c0=1e-4, erate=(1.0, 1.0, 0.0))
    o = Oracle(m)
    for n in range(1, 4):
        st = o.load_step()
        assert st["status"] == 0
        f = o.fields()
        np.testing.assert_allclose(f["p"], -2 * m.bulk * n * m.dt, rtol=1e-10)
        assert np.abs(f["txx"]).max() == 0.0 and np.abs(f["tyy"]).max() == 0.0
        assert np.all(np.isfinite(f["lambda_dot"]))


# ------------------------------------------------- direct linear solve (N2)
@pytest.mark.parametrize("ndim,n", [(2, (9, 7, 1)), (2, (15, 15, 1)), (3, (5, 6, 4)), (3, (7, 7, 7))])
def test_elastic_increment_matches_direct_solve(ndim, n):
    """A non-equilibrium initial stress (pressure anomaly plus random deviator)
    relaxed by one elastic increment: the PT fixed point must equal the direct
    sparse solution of the discrete linear problem."""
    m = homog(ndim, n=n, c0=10.0, tol=1e-13)
    o = Oracle(m)
    st0 = random_state(m, seed=7, amp_s=1e-3)
    start = {k: v for k, v in st0.items() if not k.startswith("v") and not k.endswith("_old")}
    start["p"] = start["p"] + pressure_anomaly(m, 2e-3, 0.25)
    for k, v in start.items():
        o.set(k, v)
    # walls carry no shear stress (free slip)
    st = o.load_step()
    assert st["status"] == 0
    old = {k + "_old": o.get(k + "_old") for k in start}
    ref = direct_elastic.solve(m, old)
    f = o.fields()
    for k, v in ref.items():
        scale = max(np.abs(v).max(), 1e-30)
        err = np.abs(f[k] - v).max() / scale
        assert err < 1e-9, (k, err)


def test_frozen_increment_matches_direct_solve_with_fixed_lambda():
    """Frozen plasticity (accelerated PT section): an increment frozen before
    it converged ends at the fixed point of the linear problem with the
    stored per-cell Lambda; the direct sparse solve of that linear problem
    (different code: assembled operators, LU) must give the same fields."""
    m = c1_small_2d().with_(n_check=10, dt=2e-4, tol=1e-12, freeze_iter=300,
                            incl_centre=(0.05, 0.03, 0.0))
    o = Oracle(m)
    frozen = None
    for _ in range(8):
        st = o.load_step()
        assert st["status"] == 0
        if st["frozen_at"] > 0:
            frozen = st
            break
    assert frozen is not None and frozen["frozen_at"] >= 300 and frozen["frozen_at"] % 10 == 0
    lam = o.get("lambda_frozen")
    assert lam.max() > 0
    old = {k: o.get(k) for k in ("p_old", "txx_old", "tyy_old", "txy_old")}
    ref = direct_elastic.solve(m, old, lam=lam)
    f = o.fields()
    for k in ("vx", "vy", "p", "txx", "tyy", "txy"):
        scale = max(np.abs(ref[k]).max(), 1e-30)
        err = np.abs(f[k] - ref[k]).max() / scale
        assert err < 1e-8, (k, err)
    # the frozen state is an approximation: Lambda came from a sweep before
    # convergence, so the yield condition holds only approximately
    assert 0 < frozen["max_violation"] < 0.5 * m.c0


# ------------------------------------------------------------ invariants
@pytest.fixture(scope="module")
def c1_run():
    m = c1_small_2d().with_(n_check=10)
    o = Oracle(m)
    o.record_history()
    stats, hists, states = [], [], []
    for _ in range(m.steps):
        stats.append(o.load_step())
        hists.append(o.history())
        states.append(o.fields(["vx", "vy", "p", "txx", "tyy", "txy", "tau_ii", "yield"]))
    return m, o, stats, hists, states


def test_c1_converges_every_increment(c1_run):
    m, o, stats, _, _ = c1_run
    assert all(s["status"] == 0 for s in stats)
    # the inclusion yields first (2 G a t > B c/2 at step 4), the matrix later
    assert stats[2]["n_yield"] == 0 and stats[3]["n_yield"] > 0


def test_yield_invariant_at_centres(c1_run):
    """tauII <= A p + B c at every centre after return mapping."""
    _, _, _, _, states = c1_run
    for f in states:
        assert np.all(f["tau_ii"] <= f["yield"] * (1 + 1e-12) + 1e-300)


def test_force_balance_column_integrals(c1_run):
    """Adjacent column integrals of sigma_xx differ by dx * sum_j R_x dy, and wall
    shear is zero, so every column carries the same force up to Lx Ly |R|inf."""
    m, _, stats, _, _ = c1_run
    for s in stats:
        bound = m.lx * m.ly * s["resid"] * 2
        assert abs(s["sxx_centre"] - s["sxx_left"]) <= bound + 1e-16
        assert abs(s["sxx_right"] - s["sxx_left"]) <= bound + 1e-16


def test_mirror_symmetry_before_yield(c1_run):
    """Centred inclusion and pure shear, elastic increments: the state is mirror
    symmetric (vx odd in x, vy odd in y, tau_xy odd in both, p and normal
    deviators even)."""
    m, _, _, _, states = c1_run
    for f in states[:3]:
        g = {k: f[k] for k in ("vx", "vy", "p", "txx", "tyy", "txy")}
        for axes in ((0,), (1,)):
            mm = mirror(m, g, axes)
            errs = field_errors(m, mm, g, list(g))
            assert max(errs.values()) <= 1e-10, (axes, errs)


@pytest.mark.parametrize("axes", [(0,), (1,), (0, 1)])
def test_mirror_equivariance_after_yield(axes):
    """The discrete equations commute with reflections: solving an increment from
    a mirrored (post-yield, asymmetric) state gives the mirrored solution."""
    m = c1_small_2d().with_(n_check=10, tol=1e-11)
    o = Oracle(m)
    for _ in range(5):
        assert o.load_step()["status"] == 0
    names = ["vx", "vy", "p", "txx", "tyy", "txy"]
    start = o.fields(names)
    assert o.load_step()["status"] == 0
    sol = o.fields(names)
    o2 = Oracle(m)
    for k, v in mirror(m, start, axes).items():
        o2.set(k, v)
    assert o2.load_step()["status"] == 0
    errs = field_errors(m, o2.fields(names), mirror(m, sol, axes), names)
    assert max(errs.values()) <= 1e-8, errs


def test_residual_envelope_plastic_is_bounded(c1_run):
    """Plastic increments: the PT residual oscillates and can plateau while the set
    of yielding cells reorganises, but it stays bounded by its early level and
    ends below the tolerance."""
    m, _, stats, hists, _ = c1_run
    per = m.nx // 10                      # checks per nx iterations (n_check = 10)
    for s, h in zip(stats, hists):
        if s["iters"] == 0:               # the starting state met the tolerance
            assert len(h) == 0 and s["cert"] <= m.tol * s["ref"]
            continue
        assert h[-1] <= m.tol * s["ref"]
        if len(h) > 2 * per:
            assert h[per:].max() <= 2.0 * h[:per].max()


@pytest.mark.parametrize("ndim", [2, 3])
def test_residual_envelope_elastic_decreases(ndim):
    """Elastic increment with a heterogeneous start (linear problem): sampled every
    nx iterations after the first nx, the running minimum of the residual drops by
    at least 10x every 16 nx iterations until the tolerance is met."""
    n = (31, 31, 1) if ndim == 2 else (15, 15, 15)
    m = homog(ndim, n=n, c0=10.0, tol=1e-12, n_check=1)
    o = Oracle(m)
    o.set("p", pressure_anomaly(m, 2e-3, 0.25))
    o.record_history()
    st = o.load_step()
    assert st["status"] == 0
    h = o.history()
    runmin = np.minimum.accumulate(h)
    win = 16 * m.nx
    for a in range(m.nx, len(h) - win, win):
        assert runmin[a + win] <= 0.1 * runmin[a] or runmin[a + win] <= m.tol * st["ref"]


def test_pt_parameters_do_not_move_elastic_fixed_point():
    """The converged increment does not depend on the PT parameters (cfl, Re)."""
    m = homog(2, n=(15, 13, 1), c0=10.0, tol=1e-13)
    outs = []
    for cfl, re in ((0.0, 0.0), (0.8 * 0.9 / math.sqrt(2), 1.3 * RE_OPT)):
        o = Oracle(m.with_(cfl=cfl, re=re))
        o.set("p", pressure_anomaly(m, 2e-3, 0.3))
        assert o.load_step()["status"] == 0
        outs.append(o.fields(["vx", "vy", "p", "txx", "tyy", "txy"]))
    for k in outs[0]:
        sc = np.abs(outs[0][k]).max()
        assert np.abs(outs[0][k] - outs[1][k]).max() <= 1e-9 * sc


def test_3d_deviator_stays_trace_free():
    m = homog(3, n=(9, 9, 9), c0=1.75e-3, incl_factor=0.5, incl_radius=0.3, dt=2e-4)
    o = Oracle(m)
    for _ in range(6):
        assert o.load_step()["status"] == 0
    f = o.fields()
    assert np.abs(f["txx"] + f["tyy"] + f["tzz"]).max() <= 1e-15
    assert np.all(f["tau_ii"] <= f["yield"] * (1 + 1e-12))


# ---------------------------------------------- planted-mistake sanity check
def test_direct_solve_detects_a_planted_sign_error():
    """The direct-solve pin is sharp enough to catch a flipped shear term."""
    m = homog(2, n=(9, 7, 1), c0=10.0, tol=1e-13)
    o = Oracle(m)
    o.set("p", pressure_anomaly(m, 2e-3, 0.3))
    assert o.load_step()["status"] == 0
    old = {k: o.get(k) for k in ("p_old", "txx_old", "tyy_old", "txy_old")}
    ref = direct_elastic.solve(m, old)
    wrong = dict(old)
    wrong["txy_old"] = old["txy_old"]
    good = np.abs(o.get("vx") - ref["vx"]).max()
    # a planted mistake on the reference side: drop the pressure of the old state
    bad = direct_elastic.solve(m, dict(old, p_old=0 * old["p_old"]))
    assert good < 1e-9 * np.abs(ref["vx"]).max()
    assert np.abs(o.get("vx") - bad["vx"]).max() > 1e-6 * np.abs(ref["vx"]).max()
