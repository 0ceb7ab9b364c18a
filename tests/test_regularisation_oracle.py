"""Pins of the consistency-regularised return (eta_vp > 0) in the oracle.

The constitutive section splits the strain rate into elastic and visco-plastic
parts; the introduction cites a consistency viscosity as the regularisation
of the localisation width.  Reading: a yielding point carries
    tauII = A p + B c + eta_vp lambda_dot,   lambda_dot = 2 eps_dot_p,II,
so the stress exceeds the Drucker-Prager bound by a viscous overstress.

A homogeneous model under pure shear (uniform cohesion, free-slip walls) has a
homogeneous solution; every converged increment must satisfy the continuum
increment equations in closed form, solved here by hand from the previous
increment's state (mu_s = inf, so D = 1/(G dt)):
    T = tau^/(G dt) + 2 e',  s = sqrt(J2(T)),
    lambda_dot = (s - D (A p^ + B c)) / (1 + D A C K dt + D eta_vp),
    p = p^ + K dt lambda_dot C,  tauII = A p + B c + eta_vp lambda_dot,
    tau = T tauII / s.
Besides the closed form: the overstress equals eta_vp times twice the
plastic strain rate read from the plastic-strain accumulator (an output the
return does not write), a vanishing eta_vp gives the perfect return, and a
large eta_vp approaches the elastic trial."""
import math

import numpy as np
import pytest

from ep_workloads import Model
from oracle.oracle import Oracle


def constants(ndim, phi, psi):
    sp, cp, ss = math.sin(math.radians(phi)), math.cos(math.radians(phi)), math.sin(math.radians(psi))
    if ndim == 2:
        return sp, cp, ss
    return (6 * sp / (math.sqrt(3) * (3 - sp)), 6 * cp / (math.sqrt(3) * (3 - sp)),
            6 * ss / (math.sqrt(3) * (3 - ss)))


def uniform(o, name):
    a = o.get(name)
    assert np.ptp(a) <= 1e-9 * max(np.abs(a).max(), 1e-6), name
    return float(a.ravel()[0])


def model(ndim, psi, eta_vp, steps=9):
    return Model(ndim=ndim, nx=7, ny=6, nz=5, dt=3e-4, tol=1e-11, n_check=10, incl_factor=1.0, psi_deg=psi,
                 eta_vp=eta_vp, steps=steps)


@pytest.mark.parametrize("ndim,psi,eta_vp", [(2, 0.0, 1e-4), (2, 10.0, 2e-4), (3, 0.0, 1e-4), (3, 8.0, 3e-4)],
                         ids=["2d", "2d-psi10", "3d", "3d-psi8"])
def test_homogeneous_increments_match_the_closed_form(ndim, psi, eta_vp):
    m = model(ndim, psi, eta_vp)
    A, B, C = constants(ndim, m.phi_deg, psi)
    K, G, dt, c = m.bulk, m.shear, m.dt, m.c0
    D = 1.0 / (G * dt)
    assert 0.3 <= D * eta_vp <= 1.0          # the overstress is a sizeable part of the stress
    o = Oracle(m)
    p0, txx0, tyy0, ep0 = 0.0, 0.0, 0.0, 0.0
    yielded = 0
    for n in range(m.steps):
        st = o.load_step()
        assert st["status"] == 0, (n, st)
        Txx, Tyy = txx0 / (G * dt) + 2.0, tyy0 / (G * dt) - 2.0
        Tzz = -(Txx + Tyy)
        s = math.sqrt(0.5 * (Txx ** 2 + Tyy ** 2 + (Tzz ** 2 if ndim == 3 else 0.0)))
        Y0 = A * p0 + B * c
        ld = 0.0
        if s / D <= Y0:
            p, tii = p0, s / D
        else:
            ld = (s - D * Y0) / (1 + D * A * C * K * dt + D * eta_vp)
            p = p0 + K * dt * ld * C
            tii = A * p + B * c + eta_vp * ld
            yielded += 1
        txx, tyy = Txx * tii / s, Tyy * tii / s
        got = uniform(o, "p"), uniform(o, "txx"), uniform(o, "tyy")
        scale = abs(txx)
        assert abs(got[0] - p) <= 1e-8 * scale, (n, got[0], p)
        assert abs(got[1] - txx) <= 1e-8 * scale, (n, got[1], txx)
        assert abs(got[2] - tyy) <= 1e-8 * scale, (n, got[2], tyy)
        # overstress = eta_vp * 2 eps_dot_p,II, the plastic strain rate from the accumulator
        ep = uniform(o, "eps_p")
        if ld > 0:
            over = tii - (A * got[0] + B * c)
            assert abs(over - eta_vp * 2.0 * (ep - ep0) / dt) <= 1e-7 * scale, (n, over, ep - ep0)
            assert over > 1e-3 * tii                # a real overstress, not rounding
            assert st["max_violation"] == pytest.approx(over, rel=1e-6)
        else:
            assert ep == ep0                        # elastic increment: no plastic strain
        p0, txx0, tyy0, ep0 = got[0], got[1], got[2], ep
    assert yielded >= 3
    o.close()


@pytest.mark.parametrize("ndim", [2, 3])
def test_vanishing_viscosity_reduces_to_the_perfect_return(ndim):
    """With D eta_vp far below rounding the regularised branch of the return
    (Lambda = lambda_dot / tauII from the consistency condition) must give
    the perfectly plastic return (Lambda = D (tauII_tr / Y - 1)) up to
    rounding, on an inclusion model over its first plastic increments."""
    m = Model(ndim=ndim, nx=17, ny=15, nz=13, dt=2e-4, tol=1e-9, n_check=10, incl_radius=0.25, steps=4)
    a, t = Oracle(m), Oracle(m.with_(eta_vp=1e-30))
    for _ in range(m.steps):
        sa, st = a.load_step(), t.load_step()
        assert sa["status"] == st["status"] == 0
    assert sa["n_yield"] > 0 and st["n_yield"] == sa["n_yield"]
    for k in ("txx", "tyy", "txy", "p", "eps_p"):
        ref = np.abs(a.get(k)).max()
        assert np.abs(t.get(k) - a.get(k)).max() <= 1e-6 * ref, k
    a.close()
    t.close()


def test_large_viscosity_approaches_the_elastic_trial():
    """With D eta_vp >> 1 the plastic rate vanishes like 1/(D eta_vp) and the
    stress tends to the elastic one: the deviation from the elastic stress
    falls by the same factor as eta_vp grows."""
    dev = []
    for eta in (1e-1, 1e0):
        m = model(2, 0.0, eta, steps=12)
        e = Oracle(m.with_(c0=1e3))                  # never yields: elastic reference
        o = Oracle(m)
        for _ in range(m.steps):
            assert o.load_step()["status"] == 0
            assert e.load_step()["status"] == 0
        assert o.get("eps_p").max() > 0
        dev.append(abs(uniform(o, "txx") - uniform(e, "txx")) / abs(uniform(e, "txx")))
        o.close()
        e.close()
    assert dev[0] < 2e-2
    assert dev[1] == pytest.approx(dev[0] / 10, rel=0.05)


@pytest.mark.parametrize("ndim,psi,eta_vp,depth", [
    (2, 0.0, 1e-4, 300.0), (2, 10.0, 0.0, 300.0), (2, 10.0, 1e-4, 300.0), (2, 10.0, 1e-4, 0.05),
    (3, 8.0, 2e-4, 300.0), (3, 8.0, 0.0, 0.05)],
    ids=["2d-psi0", "2d-psi10-perfect", "2d-psi10", "2d-psi10-crossing", "3d-psi8", "3d-psi8-perfect-crossing"])
def test_tension_beyond_the_apex_satisfies_the_return_equations(ndim, psi, eta_vp, depth):
    """Homogeneous pure shear started in tension, p^ = -(1 + depth) B c / A:
    the bound max(0, A p + B c) is zero until dilatancy lifts the pressure
    past the apex ("crossing": within the first increments).  The converged
    state of every increment must satisfy the three equations that define the
    return, with lambda_dot read from the plastic-strain accumulator:
        D tauII + lambda_dot = sqrt(J2(T)),
        tauII = max(0, A p + B c) + eta_vp lambda_dot,
        p = p^ + K dt C lambda_dot."""
    m = model(ndim, psi, eta_vp, steps=6)
    A, B, C = constants(ndim, m.phi_deg, psi)
    K, G, dt, c = m.bulk, m.shear, m.dt, m.c0
    D = 1.0 / (G * dt)
    p_start = -(1.0 + depth) * B * c / A
    o = Oracle(m)
    o.set("p", np.full(m.n_cells, p_start))
    p0, txx0, tyy0, ep0 = p_start, 0.0, 0.0, 0.0
    sides = set()
    for n in range(m.steps):
        st = o.load_step()
        assert st["status"] == 0, (n, st)
        Txx, Tyy = txx0 / (G * dt) + 2.0, tyy0 / (G * dt) - 2.0
        Tzz = -(Txx + Tyy)
        s = math.sqrt(0.5 * (Txx ** 2 + Tyy ** 2 + (Tzz ** 2 if ndim == 3 else 0.0)))
        p, txx, tyy, ep = uniform(o, "p"), uniform(o, "txx"), uniform(o, "tyy"), uniform(o, "eps_p")
        tzz = -(txx + tyy)
        tii = math.sqrt(0.5 * (txx ** 2 + tyy ** 2 + (tzz ** 2 if ndim == 3 else 0.0)))
        ld = 2.0 * (ep - ep0) / dt
        assert ld > 0.1 * s, (n, ld, s)                   # every increment yields
        assert abs(D * tii + ld - s) <= 1e-8 * s, (n, D * tii + ld, s)
        bound = max(0.0, A * p + B * c)
        assert abs(tii - bound - eta_vp * ld) <= 1e-8 * max(tii, B * c), (n, tii, bound, eta_vp * ld)
        assert abs(p - p0 - K * dt * C * ld) <= 1e-9 * abs(p_start), (n, p - p0, K * dt * C * ld)
        sides.add((A * p0 + B * c < 0, A * p + B * c > 0))
        p0, txx0, tyy0, ep0 = p, txx, tyy, ep
    if depth < 1:
        assert (True, True) in sides                      # an increment lifted p past the apex
    else:
        assert sides == {(True, False)}                   # every increment ended beyond the apex
    o.close()
