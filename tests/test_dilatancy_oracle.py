"""Pins of the dilatant return (psi > 0) in the oracle (paper: Plasticity
section, plastic potential Q = sqrt(J2) - C p, C from the dilation angle).

A homogeneous model under pure shear (uniform cohesion, free-slip walls) has a
homogeneous solution, so every converged increment must satisfy the continuum
increment equations in closed form, solved here by hand from the previous
increment's state:
    deviator   (tau - tau^)/(G dt) + lambda_dot tau / tauII = 2 e'      (mu_s = inf)
    pressure   (p - p^)/(K dt) = -div v + lambda_dot C = lambda_dot C   (div v = 0)
    yield      tauII = A p + B c   when the trial exceeds it.
With T = tau^/(G dt) + 2 e' and s = sqrt(J2(T)) this gives
    lambda_dot = (s - (A p^ + B c)/(G dt)) / (1 + A C K / G),
    p = p^ + K dt lambda_dot C,  tauII = A p + B c,  tau = T tauII / s.
Checked in 2D (A = sin phi, C = sin psi) and 3D (the 6 sin / (sqrt3 (3 - sin))
forms) over increments that yield; psi = 0 reduces to the plain return, and the
pressure must rise under plastic flow (dilatancy against rigid walls)."""
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


def centre(o, m, name):
    a = o.get(name)
    assert np.ptp(a) <= 1e-9 * max(np.abs(a).max(), 1e-6), name     # homogeneous (stress scale ~1e-3)
    return float(a.ravel()[0])


@pytest.mark.parametrize("ndim,psi", [(2, 10.0), (2, 0.0), (3, 8.0)], ids=["2d-psi10", "2d-psi0", "3d-psi8"])
def test_homogeneous_increments_match_the_closed_form(ndim, psi):
    m = Model(ndim=ndim, nx=7, ny=6, nz=5, dt=3e-4, tol=1e-11, n_check=10, incl_factor=1.0, psi_deg=psi,
              steps=9)
    A, B, C = constants(ndim, m.phi_deg, psi)
    K, G, dt, c = m.bulk, m.shear, m.dt, m.c0
    o = Oracle(m)
    p0, txx0, tyy0 = 0.0, 0.0, 0.0
    yielded = 0
    for n in range(m.steps):
        st = o.load_step()
        assert st["status"] == 0, (n, st)
        # closed form from the previous state; pure shear e' = (1, -1, 0)
        Txx, Tyy = txx0 / (G * dt) + 2.0, tyy0 / (G * dt) - 2.0
        Tzz = -(Txx + Tyy)
        J2 = 0.5 * (Txx ** 2 + Tyy ** 2 + (Tzz ** 2 if ndim == 3 else 0.0))
        s = math.sqrt(J2)
        Y0 = A * p0 + B * c
        if s * G * dt <= Y0:
            p, sc = p0, G * dt
        else:
            ld = (s - Y0 / (G * dt)) / (1 + A * C * K / G)
            p = p0 + K * dt * ld * C
            sc = (A * p + B * c) / s
            yielded += 1
        txx, tyy = Txx * sc, Tyy * sc
        got = centre(o, m, "p"), centre(o, m, "txx"), centre(o, m, "tyy")
        scale = max(abs(txx), 1e-12)
        assert abs(got[0] - p) <= 1e-8 * scale, (n, got[0], p)
        assert abs(got[1] - txx) <= 1e-8 * scale, (n, got[1], txx)
        assert abs(got[2] - tyy) <= 1e-8 * scale, (n, got[2], tyy)
        if psi > 0 and yielded > 1:
            assert got[0] > p0 > 0 or (yielded == 1), (n, got[0], p0)    # the pressure rises under flow
        p0, txx0, tyy0 = got
    assert yielded >= 3
    o.close()
