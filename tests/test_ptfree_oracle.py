"""Pins of the oracle against the increment's equations with the pseudo-time
terms removed (paper: accelerated pseudo-transient method, where the
quasi-static solution is the attractor of the pseudo-time iteration and Re, r
only set its convergence; return mapping section).

oracle/ptfree.py writes those equations independently (numpy, vectorised,
natural array shapes) and solves them directly on tiny grids.  The pins:

- every accepted state of the oracle is a root of them: its momentum residual
  is at most tol * ref (the certificate), and its stresses are the equations'
  stresses of its velocities (2D, 3D, per-cell G, dilatancy, regularisation);
- plausible mistakes in the reading (shear points taking the largest Lambda
  of their cells, the centre using one shear point instead of the mean of
  four, the pressure sign, the pseudo-time trial in the centre J2) make the
  oracle's states fail them;
- the converged fields do not depend on the PT parameters (Courant number,
  Re, and the weight of the pseudo-time trial in the iteration's Lambda)
  beyond the tolerance, on a heterogeneous yielding increment;
- a direct nonlinear solve (MINPACK hybrid method) from the plain guess
  reaches the oracle's state;
- elastic increments are accepted from their starting state, and the
  residual carried from one increment to the next grows at most linearly.
"""
import math

import numpy as np
import pytest

from ep_workloads import Model, c1_small_2d, c3_3d, gaussian_shear
from oracle.oracle import Oracle
from oracle.ptfree import Increment, previous_state

STRESS = ["p", "txx", "tyy", "txy", "txz", "tyz", "tzz"]


def _cases():
    base2 = c1_small_2d().with_(incl_centre=(0.05, 0.03, 0.0), dt=2e-4, tol=1e-10)
    base3 = c3_3d(17).with_(ny=15, nz=13, incl_centre=(0.05, 0.03, -0.02), dt=2e-4, tol=1e-10)
    g2 = base2.with_(nx=41, ny=37, shear=1.2)
    g3 = base3.with_(shear=1.2, psi_deg=8.0, eta_vp=1e-3)
    return {
        "2d": (base2, None),
        "2d-psi-vp": (base2.with_(psi_deg=10.0, eta_vp=1e-3), None),
        "2d-G": (g2, gaussian_shear(g2, centre=(0.03, -0.02, 0.0))),
        "3d": (base3, None),
        "3d-G-psi-vp": (g3, gaussian_shear(g3, centre=(0.03, -0.02, 0.01))),
    }


CASES = _cases()


def _increment(o, m, G):
    st = previous_state(o)
    if G is not None:
        st["shear"] = G
    inc = Increment(m, st)
    v = inc.with_walls({k: o.get(k) for k in inc.shapes()})
    return inc, v


@pytest.mark.parametrize("case", list(CASES))
def test_accepted_states_solve_the_ptfree_equations(case):
    m, G = CASES[case]
    o = Oracle(m)
    if G is not None:
        o.set_shear_modulus(G)
    yielded = 0
    for _ in range(5):
        st = o.load_step()
        assert st["status"] == 0
        inc, v = _increment(o, m, G)
        r = inc.residual_max(v)
        assert r <= m.tol * st["ref"] * (1 + 1e-9), (r, st)
        assert abs(r - st["cert"]) <= 1e-6 * st["cert"] + 1e-3 * m.tol * st["ref"]
        s = inc.stresses(v)
        scale = max(np.abs(o.get(k)).max() for k in ("txx", "tyy"))
        for k in STRESS:
            if k in s and o.get(k).size:
                assert np.abs(s[k].ravel() - o.get(k)).max() <= 1e-12 * scale, k
        yielded = max(yielded, st["n_yield"])
    assert yielded > 0


def test_planted_mistakes_break_the_equations():
    m = c1_small_2d().with_(incl_centre=(0.05, 0.03, 0.0), dt=2e-4, tol=1e-10)
    o = Oracle(m)
    for _ in range(4):
        st = o.load_step()
    assert st["n_yield"] > 100
    bar = m.tol * st["ref"]
    inc, v = _increment(o, m, None)
    assert inc.residual_max(v) <= bar * (1 + 1e-9)

    # shear points take the largest Lambda of their four cells
    class MaxLambda(Increment):
        def _stress2(self, v):
            s = super()._stress2(v)
            lam = s["lam"]
            lv = np.maximum(np.maximum(lam[:-1, :-1], lam[:-1, 1:]), np.maximum(lam[1:, :-1], lam[1:, 1:]))
            mean = 0.25 * (lam[:-1, :-1] + lam[:-1, 1:] + lam[1:, :-1] + lam[1:, 1:])
            D = self.igd[0, 0] + self.imu
            txy = s["txy"]
            txy[1:-1, 1:-1] = txy[1:-1, 1:-1] * (D + mean) / (D + lv)
            return s

    # centre J2 with the shear trial of one vertex instead of the mean of four
    class OneVertex(Increment):
        def _centre(self, nS2, sh2, p_tr):
            return super()._centre(nS2, self._one, p_tr)

        def _stress2(self, v):
            dx, dy = self.h[0], self.h[1]
            vx, vy = v["vx"], v["vy"]
            ny, nx = self.c.shape
            Sxy = np.zeros((ny + 1, nx + 1))
            exy = 0.5 * ((vx[1:, 1:-1] - vx[:-1, 1:-1]) / dy + (vy[1:-1, 1:] - vy[1:-1, :-1]) / dx)
            Sxy[1:-1, 1:-1] = self.old["txy"][1:-1, 1:-1] * self.igd[0, 0] + 2.0 * exy
            self._one = Sxy[1:, 1:] ** 2
            return super()._stress2(v)

    # pressure with the wrong sign of the divergence
    class PressureSign(Increment):
        def __init__(self, *a):
            super().__init__(*a)
            self.kdt = -self.kdt

    # the yield test on the pseudo-time trial scale: the centre J2 taken as
    # that of T = tau/(G~ dtau) + S at the fixed point of an elastic update
    # (S scaled by D/Dp), against D, in place of S against Dp
    igt = 1.0 / o.scalars()["gdtau"]

    class PseudoTimeTrial(Increment):
        def _centre(self, nS2, sh2, p_tr):
            Dp = self.igd + self.imu
            f = (igt + Dp) / Dp
            lam, p, _ = super()._centre(nS2 * f * f, sh2 * f * f, p_tr)
            return lam * Dp / (igt + Dp), p, Dp

    for cls in (MaxLambda, OneVertex, PressureSign, PseudoTimeTrial):
        bad = cls(m, previous_state(o))
        r = bad.residual_max(v)
        assert r > 100.0 * bar, (cls.__name__, r, bar)


def _c1_hetero(**kw):
    return c1_small_2d().with_(incl_centre=(0.05, 0.03, 0.0), dt=2e-4, tol=1e-10, max_iter=400000, **kw)


def test_fixed_point_independent_of_pt_parameters():
    """The heterogeneous yielding increments of an off-centre inclusion (4th
    increment: 432 yielding cells) end in the same state whatever the
    Courant number and Re: independent trajectories agree to the tolerance's
    scale (measured 6e-10 at tol 1e-10), where the previous reading moved the
    fields by 3e-3."""
    names = ["vx", "vy", "p", "txx", "tyy", "txy"]
    cfl0, re0 = 0.9 / math.sqrt(2.0), 3.0 * math.sqrt(10.0) * math.pi / 2.0
    a, b = Oracle(_c1_hetero()), Oracle(_c1_hetero(cfl=0.8 * cfl0, re=1.3 * re0))
    for _ in range(4):
        sa, sb = a.load_step(), b.load_step()
        assert sa["status"] == 0 and sb["status"] == 0
    assert sa["n_yield"] > 400 and sa["n_yield"] == sb["n_yield"]
    assert sa["iters"] != sb["iters"]              # different paths ...
    sc = max(np.abs(a.get(k)).max() for k in ("p", "txx", "tyy", "txy"))
    for k in names:
        den = sc if k[0] in "pt" else np.abs(a.get(k)).max()
        assert np.abs(a.get(k) - b.get(k)).max() <= 1e-8 * den, k   # ... one state


def test_fixed_point_independent_of_the_iteration_blend():
    """Lambda of the iteration blends the physical and the pseudo-time trial;
    from a shared start the blend changes the path, not the state."""
    names = ["vx", "vy", "p", "txx", "tyy", "txy"]
    a = Oracle(_c1_hetero())
    for _ in range(3):
        a.load_step()
    keep = names + ["p_old", "txx_old", "tyy_old", "txy_old", "ux", "uy", "exx", "eyy", "exy", "eps_p"]
    start = {k: a.get(k) for k in keep}
    out = {}
    for blend in (0.0, 0.25, 0.6):
        o = Oracle(_c1_hetero(pt_blend=blend, pt_blend_late=blend))
        for k in keep:
            o.set(k, start[k])
        st = o.load_step()
        assert st["status"] == 0
        out[blend] = (st, {k: o.get(k) for k in names})
    its = {b: out[b][0]["iters"] for b in out}
    assert len(set(its.values())) == 3, its
    ref = out[0.25][1]
    sc = max(np.abs(ref[k]).max() for k in ("p", "txx", "tyy", "txy"))
    for b in (0.0, 0.6):
        for k in names:
            den = sc if k[0] in "pt" else np.abs(ref[k]).max()
            assert np.abs(out[b][1][k] - ref[k]).max() <= 1e-8 * den, (b, k)


def test_direct_solve_reaches_the_oracle_state():
    """9 x 7 cells, yielding inclusion: the equations solved directly from
    the plain guess (the previous increment's velocities) give the oracle's
    converged velocities.  Increments 2-4 and 6 (7 to 24 yielding cells);
    in the 5th the hybrid method stalls at a kink of the return (yield
    switching on and off) and is not used."""
    m = Model(ndim=2, nx=9, ny=7, tol=1e-12, n_check=10, incl_centre=(0.08, -0.05, 0.0), incl_radius=0.2,
              dt=2e-4, steps=6, max_iter=500000)
    o = Oracle(m)
    compared = 0
    for n in range(1, 7):
        v0 = {k: o.get(k) for k in ("vx", "vy")}
        st = o.load_step()
        assert st["status"] == 0
        if n not in (2, 3, 4, 6):
            continue
        assert st["n_yield"] >= 7
        inc = Increment(m, previous_state(o))
        vs, res = inc.solve(v0)
        assert inc.residual_max(inc.with_walls(vs)) <= 1e-15
        for k in vs:
            assert np.abs(vs[k] - o.get(k)).max() <= 1e-9 * np.abs(o.get(k)).max(), (n, k)
        compared += 1
    assert compared == 4


def test_elastic_increments_accept_their_starting_state():
    """Ten elastic increments at 47^3: each starting state (previous
    velocities with their physical stresses) already meets the tolerance
    and is accepted without a sweep; the residual it carries grows by about
    one rounding unit per increment (linearly), not geometrically."""
    m = c3_3d(47).with_(incl_centre=(0.05, 0.03, -0.02))
    o = Oracle(m)
    rr = []
    for _ in range(10):
        st = o.load_step()
        assert st["status"] == 0 and st["iters"] == 0 and st["n_yield"] == 0
        assert st["cert"] == st["r_ref"]
        rr.append(st["r_ref"])
    for n, r in enumerate(rr):
        assert r <= 3.0 * (n + 1) * rr[0], rr
    assert max(rr) <= 1e-4 * m.tol * st["ref"]
