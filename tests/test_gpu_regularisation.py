"""GPU parity of the consistency-regularised return (eta_vp > 0: a yielding
point carries tauII = A p + B c + eta_vp lambda_dot, the visco-plastic strain
rate of the constitutive section) against the oracle: single sweeps from
random yielding states (alone and with dilatancy), trajectories with identical
FP64 iteration counts, frozen plasticity, and a batch of models with
different viscosities (equal to the single-model solver bit for bit)."""
import numpy as np
import pytest

from ep_workloads import Model, c1_small_2d, random_state
from gpu_common import IT2, accum_names, compare, compare_accumulators, it_names, say, set_state, solver
from oracle.oracle import Oracle

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def run_both(m, prec, sweep=0):
    g = solver(m, precision=prec, sweep=sweep)
    o = Oracle(m)
    out = []
    for _ in range(m.steps):
        sg, so = g.load_step(), o.load_step()
        out.append((sg, so))
        if sg["status"] != 0 or so["status"] != 0:
            break
    return g, o, out


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("sweep", [1, 2], ids=["fused", "unfused"])
@pytest.mark.parametrize("psi", [0.0, 10.0], ids=["psi0", "psi10"])
def test_single_sweeps_from_yielding_states(ndim, sweep, psi):
    """eta_vp = 5e-5 against D ~ 1e4 (1/(G dt) plus the pseudo-time term):
    the overstress is of the order of the bound."""
    m = (Model(ndim=2, nx=37, ny=29, psi_deg=psi, c0=1e-4, eta_vp=5e-5) if ndim == 2
         else Model(ndim=3, nx=13, ny=11, nz=9, psi_deg=psi, c0=1e-4, eta_vp=5e-5))
    say("regularised single sweeps", ndim, "sweep", sweep, "psi", psi)
    st = random_state(m, seed=37, amp_s=2e-3)
    g = solver(m, sweep=sweep)
    o = Oracle(m)
    set_state(g, m, st, settable_tzz=False)
    set_state(o, m, st, settable_tzz=True)
    for n in (1, 4):
        g.sweep(n)
        for _ in range(n):
            o.sweep()
        names = it_names(m)
        compare(m, g.fields(names), o.fields(names), names, 1e-11, f"{n} sweeps")
    # the regularisation changes the sweep (a test that compared plain sweeps would pass too)
    p = Oracle(m.with_(eta_vp=0.0))
    set_state(p, m, st, settable_tzz=True)
    for _ in range(5):
        p.sweep()
    assert np.abs(p.get("txx") - o.get("txx")).max() > 1e-3 * np.abs(o.get("txx")).max()
    g.close()
    o.close()
    p.close()


@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "fp32"])
def test_2d_trajectory(prec):
    m = c1_small_2d().with_(n_check=10, incl_centre=(0.05, 0.03, -0.02), eta_vp=5e-5)
    say("regularised 2d trajectory, prec", prec)
    g, o, out = run_both(m, prec)
    assert out[-1][1]["n_yield"] > 0
    assert out[-1][1]["max_violation"] > 0                  # overstress above the bound
    for n, (sg, so) in enumerate(out):
        assert sg["status"] == 0 and so["status"] == 0, (n, sg["status"], so["status"])
        if prec == FP64:
            assert sg["iters"] == so["iters"], (n, sg["iters"], so["iters"])
            assert sg["n_yield"] == so["n_yield"], (n, sg["n_yield"], so["n_yield"])
            assert sg["max_violation"] == pytest.approx(so["max_violation"], rel=1e-6, abs=1e-12)
    tol = 1e-6 if prec == FP64 else 1e-4
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, tol)
    compare_accumulators(m, g.fields(accum_names(m)), o.fields(accum_names(m)), tol)
    g.close()
    o.close()


def test_3d_trajectory():
    m = Model(ndim=3, nx=17, ny=15, nz=13, dt=2e-4, tol=1e-8, n_check=10, incl_radius=0.25,
              incl_centre=(0.04, -0.03, 0.02), steps=5, eta_vp=5e-5, psi_deg=6.0)
    say("regularised 3d trajectory")
    g, o, out = run_both(m, FP64)
    assert out[-1][1]["n_yield"] > 0
    for n, (sg, so) in enumerate(out):
        assert sg["status"] == 0 and so["status"] == 0
        assert sg["iters"] == so["iters"] and sg["n_yield"] == so["n_yield"], (n, sg["iters"], so["iters"])
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, 1e-6)
    compare_accumulators(m, g.fields(accum_names(m)), o.fields(accum_names(m)), 1e-6)
    g.close()
    o.close()


@pytest.mark.parametrize("sweep", [0, 2], ids=["auto", "unfused"])
def test_frozen_plasticity_2d(sweep):
    m = c1_small_2d().with_(n_check=10, incl_centre=(0.05, 0.03, -0.02), eta_vp=5e-5, freeze_iter=200, steps=9)
    say("regularised frozen 2d, sweep", sweep)
    g, o, out = run_both(m, FP64, sweep)
    assert any(so["frozen_at"] > 0 for _, so in out)
    for n, (sg, so) in enumerate(out):
        assert sg["status"] == 0 and so["status"] == 0
        assert sg["iters"] == so["iters"] and sg["frozen_at"] == so["frozen_at"], (n, sg["iters"], so["iters"])
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, 1e-6)
    g.close()
    o.close()


def test_batch_of_different_viscosities():
    """Per-model eta_vp and psi in one batch: each model equals the
    single-model solver bit for bit and the oracle to the FP64 bar."""
    from test_gpu_batch import iters_agree, run_batch, run_single
    steps = 5
    base = dict(ndim=2, dt=2e-4, tol=1e-8, n_check=10, steps=steps)
    models = [
        Model(nx=37, ny=29, lx=1.3, phi_deg=25.0, incl_radius=0.2, incl_centre=(0.07, -0.04, 0), eta_vp=2e-5,
              **base),
        Model(nx=23, ny=23, phi_deg=20.0, c0=2.5e-3, incl_radius=0.25, incl_centre=(-0.04, -0.02, 0), **base),
        Model(nx=31, ny=45, ly=1.4, incl_radius=0.12, incl_centre=(0.03, 0.06, 0), eta_vp=1e-4, psi_deg=8.0,
              **base),
    ]
    say("regularised batch")
    b, out, _ = run_batch(models, FP64, steps)
    for i, m in enumerate(models):
        g, sg = run_single(m, FP64, steps)
        view = b.model(i)
        for n in range(steps):
            assert out[n][i]["status"] == 0, (i, n)
            assert out[n][i]["iters"] == sg[n]["iters"], (i, n)
        for k in IT2 + accum_names(m):
            assert np.array_equal(view.get(k), g.get(k)), (i, k)
        g.close()
        o = Oracle(m)
        so, hist = [], []
        for _ in range(steps):
            o.record_history()
            so.append(o.load_step())
            hist.append(o.history() / so[-1]["ref"])
        assert so[-1]["n_yield"] > 0, i
        for n in range(steps):
            assert so[n]["status"] == 0, (i, n)
            assert iters_agree(out[n][i]["iters"], so[n]["iters"], hist[n], m), (i, n)
        compare(m, view.fields(IT2), o.fields(IT2), IT2, 1e-6, f"model {i}")
        compare_accumulators(m, view.fields(accum_names(m)), o.fields(accum_names(m)), 1e-6, f"model {i}")
        o.close()
    b.close()


@pytest.mark.parametrize("ndim,psi,eta_vp,depth,prec", [
    (2, 10.0, 1e-4, 0.05, FP64), (2, 10.0, 0.0, 300.0, FP64), (2, 10.0, 1e-4, 0.05, FP32),
    (3, 8.0, 2e-4, 300.0, FP64), (3, 8.0, 0.0, 0.05, FP64)],
    ids=["2d-crossing", "2d-perfect-deep", "2d-crossing-fp32", "3d-deep", "3d-perfect-crossing"])
def test_tension_beyond_the_apex(ndim, psi, eta_vp, depth, prec):
    """Homogeneous pure shear started in tension, p^ = -(1 + depth) B c / A:
    the return's apex piece (bound max(0, A p + B c) = 0), and with a small
    depth the dilatant crossing of the apex."""
    import math
    m = Model(ndim=ndim, nx=7, ny=6, nz=5, dt=3e-4, tol=1e-11 if prec == FP64 else 1e-6, n_check=10,
              incl_factor=1.0, psi_deg=psi, eta_vp=eta_vp, steps=6)
    sp, cp = math.sin(math.radians(m.phi_deg)), math.cos(math.radians(m.phi_deg))
    A, B = (sp, cp) if ndim == 2 else (6 * sp / (math.sqrt(3) * (3 - sp)), 6 * cp / (math.sqrt(3) * (3 - sp)))
    p_start = np.full(m.n_cells, -(1.0 + depth) * B * m.c0 / A)
    say("tension beyond the apex", ndim, psi, eta_vp, depth, "prec", prec)
    g = solver(m, precision=prec)
    o = Oracle(m)
    g.set("p", p_start)
    o.set("p", p_start)
    for n in range(m.steps):
        sg, so = g.load_step(), o.load_step()
        assert sg["status"] == 0 and so["status"] == 0, (n, sg, so)
        assert sg["n_yield"] == so["n_yield"] == m.n_cells, n
    tol = 1e-6 if prec == FP64 else 1e-4
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, tol)
    compare_accumulators(m, g.fields(accum_names(m)), o.fields(accum_names(m)), tol)
    g.close()
    o.close()
