"""GPU parity of the dilatant return (psi > 0; paper: Plasticity section,
plastic potential sqrt(J2) - C p) against the oracle: single sweeps from
random yielding states, trajectories with identical FP64 iteration counts,
and frozen plasticity (the pressure source of a held Lambda)."""
import numpy as np
import pytest

from ep_workloads import Model, c1_small_2d, random_state
from gpu_common import accum_names, compare, compare_accumulators, it_names, say, set_state, solver
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
def test_single_sweeps_from_yielding_states(ndim, sweep):
    m = (Model(ndim=2, nx=37, ny=29, psi_deg=12.0, c0=1e-4) if ndim == 2
         else Model(ndim=3, nx=13, ny=11, nz=9, psi_deg=9.0, c0=1e-4))
    say("dilatant single sweeps", ndim, "sweep", sweep)
    st = random_state(m, seed=31, amp_s=2e-3)
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
    g.close()
    o.close()


@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "fp32"])
def test_2d_trajectory(prec):
    m = c1_small_2d().with_(n_check=10, incl_centre=(0.05, 0.03, -0.02), psi_deg=10.0)
    say("dilatant 2d trajectory, prec", prec)
    g, o, out = run_both(m, prec)
    assert out[-1][1]["n_yield"] > 0
    for n, (sg, so) in enumerate(out):
        assert sg["status"] == 0 and so["status"] == 0, (n, sg["status"], so["status"])
        if prec == FP64:
            assert sg["iters"] == so["iters"], (n, sg["iters"], so["iters"])
            assert sg["n_yield"] == so["n_yield"], (n, sg["n_yield"], so["n_yield"])
    tol = 1e-6 if prec == FP64 else 1e-4
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, tol)
    compare_accumulators(m, g.fields(accum_names(m)), o.fields(accum_names(m)), tol)
    g.close()
    o.close()


def test_3d_trajectory():
    m = Model(ndim=3, nx=17, ny=15, nz=13, dt=2e-4, tol=1e-8, n_check=10, incl_radius=0.25,
              incl_centre=(0.04, -0.03, 0.02), steps=5, psi_deg=8.0)
    say("dilatant 3d trajectory")
    g, o, out = run_both(m, FP64)
    assert out[-1][1]["n_yield"] > 0
    for n, (sg, so) in enumerate(out):
        assert sg["status"] == 0 and so["status"] == 0
        assert sg["iters"] == so["iters"] and sg["n_yield"] == so["n_yield"]
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, 1e-6)
    g.close()
    o.close()


@pytest.mark.parametrize("sweep", [0, 2], ids=["auto", "unfused"])
def test_frozen_plasticity_2d(sweep):
    m = c1_small_2d().with_(n_check=10, incl_centre=(0.05, 0.03, -0.02), psi_deg=10.0, freeze_iter=300, steps=9)
    say("dilatant frozen 2d, sweep", sweep)
    g, o, out = run_both(m, FP64, sweep)
    assert any(so["frozen_at"] > 0 for _, so in out)
    for n, (sg, so) in enumerate(out):
        assert sg["status"] == 0 and so["status"] == 0
        assert sg["iters"] == so["iters"] and sg["frozen_at"] == so["frozen_at"], (n, sg["iters"], so["iters"])
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, 1e-6)
    g.close()
    o.close()
