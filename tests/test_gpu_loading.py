"""GPU parity of a loading schedule (ep_set_strain_rate between increments;
velocity increments of 1 % per load step) against the oracle, FP64 and FP32
fields (whose velocities are stored relative to the background field of
the current rate)."""
import pytest

from ep_workloads import c1_small_2d, Model
from gpu_common import accum_names, compare, compare_accumulators, it_names, say, solver
from oracle.oracle import Oracle

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_trajectory_with_rate_schedule(prec, ndim):
    # 2D: the matrix localises in the 8th increment, where the perfectly plastic
    # increment has a near-flat set of solutions (the iteration drifts on a
    # residual plateau of 2e-5 of the reference); frozen plasticity after
    # 16 nx iterations (the accelerated-PT section's remedy) makes it linear
    m = (c1_small_2d().with_(n_check=10, incl_centre=(0.05, 0.03, -0.02), freeze_iter=16 * 63) if ndim == 2 else
         Model(ndim=3, nx=17, ny=15, nz=13, dt=2e-4, tol=1e-8, n_check=10, incl_radius=0.25,
               incl_centre=(0.04, -0.03, 0.02), steps=5))
    say("rate schedule, ndim", ndim, "prec", prec)
    g, o = solver(m, precision=prec), Oracle(m)
    a = 1.0
    for n in range(m.steps):
        rate = (a, -a, 0.0)
        g.set_strain_rate(rate)
        o.set_strain_rate(rate)
        sg, so = g.load_step(), o.load_step()
        assert sg["status"] == 0 and so["status"] == 0, (n, sg["status"], so["status"])
        if prec == FP64:
            assert sg["iters"] == so["iters"], (n, sg["iters"], so["iters"])
        a *= 1.01
    tol = 1e-6 if prec == FP64 else 1e-4
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, tol)
    compare_accumulators(m, g.fields(accum_names(m)), o.fields(accum_names(m)), tol)
    g.close()
    o.close()
