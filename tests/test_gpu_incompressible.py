"""GPU parity of the incompressible case (paper: pseudo-transient pressure
equation A2ssP2, K = +inf) against the oracle: trajectories with identical
FP64 iteration counts, fields within 1e-6 (FP64) / 1e-4 (FP32 fields)."""
import math

import pytest

from ep_workloads import Model, c1_small_2d
from gpu_common import compare, it_names, say, solver
from oracle.oracle import Oracle

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def run_both(m, prec):
    g = solver(m, precision=prec)
    o = Oracle(m)
    out = []
    for _ in range(m.steps):
        sg, so = g.load_step(), o.load_step()
        out.append((sg, so))
        if sg["status"] != 0 or so["status"] != 0:
            break
    return g, o, out


@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "fp32"])
def test_incompressible_2d_trajectory(prec):
    """Paper: incompressible pseudo-transient pressure equation (A2ssP2),
    K = +inf: trajectory parity with the oracle."""
    m = c1_small_2d().with_(n_check=10, incl_centre=(0.05, 0.03, -0.02), bulk=math.inf, steps=8)
    say("incompressible 2d trajectory, prec", prec)
    g, o, out = run_both(m, prec)
    assert any(so["n_yield"] > 0 for _, so in out)
    for n, (sg, so) in enumerate(out):
        assert sg["status"] == 0 and so["status"] == 0, (n, sg["status"], so["status"])
        if prec == FP64:
            assert sg["iters"] == so["iters"], (n, sg["iters"], so["iters"])
    tol = 1e-6 if prec == FP64 else 1e-4
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, tol)
    g.close()
    o.close()


def test_incompressible_3d_trajectory():
    m = Model(ndim=3, nx=17, ny=15, nz=13, dt=2e-4, tol=1e-8, n_check=10, incl_radius=0.25,
              incl_centre=(0.04, -0.03, 0.02), steps=5, bulk=math.inf)
    say("incompressible 3d trajectory")
    g, o, out = run_both(m, FP64)
    for n, (sg, so) in enumerate(out):
        assert sg["status"] == 0 and so["status"] == 0
        assert sg["iters"] == so["iters"]
    names = it_names(m)
    compare(m, g.fields(names), o.fields(names), names, 1e-6)
    g.close()
    o.close()
