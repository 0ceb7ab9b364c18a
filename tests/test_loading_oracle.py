"""Pin of a loading schedule (background strain rate changed between
increments) in the oracle: homogeneous elastic pure shear accumulates
tau_xx = sum over increments of 2 G dt a_n exactly (div v = 0, no plastic
flow), p stays 0, and the velocities are the background field of the last
rate."""
import numpy as np

from ep_workloads import Model
from oracle.oracle import Oracle


def test_elastic_increments_follow_the_rate_schedule():
    m = Model(ndim=2, nx=8, ny=7, dt=1e-4, tol=1e-11, n_check=10, incl_factor=1.0, c0=1.0, steps=6)
    o = Oracle(m)
    a, total = 1.0, 0.0
    for n in range(m.steps):
        o.set_strain_rate((a, -a, 0.0))
        st = o.load_step()
        assert st["status"] == 0
        total += 2.0 * m.shear * m.dt * a
        txx = o.get("txx")
        assert np.allclose(txx, total, rtol=1e-9, atol=0), (n, txx[0], total)
        assert np.allclose(o.get("tyy"), -total, rtol=1e-9, atol=0)
        assert np.abs(o.get("p")).max() <= 1e-12 * total
        a *= 1.01
    # velocities: the background field of the last rate, v_x = a x on x-faces
    last = a / 1.01
    xn = -m.lx / 2 + (m.lx / m.nx) * np.arange(m.nx + 1)
    vx = o.get("vx").reshape(m.ny, m.nx + 1)
    assert np.allclose(vx, last * xn[None, :], rtol=1e-9, atol=1e-15)
    o.close()
