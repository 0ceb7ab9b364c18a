"""Pins of the oracle on the symmetry study's setup (section "Symmetry versus
non-symmetry"): 2D pure shear of a 2:1 domain, uniform cohesion, a central
pressure anomaly p = c/2, elastic limit.

The setup is invariant under the x-mirror (x -> -x, vx -> -vx), and so are
the equations; a discretisation that is not (a shifted index, a one-sided
average) breaks the pins below.  Once the model yields, the symmetric state
is unstable and rounding-level asymmetry grows into a single shear band, so
the solution is one of two mirror-image branches.  Perturbing the anomaly by
+/-1e-12 c on one side selects the branch: the two runs must be exact mirror
images (same iteration counts and stress integrals), each band must be
symmetric under the point reflection (x, y) -> (-x, -y), which the
perturbation does not break, and before the first yield the state must stay
x-mirror symmetric."""
import numpy as np

from ep_workloads import e2_symmetry, pressure_anomaly
from oracle.oracle import Oracle


def run(m, sign):
    p = pressure_anomaly(m, 0.5 * m.c0, 0.1).reshape(m.ny, m.nx)
    xc = -0.5 * m.lx + (np.arange(m.nx) + 0.5) * (m.lx / m.nx)
    yc = -0.5 * m.ly + (np.arange(m.ny) + 0.5) * (m.ly / m.ny)
    X, Y = np.meshgrid(xc, yc)
    p = p + sign * 1e-12 * m.c0 * ((X > 0) & (np.abs(Y) < 0.05))
    o = Oracle(m)
    o.set("p", np.ascontiguousarray(p.ravel()))
    st, eps = [], []
    for _ in range(m.steps):
        st.append(o.load_step())
        eps.append(o.get("eps_p").reshape(m.ny, m.nx).copy())
    vx = o.get("vx").reshape(m.ny, m.nx + 1)
    o.close()
    return st, eps, vx


def test_branches_are_mirror_images():
    # constant blend of the iteration's return: with the late blend the
    # bifurcating increment maps the +-perturbation to the branches
    # non-monotonically in its size (measured), so that a rounding-level
    # perturbation no longer decides the branch; the pin is about the
    # equations' mirror equivariance, which the blend does not touch
    m = e2_symmetry(7, nx=95, ny=47, tol=1e-10).with_(pt_blend_late=0.25)
    sa, ea, va = run(m, +1.0)
    sb, eb, vb = run(m, -1.0)
    assert all(s["status"] == 0 for s in sa + sb)
    first = next(n for n, s in enumerate(sa) if s["n_yield"] > 0)
    top = ea[-1].max()
    assert top > 0
    # symmetric until the model yields (the perturbation is at rounding level)
    for n in range(first):
        assert ea[n].max() == 0.0
    # a single band, not the symmetric pattern: far from x-mirror symmetric ...
    assert np.abs(ea[-1] - ea[-1][:, ::-1]).max() > 0.5 * top
    # ... but symmetric under the point reflection
    assert np.abs(ea[-1] - ea[-1][::-1, ::-1]).max() <= 1e-9 * top
    # the two branches are x-mirror images of each other
    # (iteration counts equal up to one check: the mirror images differ by
    # rounding, which can move an acceptance at the tolerance by one check)
    assert all(abs(x["iters"] - y["iters"]) <= m.n_check for x, y in zip(sa, sb))
    for x, y in zip(sa, sb):
        assert abs(x["sxx_centre"] - y["sxx_centre"]) <= 1e-9 * abs(x["sxx_centre"])
        assert x["n_yield"] == y["n_yield"]
    assert np.abs(ea[-1] - eb[-1][:, ::-1]).max() <= 1e-9 * top
    vtop = np.abs(va).max()
    assert np.abs(va + vb[:, ::-1]).max() <= 1e-9 * vtop          # vx is odd under the x-mirror
