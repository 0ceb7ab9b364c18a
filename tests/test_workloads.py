"""Seeded input generators: the heterogeneous cohesion and the symmetry
study's start (inputs only; they hold none of the solver's arithmetic)."""
import numpy as np

from ep_workloads import Model, e2_symmetry, gaussian_cohesion, pressure_anomaly


def test_gaussian_cohesion_end_values_and_shape():
    m = Model(ndim=2, nx=63, ny=63, c0=2e-3)
    c = gaussian_cohesion(m).reshape(m.ny, m.nx)
    assert c[31, 31] == m.c0                                  # lowest at the centre
    assert c.max() == 2 * m.c0 and np.all(c[:, :3] == 2 * m.c0)   # the wall band
    inner = c[4:-4, 4:-4]
    assert inner.max() < 1.2 * m.c0 and inner.max() > 1.15 * m.c0
    row = c[31, 4:32]
    assert np.all(np.diff(row) <= 0)                          # rises towards the walls
    assert np.allclose(c, c[::-1, ::-1], rtol=1e-14, atol=0) and np.allclose(c, c[:, ::-1], rtol=1e-14, atol=0)
    shifted = gaussian_cohesion(m, centre=(0.1, 0.0, 0.0)).reshape(m.ny, m.nx)
    assert shifted.argmin() % m.nx > 31
    m3 = Model(ndim=3, nx=15, ny=13, nz=11, c0=2e-3)
    c3 = gaussian_cohesion(m3)
    assert c3.size == m3.n_cells and c3.min() >= m3.c0 and c3.max() == 2 * m3.c0


def test_symmetry_study_start():
    m = e2_symmetry(7)
    assert (m.nx, m.ny, m.lx, m.ly) == (383, 191, 2.0, 1.0)
    assert abs(m.dt * 7 - 2e-3) < 1e-15 and m.visc == 1e6
    p = pressure_anomaly(m, 0.5 * m.c0, 0.1).reshape(m.ny, m.nx)
    assert set(np.unique(p)) == {0.0, 1e-3}
    assert np.array_equal(p, p[:, ::-1]) and np.array_equal(p, p[::-1, :])
