"""Pin of the incompressible pressure equation (paper: pseudo-transient
pressure equation A2ssP2, the K -> infinity limit of A2ssP) in the oracle.

The oracle takes K = +inf as the incompressible case (1/(K dt) = 0 in the
pressure update; readings for the residual and the physical evaluation).  Its
converged states must be the limit of the compressible ones: over three
increments of a small yielding 2D model (up to the point where the increment
stops having a unique solution), the gap to the K = +inf state falls by
the factor by which K grows (O(1/K)), down to 1e-4 of the field scales at
K = 1e4 — a dropped pressure term or a wrong sign would leave an O(1) gap or a
different rate."""
import math

import numpy as np

from ep_workloads import Model
from oracle.oracle import Oracle

NAMES = ["vx", "vy", "p", "txx", "tyy", "txy"]


def run(m):
    o = Oracle(m)
    st = [o.load_step() for _ in range(m.steps)]
    f = o.fields(NAMES)
    o.close()
    return st, f


def gaps(ref, got):
    sc = max(np.abs(ref[k]).max() for k in ("p", "txx", "tyy", "txy"))
    return {k: np.abs(got[k] - ref[k]).max() / (sc if k[0] in "pt" else np.abs(ref[k]).max()) for k in ref}


def test_incompressible_state_is_the_stiff_limit():
    # three increments: the inclusion yields in the second; in the fourth the
    # plastic zone reaches the walls and the increment has more than one
    # solution, so states of different K no longer compare (one branch each)
    base = Model(ndim=2, nx=31, ny=31, tol=1e-9, n_check=10, incl_centre=(0.05, 0.03, 0.0), incl_radius=0.15,
                 dt=2e-4, steps=3)
    st, ref = run(base.with_(bulk=math.inf))
    assert all(s["status"] == 0 for s in st)
    assert st[-1]["n_yield"] > 0
    g3 = gaps(ref, run(base.with_(bulk=1e3))[1])
    g4 = gaps(ref, run(base.with_(bulk=1e4))[1])
    for k in NAMES:
        assert g4[k] < 2e-4, (k, g4[k])
        assert 8.0 < g3[k] / g4[k] < 12.5, (k, g3[k], g4[k])
