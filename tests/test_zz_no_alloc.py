"""GPU check of the allocation-free residual entry point (ep_residual_noalloc)
through the C ABI: on the same state it must return exactly what ep_residual
returns (same kernels; only the counters, argument tables and tile list live
in the library's static device array), on two calls in a row, the second
with a smaller model; and it must reject a 2D model whose tile list does not
fit the array, leaving no trace."""
import pytest

from ep_workloads import Model, random_state
from gpu_common import say, set_state, solver

pytestmark = pytest.mark.gpu

KEYS = ["resid", "momentum", "physical", "vmax", "continuity", "eps_rel"]


def ep():
    from paper_2305_01701_amd import ep as E
    return E


def both(m, seed):
    E = ep()
    g = solver(m)
    set_state(g, m, random_state(m, seed=seed, amp_v=2e-3, amp_s=1.2e-3), settable_tzz=False)
    rc0, na = E.ep_residual_noalloc(g.h)       # first: nothing of this model staged yet
    rc1, ref = E.ep_residual(g.h)
    rc2, na2 = E.ep_residual_noalloc(g.h)      # again, after ep_residual
    assert rc0 == 0 and rc1 == 0 and rc2 == 0, (rc0, rc1, rc2)
    g.close()
    return na, ref, na2


@pytest.mark.parametrize("pair", [
    (Model(ndim=2, nx=130, ny=67, incl_centre=(0.1, -0.05, 0)), Model(ndim=2, nx=37, ny=29, lx=1.3)),
    (Model(ndim=3, nx=70, ny=33, nz=17, incl_radius=0.25), Model(ndim=3, nx=13, ny=11, nz=9, lz=0.8)),
], ids=["2d", "3d"])
def test_noalloc_residual_equals_residual(pair):
    """Two calls in a row, the second with a smaller model: bit for bit the
    values of ep_residual (the array keeps the previous call's contents, so
    the second call also shows that everything is cleared or rewritten)."""
    for q, m in enumerate(pair):
        say("noalloc residual", m.ndim, m.nx, m.ny, m.nz)
        na, ref, na2 = both(m, seed=5 + q)
        for k in KEYS:
            assert na[k] == ref[k], (q, k, na[k], ref[k])
            assert na2[k] == ref[k], (q, k, na2[k], ref[k])
        assert ref["physical"] > 0 and ref["continuity"] > 0


def test_noalloc_rejects_models_beyond_the_array():
    """8192 tiles of 64 x 16 cells (2048 x 4096) exceed the 8000 the array holds:
    EP_EINVAL with a message naming the limit; a model that fits still works
    afterwards."""
    E = ep()
    m = Model(ndim=2, nx=2048, ny=4096, ly=2.0)
    say("noalloc rejection", m.nx, m.ny)
    g = solver(m)
    rc, _ = E.ep_residual_noalloc(g.h)
    msg = E.lib().ep_last_error(g.h).decode()
    g.close()
    assert rc == E.EP_EINVAL and "scratch capacity" in msg, (rc, msg)
    small = Model(ndim=2, nx=37, ny=29, lx=1.3)
    na, ref, _ = both(small, seed=9)
    assert all(na[k] == ref[k] for k in KEYS)
