"""The C-ABI library loads and exports every symbol include/ep.h declares;
pure host functions (version, workspace sizing, parameter validation) behave
as documented.  No device work: runs without a GPU."""
import ctypes as C
import math
import os
import re

import pytest

from ep_workloads import c1_small_2d, c3_3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def E():
    from paper_2305_01701_amd import ep
    if not os.path.exists(ep.LIB_PATH):
        from paper_2305_01701_amd import build
        build.build()
    return ep


def declared_functions():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ep_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_binding_symbols(E):
    assert declared_functions() == sorted(E.SYMBOLS)


def test_library_exports_every_declared_symbol(E):
    L = E.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_abi_version(E):
    assert E.ep_abi_version() == 3


def test_workspace_size_scales_with_grid_and_precision(E):
    m = c1_small_2d()
    b64 = E.ep_workspace_size(E.params_from_model(m))
    b32 = E.ep_workspace_size(E.params_from_model(m, precision=E.EP_FP32_FIELDS))
    assert b32 > b64 > 0 and b64 % 256 == 0
    big = E.ep_workspace_size(E.params_from_model(c3_3d()))
    # 3D 255^3 FP64: at least the 25 algorithmic arrays (ping-pong counted twice)
    assert big > 25 * 255 ** 3 * 8


@pytest.mark.parametrize("change", [
    dict(psi_deg=-1.0), dict(psi_deg=35.0), dict(nx=2), dict(bulk=0.0), dict(shear=-1.0), dict(dt=0.0), dict(tol=0.0),
    dict(cfl=0.75), dict(ndim=4), dict(max_iter=0), dict(visc=0.0), dict(freeze_iter=-1), dict(objective=2),
    dict(eta_vp=-1e-3), dict(eta_vp=float("inf")), dict(eta_vp=float("nan")), dict(pt_blend=-0.1), dict(pt_blend=1.5),
])
def test_invalid_parameters_rejected(E, change):
    m = c1_small_2d().with_(**change)
    p = E.params_from_model(m)
    n = C.c_size_t(0)
    assert E.lib().ep_workspace_size(C.byref(p), C.byref(n)) == E.EP_EINVAL


def test_init_rejects_small_workspace_without_touching_device(E):
    m = c1_small_2d()
    p = E.params_from_model(m)
    need = E.ep_workspace_size(p)
    rc, h = E.ep_init(p, None, 0, need, 0)            # NULL workspace
    assert rc == E.EP_ENOMEM and not h.value
    rc, h = E.ep_init(p, None, 256, need - 256, 0)    # too small: rejected before any use
    assert rc == E.EP_ENOMEM and not h.value


def test_last_error_without_handle(E):
    assert E.lib().ep_last_error(None) == b"no handle"


def _batch_rc(E, models, precisions=None):
    ps = [E.params_from_model(m, precision=(precisions[i] if precisions else E.EP_FP32_FIELDS))
          for i, m in enumerate(models)]
    n = C.c_size_t(0)
    return E.lib().ep_batch_workspace_size(len(ps), E._params_array(ps), C.byref(n)), n.value


def test_batch_workspace_is_sum_of_models_plus_tables(E):
    from ep_workloads import c4_batch
    models = c4_batch(0, n_models=8)
    rc, total = _batch_rc(E, models)
    assert rc == E.EP_OK
    singles = sum(E.ep_workspace_size(E.params_from_model(m, precision=E.EP_FP32_FIELDS)) for m in models)
    assert singles < total < singles + 64 * 2 ** 20


@pytest.mark.parametrize("case", ["3d", "odd_check", "mixed_precision", "empty", "bad_model"])
def test_batch_rejects_invalid_sets(E, case):
    a, b = c1_small_2d(), c1_small_2d().with_(nx=40)
    precs = None
    if case == "3d":
        models = [a, c3_3d(7)]
    elif case == "odd_check":
        models = [a.with_(n_check=11), b.with_(n_check=11)]
    elif case == "mixed_precision":
        models, precs = [a, b], [E.EP_FP64, E.EP_FP32_FIELDS]
    elif case == "empty":
        n = C.c_size_t(0)
        assert E.lib().ep_batch_workspace_size(0, None, C.byref(n)) == E.EP_EINVAL
        return
    else:
        models = [a, b.with_(psi_deg=45.0)]          # psi > phi
    assert _batch_rc(E, models, precs)[0] == E.EP_EINVAL


def test_batch_init_rejects_small_workspace(E):
    models = [c1_small_2d(), c1_small_2d().with_(nx=40)]
    ps = [E.params_from_model(m) for m in models]
    need = E.ep_batch_workspace_size(ps)
    rc, b = E.ep_batch_init(ps, [None, None], 256, need - 256, 0)
    assert rc == E.EP_ENOMEM and not b.value
    assert E.lib().ep_batch_last_error(None) == b"no batch"


@pytest.mark.parametrize("case", ["3d", "unfused"])
def test_freeze_accepted_in_every_sweep_form(E, case):
    m = (c3_3d(7) if case == "3d" else c1_small_2d()).with_(freeze_iter=100)
    p = E.params_from_model(m, sweep=E.EP_SWEEP_UNFUSED if case == "unfused" else E.EP_SWEEP_AUTO)
    n = C.c_size_t(0)
    assert E.lib().ep_workspace_size(C.byref(p), C.byref(n)) == E.EP_OK


def _net_config(E, n, samples, base=32):
    c = E.ep_net_config()
    c.nx = c.ny = c.nz = n
    c.base, c.max_samples, c.seed = base, samples, 0
    for q, v in enumerate((1e-3, 1e-4, 1e-5, 1e-5)):
        c.scale[q] = v
    return c


def test_inference_only_network_needs_less_workspace(E):
    """max_samples = 0 holds no sample slots and no activation gradients:
    at 511^3 about half the workspace of a one-sample training network;
    negative counts are rejected."""
    L = E.lib()
    sizes = {}
    for s in (0, 1, 2):
        b = C.c_size_t(0)
        assert L.ep_net_workspace_size(C.byref(_net_config(E, 511, s)), C.byref(b)) == E.EP_OK
        sizes[s] = b.value
    assert sizes[0] < 0.55 * sizes[1] and sizes[1] < sizes[2]
    b = C.c_size_t(0)
    assert L.ep_net_workspace_size(C.byref(_net_config(E, 31, -1)), C.byref(b)) == E.EP_EINVAL


def test_init_rejects_out_of_range_shear_before_device_work(E):
    """A per-cell shear modulus outside (0, shear] fails at ep_init before the
    workspace (here a dummy address) is touched."""
    import numpy as np
    m = c1_small_2d()
    p = E.params_from_model(m)
    need = E.ep_workspace_size(p)
    for bad in (0.0, -1.0, 2.0 * m.shear, float("nan")):
        g = np.full(m.nx * m.ny, m.shear)
        g[17] = bad
        rc, h = E.ep_init(p, None, 256, need, 0, shear=g)
        assert rc == E.EP_EINVAL and not h.value, bad
