"""Shared helpers of the GPU tests: run the HIP path and the oracle on the same
seeded inputs and compare field by field."""
import sys

import numpy as np

from ep_workloads import cohesion_field, random_state
from fieldtools import field_errors
from oracle.oracle import Oracle

IT2 = ["vx", "vy", "p", "txx", "tyy", "txy"]
IT3 = ["vx", "vy", "vz", "p", "txx", "tyy", "tzz", "txy", "txz", "tyz"]


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def it_names(m):
    return IT2 if m.ndim == 2 else IT3


def old_names(m):
    return [k + "_old" for k in it_names(m) if not k.startswith("v")]


def solver(m, **kw):
    from paper_2305_01701_amd.ep import Solver
    return Solver(m, cohesion_field(m), **kw)


def set_state(target, m, state, settable_tzz):
    for k, v in state.items():
        if k in ("tzz", "tzz_old") and not settable_tzz:
            continue
        target.set(k, v)


def compare(m, got, ref, names, tol, what=""):
    errs = field_errors(m, got, ref, names)
    worst = max(errs.values())
    assert worst <= tol, (what, {k: f"{v:.2e}" for k, v in errs.items()})
    return errs


def accum_names(m):
    n = ["ux", "uy", "exx", "eyy", "exy", "eps_p"]
    if m.ndim == 3:
        n += ["uz", "ezz", "exz", "eyz"]
    return n


def compare_accumulators(m, got, ref, tol, what=""):
    """Displacements share one scale, strain components another (a component
    that is zero up to rounding, e.g. the shear strain of a homogeneous pure
    shear, is measured against the strain scale, not its own noise)."""
    names = accum_names(m)
    scale = {
        "u": max(np.abs(ref[k]).max() for k in names if k.startswith("u")),
        "e": max(np.abs(ref[k]).max() for k in names if k.startswith("e") and k != "eps_p"),
    }
    for k in names:
        if k == "eps_p":
            sc = np.abs(ref[k]).max()
            if sc == 0:
                assert np.abs(got[k]).max() == 0, (what, k)
                continue
        else:
            sc = scale["u" if k.startswith("u") else "e"]
        err = np.abs(got[k] - ref[k]).max() / max(sc, 1e-300)
        assert err <= tol, (what, k, err)
