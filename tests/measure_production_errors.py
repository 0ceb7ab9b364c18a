"""Per-field max error of the GPU increments against the FP64 oracle on the
1023 x 1023 pure-shear workload (paper: convergence study; the 2D runs of the
model configuration section), elasto-plastic and visco-plastic (Maxwell
viscosity 1e-2), FP64 and FP32 fields.

Not a test (pytest does not collect it): one oracle increment at this size
takes minutes on the host cores.  Both sides run the same increments from the
same initial state: the elastic increments of the homogeneous background
field are accepted without a sweep on both sides, so the first yielding
increment starts from the same state.  Printed per variant and precision:
status, sweeps, yielding cells, and per field max|gpu - oracle| / scale
(stresses on the common stress scale, velocities on their own), the PT-free
momentum residual of the GPU's accepted state evaluated by oracle/ptfree.py
over tol * ref, and after how many sweeps the residual histories of the two
sides first differ by 1e-9 ... 1e-1 relative.  With --control a second
oracle run, its cohesion perturbed by one part in 1e13, is compared in the
same way (the sensitivity of the increment itself).

Usage: python tests/measure_production_errors.py [--variants ep,vp] [--control] [--out FILE]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from ep_workloads import c2_2d, cohesion_field  # noqa: E402
from fieldtools import field_errors  # noqa: E402
from oracle.oracle import Oracle  # noqa: E402
from oracle.ptfree import Increment, previous_state  # noqa: E402

NAMES = ["vx", "vy", "p", "txx", "tyy", "txy"]


def log(*a):
    print(*a, flush=True)


def first_yielding(m, max_inc=12, cohesion=None):
    """Oracle increments up to and including the first one that sweeps."""
    o = Oracle(m, cohesion, progress=2000)
    o.record_history(200000)
    t0 = time.perf_counter()
    for n in range(1, max_inc + 1):
        st = o.load_step()
        log(f"oracle {m.name} increment {n}: status {st['status']} sweeps {st['iters']} "
            f"yielding {st['n_yield']} ({time.perf_counter() - t0:.0f} s)")
        if st["status"] != 0 or st["iters"] > 0:
            return o, n, st, time.perf_counter() - t0
    raise RuntimeError("no yielding increment")


def divergence(a, b, n_check):
    """Sweeps after which two residual histories first differ by more than
    1e-9, 1e-6, 1e-3 and 1e-1 relative (None: never)."""
    n = min(len(a), len(b))
    d = np.abs(a[:n] - b[:n]) / np.maximum(np.abs(b[:n]), 1e-300)
    out = {}
    for lim in (1e-9, 1e-6, 1e-3, 1e-1):
        k = np.nonzero(d > lim)[0]
        out[f"{lim:g}"] = int((k[0] + 1) * n_check) if k.size else None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--variants", default="ep,vp")
    ap.add_argument("--out", default="")
    ap.add_argument("--control", action="store_true",
                    help="also run the oracle with the cohesion perturbed by 1e-13 relative")
    a = ap.parse_args()
    from paper_2305_01701_amd import ep as E
    out = []
    for var in a.variants.split(","):
        m = c2_2d(0) if var == "ep" else c2_2d(0, visc=1e-2)
        m = m.with_(max_iter=400000)
        gpu = {}
        for prec, pname in ((E.EP_FP64, "fp64"), (E.EP_FP32_FIELDS, "fp32")):
            s = E.Solver(m, cohesion_field(m), precision=prec)
            sts = []
            while True:
                st = s.load_step()
                sts.append(st)
                if st["status"] != 0 or st["iters"] > 0 or len(sts) >= 12:
                    break
            log(f"gpu {var} {pname}: increments {len(sts)}, last: status {st['status']} sweeps {st['iters']} "
                f"(fp32 {st['iters_fp32']}) yielding {st['n_yield']} frozen_at {st['frozen_at']}")
            inc = Increment(m, previous_state(s))
            v = inc.with_walls({k: s.get(k) for k in inc.shapes()})
            ptfree = inc.residual_max(v) / (m.tol * st["ref"])
            gpu[pname] = (len(sts), st, s.fields(NAMES), ptfree, s.history()[0])
            s.close()
        o, n, so, secs = first_yielding(m)
        ref = o.fields(NAMES)
        hist_o = o.history() / so["ref"]
        rows = []
        if a.control:
            c, _, sc, _ = first_yielding(m, cohesion=cohesion_field(m) * (1.0 + 1e-13))
            hist_c = c.history() / sc["ref"]
            rows.append(("oracle-perturbed", (n, sc, c.fields(NAMES), None, hist_c)))
            c.close()
        for pname, (ng, st, f, ptfree, hist) in list(gpu.items()) + rows:
            errs = field_errors(m, f, ref, NAMES)
            row = {"variant": var, "precision": pname, "increment": n, "same_increment": ng == n,
                   "status": [st["status"], so["status"]], "sweeps": [st["iters"], so["iters"]],
                   "yielding": [st["n_yield"], so["n_yield"]], "frozen_at": [st["frozen_at"], so["frozen_at"]],
                   "max_err": {k: float(f"{v:.3e}") for k, v in errs.items()},
                   "ptfree_over_tol": None if ptfree is None else float(f"{ptfree:.3e}"),
                   "history_divergence_sweeps": divergence(hist, hist_o, so["iters"] // max(len(hist_o), 1)),
                   "history_first_checks": [[float(f"{x:.6e}") for x in hist[:8]], [float(f"{x:.6e}") for x in hist_o[:8]]],
                   "oracle_seconds": round(secs, 1)}
            log(json.dumps(row))
            out.append(row)
        o.close()
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
