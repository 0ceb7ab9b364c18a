"""Helpers for comparing staggered fields (test infrastructure)."""
import numpy as np

# parity of each field under x -> -x, y -> -y, z -> -z
_SIGN = {
    "vx": (-1, 1, 1), "vy": (1, -1, 1), "vz": (1, 1, -1),
    "p": (1, 1, 1), "txx": (1, 1, 1), "tyy": (1, 1, 1), "tzz": (1, 1, 1),
    "txy": (-1, -1, 1), "txz": (-1, 1, -1), "tyz": (1, -1, -1),
}


def shapes(m):
    nx, ny, nz = m.nx, m.ny, m.nz
    if m.ndim == 2:   # numpy order (y, x)
        return {"vx": (ny, nx + 1), "vy": (ny + 1, nx), "p": (ny, nx), "txx": (ny, nx),
                "tyy": (ny, nx), "txy": (ny + 1, nx + 1)}
    return {"vx": (nz, ny, nx + 1), "vy": (nz, ny + 1, nx), "vz": (nz + 1, ny, nx),
            "p": (nz, ny, nx), "txx": (nz, ny, nx), "tyy": (nz, ny, nx), "tzz": (nz, ny, nx),
            "txy": (nz, ny + 1, nx + 1), "txz": (nz + 1, ny, nx + 1), "tyz": (nz + 1, ny + 1, nx)}


def mirror(m, f, axes):
    """Reflect fields about the domain centre along the given axes (0=x,1=y,2=z)."""
    sh = shapes(m)
    out = {}
    for k, v in f.items():
        base = k[:-4] if k.endswith("_old") else k
        if base not in sh:
            continue
        a = np.asarray(v).reshape(sh[base])
        s = 1
        for ax in axes:
            a = np.flip(a, axis=a.ndim - 1 - ax)
            s *= _SIGN[base][ax]
        out[k] = (s * a).ravel().copy()
    return out


def rel_err(a, b, scale=None):
    a = np.asarray(a); b = np.asarray(b)
    sc = scale if scale is not None else max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / sc)


def field_errors(m, got, ref, names):
    """Per-field max|got-ref| / max|ref|; stresses share the deviator scale so
    that near-zero fields (p under pure shear) are judged on the stress scale."""
    sscale = max(np.abs(ref[k]).max() for k in names if k[0] in "pt")
    out = {}
    for k in names:
        sc = sscale if k[0] in "pt" else max(np.abs(ref[k]).max(), 1e-300)
        out[k] = rel_err(got[k], ref[k], sc)
    return out
