"""Oracle of the learned warm start: TEST INFRASTRUCTURE ONLY.

Plain float64 numpy implementation of what the warm-start network computes,
written from the definitions (no blocking, no fusion), for the parity tests of
the GPU network kernels.  Only tests/, the smoke check and the CPU baseline of
the benchmark may import it.

The warm start (an addition to the paper's method: the paper starts every
increment from the previous velocities) predicts the velocity change of the
next load increment from the current state, so that the PT iteration starts
closer to its fixed point.  The network is a 3-level encoder-decoder of
3x3x3 'same' convolutions with zero padding:

  level 0:  a0 = relu(conv(x, W0)),  s0 = relu(conv(a0, W1))
  level 1:  a1 = relu(conv(pool(s0), W2)),  s1 = relu(conv(a1, W3))
  level 2:  a2 = relu(conv(pool(s1), W4)),  b2 = relu(conv(a2, W5))
  up 1:     r6 = relu(conv(up(b2), W6)),  c1 = r6 + s1,  d1 = relu(conv(c1, W7))
  up 0:     r8 = relu(conv(up(d1), W8)),  c0 = r8 + s0,  d0 = relu(conv(c0, W9))
  head:     y = conv(d0, W10)

with channel widths cin -> C, C -> 2C -> 4C and back, C -> cout; pool is the
2x2x2 mean, up the 2x2x2 nearest-neighbour repetition.  Tensors are (D, H, W,
channels); a convolution weight is (Cout, 27, Cin) with the 27 taps (dz, dy,
dx) in {-1, 0, 1}^3, dz slowest; conv(x, W)[v, o] = b[o] + sum over taps t and
inputs i of x[v + off_t, i] W[o, t, i] (zero outside the volume).

Training minimises the mean squared error over the valid output entries with
Adam (Kingma and Ba, "Adam: a method for stochastic optimization", 2015).

Features and targets (the solver side): channels at cell (i, j, k): the
deviatoric stresses tau_xx, tau_yy, tau_zz at the centre, tau_xy, tau_xz,
tau_yz averaged from the 4 surrounding edges, the pressure, the accumulated
plastic strain, and the previous increment's velocity change at the cell's
lower x, y, z faces; each group divided by its scale.  Output channel d at
cell (i, j, k) is the velocity change of the lower face of that cell in
direction d, divided by the output scale; wall faces keep their prescribed
values.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
N_LAYERS = 11


def channels(cin: int, base: int, cout: int):
    """(Cin, Cout) of the 11 convolutions."""
    c, c2, c4 = base, 2 * base, 4 * base
    return [(cin, c), (c, c), (c, c2), (c2, c2), (c2, c4), (c4, c4),
            (c4, c2), (c2, c2), (c2, c), (c, c), (c, cout)]


# ---------------------------------------------------------------- BF16 storage
def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64:
    the value a float32 becomes when its low 16 bits are rounded away."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


# ----------------------------------------------------------------- operators
def conv3(x, w, b=None):
    """3x3x3 correlation with zero padding; x (D, H, W, Ci), w (Co, 27, Ci)."""
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((D, H, W, w.shape[0]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :]
        y += xs @ w[:, t, :].T
    if b is not None:
        y += b
    return y


def conv3_dx(g, w):
    """Gradient of conv3 with respect to its input: dx[u, i] = sum over t, o of
    g[u - off_t, o] w[o, t, i]."""
    D, H, W, _ = g.shape
    gp = np.pad(g, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dx = np.zeros((D, H, W, w.shape[2]))
    for t, (dz, dy, dxx) in enumerate(TAPS):
        gs = gp[1 - dz:1 - dz + D, 1 - dy:1 - dy + H, 1 - dxx:1 - dxx + W, :]
        dx += gs @ w[:, t, :]
    return dx


def conv3_dw(x, g):
    """Gradients of conv3 with respect to weights and bias:
    dw[o, t, i] = sum over v of g[v, o] x[v + off_t, i], db[o] = sum of g."""
    D, H, W, ci = x.shape
    co = g.shape[3]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    g2 = g.reshape(-1, co)
    dw = np.zeros((co, 27, ci))
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :].reshape(-1, ci)
        dw[:, t, :] = g2.T @ xs
    return dw, g2.sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def pool(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def pool_dx(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=0), 2, axis=1), 2, axis=2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=0), 2, axis=1), 2, axis=2)


def up_dx(g):
    D, H, W, C = g.shape
    return g.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


# ------------------------------------------------------------------- network
def init_params(cin: int, base: int, cout: int, seed: int):
    """He-normal weights (std sqrt(2 / (27 Cin))), zero biases; the head starts
    at zero so that the untrained network predicts no change."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ps = []
    for l, (ci, co) in enumerate(channels(cin, base, cout)):
        std = 0.0 if l == N_LAYERS - 1 else np.sqrt(2.0 / (27 * ci))
        ps.append((rng.standard_normal((co, 27, ci)) * std, np.zeros(co)))
    return ps


def forward(params, x, store=None):
    """Returns (y, cache).  store: None (float64 throughout) or bf16 (every
    stored tensor -- input, weights, activations -- rounded to bfloat16, as
    the GPU stores them; the output y stays float32-exact float64)."""
    q = (lambda a: a) if store is None else store
    W = [(q(w), b) for w, b in params]
    x = q(x)
    c = {}
    c["x"] = x
    c["a0"] = q(relu(conv3(x, *W[0])))
    c["s0"] = q(relu(conv3(c["a0"], *W[1])))
    c["p0"] = q(pool(c["s0"]))
    c["a1"] = q(relu(conv3(c["p0"], *W[2])))
    c["s1"] = q(relu(conv3(c["a1"], *W[3])))
    c["p1"] = q(pool(c["s1"]))
    c["a2"] = q(relu(conv3(c["p1"], *W[4])))
    c["b2"] = q(relu(conv3(c["a2"], *W[5])))
    c["u1"] = q(up(c["b2"]))
    c["r6"] = q(relu(conv3(c["u1"], *W[6])))
    c["c1"] = q(c["r6"] + c["s1"])
    c["d1"] = q(relu(conv3(c["c1"], *W[7])))
    c["u0"] = q(up(c["d1"]))
    c["r8"] = q(relu(conv3(c["u0"], *W[8])))
    c["c0"] = q(c["r8"] + c["s0"])
    c["d0"] = q(relu(conv3(c["c0"], *W[9])))
    y = conv3(c["d0"], *W[10])
    c["W"] = W
    return y, c


def loss_grad(y, target, mask):
    """Mean squared error over the entries where mask is set, and its
    gradient with respect to y."""
    n = max(int(mask.sum()), 1)
    d = (y - target) * mask
    return float((d * d).sum() / n), 2.0 * d / n


def backward(cache, gy, store=None):
    """Parameter gradients [(dW, db)] of the network for the output gradient
    gy; with store, every stored gradient tensor is rounded like the GPU's."""
    q = (lambda a: a) if store is None else store
    W = cache["W"]
    g = [None] * N_LAYERS
    gy = q(gy)
    g[10] = conv3_dw(cache["d0"], gy)
    z9 = q(conv3_dx(gy, W[10][0]) * (cache["d0"] > 0))
    g[9] = conv3_dw(cache["c0"], z9)
    gc0 = q(conv3_dx(z9, W[9][0]))
    z8 = q(gc0 * (cache["r8"] > 0))
    g[8] = conv3_dw(cache["u0"], z8)
    gd1 = q(up_dx(q(conv3_dx(z8, W[8][0]))))
    z7 = q(gd1 * (cache["d1"] > 0))
    g[7] = conv3_dw(cache["c1"], z7)
    gc1 = q(conv3_dx(z7, W[7][0]))
    z6 = q(gc1 * (cache["r6"] > 0))
    g[6] = conv3_dw(cache["u1"], z6)
    gb2 = q(up_dx(q(conv3_dx(z6, W[6][0]))))
    z5 = q(gb2 * (cache["b2"] > 0))
    g[5] = conv3_dw(cache["a2"], z5)
    z4 = q(q(conv3_dx(z5, W[5][0])) * (cache["a2"] > 0))
    g[4] = conv3_dw(cache["p1"], z4)
    gs1 = q(gc1 + pool_dx(q(conv3_dx(z4, W[4][0]))))
    z3 = q(gs1 * (cache["s1"] > 0))
    g[3] = conv3_dw(cache["a1"], z3)
    z2 = q(q(conv3_dx(z3, W[3][0])) * (cache["a1"] > 0))
    g[2] = conv3_dw(cache["p0"], z2)
    gs0 = q(gc0 + pool_dx(q(conv3_dx(z2, W[2][0]))))
    z1 = q(gs0 * (cache["s0"] > 0))
    g[1] = conv3_dw(cache["a0"], z1)
    z0 = q(q(conv3_dx(z1, W[1][0])) * (cache["a0"] > 0))
    g[0] = conv3_dw(cache["x"], z0)
    return g


class Adam:
    """Adam on float64 master weights (Kingma and Ba, Algorithm 1)."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps, self.t = lr, b1, b2, eps, 0
        self.m = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
        self.v = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]

    def step(self, params, grads):
        self.t += 1
        out = []
        for l, ((w, b), (gw, gb)) in enumerate(zip(params, grads)):
            new = []
            for k, (p, gp) in enumerate(((w, gw), (b, gb))):
                m = self.b1 * self.m[l][k] + (1 - self.b1) * gp
                v = self.b2 * self.v[l][k] + (1 - self.b2) * gp * gp
                self.m[l] = (m, self.m[l][1]) if k == 0 else (self.m[l][0], m)
                self.v[l] = (v, self.v[l][1]) if k == 0 else (self.v[l][0], v)
                mh = m / (1 - self.b1 ** self.t)
                vh = v / (1 - self.b2 ** self.t)
                new.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
            out.append(tuple(new))
        return out


# ------------------------------------------------------- features and targets
def net_dims(m):
    """Network volume: the grid rounded up to multiples of 4 (two poolings)."""
    r4 = lambda n: (n + 3) // 4 * 4
    return r4(m.nz), r4(m.ny), r4(m.nx)


def _grid(flat, shape_xyz):
    nx_, ny_, nz_ = shape_xyz
    return np.asarray(flat, dtype=np.float64).reshape(nz_, ny_, nx_)


def features(m, f, dv_prev, scales):
    """Input tensor (D, H, W, 16) from the state of a 3D model.
    f: staggered fields by name (flat, x fastest); dv_prev: the previous
    increment's velocity change {vx, vy, vz} (flat, face shapes);
    scales: (stress, plastic strain, velocity change)."""
    nx, ny, nz = m.nx, m.ny, m.nz
    ss, se, sv = scales
    D, H, W = net_dims(m)
    x = np.zeros((D, H, W, 16))
    txx = _grid(f["txx"], (nx, ny, nz))
    tyy = _grid(f["tyy"], (nx, ny, nz))
    txy = _grid(f["txy"], (nx + 1, ny + 1, nz))
    txz = _grid(f["txz"], (nx + 1, ny, nz + 1))
    tyz = _grid(f["tyz"], (nx, ny + 1, nz + 1))
    sl = (slice(0, nz), slice(0, ny), slice(0, nx))
    x[sl + (0,)] = txx / ss
    x[sl + (1,)] = tyy / ss
    x[sl + (2,)] = -(txx + tyy) / ss
    x[sl + (3,)] = 0.25 * (txy[:, :-1, :-1] + txy[:, :-1, 1:] + txy[:, 1:, :-1] + txy[:, 1:, 1:]) / ss
    x[sl + (4,)] = 0.25 * (txz[:-1, :, :-1] + txz[:-1, :, 1:] + txz[1:, :, :-1] + txz[1:, :, 1:]) / ss
    x[sl + (5,)] = 0.25 * (tyz[:-1, :-1, :] + tyz[:-1, 1:, :] + tyz[1:, :-1, :] + tyz[1:, 1:, :]) / ss
    x[sl + (6,)] = _grid(f["p"], (nx, ny, nz)) / ss
    x[sl + (7,)] = _grid(f["eps_p"], (nx, ny, nz)) / se
    x[sl + (8,)] = _grid(dv_prev["vx"], (nx + 1, ny, nz))[:, :, :nx] / sv
    x[sl + (9,)] = _grid(dv_prev["vy"], (nx, ny + 1, nz))[:, :ny, :] / sv
    x[sl + (10,)] = _grid(dv_prev["vz"], (nx, ny, nz + 1))[:nz, :, :] / sv
    return x


def targets(m, dv, scale):
    """(target, mask), each (D, H, W, 16): velocity change of the lower face
    of every cell in channels 0..2 (interior faces only), divided by scale."""
    nx, ny, nz = m.nx, m.ny, m.nz
    D, H, W = net_dims(m)
    t = np.zeros((D, H, W, 16))
    k = np.zeros((D, H, W, 16))
    t[:nz, :ny, :nx, 0] = _grid(dv["vx"], (nx + 1, ny, nz))[:, :, :nx] / scale
    t[:nz, :ny, :nx, 1] = _grid(dv["vy"], (nx, ny + 1, nz))[:, :ny, :] / scale
    t[:nz, :ny, :nx, 2] = _grid(dv["vz"], (nx, ny, nz + 1))[:nz, :, :] / scale
    k[:nz, :ny, 1:nx, 0] = 1
    k[:nz, 1:ny, :nx, 1] = 1
    k[1:nz, :ny, :nx, 2] = 1
    return t, k


def apply_guess(m, v, y, scale):
    """Velocities of the guess: v + scale * y at interior faces; walls kept."""
    nx, ny, nz = m.nx, m.ny, m.nz
    out = {}
    vx = _grid(v["vx"], (nx + 1, ny, nz)).copy()
    vx[:, :, 1:nx] += scale * y[:nz, :ny, 1:nx, 0]
    vy = _grid(v["vy"], (nx, ny + 1, nz)).copy()
    vy[:, 1:ny, :] += scale * y[:nz, 1:ny, :nx, 1]
    vz = _grid(v["vz"], (nx, ny, nz + 1)).copy()
    vz[1:nz, :, :] += scale * y[1:nz, :ny, :nx, 2]
    out["vx"], out["vy"], out["vz"] = vx.ravel(), vy.ravel(), vz.ravel()
    return out
