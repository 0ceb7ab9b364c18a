"""Pins of the warm-start network oracle (CPU): the convolution and its two
gradients against PyTorch's CPU conv3d and autograd (library routines, float64),
adjoint identities of pooling and upsampling, the whole network's parameter
gradient against central finite differences, bfloat16 rounding against
PyTorch's conversion, the first Adam step in closed form, and the feature /
target / guess maps on states with known answers."""
import numpy as np
import pytest
import torch

from ep_workloads import Model, field_shapes, random_state
from oracle import warmstart as W


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def torch_weight(w):
    co, _, ci = w.shape
    return torch.from_numpy(w.reshape(co, 3, 3, 3, ci).transpose(0, 4, 1, 2, 3).copy())


def test_tap_order_is_z_slowest():
    assert W.TAPS[0] == (-1, -1, -1) and W.TAPS[1] == (-1, -1, 0) and W.TAPS[13] == (0, 0, 0)
    assert W.TAPS[26] == (1, 1, 1) and W.TAPS[3] == (-1, 0, -1)


def test_conv_and_gradients_match_torch():
    r = rng(1)
    x = r.standard_normal((5, 6, 7, 3))
    w = r.standard_normal((4, 27, 3))
    b = r.standard_normal(4)
    g = r.standard_normal((5, 6, 7, 4))
    xt = torch.from_numpy(x.transpose(3, 0, 1, 2)[None].copy()).requires_grad_(True)
    wt = torch_weight(w).requires_grad_(True)
    bt = torch.from_numpy(b).requires_grad_(True)
    yt = torch.nn.functional.conv3d(xt, wt, bt, padding=1)
    y = W.conv3(x, w, b)
    assert np.allclose(y, yt[0].detach().numpy().transpose(1, 2, 3, 0), rtol=1e-12, atol=1e-12)
    yt.backward(torch.from_numpy(g.transpose(3, 0, 1, 2)[None].copy()))
    dx = W.conv3_dx(g, w)
    dw, db = W.conv3_dw(x, g)
    assert np.allclose(dx, xt.grad[0].numpy().transpose(1, 2, 3, 0), rtol=1e-12, atol=1e-12)
    dwt = wt.grad.numpy().transpose(0, 2, 3, 4, 1).reshape(4, 27, 3)
    assert np.allclose(dw, dwt, rtol=1e-12, atol=1e-12)
    assert np.allclose(db, bt.grad.numpy(), rtol=1e-12)


def test_pool_and_up_adjoints():
    r = rng(2)
    a = r.standard_normal((2, 3, 4, 5))
    b = r.standard_normal((4, 6, 8, 5))
    assert np.isclose((W.up(a) * b).sum(), (a * W.up_dx(b)).sum())
    assert np.isclose((W.pool(b) * a).sum(), (b * W.pool_dx(a)).sum())
    assert np.allclose(W.pool(W.up(a)), a)


def small_net(seed=3, base=4):
    params = W.init_params(16, base, 16, seed)
    r = rng(seed + 1)
    # a nonzero head so that every layer receives gradient
    params[-1] = (r.standard_normal(params[-1][0].shape) * 0.1, r.standard_normal(16) * 0.1)
    x = r.standard_normal((8, 8, 8, 16))
    t = r.standard_normal((8, 8, 8, 16))
    mask = (r.random((8, 8, 8, 16)) < 0.5).astype(float)
    return params, x, t, mask


def net_loss(params, x, t, mask):
    y, _ = W.forward(params, x)
    return W.loss_grad(y, t, mask)[0]


def test_network_gradient_matches_finite_differences():
    params, x, t, mask = small_net()
    y, cache = W.forward(params, x)
    _, gy = W.loss_grad(y, t, mask)
    grads = W.backward(cache, gy)
    r = rng(7)
    for l in range(W.N_LAYERS):
        w, b = params[l]
        for _ in range(3):
            idx = tuple(r.integers(0, s) for s in w.shape)
            h = 1e-6
            wp, wm = w.copy(), w.copy()
            wp[idx] += h
            wm[idx] -= h
            pp = list(params); pp[l] = (wp, b)
            pm = list(params); pm[l] = (wm, b)
            fd = (net_loss(pp, x, t, mask) - net_loss(pm, x, t, mask)) / (2 * h)
            assert grads[l][0][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9), (l, idx)
        o = int(r.integers(0, b.shape[0]))
        bp, bm = b.copy(), b.copy()
        bp[o] += 1e-6
        bm[o] -= 1e-6
        pp = list(params); pp[l] = (w, bp)
        pm = list(params); pm[l] = (w, bm)
        fd = (net_loss(pp, x, t, mask) - net_loss(pm, x, t, mask)) / 2e-6
        assert grads[l][1][o] == pytest.approx(fd, rel=1e-5, abs=1e-9), (l, "bias")


def test_planted_gradient_mistake_is_detected():
    """A dropped skip-connection gradient (a plausible slip) breaks the
    finite-difference agreement of the first layers."""
    params, x, t, mask = small_net()
    y, cache = W.forward(params, x)
    _, gy = W.loss_grad(y, t, mask)
    cache_bad = dict(cache)
    good = W.backward(cache, gy)
    cache_bad["s0"] = np.zeros_like(cache["s0"])      # kills the level-0 relu mask
    bad = W.backward(cache_bad, gy)
    assert not np.allclose(good[1][0], bad[1][0])


def test_bf16_rounding_matches_torch():
    r = rng(4)
    x = np.concatenate([r.standard_normal(1000) * 10.0 ** r.integers(-20, 20, 1000),
                        [1 + 2 ** -8, 1 + 2 ** -8 + 2 ** -20, 1 + 3 * 2 ** -8, -0.0, 0.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(W.bf16(x), ref)
    assert W.bf16(np.array([1 + 2 ** -8]))[0] == 1.0              # tie to even
    assert W.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6  # tie to even (up)


def test_first_adam_step_closed_form():
    params = [(np.array([[[1.0, -2.0]]]), np.array([0.5]))]
    grads = [(np.array([[[0.3, -4.0]]]), np.array([1e-3]))]
    opt = W.Adam(params, lr=0.01)
    new = opt.step(params, grads)
    # m^ = g, v^ = g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(new[0][0], [[[1.0 - 0.01 * 0.3 / (0.3 + 1e-8), -2.0 + 0.01 * 4.0 / (4.0 + 1e-8)]]])
    assert np.allclose(new[0][1], [0.5 - 0.01 * 1e-3 / (1e-3 + 1e-8)])


def test_features_of_homogeneous_pure_shear():
    m = Model(ndim=3, nx=6, ny=5, nz=7)
    sh = field_shapes(m)
    tau, p = 3e-4, -1e-4
    f = {k: np.zeros(int(np.prod(s))) for k, s in sh.items()}
    f["txx"][:] = tau
    f["tyy"][:] = -tau
    f["p"][:] = p
    f["eps_p"] = np.full(m.nx * m.ny * m.nz, 2e-5)
    dv = {k: np.full(int(np.prod(sh[k])), 1e-6) for k in ("vx", "vy", "vz")}
    x = W.features(m, f, dv, (1e-3, 1e-4, 1e-6))
    assert x.shape == (8, 8, 8, 16)
    inside = x[:7, :5, :6]
    assert np.allclose(inside[..., 0], 0.3) and np.allclose(inside[..., 1], -0.3)
    assert np.allclose(inside[..., 2], 0.0) and np.allclose(inside[..., 3:6], 0.0)
    assert np.allclose(inside[..., 6], -0.1) and np.allclose(inside[..., 7], 0.2)
    assert np.allclose(inside[..., 8:11], 1.0) and np.allclose(inside[..., 11:], 0.0)
    assert np.all(x[7:] == 0) and np.all(x[:, 5:] == 0) and np.all(x[:, :, 6:] == 0)


def test_guess_from_exact_targets_reproduces_the_new_velocities():
    m = Model(ndim=3, nx=6, ny=5, nz=7)
    old = random_state(m, seed=5)
    new = random_state(m, seed=6)
    sh = field_shapes(m)
    for k in ("vx", "vy", "vz"):            # walls are prescribed: equal in both
        a_old = old[k].reshape(sh[k][::-1])
        a_new = new[k].reshape(sh[k][::-1])
        ax = {"vx": 2, "vy": 1, "vz": 0}[k]
        for idx in (0, -1):
            sl = [slice(None)] * 3
            sl[ax] = idx
            a_new[tuple(sl)] = a_old[tuple(sl)]
    dv = {k: new[k] - old[k] for k in ("vx", "vy", "vz")}
    t, mask = W.targets(m, dv, 1e-3)
    g = W.apply_guess(m, {k: old[k] for k in ("vx", "vy", "vz")}, t, 1e-3)
    for k in ("vx", "vy", "vz"):
        assert np.allclose(g[k], new[k], rtol=0, atol=1e-15), k
    assert mask[..., 3:].sum() == 0
    assert mask[..., 0].sum() == (m.nx - 1) * m.ny * m.nz
