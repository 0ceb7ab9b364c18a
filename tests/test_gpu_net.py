"""GPU parity of the warm-start network kernels (through the C ABI) against the
float64 oracle of oracle/warmstart.py.

The oracle is run with bfloat16 rounding at the points where the GPU stores
bfloat16 tensors (input, weights, activations, gradients), so the remaining
differences are FP32 versus float64 accumulation (relative ~1e-6) and the
rare bfloat16 rounding flips they cause (one unit in the last place,
2^-8 relative, at isolated entries).  Bars, relative to the norm of the
reference: outputs and gradients within 2e-2 in L2 norm, and every entry of
a layer's gradient within 3e-2 of that layer's largest entry; features within
one bfloat16 unit; the Adam update to FP32 rounding.
"""
import ctypes as C

import numpy as np
import pytest

from ep_workloads import Model, random_state
from gpu_common import say
from oracle import warmstart as W

pytestmark = pytest.mark.gpu


def net(nx, ny, nz, base=16, samples=2, seed=1, scale=(1e-3, 1e-4, 1e-5, 1e-5)):
    from paper_2305_01701_amd.ep import Net
    return Net(nx, ny, nz, base=base, max_samples=samples, scale=scale, seed=seed)


def to_list(flat, base):
    out, o = [], 0
    for ci, co in W.channels(16, base, 16):
        n = co * 27 * ci
        w = flat[o:o + n].reshape(co, 27, ci).astype(np.float64)
        o += n
        out.append((w, flat[o:o + co].astype(np.float64)))
        o += co
    return out


def to_flat(params):
    return np.concatenate([np.concatenate([w.ravel(), b]) for w, b in params]).astype(np.float32)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


def random_net(n, base, seed):
    """Random weights everywhere, including a nonzero head and biases."""
    r = np.random.Generator(np.random.PCG64(seed))
    ps = to_list(n.get_params(), base)
    ps[-1] = (r.standard_normal(ps[-1][0].shape) * 0.05, r.standard_normal(16) * 0.01)
    ps = [(w, r.standard_normal(b.shape) * 0.01) for w, b in ps]
    n.set_params(to_flat(ps))
    return to_list(n.get_params(), base)


GRIDS = [(8, 8, 8), (12, 8, 16), (13, 9, 11)]


@pytest.mark.parametrize("grid", GRIDS, ids=["8^3", "12x8x16", "13x9x11"])
@pytest.mark.parametrize("base", [16, 32])
def test_forward_matches_oracle(grid, base):
    nx, ny, nz = grid
    say("net forward", grid, base)
    n = net(nx, ny, nz, base=base)
    ps = random_net(n, base, seed=2)
    r = np.random.Generator(np.random.PCG64(3))
    x = r.standard_normal(n.dims + (16,))
    n.set_sample(0, x=x)
    y = n.forward(0)
    yr, _ = W.forward(ps, x, store=W.bf16)
    err = rel(y, yr)
    say("forward rel err", err)
    assert err < 2e-2
    assert np.abs(y - yr).max() < 5e-2 * np.abs(yr).max()
    n.close()


@pytest.mark.parametrize("grid,base", [((67, 35, 29), 32), ((95, 63, 45), 16)], ids=["67x35x29-C32", "95x63x45-C16"])
def test_forward_matches_oracle_many_blocks(grid, base):
    """Volumes of many convolution blocks (16 x 4 x 4 voxels) with ragged
    x blocks at some level (68 = 4 x 16 + 4 at level 0; 24 = 16 + 8 at level
    2 of 96 x 64 x 48): every output voxel against the oracle."""
    nx, ny, nz = grid
    say("net forward", grid, base)
    n = net(nx, ny, nz, base=base)
    ps = random_net(n, base, seed=5)
    r = np.random.Generator(np.random.PCG64(6))
    x = r.standard_normal(n.dims + (16,))
    n.set_sample(0, x=x)
    y = n.forward(0)
    yr, _ = W.forward(ps, x, store=W.bf16)
    err = rel(y, yr)
    say("forward rel err", err, "max", np.abs(y - yr).max() / np.abs(yr).max())
    assert err < 2e-2
    assert np.abs(y - yr).max() < 5e-2 * np.abs(yr).max()
    n.close()


@pytest.mark.parametrize("grid", GRIDS[1:], ids=["12x8x16", "13x9x11"])
def test_gradient_matches_oracle(grid):
    nx, ny, nz = grid
    base = 16
    n = net(nx, ny, nz, base=base)
    ps = random_net(n, base, seed=4)
    r = np.random.Generator(np.random.PCG64(5))
    x = r.standard_normal(n.dims + (16,))
    t = r.standard_normal(n.dims + (4,)) * 0.1
    n.set_sample(1, x=x, t=t)
    loss, g = n.gradient(1)
    m = Model(ndim=3, nx=nx, ny=ny, nz=nz)
    zero = {k: np.zeros((nx + (k == "vx")) * (ny + (k == "vy")) * (nz + (k == "vz"))) for k in ("vx", "vy", "vz")}
    _, mask = W.targets(m, zero, 1.0)
    t16 = np.zeros(n.dims + (16,))
    t16[..., :3] = t[..., :3].astype(np.float32)
    yr, cache = W.forward(ps, x, store=W.bf16)
    lr_, gy = W.loss_grad(yr, t16, mask)
    gr = W.backward(cache, gy, store=W.bf16)
    say("loss", loss, lr_)
    assert loss == pytest.approx(lr_, rel=1e-3)
    gl = to_list(g, base)
    for l in range(W.N_LAYERS):
        ew, eb = rel(gl[l][0], gr[l][0]), rel(gl[l][1], gr[l][1])
        # element by element: the largest entry error of the layer against the
        # layer's largest entry (a wrong tap, channel or boundary voxel shows
        # here even when the layer's L2 norm hides it)
        mw = float(np.abs(gl[l][0] - gr[l][0]).max() / max(np.abs(gr[l][0]).max(), 1e-30))
        mb = float(np.abs(gl[l][1] - gr[l][1]).max() / max(np.abs(gr[l][1]).max(), 1e-30))
        say("layer", l, "dW rel", ew, "db rel", eb, "dW max", mw, "db max", mb)
        assert ew < 2e-2 and eb < 2e-2, (l, ew, eb)
        assert mw < 3e-2 and mb < 3e-2, (l, mw, mb)
    n.close()


def test_gradients_and_training_are_reproducible():
    """The parameter gradients are summed over voxel chunks and workgroups in
    a fixed order (no floating-point atomics), so they repeat bit for bit: on
    a grid of several voxel chunks per tap, two gradients of one sample agree
    exactly, and two networks trained from the same start report the same
    losses and end with the same parameters."""
    base = 16
    nets = [net(40, 24, 20, base=base, samples=1, seed=3) for _ in range(2)]
    r = np.random.Generator(np.random.PCG64(8))
    x = r.standard_normal(nets[0].dims + (16,))
    t = r.standard_normal(nets[0].dims + (4,)) * 0.1
    for n in nets:
        random_net(n, base, seed=9)
        n.set_sample(0, x=x, t=t)
    _, g0 = nets[0].gradient(0)
    _, g1 = nets[0].gradient(0)
    assert np.abs(g0).max() > 0
    assert np.array_equal(g0, g1)
    la, lb = (n.train([0], 20, lr=1e-3) for n in nets)
    assert np.array_equal(la, lb)
    assert np.array_equal(nets[0].get_params(), nets[1].get_params())
    for n in nets:
        n.close()


def test_adam_step_matches_oracle_and_training_reduces_loss():
    base = 16
    n = net(12, 8, 16, base=base)
    ps = random_net(n, base, seed=6)
    r = np.random.Generator(np.random.PCG64(7))
    n.set_sample(0, x=r.standard_normal(n.dims + (16,)), t=r.standard_normal(n.dims + (4,)) * 0.1)
    _, g = n.gradient(0)
    losses = n.train([0], 1, lr=1e-3)
    after = to_list(n.get_params(), base)
    opt = W.Adam(ps, lr=1e-3)
    ref = opt.step(ps, to_list(g, base))
    for l in range(W.N_LAYERS):
        assert np.allclose(after[l][0], ref[l][0], rtol=1e-5, atol=1e-7), l
        assert np.allclose(after[l][1], ref[l][1], rtol=1e-5, atol=1e-7), l
    more = n.train([0], 30, lr=1e-3)
    say("losses", losses[0], more[0], more[-1])
    assert more[-1] < 0.5 * losses[0]
    n.close()


def test_features_and_tracking_match_oracle():
    from paper_2305_01701_amd.ep import Solver
    m = Model(ndim=3, nx=13, ny=9, nz=11, incl_radius=0.3)
    scale = (1e-3, 1e-4, 1e-3, 1e-3)
    g = Solver(m)
    st1 = random_state(m, seed=8)
    st2 = random_state(m, seed=9)
    for k in ("vx", "vy", "vz", "p", "txx", "tyy", "txy", "txz", "tyz"):
        g.set(k, st1[k])
    eps = np.abs(random_state(m, seed=10)["p"]) * 0.1
    g.set("eps_p", eps)
    n = net(m.nx, m.ny, m.nz, scale=scale)
    n.observe(g)                                   # starts tracking (change 0)
    for k in ("vx", "vy", "vz"):
        g.set(k, st2[k])
    n.observe(g, slot=1)                           # change = st2 - st1, also the target of slot 1
    n.record(g, 0)
    x, _ = n.get_sample(0)
    _, t = n.get_sample(1)
    f = g.fields(["p", "txx", "tyy", "txy", "txz", "tyz", "eps_p"])
    dv = {k: st2[k] - st1[k] for k in ("vx", "vy", "vz")}
    xr = W.bf16(W.features(m, f, dv, scale[:3]))
    assert np.allclose(x, xr, rtol=2 ** -7, atol=1e-30)
    tr, _ = W.targets(m, dv, scale[3])
    assert np.allclose(t[..., :3], tr[..., :3], rtol=1e-6, atol=1e-9)
    n.close()
    g.close()


def test_warm_start_pipeline_converges_to_the_plain_solution():
    """The learned warm start end to end on the GPU: trajectories of two 3D
    models generate the training samples, the network trains on them, and a
    held-out model is solved from the network's guesses (accepted only when
    their physical residual is lower than that of the plain guess).  Every
    increment must converge to the tolerance and end where the plain run ends;
    the iteration counts of both runs are reported (the gain)."""
    from paper_2305_01701_amd.ep import Solver
    N, steps = 15, 8

    def model(c):
        return Model(ndim=3, nx=N, ny=N, nz=N, dt=2e-4, tol=1e-6, n_check=10, incl_radius=0.2,
                     incl_centre=c, max_iter=100000)

    train_models = [model((0.05, -0.03, 0.02)), model((-0.04, 0.06, -0.01))]
    held = model((0.02, 0.02, -0.05))
    n = net(N, N, N, base=16, samples=len(train_models) * steps, scale=(3.5e-3, 3e-2, 0.5, 0.5))
    slots = []
    for q, m in enumerate(train_models):
        s = Solver(m)
        n.reset()
        n.observe(s)
        for k in range(steps):
            n.record(s, q * steps + k)
            assert s.load_step()["status"] == 0
            n.observe(s, q * steps + k)
            slots.append(q * steps + k)
        s.close()
    losses = n.train(slots, 1600, lr=3e-4)
    first, last = losses[:len(slots)].mean(), losses[-len(slots):].mean()
    say("training loss", first, "->", last)
    assert last < 0.5 * first

    plain = Solver(held)
    warm = Solver(held)
    n.reset()
    n.observe(warm)
    it_p, it_w, used = [], [], []
    for k in range(steps):
        sp = plain.load_step()
        n.predict(warm)
        sw = warm.load_step()
        n.observe(warm)
        assert sp["status"] == 0 and sw["status"] == 0, (k, sp["status"], sw["status"])
        assert sw["resid"] <= held.tol * sw["ref"]
        it_p.append(sp["iters"])
        it_w.append(sw["iters"])
        used.append(sw["guess_used"])
    say("iterations plain", it_p, sum(it_p), "warm", it_w, sum(it_w), "guess used", used)
    names = ["vx", "vy", "vz", "p", "txx", "tyy", "txy", "txz", "tyz"]
    a, b = plain.fields(names), warm.fields(names)
    for k in names:
        err = np.abs(a[k] - b[k]).max() / max(np.abs(a[k]).max(), 1e-30)
        assert err < 1e-3, (k, err)
    n.close()


def test_inference_only_network_matches_training_network():
    """An inference-only network (max_samples = 0) with the parameters of a
    training network gives bitwise the same forward pass and the same guess;
    its training entry points are rejected."""
    from paper_2305_01701_amd.ep import Solver, EP_EINVAL, lib
    N = 15
    m = Model(ndim=3, nx=N, ny=N, nz=N, dt=2e-4, tol=1e-6, n_check=10, incl_radius=0.2,
              incl_centre=(0.05, -0.03, 0.02))
    a = net(N, N, N, base=16, samples=1, scale=(3.5e-3, 3e-2, 0.5, 0.5))
    ps = random_net(a, 16, seed=4)
    b = net(N, N, N, base=16, samples=0, scale=(3.5e-3, 3e-2, 0.5, 0.5))
    b.set_params(to_flat(ps))
    sa, sb = Solver(m), Solver(m)
    for s in (sa, sb):
        for _ in range(3):
            assert s.load_step()["status"] == 0
    for n_, s in ((a, sa), (b, sb)):
        n_.reset()
        n_.observe(s)
        n_.record(s, -1)
    ya, yb = a.forward(-1), b.forward(-1)
    assert np.array_equal(ya, yb)
    a.predict(sa)
    b.predict(sb)
    fa, fb = sa.load_step(), sb.load_step()
    assert fa["guess_used"] == fb["guess_used"] and fa["iters"] == fb["iters"] and fa["r_guess"] == fb["r_guess"]
    slots = np.zeros(1, dtype=np.int32)
    assert lib().ep_net_train(b.h, slots.ctypes.data_as(C.POINTER(C.c_int)), 1, 1, 1e-3, None) == EP_EINVAL
    for x in (a, b, sa, sb):
        x.close()
