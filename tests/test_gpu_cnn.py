"""GPU parity of the learned-predictor network against the float64 oracle.

Both sides use the same bfloat16-rounded weights and round activations and
matrix-instruction operands to bfloat16 at the same points; they differ in
the accumulation (float32 on the GPU, float64 in the oracle).  A float32 sum
can land on the other side of a bfloat16 rounding boundary than the float64
sum, which changes that value by one bfloat16 ulp (2^-8 relative) and
propagates.  The tolerance is measured, not guessed: the oracle is run again
with float32 accumulation in two summation orders (the input as given, and
turned by 180 degrees with turned kernels: the same network in exact
arithmetic), and the GPU must agree with the float64 oracle to within twice
the larger float32-vs-float64 distance (plus 1e-4).  Which rounding
decisions flip depends on the order, so one order alone under-estimates
the spread (for the gradient here by a factor of three).
"""

import numpy as np
import pytest
import torch

from oracle import cnn
from paper_2001_06613_amd import synth
from paper_2001_06613_amd.binding import Net

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _oracle32(fn, *args, **kw):
    cnn.ACCUM = np.float32
    try:
        return fn(*args, **kw)
    finally:
        cnn.ACCUM = np.float64


def _flip_kernels(params, dim=2):
    """3^d kernels turned by 180 degrees about every axis (tap t ->
    3^d - 1 - t); biases kept."""
    P = cnn.unpack(params, dim)
    flat = []
    for name, ci, co, k in cnn.layers(dim):
        W, b = P[name]
        flat += [(W[::-1] if k == 3 else W).ravel(), b]
    return np.concatenate(flat)


def _turn(a, dim):
    """Every spatial axis of a (B, *spatial, C) array reversed."""
    return a[(slice(None),) + (slice(None, None, -1),) * dim].copy()


def _noise(fn, params, x, *rest):
    """Spread of float32 accumulation: the largest distance from the float64
    result over two summation orders (as given, and on the frames turned by
    180 degrees about every axis with turned kernels, which computes the
    same network in exact arithmetic but sums in another order).  Returns a
    function of the float64 result and the selection slice."""
    dim = x.ndim - 2
    a = _oracle32(fn, params, x, *rest)
    xf = _turn(x, dim)
    rf = [_turn(r, dim) for r in rest]
    b = _oracle32(fn, _flip_kernels(params, dim).astype(np.float32), xf, *rf)
    if isinstance(a, tuple) and np.ndim(a[1]) == 1:       # (loss, grad)
        runs = [a[1], _flip_kernels(b[1], dim)]
    else:                                                  # (out, ...)
        runs = [a[0], _turn(b[0], dim)]
    return lambda ref, sl=slice(None): max(_rel(r[sl], ref[sl]) for r in runs)


def _batch(B, H, W, seed):
    rng = np.random.default_rng(seed)
    x = np.empty((B, 7, H, W), np.float32)
    for b in range(B):
        img = synth.base_image(rng, (H, W))
        x[b, 0:3] = img[None] * (1 + 0.05 * rng.standard_normal((3, H, W)))
        x[b, 3:7] = rng.uniform(-2, 2, (4, H, W))
    tgt = (0.3 * rng.standard_normal((B, H, W, 2))).astype(np.float32)
    return x, tgt


@pytest.mark.parametrize("B,H,W", [(2, 32, 32), (1, 64, 48), (3, 16, 24)])
def test_forward_parity(B, H, W):
    net = Net(4, (64, 64))
    params = cnn.init_params(1)
    params[-2:] = 0.05           # non-zero head bias
    net.set_params(torch.from_numpy(params))
    x, _ = _batch(B, H, W, 2)
    net.set_input(torch.from_numpy(x))
    print(f"cnn forward {B}x{H}x{W}", flush=True)
    out = net.forward().cpu().numpy()
    xn = x.transpose(0, 2, 3, 1)
    ref, _ = cnn.forward(params, xn, bf16=True)
    noise = _noise(cnn.forward, params, xn)(ref)
    print(f"gpu {_rel(out, ref):.2e}, f32-accumulation noise {noise:.2e}")
    assert _rel(out, ref) <= 2 * noise + 1e-4


def test_gradient_parity():
    B, H, W = 2, 32, 32
    net = Net(2, (32, 32))
    params = cnn.init_params(3)
    net.set_params(torch.from_numpy(params))
    x, tgt = _batch(B, H, W, 4)
    net.set_input(torch.from_numpy(x), torch.from_numpy(tgt))
    print("cnn gradient", flush=True)
    loss, g = net.gradient()
    g = g.cpu().numpy().astype(np.float64)
    xn = x.transpose(0, 2, 3, 1)
    ref_loss, ref_g = cnn.loss_and_grad(params, xn, tgt, bf16=True)
    l32, _ = _oracle32(cnn.loss_and_grad, params, xn, tgt, bf16=True)
    noise = _noise(cnn.loss_and_grad, params, xn, tgt)
    # layer by layer (weights of each layer), then the whole vector
    o = 0
    bad = []
    for name, ci, co, k in cnn.LAYERS:
        nw = k * k * co * ci
        sl = slice(o, o + nw)
        e, n = _rel(g[sl], ref_g[sl]), noise(ref_g, sl)
        print(f"{name}: gpu {e:.2e} noise {n:.2e}")
        if e > 2 * n + 1e-4:
            bad.append(name)
        o += nw + co
    print(f"all: gpu {_rel(g, ref_g):.2e} noise {noise(ref_g):.2e}")
    assert not bad, bad
    assert _rel(g, ref_g) <= 2 * noise(ref_g) + 1e-4
    assert abs(loss - ref_loss) <= 2 * abs(l32 - ref_loss) + 1e-4 * ref_loss


def test_adam_step_and_loss_decrease():
    B, H, W = 2, 32, 32
    net = Net(2, (32, 32))
    params = cnn.init_params(5)
    net.set_params(torch.from_numpy(params))
    x, _ = _batch(B, H, W, 6)
    # a learnable target: the mean of the two neighbour displacements
    tgt = (0.5 * (x[:, 3:5] + x[:, 5:7])).transpose(0, 2, 3, 1).copy()
    net.set_input(torch.from_numpy(x), torch.from_numpy(tgt))
    _, g = net.gradient()
    g = g.cpu().numpy().astype(np.float64)
    lr = 1e-3
    net.train_step(lr)
    p1 = net.get_params().cpu().numpy().astype(np.float64)
    ref, _, _ = cnn.adam(params.astype(np.float64), 0 * g, 0 * g, g, 1, lr)
    np.testing.assert_allclose(p1, ref, rtol=1e-5, atol=1e-6)
    losses = [net.train_step(lr) for _ in range(60)]
    print("losses", losses[0], losses[-1])
    assert losses[-1] < 0.5 * losses[0]


def test_assemble_and_emit():
    n, H, W = 9, 16, 32
    rng = np.random.default_rng(7)
    frames = rng.uniform(0.2, 1, (n, H, W)).astype(np.float32)
    u = rng.uniform(-3, 3, (n, 2, H, W)).astype(np.float32)
    h = 2.0
    triples = [(3, 0, 4), (5, 4, 8), (1, 0, 2)]
    net = Net(4, (32, 32))
    net.set_params(torch.from_numpy(cnn.init_params(8)))
    fd = torch.from_numpy(frames).cuda()
    ud = torch.from_numpy(u).cuda()
    net.assemble(fd, ud, h, triples, with_target=True)
    out = net.forward().cpu().numpy()
    x = np.zeros((3, 7, H, W), np.float32)
    base = np.zeros((3, 2, H, W))
    for b, (t, l, r) in enumerate(triples):
        x[b, 0], x[b, 1], x[b, 2] = frames[l], frames[t], frames[r]
        x[b, 3:5] = u[l] / h
        x[b, 5:7] = u[r] / h
        wl, wr = (r - t) / (r - l), (t - l) / (r - l)
        base[b] = wl * u[l].astype(np.float64) + wr * u[r]
    xn = x.transpose(0, 2, 3, 1)
    ref, _ = cnn.forward(cnn.init_params(8), xn)
    assert _rel(out, ref) <= 2 * _noise(cnn.forward, cnn.init_params(8),
                                        xn)(ref) + 1e-4
    unew = ud.clone()
    net.emit(h, unew)
    unew = unew.cpu().numpy()
    for b, (t, l, r) in enumerate(triples):
        expect = base[b] + h * out[b].transpose(2, 0, 1)
        np.testing.assert_allclose(unew[t], expect, rtol=1e-5, atol=1e-5)
    untouched = [k for k in range(n) if k not in (3, 5, 1)]
    np.testing.assert_array_equal(unew[untouched], u[untouched])


# ------------------------------------------------------------------- 3-D


def _batch3(B, ext, seed):
    rng = np.random.default_rng(seed)
    x = np.empty((B, 9) + ext, np.float32)
    for b in range(B):
        img = synth.base_image(rng, ext)
        x[b, 0:3] = img[None] * (1 + 0.05 * rng.standard_normal((3,) + ext))
        x[b, 3:9] = rng.uniform(-2, 2, (6,) + ext)
    tgt = (0.3 * rng.standard_normal((B,) + ext + (3,))).astype(np.float32)
    return x, tgt


@pytest.mark.parametrize("B,ext", [(1, (16, 16, 24)), (2, (8, 16, 16))])
def test_forward_parity_3d(B, ext):
    net = Net(2, (16, 16, 24), dim=3)
    params = cnn.init_params(11, dim=3)
    params[-3:] = 0.05
    net.set_params(torch.from_numpy(params))
    x, _ = _batch3(B, ext, 12)
    net.set_input(torch.from_numpy(x))
    print(f"cnn forward 3d {B}x{ext}", flush=True)
    out = net.forward().cpu().numpy()
    xn = np.moveaxis(x, 1, -1)
    ref, _ = cnn.forward(params, xn, bf16=True)
    noise = _noise(cnn.forward, params, xn)(ref)
    print(f"gpu {_rel(out, ref):.2e}, f32-accumulation noise {noise:.2e}")
    assert out.shape == ref.shape
    assert _rel(out, ref) <= 2 * noise + 1e-4


def test_gradient_parity_3d():
    ext = (8, 16, 16)
    net = Net(1, ext, dim=3)
    params = cnn.init_params(13, dim=3)
    net.set_params(torch.from_numpy(params))
    x, tgt = _batch3(1, ext, 14)
    net.set_input(torch.from_numpy(x), torch.from_numpy(tgt))
    print("cnn gradient 3d", flush=True)
    loss, g = net.gradient()
    g = g.cpu().numpy().astype(np.float64)
    xn = np.moveaxis(x, 1, -1)
    ref_loss, ref_g = cnn.loss_and_grad(params, xn, tgt, bf16=True)
    l32, _ = _oracle32(cnn.loss_and_grad, params, xn, tgt, bf16=True)
    noise = _noise(cnn.loss_and_grad, params, xn, tgt)
    o = 0
    bad = []
    for name, ci, co, k in cnn.layers(3):
        nw = k ** 3 * co * ci
        sl = slice(o, o + nw)
        e, n = _rel(g[sl], ref_g[sl]), noise(ref_g, sl)
        print(f"{name}: gpu {e:.2e} noise {n:.2e}")
        if e > 2 * n + 1e-4:
            bad.append(name)
        o += nw + co
    print(f"all: gpu {_rel(g, ref_g):.2e} noise {noise(ref_g):.2e}")
    assert not bad, bad
    assert _rel(g, ref_g) <= 2 * noise(ref_g) + 1e-4
    assert abs(loss - ref_loss) <= 2 * abs(l32 - ref_loss) + 1e-4 * ref_loss


def test_assemble_and_emit_3d():
    n, ext = 7, (8, 16, 24)
    rng = np.random.default_rng(15)
    frames = rng.uniform(0.2, 1, (n,) + ext).astype(np.float32)
    u = rng.uniform(-3, 3, (n, 3) + ext).astype(np.float32)
    h = 2.0
    triples = [(3, 0, 4), (5, 4, 6)]
    net = Net(2, ext, dim=3)
    params = cnn.init_params(16, dim=3)
    net.set_params(torch.from_numpy(params))
    fd = torch.from_numpy(frames).cuda()
    ud = torch.from_numpy(u).cuda()
    net.assemble(fd, ud, h, triples, with_target=True)
    out = net.forward().cpu().numpy()
    x = np.zeros((2, 9) + ext, np.float32)
    base = np.zeros((2, 3) + ext)
    for b, (t, l, r) in enumerate(triples):
        x[b, 0], x[b, 1], x[b, 2] = frames[l], frames[t], frames[r]
        x[b, 3:6] = u[l] / h
        x[b, 6:9] = u[r] / h
        wl, wr = (r - t) / (r - l), (t - l) / (r - l)
        base[b] = wl * u[l].astype(np.float64) + wr * u[r]
    xn = np.moveaxis(x, 1, -1)
    ref, _ = cnn.forward(params, xn)
    assert _rel(out, ref) <= 2 * _noise(cnn.forward, params, xn)(ref) + 1e-4
    unew = ud.clone()
    net.emit(h, unew)
    unew = unew.cpu().numpy()
    for b, (t, l, r) in enumerate(triples):
        expect = base[b] + h * np.moveaxis(out[b], -1, 0)
        np.testing.assert_allclose(unew[t], expect, rtol=1e-5, atol=1e-5)
    untouched = [k for k in range(n) if k not in (3, 5)]
    np.testing.assert_array_equal(unew[untouched], u[untouched])


# ------------------------------------------ workload row widths, 2-D and 3-D


def _noise_elementwise(fn, params, x, ref):
    """Largest element-wise distance of the two float32-accumulation oracle
    runs (the orders of _noise) from the float64 result."""
    dim = x.ndim - 2
    a = _oracle32(fn, params, x)[0]
    b = _turn(_oracle32(fn, _flip_kernels(params, dim).astype(np.float32),
                        _turn(x, dim))[0], dim)
    return max(float(np.max(np.abs(a - ref))), float(np.max(np.abs(b - ref))))


def _check_forward(net, params, x, label):
    net.set_params(torch.from_numpy(params))
    net.set_input(torch.from_numpy(x))
    print(f"cnn forward {label}", flush=True)
    out = net.forward().cpu().numpy()
    xn = np.moveaxis(x, 1, -1).copy()
    ref, _ = cnn.forward(params, xn, bf16=True)
    noise = _noise(cnn.forward, params, xn)(ref)
    emax = float(np.max(np.abs(out - ref)))
    nmax = _noise_elementwise(cnn.forward, params, xn, ref)
    print(f"  norm: gpu {_rel(out, ref):.2e}, noise {noise:.2e}; "
          f"element-wise: gpu {emax:.2e}, noise {nmax:.2e}, "
          f"max|ref| {np.max(np.abs(ref)):.2e}", flush=True)
    assert out.shape == ref.shape
    assert _rel(out, ref) <= 2 * noise + 1e-4
    assert emax <= 2 * nmax + 1e-4 * float(np.max(np.abs(ref)))


def test_forward_parity_full_width_image():
    # 256-pixel rows: the widest LDS halo of the 2-D convolution
    params = cnn.init_params(21)
    params[-2:] = 0.05
    x, _ = _batch(1, 256, 256, 22)
    _check_forward(Net(1, (256, 256)), params, x, "1x256x256")


def test_forward_parity_volume_slab():
    # a 16-plane slab of the 128 x 128 x 64 volume at its row and plane size
    params = cnn.init_params(23, dim=3)
    params[-3:] = 0.05
    x, _ = _batch3(1, (16, 128, 64), 24)
    _check_forward(Net(1, (16, 128, 64), dim=3), params, x, "1x16x128x64")


def test_gradient_parity_full_width():
    B, H, W = 1, 64, 256
    net = Net(1, (H, W))
    params = cnn.init_params(25)
    net.set_params(torch.from_numpy(params))
    x, tgt = _batch(B, H, W, 26)
    net.set_input(torch.from_numpy(x), torch.from_numpy(tgt))
    print("cnn gradient 1x64x256", flush=True)
    loss, g = net.gradient()
    g = g.cpu().numpy().astype(np.float64)
    xn = x.transpose(0, 2, 3, 1)
    ref_loss, ref_g = cnn.loss_and_grad(params, xn, tgt, bf16=True)
    noise = _noise(cnn.loss_and_grad, params, xn, tgt)
    o, bad = 0, []
    for name, ci, co, k in cnn.LAYERS:
        nw = k * k * co * ci
        sl = slice(o, o + nw)
        e, n = _rel(g[sl], ref_g[sl]), noise(ref_g, sl)
        print(f"{name}: gpu {e:.2e} noise {n:.2e}")
        if e > 2 * n + 1e-4:
            bad.append(name)
        o += nw + co
    assert not bad, bad
    assert _rel(g, ref_g) <= 2 * noise(ref_g) + 1e-4
