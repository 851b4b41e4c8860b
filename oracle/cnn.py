"""Plain float64 reference of the learned temporal predictor network.

Test infrastructure only (see ``oracle/__init__.py``).

The paper predicts the transformations of frames left out of K_q by linear
interpolation (Sec. 3) or by the least-squares problem eq. (2).  The learned
predictor replaces that guess by the linear interpolation plus a correction
computed by a small convolutional encoder-decoder from the neighbouring
frames and their registered displacements.  The network is not in the paper;
the definition here is the one the HIP kernels implement, for images (d = 2)
and volumes (d = 3):

* input (3 + 2d channels): frame_l, frame_t, frame_r, u_l / h, u_r / h
  (displacements in pixels of the level), channels last;
* encoder: 2 convolutions per level (3^d taps, zero padding, ReLU) with 32,
  64, 128, 128 channels; 2^d average pooling between levels;
* decoder: nearest 2x upsampling, concatenation [skip, upsampled], 2
  convolutions per level (128, 64, 32 channels);
* head: 1x1 convolution to d channels (the correction in level pixels).

Parameters are one float32 vector, layer by layer in the order of
``layers(d)``, each layer W[tap][c_out][c_in] followed by b[c_out]; the tap
index runs over the offsets -1..1 of every axis in row-major order (tap =
3 dy + dx in 2-D, 9 dz + 3 dy + dx in 3-D).

Precision points mirror the GPU path: weights and activations are rounded
to bfloat16 (round to nearest even) where the GPU stores them in bfloat16,
sums are exact (float64 here); the head output is not rounded.  With
``bf16=False`` every rounding is skipped (used by the finite-difference pin).
``ACCUM`` selects the accumulation type of the convolutions: float64 by
default; the parity tests also run float32 once to measure how far a
float32 accumulation moves the bfloat16 roundings (their noise floor).
"""

import numpy as np


def layers(dim=2):
    """(name, c_in, c_out, kernel size) of the network for d = dim."""
    return [
        ("e1a", 3 + 2 * dim, 32, 3), ("e1b", 32, 32, 3),
        ("e2a", 32, 64, 3), ("e2b", 64, 64, 3),
        ("e3a", 64, 128, 3), ("e3b", 128, 128, 3),
        ("e4a", 128, 128, 3), ("e4b", 128, 128, 3),
        ("d3a", 256, 128, 3), ("d3b", 128, 128, 3),
        ("d2a", 192, 64, 3), ("d2b", 64, 64, 3),
        ("d1a", 96, 32, 3), ("d1b", 32, 32, 3),
        ("head", 32, dim, 1),
    ]


LAYERS = layers(2)


def param_count(dim=2):
    return sum(k ** dim * ci * co + co for _, ci, co, k in layers(dim))


def unpack(params, dim=2):
    """Flat vector -> {name: (W[taps][co][ci], b[co])} in float64."""
    params = np.asarray(params, dtype=np.float64)
    out = {}
    o = 0
    for name, ci, co, k in layers(dim):
        nw = k ** dim * co * ci
        W = params[o:o + nw].reshape(k ** dim, co, ci)
        o += nw
        b = params[o:o + co]
        o += co
        out[name] = (W, b)
    assert o == params.size
    return out


def to_bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, bf16):
    return to_bf16(x) if bf16 else np.asarray(x, dtype=np.float64)


ACCUM = np.float64


def _taps(k, d):
    """Offsets of every tap (each axis 0..k-1, i.e. -k//2..k//2 shifted) in
    row-major tap order."""
    return list(np.ndindex(*((k,) * d)))


def conv(x, W, b, k):
    """Zero-padded convolution (cross-correlation), channels last.

    x: (B, *spatial, ci) with d spatial axes; W: (k^d, co, ci); b: (co,).
    y[p, co] = b[co] + sum_tap sum_ci x[p + off(tap), ci] W[tap, co, ci].
    """
    d = x.ndim - 2
    sp = x.shape[1:-1]
    co = W.shape[1]
    y = (np.zeros(x.shape[:-1] + (co,)) + b).astype(ACCUM)
    r = k // 2
    xp = np.pad(x, ((0, 0),) + ((r, r),) * d + ((0, 0),)).astype(ACCUM)
    Wa = W.astype(ACCUM)
    for tap, off in enumerate(_taps(k, d)):
        sl = tuple(slice(o, o + n) for o, n in zip(off, sp))
        xs = xp[(slice(None),) + sl]
        y += np.tensordot(xs, Wa[tap], axes=([d + 1], [1])).astype(ACCUM)
    return y.astype(np.float64)


def conv_backward(x, W, k, dy):
    """Gradients of conv wrt x, W and b for upstream gradient dy."""
    d = x.ndim - 2
    sp = x.shape[1:-1]
    r = k // 2
    xp = np.pad(x, ((0, 0),) + ((r, r),) * d + ((0, 0),)).astype(ACCUM)
    dya = dy.astype(ACCUM)
    Wa = W.astype(ACCUM)
    dxp = np.zeros_like(xp)
    dW = np.zeros(W.shape, dtype=ACCUM)
    axes = list(range(d + 1))
    for tap, off in enumerate(_taps(k, d)):
        sl = (slice(None),) + tuple(slice(o, o + n) for o, n in zip(off, sp))
        xs = xp[sl]
        dW[tap] = np.tensordot(dya, xs, axes=(axes, axes))
        dxp[sl] += np.tensordot(dya, Wa[tap], axes=([d + 1], [0]))
    dx = dxp[(slice(None),) + tuple(slice(r, r + n) for n in sp)]
    db = dya.sum(axis=tuple(axes))
    return (dx.astype(np.float64), dW.astype(np.float64),
            db.astype(np.float64))


def _blocks(x):
    """(B, *spatial, C) -> (B, s0/2, 2, s1/2, 2, ..., C) and the axes of
    the 2-blocks."""
    d = x.ndim - 2
    shape = [x.shape[0]]
    for n in x.shape[1:-1]:
        shape += [n // 2, 2]
    shape.append(x.shape[-1])
    return x.reshape(shape), tuple(2 + 2 * a for a in range(d))


def pool(x):
    xb, ax = _blocks(x)
    return xb.mean(axis=ax)


def up(x):
    for a in range(1, x.ndim - 1):
        x = np.repeat(x, 2, axis=a)
    return x


def pool_backward(dy):
    return up(dy) / float(2 ** (dy.ndim - 2))


def up_backward(dy):
    yb, ax = _blocks(dy)
    return yb.sum(axis=ax)


def forward(params, x, bf16=True):
    """Network output (B, *spatial, d) and the rounded parameters."""
    d = x.ndim - 2
    lay = layers(d)
    P = unpack(params, d)
    if bf16:
        P = {n: (to_bf16(W), b) for n, (W, b) in P.items()}
    act = {"in": _r(x, bf16)}

    def cr(name, inp):
        W, b = P[name]
        k = dict((l[0], l[3]) for l in lay)[name]
        return _r(np.maximum(conv(inp, W, b, k), 0.0), bf16)

    e1 = cr("e1b", cr("e1a", act["in"]))
    p1 = _r(pool(e1), bf16)
    e2 = cr("e2b", cr("e2a", p1))
    p2 = _r(pool(e2), bf16)
    e3 = cr("e3b", cr("e3a", p2))
    p3 = _r(pool(e3), bf16)
    e4 = cr("e4b", cr("e4a", p3))
    c3 = np.concatenate([e3, up(e4)], axis=-1)
    d3 = cr("d3b", cr("d3a", c3))
    c2 = np.concatenate([e2, up(d3)], axis=-1)
    d2 = cr("d2b", cr("d2a", c2))
    c1 = np.concatenate([e1, up(d2)], axis=-1)
    d1 = cr("d1b", cr("d1a", c1))
    W, b = P["head"]
    out = conv(d1, W, b, 1)
    return out, P


def loss_and_grad(params, x, target, bf16=True):
    """Mean squared error over (B, *spatial, d) and its gradient wrt params.

    The backward pass rounds every upstream gradient to bfloat16 where the
    GPU feeds it to a bfloat16 matrix instruction.
    """
    d = x.ndim - 2
    lay = layers(d)
    P = unpack(params, d)
    if bf16:
        P = {n: (to_bf16(W), b) for n, (W, b) in P.items()}
    ks = dict((l[0], l[3]) for l in lay)
    acts = {}

    def cr(name, inp):
        W, b = P[name]
        acts[name] = inp
        y = _r(np.maximum(conv(inp, W, b, ks[name]), 0.0), bf16)
        acts[name + ":out"] = y
        return y

    xin = _r(x, bf16)
    e1 = cr("e1b", cr("e1a", xin))
    p1 = _r(pool(e1), bf16)
    e2 = cr("e2b", cr("e2a", p1))
    p2 = _r(pool(e2), bf16)
    e3 = cr("e3b", cr("e3a", p2))
    p3 = _r(pool(e3), bf16)
    e4 = cr("e4b", cr("e4a", p3))
    c3 = np.concatenate([e3, up(e4)], axis=-1)
    d3 = cr("d3b", cr("d3a", c3))
    c2 = np.concatenate([e2, up(d3)], axis=-1)
    d2 = cr("d2b", cr("d2a", c2))
    c1 = np.concatenate([e1, up(d2)], axis=-1)
    d1 = cr("d1b", cr("d1a", c1))
    Wh, bh = P["head"]
    out = conv(d1, Wh, bh, 1)
    diff = out - target
    loss = float(np.mean(diff * diff))
    dout = 2.0 * diff / diff.size

    grads = {}

    def back(name, dpost):
        """Through ReLU and conv `name`; returns the gradient of its input."""
        y = acts[name + ":out"]
        dpre = _r(dpost * (y > 0), bf16)
        dx, dW, db = conv_backward(acts[name], P[name][0], ks[name], dpre)
        grads[name] = (dW, db)
        return dx

    dxh, dWh, dbh = conv_backward(d1, Wh, 1, _r(dout, bf16))
    grads["head"] = (dWh, dbh)
    dc1 = back("d1a", back("d1b", dxh))
    de1 = dc1[..., :32]
    dd2 = up_backward(dc1[..., 32:])
    dc2 = back("d2a", back("d2b", dd2))
    de2 = dc2[..., :64]
    dd3 = up_backward(dc2[..., 64:])
    dc3 = back("d3a", back("d3b", dd3))
    de3 = dc3[..., :128]
    de4 = up_backward(dc3[..., 128:])
    dp3 = back("e4a", back("e4b", de4))
    de3 = de3 + pool_backward(dp3)
    dp2 = back("e3a", back("e3b", de3))
    de2 = de2 + pool_backward(dp2)
    dp1 = back("e2a", back("e2b", de2))
    de1 = de1 + pool_backward(dp1)
    back("e1a", back("e1b", de1))

    flat = []
    for name, ci, co, k in lay:
        dW, db = grads[name]
        flat.append(dW.ravel())
        flat.append(db.ravel())
    return loss, np.concatenate(flat)


def init_params(seed, dim=2):
    """He-normal weights, zero biases, float32 (the GPU uses the same)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for name, ci, co, k in layers(dim):
        std = np.sqrt(2.0 / (k ** dim * ci))
        if name == "head":
            std *= 0.1
        out.append(rng.standard_normal(k ** dim * co * ci) * std)
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def adam(params, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), float64; returns (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
