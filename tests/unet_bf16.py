"""The U-Net of the learned warm start in float32 with BF16 rounding where
the GPU kernels store BF16: a model of the kernels' number format, for
element-wise comparison (test helper, not the oracle; the FP64 oracle in
oracle/unet.py remains the reference of the network's mathematics).

Rounding points (round to nearest even, as the kernels' converter):
  forward   the first convolution in float32 from the float32 input and
            float32 weights; every other convolution from BF16 inputs and
            BF16 weights, float32 sums plus the float32 bias; each layer's
            ReLU output stored as BF16; pooling averages BF16 values in
            float32 and stores BF16; upsampling and concatenation copy;
            the 1x1 head sums BF16 features with float32 weights.
  backward  the output gradient 2 (out - t) / V in float32; the head's
            input gradient gout * w stored as BF16; per layer the ReLU
            mask of the BF16 output, the weight gradient summed in float32
            from BF16 operands (the first layer's from the float32 input),
            the input gradient summed in float32 from BF16 operands and
            stored as BF16; the upsampling gradient (sum of 8 children) and
            the skip-plus-pooling gradient (skip + coarse / 8) stored as
            BF16.
Summation order differs from the matrix cores', so values that sit on a
BF16 rounding boundary may round the other way: the comparison is to a
few BF16 units, not bit for bit.
"""
import numpy as np

from oracle import unet as U


def bf(x):
    """Round float32 values to BF16 (nearest even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    u = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return u.view(np.float32)


def _shift(x, dz, dy, dx):
    return U.shift(x, dz, dy, dx)


def _conv(x, W, b):
    """float32 convolution: W (co, 27, ci), x (D, H, W, ci)."""
    out = np.broadcast_to(b.astype(np.float32), x.shape[:3] + (W.shape[0],)).copy()
    for t, (dz, dy, dx) in enumerate(U.TAPS):
        out += _shift(x, dz, dy, dx) @ W[:, t, :].T
    return out


def _conv_back(x, W, g):
    dW = np.zeros(W.shape, np.float32)
    gx = np.zeros(x.shape, np.float32)
    for t, (dz, dy, dx) in enumerate(U.TAPS):
        s = _shift(x, dz, dy, dx).reshape(-1, x.shape[-1])
        dW[:, t, :] = g.reshape(-1, g.shape[-1]).T @ s
        gx += _shift(g @ W[:, t, :], -dz, -dy, -dx)
    return gx, dW, g.sum(axis=(0, 1, 2), dtype=np.float32)


def _pool(x):
    D, H, W, C = x.shape
    s = x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5), dtype=np.float32)
    return bf(s * np.float32(0.125))


def _up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def _up_back(g):
    D, H, W, C = g.shape
    return bf(g.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5), dtype=np.float32))


def forward(params, x):
    P = {k: v.astype(np.float32) for k, v in U.unpack(params).items()}
    x = np.asarray(x, np.float32)
    cache = {"x": x}

    def layer(name, inp, first=False):
        W = P[(name, "W")] if first else bf(P[(name, "W")])
        y = bf(np.maximum(_conv(inp, W, P[(name, "b")]), np.float32(0.0)))
        cache[name] = (inp, y, W)
        return y

    e0 = layer("e0b", layer("e0a", x, first=True))
    e1 = layer("e1b", layer("e1a", _pool(e0)))
    e2 = layer("e2b", layer("e2a", _pool(e1)))
    bt = layer("bb", layer("ba", _pool(e2)))
    d2 = layer("d2b", layer("d2a", np.concatenate([_up(bt), e2], -1)))
    d1 = layer("d1b", layer("d1a", np.concatenate([_up(d2), e1], -1)))
    d0 = layer("d0b", layer("d0a", np.concatenate([_up(d1), e0], -1)))
    cache["d0"] = d0
    out = d0 @ P[("head", "W")] + P[("head", "b")][0]
    return out.astype(np.float32), cache


def backward(params, cache, g_out):
    P = {k: v.astype(np.float32) for k, v in U.unpack(params).items()}
    g_out = np.asarray(g_out, np.float32)
    grads = {}

    def layer_back(name, gy, want_gx=True):
        inp, y, W = cache[name]
        gpre = np.where(y > 0, gy, np.float32(0.0)).astype(np.float32)
        gx, dW, db = _conv_back(inp, W, gpre)
        grads[(name, "W")] = dW
        grads[(name, "b")] = db
        return bf(gx) if want_gx else None

    d0 = cache["d0"]
    grads[("head", "W")] = np.einsum("zyx,zyxc->c", g_out, d0)
    grads[("head", "b")] = np.array([g_out.sum(dtype=np.float32)], np.float32)
    g = bf(g_out[..., None] * P[("head", "W")])
    gc = layer_back("d0a", layer_back("d0b", g))
    g_e0 = gc[..., 32:]
    gc = layer_back("d1a", layer_back("d1b", _up_back(gc[..., :32])))
    g_e1 = gc[..., 64:]
    gc = layer_back("d2a", layer_back("d2b", _up_back(gc[..., :64])))
    g_e2 = gc[..., 128:]
    g = layer_back("ba", layer_back("bb", _up_back(gc[..., :128])))
    g = layer_back("e2a", layer_back("e2b", bf(g_e2 + _up(g) * np.float32(0.125))))
    g = layer_back("e1a", layer_back("e1b", bf(g_e1 + _up(g) * np.float32(0.125))))
    layer_back("e0a", layer_back("e0b", bf(g_e0 + _up(g) * np.float32(0.125))), want_gx=False)
    lay, n = U.param_layout()
    vec = np.zeros(n, np.float32)
    for name, kind, off, shape in lay:
        vec[off:off + int(np.prod(shape))] = grads[(name, kind)].reshape(-1)
    return vec


def loss_and_grad(params, x, target):
    out, cache = forward(params, x)
    diff = (out - np.asarray(target, np.float32)).astype(np.float32)
    loss = float(np.mean(diff.astype(np.float64) ** 2))
    g_out = (np.float32(2.0) * diff / np.float32(diff.size)).astype(np.float32)
    return loss, backward(params, cache, g_out), out


def residual_output_grad(out, target, k0):
    """Output gradient of the residual loss as the kernels form it, in
    float32: q = A e on the unknown planes (e = out - target, zero below k0
    and beyond the top plane; a Neumann bottom, k0 = 0, mirrors plane 1),
    then (2 / V) A^T q."""
    f = np.float32
    e = (np.asarray(out, f) - np.asarray(target, f)).astype(f)
    D = e.shape[0]
    z = np.arange(D)[:, None, None]
    e = np.where(z >= k0, e, f(0.0)).astype(f)
    ep = np.concatenate([e, np.zeros_like(e[:1])], 0)          # plane D is zero

    def xy_sum(a):
        s = np.roll(a, 1, axis=2) + np.roll(a, -1, axis=2)
        return (s + (np.roll(a, 1, axis=1) + np.roll(a, -1, axis=1))).astype(f)

    zz = np.zeros_like(e)
    for k in range(D):
        if k == 0:
            zz[0] = f(2.0) * ep[1]
        else:
            zz[k] = ep[k - 1] + ep[k + 1]
    q = ((f(6.0) * e - xy_sum(e)) - zz).astype(f)
    q = np.where(z >= k0, q, f(0.0)).astype(f)
    zz = np.zeros_like(q)
    for k in range(D):
        lo = (f(2.0) if k - 1 == 0 else f(1.0)) * q[k - 1] if k - 1 >= k0 else np.zeros_like(q[0])
        zz[k] = lo + (q[k + 1] if k + 1 < D else np.zeros_like(q[0]))
    g = (((f(6.0) * q - xy_sum(q)) - zz) * f(2.0 / q.size)).astype(f)
    return np.where(z >= k0, g, f(0.0)).astype(f)
