"""FP64 reference of the learned Poisson warm start (3-D U-Net).

Test infrastructure only (see the package docstring).  Not in the paper:
the learned warm start is a production form of the field solve whose
multigrid always finishes the solve to the same residual.

Architecture (four levels of 16/32/64/128 channels, 3x3x3 convolutions):
  encoder   e0a 2->16, e0b 16->16 | avg-pool 2^3 | e1a 16->32, e1b 32->32 |
            pool | e2a 32->64, e2b 64->64 | pool | ba 64->128, bb 128->128
  decoder   nearest upsampling x2, concatenation [up, skip], two convs:
            d2a 192->64, d2b 64->64 | d1a 96->32, d1b 32->32 |
            d0a 48->16, d0b 16->16
  head      1x1x1 convolution 16->1, no activation.
Every 3x3x3 convolution has a bias and a ReLU.  Padding is circular in x and
y (periodic gap) and zero in z.  Tensors are (D, H, W, C) = (z, y, x, c).

Parameter vector: for each convolution in the order above, W[co][tap][ci]
(tap = (dz+1)*9 + (dy+1)*3 + (dx+1)) then b[co]; then the head's w[16] and
b.  The loss is the mean squared error of the output against the target.
"""
import numpy as np

LAYERS = (("e0a", 2, 16), ("e0b", 16, 16), ("e1a", 16, 32), ("e1b", 32, 32),
          ("e2a", 32, 64), ("e2b", 64, 64), ("ba", 64, 128), ("bb", 128, 128),
          ("d2a", 192, 64), ("d2b", 64, 64), ("d1a", 96, 32), ("d1b", 32, 32),
          ("d0a", 48, 16), ("d0b", 16, 16))
HEAD_IN = 16
TAPS = tuple((dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1)
             for dx in (-1, 0, 1))


def param_layout():
    """[(name, kind, offset, shape)] of the flat parameter vector."""
    out, off = [], 0
    for name, ci, co in LAYERS:
        out.append((name, "W", off, (co, 27, ci)))
        off += co * 27 * ci
        out.append((name, "b", off, (co,)))
        off += co
    out.append(("head", "W", off, (HEAD_IN,)))
    off += HEAD_IN
    out.append(("head", "b", off, (1,)))
    off += 1
    return out, off


def unpack(params):
    lay, _ = param_layout()
    d = {}
    for name, kind, off, shape in lay:
        n = int(np.prod(shape))
        d[(name, kind)] = np.asarray(params[off:off + n], np.float64).reshape(shape)
    return d


def shift(x, dz, dy, dx):
    """s[z, y, x] = x[z+dz, y+dy, x+dx]: circular in y, x, zero outside z."""
    s = np.roll(x, shift=(-dy, -dx), axis=(1, 2))
    if dz == 1:
        s = np.concatenate([s[1:], np.zeros_like(s[:1])], axis=0)
    elif dz == -1:
        s = np.concatenate([np.zeros_like(s[:1]), s[:-1]], axis=0)
    return s


def conv(x, W, b):
    out = np.broadcast_to(b, x.shape[:3] + (W.shape[0],)).copy()
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += shift(x, dz, dy, dx) @ W[:, t, :].T
    return out


def conv_backward(x, W, g):
    """Gradients of sum(g * conv(x)) w.r.t. x, W, b."""
    dW = np.zeros_like(W)
    dx_ = np.zeros_like(x)
    for t, (dz, dy, dx) in enumerate(TAPS):
        dW[:, t, :] = np.einsum("zyxo,zyxi->oi", g, shift(x, dz, dy, dx))
        # Adjoint of the shift: shift back by the opposite tap.
        dx_ += shift(g @ W[:, t, :], -dz, -dy, -dx)
    return dx_, dW, g.sum(axis=(0, 1, 2))


def pool(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def pool_backward(g):
    return np.repeat(np.repeat(np.repeat(g, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_backward(g):
    D, H, W, C = g.shape
    return g.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


def forward(params, x):
    """x: (D, H, W, 2) -> (out (D, H, W), cache)."""
    P = unpack(params)
    cache = {"x": x}

    def layer(name, inp):
        y = relu(conv(inp, P[(name, "W")], P[(name, "b")]))
        cache[name] = (inp, y)
        return y

    e0 = layer("e0b", layer("e0a", x))
    e1 = layer("e1b", layer("e1a", pool(e0)))
    e2 = layer("e2b", layer("e2a", pool(e1)))
    bt = layer("bb", layer("ba", pool(e2)))
    d2 = layer("d2b", layer("d2a", np.concatenate([up(bt), e2], -1)))
    d1 = layer("d1b", layer("d1a", np.concatenate([up(d2), e1], -1)))
    d0 = layer("d0b", layer("d0a", np.concatenate([up(d1), e0], -1)))
    cache["d0"] = d0
    out = d0 @ P[("head", "W")] + P[("head", "b")][0]
    return out, cache


def backward(params, cache, g_out):
    """Gradient of sum(g_out * out) w.r.t. the parameter vector."""
    P = unpack(params)
    grads = {}

    def layer_back(name, gy):
        inp, y = cache[name]
        gpre = gy * (y > 0)
        gx, dW, db = conv_backward(inp, P[(name, "W")], gpre)
        grads[(name, "W")] = dW
        grads[(name, "b")] = db
        return gx

    d0 = cache["d0"]
    grads[("head", "W")] = np.einsum("zyx,zyxc->c", g_out, d0)
    grads[("head", "b")] = np.array([g_out.sum()])
    g = g_out[..., None] * P[("head", "W")]
    gc = layer_back("d0a", layer_back("d0b", g))
    g_e0 = gc[..., 32:]
    gc = layer_back("d1a", layer_back("d1b", up_backward(gc[..., :32])))
    g_e1 = gc[..., 64:]
    gc = layer_back("d2a", layer_back("d2b", up_backward(gc[..., :64])))
    g_e2 = gc[..., 128:]
    g = layer_back("ba", layer_back("bb", up_backward(gc[..., :128])))
    g = layer_back("e2a", layer_back("e2b", pool_backward(g) + g_e2))
    g = layer_back("e1a", layer_back("e1b", pool_backward(g) + g_e1))
    layer_back("e0a", layer_back("e0b", pool_backward(g) + g_e0))
    lay, n = param_layout()
    vec = np.zeros(n)
    for name, kind, off, shape in lay:
        vec[off:off + int(np.prod(shape))] = grads[(name, kind)].reshape(-1)
    return vec


def loss_and_grad(params, x, target):
    out, cache = forward(params, x)
    diff = out - target
    loss = float(np.mean(diff * diff))
    g_out = 2.0 * diff / diff.size
    return loss, backward(params, cache, g_out), out


def adam_step(params, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) in place; t counts from 1."""
    m[:] = beta1 * m + (1.0 - beta1) * grad
    v[:] = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    params[:] = params - lr * mh / (np.sqrt(vh) + eps)


# --------------------------------------------------------------------------
# Residual loss: the scaled 7-point operator applied to the error
# --------------------------------------------------------------------------
def _net_grid(shape, k0):
    """Poisson grid of the network's planes: nz = D with a Dirichlet top
    (the plane beyond the network is zero) and a Dirichlet (k0 = 1) or
    Neumann (k0 = 0) bottom."""
    from .poisson import DIRICHLET, NEUMANN, Grid
    D, H, W = shape
    return Grid(W, H, D, 1.0, DIRICHLET if k0 == 1 else NEUMANN, DIRICHLET)


def _embed(e, k0):
    """Network planes (D, H, W) -> node array (D+1, H, W) with the planes
    below k0 and the top plane zero."""
    D, H, W = e.shape
    out = np.zeros((D + 1, H, W))
    out[k0:D] = e[k0:D]
    return out


def residual_loss_and_grad(params, x, target, k0):
    """Loss = sum over the unknown planes of (A (c - t))^2 / V, with A the
    scaled Poisson operator of the network grid (x, y periodic, zero beyond
    the top plane, Dirichlet or mirror Neumann bottom); it is the squared
    residual of the start phi_prev + sigma c over sigma^2, per voxel.
    Returns (loss, parameter gradient, output)."""
    from .poisson import apply_operator
    out, cache = forward(params, x)
    D, H, W = out.shape
    g = _net_grid(out.shape, k0)
    q = apply_operator(_embed(out - target, k0), g)[:D]
    q[:k0] = 0.0
    V = out.size
    loss = float(np.sum(q * q) / V)
    # d loss / d c = (2 / V) A^T q on the unknowns: A^T through the
    # operator's definition (rows of A), taken column by column as the
    # adjoint of apply_operator.
    g_out = (2.0 / V) * _adjoint(q, g, k0)
    return loss, backward(params, cache, g_out), out


def _adjoint(q, g, k0):
    """A^T q restricted to the unknown planes, from A's rows: A e at an
    unknown node is 6 e - (x, y neighbours) - (z neighbours, the lower one
    mirrored at a Neumann bottom), so each row entry is sent back to the
    node it multiplies."""
    D, H, W = q.shape
    r = np.zeros((D + 1, H, W))
    for k in range(k0, D):
        qk = q[k]
        r[k] += 6.0 * qk
        r[k] -= np.roll(qk, 1, axis=1) + np.roll(qk, -1, axis=1)
        r[k] -= np.roll(qk, 1, axis=0) + np.roll(qk, -1, axis=0)
        if k == 0:
            r[1] -= 2.0 * qk          # mirror ghost phi_-1 = phi_1
        else:
            r[k - 1] -= qk
            r[k + 1] -= qk
    out = r[:D]
    out[:k0] = 0.0
    return out
