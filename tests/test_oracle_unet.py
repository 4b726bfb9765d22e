"""Pins of the FP64 U-Net reference: central finite differences of the
loss, and an independent PyTorch CPU autograd evaluation of the same
network (test-only cross-check)."""
import numpy as np
import pytest

import workloads as W
from oracle import unet as U


def small_case(seed=0, shape=(8, 8, 16)):
    rng = np.random.default_rng(seed)
    params = W.unet_init(seed).astype(np.float64)
    # Non-zero biases so every term of the gradient is exercised.
    lay, n = U.param_layout()
    for name, kind, off, shape_ in lay:
        if kind == "b":
            k = int(np.prod(shape_))
            params[off:off + k] = rng.standard_normal(k) * 0.05
    x = rng.standard_normal(shape + (2,))
    t = rng.standard_normal(shape)
    return params, x, t


def test_param_count_matches_init():
    _, n = U.param_layout()
    assert W.unet_init(0).size == n


def test_gradient_finite_differences():
    params, x, t = small_case()
    loss, grad, _ = U.loss_and_grad(params, x, t)
    rng = np.random.default_rng(1)
    lay, n = U.param_layout()
    # Check a sample of parameters in every tensor.
    idx = []
    for name, kind, off, shape in lay:
        k = int(np.prod(shape))
        idx += list(off + rng.choice(k, size=min(3, k), replace=False))
    h = 1e-6
    for i in idx:
        p1 = params.copy()
        p1[i] += h
        p2 = params.copy()
        p2[i] -= h
        fd = (U.loss_and_grad(p1, x, t)[0] - U.loss_and_grad(p2, x, t)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, grad[i])


def test_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    params, x, t = small_case(2)
    loss, grad, out = U.loss_and_grad(params, x, t)
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True)
         for k, v in U.unpack(params).items()}

    def conv(inp, name):
        # inp: (1, C, D, H, W); circular padding in H, W, zeros in D.
        w = P[(name, "W")]                       # (co, 27, ci)
        co, _, ci = w.shape
        k = w.reshape(co, 3, 3, 3, ci).permute(0, 4, 1, 2, 3)
        y = F.pad(inp, (1, 1, 1, 1, 0, 0), mode="circular")
        y = F.pad(y, (0, 0, 0, 0, 1, 1))
        return F.relu(F.conv3d(y, k) + P[(name, "b")].view(1, -1, 1, 1, 1))

    xt = torch.tensor(np.transpose(x, (3, 0, 1, 2))[None])
    up = lambda a: F.interpolate(a, scale_factor=2, mode="nearest")
    e0 = conv(conv(xt, "e0a"), "e0b")
    e1 = conv(conv(F.avg_pool3d(e0, 2), "e1a"), "e1b")
    e2 = conv(conv(F.avg_pool3d(e1, 2), "e2a"), "e2b")
    bt = conv(conv(F.avg_pool3d(e2, 2), "ba"), "bb")
    d2 = conv(conv(torch.cat([up(bt), e2], 1), "d2a"), "d2b")
    d1 = conv(conv(torch.cat([up(d2), e1], 1), "d1a"), "d1b")
    d0 = conv(conv(torch.cat([up(d1), e0], 1), "d0a"), "d0b")
    o = torch.einsum("bczyx,c->bzyx", d0, P[("head", "W")]) + P[("head", "b")]
    lt = torch.mean((o[0] - torch.tensor(t)) ** 2)
    lt.backward()
    assert abs(lt.item() - loss) <= 1e-12 * abs(loss)
    assert np.allclose(o[0].detach().numpy(), out, rtol=1e-12, atol=1e-12)
    lay, n = U.param_layout()
    for name, kind, off, shape in lay:
        k = int(np.prod(shape))
        ref = P[(name, kind)].grad.numpy().reshape(-1)
        assert np.allclose(grad[off:off + k], ref, rtol=1e-9, atol=1e-14), name


def test_adam_against_closed_form_first_step():
    """First Adam step moves every parameter by -lr * sign(grad) (bias-
    corrected moments of one gradient)."""
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -0.25, 1e-3])
    m, v = np.zeros(3), np.zeros(3)
    U.adam_step(p, m, v, g, 1, lr=0.1, eps=0.0)
    assert np.allclose(p, [0.9, -1.9, 2.9], rtol=0, atol=1e-15)


@pytest.mark.parametrize("k0", [0, 1])
def test_residual_loss_pins(k0):
    """The residual loss is the squared residual of the Poisson operator
    (its own pinned implementation) over the unknowns; its gradient with
    respect to the output matches finite differences, which checks the
    adjoint (including the Neumann mirror)."""
    from oracle import poisson as P
    rng = np.random.default_rng(4)
    shape = (8, 8, 8)
    c = rng.standard_normal(shape)
    t = rng.standard_normal(shape)
    g = U._net_grid(shape, k0)
    e = U._embed(c - t, k0)
    q = P.apply_operator(e, g)[:8]
    q[:k0] = 0.0
    loss = np.sum(q * q) / c.size
    # Finite differences of the loss w.r.t. a few output entries.
    def L(cc):
        qq = P.apply_operator(U._embed(cc - t, k0), g)[:8]
        qq[:k0] = 0.0
        return np.sum(qq * qq) / c.size
    grad = (2.0 / c.size) * U._adjoint(q, g, k0)
    for idx in [(0, 0, 0), (1, 2, 3), (7, 7, 7), (0, 5, 1), (3, 0, 7)]:
        h = 1e-6
        cp = c.copy(); cp[idx] += h
        cm = c.copy(); cm[idx] -= h
        fd = (L(cp) - L(cm)) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, grad[idx])
    assert abs(L(c) - loss) < 1e-12
    # Zero error, zero loss.
    assert L(t) == 0.0


def test_residual_loss_and_grad_matches_finite_differences():
    p = W.unet_init(5).astype(np.float64)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((8, 8, 8, 2))
    t = rng.standard_normal((8, 8, 8))
    loss, g, _ = U.residual_loss_and_grad(p, x, t, 1)
    lay, n = U.param_layout()
    for name, kind, off, shape in lay[-4:]:
        j = off
        h = 1e-5
        pp = p.copy(); pp[j] += h
        pm = p.copy(); pm[j] -= h
        fd = (U.residual_loss_and_grad(pp, x, t, 1)[0] -
              U.residual_loss_and_grad(pm, x, t, 1)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-5 * max(1.0, abs(fd)), (name, kind, fd, g[j])
