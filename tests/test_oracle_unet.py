"""Pins of the surrogate network's oracle (oracle/unet.py) against
definitions it does not share code with: a convolution summed by hand, the
transpose of a linear map, autograd of the same network, finite
differences, and the closed form of Adam under a constant gradient."""
import numpy as np
import pytest
import torch

from oracle import unet

SMALL = dict(c0=4, c1=6, c2=8)


def _params(seed, scale=0.3, **cfg):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(unet.param_count(**cfg)) * scale).astype(np.float32)


def test_param_count_of_the_standard_network():
    """c0, c1, c2 = 32, 64, 128: about half a million parameters."""
    n = unet.param_count()
    assert n == (9 * 3 * 32 + 32 + 9 * 32 * 32 + 32 + 9 * 32 * 64 + 64 + 9 * 64 * 64 + 64 + 9 * 64 * 128 + 128
                 + 9 * 128 * 128 + 128 + 9 * 192 * 64 + 64 + 9 * 64 * 64 + 64 + 9 * 96 * 32 + 32
                 + 9 * 32 * 32 + 32 + 32 * 3 + 3)
    assert 450_000 < n < 550_000


def test_conv_is_the_periodic_correlation_summed_by_hand():
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.standard_normal((2, 5, 6, 3)))
    w = torch.tensor(rng.standard_normal((9, 3, 4)))
    b = torch.tensor(rng.standard_normal(4))
    z = unet.conv(x, w, b, rounding=False).numpy()
    ref = np.zeros((2, 5, 6, 4))
    for n in range(2):
        for yy in range(5):
            for xx in range(6):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        ref[n, yy, xx] += x[n, (yy + dy) % 5, (xx + dx) % 6].numpy() @ w[3 * (dy + 1) + dx + 1].numpy()
                ref[n, yy, xx] += b.numpy()
    assert np.abs(z - ref).max() < 1e-12


def test_bf16_rounding_is_round_to_nearest_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to the even mantissa (1)
    x = torch.tensor([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -(1 + 2 ** -7)], dtype=torch.float64)
    assert unet.bf16(x).tolist() == [1.0, 1 + 2 ** -6, 1.0, -(1 + 2 ** -7)]


def test_input_gradient_is_the_adjoint_of_the_convolution():
    """<conv(x), dz> = <x, conv_input_grad(dz)> for the bias-free map."""
    rng = np.random.default_rng(1)
    for taps in (9, 1):
        x = torch.tensor(rng.standard_normal((2, 4, 8, 3)))
        dz = torch.tensor(rng.standard_normal((2, 4, 8, 5)))
        w = torch.tensor(rng.standard_normal((taps, 3, 5)))
        lhs = (unet.conv(x, w, torch.zeros(5, dtype=torch.float64), rounding=False) * dz).sum()
        rhs = (x * unet._conv_input_grad(dz, w, rounding=False)).sum()
        assert abs(float(lhs - rhs)) < 1e-10 * abs(float(lhs))


def test_backward_matches_autograd():
    """The hand-written backward (rounding off) equals torch autograd of the
    forward pass, for every parameter."""
    cfg = SMALL
    p = _params(2, **cfg)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 8, 12, 3))
    t = rng.standard_normal((2, 8, 12, 3))
    loss, g, _ = unet.loss_and_grads(p, x, t, rounding=False, **cfg)
    pt = torch.tensor(p.astype(np.float64), requires_grad=True)
    # autograd through the same forward: rebuild it on a differentiable vector
    orig_unpack = unet.unpack

    def unpack_diff(params, c0, c1, c2, cin):
        out, off = {}, 0
        for name, ci, co, taps, _ in unet.layers(c0, c1, c2, cin):
            w = pt[off:off + taps * ci * co].reshape(taps, ci, co)
            off += taps * ci * co
            out[name] = (w, pt[off:off + co])
            off += co
        return out

    unet.unpack = unpack_diff
    try:
        y, _ = unet.forward(p, x, rounding=False, **cfg)
        l2 = ((y - torch.tensor(t)) ** 2).mean()
        l2.backward()
    finally:
        unet.unpack = orig_unpack
    assert abs(float(l2.detach()) - loss) < 1e-12
    assert np.abs(pt.grad.numpy() - g).max() < 1e-10 * max(1.0, np.abs(g).max())


def test_backward_matches_finite_differences():
    cfg = SMALL
    p = _params(4, **cfg)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((1, 8, 8, 3))
    t = rng.standard_normal((1, 8, 8, 3))
    _, g, _ = unet.loss_and_grads(p, x, t, rounding=False, **cfg)
    p64 = p.astype(np.float64)
    idx = np.random.default_rng(6).choice(p.size, 25, replace=False)
    for i in idx:
        h = 1e-6  # small enough that no ReLU switches between the two evaluations
        pp, pm = p64.copy(), p64.copy()
        pp[i] += h
        pm[i] -= h
        # forward in FP64 on unrounded parameters
        lp = float(((unet.forward(pp, x, rounding=False, **cfg)[0] - torch.tensor(t)) ** 2).mean())
        lm = float(((unet.forward(pm, x, rounding=False, **cfg)[0] - torch.tensor(t)) ** 2).mean())
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) < 1e-5 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_rounding_changes_results_only_at_bf16_precision():
    """With rounding on, outputs and gradients move by about 2^-8 relative,
    not more: the rounding points are where the GPU rounds, not a change of
    the network."""
    cfg = SMALL
    p = _params(7, scale=0.2, **cfg)
    rng = np.random.default_rng(8)
    x = rng.standard_normal((1, 8, 8, 3))
    t = rng.standard_normal((1, 8, 8, 3))
    l0, g0, y0 = unet.loss_and_grads(p, x, t, rounding=False, **cfg)
    l1, g1, y1 = unet.loss_and_grads(p, x, t, rounding=True, **cfg)
    assert 0 < np.abs(y1 - y0).max() < 0.05 * np.abs(y0).max()
    assert np.linalg.norm(g1 - g0) < 0.05 * np.linalg.norm(g0)


def test_residual_identity_when_the_head_is_zero():
    """y = x + head(...): zero head weights and bias give y = x exactly."""
    cfg = SMALL
    p = _params(9, **cfg)
    n_head = 4 * 3 + 3
    p[-n_head:] = 0
    x = np.random.default_rng(10).standard_normal((1, 8, 8, 3))
    y, _ = unet.forward(p, x, **cfg)
    assert np.array_equal(y.numpy(), x)


def test_adam_closed_form_for_a_constant_gradient():
    """With a constant gradient g, the bias-corrected moments are g and g^2
    at every step, so each step moves a parameter by lr g / (|g| + eps)."""
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    q = p.copy()
    for step in range(1, 6):
        q, m, v = unet.adam(q, g, m, v, step, lr=0.01)
    expect = p - 5 * 0.01 * g / (np.abs(g) + 1e-8)
    assert np.abs(q - expect).max() < 1e-12
