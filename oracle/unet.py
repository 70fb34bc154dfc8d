"""FP64 CPU oracle of the surrogate network.  Test infrastructure only: the
tests, the smoke check and the benchmark's CPU baseline use it; the library
never does.

The surrogate maps the state (phi, rho u_x, rho u_y) of a periodic D2Q9
lattice, as a [batch, height, width, 3] tensor in normalised units, to the
state 50 lattice Boltzmann steps later.  It is a small U-Net with periodic
3x3 convolutions:

    e0a  3 -> c0      e0b  c0 -> c0           (full resolution; e0b is skip 0)
    pool (2x2 mean)
    e1a  c0 -> c1     e1b  c1 -> c1           (1/2; e1b is skip 1)
    pool
    b2a  c1 -> c2     b2b  c2 -> c2           (1/4)
    upsample (nearest, 2x), concatenate [up, skip 1]
    d1a  c2+c1 -> c1  d1b  c1 -> c1           (1/2)
    upsample, concatenate [up, skip 0]
    d0a  c1+c0 -> c0  d0b  c0 -> c0           (full resolution)
    head 1x1 c0 -> 3, no activation;  y = x + head

Every 3x3 convolution is followed by a bias and ReLU.  Convolutions take
their input and weights rounded to bfloat16 (round to nearest even) and
accumulate exactly (here in FP64); biases stay FP32.  The backward pass
rounds to bfloat16 at the same places: the incoming gradient and the
weights for the input gradient, the layer input and the incoming gradient
for the weight gradient.  ``rounding=False`` turns the rounding off, which
the pins use to compare the hand-written backward with autograd.

Parameters are one flat FP32 vector: for each layer in the order above,
W[tap][cin][cout] (tap = 3 dy + dx for offsets dy, dx in -1..1, or a single
tap for the head) then b[cout].
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

DT = torch.float64


def layers(c0=32, c1=64, c2=128, cin=3):
    """(name, cin, cout, taps, relu) of every convolution, in parameter order."""
    return [
        ("e0a", cin, c0, 9, True), ("e0b", c0, c0, 9, True),
        ("e1a", c0, c1, 9, True), ("e1b", c1, c1, 9, True),
        ("b2a", c1, c2, 9, True), ("b2b", c2, c2, 9, True),
        ("d1a", c2 + c1, c1, 9, True), ("d1b", c1, c1, 9, True),
        ("d0a", c1 + c0, c0, 9, True), ("d0b", c0, c0, 9, True),
        ("head", c0, cin, 1, False),
    ]


def param_count(c0=32, c1=64, c2=128, cin=3) -> int:
    return sum(t * ci * co + co for _, ci, co, t, _ in layers(c0, c1, c2, cin))


def unpack(params, c0=32, c1=64, c2=128, cin=3):
    """Flat parameter vector -> {name: (W[taps, cin, cout], b[cout])} as FP64 tensors."""
    p = torch.as_tensor(np.asarray(params)).to(DT)  # FP32 master values are exact in FP64
    out, off = {}, 0
    for name, ci, co, t, _ in layers(c0, c1, c2, cin):
        w = p[off:off + t * ci * co].reshape(t, ci, co)
        off += t * ci * co
        b = p[off:off + co]
        off += co
        out[name] = (w, b)
    assert off == p.numel()
    return out


def bf16(x, rounding=True):
    """x rounded to the nearest bfloat16 (ties to even), as FP64."""
    return x.to(torch.bfloat16).to(DT) if rounding else x


def _nchw(x):
    return x.permute(0, 3, 1, 2)


def _nhwc(x):
    return x.permute(0, 2, 3, 1)


def _kernel(w):
    """W[tap][cin][cout] -> conv2d weight [cout, cin, kh, kw]."""
    t, ci, co = w.shape
    k = 3 if t == 9 else 1
    return w.permute(2, 1, 0).reshape(co, ci, k, k)


def conv(x, w, b, rounding=True):
    """Periodic convolution (cross-correlation) of NHWC x with W[tap][cin][cout]:
    z[p][co] = b[co] + sum_{tap, ci} x[p + (dy, dx)][ci] W[tap][ci][co]."""
    xn = _nchw(bf16(x, rounding))
    k = _kernel(bf16(w, rounding))
    if k.shape[-1] == 3:
        xn = F.pad(xn, (1, 1, 1, 1), mode="circular")
    return _nhwc(F.conv2d(xn, k)) + b


def pool(x):
    """2x2 mean."""
    return _nhwc(F.avg_pool2d(_nchw(x), 2))


def up(x):
    """Nearest-neighbour 2x upsampling."""
    return x.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)


def forward(params, x, c0=32, c1=64, c2=128, rounding=True):
    """Returns (y, activations) for x [B, H, W, 3] (H, W multiples of 4)."""
    P = unpack(params, c0, c1, c2, x.shape[-1])
    x = torch.as_tensor(np.asarray(x)).to(DT)
    act = {"x": x}

    def layer(name, inp):
        w, b = P[name]
        z = conv(inp, w, b, rounding)
        a = torch.relu(z) if name != "head" else z
        act[name] = a
        return a

    e0 = layer("e0b", layer("e0a", x))
    e1 = layer("e1b", layer("e1a", pool(e0)))
    b2 = layer("b2b", layer("b2a", pool(e1)))
    u1 = torch.cat([up(b2), e1], dim=-1)
    act["u1"] = u1
    d1 = layer("d1b", layer("d1a", u1))
    u0 = torch.cat([up(d1), e0], dim=-1)
    act["u0"] = u0
    d0 = layer("d0b", layer("d0a", u0))
    y = x + layer("head", d0)
    return y, act


def _conv_input_grad(dz, w, rounding):
    """d(loss)/d(input) of conv: dx[q][ci] = sum_{tap, co} dz[q - tap][co] W[tap][ci][co]."""
    k = _kernel(bf16(w, rounding))
    dzn = _nchw(bf16(dz, rounding))
    if k.shape[-1] == 3:
        # the adjoint of a periodic correlation is a periodic convolution
        dzn = F.pad(dzn, (1, 1, 1, 1), mode="circular")
        return _nhwc(F.conv2d(dzn, k.flip(-1, -2).transpose(0, 1)))
    return _nhwc(F.conv2d(dzn, k.transpose(0, 1)))


def _conv_weight_grad(x, dz, taps, rounding):
    """dW[tap][ci][co] = sum_p x[p + tap][ci] dz[p][co];  db[co] = sum_p dz[p][co]."""
    xb, dzb = bf16(x, rounding), bf16(dz, rounding)
    if taps == 1:
        dw = torch.einsum("bhwi,bhwo->io", xb, dzb)[None]
    else:
        dw = torch.zeros(9, x.shape[-1], dz.shape[-1], dtype=DT)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                xs = torch.roll(xb, shifts=(-dy, -dx), dims=(1, 2))  # xs[p] = x[p + (dy, dx)]
                dw[3 * (dy + 1) + (dx + 1)] = torch.einsum("bhwi,bhwo->io", xs, dzb)
    return dw, dz.sum(dim=(0, 1, 2))


def loss_and_grads(params, x, target, c0=32, c1=64, c2=128, rounding=True):
    """Mean squared error over every element of y and the gradient of the
    loss with respect to the flat parameter vector (FP64), by the backward
    pass written out layer by layer."""
    P = unpack(params, c0, c1, c2, x.shape[-1])
    y, A = forward(params, x, c0, c1, c2, rounding)
    t = torch.as_tensor(np.asarray(target)).to(DT)
    diff = y - t
    loss = float((diff ** 2).mean())
    G = {}

    def back(name, inp, da):
        """Gradient through layer `name` (input `inp`, output A[name]); returns d(inp)."""
        w, _ = P[name]
        dz = da * (A[name] > 0) if name != "head" else da
        G[name] = _conv_weight_grad(inp, dz, w.shape[0], rounding)
        return _conv_input_grad(dz, w, rounding)

    c1_ = P["e1b"][0].shape[2]
    dd0 = back("head", A["d0b"], 2.0 * diff / diff.numel())
    du0 = back("d0a", A["u0"], back("d0b", A["d0a"], dd0))
    dd1 = du0[..., :c1_].reshape(du0.shape[0], du0.shape[1] // 2, 2, du0.shape[2] // 2, 2, c1_).sum(dim=(2, 4))
    de0 = du0[..., c1_:]
    du1 = back("d1a", A["u1"], back("d1b", A["d1a"], dd1))
    c2_ = P["b2b"][0].shape[2]
    db2 = du1[..., :c2_].reshape(du1.shape[0], du1.shape[1] // 2, 2, du1.shape[2] // 2, 2, c2_).sum(dim=(2, 4))
    de1 = du1[..., c2_:]
    dp1 = back("b2a", pool(A["e1b"]), back("b2b", A["b2a"], db2))
    de1 = de1 + up(dp1) / 4.0
    dp0 = back("e1a", pool(A["e0b"]), back("e1b", A["e1a"], de1))
    de0 = de0 + up(dp0) / 4.0
    back("e0a", A["x"], back("e0b", A["e0a"], de0))
    flat = []
    for name, *_ in layers(c0, c1, c2, x.shape[-1]):
        dw, db = G[name]
        flat += [dw.reshape(-1), db.reshape(-1)]
    return loss, torch.cat(flat).numpy(), y.numpy()


def adam(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) of FP64 copies; step
    counts from 1.  Returns (params, m, v)."""
    params, grads = np.asarray(params, np.float64), np.asarray(grads, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * grads
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * grads * grads
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
