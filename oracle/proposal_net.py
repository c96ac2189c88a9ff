"""CPU oracle of the learned proposal network -- TEST INFRASTRUCTURE ONLY.

The network is a project addition (the paper's method is model-free,
Section 3.1), so it has no passage to follow; this file is its plain
definition, in PyTorch CPU fp64, written independently of the GPU kernels:

  input   6 channels (source RGB, target RGB) in [0, 1], NHWC [B][h][w][6],
          centred to 2x - 1 by the network
  enc     (32, 48, 96, 192) channels, two 3x3 conv (padding 1) + ReLU per
          level, 2x2 average pooling between levels
  dec     nearest 2x upsampling, concatenation [upsampled, skip], two 3x3
          conv + ReLU per level
  head    3x3 conv to 2 channels (offset row, col), no activation
  loss    sum(mask * |pred - target|_1) / max(sum(mask), 1)

Parameters are one flat vector: for each of the 15 convolutions in order,
weight [cout][cin][3][3] then bias [cout].

``emulate_bf16=True`` rounds to bfloat16 (round to nearest even) exactly
where the GPU path stores bf16: the network input, every weight used by a
convolution, every stored activation and activation gradient.  With
``emulate_bf16=False`` everything is plain fp64, which is what the finite-
difference and autograd pins check.  The backward pass is written out by
hand (data and weight gradients of each convolution as library primitives).
"""
from __future__ import annotations

import torch
import torch.nn.functional as Fn

LAYERS = [  # (cin, cout, relu)
    (6, 32, True), (32, 32, True),
    (32, 48, True), (48, 48, True),
    (48, 96, True), (96, 96, True),
    (96, 192, True), (192, 192, True),
    (288, 96, True), (96, 96, True),
    (144, 48, True), (48, 48, True),
    (80, 32, True), (32, 32, True),
    (32, 2, False),
]


def param_count() -> int:
    return sum(9 * ci * co + co for ci, co, _ in LAYERS)


def unflatten(flat: torch.Tensor, dt=torch.float64):
    flat = flat.to(dt)
    out, off = [], 0
    for ci, co, _ in LAYERS:
        w = flat[off:off + 9 * ci * co].reshape(co, ci, 3, 3)
        off += 9 * ci * co
        b = flat[off:off + co]
        off += co
        out.append((w, b))
    assert off == flat.numel()
    return out


def init_params(seed: int) -> torch.Tensor:
    """Kaiming-uniform weights (fan-in, ReLU gain), zero biases, seeded."""
    g = torch.Generator().manual_seed(seed)
    parts = []
    for ci, co, _ in LAYERS:
        bound = (6.0 / (9 * ci)) ** 0.5
        parts.append((torch.rand(co * ci * 9, generator=g, dtype=torch.float64) * 2 - 1) * bound)
        parts.append(torch.zeros(co, dtype=torch.float64))
    return torch.cat(parts).to(torch.float32)


def rb(x: torch.Tensor, emulate: bool) -> torch.Tensor:
    return x.to(torch.bfloat16).to(x.dtype) if emulate else x


def _conv(x, w, b, emulate):
    return Fn.conv2d(x, rb(w, emulate), b, padding=1)


def forward(flat, pair6, emulate_bf16: bool = True, acc=torch.float64):
    """Returns (pred NHWC [B][h][w][2], cache for backward).

    acc is the type every sum is accumulated in: fp64 (the reference), or
    fp32 to measure how far a change of accumulation precision alone moves
    the bf16-rounded results (the tolerance of the GPU comparison is derived
    from that spread)."""
    e = emulate_bf16
    P = unflatten(flat, acc)
    x = rb(2.0 * pair6.to(acc).permute(0, 3, 1, 2) - 1.0, e)
    acts = {"x0": x}

    def conv(i, inp):
        y = _conv(inp, *P[i], e)
        if LAYERS[i][2]:
            y = rb(torch.relu(y), e)
        return y

    a0 = conv(0, x); e1 = conv(1, a0); p1 = rb(Fn.avg_pool2d(e1, 2), e)
    a2 = conv(2, p1); e2 = conv(3, a2); p2 = rb(Fn.avg_pool2d(e2, 2), e)
    a4 = conv(4, p2); e3 = conv(5, a4); p3 = rb(Fn.avg_pool2d(e3, 2), e)
    a6 = conv(6, p3); bt = conv(7, a6)
    c3 = torch.cat([Fn.interpolate(bt, scale_factor=2, mode="nearest"), e3], 1)
    a8 = conv(8, c3); d3 = conv(9, a8)
    c2 = torch.cat([Fn.interpolate(d3, scale_factor=2, mode="nearest"), e2], 1)
    a10 = conv(10, c2); d2 = conv(11, a10)
    c1 = torch.cat([Fn.interpolate(d2, scale_factor=2, mode="nearest"), e1], 1)
    a12 = conv(12, c1); d1 = conv(13, a12)
    pred = _conv(d1, *P[14], e)  # fp32 output on the GPU: not rounded to bf16
    acts.update(a0=a0, e1=e1, p1=p1, a2=a2, e2=e2, p2=p2, a4=a4, e3=e3, p3=p3, a6=a6, bt=bt, c3=c3,
                a8=a8, d3=d3, c2=c2, a10=a10, d2=d2, c1=c1, a12=a12, d1=d1)
    return pred.permute(0, 2, 3, 1), (P, acts)


def loss_value(pred, target, mask):
    dt = pred.dtype if pred.dtype in (torch.float32, torch.float64) else torch.float64
    pred, target, mask = pred.to(dt), target.to(dt), mask.to(dt)
    d = torch.clamp(mask.sum(), min=1.0)
    return (mask[..., None] * (pred - target).abs()).sum() / d


def loss_and_grads(flat, pair6, target, mask, emulate_bf16: bool = True, acc=torch.float64):
    """(loss, flat gradient) by the hand-derived backward pass, accumulated in acc."""
    e = emulate_bf16
    pred, (P, A) = forward(flat, pair6, e, acc)
    target = target.to(acc)
    mask = mask.to(acc)
    loss = loss_value(pred, target, mask)
    d = torch.clamp(mask.sum(), min=1.0)
    gpred = rb(mask[..., None] * torch.sign(pred - target) / d, e).permute(0, 3, 1, 2)
    grads = [None] * len(LAYERS)

    def conv_bwd(i, inp, g, need_input_grad=True):
        w, _ = P[i]
        gw = torch.nn.grad.conv2d_weight(inp, w.shape, g, padding=1)
        gb = g.sum(dim=(0, 2, 3))
        grads[i] = (gw, gb)
        if not need_input_grad:
            return None
        return rb(torch.nn.grad.conv2d_input(inp.shape, rb(w, e), g, padding=1), e)

    def relu_conv_bwd(i, inp, out, g, need_input_grad=True):
        return conv_bwd(i, inp, g * (out > 0), need_input_grad)

    def up_bwd(g, c_deep):
        gd = g[:, :c_deep]
        n, c, h, w = gd.shape
        gdeep = rb(gd.reshape(n, c, h // 2, 2, w // 2, 2).sum(dim=(3, 5)), e)
        return gdeep, g[:, c_deep:]

    def pool_bwd_add(gin, gout):
        return rb(gin + 0.25 * Fn.interpolate(gout, scale_factor=2, mode="nearest"), e)

    g = conv_bwd(14, A["d1"], gpred)
    g = relu_conv_bwd(13, A["a12"], A["d1"], g)
    g = relu_conv_bwd(12, A["c1"], A["a12"], g)
    g_d2, g_e1 = up_bwd(g, 48)
    g = relu_conv_bwd(11, A["a10"], A["d2"], g_d2)
    g = relu_conv_bwd(10, A["c2"], A["a10"], g)
    g_d3, g_e2 = up_bwd(g, 96)
    g = relu_conv_bwd(9, A["a8"], A["d3"], g_d3)
    g = relu_conv_bwd(8, A["c3"], A["a8"], g)
    g_bt, g_e3 = up_bwd(g, 192)
    g = relu_conv_bwd(7, A["a6"], A["bt"], g_bt)
    g_p3 = relu_conv_bwd(6, A["p3"], A["a6"], g)
    g_e3 = pool_bwd_add(g_e3, g_p3)
    g = relu_conv_bwd(5, A["a4"], A["e3"], g_e3)
    g_p2 = relu_conv_bwd(4, A["p2"], A["a4"], g)
    g_e2 = pool_bwd_add(g_e2, g_p2)
    g = relu_conv_bwd(3, A["a2"], A["e2"], g_e2)
    g_p1 = relu_conv_bwd(2, A["p1"], A["a2"], g)
    g_e1 = pool_bwd_add(g_e1, g_p1)
    g = relu_conv_bwd(1, A["a0"], A["e1"], g_e1)
    relu_conv_bwd(0, A["x0"], A["a0"], g, need_input_grad=False)
    flat_g = torch.cat([t.reshape(-1) for gw, gb in grads for t in (gw, gb)])
    return loss, flat_g


def layer_slices():
    """(start, stop) of every layer's weights+bias in the flat vector."""
    out, off = [], 0
    for ci, co, _ in LAYERS:
        n = 9 * ci * co + co
        out.append((off, off + n))
        off += n
    return out
