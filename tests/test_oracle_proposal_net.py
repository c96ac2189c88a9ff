"""Pins of the proposal network's CPU oracle: its hand-written backward pass
against PyTorch autograd and against central finite differences (fp64, no
bf16 rounding), plus its parameter count and layer layout."""
import numpy as np
import pytest
import torch

from oracle import proposal_net as net


def _batch(B=1, h=8, w=8, seed=0):
    g = torch.Generator().manual_seed(seed)
    x = torch.rand(B, h, w, 6, generator=g, dtype=torch.float64)
    t = (torch.rand(B, h, w, 2, generator=g, dtype=torch.float64) - 0.5) * 4
    m = (torch.rand(B, h, w, generator=g, dtype=torch.float64) > 0.3).to(torch.float64)
    return x, t, m


def test_parameter_count_and_layout():
    assert net.param_count() == 1116226
    sl = net.layer_slices()
    assert sl[0] == (0, 9 * 6 * 32 + 32) and sl[-1][1] == net.param_count()


def test_backward_matches_autograd():
    flat = net.init_params(3).to(torch.float64)
    x, t, m = _batch(B=2, h=16, w=8, seed=1)
    loss, g = net.loss_and_grads(flat, x, t, m, emulate_bf16=False)
    p = flat.clone().requires_grad_(True)
    pred, _ = net.forward(p, x, emulate_bf16=False)
    ref = net.loss_value(pred, t, m)
    ref.backward()
    assert abs(float(loss) - float(ref.detach())) < 1e-12
    rel = (g - p.grad).norm() / p.grad.norm()
    assert rel < 1e-10, rel
    for a, b in net.layer_slices():
        assert (g[a:b] - p.grad[a:b]).abs().max() <= 1e-10 * max(1.0, float(p.grad[a:b].abs().max()))


def test_backward_matches_finite_differences():
    torch.manual_seed(0)
    flat = net.init_params(5).to(torch.float64) * 0.5
    x, t, m = _batch(B=1, h=16, w=16, seed=2)
    _, g = net.loss_and_grads(flat, x, t, m, emulate_bf16=False)
    rng = np.random.default_rng(4)
    eps = 1e-6
    checked = 0
    for a, b in net.layer_slices():
        for idx in rng.integers(a, b, size=6):
            e = torch.zeros_like(flat)
            e[idx] = eps
            lp = net.loss_value(net.forward(flat + e, x, False)[0], t, m)
            lm = net.loss_value(net.forward(flat - e, x, False)[0], t, m)
            fd = float(lp - lm) / (2 * eps)
            an = float(g[idx])
            if abs(an) < 1e-7 and abs(fd) < 1e-7:
                continue
            assert abs(fd - an) <= 1e-5 * max(abs(fd), abs(an)) + 1e-9, (a, idx, fd, an)
            checked += 1
    assert checked >= 30


def test_bf16_emulation_stays_close_to_fp64():
    flat = net.init_params(7)
    x, t, m = _batch(B=1, h=16, w=16, seed=3)
    p64, _ = net.forward(flat, x, emulate_bf16=False)
    p16, _ = net.forward(flat, x, emulate_bf16=True)
    rel = float((p16 - p64).norm() / p64.norm())
    assert 0 < rel < 5e-2, rel
