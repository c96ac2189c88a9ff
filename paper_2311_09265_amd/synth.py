"""Seeded synthetic videos shaped like the FastBlend workloads.

This module only produces inputs (uint8 guide and style frames).  It holds
none of the method's arithmetic, so that both the CPU oracle and the HIP path
can be fed from it.

The paper evaluates on real videos restyled by diffusion models (Pixabay100,
Section 4.4) and times 512x768 videos (Section 4.6).  Neither the videos nor
the models are available, so these generators stand in for them:

* value noise: a sum of bilinearly interpolated random lattices (cells 16, 8,
  4 pixels; weights 1, 1/2, 1/4), normalised to 0..255 per channel;
* sprite videos: textured rectangles moving at integer velocities over a
  static (optionally panning) noise background, reflected at the borders;
* styles: a per-channel monotone piecewise-linear colour LUT, optionally with
  per-frame gain/offset jitter (flicker) or a Gaussian blur.

Every function takes an explicit seed and is deterministic.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "value_noise", "random_lut", "apply_lut", "flicker", "gaussian_blur",
    "translation_pair", "sprite_video", "blend_workload", "interp_workload",
    "mixed_pairs", "CONFIG_SEED", "PHILOX_SEED",
]

#: data seed of workload k (1-based, in the order the workloads are listed)
CONFIG_SEED = {k: 0xFB000000 + k for k in range(1, 6)}
#: Philox key used for workload k
PHILOX_SEED = {k: 0xFB5EED00 + k for k in range(1, 6)}


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))


def value_noise(h: int, w: int, seed: int, cells: Sequence[int] = (16, 8, 4),
                weights: Sequence[float] = (1.0, 0.5, 0.25), channels: int = 3) -> np.ndarray:
    """Smooth random texture, uint8 [h][w][channels]."""
    rng = _rng(seed)
    acc = np.zeros((h, w, channels), np.float64)
    for cell, wt in zip(cells, weights):
        gh, gw = h // cell + 2, w // cell + 2
        lat = rng.random((gh, gw, channels))
        ys = np.arange(h) / cell
        xs = np.arange(w) / cell
        y0 = np.floor(ys).astype(np.int64)
        x0 = np.floor(xs).astype(np.int64)
        fy = (ys - y0)[:, None, None]
        fx = (xs - x0)[None, :, None]
        a = lat[y0][:, x0]
        b = lat[y0][:, x0 + 1]
        c = lat[y0 + 1][:, x0]
        d = lat[y0 + 1][:, x0 + 1]
        acc += wt * ((a * (1 - fx) + b * fx) * (1 - fy) + (c * (1 - fx) + d * fx) * fy)
    lo = acc.min(axis=(0, 1), keepdims=True)
    hi = acc.max(axis=(0, 1), keepdims=True)
    out = (acc - lo) / np.maximum(hi - lo, 1e-12) * 255.0
    return np.clip(np.rint(out), 0, 255).astype(np.uint8)


def random_lut(seed: int, knots: int = 5) -> np.ndarray:
    """Per-channel monotone piecewise-linear LUT, uint8 [3][256]."""
    rng = _rng(seed)
    lut = np.empty((3, 256), np.uint8)
    x = np.linspace(0, 255, knots)
    for ch in range(3):
        y = np.sort(rng.random(knots)) * 255.0
        y[0] = min(y[0], 40.0)
        y[-1] = max(y[-1], 215.0)
        lut[ch] = np.clip(np.rint(np.interp(np.arange(256), x, y)), 0, 255).astype(np.uint8)
    return lut


def apply_lut(frames: np.ndarray, lut: np.ndarray) -> np.ndarray:
    out = np.empty_like(frames)
    for ch in range(3):
        out[..., ch] = lut[ch][frames[..., ch]]
    return out


def flicker(frames: np.ndarray, seed: int, gain: float = 0.1, offset: float = 0.1) -> np.ndarray:
    """Per-frame, per-channel gain U[1-gain,1+gain] and offset U[-offset,offset]*255."""
    rng = _rng(seed)
    n = frames.shape[0]
    g = rng.uniform(1 - gain, 1 + gain, size=(n, 1, 1, 3))
    o = rng.uniform(-offset, offset, size=(n, 1, 1, 3)) * 255.0
    return np.clip(np.rint(frames.astype(np.float64) * g + o), 0, 255).astype(np.uint8)


def gaussian_blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur of an HWC uint8 image, radius ceil(3 sigma), clamped borders."""
    rad = int(np.ceil(3 * sigma))
    k = np.exp(-0.5 * (np.arange(-rad, rad + 1) / sigma) ** 2)
    k /= k.sum()
    x = img.astype(np.float64)
    h, w = x.shape[:2]
    pad = np.pad(x, ((rad, rad), (0, 0), (0, 0)), mode="edge")
    x = sum(k[i] * pad[i:i + h] for i in range(2 * rad + 1))
    pad = np.pad(x, ((0, 0), (rad, rad), (0, 0)), mode="edge")
    x = sum(k[i] * pad[:, i:i + w] for i in range(2 * rad + 1))
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def translation_pair(seed: int, size: int = 64, shift: Tuple[int, int] = (3, -2),
                     noise: int = 4, margin: int = 8):
    """Guide A, guide B = A moved by ``shift`` (rows, cols) plus U{-noise..noise}, style LUT(A).

    Both guides are crops of one larger canvas, so B(r, c) = A(r - dr, c - dc)
    holds wherever both sides exist, with no fill.  Returns (A, B, style).
    """
    dr, dc = shift
    canvas = value_noise(size + 2 * margin, size + 2 * margin, seed)
    a = canvas[margin:margin + size, margin:margin + size]
    b = canvas[margin - dr:margin - dr + size, margin - dc:margin - dc + size].astype(np.int32)
    rng = _rng(seed ^ 0x5A5A)
    if noise:
        b = b + rng.integers(-noise, noise + 1, size=b.shape)
    b = np.clip(b, 0, 255).astype(np.uint8)
    style = apply_lut(a, random_lut(seed ^ 0x1234))
    return np.ascontiguousarray(a), np.ascontiguousarray(b), np.ascontiguousarray(style)


@dataclasses.dataclass
class _Sprite:
    h: int
    w: int
    r: float
    c: float
    vr: int
    vc: int
    tex: np.ndarray


def sprite_video(n: int, h: int, w: int, seed: int, n_sprites: int = 6,
                 side: Tuple[int, int] = (32, 128), vmax: int = 8, pan: int = 0) -> np.ndarray:
    """Textured sprites moving over a noise background; uint8 [n][h][w][3].

    ``pan`` > 0 crops the background from a canvas ``pan*(n-1)`` pixels wider,
    moving the crop window by ``pan`` columns per frame.
    """
    rng = _rng(seed)
    bw = w + pan * max(n - 1, 0)
    bg = value_noise(h, bw, seed ^ 0xB6)
    speeds = np.array([v for v in range(-vmax, vmax + 1) if v != 0])
    sprites: List[_Sprite] = []
    # sprite sides are limited to the frame (small test frames)
    lo_h, lo_w = max(1, min(side[0], h // 3)), max(1, min(side[0], w // 3))
    for k in range(n_sprites):
        sh = int(rng.integers(lo_h, max(lo_h, min(side[1], h - 1)) + 1))
        sw = int(rng.integers(lo_w, max(lo_w, min(side[1], w - 1)) + 1))
        sprites.append(_Sprite(sh, sw, float(rng.integers(0, h - sh + 1)),
                               float(rng.integers(0, w - sw + 1)),
                               int(rng.choice(speeds)), int(rng.choice(speeds)),
                               value_noise(sh, sw, seed ^ (0x51 + 97 * k))))
    out = np.empty((n, h, w, 3), np.uint8)
    for t in range(n):
        frame = bg[:, pan * t:pan * t + w].copy()
        for s in sprites:
            r, c = int(s.r), int(s.c)
            frame[r:r + s.h, c:c + s.w] = s.tex
            # advance with reflection at the borders
            nr, nc = s.r + s.vr, s.c + s.vc
            if nr < 0 or nr > h - s.h:
                s.vr = -s.vr
                nr = s.r + s.vr
            if nc < 0 or nc > w - s.w:
                s.vc = -s.vc
                nc = s.c + s.vc
            s.r, s.c = float(min(max(nr, 0), h - s.h)), float(min(max(nc, 0), w - s.w))
        out[t] = frame
    return out


def blend_workload(n: int = 32, h: int = 512, w: int = 512, seed: int = CONFIG_SEED[2]):
    """Guide sprite video and flickering LUT-recoloured style video (blending mode)."""
    guides = sprite_video(n, h, w, seed)
    styles = flicker(apply_lut(guides, random_lut(seed ^ 0x77)), seed ^ 0x99)
    return guides, styles


def interp_workload(n: int = 64, h: int = 576, w: int = 1024, key_every: int = 16,
                    seed: int = CONFIG_SEED[3]):
    """Panning sprite video, keyframe indices and blurred LUT keyframe styles (interpolation mode)."""
    guides = sprite_video(n, h, w, seed, pan=2)
    keys = np.arange(0, n, key_every, dtype=np.int32)
    lut = random_lut(seed ^ 0x77)
    rng = _rng(seed ^ 0x3C)
    key_styles = np.stack([gaussian_blur(apply_lut(guides[k], lut), float(rng.uniform(0.8, 2.0)))
                           for k in keys])
    return guides, keys, key_styles


def mixed_pairs(per_size: int = 12, seed: int = CONFIG_SEED[4],
                sizes=((256, 256, 3), (512, 512, 3), (576, 1024, 4), (720, 1280, 4)), frames: int = 12):
    """(source, target, levels) guide pairs (t, t+delta), delta ~ U{1..5}, at mixed sizes."""
    rng = _rng(seed)
    pairs = []
    for si, (h, w, lv) in enumerate(sizes):
        vid = sprite_video(frames, h, w, seed ^ (0x100 * (si + 1)))
        for _ in range(per_size):
            d = int(rng.integers(1, 6))
            t = int(rng.integers(0, frames - d))
            pairs.append((vid[t], vid[t + d], lv))
    return pairs
