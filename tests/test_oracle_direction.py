"""Pins of the pair direction in Eq. 2 (Sec. 3.4) and Eq. 9 (Sec. 3.5), and
in every mode built on them.

Sec. 3.2 defines the NNF of a pair (S, T) on the target: its entry at target
pixel v is the centre u of the source patch that matches T's patch at v.  The
blend brings style S_j to frame i through the NNF of (G_j, G_i).

Here the guides are crops of one uniform-noise canvas, moved by t per frame:
G_k(v) = C(v + k t).  The styles are a per-channel LUT of the guides,
S_k = LUT(G_k).  Then G_j(v + (i - j) t) = G_i(v), so NNF(G_j, G_i)(v) =
v + (i - j) t, and remapping S_j through it gives S_i at every pixel whose
remap neighbourhood matched exactly.  In the interior, every blend and
interpolation must therefore return S_i / 255.

Remapping through the reverse field NNF(G_i, G_j) gives S_i shifted by
2 (i - j) t instead.  The same check rejects that (the last test).
"""
import numpy as np
import pytest

import pins

P, LEVELS, ITERS, SEED = 2, 2, 16, 0xFB0D1
T = (1, 2)            # translation per frame (rows, cols)
N, M = 5, 2
H, W = 44, 56


def _lut(seed):
    rng = np.random.default_rng(seed)
    lut = np.zeros((3, 256), np.uint8)
    for ch in range(3):
        # strictly increasing knots: the LUT is injective, so S_k determines G_k
        knots = np.sort(rng.choice(np.arange(1, 255), 3, replace=False))
        xs = np.concatenate([[0], knots, [255]])
        ys = np.sort(rng.choice(np.arange(0, 256), 5, replace=False))
        lut[ch] = np.round(np.interp(np.arange(256), xs, ys)).astype(np.uint8)
    return lut


def _video(n=N, seed=0xFB0D):
    canvas = pins.noise_image(H + (n - 1) * T[0], W + (n - 1) * T[1], seed)
    g = np.stack([canvas[k * T[0]:k * T[0] + H, k * T[1]:k * T[1] + W] for k in range(n)])
    lut = _lut(seed + 1)
    s = np.stack([np.stack([lut[ch][g[k][..., ch]] for ch in range(3)], -1) for k in range(n)])
    return g, s


def _interior(shift_frames, depth=1):
    """Pixels whose remap neighbourhood (depth chained remaps) lies, shifted
    by up to shift_frames * t, inside both frames with full patches."""
    rr, cc = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    mr = 2 * P * depth + shift_frames * T[0]
    mc = 2 * P * depth + shift_frames * T[1]
    return (rr >= mr) & (rr < H - mr) & (cc >= mc) & (cc < W - mc)


def _assert_rebuilds_styles(out, s, frames, shift_frames, depth=1, tol=1e-12):
    inner = _interior(shift_frames, depth)
    assert inner.sum() > 200
    for i in frames:
        err = np.abs(out[i] - s[i] / 255.0).max(axis=-1)[inner]
        assert err.max() <= tol, (i, float(err.max()), float((err > tol).mean()))


def test_translation_fields_point_from_target_into_source(orc):
    """The field of (G_j, G_i) holds v + (i - j) t in the interior: the source
    coordinates that match each target pixel (Sec. 3.2), not the reverse."""
    g, _ = _video()
    rr, cc = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for j, i in ((0, 2), (3, 1)):
        F, E = orc.patchmatch(g[j], g[i], P, LEVELS, ITERS, SEED, j * N + i)
        inner = _interior(abs(i - j))
        assert (F[..., 0][inner] == (rr + (i - j) * T[0])[inner]).all()
        assert (F[..., 1][inner] == (cc + (i - j) * T[1])[inner]).all()
        assert (E[inner] == 0).all()


def test_balanced_blend_rebuilds_each_frame(orc):
    g, s = _video()
    _assert_rebuilds_styles(orc.blend_window(g, s, M, P, LEVELS, ITERS, SEED), s, range(N), M)


def test_style_loss_blend_rebuilds_each_frame(orc):
    """Eq. 3 (guide + style loss, S^ refreshed every iteration)."""
    g, s = _video()
    out = orc.blend_window_style(g, s, M, P, LEVELS, ITERS, SEED, 16)
    _assert_rebuilds_styles(out, s, range(N), M)


def test_accurate_blend_rebuilds_each_frame(orc):
    """Eq. 7-8: T^- of the window is S_i itself in the interior, and the
    second estimation keeps the translation fields."""
    g, s = _video()
    out, tbar = orc.blend_window_accurate(g, s, M, P, LEVELS, ITERS, SEED, 16, return_tbar=True)
    inner = _interior(M)
    for i in range(N):
        assert (tbar[i][inner] == s[i][inner]).all()
    _assert_rebuilds_styles(out, s, range(N), M, depth=2)


def test_fast_blend_rebuilds_each_frame(orc):
    """Alg. 3-5 / Eq. 6: a query remaps table entries that are themselves
    sums of remaps (two chained remaps, the frames of a block all inside the
    window), so the interior keeps two remap neighbourhoods from the edges."""
    g, s = _video()
    out = orc.blend_window_fast(g, s, M, P, LEVELS, ITERS, SEED)
    _assert_rebuilds_styles(out, s, range(N), M, depth=2)


@pytest.mark.parametrize("track,align", [(False, False), (True, False), (True, True)])
def test_interpolation_rebuilds_each_frame(orc, track, align):
    """Eq. 9 (and the tracking / Eq. 10 extras): keys 0 and 4 rebuild the
    frames between them, whose weights sum to 1."""
    g, s = _video()
    keys = np.array([0, N - 1], np.int32)
    if track or align:
        out = orc.interpolate_ext(g, keys, s[keys], P, LEVELS, ITERS, SEED, 16, track=track, align=align)
    else:
        out = orc.interpolate(g, keys, s[keys], P, LEVELS, ITERS, SEED)
    _assert_rebuilds_styles(out, s, range(N), N - 1)


def test_reverse_field_is_caught(orc):
    """The check above rejects a swapped direction: S_j remapped through
    NNF(G_i, G_j) is S_i moved by 2 (i - j) t, wrong on nearly every
    interior pixel, and so is a blend that averaged such remaps."""
    g, s = _video()
    i = 2
    inner = _interior(M)
    outs = [s[i] / 255.0]
    for j in (0, 1, 3, 4):
        Fw, _ = orc.patchmatch(g[i], g[j], P, LEVELS, ITERS, SEED, i * N + j)   # the reverse pair
        r = orc.remap(s[j], Fw, P)
        wrong = np.abs(r - s[i] / 255.0).max(axis=-1)[inner] > 0
        assert wrong.mean() > 0.9, (j, wrong.mean())
        outs.append(r)
        # the right direction rebuilds S_i there
        Fr, _ = orc.patchmatch(g[j], g[i], P, LEVELS, ITERS, SEED, j * N + i)
        assert (orc.remap(s[j], Fr, P)[inner] == (s[i] / 255.0)[inner]).all()
    swapped = np.mean(outs, axis=0)
    assert (np.abs(swapped - s[i] / 255.0).max(axis=-1)[inner] > 0).mean() > 0.9
