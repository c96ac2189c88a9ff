"""Pins of the oracle's remapping (Alg. 2), window blending (Eq. 2) and keyframe
interpolation (Eq. 9): the patch-placement definition of Section 3.3, identity
and translation fields, constant images, and closed forms for the window and
keyframe weights.
"""
import numpy as np
import pytest

import pins
from paper_2311_09265_amd import synth


def _field(h, w, rng):
    return np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_remap_equals_patch_placement_definition(orc, p):
    rng = np.random.default_rng(p)
    for h, w in ((9, 13), (16, 16), (5, 7)):
        style = pins.noise_image(h, w, 10 * p + h)
        F = _field(h, w, rng)
        got = orc.remap(style, F, p)
        ref = pins.remap_by_patches(style, F, p)
        assert np.array_equal(got, ref)     # identical integer sums and divisions


def test_remap_identity_translation_constant(orc):
    style = pins.noise_image(20, 24, 5)
    rr, cc = np.meshgrid(np.arange(20), np.arange(24), indexing="ij")
    ident = np.stack([rr, cc], -1).astype(np.int32)
    assert np.array_equal(orc.remap(style, ident, 2), style / 255.0)
    # a constant translation field rebuilds the shifted image away from the borders
    F = np.stack([np.clip(rr + 2, 0, 19), np.clip(cc - 3, 0, 23)], -1).astype(np.int32)
    out = orc.remap(style, F, 2)
    inner = (rr >= 2) & (rr < 16) & (cc >= 5) & (cc < 22)
    shifted = style[np.clip(rr + 2, 0, 19), np.clip(cc - 3, 0, 23)] / 255.0
    assert np.array_equal(out[inner], shifted[inner])
    # a constant image stays constant under any field
    const = np.full((20, 24, 3), (12, 200, 77), np.uint8)
    out = orc.remap(const, _field(20, 24, np.random.default_rng(0)), 2)
    assert np.allclose(out, np.array([12, 200, 77]) / 255.0, rtol=0, atol=1e-15)


def test_blend_window_closed_forms(orc):
    N, h, w, M = 7, 24, 20, 2
    guides = synth.sprite_video(N, h, w, 3, n_sprites=1, side=(6, 10), vmax=2)
    # per-frame constant styles: any remap keeps them constant, so frame i is the
    # plain mean of the constants over the window truncated to [0, N-1]
    consts = np.arange(N) * 30 + 5
    styles = np.broadcast_to(consts[:, None, None, None], (N, h, w, 3)).astype(np.uint8).copy()
    out = orc.blend_window(guides, styles, M, 2, 2, 3, 1)
    for i in range(N):
        lo, hi = max(0, i - M), min(N - 1, i + M)
        assert np.allclose(out[i], consts[lo:hi + 1].mean() / 255.0, rtol=0, atol=1e-15), i
    # M = 0 returns every style frame itself; N = 1 likewise
    styles = np.stack([pins.noise_image(h, w, 60 + i) for i in range(N)])
    assert np.array_equal(orc.blend_window(guides, styles, 0, 2, 2, 3, 1), styles / 255.0)
    assert np.array_equal(orc.blend_window(guides[:1], styles[:1], 3, 2, 2, 3, 1), styles[:1] / 255.0)


def test_blend_identical_guides_is_temporal_mean(orc):
    """With every guide frame equal (a uniform-noise texture), the NNFs converge to
    the identity, and Eq. (2) reduces to the per-pixel temporal mean of the styles."""
    N, h, w, M = 5, 16, 16, 2
    g = pins.noise_image(h, w, 77)
    guides = np.stack([g] * N)
    styles = np.stack([pins.noise_image(h, w, 80 + i) for i in range(N)])
    out = orc.blend_window(guides, styles, M, 2, 1, 12, 5)
    for i in range(N):
        lo, hi = max(0, i - M), min(N - 1, i + M)
        ref = styles[lo:hi + 1].astype(np.float64).sum(0) / 255.0 / (hi - lo + 1)
        assert np.allclose(out[i], ref, rtol=0, atol=1e-12), i


def test_interpolate_closed_forms(orc):
    N, h, w = 11, 20, 18
    guides = synth.sprite_video(N, h, w, 4, n_sprites=1, side=(6, 10), vmax=2)
    keys = np.array([2, 6, 9], np.int32)
    kc = np.array([10, 130, 250])
    kstyles = np.broadcast_to(kc[:, None, None, None], (3, h, w, 3)).astype(np.uint8).copy()
    out = orc.interpolate(guides, keys, kstyles, 2, 2, 3, 1)
    for i in range(N):
        if i in keys:
            exp = kc[list(keys).index(i)]
        elif i < keys[0]:
            exp = kc[0]
        elif i > keys[-1]:
            exp = kc[-1]
        else:
            k = np.searchsorted(keys, i)
            l, r = keys[k - 1], keys[k]
            exp = (r - i) / (r - l) * kc[k - 1] + (i - l) / (r - l) * kc[k]
        assert np.allclose(out[i], exp / 255.0, rtol=0, atol=1e-14), i
    # keyframes pass through bit-exact, for any content
    kstyles = np.stack([pins.noise_image(h, w, 90 + k) for k in range(3)])
    out = orc.interpolate(guides, keys, kstyles, 2, 2, 3, 1)
    for k, i in enumerate(keys):
        assert np.array_equal(out[i], kstyles[k] / 255.0)
