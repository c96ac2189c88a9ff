"""Pins of the oracle's fast mode (remapping table Alg. 3, blending table
Alg. 4, interval query Alg. 5, sliding window Eq. 6)."""
import numpy as np
import pytest

import oracle
from paper_2311_09265_amd import synth


def _window_mean(styles, M):
    N = len(styles)
    x = styles.astype(np.float64) / 255.0
    return np.stack([x[max(0, i - M):min(N - 1, i + M) + 1].mean(0) for i in range(N)])


@pytest.mark.parametrize("N,M", [(1, 3), (2, 1), (5, 2), (7, 7), (8, 3), (13, 4), (16, 5), (31, 9), (33, 1), (40, 30)])
def test_identity_fields_give_the_exact_window_mean(N, M):
    """With every NNF the identity, every remap (Alg. 2) is exact, so the
    tables and queries must reproduce the truncated window mean exactly:
    a frame counted twice or missed by the table or query indexing shows."""
    rng = np.random.default_rng(N * 100 + M)
    h, w = 6, 7
    g = rng.integers(0, 256, (N, h, w, 3)).astype(np.uint8)
    s = rng.integers(0, 256, (N, h, w, 3)).astype(np.uint8)
    out = oracle.blend_window_fast(g, s, M, 2, 1, 1, 5, identity_nnf=True)
    assert np.abs(out - _window_mean(s, M)).max() < 1e-12


def test_identity_remap_of_float_image_is_exact():
    rng = np.random.default_rng(3)
    X = rng.random((9, 11, 3))
    r, c = np.meshgrid(np.arange(9), np.arange(11), indexing="ij")
    F = np.stack([r, c], -1).astype(np.int32)
    assert np.abs(oracle.remap_f64(X, F, 2) - X).max() < 1e-15


def test_float_remap_equals_the_uint8_remap_on_uint8_values():
    """Alg. 2 on a float image holding uint8 values / 255 equals the pinned
    uint8 remap (the same averaging, the same clamping)."""
    rng = np.random.default_rng(4)
    h, w = 17, 23
    S = rng.integers(0, 256, (h, w, 3)).astype(np.uint8)
    F = np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    assert np.abs(oracle.remap_f64(S / 255.0, F, 2) - oracle.remap(S, F, 2)).max() < 1e-13


def test_constant_styles_give_the_window_mean_with_real_fields():
    """Real PatchMatch fields: a remap of a constant frame is that constant,
    so the result is still the window mean of the constants."""
    g = synth.sprite_video(9, 24, 28, 5, n_sprites=2, side=(4, 9))
    c = np.arange(9) * 25 + 10
    s = np.ones_like(g) * c[:, None, None, None].astype(np.uint8)
    out = oracle.blend_window_fast(g, s, 3, 2, 2, 2, 7)
    assert np.abs(out - _window_mean(s, 3)).max() < 1e-12


def test_fast_mode_approximates_the_balanced_blend():
    """Eq. 4-5 are approximations, so the fast result is not the balanced
    one; it is a blend of the same window, much closer to the balanced
    result than the unblended styles are."""
    g = synth.sprite_video(8, 32, 40, 9, n_sprites=2, side=(5, 12))
    s = synth.flicker(synth.apply_lut(g, synth.random_lut(3)), 4)
    fast = oracle.blend_window_fast(g, s, 2, 2, 2, 3, 11)
    bal = oracle.blend_window(g, s, 2, 2, 2, 3, 11)
    raw = s / 255.0
    assert np.abs(fast - bal).mean() < 0.5 * np.abs(raw - bal).mean()


@pytest.mark.parametrize("M", [1, 2])
def test_two_frames_equal_the_balanced_blend(M):
    """With two frames every window is the whole video, and the tables and
    queries of Eq. 6 reduce to each frame plus the other one remapped through
    the NNF Eq. 2 uses: fast mode equals the balanced blend up to rounding."""
    g = synth.sprite_video(2, 40, 56, 3, n_sprites=2, side=(8, 20))
    s = synth.sprite_video(2, 40, 56, 4, n_sprites=2, side=(8, 20))
    a = oracle.blend_window_fast(g, s, M, 2, 2, 3, 9)
    b = oracle.blend_window(g, s, M, 2, 2, 3, 9)
    assert np.abs(a - b).max() < 1e-12
