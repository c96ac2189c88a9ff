"""Pins of the oracle's guide + style loss (Eq. 3, Section 3.4): the remapped
style S^ against the separately pinned Alg. 2 remap, the loss against the
pinned Eq. 1 SSD, special cases that reduce to the plain guide-only method,
and the per-level composition of the coarse-to-fine run."""
import numpy as np
import pytest

import oracle
from paper_2311_09265_amd import synth


def _video(n, h, w, seed):
    return synth.sprite_video(n, h, w, seed, n_sprites=2, side=(4, max(5, min(h, w) // 3)))


def _styles(guides, seed):
    rng = np.random.default_rng(seed)
    lut = np.sort(rng.integers(0, 256, (3, 256)), axis=1).astype(np.uint8)
    return np.stack([np.stack([lut[c][g[..., c]] for c in range(3)], -1) for g in guides])


def _identity(h, w):
    r, c = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    return np.stack([r, c], -1).astype(np.int32)


def test_remapped_style_is_rounded_alg2_remap():
    """S^ equals the Alg. 2 remap (pinned against the literal patch placement
    in the remap tests) rounded half up, wherever the fp64 value is not within
    rounding noise of a half."""
    rng = np.random.default_rng(1)
    h, w, p = 23, 31, 2
    S = rng.integers(0, 256, (h, w, 3)).astype(np.uint8)
    F = np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    got = oracle.remap_u8(S, F, p).astype(np.int64)
    x = oracle.remap(S, F, p) * 255.0
    want = np.floor(x + 0.5).astype(np.int64)
    ok = np.abs(x - np.floor(x) - 0.5) > 1e-7
    assert ok.mean() > 0.9
    assert np.array_equal(got[ok], want[ok])
    # exact halves round up
    assert np.all(got[~ok] == np.ceil(x[~ok] - 1e-7))
    # the identity field reproduces the image
    assert np.array_equal(oracle.remap_u8(S, _identity(h, w), p), S)


@pytest.mark.parametrize("alpha16", [1, 16, 37])
def test_constant_style_reduces_to_guide_only_patchmatch(alpha16):
    """With a constant source style, S^ is that constant, the style term is 0
    for every candidate, and Eq. 3 orders candidates exactly as Eq. 1: the
    field equals the plain method's and E = alpha16 * E_plain."""
    g = _video(2, 40, 48, 3)
    S = np.full_like(g[0], 97)
    seed, K, n = 11, 2, 3
    F, E, Sh = oracle.patchmatch_style(g[0], g[1], S, 2, K, n, seed, 5, alpha16)
    Fp, Ep = oracle.patchmatch(g[0], g[1], 2, K, n, seed, 5)
    assert np.array_equal(F, Fp)
    assert np.array_equal(E.astype(np.int64), alpha16 * Ep.astype(np.int64))
    assert np.all(Sh == 97)


@pytest.mark.parametrize("alpha16", [0, 16, 100])
def test_iteration_energy_is_the_loss_under_the_refreshed_style(alpha16):
    """One iteration: S^ is the refresh of the previous field; every returned
    E is alpha16 * SSD(G) + 16 * SSD(S, S^) at the returned match (the pinned
    Eq. 1 SSD); and no pixel ends above its incumbent's loss under that S^."""
    g = _video(2, 32, 40, 7)
    s = _styles(g, 8)
    rng = np.random.default_rng(2)
    h, w = g.shape[1:3]
    Fo = np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    Fn, En, Sh = oracle.pm_iteration_style(g[0], g[1], s[0], 2, alpha16, 0, 0, 21, 3, Fo)
    assert np.array_equal(Sh, oracle.remap_u8(s[0], Fo, 2))
    want = (alpha16 * oracle.energy(g[0], g[1], Fn, 2).astype(np.int64)
            + 16 * oracle.energy(s[0], Sh, Fn, 2).astype(np.int64))
    assert np.array_equal(En.astype(np.int64), want)
    incumbent = (alpha16 * oracle.energy(g[0], g[1], Fo, 2).astype(np.int64)
                 + 16 * oracle.energy(s[0], Sh, Fo, 2).astype(np.int64))
    assert np.all(En.astype(np.int64) <= incumbent)
    assert np.any(En.astype(np.int64) < incumbent)


def test_identity_is_a_fixed_point_of_a_frame_with_itself():
    """Matching a frame to itself from the identity field: S^ = S, the loss of
    the identity is 0, and strict '<' keeps it at every pixel."""
    g = _video(1, 24, 30, 9)[0]
    s = _styles(g[None], 4)[0]
    F0 = _identity(*g.shape[:2])
    Fn, En, Sh = oracle.pm_iteration_style(g, g, s, 2, 16, 0, 0, 5, 0, F0)
    assert np.array_equal(Sh, s)
    assert np.array_equal(Fn, F0)
    assert not En.any()


def test_ties_keep_the_incumbent():
    """Constant guides and style: every candidate has loss 0, so strict '<'
    leaves any starting field untouched (propagation and random search)."""
    h, w = 20, 26
    g = np.full((h, w, 3), 40, np.uint8)
    s = np.full((h, w, 3), 180, np.uint8)
    rng = np.random.default_rng(6)
    F0 = np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    Fn, En, _ = oracle.pm_iteration_style(g, g, s, 2, 16, 0, 0, 3, 1, F0)
    assert np.array_equal(Fn, F0)
    assert not En.any()


def test_coarse_to_fine_run_is_the_composition_of_its_steps():
    """patchmatch_style over 2 levels equals: random init at level 1 on the
    downsampled guides, iterations on the downsampled guides and style (level
    index 1), upsampling, iterations at level 0 -- so the style pyramid, the
    level numbers in the draws and the order of refresh and search are wired
    as stated."""
    g = _video(2, 36, 44, 12)
    s = _styles(g, 13)
    p, seed, pid, a16, n = 2, 77, 9, 24, 2
    F, E, Sh = oracle.patchmatch_style(g[0], g[1], s[0], p, 2, n, seed, pid, a16)
    G1 = [oracle.downsample(x) for x in (g[0], g[1], s[0])]
    Fc, _ = oracle.nnf_init_random(G1[0], G1[1], p, 1, seed, pid)
    for it in range(n):
        Fc, Ec, _ = oracle.pm_iteration_style(G1[0], G1[1], G1[2], p, a16, 1, it, seed, pid, Fc)
    Ff, _ = oracle.nnf_upsample(Fc, g[0], g[1], p)
    for it in range(n):
        Ff, Ef, Shf = oracle.pm_iteration_style(g[0], g[1], s[0], p, a16, 0, it, seed, pid, Ff)
    assert np.array_equal(F, Ff) and np.array_equal(E, Ef) and np.array_equal(Sh, Shf)


def test_blend_with_constant_styles_is_the_window_mean():
    """Eq. 2 under the Eq. 3 loss: with constant style frames every remap is
    that constant whatever the field, so each output frame is the truncated
    window mean of the constants / 255."""
    g = _video(5, 20, 24, 15)
    c = np.array([10, 60, 120, 200, 255])
    s = np.ones_like(g) * c[:, None, None, None].astype(np.uint8)
    M = 2
    out = oracle.blend_window_style(g, s, M, 2, 1, 2, 3, 16)
    for i in range(5):
        lo, hi = max(0, i - M), min(4, i + M)
        assert np.allclose(out[i], c[lo:hi + 1].mean() / 255.0, atol=1e-12)


def test_invalid_arguments_are_rejected():
    g = _video(2, 16, 16, 1)
    with pytest.raises(RuntimeError):
        oracle.patchmatch_style(g[0], g[1], g[0], 2, 1, 0, 1, 0, 16)   # no iteration
    with pytest.raises(RuntimeError):
        oracle.patchmatch_style(g[0], g[1], g[0], 2, 1, 1, 1, 0, 513)  # alpha16 out of range


# ---- the range of the scaled loss (Eq. 3; the same loss form serves Eq. 8 and Eq. 10) ----

def _saturated(h, w, seed):
    """Random 0 / 255 images: every channel difference is 0 or 255, so patch
    SSDs reach the extreme 3 * 255^2 * (2p+1)^2 where the images are complements."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 2, (h, w, 3)) * 255).astype(np.uint8)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_alpha16_bound_is_the_largest_that_fits_uint32(p):
    """The accepted alpha16 range is exactly the one for which the worst-case
    loss (alpha16 + 16) * 3 * 255^2 * (2p+1)^2, computed with Python's
    unbounded integers, is below 2^32 (or the 512 cap)."""
    worst = 3 * 255 * 255 * (2 * p + 1) ** 2
    amax = oracle.alpha16_max(p)
    assert (amax + 16) * worst < 2 ** 32
    assert amax == 512 or (amax + 17) * worst >= 2 ** 32
    assert {1: 512, 2: 512, 3: 433, 4: 255}[p] == amax


@pytest.mark.parametrize("p", [3, 4])
def test_loss_is_exact_at_the_largest_alpha16(p):
    """On saturated patches at the largest accepted alpha16 the oracle's loss
    equals alpha16 SSD(G) + 16 SSD(S, S^) evaluated with Python integers from
    an independent vectorised SSD, including the worst case (complementary
    images, every difference 255) that a uint32 sum would wrap for larger
    alpha16.  Above the bound the loss is still exact (64-bit), but the
    coarse-to-fine run rejects the parameter because energies are uint32."""
    from pins import ssd
    h, w = 13, 14
    amax = oracle.alpha16_max(p)
    Gs, Ss = _saturated(h, w, 1), _saturated(h, w, 2)
    Gt, Sh = 255 - Gs, 255 - Ss
    worst = 3 * 255 * 255 * (2 * p + 1) ** 2
    c = (6, 7)
    assert oracle.style_loss(Gs, Gt, Ss, Sh, p, amax, c, c) == (amax + 16) * worst
    assert oracle.style_loss(Gs, Gt, Ss, Sh, p, 512, c, c) == (512 + 16) * worst  # > 2^32 - 1, not wrapped
    Gt2, Sh2 = _saturated(h, w, 3), _saturated(h, w, 4)
    rng = np.random.default_rng(5)
    for _ in range(20):
        u = (int(rng.integers(0, h)), int(rng.integers(0, w)))
        v = (int(rng.integers(0, h)), int(rng.integers(0, w)))
        want = amax * ssd(Gs, Gt2, p, u, v) + 16 * ssd(Ss, Sh2, p, u, v)
        assert oracle.style_loss(Gs, Gt2, Ss, Sh2, p, amax, u, v) == want
    # the coarse-to-fine runs accept the bound and reject one more
    F, E, _ = oracle.patchmatch_style(Gs, Gt, Ss, p, 1, 1, 3, 0, amax)
    assert E.max() <= (amax + 16) * worst
    with pytest.raises(RuntimeError):
        oracle.patchmatch_style(Gs, Gt, Ss, p, 1, 1, 3, 0, amax + 1)
    with pytest.raises(RuntimeError):
        oracle.patchmatch_target(Gs, Gt, Ss, Sh, p, 1, 1, 3, 0, amax + 1)
    with pytest.raises(ValueError):
        oracle.pm_iteration_style(Gs, Gt, Ss, p, amax + 1, 0, 0, 3, 0, F)


@pytest.mark.parametrize("p", [3, 4])
def test_saturated_run_at_the_bound_keeps_exact_energies(p):
    """A whole Eq. 3 run at the largest alpha16 on saturated data: every
    energy equals alpha16 SSD(G) + 16 SSD(S, S^) of its match, computed with
    Python integers from the independent SSD and the final refresh S^."""
    from pins import energy
    h, w = 15, 17
    amax = oracle.alpha16_max(p)
    Gs, Gt, Ss = _saturated(h, w, 11), _saturated(h, w, 12), _saturated(h, w, 13)
    F, E, Sh = oracle.patchmatch_style(Gs, Gt, Ss, p, 1, 2, 9, 4, amax)
    want = amax * energy(Gs, Gt, F, p) + 16 * energy(Ss, Sh, F, p)
    assert want.max() < 2 ** 32
    assert np.array_equal(E.astype(np.int64), want)
