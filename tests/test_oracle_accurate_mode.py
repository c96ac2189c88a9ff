"""Pins of the oracle's accurate mode (Eq. 7-8, Section 3.4): the averaged
remap T^- against the pinned balanced blend, the Eq. 8 loss against the
pinned SSD and the plain method, and the composition of the whole mode."""
import numpy as np
import pytest

import oracle
from paper_2311_09265_amd import synth


def _video(N, h, w, seed):
    g = synth.sprite_video(N, h, w, seed, n_sprites=2, side=(4, max(5, min(h, w) // 3)))
    s = synth.flicker(synth.apply_lut(g, synth.random_lut(seed ^ 5)), seed ^ 9)
    return g, s


def test_tbar_is_the_rounded_balanced_blend():
    """T^- of every frame equals the balanced blend (Eq. 2 with the Eq. 1
    NNFs, pinned separately) x 255 rounded half up, away from exact halves."""
    g, s = _video(6, 28, 34, 3)
    M, K, n, seed = 2, 2, 2, 13
    _, tb = oracle.blend_window_accurate(g, s, M, 2, K, n, seed, 16, return_tbar=True)
    x = oracle.blend_window(g, s, M, 2, K, n, seed) * 255.0
    ok = np.abs(x - np.floor(x) - 0.5) > 1e-6
    assert ok.mean() > 0.9
    assert np.array_equal(tb[ok].astype(np.int64), np.floor(x[ok] + 0.5).astype(np.int64))
    assert np.all(tb[~ok] == np.ceil(x[~ok] - 1e-6))


@pytest.mark.parametrize("alpha16", [1, 16])
def test_constant_style_and_target_reduce_to_the_plain_method(alpha16):
    g, _ = _video(2, 36, 40, 5)
    S = np.full_like(g[0], 120)
    F, E = oracle.patchmatch_target(g[0], g[1], S, S, 2, 2, 3, 7, 4, alpha16)
    Fp, Ep = oracle.patchmatch(g[0], g[1], 2, 2, 3, 7, 4)
    assert np.array_equal(F, Fp)
    assert np.array_equal(E.astype(np.int64), alpha16 * Ep.astype(np.int64))


def test_iteration_energy_is_the_eq8_loss():
    g, s = _video(2, 30, 36, 8)
    rng = np.random.default_rng(1)
    h, w = g.shape[1:3]
    Tb = rng.integers(0, 256, (h, w, 3)).astype(np.uint8)
    Fo = np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    Fn, En = oracle.pm_iteration_target(g[0], g[1], s[0], Tb, 2, 24, 0, 1, 9, 2, Fo)
    want = 24 * oracle.energy(g[0], g[1], Fn, 2).astype(np.int64) + 16 * oracle.energy(s[0], Tb, Fn, 2).astype(np.int64)
    assert np.array_equal(En.astype(np.int64), want)
    inc = 24 * oracle.energy(g[0], g[1], Fo, 2).astype(np.int64) + 16 * oracle.energy(s[0], Tb, Fo, 2).astype(np.int64)
    assert np.all(En.astype(np.int64) <= inc) and np.any(En.astype(np.int64) < inc)


def test_accurate_blend_is_the_composition_of_its_steps():
    g, s = _video(5, 24, 30, 11)
    N, M, K, n, seed, a16 = 5, 1, 2, 2, 3, 16
    out, tb = oracle.blend_window_accurate(g, s, M, 2, K, n, seed, a16, return_tbar=True)
    for i in range(N):
        js = [j for j in range(max(0, i - M), min(N - 1, i + M) + 1) if j != i]
        F1 = [oracle.patchmatch(g[j], g[i], 2, K, n, seed, j * N + i)[0] for j in js]
        tbi = oracle.window_mean_u8(s, i, js, F1, 2)
        assert np.array_equal(tbi, tb[i])
        acc = s[i] / 255.0
        for j in js:
            F2, _ = oracle.patchmatch_target(g[j], g[i], s[j], tbi, 2, K, n, seed, j * N + i, a16)
            acc = acc + oracle.remap(s[j], F2, 2)
        assert np.abs(out[i] - acc / (len(js) + 1)).max() < 1e-12


def test_constant_styles_give_the_window_mean():
    g, _ = _video(6, 20, 26, 2)
    c = np.array([5, 50, 90, 140, 200, 250])
    s = np.ones_like(g) * c[:, None, None, None].astype(np.uint8)
    out = oracle.blend_window_accurate(g, s, 2, 2, 1, 2, 3, 16)
    for i in range(6):
        lo, hi = max(0, i - 2), min(5, i + 2)
        assert np.allclose(out[i], c[lo:hi + 1].mean() / 255.0, atol=1e-12)


def test_ties_keep_the_incumbent():
    h, w = 18, 22
    g = np.full((h, w, 3), 70, np.uint8)
    s = np.full((h, w, 3), 30, np.uint8)
    tb = np.full((h, w, 3), 30, np.uint8)
    rng = np.random.default_rng(5)
    F0 = np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    Fn, En = oracle.pm_iteration_target(g, g, s, tb, 2, 16, 0, 0, 3, 1, F0)
    assert np.array_equal(Fn, F0) and not En.any()


def test_coarse_to_fine_target_run_is_the_composition_of_its_steps():
    """Two levels: the guides, the source style and T^- are all downsampled
    with the pyramid filter for level 1."""
    g, s = _video(2, 36, 44, 17)
    rng = np.random.default_rng(3)
    tb = rng.integers(0, 256, g[0].shape).astype(np.uint8)
    p, seed, pid, a16, n = 2, 41, 6, 20, 2
    F, E = oracle.patchmatch_target(g[0], g[1], s[0], tb, p, 2, n, seed, pid, a16)
    D = [oracle.downsample(x) for x in (g[0], g[1], s[0], tb)]
    Fc, _ = oracle.nnf_init_random(D[0], D[1], p, 1, seed, pid)
    for it in range(n):
        Fc, _ = oracle.pm_iteration_target(D[0], D[1], D[2], D[3], p, a16, 1, it, seed, pid, Fc)
    Ff, _ = oracle.nnf_upsample(Fc, g[0], g[1], p)
    for it in range(n):
        Ff, Ef = oracle.pm_iteration_target(g[0], g[1], s[0], tb, p, a16, 0, it, seed, pid, Ff)
    assert np.array_equal(F, Ff) and np.array_equal(E, Ef)
