"""Pins of the oracle's PatchMatch (Alg. 1, Section 3.2) against what the paper
and the mathematics fix: brute-force exhaustive NNFs, exact recovery of
integer translations, per-iteration monotonicity, the direction of
propagation and the concurrent (Jacobi) update.
"""
import numpy as np
import pytest

import pins
from paper_2311_09265_amd import synth


def _iterate(orc, S, T, p, level, n, seed, pair, F, E, collect=False):
    hist = []
    for it in range(n):
        F, E = orc.pm_iteration(S, T, p, level, it, seed, pair, F, E)
        if collect:
            hist.append((F, E))
    return (F, E, hist) if collect else (F, E)


def test_energy_non_increasing_and_consistent(orc):
    S = synth.value_noise(40, 36, 5)
    T = synth.value_noise(40, 36, 6)
    F, E = orc.nnf_init_random(S, T, 2, 0, 99, 3)
    prevE = E.copy()
    for it in range(6):
        F, E = orc.pm_iteration(S, T, 2, 0, it, 99, 3, F, E)
        assert (E <= prevE).all(), it          # F(E' < E) <- F' never raises a pixel's loss
        assert np.array_equal(E.astype(np.int64), pins.energy(S, T, F, 2))
        prevE = E.copy()
    assert E.mean() < 0.5 * pins.energy(S, T, orc.nnf_init_random(S, T, 2, 0, 99, 3)[0], 2).mean()


def test_never_below_brute_force_and_reaches_it_on_tiny_frames(orc):
    """E >= the exhaustive minimum everywhere (it is a real patch loss).  On a
    coherent tiny pair (four translated blocks: rows and columns cyclically
    rotated) 30 iterations reach the exhaustive minimum on >= 95% of pixels."""
    hits = []
    for seed in range(3):
        S = pins.noise_image(16, 16, 100 + seed)
        U = pins.noise_image(16, 16, 200 + seed)          # unrelated: incoherent NNF
        T = np.roll(np.roll(S, -8, axis=1), -5, axis=0)   # coherent: block translations
        for tgt, need in ((U, None), (T, 0.95)):
            Fb, Eb = pins.brute_force_nnf(S, tgt, 2)
            F, E = orc.nnf_init_random(S, tgt, 2, 0, seed, 0)
            F, E = _iterate(orc, S, tgt, 2, 0, 30, seed, 0, F, E)
            assert (E.astype(np.int64) >= Eb).all()
            assert np.array_equal(E.astype(np.int64), pins.energy(S, tgt, F, 2))
            if need is not None:
                hits.append((E.astype(np.int64) == Eb).mean())
    assert np.mean(hits) >= 0.95, hits


@pytest.mark.parametrize("shift", [(3, -2), (-2, 3), (5, 4)])
def test_exact_translation_recovery(orc, shift):
    """T(r,c) = S(r - dr, c - dc) on uniform noise: interior pixels reach F(v) = v - shift, E = 0.

    That answer is also what exhaustive search returns (checked on a crop).
    """
    dr, dc = shift
    canvas = pins.noise_image(80, 80, 7)
    S = canvas[8:72, 8:72]
    T = canvas[8 - dr:72 - dr, 8 - dc:72 - dc]
    F, E = orc.patchmatch(S, T, 2, 2, 16, 17, 5)   # Jacobi needs enough iterations to converge
    rr, cc = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    p = 2
    inner = ((rr - dr >= p) & (rr - dr < 64 - p) & (cc - dc >= p) & (cc - dc < 64 - p)
             & (rr >= p) & (rr < 64 - p) & (cc >= p) & (cc < 64 - p))
    ok = (F[..., 0] == rr - dr) & (F[..., 1] == cc - dc) & (E == 0)
    assert ok[inner].mean() == 1.0, ok[inner].mean()
    n = 24
    Fb, Eb = pins.brute_force_nnf(S[:n, :n], T[:n, :n], 2)
    r2, c2 = rr[:n, :n], cc[:n, :n]
    sub = ((r2 - dr >= p) & (r2 - dr < n - p) & (c2 - dc >= p) & (c2 - dc < n - p)
           & (r2 >= p) & (r2 < n - p) & (c2 >= p) & (c2 < n - p))
    assert (Eb[sub] == 0).all()
    assert (Fb[..., 0][sub] == (r2 - dr)[sub]).all() and (Fb[..., 1][sub] == (c2 - dc)[sub]).all()


def test_propagation_repairs_a_single_wrong_pixel(orc):
    """With the field right everywhere but one pixel, one iteration repairs it via
    F'(v) = F(v + d) - d -- a flipped sign or axis in propagation would not."""
    canvas = pins.noise_image(72, 72, 8)
    dr, dc = 2, -3
    S = canvas[4:68, 4:68]
    T = canvas[4 - dr:68 - dr, 4 - dc:68 - dc]
    rr, cc = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    F = np.stack([np.clip(rr - dr, 0, 63), np.clip(cc - dc, 0, 63)], -1).astype(np.int32)
    for v in [(30, 30), (10, 50), (50, 12)]:
        Fw = F.copy()
        Fw[v] = (63 - v[0], 5)  # far from the right match
        Ew = orc.energy(S, T, Fw, 2)
        assert Ew[v] > 0
        for seed in range(4):
            F1, E1 = orc.pm_iteration(S, T, 2, 0, 0, seed, 0, Fw, Ew)
            assert tuple(F1[v]) == (v[0] - dr, v[1] - dc) and E1[v] == 0


def test_update_is_concurrent_not_in_scan_order(orc):
    """Seeding the right match at one pixel, the right region grows by one pixel
    (in L1 distance) per iteration, as every pixel reads only the previous field.
    A scan-order (in-place) update would carry it across the image in one pass."""
    canvas = pins.noise_image(72, 72, 9)
    dr, dc = 1, 2
    S = canvas[4:68, 4:68]
    T = canvas[4 - dr:68 - dr, 4 - dc:68 - dc]
    rng = np.random.default_rng(0)
    F = np.stack([rng.integers(0, 64, (64, 64)), rng.integers(0, 64, (64, 64))], -1).astype(np.int32)
    c0 = (32, 32)
    F[c0] = (c0[0] - dr, c0[1] - dc)
    E = orc.energy(S, T, F, 2)
    rr, cc = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    dist = np.abs(rr - c0[0]) + np.abs(cc - c0[1])
    for it in range(3):
        F, E = orc.pm_iteration(S, T, 2, 0, it, 5, 1, F, E)
        right = (F[..., 0] == rr - dr) & (F[..., 1] == cc - dc)
        k = it + 1
        assert right[dist <= k].all(), it          # the diamond of radius k is reached
        far = dist > k + 1
        # only random hits (and their own growth) beyond it; a scan-order pass would
        # already have carried the match over the whole lower-right part of the image
        assert right[far].mean() < 0.1, (it, right[far].mean())


def test_update_reads_only_the_previous_field_of_the_4_neighbourhood(orc):
    """Two fields that agree on a block give identical results after one iteration
    at every pixel whose 4-neighbourhood lies in the block (concurrent update)."""
    S = synth.value_noise(48, 48, 21)
    T = synth.value_noise(48, 48, 22)
    rng = np.random.default_rng(3)
    Fa = np.stack([rng.integers(0, 48, (48, 48)), rng.integers(0, 48, (48, 48))], -1).astype(np.int32)
    Fb = np.stack([rng.integers(0, 48, (48, 48)), rng.integers(0, 48, (48, 48))], -1).astype(np.int32)
    block = np.zeros((48, 48), bool)
    block[10:30, 14:40] = True
    Fb[block] = Fa[block]
    Ea, Eb = orc.energy(S, T, Fa, 2), orc.energy(S, T, Fb, 2)
    Fa1, Ea1 = orc.pm_iteration(S, T, 2, 0, 0, 8, 2, Fa, Ea)
    Fb1, Eb1 = orc.pm_iteration(S, T, 2, 0, 0, 8, 2, Fb, Eb)
    core = np.zeros((48, 48), bool)
    core[11:29, 15:39] = True
    assert np.array_equal(Fa1[core], Fb1[core]) and np.array_equal(Ea1[core], Eb1[core])
    assert (Fa1[~block] != Fb1[~block]).any()


def test_config1_translation_with_noise(orc):
    """Value-noise pair shifted by (3,-2) plus U{-4..4} noise (the 64x64 workload).
    At the true shift the expected energy is 75 * E[n^2] = 75 * 60/9 = 500."""
    A, B, _ = synth.translation_pair(synth.CONFIG_SEED[1])
    rr, cc = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    inner = (rr >= 5) & (rr < 62) & (cc >= 2) & (cc < 59)
    true_e = pins.energy(A, B, np.stack([np.clip(rr - 3, 0, 63), np.clip(cc + 2, 0, 63)], -1), 2)
    assert abs(true_e[inner].mean() - 500) < 40
    # the workload's 5 iterations: most interior pixels already hold the true shift
    F, E = orc.patchmatch(A, B, 2, 1, 5, synth.PHILOX_SEED[1], 0)
    hold = (F[..., 0] == rr - 3) & (F[..., 1] == cc + 2)
    assert hold[inner].mean() > 0.9
    assert (E[hold] == true_e[hold]).all()
    # run longer and every interior pixel converges to it
    F, E = orc.patchmatch(A, B, 2, 1, 12, synth.PHILOX_SEED[1], 0)
    hold = (F[..., 0] == rr - 3) & (F[..., 1] == cc + 2)
    assert hold[inner].all() and (E[inner] <= true_e[inner]).all()


def test_pyramid_path_matches_per_level_composition(orc):
    """fbo_patchmatch == composing downsample / init / iterate / upsample by hand (Alg. 1 order)."""
    S = synth.value_noise(45, 38, 11)
    T = synth.value_noise(45, 38, 12)
    K, n, seed, pair = 3, 3, 77, 9
    F, E = orc.patchmatch(S, T, 2, K, n, seed, pair)
    Sp, Tp = orc.pyramid(S, K), orc.pyramid(T, K)
    Fl, El = orc.nnf_init_random(Sp[K - 1], Tp[K - 1], 2, K - 1, seed, pair)
    for l in range(K - 1, -1, -1):
        if l < K - 1:
            Fl, El = orc.nnf_upsample(Fl, Sp[l], Tp[l], 2)
        Fl, El = _iterate(orc, Sp[l], Tp[l], 2, l, n, seed, pair, Fl, El)
    assert np.array_equal(F, Fl) and np.array_equal(E, El)


def test_seeded_init_with_true_shift(orc):
    """An offset field seeding the coarsest level (instead of the random draw)
    that holds the true shift carries it to level 0 through upsampling."""
    canvas = pins.noise_image(72, 72, 12)
    S = canvas[3:67, 3:67]
    T = canvas[1:65, 7:71]   # T(r,c) = S(r-2, c+4)
    off = np.zeros((32, 32, 2), np.int32)
    off[..., 0] = -1
    off[..., 1] = 2          # the shift at half resolution
    F, E = orc.patchmatch(S, T, 2, 2, 2, 1, 0, seed_offsets=off)
    rr, cc = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    inner = (rr >= 4) & (rr < 62) & (cc >= 2) & (cc < 58)
    assert ((F[..., 0] == rr - 2) & (F[..., 1] == cc + 4))[inner].all()
    assert (E[inner] == 0).all()


def test_ties_keep_the_incumbent(orc):
    """The update F(E' < E) <- F' is strict: on a constant image pair every
    candidate ties at loss 0, so iterations never move the field."""
    S = np.full((24, 30, 3), 90, np.uint8)
    F, E = orc.nnf_init_random(S, S, 2, 0, 4, 1)
    assert (E == 0).all()
    F1, E1 = F, E
    for it in range(3):
        F1, E1 = orc.pm_iteration(S, S, 2, 0, it, 4, 1, F1, E1)
    assert np.array_equal(F1, F) and (E1 == 0).all()
