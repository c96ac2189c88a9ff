"""Pins of the oracle's guard of a seeded run (a project addition that protects
the learned seed; the paper's Alg. 1 starts from random fields).

The rule: at the coarsest level the seeded start followed by `iters`
iterations races the random start followed by one more iteration,
min(iters + 1, plain_iters).  If the seeded level's summed energy is the
larger, the seed is rejected and the whole result is the plain run
(plain_iters iterations at every level); otherwise it is the seeded run.  The guard is
checked against that rule restated here on top of the pinned init and single
iteration, and by its behaviour: a seed that is the pair's true motion is
kept, a random seed is rejected, and a rejected run is the plain run exactly.
"""
import numpy as np
import pytest

import pins
from paper_2311_09265_amd import synth


def _coarse_sum(orc, S, T, p, levels, iters, seed, pair, off):
    """Summed energy of the coarsest level after `iters` iterations from the
    seeded (off) or random (off None) start, composed from the pinned steps."""
    l = levels - 1
    Sl, Tl = orc.pyramid(S, levels)[l], orc.pyramid(T, levels)[l]
    if off is None:
        F, E = orc.nnf_init_random(Sl, Tl, p, l, seed, pair)
    else:
        F, E = orc.nnf_init_offsets(Sl, Tl, p, off)
    for it in range(iters):
        F, E = orc.pm_iteration(Sl, Tl, p, l, it, seed, pair, F, E)
    assert np.array_equal(E.astype(np.int64), pins.energy(Sl, Tl, F, p))
    return int(E.astype(np.int64).sum())


def _pair(h=48, w=64, seed=3):
    v = synth.sprite_video(4, h, w, seed, n_sprites=3, side=(8, 20))
    return v[0], v[3]


def _coarse(h, w, levels):
    return -(-h // (1 << (levels - 1))), -(-w // (1 << (levels - 1)))


@pytest.mark.parametrize("levels,iters,plain_iters,amp", [(2, 1, 3, 2), (3, 2, 6, 9), (1, 2, 5, 30), (2, 2, 2, 0)])
def test_guard_follows_its_rule(orc, levels, iters, plain_iters, amp):
    S, T = _pair()
    hc, wc = _coarse(48, 64, levels)
    off = np.random.default_rng(amp).integers(-amp, amp + 1, (hc, wc, 2)).astype(np.int32)
    F, E, rej, sums = orc.patchmatch_raced(S, T, 2, levels, iters, plain_iters, 77, 5, off)
    ss = _coarse_sum(orc, S, T, 2, levels, iters, 77, 5, off)
    sp = _coarse_sum(orc, S, T, 2, levels, min(iters + 1, plain_iters), 77, 5, None)
    assert sums == (ss, sp)
    assert rej == (ss > sp)
    if rej:
        Fr, Er = orc.patchmatch(S, T, 2, levels, plain_iters, 77, 5)
    else:
        Fr, Er = orc.patchmatch(S, T, 2, levels, iters, 77, 5, seed_offsets=off)
    assert np.array_equal(F, Fr) and np.array_equal(E, Er)
    assert np.array_equal(E.astype(np.int64), pins.energy(S, T, F, 2))


def test_guard_keeps_the_true_motion(orc):
    """A shifted noise pair seeded with its exact translation: the seeded
    coarse level is already at its minimum in the interior, so it beats the
    random start at any iteration count and the seeded run is kept."""
    canvas = pins.noise_image(88, 88, 5)
    S, T = canvas[8:72, 8:80], canvas[5:69, 10:82]   # T(r, c) = S(r - 3, c + 2)
    levels = 1
    off = np.zeros((64, 72, 2), np.int32)
    off[..., 0], off[..., 1] = -3, 2
    F, E, rej, (ss, sp) = orc.patchmatch_raced(S, T, 2, levels, 2, 6, 21, 0, off)
    assert not rej and ss < sp
    F0, E0 = orc.patchmatch(S, T, 2, levels, 2, 21, 0, seed_offsets=off)
    assert np.array_equal(F, F0) and np.array_equal(E, E0)
    # the interior holds the true shift with zero energy (Sec. 3.2: E = 0 at an exact match)
    inner = (slice(5, 59), slice(4, 66))
    assert (F[inner][..., 0] == np.arange(64)[inner[0], None] - 3).all()
    assert (E[inner] == 0).all()


def test_guard_rejects_a_random_seed_for_the_plain_run(orc):
    """Offsets drawn at random over the whole coarse level lose the race: the
    result is the plain random-start run with plain_iters iterations, exactly."""
    S, T = _pair(64, 80, 11)
    hc, wc = _coarse(64, 80, 3)
    rng = np.random.default_rng(4)
    off = np.stack([rng.integers(-hc, hc, (hc, wc)), rng.integers(-wc, wc, (hc, wc))], -1).astype(np.int32)
    F, E, rej, (ss, sp) = orc.patchmatch_raced(S, T, 2, 3, 2, 6, 31, 2, off)
    assert rej and ss > sp
    F0, E0 = orc.patchmatch(S, T, 2, 3, 6, 31, 2)
    assert np.array_equal(F, F0) and np.array_equal(E, E0)


def test_guard_with_equal_sums_keeps_the_seed(orc):
    """Ties go to the seed (strict '>'): seeding with the plain run's own
    coarsest-level field and running as many iterations as the race gives the
    plain start (plain_iters = iters, so the race runs iters) reproduces the
    plain coarse level exactly (the random start is only the draw at the
    start), so both sums are equal."""
    S, T = _pair()
    levels, it = 2, 3
    l = levels - 1
    Sl, Tl = orc.pyramid(S, levels)[l], orc.pyramid(T, levels)[l]
    F, E = orc.nnf_init_random(Sl, Tl, 2, l, 9, 1)
    hc, wc = Sl.shape[:2]
    off = F - np.stack(np.meshgrid(np.arange(hc), np.arange(wc), indexing="ij"), -1).astype(np.int32)
    Fs, Es, rej, (ss, sp) = orc.patchmatch_raced(S, T, 2, levels, it, it, 9, 1, off)
    assert ss == sp and not rej
