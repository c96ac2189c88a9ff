"""Pins of the oracle's convergence guard for seeded PatchMatch (a project
addition that protects the learned seed; the paper's Alg. 1 starts from
random fields).

The rule: at the finest level, with P the summed energy before the last
iteration and C after it, one more iteration runs (with the next iteration
index) while 100 (P - C) > tau_pct P, at most max_extra times.  The guard is
checked against that rule restated here on top of the pinned single
iteration, init and upsample, and by its behaviour: it stays silent when the
seed is already right, fires on a bad seed, and then only lowers the energy.
"""
import numpy as np
import pytest

import pins
from paper_2311_09265_amd import synth


def _by_rule(orc, S, T, p, levels, iters, seed, pair, off, max_extra, tau):
    """The guarded run composed from the oracle's pinned steps, the rule in
    Python integers."""
    Sl, Tl = orc.pyramid(S, levels), orc.pyramid(T, levels)
    F = E = None
    for l in range(levels - 1, -1, -1):
        if l == levels - 1:
            F, E = orc.nnf_init_offsets(Sl[l], Tl[l], p, off)
        else:
            F, E = orc.nnf_upsample(F, Sl[l], Tl[l], p)
        prev = E
        for it in range(iters):
            prev = E
            F, E = orc.pm_iteration(Sl[l], Tl[l], p, l, it, seed, pair, F, E)
    P, C = int(prev.astype(np.int64).sum()), int(E.astype(np.int64).sum())
    extra = 0
    while extra < max_extra and 100 * (P - C) > tau * P:
        F, E = orc.pm_iteration(Sl[0], Tl[0], p, 0, iters + extra, seed, pair, F, E)
        P, C = C, int(E.astype(np.int64).sum())
        extra += 1
    return F, E, extra


def _pair(h=48, w=64, seed=3):
    v = synth.sprite_video(4, h, w, seed, n_sprites=3, side=(8, 20))
    return v[0], v[3]


@pytest.mark.parametrize("levels,iters,tau", [(2, 1, 1), (3, 2, 1), (1, 2, 5), (2, 2, 0)])
def test_guard_follows_its_rule(orc, levels, iters, tau):
    S, T = _pair()
    hc, wc = -(-48 // (1 << (levels - 1))), -(-64 // (1 << (levels - 1)))
    off = np.zeros((hc, wc, 2), np.int32)
    F, E, extra = orc.patchmatch_guarded(S, T, 2, levels, iters, 77, 5, off, 4, tau)
    Fr, Er, xr = _by_rule(orc, S, T, 2, levels, iters, 77, 5, off, 4, tau)
    assert extra == xr
    assert np.array_equal(F, Fr) and np.array_equal(E, Er)
    assert np.array_equal(E.astype(np.int64), pins.energy(S, T, F, 2))


def test_guard_off_equals_plain_seeded_run(orc):
    S, T = _pair()
    off = np.random.default_rng(1).integers(-3, 4, (24, 32, 2)).astype(np.int32)
    F0, E0 = orc.patchmatch(S, T, 2, 2, 2, 9, 1, seed_offsets=off)
    F, E, extra = orc.patchmatch_guarded(S, T, 2, 2, 2, 9, 1, off, max_extra=0)
    assert extra == 0 and np.array_equal(F, F0) and np.array_equal(E, E0)


def test_guard_is_silent_on_a_converged_seed(orc):
    """Seeded with the exact translation of a shifted noise pair (1 level),
    the interior is right from the start and 6 iterations settle the border:
    the last iteration lowers the summed energy by at most tau, no extra
    iteration runs, and the result is the unguarded one."""
    canvas = pins.noise_image(72, 72, 5)
    S, T = canvas[4:68, 4:68], canvas[1:65, 6:70]   # T(r, c) = S(r - 3, c + 2)
    off = np.zeros((64, 64, 2), np.int32)
    off[..., 0], off[..., 1] = -3, 2
    Sl, Tl = orc.pyramid(S, 1), orc.pyramid(T, 1)
    F, E = orc.nnf_init_offsets(Sl[0], Tl[0], 2, off)
    sums = [int(E.astype(np.int64).sum())]
    for it in range(6):
        F, E = orc.pm_iteration(Sl[0], Tl[0], 2, 0, it, 21, 0, F, E)
        sums.append(int(E.astype(np.int64).sum()))
    assert 100 * (sums[-2] - sums[-1]) <= sums[-2]      # the case: the last drop is within 1%
    F0, E0 = orc.patchmatch(S, T, 2, 1, 6, 21, 0, seed_offsets=off)
    F, E, extra = orc.patchmatch_guarded(S, T, 2, 1, 6, 21, 0, off)
    assert extra == 0 and np.array_equal(F, F0) and np.array_equal(E, E0)


def test_guard_fires_on_a_bad_seed_and_only_lowers_energy(orc):
    """A zero offset field on a pair with moving sprites leaves the finest
    level far from converged after 2 iterations: the guard adds iterations,
    and every pixel's energy is at most the unguarded one."""
    S, T = _pair(64, 64, 11)
    off = np.zeros((16, 16, 2), np.int32)
    F0, E0 = orc.patchmatch(S, T, 2, 3, 2, 31, 2, seed_offsets=off)
    F, E, extra = orc.patchmatch_guarded(S, T, 2, 3, 2, 31, 2, off, 4, 1)
    assert extra >= 1
    assert (E <= E0).all() and E.astype(np.int64).sum() < E0.astype(np.int64).sum()
