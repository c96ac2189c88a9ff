"""Pins of the oracle's interpolation extras (Section 3.5): tracking (the
neighbouring target frames' matches as candidates) and the pairwise
alignment loss (Eq. 10), both with the pairs estimated jointly."""
import numpy as np
import pytest

import oracle
from paper_2311_09265_amd import synth


def _interp_video(N, h, w, seed):
    g = synth.sprite_video(N, h, w, seed, n_sprites=2, side=(4, max(5, min(h, w) // 3)))
    return g


def test_no_option_equals_the_plain_interpolation():
    g = _interp_video(9, 24, 30, 2)
    keys = np.array([0, 4, 8])
    ks = synth.apply_lut(g[keys], synth.random_lut(4))
    a = oracle.interpolate_ext(g, keys, ks, 2, 2, 2, 5)
    b = oracle.interpolate(g, keys, ks, 2, 2, 2, 5)
    assert np.abs(a - b).max() < 1e-15


def _shift_setup(seed=3, h=28, w=34, a=3, b=-2):
    canvas = synth.value_noise(h + 16, w + 16, seed)
    S = np.ascontiguousarray(canvas[8:8 + h, 8:8 + w])
    T = np.ascontiguousarray(canvas[8 - a:8 - a + h, 8 - b:8 - b + w])   # T(v) = S(v - (a, b))
    r, c = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    exact = np.stack([np.clip(r - a, 0, h - 1), np.clip(c - b, 0, w - 1)], -1).astype(np.int32)
    inner = (r - a >= 2) & (r - a < h - 2) & (c - b >= 2) & (c - b < w - 2) & (r >= 2) & (r < h - 2) & (c >= 2) & (c < w - 2)
    return S, T, exact, inner


@pytest.mark.parametrize("side", ["prev", "next"])
def test_tracking_takes_the_neighbouring_frames_match(side):
    """Pair q = (key, frame i), its neighbour holds the exact translation
    (loss 0 in the interior) while q starts from a random field: one
    iteration with tracking gives loss 0 at every interior pixel, with the
    neighbour's match taken as is; without tracking it does not."""
    S, T, exact, inner = _shift_setup()
    h, w = S.shape[:2]
    rng = np.random.default_rng(1)
    Fq = np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    fields = [Fq, exact]
    energies = [oracle.energy(S, T, Fq, 2), oracle.energy(S, T, exact, 2)]
    kw = {"prev": 1} if side == "prev" else {"nxt": 1}
    Fn, En = oracle.pm_iteration_ext(S, T, S, S, 2, 16, oracle.TRACK, 0, 0, 9, 1, fields, energies, 0, **kw)
    assert not En[inner].any()
    assert np.array_equal(Fn[inner], exact[inner])
    F0, E0 = oracle.pm_iteration_ext(S, T, S, S, 2, 16, 0, 0, 0, 9, 1, fields, energies, 0, **kw)
    assert E0[inner].any()


def _patch_ssd_field(A, B, FA, FB, p):
    h, w = FA.shape[:2]
    out = np.zeros((h, w), np.int64)
    for r in range(h):
        for c in range(w):
            out[r, c] = oracle.patch_ssd(A, B, p, FA[r, c], FB[r, c])
    return out


def test_alignment_energy_is_the_pairwise_loss():
    """En = alpha16 SSD(G_a[F], G_i[v]) + 16 SSD(S_a[F], S_b[F_b(v)]), with the
    partner's previous field F_b; no pixel ends above its re-scored
    incumbent."""
    g = _interp_video(3, 16, 20, 6)
    rng = np.random.default_rng(2)
    Sa = rng.integers(0, 256, g[0].shape).astype(np.uint8)
    Sb = rng.integers(0, 256, g[0].shape).astype(np.uint8)
    h, w = g.shape[1:3]
    rf = lambda: np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    Fa, Fb = rf(), rf()
    Ea, Eb = oracle.energy(g[0], g[1], Fa, 2), oracle.energy(g[2], g[1], Fb, 2)
    a16 = 24
    Fn, En = oracle.pm_iteration_ext(g[0], g[1], Sa, Sb, 2, a16, oracle.ALIGN, 0, 0, 4, 1, [Fa, Fb], [Ea, Eb], 0,
                                     partner=1)
    r, c = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    V = np.stack([r, c], -1)
    want = a16 * oracle.energy(g[0], g[1], Fn, 2).astype(np.int64) + 16 * _patch_ssd_field(Sa, Sb, Fn, Fb, 2)
    assert np.array_equal(En.astype(np.int64), want)
    inc = a16 * oracle.energy(g[0], g[1], Fa, 2).astype(np.int64) + 16 * _patch_ssd_field(Sa, Sb, Fa, Fb, 2)
    assert np.all(En.astype(np.int64) <= inc) and np.any(En.astype(np.int64) < inc)
    del V


def test_constant_keyframe_styles_reduce_alignment_to_the_plain_iteration():
    g = _interp_video(3, 20, 24, 8)
    S = np.full_like(g[0], 77)
    rng = np.random.default_rng(5)
    h, w = g.shape[1:3]
    Fa = np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    Fb = np.stack([rng.integers(0, h, (h, w)), rng.integers(0, w, (h, w))], -1).astype(np.int32)
    Ea = oracle.energy(g[0], g[1], Fa, 2)
    Eb = oracle.energy(g[2], g[1], Fb, 2)
    Fn, En = oracle.pm_iteration_ext(g[0], g[1], S, S, 2, 16, oracle.ALIGN, 0, 2, 7, 3, [Fa, Fb], [Ea, Eb], 0,
                                     partner=1)
    Fp, Ep = oracle.pm_iteration(g[0], g[1], 2, 0, 2, 7, 3, Fa, Ea)
    assert np.array_equal(Fn, Fp)
    assert np.array_equal(En.astype(np.int64), 16 * Ep.astype(np.int64))


@pytest.mark.parametrize("track,align", [(True, False), (False, True), (True, True)])
def test_constant_keys_give_the_eq9_weights(track, align):
    g = _interp_video(9, 20, 24, 11)
    keys = np.array([1, 5, 8])
    cols = np.array([30, 130, 230])
    ks = np.ones((3,) + g.shape[1:], np.uint8) * cols[:, None, None, None].astype(np.uint8)
    out = oracle.interpolate_ext(g, keys, ks, 2, 2, 2, 3, 16, track=track, align=align)
    for i in range(9):
        if i in keys:
            want = cols[list(keys).index(i)]
        elif i < 1:
            want = cols[0]
        elif i < 5:
            want = ((5 - i) * cols[0] + (i - 1) * cols[1]) / 4
        else:
            want = ((8 - i) * cols[1] + (i - 5) * cols[2]) / 3
        assert np.allclose(out[i], want / 255.0, atol=1e-12), i


def test_invalid_arguments_are_rejected():
    g = _interp_video(4, 16, 16, 1)
    ks = g[[0, 3]]
    with pytest.raises(RuntimeError):
        oracle.interpolate_ext(g, np.array([0, 3]), ks, 2, 1, 0, 1, 16, align=True)   # no iteration
    with pytest.raises(RuntimeError):
        oracle.interpolate_ext(g, np.array([0, 3]), ks, 2, 1, 1, 1, 0, align=True)    # alpha16 < 1


def test_joint_run_is_the_lockstep_composition():
    """One level, tracking + alignment: the joint estimation equals pairs
    initialised by their own draws and iterated in lockstep, each reading
    the previous fields of its neighbours (same key, adjacent frames) and of
    its partner (same frame, the other key), then Eq. 9."""
    g = _interp_video(7, 18, 22, 13)
    keys = [0, 3, 6]
    ks = synth.apply_lut(g[keys], synth.random_lut(7))
    N, p, n, seed, a16 = 7, 2, 2, 9, 20
    pairs = []  # (key index, frame)
    for i in range(N):
        if i in keys:
            continue
        kl = max(k for k in range(3) if keys[k] < i)
        kr = min(k for k in range(3) if keys[k] > i)
        pairs += [(kl, i), (kr, i)]
    idx = {pr: q for q, pr in enumerate(pairs)}
    F, E = [], []
    for (k, i) in pairs:
        f, e = oracle.nnf_init_random(g[keys[k]], g[i], p, 0, seed, keys[k] * N + i)
        F.append(f)
        E.append(e)
    for it in range(n):
        new = []
        for q, (k, i) in enumerate(pairs):
            other = [t for t, (k2, i2) in enumerate(pairs) if i2 == i and t != q][0]
            new.append(oracle.pm_iteration_ext(g[keys[k]], g[i], ks[k], ks[pairs[other][0]], p, a16,
                                               oracle.TRACK | oracle.ALIGN, 0, it, seed, keys[k] * N + i, F, E, q,
                                               idx.get((k, i - 1), -1), idx.get((k, i + 1), -1), other))
        F, E = [x[0] for x in new], [x[1] for x in new]
    want = np.zeros((N,) + g.shape[1:], np.float64)
    for i in range(N):
        if i in keys:
            want[i] = ks[keys.index(i)] / 255.0
            continue
        (kl, _), (kr, _) = [pr for pr in pairs if pr[1] == i]
        l, r = keys[kl], keys[kr]
        want[i] = ((r - i) / (r - l)) * oracle.remap(ks[kl], F[idx[(kl, i)]], p) + \
                  ((i - l) / (r - l)) * oracle.remap(ks[kr], F[idx[(kr, i)]], p)
    got = oracle.interpolate_ext(g, np.array(keys), ks, p, 1, n, seed, a16, track=True, align=True)
    assert np.abs(got - want).max() < 1e-12
