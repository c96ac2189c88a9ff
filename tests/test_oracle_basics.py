"""Pins of the oracle's building blocks: Philox, pyramid, patch SSD, init, upsample.

Each test checks the oracle against something other than itself: an
independent library implementation, a hand-derived fixture, a closed form, an
invariant, or a vectorised numpy formulation (``pins``).
"""
import json
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

_ROCRAND_PROG = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
  unsigned long long k0, k1, c0, c1, c2, c3;
  while (scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    rocrand_state_philox4x32_10 st;
    /* key = seed; counter words (x, y) from the offset / 4, (z, w) from the subsequence */
    rocrand_init(k0 | (k1 << 32), c2 | (c3 << 32), 4ull * (c0 | (c1 << 32)), &st);
    uint4 r = rocrand4(&st);
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc (rocRAND host build) not available")
def test_philox_matches_rocrand_host_implementation(orc):
    """Philox4x32-10 against rocRAND's independent host-callable implementation."""
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    cases[0] = 0
    cases[1] = 2**32 - 1
    # rocRAND takes counter words (x, y) as an element offset of 4 * (x | y << 32),
    # which must fit in 64 bits: keep y below 2^30
    cases[:, 3] &= 2**30 - 1
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "p.cpp")
        exe = os.path.join(td, "p")
        with open(src, "w") as f:
            f.write(_ROCRAND_PROG)
        subprocess.check_call(["hipcc", "-O1", "-o", exe, src], stdout=subprocess.DEVNULL,
                              stderr=subprocess.DEVNULL)
        txt = "\n".join(" ".join(str(int(x)) for x in row) for row in cases)
        out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()], np.uint64)
    assert ref.shape == (300, 4)
    for row, exp in zip(cases, ref):
        got = orc.philox4x32_10([int(row[2]), int(row[3]), int(row[4]), int(row[5])],
                                [int(row[0]), int(row[1])])
        assert np.array_equal(got.astype(np.uint64), exp), (row, got, exp)


def test_uniform16_range_and_chi2(orc):
    # closed form: the map (u * n) >> 16 never reaches n and covers [0, n)
    for n in (1, 2, 3, 7, 129, 1025, 65535):
        assert orc.uniform16(0, n) == 0
        assert orc.uniform16(0xFFFF, n) == n - 1
    # chi-squared of 16-bit Philox draws mapped to 9 and 33 bins
    words = np.array([orc.philox4x32_10([i, 3, 5, 0], [11, 13]) for i in range(4000)], np.uint32).reshape(-1)
    u16 = np.concatenate([words & 0xFFFF, words >> 16]).astype(np.uint64)
    for n in (9, 33):
        bins = np.bincount(((u16 * n) >> 16).astype(np.int64), minlength=n)
        exp = len(u16) / n
        chi2 = ((bins - exp) ** 2 / exp).sum()
        # generous bound: p < 1e-6 for df <= 32
        assert chi2 < 90, (n, chi2)


def test_pyramid_golden(orc):
    g = json.load(open(os.path.join(GOLDEN, "pyramid_3x3.json")))
    img = np.stack(g["input_channels"], axis=-1).astype(np.uint8)
    exp = np.stack(g["output_channels"], axis=-1).astype(np.uint8)
    assert np.array_equal(orc.downsample(img), exp)


def test_pyramid_invariants(orc):
    # a constant image stays constant, at ceil sizes
    c = np.full((13, 10, 3), 77, np.uint8)
    d = orc.downsample(c)
    assert d.shape == (7, 5, 3) and (d == 77).all()
    # a 2x2-replicated image downsamples to the original
    base = pins.noise_image(9, 11, 3)
    rep = np.repeat(np.repeat(base, 2, axis=0), 2, axis=1)
    assert np.array_equal(orc.downsample(rep), base)
    # numpy formulation on even interior blocks
    x = pins.noise_image(16, 12, 4).astype(np.int64)
    blk = x.reshape(8, 2, 6, 2, 3).sum(axis=(1, 3))
    assert np.array_equal(orc.downsample(x.astype(np.uint8)), ((blk + 2) >> 2).astype(np.uint8))
    levels = orc.pyramid(pins.noise_image(37, 21, 5), 4)
    assert [l.shape[:2] for l in levels] == [(37, 21), (19, 11), (10, 6), (5, 3)]


def test_ssd_golden(orc):
    g = json.load(open(os.path.join(GOLDEN, "ssd_3x3.json")))
    T = np.zeros((3, 3, 3), np.uint8)
    T[0, 0] = (1, 2, 3)
    T[2, 2] = (0, 0, 4)
    imgs = {"zero": np.zeros((3, 3, 3), np.uint8), "ten": np.full((3, 3, 3), 10, np.uint8)}
    for case in g["cases"]:
        got = orc.patch_ssd(imgs[case["S"]], T, case["p"], case["u"], case["v"])
        assert got == case["ssd"], case


def test_ssd_matches_vectorised_and_symmetry(orc):
    rng = np.random.default_rng(1)
    S = pins.noise_image(11, 14, 10)
    T = pins.noise_image(11, 14, 11)
    for p in (0, 1, 2, 3):
        for _ in range(40):
            u = (int(rng.integers(0, 11)), int(rng.integers(0, 14)))
            v = (int(rng.integers(0, 11)), int(rng.integers(0, 14)))
            d = orc.patch_ssd(S, T, p, u, v)
            assert d == pins.ssd(S, T, p, u, v)
            assert d == orc.patch_ssd(T, S, p, v, u)
            assert orc.patch_ssd(S, S, p, u, u) == 0


def test_energy_matches_vectorised(orc):
    S = pins.noise_image(17, 23, 20)
    T = pins.noise_image(17, 23, 21)
    rng = np.random.default_rng(2)
    F = np.stack([rng.integers(0, 17, (17, 23)), rng.integers(0, 23, (17, 23))], -1).astype(np.int32)
    assert np.array_equal(orc.energy(S, T, F, 2).astype(np.int64), pins.energy(S, T, F, 2))


def test_init_random_range_energy_and_determinism(orc):
    S = pins.noise_image(33, 40, 30)
    T = pins.noise_image(33, 40, 31)
    F, E = orc.nnf_init_random(S, T, 2, 2, 1234, 7)
    assert F[..., 0].min() >= 0 and F[..., 0].max() < 33
    assert F[..., 1].min() >= 0 and F[..., 1].max() < 40
    assert np.array_equal(E.astype(np.int64), pins.energy(S, T, F, 2))
    F2, _ = orc.nnf_init_random(S, T, 2, 2, 1234, 7)
    assert np.array_equal(F, F2)
    F3, _ = orc.nnf_init_random(S, T, 2, 2, 1234, 8)
    assert (F3 != F).any(axis=-1).mean() > 0.9  # another pair id draws another field
    # rows and columns are spread over the whole image
    assert len(np.unique(F[..., 0])) == 33 and len(np.unique(F[..., 1])) == 40


def test_init_offsets(orc):
    S = pins.noise_image(12, 9, 40)
    T = pins.noise_image(12, 9, 41)
    off = np.zeros((12, 9, 2), np.int32)
    off[..., 0] = -3
    off[..., 1] = 100
    F, E = orc.nnf_init_offsets(S, T, 1, off)
    rr, cc = np.meshgrid(np.arange(12), np.arange(9), indexing="ij")
    assert np.array_equal(F[..., 0], np.clip(rr - 3, 0, 11))
    assert (F[..., 1] == 8).all()
    assert np.array_equal(E.astype(np.int64), pins.energy(S, T, F, 1))


def test_upsample_identity_and_offsets(orc):
    # identity at the coarse level -> identity at the fine level (odd sizes too)
    for h, w in ((16, 16), (15, 9)):
        hc, wc = (h + 1) // 2, (w + 1) // 2
        rr, cc = np.meshgrid(np.arange(hc), np.arange(wc), indexing="ij")
        Fc = np.stack([rr, cc], -1).astype(np.int32)
        S = pins.noise_image(h, w, 50)
        T = pins.noise_image(h, w, 51)
        F, E = orc.nnf_upsample(Fc, S, T, 2)
        fr, fcol = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
        assert np.array_equal(F[..., 0], fr) and np.array_equal(F[..., 1], fcol)
        assert np.array_equal(E.astype(np.int64), pins.energy(S, T, F, 2))
    # a constant coarse offset t becomes 2t at the fine level (where not clamped)
    h, w = 20, 24
    rr, cc = np.meshgrid(np.arange(10), np.arange(12), indexing="ij")
    Fc = np.stack([np.clip(rr + 2, 0, 9), np.clip(cc - 1, 0, 11)], -1).astype(np.int32)
    S = pins.noise_image(h, w, 52)
    F, _ = orc.nnf_upsample(Fc, S, S, 1)
    fr, fcol = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    inner = (fr < 16) & (fcol >= 2)
    assert (F[..., 0] - fr)[inner].tolist() == [4] * int(inner.sum())
    assert (F[..., 1] - fcol)[inner].tolist() == [-2] * int(inner.sum())
