"""GPU parity of the accurate-mode window blend (FB_ACCURATE_BLEND, Eq. 7-8)
against the CPU oracle, within 1e-5 on [0, 1], through the C ABI.  The
second-pass NNFs depend on T^- bit for bit, so agreement within 1e-5 also
shows that T^- and the Eq. 8 fields are exact."""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_09265_amd import fastblend as fbm
from paper_2311_09265_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fbm.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _video(N, h, w, seed):
    g = synth.sprite_video(N, h, w, seed, n_sprites=2, side=(max(2, min(h, w) // 6), max(3, min(h, w) // 3)))
    s = synth.flicker(synth.apply_lut(g, synth.random_lut(seed ^ 5)), seed ^ 9)
    return g, s


@pytest.mark.parametrize("N,h,w,M,K,iters,alpha16", [(5, 40, 48, 2, 2, 2, 16), (4, 33, 45, 1, 1, 3, 5),
                                                     (6, 32, 40, 3, 2, 2, 64), (1, 20, 20, 2, 1, 1, 16)])
def test_accurate_blend_matches_oracle(ctx, N, h, w, M, K, iters, alpha16):
    g, s = _video(N, h, w, N * 11 + w)
    seed = 29
    prm = fbm.make_params(2, K, iters, seed, fbm.FB_ACCURATE_BLEND, alpha16)
    out = host(ctx.fb_blend_window(dev(g), dev(s), M, prm))
    ref = oracle.blend_window_accurate(g, s, M, 2, K, iters, seed, alpha16)
    assert np.abs(out - ref).max() <= TOL


@pytest.mark.parametrize("p", [1, 3])
def test_accurate_blend_other_patch_radii(ctx, p):
    """3x3 and 7x7 patches: their own bound tables, patch-sum quantisation
    and unrolled row loops in both passes."""
    g, s = _video(4, 30, 37, 70 + p)
    prm = fbm.make_params(p, 2, 2, 31, fbm.FB_ACCURATE_BLEND, 16)
    out = host(ctx.fb_blend_window(dev(g), dev(s), 1, prm))
    ref = oracle.blend_window_accurate(g, s, 1, p, 2, 2, 31, 16)
    assert np.abs(out - ref).max() <= TOL


def test_accurate_blend_full_size_frames(ctx):
    """The first 4 frames of the 512x512 blend workload, 3 levels x 6
    iterations, window radius 5 (truncated), alpha = 1."""
    guides, styles = synth.blend_workload(4, 512, 512)
    seed = synth.PHILOX_SEED[2]
    prm = fbm.make_params(2, 3, 6, seed, fbm.FB_ACCURATE_BLEND, 16)
    out = host(ctx.fb_blend_window(dev(guides), dev(styles), 5, prm))
    ref = oracle.blend_window_accurate(guides, styles, 5, 2, 3, 6, seed, 16)
    assert np.abs(out - ref).max() <= TOL


def test_accurate_blend_graph_replay_matches_eager(ctx):
    g, s = _video(5, 32, 48, 7)
    prm = fbm.make_params(2, 2, 2, 3, fbm.FB_ACCURATE_BLEND, 16)
    ref = host(ctx.fb_blend_window(dev(g), dev(s), 2, prm))
    gprm = fbm.make_params(2, 2, 2, 3, fbm.FB_ACCURATE_BLEND | fbm.FB_USE_GRAPH, 16)
    for rep in range(3):
        assert np.array_equal(host(ctx.fb_blend_window(dev(g), dev(s), 2, gprm)), ref), rep


def test_accurate_blend_rejects_bad_arguments(ctx):
    g, s = _video(3, 16, 16, 1)
    for flags, iters, a16 in ((fbm.FB_ACCURATE_BLEND, 0, 16), (fbm.FB_ACCURATE_BLEND, 1, 513),
                              (fbm.FB_ACCURATE_BLEND | fbm.FB_FAST_BLEND, 1, 16),
                              (fbm.FB_ACCURATE_BLEND | fbm.FB_STYLE_LOSS, 1, 16)):
        with pytest.raises(fbm.FastBlendError):
            ctx.fb_blend_window(dev(g), dev(s), 1, fbm.make_params(2, 1, iters, 1, flags, a16))
