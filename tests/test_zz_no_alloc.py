"""GPU test of fb_patchmatch_level_noalloc, the variant of fb_patchmatch_level
that allocates nothing (its working memory is the library's fixed per-GPU
array): through the C ABI it returns exactly what fb_patchmatch_level
returns, on two calls in a row, the second with a smaller level, and it
refuses a level above its stated maximum."""
import numpy as np
import pytest
import torch

from paper_2311_09265_amd import fastblend as fbm
from paper_2311_09265_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fbm.Context(0)
    yield c
    c.close()


def _level_pair(ctx, h, w, levels, seed):
    v = synth.sprite_video(2, h, w, seed, n_sprites=3, side=(8, 24))
    g = torch.from_numpy(v).cuda()
    return ctx.fb_build_pyramid(g[0], levels), ctx.fb_build_pyramid(g[1], levels)


@pytest.mark.parametrize("iters", [3, 4])
def test_noalloc_level_equals_the_allocating_call(ctx, iters):
    """Two calls in a row (a 200x264 level from its upsampled coarse field,
    then a 40x52 level from a given field and energy), each against
    fb_patchmatch_level on the same inputs: bit-identical."""
    seed = 0xFB5EED11
    prm = fbm.make_params(2, 2, iters, seed)
    cases = []
    # first call: level 0 of 200x264 upsampled from level 1
    sp, tp = _level_pair(ctx, 200, 264, 2, 3)
    coarse, _ = ctx.fb_patchmatch_level(sp, tp, 200, 264, 1, prm, 7,
                                        nnf=torch.zeros((100, 132, 2), dtype=torch.int32, device="cuda"),
                                        energy=torch.full((100, 132), 2 ** 31 - 1, dtype=torch.int32,
                                                          device="cuda"))
    cases.append((sp, tp, 200, 264, 0, coarse, None, None, 7))
    # second call, smaller: level 0 of 40x52 from a given start
    sp2, tp2 = _level_pair(ctx, 40, 52, 1, 5)
    rng = np.random.default_rng(1)
    f0 = np.stack([rng.integers(0, 40, (40, 52)), rng.integers(0, 52, (40, 52))], -1).astype(np.int32)
    e0 = np.full((40, 52), 2 ** 30, np.int32)
    cases.append((sp2, tp2, 40, 52, 0, None, f0, e0, 9))
    for sp_, tp_, h, w, level, nc, f0_, e0_, pid in cases:
        hl, wl = fbm.level_size(h, w, level)
        def start():
            if f0_ is None:
                return (torch.empty((hl, wl, 2), dtype=torch.int32, device="cuda"),
                        torch.empty((hl, wl), dtype=torch.int32, device="cuda"))
            return torch.from_numpy(f0_.copy()).cuda(), torch.from_numpy(e0_.copy()).cuda()
        na, ea = start()
        ctx.fb_patchmatch_level_noalloc(sp_, tp_, h, w, level, prm, pid, na, ea, nnf_coarse=nc)
        nb, eb = start()
        ctx.fb_patchmatch_level(sp_, tp_, h, w, level, prm, pid, nnf=nb, energy=eb, nnf_coarse=nc)
        torch.cuda.synchronize()
        assert torch.equal(na, nb), (h, w)
        assert torch.equal(ea, eb), (h, w)


def test_noalloc_level_refuses_a_level_above_the_maximum(ctx):
    """A 1024x1025 level (1,049,600 pixels) is above the 1,048,576 the array
    holds: FB_E_UNSUPPORTED before anything is enqueued."""
    h, w = 1024, 1025
    z = torch.zeros(fbm.load_library().fb_pyramid_bytes(h, w, 2, 2), dtype=torch.uint8, device="cuda")
    nnf = torch.zeros((h, w, 2), dtype=torch.int32, device="cuda")
    en = torch.zeros((h, w), dtype=torch.int32, device="cuda")
    with pytest.raises(fbm.FastBlendError) as ei:
        ctx.fb_patchmatch_level_noalloc(z, z, h, w, 0, fbm.make_params(2, 2, 1, 0), 0, nnf, en)
    assert ei.value.status == -3
