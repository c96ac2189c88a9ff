"""GPU tests of the library's runtime: contexts release all the device memory
they allocate, and launch tables uploaded stream-ordered (a ring of table
slots) serve calls on several streams and many changing plans correctly."""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_09265_amd import fastblend as fbm
from paper_2311_09265_amd import synth

pytestmark = pytest.mark.gpu


def _small_workload(N=4, h=48, w=64, seed=5):
    g = synth.sprite_video(N, h, w, seed, n_sprites=2, side=(8, 20))
    s = synth.sprite_video(N, h, w, seed + 1, n_sprites=2, side=(8, 20))
    return torch.from_numpy(g).cuda(), torch.from_numpy(s).cuda()


def test_create_run_destroy_does_not_leak():
    """Every buffer a context allocates (pyramids, fields, the Eq. 3 S^ and
    fast-mode tables, the guard's buffers, launch-table slots) is freed by
    fb_destroy: free device memory after the fifth create/run/destroy cycle
    equals that after the first."""
    g, s = _small_workload()
    free = []
    for rep in range(5):
        ctx = fbm.Context(0)
        prm = fbm.make_params(2, 2, 2, 3)
        ctx.fb_blend_window(g, s, 1, prm)
        ctx.fb_blend_window(g, s, 1, fbm.make_params(2, 2, 2, 3, fbm.FB_STYLE_LOSS, 16))
        ctx.fb_blend_window(g, s, 2, fbm.make_params(2, 2, 2, 3, fbm.FB_FAST_BLEND))
        ctx.fb_blend_window(g, s, 1, fbm.make_params(2, 2, 2, 3, fbm.FB_ACCURATE_BLEND, 16))
        pyrs = [ctx.fb_build_pyramid(g[f], 2) for f in range(2)]
        off = torch.zeros((24, 32, 2), dtype=torch.int32, device="cuda")
        ctx.fb_patchmatch_batch([dict(src_pyr=pyrs[0], tgt_pyr=pyrs[1], h=48, w=64, levels=2, pair_id=1,
                                      seed_offsets=off)], fbm.make_params(2, 2, 2, 3, fbm.FB_LEARNED_SEED))
        torch.cuda.synchronize()
        ctx.close()
        del pyrs, off
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
    assert free[-1] >= free[0] - (1 << 20), [f >> 20 for f in free]


def test_plans_alternate_across_streams():
    """Three different plans (changing outputs and shapes), called in turn on
    two streams without synchronising in between, more times than the ring
    has slots: every result equals the oracle's."""
    ctx = fbm.Context(0)
    try:
        N, M = 4, 1
        shapes = [(40, 56), (48, 64), (32, 40)]
        works = [_small_workload(N, h, w, 7 + k) for k, (h, w) in enumerate(shapes)]
        prm = fbm.make_params(2, 2, 2, 11)
        streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        outs = []
        for rep in range(12):
            k = rep % 3
            st = streams[rep % 2]
            with torch.cuda.stream(st):
                g, s = works[k]
                # the inputs were made on the default stream
                st.wait_stream(torch.cuda.default_stream())
                outs.append((k, ctx.fb_blend_window(g, s, M, prm)))
        torch.cuda.synchronize()
        refs = {}
        for k, out in outs:
            if k not in refs:
                g, s = works[k]
                refs[k] = oracle.blend_window(g.cpu().numpy(), s.cpu().numpy(), M, 2, 2, 2, 11)
            assert float(np.abs(out.cpu().numpy().astype(np.float64) - refs[k]).max()) <= 1e-5, k
    finally:
        ctx.close()
