"""GPU tests of the library's runtime: contexts release all the device memory
they allocate, and launch tables uploaded stream-ordered (a ring of table
slots) serve calls on several streams and many changing plans correctly."""
import ctypes

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


def test_failed_graph_capture_runs_eagerly():
    """FB_USE_GRAPH with a capture that fails (forced with
    FB_DEBUG_FAIL_CAPTURE) runs the launches eagerly: the call succeeds, the
    blend equals the eager one, and the fallback is counted; a normal graph
    call afterwards replays a captured graph again."""
    g, s = _small_workload(5, 40, 56, 13)
    ctx = fbm.Context(0)
    try:
        ref = ctx.fb_blend_window(g, s, 2, fbm.make_params(2, 2, 2, 17))
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.default_stream())
        with torch.cuda.stream(side):
            got = ctx.fb_blend_window(g, s, 2, fbm.make_params(2, 2, 2, 17,
                                                               fbm.FB_USE_GRAPH | fbm.FB_DEBUG_FAIL_CAPTURE))
            side.synchronize()
            assert ctx.fb_graph_fallbacks() == 1
            assert torch.equal(got, ref)
            for _ in range(2):
                again = ctx.fb_blend_window(g, s, 2, fbm.make_params(2, 2, 2, 17, fbm.FB_USE_GRAPH))
                side.synchronize()
                assert torch.equal(again, ref)
        assert ctx.fb_graph_fallbacks() == 1
    finally:
        ctx.close()


def test_tuning_results_persist_across_contexts(tmp_path):
    """A batch shape tuned by one context and saved is not timed again by a
    context that loads the file, and the results are the same."""
    g, s = _small_workload(4, 48, 64, 21)
    prm = fbm.make_params(2, 2, 2, 5)
    a = fbm.Context(0)
    try:
        ra = a.fb_blend_window(g, s, 1, prm)
        assert a.fb_autotune_runs() == 1
        path = str(tmp_path / "tuning.json")
        a.tuning_save(path)
        text = a.tuning_export()
    finally:
        a.close()
    b = fbm.Context(0)
    try:
        assert b.tuning_load(path)
        assert b.tuning_export() == text
        rb = b.fb_blend_window(g, s, 1, prm)
        assert b.fb_autotune_runs() == 0
        assert torch.equal(ra, rb)
        with pytest.raises(fbm.FastBlendError):
            b.tuning_import("p2;48x64*6=99\n")
    finally:
        b.close()


def test_gather_probe_reports_rates():
    """The measurement entry point: positive row rates, random rows no faster
    than consecutive ones, and patch radii other than 2 refused."""
    g, _ = _small_workload(1, 128, 160, 25)
    ctx = fbm.Context(0)
    try:
        pyr = ctx.fb_build_pyramid(g[0], 1, 2)
        div = ctx.fb_gather_probe(pyr, 128, 160, True, 32)
        coh = ctx.fb_gather_probe(pyr, 128, 160, False, 32)
        assert 0 < div <= coh * 1.05, (div, coh)
        L = fbm.load_library()
        r = ctypes.c_double(0.0)
        assert L.fb_gather_probe(ctx.handle, ctypes.c_void_p(pyr.data_ptr()), 128, 160, 3, 1, 32, ctypes.byref(r),
                                 None) == -3
    finally:
        ctx.close()
