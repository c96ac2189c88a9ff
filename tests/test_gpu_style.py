"""GPU parity of the guide + style loss (Eq. 3, FB_STYLE_LOSS) against the CPU
oracle: fields and energies bit-exact, blends within 1e-5, through the C ABI."""
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


def _video(n, h, w, seed):
    return synth.sprite_video(n, h, w, seed, n_sprites=2, side=(max(2, min(h, w) // 6), max(3, min(h, w) // 3)))


def _styles(guides, seed):
    rng = np.random.default_rng(seed)
    lut = np.sort(rng.integers(0, 256, (3, 256)), axis=1).astype(np.uint8)
    gain = rng.uniform(0.9, 1.1, (len(guides), 1, 1, 3))
    out = np.stack([np.stack([lut[c][g[..., c]] for c in range(3)], -1) for g in guides]).astype(np.float64)
    return np.clip(np.rint(out * gain), 0, 255).astype(np.uint8)


def _style_params(p, K, iters, seed, alpha16, flags=0):
    return fbm.make_params(p, K, iters, seed, flags | fbm.FB_STYLE_LOSS, alpha16)


def _run_pairs(ctx, cases, prm):
    descs = []
    for g, s, h, w, K, pid in cases:
        p = prm.patch_radius
        descs.append(dict(src_pyr=ctx.fb_build_pyramid(dev(g[0]), K, p), tgt_pyr=ctx.fb_build_pyramid(dev(g[1]), K, p),
                          src_style_pyr=ctx.fb_build_pyramid(dev(s), K, p), h=h, w=w, levels=K, pair_id=pid))
    return ctx.fb_patchmatch_batch(descs, prm)


@pytest.mark.parametrize("p,alpha16", [(2, 16), (2, 0), (1, 40), (3, 7)])
def test_style_batch_matches_oracle(ctx, p, alpha16):
    """Mixed sizes and level counts in one batch (ragged tiles, odd sizes)."""
    seed, iters = 31, 3
    cases = []
    for (h, w, K, vs) in ((40, 56, 2, 1), (37, 29, 1, 2), (64, 80, 3, 3)):
        g = _video(2, h, w, vs)
        s = _styles(g, vs + 10)
        cases.append((g, s[0], h, w, K, 7 * vs))
    outs = _run_pairs(ctx, cases, _style_params(p, 3, iters, seed, alpha16))
    for (g, s, h, w, K, pid), (nnf, en) in zip(cases, outs):
        F, E, _ = oracle.patchmatch_style(g[0], g[1], s, p, K, iters, seed, pid, alpha16)
        n, e = host(nnf), host(en).astype(np.uint32)
        bad = np.argwhere((n != F).any(-1) | (e != E))
        assert bad.size == 0, ((h, w, K), len(bad), bad[:3])


@pytest.mark.parametrize("p", [2, 4])
def test_style_batch_degenerate_shapes(ctx, p):
    """One-row, one-column and tiny frames (every patch clamped, tiles mostly
    empty) in one batch, with the style loss."""
    seed, iters = 5, 3
    cases = []
    for k, (h, w) in enumerate(((1, 17), (13, 1), (2, 3), (1, 1))):
        rng = np.random.default_rng(100 + k)
        g = rng.integers(0, 256, (2, h, w, 3), dtype=np.uint8)
        s = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
        cases.append((g, s, h, w, 1, 11 + k))
    outs = _run_pairs(ctx, cases, _style_params(p, 1, iters, seed, 16))
    for (g, s, h, w, K, pid), (nnf, en) in zip(cases, outs):
        F, E, _ = oracle.patchmatch_style(g[0], g[1], s, p, K, iters, seed, pid, 16)
        n, e = host(nnf), host(en).astype(np.uint32)
        assert np.array_equal(n, F) and np.array_equal(e, E), (h, w, p)


def test_style_tile_shapes_and_graph_replay_agree(ctx):
    g = _video(2, 48, 72, 5)
    s = _styles(g, 6)
    cases = [(g, s[0], 48, 72, 2, 3)]
    ref = None
    for cfg in range(fbm.load_library().fb_num_tile_configs()):
        ctx.fb_set_tile_config(cfg)
        (nnf, en), = _run_pairs(ctx, cases, _style_params(2, 2, 2, 9, 16))
        cur = (host(nnf), host(en))
        if ref is None:
            ref = cur
        assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1]), cfg
    ctx.fb_set_tile_config(-1)
    for rep in range(3):
        (nnf, en), = _run_pairs(ctx, cases, _style_params(2, 2, 2, 9, 16, fbm.FB_USE_GRAPH))
        assert np.array_equal(host(nnf), ref[0]) and np.array_equal(host(en), ref[1]), rep


@pytest.mark.parametrize("N,h,w,M,K,iters", [(5, 40, 48, 2, 2, 2), (3, 33, 45, 1, 1, 3)])
def test_style_blend_matches_oracle(ctx, N, h, w, M, K, iters):
    g = _video(N, h, w, N + h)
    s = _styles(g, w)
    seed = 17
    out = host(ctx.fb_blend_window(dev(g), dev(s), M, _style_params(2, K, iters, seed, 16)))
    ref = oracle.blend_window_style(g, s, M, 2, K, iters, seed, 16)
    assert np.abs(out - ref).max() <= TOL


def test_style_full_size_pair(ctx):
    """One 512x512 pair of the blend workload, 3 levels x 6 iterations, under
    Eq. 3 with alpha = 1: bit-exact with the oracle."""
    guides, styles = synth.blend_workload()
    seed = synth.PHILOX_SEED[2]
    j, i = 3, 0
    cases = [((guides[j], guides[i]), styles[j], 512, 512, 3, j * 32 + i)]
    (nnf, en), = _run_pairs(ctx, cases, _style_params(2, 3, 6, seed, 16))
    F, E, _ = oracle.patchmatch_style(guides[j], guides[i], styles[j], 2, 3, 6, seed, j * 32 + i, 16)
    assert np.array_equal(host(nnf), F)
    assert np.array_equal(host(en).astype(np.uint32), E)


def test_style_invalid_arguments(ctx):
    g = _video(2, 24, 24, 1)
    s = _styles(g, 2)
    cases = [(g, s[0], 24, 24, 1, 0)]
    with pytest.raises(fbm.FastBlendError):
        _run_pairs(ctx, cases, _style_params(2, 1, 0, 1, 16))      # no iteration
    with pytest.raises(fbm.FastBlendError):
        _run_pairs(ctx, cases, _style_params(2, 1, 1, 1, 600))     # alpha16 out of range
    pa, pb = ctx.fb_build_pyramid(dev(g[0]), 1), ctx.fb_build_pyramid(dev(g[1]), 1)
    with pytest.raises(fbm.FastBlendError):                               # no style pyramid
        ctx.fb_patchmatch_batch([dict(src_pyr=pa, tgt_pyr=pb, h=24, w=24, levels=1, pair_id=0)],
                                _style_params(2, 1, 1, 1, 16))
    with pytest.raises(fbm.FastBlendError):                               # per-level calls keep Eq. 1
        ctx.fb_nnf_init(pa, pb, 24, 24, 0, _style_params(2, 1, 1, 1, 16), 0)
