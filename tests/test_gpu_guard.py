"""GPU tests of the guard of seeded PatchMatch (FB_LEARNED_SEED): every seeded
pair races its coarsest level against the plain random start, and a seed that
loses is replaced by the plain run.  Checked bit-exact against the oracle's
guarded run (oracle.patchmatch_raced), through the batch call and the window
blend, with network weights loaded from the host that predict a bad field."""
import numpy as np
import pytest
import torch

import oracle
from oracle import proposal_net as net
from paper_2311_09265_amd import fastblend as fbm
from paper_2311_09265_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = fbm.Context(0)
    yield c
    c.close()


def _video(N=4, h=72, w=100, seed=17):
    return synth.sprite_video(N, h, w, seed, n_sprites=3, side=(10, 28))


def _seeds(kind, hc, wc, rng):
    if kind == "random":      # unrelated to the video's motion
        return np.stack([rng.integers(-hc, hc, (hc, wc)), rng.integers(-wc, wc, (hc, wc))], -1).astype(np.int32)
    if kind == "corner":      # every pixel starts at the last source pixel
        off = np.zeros((hc, wc, 2), np.int32)
        off[..., 0], off[..., 1] = hc, wc
        return off
    if kind == "zero":        # the static background matches
        return np.zeros((hc, wc, 2), np.int32)
    return rng.integers(-2, 3, (hc, wc, 2)).astype(np.int32)   # "small": near the truth


def _converged_seed(S, T, levels, plain_iters, seed, pair_id):
    """Offsets of the plain run's own coarsest level after plain_iters
    iterations: the seeded start is that field, so the seeded sum can only be
    lower or equal (iterations never raise a pixel's energy) and the seed is
    kept (ties go to the seed)."""
    l = levels - 1
    Sl, Tl = oracle.pyramid(S, levels)[l], oracle.pyramid(T, levels)[l]
    F, E = oracle.nnf_init_random(Sl, Tl, 2, l, seed, pair_id)
    for it in range(plain_iters):
        F, E = oracle.pm_iteration(Sl, Tl, 2, l, it, seed, pair_id, F, E)
    hc, wc = Sl.shape[:2]
    return (F - np.stack(np.meshgrid(np.arange(hc), np.arange(wc), indexing="ij"), -1)).astype(np.int32)


@pytest.mark.parametrize("levels,iters,plain_iters", [(3, 2, 6), (2, 3, 2), (1, 1, 4), (2, 2, 5), (3, 0, 3)])
def test_guarded_batch_matches_oracle(ctx, levels, iters, plain_iters):
    """Rejected and kept seeds in one batch, run lengths in both orders and of
    odd difference, a single level (the race decides the final field) and no
    seeded iterations at all: fields, energies and the two sums of every pair
    equal the oracle's guarded run."""
    N, h, w = 4, 72, 100
    guides = _video(N, h, w)
    g = torch.from_numpy(guides).cuda()
    pyrs = [ctx.fb_build_pyramid(g[f], levels) for f in range(N)]
    hc, wc = fbm.level_size(h, w, levels - 1)
    pairs = [(0, 1, "random"), (1, 0, "zero"), (2, 3, "converged"), (3, 1, "corner"), (1, 2, "small")]
    rng = np.random.default_rng(levels * 100 + iters * 10 + plain_iters)
    seed = 0xFB5EED42
    seeds = [_converged_seed(guides[j], guides[i], levels, plain_iters, seed, j * N + i) if kind == "converged"
             else _seeds(kind, hc, wc, rng) for j, i, kind in pairs]
    descs = [dict(src_pyr=pyrs[j], tgt_pyr=pyrs[i], h=h, w=w, levels=levels, pair_id=j * N + i,
                  seed_offsets=torch.from_numpy(s).cuda()) for (j, i, _), s in zip(pairs, seeds)]
    prm = fbm.make_params(2, levels, iters, seed, fbm.FB_LEARNED_SEED, plain_iters=plain_iters)
    outs = ctx.fb_patchmatch_batch(descs, prm)
    sums = ctx.fb_guard_read()
    assert sums.shape == (len(pairs), 2)
    rejected = []
    for k, (j, i, _) in enumerate(pairs):
        F, E, rej, (ss, sp) = oracle.patchmatch_raced(guides[j], guides[i], 2, levels, iters, plain_iters, seed,
                                                      j * N + i, seeds[k])
        assert (int(sums[k, 0]), int(sums[k, 1])) == (ss, sp), k
        assert np.array_equal(outs[k][0].cpu().numpy(), F), k
        assert np.array_equal(fbm.energy_u32(outs[k][1]).cpu().numpy(), E.astype(np.int64)), k
        rejected.append(rej)
    assert not rejected[2]                           # the converged seed is kept
    assert rejected[3] or plain_iters <= iters       # the corner seed loses to a longer plain run


def test_no_guard_flag_takes_the_seed(ctx):
    N, h, w, levels = 4, 72, 100, 3
    guides = _video(N, h, w)
    g = torch.from_numpy(guides).cuda()
    pyrs = [ctx.fb_build_pyramid(g[f], levels) for f in range(N)]
    hc, wc = fbm.level_size(h, w, levels - 1)
    off = _seeds("random", hc, wc, np.random.default_rng(3))
    d = [dict(src_pyr=pyrs[0], tgt_pyr=pyrs[2], h=h, w=w, levels=levels, pair_id=2,
              seed_offsets=torch.from_numpy(off).cuda())]
    prm = fbm.make_params(2, levels, 2, 5, fbm.FB_LEARNED_SEED | fbm.FB_NO_GUARD)
    (nnf, en), = ctx.fb_patchmatch_batch(d, prm)
    F, E = oracle.patchmatch(guides[0], guides[2], 2, levels, 2, 5, 2, seed_offsets=off)
    assert np.array_equal(nnf.cpu().numpy(), F)
    assert int(ctx.fb_guard_read().abs().sum()) == 0


def _bad_network(shift=(37, -29)):
    """Weights that predict one constant offset everywhere (all weights zero,
    the head's biases the offset): a field unrelated to the video's motion."""
    flat = torch.zeros(net.param_count(), dtype=torch.float32)
    a, b = net.layer_slices()[-1]
    flat[b - 2], flat[b - 1] = float(shift[0]), float(shift[1])
    return flat


def test_bad_network_falls_back_to_plain(ctx):
    """A network loaded from the host that predicts a bad field: the guard
    rejects every pair's seed, and the blend (and each NNF) equals the plain
    method with 6 iterations per level exactly -- final energy within margin 0
    of plain@6."""
    N, h, w, levels, M = 5, 64, 96, 3, 2
    guides = _video(N, h, w, 29)
    styles = synth.sprite_video(N, h, w, 31, n_sprites=2, side=(8, 20))
    g, s = torch.from_numpy(guides).cuda(), torch.from_numpy(styles).cuda()
    ctx.fb_unet_load(_bad_network().cuda())
    seed = 0xFB5EED77
    lprm = fbm.make_params(2, levels, 2, seed, fbm.FB_LEARNED_SEED, plain_iters=6)
    pprm = fbm.make_params(2, levels, 6, seed)
    out_l = ctx.fb_blend_window(g, s, M, lprm)
    sums = ctx.fb_guard_read()
    out_p = ctx.fb_blend_window(g, s, M, pprm)
    n_pairs = sum(min(N - 1, i + M) - max(0, i - M) for i in range(N))
    assert sums.shape == (n_pairs, 2)
    assert bool((sums[:, 0] > sums[:, 1]).all()), sums
    assert torch.equal(out_l, out_p)
    pyrs = [ctx.fb_build_pyramid(g[f], levels) for f in range(N)]
    pairs = [(j, i) for i in range(N) for j in range(max(0, i - M), min(N - 1, i + M) + 1) if j != i]
    descs = [dict(src_pyr=pyrs[j], tgt_pyr=pyrs[i], h=h, w=w, levels=levels, pair_id=j * N + i) for j, i in pairs]
    for (fl, el), (fp, ep) in zip(ctx.fb_patchmatch_batch(descs, lprm), ctx.fb_patchmatch_batch(descs, pprm)):
        assert torch.equal(fl, fp) and torch.equal(el, ep)


def test_interpolation_with_learned_seeds(ctx):
    """fb_interpolate under FB_LEARNED_SEED, on a still video (one frame plus
    independent noise of +-4 per frame, so zero is the true motion).  Every
    pair's two race sums equal the oracle's for the same seed field.  A
    network that predicts a constant, wrong offset loses every race: the
    frames equal plain interpolation with plain_iters iterations exactly.  A
    network that predicts zero offsets keeps every seed: the guarded frames
    equal the unguarded ones (FB_NO_GUARD) and differ from plain's."""
    N, h, w, levels = 9, 48, 64, 2
    keys = [0, 4, 8]
    base = _video(1, h, w, 41)[0].astype(np.int32)
    noise = np.random.default_rng(5).integers(-4, 5, (N, h, w, 3))
    frames = np.clip(base[None] + noise, 0, 255).astype(np.uint8)
    guides = torch.from_numpy(frames).cuda()
    kst = torch.from_numpy(synth.sprite_video(len(keys), h, w, 43, n_sprites=2, side=(8, 20))).cuda()
    # the pairs in the order the call plans them: frame, then left before right key
    pairs = [(k, i) for i in range(N) if i not in keys
             for k in (max(k for k in keys if k < i), min(k for k in keys if k > i))]
    hc, wc = fbm.level_size(h, w, levels - 1)
    seed = 0xFB5EED78

    def oracle_sums(shift, plain_iters):
        off = np.zeros((hc, wc, 2), np.int32)
        off[..., 0], off[..., 1] = shift
        return torch.tensor([list(oracle.patchmatch_raced(frames[k], frames[i], 2, levels, 2, plain_iters, seed,
                                                          k * N + i, off)[3]) for k, i in pairs], dtype=torch.int64)

    ctx.fb_unet_load(_bad_network((37, -29)).cuda())
    out_l = ctx.fb_interpolate(guides, keys, kst, fbm.make_params(2, levels, 2, seed, fbm.FB_LEARNED_SEED,
                                                                  plain_iters=5))
    sums = ctx.fb_guard_read()
    assert torch.equal(sums, oracle_sums((37, -29), 5))
    assert bool((sums[:, 0] > sums[:, 1]).all()), sums
    assert torch.equal(out_l, ctx.fb_interpolate(guides, keys, kst, fbm.make_params(2, levels, 5, seed)))
    ctx.fb_unet_load(_bad_network((0, 0)).cuda())
    out_g = ctx.fb_interpolate(guides, keys, kst, fbm.make_params(2, levels, 2, seed, fbm.FB_LEARNED_SEED))
    sums = ctx.fb_guard_read()
    assert torch.equal(sums, oracle_sums((0, 0), 6))
    assert bool((sums[:, 0] <= sums[:, 1]).all()), sums
    out_u = ctx.fb_interpolate(guides, keys, kst, fbm.make_params(2, levels, 2, seed,
                                                                  fbm.FB_LEARNED_SEED | fbm.FB_NO_GUARD))
    assert torch.equal(out_g, out_u)
    assert not torch.equal(out_g, ctx.fb_interpolate(guides, keys, kst, fbm.make_params(2, levels, 2, seed)))


def test_guarded_graph_replay_matches_eager(ctx):
    """The guarded launch sequence is fixed: a captured graph replays it with
    the same fields, whichever seeds lose."""
    N, h, w, levels = 4, 72, 100, 3
    guides = _video(N, h, w)
    g = torch.from_numpy(guides).cuda()
    pyrs = [ctx.fb_build_pyramid(g[f], levels) for f in range(N)]
    hc, wc = fbm.level_size(h, w, levels - 1)
    rng = np.random.default_rng(8)
    kinds = ["random", "small", "random", "zero"]
    descs = [dict(src_pyr=pyrs[j], tgt_pyr=pyrs[(j + 1) % N], h=h, w=w, levels=levels, pair_id=j,
                  seed_offsets=torch.from_numpy(_seeds(k, hc, wc, rng)).cuda()) for j, k in enumerate(kinds)]
    eager = ctx.fb_patchmatch_batch(descs, fbm.make_params(2, levels, 2, 9, fbm.FB_LEARNED_SEED))
    gprm = fbm.make_params(2, levels, 2, 9, fbm.FB_LEARNED_SEED | fbm.FB_USE_GRAPH)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for rep in range(3):
            got = ctx.fb_patchmatch_batch(descs, gprm)
            side.synchronize()
            for (a, ea), (b, eb) in zip(got, eager):
                assert torch.equal(a, b) and torch.equal(ea, eb), rep


def test_guarded_mixed_sizes_and_levels_match_oracle(ctx):
    """Pairs of different sizes and level counts in one batch, so that their
    races are decided at different passes (a 3-level pair's coarsest pass
    comes before a 2-level pair's): every pair equals the oracle's guarded
    run, rejected and kept alike."""
    seed, iters, plain = 0xFB5EED55, 2, 5
    specs = [(48, 64, 2, "random", 21), (96, 128, 3, "converged", 22), (96, 128, 3, "random", 23),
             (48, 64, 2, "converged", 24), (72, 100, 3, "zero", 25)]
    descs, refs = [], []
    for k, (h, w, levels, kind, vs) in enumerate(specs):
        v = _video(2, h, w, vs)
        g = torch.from_numpy(v).cuda()
        hc, wc = fbm.level_size(h, w, levels - 1)
        if kind == "converged":
            off = _converged_seed(v[0], v[1], levels, plain, seed, k)
        else:
            off = _seeds(kind, hc, wc, np.random.default_rng(k))
        descs.append(dict(src_pyr=ctx.fb_build_pyramid(g[0], levels), tgt_pyr=ctx.fb_build_pyramid(g[1], levels),
                          h=h, w=w, levels=levels, pair_id=k, seed_offsets=torch.from_numpy(off).cuda()))
        refs.append(oracle.patchmatch_raced(v[0], v[1], 2, levels, iters, plain, seed, k, off))
    outs = ctx.fb_patchmatch_batch(descs, fbm.make_params(2, 3, iters, seed, fbm.FB_LEARNED_SEED, plain_iters=plain))
    sums = ctx.fb_guard_read()
    rejected = []
    for k, ((nnf, en), (F, E, rej, (ss, sp))) in enumerate(zip(outs, refs)):
        assert (int(sums[k, 0]), int(sums[k, 1])) == (ss, sp), k
        assert np.array_equal(nnf.cpu().numpy(), F), k
        assert np.array_equal(fbm.energy_u32(en).cpu().numpy(), E.astype(np.int64)), k
        rejected.append(rej)
    assert rejected[0] and rejected[2] and not rejected[1] and not rejected[3]
