#!/usr/bin/env python3
"""Benchmark of the FastBlend blending hot path on one MI355X.

Workload (one step): blending mode over a 32-frame 512x512 RGB uint8 video,
window radius 5 (290 ordered frame pairs), patch 5x5, 3 pyramid levels x 6
PatchMatch iterations: pyramids of all frames, batched PatchMatch of every
pair, remapping and the window average of Eq. 2, from uint8 guides/styles
resident in HBM to fp32 blended frames.  Inputs are seeded synthetic sprite
videos with flickering LUT styles (paper_2311_09265_amd.synth).

Prints one JSON line:
  value      whole-job PatchMatch throughput, Mpix*iter/s = pixel-iterations
             of all pairs and levels per step / step wall time
  roofline   the dominant kernel (the PatchMatch iteration) against the
             integer dot-product ALU peak: algorithmic byte-terms (one per
             squared channel difference of Eq. 1) / summed HIP-event time of
             its launches in the timed region
  cpu_baseline  the CPU oracle on a bounded sample of the same pairs
  learned    the same blend with the proposal network seeding PatchMatch
  style_loss the same blend with every NNF under the guide + style loss (Eq. 3)
  fast_mode  the fast-mode blend (tables and queries, Alg. 3-5) against the
             balanced one at window radius 5 and 15
  accurate_mode  the accurate-mode blend (Eq. 7-8)
  interpolation  the 1024x576 keyframe interpolation (Eq. 9), plain, with
             tracking, and with tracking + pairwise alignment (Eq. 10)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpix·iter/s of PatchMatch + blended frames/s at 512², window 5; learned vs plain"
# v_dot4_u32_u8: 4 byte multiply-accumulates per lane per clock,
# 256 CUs x 64 lanes x 2.4 GHz x 4
DOT4_PEAK_TOPS = 256 * 64 * 2.4e9 * 4 / 1e12
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def level_sizes(h, w, levels):
    return [(-(-h // (1 << l)), -(-w // (1 << l))) for l in range(levels)]


def window_pairs(N, M):
    return [(j, i) for i in range(N) for j in range(max(0, i - M), min(N - 1, i + M) + 1) if j != i]


def pm_work(n_pairs, h, w, levels, iters, p):
    """(pixel-iterations, algorithmic byte-terms of the iteration kernel) per step."""
    pix, terms = 0, 0
    K = (2 * p + 1) ** 2 * 3
    for hl, wl in level_sizes(h, w, levels):
        R = max(hl, wl)
        n_random = R.bit_length()               # radii R >> m >= 1
        n_prop = 4 * hl * wl - 2 * hl - 2 * wl  # in-image neighbours, summed over pixels
        pix += n_pairs * hl * wl * iters
        terms += n_pairs * iters * (n_prop + hl * wl * n_random) * K
    return pix, terms


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and its logical CPU count."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def cpu_baseline(guides, pairs, p, levels, iters, seed, N, budget_s):
    """The oracle on the host: as many of the blend's pairs as fit the time
    budget on all threads, then one pair on one thread and the 64x64 pair
    (1 level, 5 iterations) on one thread, median of 20."""
    import numpy as np
    import oracle
    from paper_2311_09265_amd import synth
    h, w = guides.shape[1:3]
    threads = oracle.get_threads()
    done, t0 = 0, time.perf_counter()
    for (j, i) in pairs:
        oracle.patchmatch(guides[j], guides[i], p, levels, iters, seed, j * N + i)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    pix, _ = pm_work(done, h, w, levels, iters, p)
    model, ncpu = cpu_model()
    single = {}
    try:
        oracle.set_threads(1)
        (j, i) = pairs[0]
        t1 = time.perf_counter()
        oracle.patchmatch(guides[j], guides[i], p, levels, iters, seed, j * N + i)
        d1 = time.perf_counter() - t1
        pix1, _ = pm_work(1, h, w, levels, iters, p)
        single["blend_pair"] = {"ms": round(d1 * 1e3, 2), "mpix_iter_per_s": round(pix1 / d1 / 1e6, 3),
                                "pair": "%dx%d, %d levels x %d iterations" % (h, w, levels, iters)}
        a, b, _ = synth.translation_pair(synth.CONFIG_SEED[1])
        ts = []
        for _ in range(20):
            t1 = time.perf_counter()
            oracle.patchmatch(a, b, p, 1, 5, synth.PHILOX_SEED[1], 0)
            ts.append(time.perf_counter() - t1)
        d1 = float(np.median(ts))
        single["pair_64x64"] = {"ms_median_of_20": round(d1 * 1e3, 3),
                                "mpix_iter_per_s": round(64 * 64 * 5 / d1 / 1e6, 3)}
    finally:
        oracle.set_threads(threads)
    return {"value": round(pix / dt / 1e6, 3), "unit": "Mpix·iter/s", "cores": threads,
            "kind": "oracle", "cpu_model": model, "logical_cpus": ncpu,
            "build": "gcc -O3, OpenMP over rows, no hand-written SIMD",
            "sample": "%d of %d pairs, each the full %d-level x %d-iteration PatchMatch of a %dx%d pair "
                      "(C oracle, %d threads), %.1f s" % (done, len(pairs), levels, iters, h, w, threads, dt),
            "single_thread": single}


def bench_learned(ctx, fbm, g, s, out, M, p, levels, seed, wpath, args, pairs, N, h, w, plain_energy):
    """The same blend with every pair's coarsest level seeded by the proposal
    network (FB_LEARNED_SEED) and args.learned_iters iterations per level."""
    import numpy as np
    import torch
    from paper_2311_09265_amd import proposal
    params, meta = proposal.load(wpath)
    ctx.fb_unet_load(torch.from_numpy(params).cuda())
    lprm = fbm.make_params(p, levels, args.learned_iters, seed, fbm.FB_LEARNED_SEED)
    for _ in range(max(args.warmup, 1)):
        ctx.fb_blend_window(g, s, M, lprm, out=out)
    torch.cuda.synchronize()
    ctx.fb_profile_enable(True)
    ctx.fb_profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.fb_blend_window(g, s, M, lprm, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    prof = ctx.fb_profile_read(reset=True)
    ctx.fb_profile_enable(False)
    log("learned: %.2f ms/step" % ms)
    # the guard: each seeded pair's coarsest level raced against plain@6 there
    gs = ctx.fb_guard_read()
    rejected = int((gs[:, 0] > gs[:, 1]).sum())
    nprm = fbm.make_params(p, levels, args.learned_iters, seed, fbm.FB_LEARNED_SEED | fbm.FB_NO_GUARD)
    ctx.fb_blend_window(g, s, M, nprm, out=out)
    torch.cuda.synchronize()
    # timed like the guarded steps (HIP events around every launch), so the
    # difference is the guard's work alone
    ctx.fb_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.fb_blend_window(g, s, M, nprm, out=out)
    torch.cuda.synchronize()
    ms_unguarded = (time.perf_counter() - t0) / args.steps * 1e3
    ctx.fb_profile_read(reset=True)
    ctx.fb_profile_enable(False)
    log("learned without the guard: %.2f ms/step" % ms_unguarded)
    graph_ms = None
    if not args.no_graph:
        # the guarded learned steps replayed as one HIP graph per step
        gprm = fbm.make_params(p, levels, args.learned_iters, seed, fbm.FB_LEARNED_SEED | fbm.FB_USE_GRAPH)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            ctx.fb_blend_window(g, s, M, gprm, out=out)
            side.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                ctx.fb_blend_window(g, s, M, gprm, out=out)
            side.synchronize()
            graph_ms = round((time.perf_counter() - t0) / args.steps * 1e3, 3)
        torch.cuda.current_stream().wait_stream(side)
        log("learned, graph replay: %.2f ms/step" % graph_ms)
    guard = {"rule": "each seeded pair's coarsest level (seeded start, %d iterations) is raced against the "
                     "plain random start with one iteration more (%d); a seed whose summed energy is the larger "
                     "is rejected and the pair's result is plain@6 exactly" % (args.learned_iters,
                                                                                min(args.learned_iters + 1, 6)),
             "pairs": int(gs.shape[0]), "rejected": rejected,
             "firing_rate": round(rejected / max(int(gs.shape[0]), 1), 4),
             "seeded_over_plain_coarse_energy_mean": round(float((gs[:, 0].double() / gs[:, 1].double()).mean()), 4),
             "ms_per_step_without_guard": round(ms_unguarded, 3),
             "guard_cost_ms_per_step": round(ms - ms_unguarded, 3)}
    energy = plain_same = None
    if not args.no_energy:
        pyrs = [ctx.fb_build_pyramid(g[f], levels, p) for f in range(N)]
        descs = [dict(src_pyr=pyrs[j], tgt_pyr=pyrs[i], h=h, w=w, levels=levels, pair_id=j * N + i)
                 for (j, i) in pairs]
        energies = [e for _, e in ctx.fb_patchmatch_batch(descs, lprm)]
        energy = round(float(fbm.energy_u32(torch.stack(energies)).double().mean().item()), 2)
        pprm = fbm.make_params(p, levels, args.learned_iters, seed)
        energies = [e for _, e in ctx.fb_patchmatch_batch(descs, pprm)]
        plain_same = round(float(fbm.energy_u32(torch.stack(energies)).double().mean().item()), 2)
        del energies, pyrs
    hc, wc = -(-h // (1 << (levels - 1))), -(-w // (1 << (levels - 1)))
    flops = fbm.load_library().fb_unet_forward_flops(len(pairs), -(-hc // 8) * 8, -(-wc // 8) * 8)
    unet_ms = prof["unet"][1] / args.steps
    pix, _ = pm_work(len(pairs), h, w, levels, args.learned_iters, p)
    tf = flops / (unet_ms / 1e3) / 1e12 if unet_ms > 0 else 0.0
    margin = 0.0
    accepted = (energy is not None and plain_energy is not None and energy <= plain_energy * (1 + margin))
    return {"ms_per_step": round(ms, 3), "blended_frames_per_s": round(N / (ms / 1e3), 3),
            "graph_ms_per_step": graph_ms,
            "iters_per_level": args.learned_iters, "pixel_iterations_per_step": pix,
            "mean_level0_patch_energy": energy, "plain_mean_level0_patch_energy": plain_energy,
            "plain_same_iters_mean_level0_patch_energy": plain_same,
            "energy_margin": margin, "accepted": accepted, "guard": guard,
            "speedup_vs_plain": None,
            "kernel_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in prof.items() if v[0]},
            "network_roofline": {"bound": "mfma", "kernel": "k_conv3x3 (forward)", "achieved": round(tf, 3),
                                 "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tf / 2500.0, 5),
                                 "flops_per_step": flops},
            "weights": os.path.relpath(wpath, ROOT), "training": {k: meta.get(k) for k in
                                                                   ("pairs", "steps", "val_loss", "train_seconds")}}


def bench_style(ctx, fbm, g, s, out, M, p, levels, iters, seed, args, pairs, N, h, w):
    """The same blend with every NNF estimated under the guide + style loss of
    Eq. 3 (FB_STYLE_LOSS, alpha = 1): a refresh of the remapped style before
    each iteration launch, and twice the byte-terms per candidate."""
    import torch
    sprm = fbm.make_params(p, levels, iters, seed, fbm.FB_STYLE_LOSS, 16)
    for _ in range(max(args.warmup, 1)):
        ctx.fb_blend_window(g, s, M, sprm, out=out)
    torch.cuda.synchronize()
    ctx.fb_profile_enable(True)
    ctx.fb_profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.fb_blend_window(g, s, M, sprm, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    prof = ctx.fb_profile_read(reset=True)
    ctx.fb_profile_enable(False)
    log("style loss: %.2f ms/step" % ms)
    pix, terms = pm_work(len(pairs), h, w, levels, iters, p)
    terms *= 2  # guide and style patches
    iter_ms = prof["pm_iter"][1] / args.steps
    tf = terms / (iter_ms / 1e3) / 1e12 if iter_ms > 0 else 0.0
    loss = None
    if not args.no_energy:
        pyrs = [ctx.fb_build_pyramid(g[f], levels, p) for f in range(N)]
        spyrs = [ctx.fb_build_pyramid(s[f], levels, p) for f in range(N)]
        descs = [dict(src_pyr=pyrs[j], tgt_pyr=pyrs[i], src_style_pyr=spyrs[j], h=h, w=w, levels=levels,
                      pair_id=j * N + i) for (j, i) in pairs]
        energies = [e for _, e in ctx.fb_patchmatch_batch(descs, sprm)]
        loss = round(float(fbm.energy_u32(torch.stack(energies)).double().mean().item()) / 16.0, 2)
        del energies, pyrs, spyrs
    return {"alpha": 1.0, "ms_per_step": round(ms, 3), "blended_frames_per_s": round(N / (ms / 1e3), 3),
            "mpix_iter_per_s": round(pix / (ms / 1e3) / 1e6, 3),
            "kernel_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in prof.items() if v[0]},
            "iteration_roofline": {"bound": "alu", "kernel": "k_pm_iter (Eq. 3)", "achieved": round(tf, 3),
                                   "peak": round(DOT4_PEAK_TOPS, 1), "unit": "TOP/s",
                                   "frac": round(tf / DOT4_PEAK_TOPS, 4)},
            "mean_level0_eq3_loss": loss}


def fast_mode_nnfs(N, M):
    """Distinct NNFs the fast mode estimates (tables of Alg. 3 in both frame
    orders, plus the remaps of Alg. 5's queries)."""
    Lmax = max(0, (N - 1).bit_length())
    need = set()
    frame = lambda d, k: N - 1 - k if d else k
    for d in (0, 1):
        for i in range(N):
            j = i
            for L in range(Lmax):
                if (i >> L) & 1:
                    continue
                j |= 1 << L
                if j < N:
                    need.add((frame(d, i), frame(d, j)))
    for i in range(N):
        lo, hi = max(0, i - M), min(N - 1, i + M)
        for d, (l, r) in ((0, (lo, i)), (1, (N - 1 - hi, N - 1 - i))):
            k = r
            while k >= l:
                L = 0
                while (k >> L) & 1 and k - (1 << (L + 1)) + 1 >= l:
                    L += 1
                if k != r:
                    need.add((frame(d, k), i))
                k -= 1 << L
    return len(need)


def bench_fast(ctx, fbm, g, s, out, p, levels, iters, seed, args, N, h, w):
    """Fast mode (FB_FAST_BLEND, Alg. 3-5 with Eq. 6) against the balanced
    window blend, at window radius 5 and 15."""
    import torch
    res = {}
    for M in (5, 15):
        row = {}
        for name, flags in (("fast", fbm.FB_FAST_BLEND), ("balanced", 0)):
            prm = fbm.make_params(p, levels, iters, seed, flags)
            ctx.fb_blend_window(g, s, M, prm, out=out)
            torch.cuda.synchronize()
            steps = max(1, args.steps // 2)
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.fb_blend_window(g, s, M, prm, out=out)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            nnfs = fast_mode_nnfs(N, M) if flags else len(window_pairs(N, M))
            row[name] = {"ms_per_step": round(ms, 3), "blended_frames_per_s": round(N / (ms / 1e3), 3), "nnfs": nnfs}
            log("window radius %d, %s: %.2f ms/step, %d NNFs" % (M, name, ms, nnfs))
        row["speedup_fast_vs_balanced"] = round(row["balanced"]["ms_per_step"] / row["fast"]["ms_per_step"], 3)
        res["M=%d" % M] = row
    return res


def bench_accurate(ctx, fbm, g, s, out, M, p, levels, iters, seed, args, N):
    """Accurate mode (FB_ACCURATE_BLEND, Eq. 7-8, alpha = 1) on the same blend:
    the window NNFs twice (Eq. 1, then Eq. 8 against T^-) and two remap
    passes."""
    import torch
    prm = fbm.make_params(p, levels, iters, seed, fbm.FB_ACCURATE_BLEND, 16)
    ctx.fb_blend_window(g, s, M, prm, out=out)
    torch.cuda.synchronize()
    ctx.fb_profile_enable(True)
    ctx.fb_profile_read(reset=True)
    steps = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.fb_blend_window(g, s, M, prm, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    prof = ctx.fb_profile_read(reset=True)
    ctx.fb_profile_enable(False)
    log("accurate mode: %.2f ms/step" % ms)
    return {"alpha": 1.0, "ms_per_step": round(ms, 3), "blended_frames_per_s": round(N / (ms / 1e3), 3),
            "kernel_ms_per_step": {k: round(v[1] / steps, 3) for k, v in prof.items() if v[0]}}


def bench_interp(ctx, fbm, args):
    """The interpolation workload (64 frames of 1024x576, keyframes every 16
    frames, 4 levels x 6 iterations; Eq. 9): plain, with tracking, and with
    tracking + the pairwise alignment loss (Eq. 10, alpha = 1)."""
    import torch
    from paper_2311_09265_amd import synth
    guides, keys, key_styles = synth.interp_workload()
    N, h, w = guides.shape[:3]
    g = torch.from_numpy(guides).cuda()
    ks = torch.from_numpy(key_styles).cuda()
    out = torch.empty((N, h, w, 3), dtype=torch.float32, device=g.device)
    seed = synth.PHILOX_SEED[3]
    res = {"workload": "interpolation %d frames %dx%d, keys %s, 4 levels x 6 iterations" % (N, w, h, [int(k) for k in keys])}
    for name, flags in (("plain", 0), ("tracking", fbm.FB_TRACKING),
                        ("tracking_align", fbm.FB_TRACKING | fbm.FB_ALIGN)):
        prm = fbm.make_params(2, 4, 6, seed, flags, 16)
        ctx.fb_interpolate(g, list(keys), ks, prm, out=out)
        torch.cuda.synchronize()
        steps = max(1, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.fb_interpolate(g, list(keys), ks, prm, out=out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        res[name] = {"ms_per_call": round(ms, 3), "frames_per_s": round(N / (ms / 1e3), 3)}
        log("interpolation %s: %.2f ms per call" % (name, ms))
    del g, ks, out
    return res


def bench_pair64(ctx, fbm, args):
    """The 64x64 pair (value noise shifted by (3, -2) plus noise, 1 level, patch
    5x5, 5 iterations): one fb_patchmatch_batch call, eager and replayed as a
    HIP graph, median of 100 calls each (a latency figure: 20,480
    pixel-iterations per call)."""
    import numpy as np
    import torch
    from paper_2311_09265_amd import synth
    a, b, _ = synth.translation_pair(synth.CONFIG_SEED[1])
    pa = ctx.fb_build_pyramid(torch.from_numpy(a).cuda(), 1, 2)
    pb = ctx.fb_build_pyramid(torch.from_numpy(b).cuda(), 1, 2)
    desc = [dict(src_pyr=pa, tgt_pyr=pb, h=64, w=64, levels=1, pair_id=0)]
    res = {"workload": "one 64x64 pair, 1 level, patch 5x5, 5 iterations", "pixel_iterations_per_call": 64 * 64 * 5}
    for name, flags in (("eager", 0), ("graph", fbm.FB_USE_GRAPH)):
        prm = fbm.make_params(2, 1, 5, synth.PHILOX_SEED[1], flags)
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            for _ in range(5):
                ctx.fb_patchmatch_batch(desc, prm)
            side.synchronize()
            ts = []
            for _ in range(100):
                t0 = time.perf_counter()
                ctx.fb_patchmatch_batch(desc, prm)
                side.synchronize()
                ts.append(time.perf_counter() - t0)
        med = float(np.median(ts))
        res[name] = {"ms_median_of_100": round(med * 1e3, 4), "mpix_iter_per_s": round(64 * 64 * 5 / med / 1e6, 3)}
        log("64x64 pair, %s: %.3f ms per call" % (name, med * 1e3))
    return res


def bench_pairs_512(ctx, fbm, g, p, levels, iters, learned_iters, seed, args, pairs, N, h, w, learned):
    """PatchMatch alone for the 290 window pairs of the 512x512 blend (pyramids
    built beforehand), batched in one fb_patchmatch_batch call against one
    call per pair, for plain (6 iterations per level) and, when the network
    is loaded, learned seeds (2 per level, guarded)."""
    import torch
    pyrs = [ctx.fb_build_pyramid(g[f], levels, p) for f in range(N)]
    descs = [dict(src_pyr=pyrs[j], tgt_pyr=pyrs[i], h=h, w=w, levels=levels, pair_id=j * N + i) for (j, i) in pairs]
    res = {"workload": "%d pairs of %dx%d, %d levels, PatchMatch only" % (len(pairs), h, w, levels)}
    modes = [("plain", iters, 0)]
    if learned:
        modes.append(("learned", learned_iters, fbm.FB_LEARNED_SEED))
    steps = max(1, args.steps // 2)
    for name, its, flags in modes:
        pix, _ = pm_work(len(pairs), h, w, levels, its, p)
        prm = fbm.make_params(p, levels, its, seed, flags)
        out = {"pixel_iterations_per_call": pix}
        for how in ("batched", "per_pair"):
            if how == "per_pair":
                def run():
                    for d in descs:
                        ctx.fb_patchmatch_batch([d], prm)
            else:
                def run():
                    ctx.fb_patchmatch_batch(descs, prm)
            run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                run()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / steps * 1e3
            out[how] = {"ms_per_call": round(ms, 3), "mpix_iter_per_s": round(pix / (ms / 1e3) / 1e6, 3)}
            log("%d pairs, %s, %s: %.2f ms per call" % (len(pairs), name, how, ms))
        out["speedup_batched_vs_per_pair"] = round(out["per_pair"]["ms_per_call"] / out["batched"]["ms_per_call"], 3)
        res[name] = out
    del descs, pyrs
    return res


def bench_mixed(ctx, fbm, args):
    """The mixed-size batch: 12 pairs (t, t + d), d in 1..5, of each of 256x256
    and 512x512 (3 levels) and 1024x576 and 1280x720 (4 levels), 6 iterations:
    all 48 whole pyramids in one fb_patchmatch_batch call (grouped launches,
    eager and replayed as a graph) against one call per pair."""
    import torch
    from paper_2311_09265_amd import synth
    p, iters = 2, 6
    seed = synth.PHILOX_SEED[4]
    pairs = synth.mixed_pairs()
    descs, pix = [], 0
    for k, (a, b, lv) in enumerate(pairs):
        h, w = a.shape[:2]
        descs.append(dict(src_pyr=ctx.fb_build_pyramid(torch.from_numpy(a).cuda(), lv, p),
                          tgt_pyr=ctx.fb_build_pyramid(torch.from_numpy(b).cuda(), lv, p),
                          h=h, w=w, levels=lv, pair_id=k))
        pix += n_pix_iters(h, w, lv, iters)
    res = {"workload": "48 pairs: 12 each of 256x256 and 512x512 (3 levels), 1024x576 and 1280x720 "
                       "(4 levels), patch 5x5, 6 iterations",
           "pixel_iterations_per_call": pix}
    steps = max(1, args.steps // 2)
    for name, flags, per_pair in (("batched", 0, False), ("batched_graph", fbm.FB_USE_GRAPH, False),
                                  ("per_pair", 0, True)):
        prm = fbm.make_params(p, 4, iters, seed, flags)
        if per_pair:
            def run():
                for d in descs:
                    ctx.fb_patchmatch_batch([d], prm)
        else:
            def run():
                ctx.fb_patchmatch_batch(descs, prm)
        run()  # tunes the tile shape of every batch shape; captures the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        res[name] = {"ms_per_call": round(ms, 3), "mpix_iter_per_s": round(pix / (ms / 1e3) / 1e6, 3)}
        log("mixed batch, %s: %.2f ms per call" % (name, ms))
    res["speedup_batched_graph_vs_per_pair"] = round(res["per_pair"]["ms_per_call"] /
                                                     res["batched_graph"]["ms_per_call"], 3)
    del descs
    return res


def n_pix_iters(h, w, levels, iters):
    return sum(hl * wl for hl, wl in level_sizes(h, w, levels)) * iters


# the sources that decide what the iteration kernel does (its code, the
# shared constants and the pyramid layout it reads)
ITER_KERNEL_SOURCES = ("patchmatch.hip", "fb_common.h", "pyramid.hip")


def iter_kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for name in ITER_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_09265_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def iter_kernel_traffic():
    """HBM bytes per launch of the PatchMatch iteration kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel sources."""
    summ = os.path.join(ROOT, "profiles", "pm_iter_counters_blend512.json")
    if not os.path.exists(summ):
        return None, "no counter summary"
    with open(summ) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256") != iter_kernel_sha():
        return None, "counters were taken on another version of the kernel"
    return d["hbm_bytes_per_launch"], d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=32)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--no-energy", action="store_true", help="skip the mean-energy pass")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2311_09265_amd", "weights", "proposal_unet.npz"),
                    help="trained proposal network; the learned comparison is skipped if absent")
    ap.add_argument("--learned-iters", type=int, default=2)
    ap.add_argument("--no-style", action="store_true", help="skip the Eq. 3 (guide + style loss) comparison")
    ap.add_argument("--no-fast", action="store_true", help="skip the fast-mode comparison")
    ap.add_argument("--no-accurate", action="store_true", help="skip the accurate-mode timing")
    ap.add_argument("--no-interp", action="store_true", help="skip the interpolation timings")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-size batch timings")
    ap.add_argument("--no-pair64", action="store_true", help="skip the 64x64 single-pair latency")
    ap.add_argument("--no-pairs512", action="store_true",
                    help="skip PatchMatch of the 290 blend pairs batched vs per pair")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB once (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2311_09265_amd import fastblend as fbm
    from paper_2311_09265_amd import synth

    N, h, w, M, p, levels, iters = args.frames, args.size, args.size, 5, 2, 3, 6
    seed = synth.PHILOX_SEED[2]
    log("generating %d-frame %dx%d synthetic video" % (N, h, w))
    guides, styles = synth.blend_workload(N, h, w)
    pairs = window_pairs(N, M)
    pix, terms = pm_work(len(pairs), h, w, levels, iters, p)

    dev = torch.device("cuda", 0)
    ctx = fbm.Context(0)
    g = torch.from_numpy(guides).to(dev)
    s = torch.from_numpy(styles).to(dev)
    out = torch.empty((N, h, w, 3), dtype=torch.float32, device=dev)
    prm = fbm.make_params(p, levels, iters, seed)
    for k in range(args.warmup):
        ctx.fb_blend_window(g, s, M, prm, out=out)
        torch.cuda.synchronize()
        log("warmup step %d done" % k)

    # timed region: eager launches, every launch bracketed by HIP events on the library's stream
    ctx.fb_profile_enable(True)
    ctx.fb_profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.fb_blend_window(g, s, M, prm, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.fb_profile_read(reset=True)
    ctx.fb_profile_enable(False)
    ms = (t1 - t0) / args.steps * 1e3
    log("timed %d steps: %.2f ms/step" % (args.steps, ms))

    graph_ms = None
    if not args.no_graph:
        # the same steps replayed as one HIP graph per step
        gprm = fbm.make_params(p, levels, iters, seed, fbm.FB_USE_GRAPH)
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            ctx.fb_blend_window(g, s, M, gprm, out=out)
            side.synchronize()
            t2 = time.perf_counter()
            for _ in range(args.steps):
                ctx.fb_blend_window(g, s, M, gprm, out=out)
            side.synchronize()
            t3 = time.perf_counter()
        graph_ms = round((t3 - t2) / args.steps * 1e3, 3)
        log("graph replay: %.2f ms/step" % graph_ms)

    mean_energy = None
    if not args.no_energy:
        # quality: mean level-0 patch energy of all pairs (outside the timed region)
        pyrs = [ctx.fb_build_pyramid(g[f], levels, p) for f in range(N)]
        descs = [dict(src_pyr=pyrs[j], tgt_pyr=pyrs[i], h=h, w=w, levels=levels, pair_id=j * N + i)
                 for (j, i) in pairs]
        energies = [e for _, e in ctx.fb_patchmatch_batch(descs, prm)]
        mean_energy = round(float(fbm.energy_u32(torch.stack(energies)).double().mean().item()), 2)
        del energies, pyrs

    fast = None
    if not args.no_fast:
        fast = bench_fast(ctx, fbm, g, s, out, p, levels, iters, seed, args, N, h, w)

    interp = None
    if not args.no_interp:
        interp = bench_interp(ctx, fbm, args)

    mixed = None
    if not args.no_mixed:
        mixed = bench_mixed(ctx, fbm, args)

    pair64 = None
    if not args.no_pair64:
        pair64 = bench_pair64(ctx, fbm, args)

    # the row-gather rate that bounds the iteration kernel, measured on level 0
    # of frame 0's pyramid (1 MB, L2-resident like a pair's source level)
    probe_pyr = ctx.fb_build_pyramid(g[0], 1, p)
    torch.cuda.synchronize()
    gather = {"divergent_rows_per_s": ctx.fb_gather_probe(probe_pyr, h, w, True),
              "coherent_rows_per_s": ctx.fb_gather_probe(probe_pyr, h, w, False)}
    del probe_pyr

    accurate = None
    if not args.no_accurate:
        accurate = bench_accurate(ctx, fbm, g, s, out, M, p, levels, iters, seed, args, N)

    style = None
    if not args.no_style:
        style = bench_style(ctx, fbm, g, s, out, M, p, levels, iters, seed, args, pairs, N, h, w)

    learned = None
    wpath = args.weights
    if wpath and os.path.exists(wpath):
        learned = bench_learned(ctx, fbm, g, s, out, M, p, levels, seed, wpath, args, pairs, N, h, w, mean_energy)

    pairs512 = None
    if not args.no_pairs512:
        pairs512 = bench_pairs_512(ctx, fbm, g, p, levels, iters, args.learned_iters, seed, args, pairs, N, h, w,
                                   learned is not None)

    n_iter, iter_ms = prof["pm_iter"]
    iter_ms_step = iter_ms / args.steps
    # the remap and window sum (Alg. 2, Eq. 2) against HBM: its compulsory
    # bytes are every pair's field (4 bytes per pixel, packed) and every padded
    # 4-byte style frame read once, and the fp32 RGB outputs written once
    pitch = (w + 2 * p + 15) // 16 * 16
    remap_bytes = len(pairs) * h * w * 4 + N * (h + 2 * p) * pitch * 4 + N * h * w * 12
    remap_ms_step = prof["remap"][1] / args.steps
    remap_gbs = remap_bytes / (remap_ms_step / 1e3) / 1e9 if remap_ms_step > 0 else 0.0
    traffic, traffic_info = iter_kernel_traffic()
    achieved = terms / (iter_ms_step / 1e3) / 1e12
    kernel_ms = {k: round(v[1] / args.steps, 3) for k, v in prof.items() if v[0]}

    if args.calib_copy_mib:
        x = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("calibration copy of %d MiB done" % args.calib_copy_mib)
        del x, y

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) for up to %.0f s" % args.cpu_seconds)
        cpu = cpu_baseline(guides, pairs, p, levels, iters, seed, N, args.cpu_seconds)
        log("cpu baseline: %s" % cpu)

    res = {
        "metric": METRIC,
        "value": round(pix / (ms / 1e3) / 1e6, 3),
        "unit": "Mpix·iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "blend %d frames %dx%d RGB u8, window radius %d (%d pairs), patch %dx%d, "
                               "%d levels x %d iterations, plain random init" % (
                                   N, h, w, M, len(pairs), 2 * p + 1, 2 * p + 1, levels, iters),
                   "frames": N, "height": h, "width": w, "window_radius": M, "pairs": len(pairs),
                   "patch": 2 * p + 1, "levels": levels, "iters": iters},
        "blended_frames_per_s": round(N / (ms / 1e3), 3),
        "graph_ms_per_step": graph_ms,
        "pixel_iterations_per_step": pix,
        "mean_level0_patch_energy": mean_energy,
        "kernel_ms_per_step": kernel_ms,
        "roofline": {"bound": "alu", "kernel": "k_pm_iter",
                     "achieved": round(achieved, 3), "peak": round(DOT4_PEAK_TOPS, 1), "unit": "TOP/s",
                     "frac": round(achieved / DOT4_PEAK_TOPS, 4), "traffic": traffic,
                     "traffic_note": ("L2-to-fabric bytes per launch (includes Infinity-Cache hits, so an upper "
                                      "bound on HBM bytes), rocprofv3 FETCH_SIZE x %.2f + WRITE_SIZE x %.2f "
                                      "(copy-calibrated), %s" % (traffic_info["fetch_scale"], traffic_info["write_scale"],
                                                                 traffic_info["summary"])
                                      if traffic is not None else traffic_info),
                     "work": "byte-terms of Eq. 1 (one per squared channel difference) per step: %d" % terms,
                     "avg_launch_ms": round(iter_ms / max(n_iter, 1), 4), "launches": n_iter},
        "remap_roofline": {"bound": "hbm", "kernel": "k_remap_sum", "achieved": round(remap_gbs, 1),
                           "peak": 8000.0, "unit": "GB/s", "frac": round(remap_gbs / 8000.0, 4),
                           "work": "compulsory bytes per step: %d (fields, padded styles, fp32 outputs); the "
                                   "kernel is bound by L1 gathers of (2p+1)^2 source pixels per remapped pixel"
                                   % remap_bytes},
        "gather_roof": {
            "kernel": "k_gather_probe",
            "divergent_rows_per_s": round(gather["divergent_rows_per_s"], 0),
            "coherent_rows_per_s": round(gather["coherent_rows_per_s"], 0),
            "note": "lane-rows per second: 5-pixel rows (a 16-byte and a 4-byte load each, folded with v_dot4) "
                    "gathered from a 512x512 padded level by 2048 x 256 lanes, every lane at its own random "
                    "position (random-search candidates) or each wave at 64 consecutive pixels (propagation "
                    "candidates): the two ends of the gather rate that bounds k_pm_iter"},
        "cpu_baseline": cpu,
        "learned": learned,
        "style_loss": style,
        "fast_mode": fast,
        "accurate_mode": accurate,
        "interpolation": interp,
        "mixed_batch": mixed,
        "pairs_512": pairs512,
        "pair_64x64": pair64,
    }
    if learned:
        learned["speedup_vs_plain"] = round(ms / learned["ms_per_step"], 3)
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
