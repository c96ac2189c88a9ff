"""Training and evaluation of the learned PatchMatch proposal.

The network (kernels in csrc/unet*.hip, C ABI fb_unet_*) maps a frame pair at
the coarsest pyramid level to the offset field of its matches.  It is trained
on NNFs that the plain method computes (fb_patchmatch_batch: random
initialisation, levels x iters concurrent PatchMatch), then seeds the
coarsest level of PatchMatch in place of the random draw (FB_LEARNED_SEED),
which lets the finer levels run fewer iterations.  Plain PatchMatch stays the
default, the fallback and the reference a model is measured against: ``evaluate`` measures the mean level-0
patch energy of the seeded, shorter run against the plain run, and a model is
accepted only if it stays within the stated margin.

Data: seeded synthetic 512x512 pairs, half value-noise translations (random
integer shift in [-16, 16]^2, +-4 pixel noise), half frame pairs (t, t+d),
d in [1, 5], of sprite videos; the sprite half is a deliberate addition so
the network sees the local motion of the blending workload.

Label of coarse pixel (r, c) at level K-1 (scale s = 2^(K-1)): the mean level-0
offset F(v) - v over its s x s block, divided by s; weight 1 where the block's
mean energy is at most twice the pair's median block energy and its offsets
spread by at most one coarse pixel, else 0.

Everything that runs on the GPU goes through the library: pyramids, plain
PatchMatch, the network input, forward, backward and Adam.  PyTorch only
holds the tensors and forms the per-block label statistics.

Usage:  python -m paper_2311_09265_amd.proposal train --out WEIGHTS.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

from . import synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "proposal_unet.npz")

SIZE, LEVELS, P, ITERS = 512, 3, 2, 6
TRAIN_SEED = 0xFB0C0DE5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- data ----
def _translation_pairs(seed: int, n: int):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        d = tuple(int(v) for v in rng.integers(-16, 17, size=2))
        a, b, _ = synth.translation_pair(seed * 131 + k, size=SIZE, shift=d, noise=4, margin=16)
        out.append((a, b))
    return out


def _sprite_pairs(seed: int, n: int):
    rng = np.random.default_rng(seed)
    vid = synth.sprite_video(16, SIZE, SIZE, seed)
    out = []
    for _ in range(n):
        d = int(rng.integers(1, 6))
        t = int(rng.integers(0, 16 - d))
        out.append((vid[t], vid[t + d]) if rng.random() < 0.5 else (vid[t + d], vid[t]))
    return out


def _job(args):
    kind, seed, n = args
    return _translation_pairs(seed, n) if kind == "t" else _sprite_pairs(seed, n)


def training_pairs(n_pairs: int, seed: int = TRAIN_SEED, workers: int = 8):
    """n_pairs seeded (source, target) uint8 frame pairs (half translations, half sprites)."""
    jobs = []
    per = 16
    for k in range((n_pairs // 2 + per - 1) // per):
        jobs.append(("t", seed + 2 * k, per))
        jobs.append(("s", seed + 2 * k + 1, per))
    with get_context("fork").Pool(workers) as pool:
        chunks = pool.map(_job, jobs)
    trans = [p for c, j in zip(chunks, jobs) if j[0] == "t" for p in c][: n_pairs // 2]
    spr = [p for c, j in zip(chunks, jobs) if j[0] == "s" for p in c][: n_pairs - n_pairs // 2]
    pairs = [x for ab in zip(trans, spr) for x in ab]
    return pairs[:n_pairs]


def prepare(ctx, pairs, chunk: int = 64):
    """GPU tensors (x6 [n][H][W][6], target [n][H][W][2], mask [n][H][W]) from plain PatchMatch."""
    import torch
    import torch.nn.functional as F
    from . import fastblend as fbm
    dev = ctx.device
    s = 1 << (LEVELS - 1)
    prm = fbm.make_params(P, LEVELS, ITERS, TRAIN_SEED)
    xs, ts, ms = [], [], []
    rr = torch.arange(SIZE, device=dev, dtype=torch.float32)
    for c0 in range(0, len(pairs), chunk):
        part = pairs[c0:c0 + chunk]
        frames = torch.from_numpy(np.stack([f for ab in part for f in ab])).to(dev)
        pyrs = [ctx.fb_build_pyramid(frames[k], LEVELS, P) for k in range(len(frames))]
        descs = [dict(src_pyr=pyrs[2 * k], tgt_pyr=pyrs[2 * k + 1], h=SIZE, w=SIZE, levels=LEVELS,
                      pair_id=c0 + k) for k in range(len(part))]
        outs = ctx.fb_patchmatch_batch(descs, prm)
        for k, (nnf, en) in enumerate(outs):
            xs.append(ctx.fb_unet_pair_input(pyrs[2 * k], pyrs[2 * k + 1], SIZE, SIZE, LEVELS, P))
            off = nnf.float() - torch.stack(torch.meshgrid(rr, rr, indexing="ij"), -1)
            o = off.permute(2, 0, 1)[None]
            mean = F.avg_pool2d(o, s)[0]
            var = (F.avg_pool2d(o * o, s)[0] - mean * mean).clamp(min=0)
            eb = F.avg_pool2d(en.float()[None, None], s)[0, 0]
            ok = (eb <= 2 * eb.median()) & (var.sum(0).sqrt() <= s)
            ts.append((mean / s).permute(1, 2, 0).contiguous())
            ms.append(ok.float())
        log("prepared %d / %d pairs" % (min(c0 + chunk, len(pairs)), len(pairs)))
    return torch.stack(xs), torch.stack(ts), torch.stack(ms)


# ------------------------------------------------------------- training ----
CHECKPOINT_VERSION = 1


def save_checkpoint(ctx, path, step: int, steps: int, batch: int, lr: float, seed: int, gen):
    """Everything training needs to continue exactly: the parameters and Adam
    moments (flat fp32), Adam's step count, the minibatch generator's state,
    the loop position and the schedule's arguments (version-tagged npz)."""
    params, m, v, adam_step = ctx.fb_unet_save_state()
    meta = {"version": CHECKPOINT_VERSION, "step": int(step), "steps": int(steps), "batch": int(batch),
            "lr": float(lr), "seed": int(seed), "adam_step": int(adam_step)}
    tmp = path + ".tmp.npz"
    np.savez(tmp, params=params.cpu().numpy(), adam_m=m.cpu().numpy(), adam_v=v.cpu().numpy(),
             rng=gen.get_state().numpy(), meta=np.frombuffer(json.dumps(meta).encode(), np.uint8))
    os.replace(tmp, path)


def load_checkpoint(ctx, path, gen):
    """Restore a checkpoint written by save_checkpoint into the context and the
    generator; returns its meta (step, steps, batch, lr, seed)."""
    import torch
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(bytes(z["meta"]).decode())
        if meta.get("version") != CHECKPOINT_VERSION:
            raise ValueError("checkpoint version %r, expected %d" % (meta.get("version"), CHECKPOINT_VERSION))
        dev = ctx.device
        ctx.fb_unet_load_state(torch.from_numpy(z["params"]).to(dev), torch.from_numpy(z["adam_m"]).to(dev),
                               torch.from_numpy(z["adam_v"]).to(dev), meta["adam_step"])
        gen.set_state(torch.from_numpy(np.array(z["rng"])))
    return meta


def train(ctx, x, t, m, steps: int = 6000, batch: int = 32, lr: float = 1e-3, seed: int = 0, log_every: int = 500,
          ckpt: str = None, ckpt_every: int = 0, resume: bool = False, stop_after: int = None):
    """Adam on random minibatches, cosine-decayed learning rate; returns the
    mean training loss of every log_every steps.  With ckpt, a checkpoint is
    written every ckpt_every steps (and at the end); resume=True continues
    from it (the same parameters, Adam state, minibatch stream and schedule,
    so the result equals an uninterrupted run).  stop_after ends the loop
    after that many steps of this call (for a planned interruption)."""
    import torch
    g = torch.Generator().manual_seed(seed)
    n = x.shape[0]
    hist, losses = [], []
    start = 0
    if resume:
        meta = load_checkpoint(ctx, ckpt, g)
        if (meta["steps"], meta["batch"], meta["lr"], meta["seed"]) != (steps, batch, float(lr), seed):
            raise ValueError("checkpoint was written by a run with other arguments: %s" % meta)
        start = meta["step"]
    done = 0
    for step in range(start, steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(x.device)
        cur_lr = lr * 0.5 * (1 + np.cos(np.pi * step / steps))
        losses.append(ctx.fb_unet_train_step(x[idx].contiguous(), t[idx].contiguous(), m[idx].contiguous(),
                                             float(cur_lr)))
        done += 1
        last = step + 1 == steps or (stop_after is not None and done == stop_after)
        if (step + 1) % log_every == 0 or last:
            hist.append(float(torch.cat(losses).mean().cpu()))
            losses = []
            log("step %d loss %.4f" % (step + 1, hist[-1]))
        if ckpt and ((ckpt_every and (step + 1) % ckpt_every == 0) or last):
            save_checkpoint(ctx, ckpt, step + 1, steps, batch, lr, seed, g)
        if last:
            break
    return hist


def validation_loss(ctx, x, t, m, batch: int = 32):
    """Mean masked-L1 of the current parameters over (x, t, m), no update."""
    import torch
    vals = []
    for b0 in range(0, x.shape[0], batch):
        sl = slice(b0, b0 + batch)
        pred = ctx.fb_unet_forward(x[sl].contiguous())
        d = torch.clamp(m[sl].sum(), min=1.0)
        vals.append(float(((pred - t[sl]).abs().sum(-1) * m[sl]).sum() / d))
    return float(np.mean(vals))


def init_params(seed: int):
    """Kaiming-uniform initial parameters in the flat layout of fb_unet_load."""
    rng = np.random.default_rng(seed)
    layers = [(6, 32), (32, 32), (32, 48), (48, 48), (48, 96), (96, 96), (96, 192), (192, 192),
              (288, 96), (96, 96), (144, 48), (48, 48), (80, 32), (32, 32), (32, 2)]
    parts = []
    for ci, co in layers:
        bound = (6.0 / (9 * ci)) ** 0.5
        parts.append(rng.uniform(-bound, bound, size=co * ci * 9).astype(np.float32))
        parts.append(np.zeros(co, np.float32))
    return np.concatenate(parts)


def save(path, params, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=np.asarray(params, np.float32), meta=np.frombuffer(json.dumps(meta).encode(), np.uint8))


def load(path=DEFAULT_WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        return z["params"], json.loads(bytes(z["meta"]).decode())


# ----------------------------------------------------------- evaluation ----
def evaluate_blend_pairs(ctx, guides, pairs, iters_plain: int = ITERS, iters_learned: int = 2, seed: int = 0):
    """Mean level-0 energy over the pairs: plain random init at iters_plain,
    network seed at iters_learned (same pair ids and Philox key)."""
    import torch
    from . import fastblend as fbm
    N = guides.shape[0]
    h, w = guides.shape[1:3]
    pyrs = [ctx.fb_build_pyramid(guides[f], LEVELS, P) for f in range(N)]
    descs = [dict(src_pyr=pyrs[j], tgt_pyr=pyrs[i], h=h, w=w, levels=LEVELS, pair_id=j * N + i) for j, i in pairs]
    plain = ctx.fb_patchmatch_batch(descs, fbm.make_params(P, LEVELS, iters_plain, seed))
    learned = ctx.fb_patchmatch_batch(descs, fbm.make_params(P, LEVELS, iters_learned, seed, fbm.FB_LEARNED_SEED))
    e_plain = float(torch.stack([e for _, e in plain]).double().mean())
    e_learned = float(torch.stack([e for _, e in learned]).double().mean())
    return e_plain, e_learned


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--out", default=DEFAULT_WEIGHTS)
    tr.add_argument("--pairs", type=int, default=4000)
    tr.add_argument("--val", type=int, default=200)
    tr.add_argument("--steps", type=int, default=6000)
    tr.add_argument("--batch", type=int, default=32)
    tr.add_argument("--lr", type=float, default=1e-3)
    args = ap.parse_args()

    t0 = time.time()
    log("generating %d training pairs" % args.pairs)
    pairs = training_pairs(args.pairs, workers=min(16, os.cpu_count() or 1))
    log("generated in %.1f s" % (time.time() - t0))
    import torch
    from . import fastblend as fbm
    ctx = fbm.Context(0)
    x, t, m = prepare(ctx, pairs)
    del pairs
    nv = args.val
    xv, tv, mv = x[-nv:], t[-nv:], m[-nv:]
    x, t, m = x[:-nv], t[:-nv], m[:-nv]
    ctx.fb_unet_load(torch.from_numpy(init_params(TRAIN_SEED)).cuda())
    v0 = validation_loss(ctx, xv, tv, mv)
    t1 = time.time()
    hist = train(ctx, x, t, m, steps=args.steps, batch=args.batch, lr=args.lr)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    v1 = validation_loss(ctx, xv, tv, mv)
    log("validation loss %.4f -> %.4f, training %.1f s" % (v0, v1, train_s))
    # acceptance on the 512x512 blending workload's pairs
    guides, _ = synth.blend_workload()
    g = torch.from_numpy(guides).cuda()
    wpairs = [(j, i) for i in range(32) for j in range(max(0, i - 5), min(31, i + 5) + 1) if j != i]
    e_plain, e_learned = evaluate_blend_pairs(ctx, g, wpairs, seed=synth.PHILOX_SEED[2])
    log("blend pairs: plain@%d mean energy %.1f, learned@2 %.1f" % (ITERS, e_plain, e_learned))
    params = ctx.fb_unet_save().cpu().numpy()
    meta = dict(pairs=args.pairs - nv, val_pairs=nv, steps=args.steps, batch=args.batch, lr=args.lr,
                train_loss=hist, val_loss_init=v0, val_loss=v1, train_seconds=train_s,
                blend_energy_plain6=e_plain, blend_energy_learned2=e_learned,
                levels=LEVELS, iters_plain=ITERS, size=SIZE, seed=TRAIN_SEED)
    save(args.out, params, meta)
    print(json.dumps({k: v for k, v in meta.items() if k != "train_loss"}))
    ctx.close()


if __name__ == "__main__":
    main()
