"""Independent numpy formulations used to pin the oracle.

None of these calls the oracle or the GPU library.  They compute the same
quantities by a different route (whole-image vectorised patches, exhaustive
search, patch placement), so that a slip in the oracle's loops (a dropped
term, a wrong sign or index, a transposed operand) shows up as a mismatch.
"""
from __future__ import annotations

import numpy as np


def pad_edge(img: np.ndarray, p: int) -> np.ndarray:
    return np.pad(np.asarray(img, np.int64), ((p, p), (p, p), (0, 0)), mode="edge")


def all_patches(img: np.ndarray, p: int) -> np.ndarray:
    """Every (2p+1)x(2p+1)x3 clamp-to-edge patch, flattened: int64 [h*w][K]."""
    h, w = img.shape[:2]
    k = 2 * p + 1
    win = np.lib.stride_tricks.sliding_window_view(pad_edge(img, p), (k, k), axis=(0, 1))
    # win: [h][w][3][k][k]
    return win.reshape(h * w, -1)


def ssd(S, T, p, u, v) -> int:
    ps = all_patches(S, p)
    pt = all_patches(T, p)
    w = S.shape[1]
    d = ps[u[0] * w + u[1]] - pt[v[0] * w + v[1]]
    return int((d * d).sum())


def energy(S, T, F, p) -> np.ndarray:
    h, w = S.shape[:2]
    ps = all_patches(S, p)
    pt = all_patches(T, p)
    idx = (F[..., 0].astype(np.int64) * w + F[..., 1]).reshape(-1)
    d = ps[idx] - pt
    return (d * d).sum(axis=1).reshape(h, w)


def brute_force_nnf(S, T, p):
    """Exact NNF by exhaustive search; ties go to the lowest row-major source index.

    Returns (F int32 [h][w][2], E int64 [h][w]).
    """
    h, w = S.shape[:2]
    ps = all_patches(S, p)
    pt = all_patches(T, p)
    d = (pt * pt).sum(1)[:, None] + (ps * ps).sum(1)[None, :] - 2 * (pt @ ps.T)
    arg = d.argmin(axis=1)
    F = np.stack([arg // w, arg % w], axis=-1).reshape(h, w, 2).astype(np.int32)
    return F, d.min(axis=1).reshape(h, w)


def remap_by_patches(style, F, p) -> np.ndarray:
    """Remapping as first described in Section 3.3: cut the source into patches,
    place patch S[F(q)] centred at every target position q, and average where
    the placed patches overlap (only in-image positions count)."""
    h, w = style.shape[:2]
    k = 2 * p + 1
    sp = pad_edge(style, p)
    acc = np.zeros((h + 2 * p, w + 2 * p, 3), np.int64)
    cnt = np.zeros((h + 2 * p, w + 2 * p), np.int64)
    for qr in range(h):
        for qc in range(w):
            fr, fc = int(F[qr, qc, 0]), int(F[qr, qc, 1])
            acc[qr:qr + k, qc:qc + k] += sp[fr:fr + k, fc:fc + k]
            cnt[qr:qr + k, qc:qc + k] += 1
    acc = acc[p:p + h, p:p + w]
    cnt = cnt[p:p + h, p:p + w]
    return acc / (255.0 * cnt[..., None])


def noise_image(h, w, seed, lo=0, hi=256):
    return np.random.default_rng(seed).integers(lo, hi, size=(h, w, 3)).astype(np.uint8)
