"""CPU oracle for the FastBlend hot path -- TEST INFRASTRUCTURE ONLY.

Plain C (``fb_oracle.c``, compiled with gcc) driven through ctypes.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package; the product library never does, and the two share no
code.  Each wrapper names the passage of the paper (arXiv 2311.09265) that the
C function follows; the C file states every reading taken where the paper is
silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``fb_oracle.c`` into ``liboracle.so`` next to it (gcc, -O3, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c99", "-O3", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        I, U32, U64 = ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64
        L.fbo_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.fbo_philox4x32_10.restype = None
        L.fbo_uniform16.argtypes = [U32, U32]
        L.fbo_uniform16.restype = U32
        L.fbo_downsample.argtypes = [u8p, I, I, u8p]
        L.fbo_downsample.restype = None
        L.fbo_patch_ssd.argtypes = [u8p, u8p, I, I, I, I, I, I, I]
        L.fbo_patch_ssd.restype = U32
        L.fbo_energy.argtypes = [u8p, u8p, I, I, I, i32p, u32p]
        L.fbo_energy.restype = None
        L.fbo_nnf_init_random.argtypes = [u8p, u8p, I, I, I, I, U64, U32, i32p, u32p]
        L.fbo_nnf_init_random.restype = None
        L.fbo_nnf_init_offsets.argtypes = [u8p, u8p, I, I, I, i32p, i32p, u32p]
        L.fbo_nnf_init_offsets.restype = None
        L.fbo_nnf_upsample.argtypes = [i32p, I, I, u8p, u8p, I, I, I, i32p, u32p]
        L.fbo_nnf_upsample.restype = None
        L.fbo_pm_iteration.argtypes = [u8p, u8p, I, I, I, I, I, U64, U32, i32p, u32p, i32p, u32p]
        L.fbo_pm_iteration.restype = None
        L.fbo_patchmatch.argtypes = [u8p, u8p, I, I, I, I, I, U64, U32, ctypes.c_void_p, i32p, u32p]
        L.fbo_patchmatch.restype = I
        L.fbo_patchmatch_raced.argtypes = [u8p, u8p, I, I, I, I, I, I, U64, U32, ctypes.c_void_p, i32p, u32p,
                                           ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int)]
        L.fbo_patchmatch_raced.restype = I
        L.fbo_remap.argtypes = [u8p, i32p, I, I, I, f64p]
        L.fbo_remap.restype = None
        L.fbo_blend_window.argtypes = [u8p, u8p, I, I, I, I, I, I, I, U64, f64p]
        L.fbo_blend_window.restype = I
        L.fbo_interpolate.argtypes = [u8p, I, I, I, i32p, u8p, I, I, I, I, U64, f64p]
        L.fbo_interpolate.restype = I
        L.fbo_remap_u8.argtypes = [u8p, i32p, I, I, I, u8p]
        L.fbo_remap_u8.restype = None
        L.fbo_style_loss.argtypes = [u8p, u8p, u8p, u8p, I, I, I, I, I, I, I, I]
        L.fbo_style_loss.restype = U64
        L.fbo_alpha16_max.argtypes = [I]
        L.fbo_alpha16_max.restype = I
        L.fbo_pm_iteration_style.argtypes = [u8p, u8p, u8p, I, I, I, I, I, I, U64, U32, i32p, i32p, u32p, u8p]
        L.fbo_pm_iteration_style.restype = None
        L.fbo_patchmatch_style.argtypes = [u8p, u8p, u8p, I, I, I, I, I, U64, U32, I, i32p, u32p,
                                           ctypes.c_void_p]
        L.fbo_patchmatch_style.restype = I
        L.fbo_blend_window_style.argtypes = [u8p, u8p, I, I, I, I, I, I, I, U64, I, f64p]
        L.fbo_blend_window_style.restype = I
        L.fbo_remap_f64.argtypes = [f64p, i32p, I, I, I, f64p]
        L.fbo_remap_f64.restype = None
        L.fbo_blend_window_fast.argtypes = [u8p, u8p, I, I, I, I, I, I, I, U64, I, f64p]
        L.fbo_blend_window_fast.restype = I
        L.fbo_window_mean_u8.argtypes = [u8p, I, ctypes.c_void_p, ctypes.c_void_p, I, I, I, I, u8p]
        L.fbo_window_mean_u8.restype = None
        L.fbo_pm_iteration_target.argtypes = [u8p, u8p, u8p, u8p, I, I, I, I, I, I, U64, U32, i32p, i32p, u32p]
        L.fbo_pm_iteration_target.restype = None
        L.fbo_patchmatch_target.argtypes = [u8p, u8p, u8p, u8p, I, I, I, I, I, U64, U32, I, i32p, u32p]
        L.fbo_patchmatch_target.restype = I
        L.fbo_blend_window_accurate.argtypes = [u8p, u8p, I, I, I, I, I, I, I, U64, I, f64p, ctypes.c_void_p]
        L.fbo_blend_window_accurate.restype = I
        L.fbo_pm_iteration_ext.argtypes = [u8p, u8p, u8p, u8p, I, I, I, I, I, I, I, U64, U32, ctypes.c_void_p,
                                           ctypes.c_void_p, I, I, I, I, i32p, u32p]
        L.fbo_pm_iteration_ext.restype = None
        L.fbo_interpolate_ext.argtypes = [u8p, I, I, I, i32p, u8p, I, I, I, I, U64, I, I, f64p]
        L.fbo_interpolate_ext.restype = I
        L.fbo_set_threads.argtypes = [I]
        L.fbo_set_threads.restype = None
        L.fbo_get_threads.argtypes = []
        L.fbo_get_threads.restype = I
        _lib = L
    return _lib


def _img(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint8)
    assert a.ndim == 3 and a.shape[2] == 3, a.shape
    return a


def set_threads(n: int) -> None:
    lib().fbo_set_threads(int(n))


def get_threads() -> int:
    return int(lib().fbo_get_threads())


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    out = np.zeros(4, np.uint32)
    lib().fbo_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def uniform16(u16: int, n: int) -> int:
    return int(lib().fbo_uniform16(int(u16), int(n)))


def downsample(img) -> np.ndarray:
    """One pyramid step (Alg. 1, "resize images")."""
    img = _img(img)
    h, w = img.shape[:2]
    out = np.zeros(((h + 1) // 2, (w + 1) // 2, 3), np.uint8)
    lib().fbo_downsample(img, h, w, out)
    return out


def pyramid(img, levels: int):
    out = [_img(img)]
    for _ in range(1, levels):
        out.append(downsample(out[-1]))
    return out


def patch_ssd(S, T, p: int, u, v) -> int:
    """Eq. (1) for one match: ||S[u] - T[v]||^2 over (2p+1)^2 x 3 patches."""
    S, T = _img(S), _img(T)
    h, w = S.shape[:2]
    return int(lib().fbo_patch_ssd(S, T, h, w, p, int(u[0]), int(u[1]), int(v[0]), int(v[1])))


def energy(S, T, F, p: int) -> np.ndarray:
    S, T = _img(S), _img(T)
    h, w = S.shape[:2]
    E = np.zeros((h, w), np.uint32)
    lib().fbo_energy(S, T, h, w, p, np.ascontiguousarray(F, np.int32), E)
    return E


def nnf_init_random(S, T, p: int, level: int, seed: int, pair_id: int):
    """Random initialisation of F at a level (Alg. 1), with its energy."""
    S, T = _img(S), _img(T)
    h, w = S.shape[:2]
    F = np.zeros((h, w, 2), np.int32)
    E = np.zeros((h, w), np.uint32)
    lib().fbo_nnf_init_random(S, T, h, w, p, level, seed, pair_id, F, E)
    return F, E


def nnf_init_offsets(S, T, p: int, offsets):
    S, T = _img(S), _img(T)
    h, w = S.shape[:2]
    F = np.zeros((h, w, 2), np.int32)
    E = np.zeros((h, w), np.uint32)
    lib().fbo_nnf_init_offsets(S, T, h, w, p, np.ascontiguousarray(offsets, np.int32), F, E)
    return F, E


def nnf_upsample(Fc, S, T, p: int):
    """Upsample a coarse NNF onto the finer level of S, T (Alg. 1), with energy."""
    S, T = _img(S), _img(T)
    h, w = S.shape[:2]
    Fc = np.ascontiguousarray(Fc, np.int32)
    F = np.zeros((h, w, 2), np.int32)
    E = np.zeros((h, w), np.uint32)
    lib().fbo_nnf_upsample(Fc, Fc.shape[0], Fc.shape[1], S, T, h, w, p, F, E)
    return F, E


def pm_iteration(S, T, p: int, level: int, it: int, seed: int, pair_id: int, F, E):
    """One concurrent PatchMatch iteration (Alg. 1 inner loop, Section 3.2)."""
    S, T = _img(S), _img(T)
    h, w = S.shape[:2]
    Fn = np.zeros((h, w, 2), np.int32)
    En = np.zeros((h, w), np.uint32)
    lib().fbo_pm_iteration(S, T, h, w, p, level, it, seed, pair_id,
                           np.ascontiguousarray(F, np.int32), np.ascontiguousarray(E, np.uint32), Fn, En)
    return Fn, En


def patchmatch(S, T, p: int, levels: int, iters: int, seed: int, pair_id: int,
               seed_offsets: Optional[np.ndarray] = None):
    """NNF(S, T) by the coarse-to-fine Alg. 1; returns level-0 F (int32 [h][w][2]) and E."""
    S, T = _img(S), _img(T)
    h, w = S.shape[:2]
    F = np.zeros((h, w, 2), np.int32)
    E = np.zeros((h, w), np.uint32)
    off = None
    if seed_offsets is not None:
        off = np.ascontiguousarray(seed_offsets, np.int32)
        ptr = off.ctypes.data_as(ctypes.c_void_p)
    else:
        ptr = None
    st = lib().fbo_patchmatch(S, T, h, w, p, levels, iters, seed, pair_id, ptr, F, E)
    if st != 0:
        raise RuntimeError("fbo_patchmatch failed: %d" % st)
    del off
    return F, E


def patchmatch_raced(S, T, p: int, levels: int, iters: int, plain_iters: int, seed: int, pair_id: int,
                     seed_offsets):
    """Seeded NNF(S, T) under the guard of a seeded run: at the coarsest level
    the seeded start with `iters` iterations races the random start with
    min(iters + 1, plain_iters) iterations; if the seeded level's summed
    energy is the larger, the whole result is the plain run (plain_iters
    iterations per level), else the seeded run.  Returns (F, E, rejected,
    (seeded sum, plain sum))."""
    S, T = _img(S), _img(T)
    h, w = S.shape[:2]
    F = np.zeros((h, w, 2), np.int32)
    E = np.zeros((h, w), np.uint32)
    off = np.ascontiguousarray(seed_offsets, np.int32)
    sums = (ctypes.c_uint64 * 2)()
    rej = ctypes.c_int(0)
    st = lib().fbo_patchmatch_raced(S, T, h, w, p, levels, iters, plain_iters, seed, pair_id,
                                    off.ctypes.data_as(ctypes.c_void_p), F, E, sums, ctypes.byref(rej))
    if st != 0:
        raise RuntimeError("fbo_patchmatch_raced failed: %d" % st)
    return F, E, bool(rej.value), (int(sums[0]), int(sums[1]))


def remap(style, F, p: int) -> np.ndarray:
    """Alg. 2 over the whole image, fp64 [h][w][3] in [0, 1]."""
    style = _img(style)
    h, w = style.shape[:2]
    out = np.zeros((h, w, 3), np.float64)
    lib().fbo_remap(style, np.ascontiguousarray(F, np.int32), h, w, p, out)
    return out


def blend_window(guides, styles, M: int, p: int, levels: int, iters: int, seed: int) -> np.ndarray:
    """Eq. (2) over a whole video, fp64 [N][h][w][3]."""
    guides = np.ascontiguousarray(guides, np.uint8)
    styles = np.ascontiguousarray(styles, np.uint8)
    N, h, w = guides.shape[:3]
    out = np.zeros((N, h, w, 3), np.float64)
    st = lib().fbo_blend_window(guides, styles, N, h, w, M, p, levels, iters, seed, out)
    if st != 0:
        raise RuntimeError("fbo_blend_window failed: %d" % st)
    return out


def remap_u8(style, F, p: int) -> np.ndarray:
    """S^ of Eq. (3): the Alg. 2 remap of `style` through F as a uint8 image
    (each channel's average rounded half up)."""
    style = _img(style)
    h, w = style.shape[:2]
    out = np.zeros((h, w, 3), np.uint8)
    lib().fbo_remap_u8(style, np.ascontiguousarray(F, np.int32), h, w, p, out)
    return out


def alpha16_max(p: int) -> int:
    """Largest alpha16 whose scaled Eq. 3 / 8 / 10 losses fit the uint32
    energies, min(512, floor((2^32 - 1) / (3 * 255^2 * (2p+1)^2)) - 16)."""
    return int(lib().fbo_alpha16_max(int(p)))


def _check_alpha16(p: int, alpha16: int) -> None:
    if not 0 <= alpha16 <= alpha16_max(p):
        raise ValueError("alpha16 must be in [0, %d] for p = %d" % (alpha16_max(p), p))


def style_loss(Gs, Gt, Ss, Sh, p: int, alpha16: int, u, v) -> int:
    """Eq. (3) for one match, scaled by 16: alpha16 SSD(G) + 16 SSD(S, S^),
    exact (64-bit) for any alpha16."""
    Gs, Gt, Ss, Sh = _img(Gs), _img(Gt), _img(Ss), _img(Sh)
    h, w = Gs.shape[:2]
    return int(lib().fbo_style_loss(Gs, Gt, Ss, Sh, h, w, p, alpha16, int(u[0]), int(u[1]), int(v[0]), int(v[1])))


def pm_iteration_style(Gs, Gt, Ss, p: int, alpha16: int, level: int, it: int, seed: int, pair_id: int, F):
    """One iteration under the Eq. (3) loss; returns (F, E, S^ of its refresh)."""
    _check_alpha16(p, alpha16)
    Gs, Gt, Ss = _img(Gs), _img(Gt), _img(Ss)
    h, w = Gs.shape[:2]
    Fn = np.zeros((h, w, 2), np.int32)
    En = np.zeros((h, w), np.uint32)
    Sh = np.zeros((h, w, 3), np.uint8)
    lib().fbo_pm_iteration_style(Gs, Gt, Ss, h, w, p, alpha16, level, it, seed, pair_id,
                                 np.ascontiguousarray(F, np.int32), Fn, En, Sh)
    return Fn, En, Sh


def patchmatch_style(Gs, Gt, Ss, p: int, levels: int, iters: int, seed: int, pair_id: int, alpha16: int):
    """NNF(G_j, G_i) under the Eq. (3) loss; returns level-0 F, E and the last S^."""
    Gs, Gt, Ss = _img(Gs), _img(Gt), _img(Ss)
    h, w = Gs.shape[:2]
    F = np.zeros((h, w, 2), np.int32)
    E = np.zeros((h, w), np.uint32)
    Sh = np.zeros((h, w, 3), np.uint8)
    st = lib().fbo_patchmatch_style(Gs, Gt, Ss, h, w, p, levels, iters, seed, pair_id, alpha16, F, E,
                                    Sh.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise RuntimeError("fbo_patchmatch_style failed: %d" % st)
    return F, E, Sh


def blend_window_style(guides, styles, M: int, p: int, levels: int, iters: int, seed: int,
                       alpha16: int) -> np.ndarray:
    """Eq. (2) with every NNF under the Eq. (3) loss, fp64 [N][h][w][3]."""
    guides = np.ascontiguousarray(guides, np.uint8)
    styles = np.ascontiguousarray(styles, np.uint8)
    N, h, w = guides.shape[:3]
    out = np.zeros((N, h, w, 3), np.float64)
    st = lib().fbo_blend_window_style(guides, styles, N, h, w, M, p, levels, iters, seed, alpha16, out)
    if st != 0:
        raise RuntimeError("fbo_blend_window_style failed: %d" % st)
    return out


def remap_f64(X, F, p: int) -> np.ndarray:
    """Alg. 2 on a floating-point image X [h][w][3] (fast mode, Eq. 4-5)."""
    X = np.ascontiguousarray(X, np.float64)
    h, w = X.shape[:2]
    out = np.zeros((h, w, 3), np.float64)
    lib().fbo_remap_f64(X, np.ascontiguousarray(F, np.int32), h, w, p, out)
    return out


def blend_window_fast(guides, styles, M: int, p: int, levels: int, iters: int, seed: int,
                      identity_nnf: bool = False) -> np.ndarray:
    """Fast mode (Alg. 3-5 with Eq. 6) over a whole video, fp64 [N][h][w][3].
    identity_nnf replaces every NNF by the identity (a test hook)."""
    guides = np.ascontiguousarray(guides, np.uint8)
    styles = np.ascontiguousarray(styles, np.uint8)
    N, h, w = guides.shape[:3]
    out = np.zeros((N, h, w, 3), np.float64)
    st = lib().fbo_blend_window_fast(guides, styles, N, h, w, M, p, levels, iters, seed, int(identity_nnf), out)
    if st != 0:
        raise RuntimeError("fbo_blend_window_fast failed: %d" % st)
    return out


def window_mean_u8(styles, i: int, js, fields, p: int) -> np.ndarray:
    """T^- of Eq. 7 for target frame i: the exact average of S_i and the
    styles js[k] remapped with fields[k], rounded half up, as uint8."""
    styles = np.ascontiguousarray(styles, np.uint8)
    N, h, w = styles.shape[:3]
    fs = [np.ascontiguousarray(f, np.int32) for f in fields]
    ptrs = (ctypes.c_void_p * max(1, len(fs)))(*[f.ctypes.data for f in fs])
    js_a = np.ascontiguousarray(js, np.int32)
    out = np.zeros((h, w, 3), np.uint8)
    lib().fbo_window_mean_u8(styles, i, js_a.ctypes.data_as(ctypes.c_void_p), ctypes.cast(ptrs, ctypes.c_void_p),
                             len(fs), h, w, p, out)
    return out


def pm_iteration_target(Gs, Gt, Ss, Tb, p: int, alpha16: int, level: int, it: int, seed: int, pair_id: int, F):
    """One iteration under the Eq. 8 loss against a fixed T^- level."""
    _check_alpha16(p, alpha16)
    Gs, Gt, Ss, Tb = _img(Gs), _img(Gt), _img(Ss), _img(Tb)
    h, w = Gs.shape[:2]
    Fn = np.zeros((h, w, 2), np.int32)
    En = np.zeros((h, w), np.uint32)
    lib().fbo_pm_iteration_target(Gs, Gt, Ss, Tb, h, w, p, alpha16, level, it, seed, pair_id,
                                  np.ascontiguousarray(F, np.int32), Fn, En)
    return Fn, En


def patchmatch_target(Gs, Gt, Ss, Tb, p: int, levels: int, iters: int, seed: int, pair_id: int, alpha16: int):
    """NNF(G_j, G_i) under the Eq. 8 loss against T^-; returns level-0 F and E."""
    Gs, Gt, Ss, Tb = _img(Gs), _img(Gt), _img(Ss), _img(Tb)
    h, w = Gs.shape[:2]
    F = np.zeros((h, w, 2), np.int32)
    E = np.zeros((h, w), np.uint32)
    st = lib().fbo_patchmatch_target(Gs, Gt, Ss, Tb, h, w, p, levels, iters, seed, pair_id, alpha16, F, E)
    if st != 0:
        raise RuntimeError("fbo_patchmatch_target failed: %d" % st)
    return F, E


def blend_window_accurate(guides, styles, M: int, p: int, levels: int, iters: int, seed: int, alpha16: int,
                          return_tbar: bool = False):
    """Accurate mode (Eq. 7-8 then Eq. 2), fp64 [N][h][w][3] (and T^- per frame)."""
    guides = np.ascontiguousarray(guides, np.uint8)
    styles = np.ascontiguousarray(styles, np.uint8)
    N, h, w = guides.shape[:3]
    out = np.zeros((N, h, w, 3), np.float64)
    tb = np.zeros((N, h, w, 3), np.uint8)
    st = lib().fbo_blend_window_accurate(guides, styles, N, h, w, M, p, levels, iters, seed, alpha16, out,
                                         tb.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise RuntimeError("fbo_blend_window_accurate failed: %d" % st)
    return (out, tb) if return_tbar else out


TRACK, ALIGN = 1, 2


def pm_iteration_ext(Gs, Gt, Ss, Sp, p: int, alpha16: int, flags: int, level: int, it: int, seed: int,
                     pair_id: int, fields, energies, q: int, prev: int = -1, nxt: int = -1, partner: int = -1):
    """One iteration of pair q of a jointly estimated interpolation (tracking
    and / or alignment, Section 3.5, Eq. 10); fields / energies: the previous
    fields and energies of all pairs.  Returns (F, E)."""
    if flags & ALIGN:
        _check_alpha16(p, alpha16)
    Gs, Gt, Ss, Sp = _img(Gs), _img(Gt), _img(Ss), _img(Sp)
    h, w = Gs.shape[:2]
    fs = [np.ascontiguousarray(f, np.int32) for f in fields]
    es = [np.ascontiguousarray(e, np.uint32) for e in energies]
    fp = (ctypes.c_void_p * len(fs))(*[f.ctypes.data for f in fs])
    ep = (ctypes.c_void_p * len(es))(*[e.ctypes.data for e in es])
    Fn = np.zeros((h, w, 2), np.int32)
    En = np.zeros((h, w), np.uint32)
    lib().fbo_pm_iteration_ext(Gs, Gt, Ss, Sp, h, w, p, alpha16, flags, level, it, seed, pair_id,
                               ctypes.cast(fp, ctypes.c_void_p), ctypes.cast(ep, ctypes.c_void_p), q, prev, nxt,
                               partner, Fn, En)
    return Fn, En


def interpolate_ext(guides, keys, key_styles, p: int, levels: int, iters: int, seed: int, alpha16: int = 16,
                    track: bool = False, align: bool = False) -> np.ndarray:
    """Eq. (9) with the NNFs estimated jointly with tracking and / or the
    pairwise alignment loss (Eq. 10), fp64 [N][h][w][3]."""
    guides = np.ascontiguousarray(guides, np.uint8)
    keys = np.ascontiguousarray(keys, np.int32)
    key_styles = np.ascontiguousarray(key_styles, np.uint8)
    N, h, w = guides.shape[:3]
    out = np.zeros((N, h, w, 3), np.float64)
    flags = (TRACK if track else 0) | (ALIGN if align else 0)
    st = lib().fbo_interpolate_ext(guides, N, h, w, keys, key_styles, len(keys), p, levels, iters, seed, alpha16,
                                   flags, out)
    if st != 0:
        raise RuntimeError("fbo_interpolate_ext failed: %d" % st)
    return out


def interpolate(guides, keys, key_styles, p: int, levels: int, iters: int, seed: int) -> np.ndarray:
    """Eq. (9) over a whole video, fp64 [N][h][w][3]."""
    guides = np.ascontiguousarray(guides, np.uint8)
    keys = np.ascontiguousarray(keys, np.int32)
    key_styles = np.ascontiguousarray(key_styles, np.uint8)
    N, h, w = guides.shape[:3]
    out = np.zeros((N, h, w, 3), np.float64)
    st = lib().fbo_interpolate(guides, N, h, w, keys, key_styles, len(keys), p, levels, iters, seed, out)
    if st != 0:
        raise RuntimeError("fbo_interpolate failed: %d" % st)
    return out
