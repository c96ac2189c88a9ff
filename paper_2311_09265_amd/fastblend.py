"""Thin Python binding of the FastBlend C ABI (``include/fastblend.h``).

Only argument marshalling happens here: tensors are checked (device, dtype,
shape, contiguity) and their device pointers, together with the current HIP
stream of PyTorch, are handed to ``libfastblend.so``.  Every step of the hot
path runs in the library's HIP kernels.  If the library is not built, every
call raises; there is no fallback.

The function names are the C names (``fb_nnf_init`` ...), taking tensors.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastblend.so")

FB_OK = 0
FB_USE_GRAPH = 0x1
FB_NO_AUTOTUNE = 0x2
FB_LEARNED_SEED = 0x4
FB_STYLE_LOSS = 0x8
FB_FAST_BLEND = 0x10
FB_ACCURATE_BLEND = 0x20
FB_TRACKING = 0x40
FB_ALIGN = 0x80
FB_NO_GUARD = 0x100
FB_DEBUG_FAIL_CAPTURE = 0x80000000
STATUS = {0: "FB_OK", -1: "FB_E_INVALID", -2: "FB_E_SHAPE", -3: "FB_E_UNSUPPORTED",
          -4: "FB_E_ALLOC", -5: "FB_E_HIP"}


class FastBlendError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s: %s (%s)" % (where, STATUS.get(status, status), msg))
        self.status = status


class fb_params(ctypes.Structure):
    _fields_ = [("patch_radius", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("flags", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("alpha16", ctypes.c_int32), ("plain_iters", ctypes.c_int32)]


class fb_pair_desc(ctypes.Structure):
    _fields_ = [("src_pyr", ctypes.c_void_p), ("tgt_pyr", ctypes.c_void_p),
                ("h", ctypes.c_int32), ("w", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("pair_id", ctypes.c_uint32), ("seed_offsets", ctypes.c_void_p),
                ("nnf", ctypes.c_void_p), ("energy", ctypes.c_void_p),
                ("src_style_pyr", ctypes.c_void_p)]


class fb_frame(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("row_stride_bytes", ctypes.c_int64)]


KERNEL_KINDS = ["pyramid", "pm_start", "pm_iter", "pm_export", "remap", "other", "unet", "style"]


class fb_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 8), ("milliseconds", ctypes.c_double * 8)]


_lib = None
_EXPORTS = ["fb_create", "fb_destroy", "fb_last_error", "fb_alpha16_max", "fb_num_tile_configs",
            "fb_set_tile_config",
            "fb_pyramid_bytes", "fb_build_pyramid", "fb_nnf_init", "fb_patchmatch_level", "fb_remap",
            "fb_blend_window", "fb_interpolate", "fb_patchmatch_batch", "fb_profile_enable",
            "fb_profile_read", "fb_unet_param_count", "fb_unet_forward_flops", "fb_unet_load", "fb_unet_save",
            "fb_unet_forward", "fb_unet_gradients", "fb_unet_train_step", "fb_unet_pair_input", "fb_guard_read", "fb_unet_save_state", "fb_unet_load_state",
            "fb_tuning_export", "fb_tuning_import", "fb_autotune_runs", "fb_graph_fallbacks",
            "fb_build_pyramid_strided", "fb_blend_window_frames", "fb_interpolate_frames", "fb_remap_strided",
            "fb_gather_probe",
            "fb_patchmatch_level_noalloc"]


def load_library(path: str = LIB_PATH):
    """Load ``libfastblend.so`` and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libfastblend.so is not built (%s); run python -m paper_2311_09265_amd.build" % path)
    L = ctypes.CDLL(path)
    vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    P = ctypes.POINTER(fb_params)
    sig = {
        "fb_create": (i32, [i32, ctypes.POINTER(vp)]),
        "fb_destroy": (None, [vp]),
        "fb_last_error": (ctypes.c_char_p, []),
        "fb_alpha16_max": (i32, [i32]),
        "fb_num_tile_configs": (i32, []),
        "fb_set_tile_config": (i32, [vp, i32]),
        "fb_pyramid_bytes": (sz, [i32, i32, i32, i32]),
        "fb_build_pyramid": (i32, [vp, vp, i32, i32, i32, i32, vp, vp]),
        "fb_nnf_init": (i32, [vp, vp, vp, i32, i32, i32, P, u32, vp, vp, vp, vp]),
        "fb_patchmatch_level": (i32, [vp, vp, vp, i32, i32, i32, P, u32, vp, vp, vp, vp]),
        "fb_patchmatch_level_noalloc": (i32, [vp, vp, vp, i32, i32, i32, P, u32, vp, vp, vp, vp]),
        "fb_remap": (i32, [vp, vp, vp, i32, i32, i32, vp, vp]),
        "fb_blend_window": (i32, [vp, vp, vp, i32, i32, i32, i32, P, vp, vp]),
        "fb_interpolate": (i32, [vp, vp, i32, i32, i32, vp, vp, i32, P, vp, vp]),
        "fb_patchmatch_batch": (i32, [vp, ctypes.POINTER(fb_pair_desc), i32, P, vp]),
        "fb_profile_enable": (i32, [vp, i32]),
        "fb_profile_read": (i32, [vp, ctypes.POINTER(fb_profile), i32]),
        "fb_unet_param_count": (ctypes.c_int64, []),
        "fb_unet_forward_flops": (ctypes.c_double, [i32, i32, i32]),
        "fb_unet_load": (i32, [vp, vp, vp]),
        "fb_unet_save": (i32, [vp, vp, vp]),
        "fb_unet_forward": (i32, [vp, vp, i32, i32, i32, vp, vp]),
        "fb_unet_gradients": (i32, [vp, vp, vp, vp, i32, i32, i32, vp, vp, vp]),
        "fb_unet_train_step": (i32, [vp, vp, vp, vp, i32, i32, i32, ctypes.c_float, vp, vp]),
        "fb_unet_pair_input": (i32, [vp, vp, vp, i32, i32, i32, i32, vp, vp]),
        "fb_guard_read": (i32, [vp, ctypes.POINTER(ctypes.c_uint64), i32, ctypes.POINTER(i32), vp]),
        "fb_unet_save_state": (i32, [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64), vp]),
        "fb_tuning_export": (ctypes.c_int64, [vp, ctypes.c_char_p, ctypes.c_int64]),
        "fb_build_pyramid_strided": (i32, [vp, vp, i32, i32, ctypes.c_int64, i32, i32, vp, vp]),
        "fb_remap_strided": (i32, [vp, vp, ctypes.c_int64, vp, i32, i32, i32, vp, vp]),
        "fb_gather_probe": (i32, [vp, vp, i32, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_double), vp]),
        "fb_blend_window_frames": (i32, [vp, ctypes.POINTER(fb_frame), ctypes.POINTER(fb_frame), i32, i32, i32, i32,
                                         P, vp, vp]),
        "fb_interpolate_frames": (i32, [vp, ctypes.POINTER(fb_frame), i32, i32, i32, vp, ctypes.POINTER(fb_frame), i32,
                                        P, vp, vp]),
        "fb_tuning_import": (i32, [vp, ctypes.c_char_p]),
        "fb_autotune_runs": (ctypes.c_int64, [vp]),
        "fb_graph_fallbacks": (ctypes.c_int64, [vp]),
        "fb_unet_load_state": (i32, [vp, vp, vp, vp, ctypes.c_int64, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int, where: str):
    if status != FB_OK:
        msg = load_library().fb_last_error()
        raise FastBlendError(status, where, msg.decode() if msg else "")


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev(t: Optional[torch.Tensor], name: str, dtype=None, shape=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _as_frames(t: torch.Tensor, name: str, n: int, h: int, w: int):
    """fb_frame array of a uint8 [n][h][w][3] GPU tensor whose pixels are
    packed (strides 3, 1) and whose rows and frames may have any stride."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.uint8:
        raise TypeError("%s must be a uint8 GPU tensor" % name)
    if tuple(t.shape) != (n, h, w, 3):
        raise ValueError("%s must have shape %s, got %s" % (name, (n, h, w, 3), tuple(t.shape)))
    sf, sr, sc, sch = t.stride()
    if sc != 3 or sch != 1 or sr < 3 * w:
        raise ValueError("%s: pixels must be packed RGB (strides (.., .., 3, 1)) with rows of at least 3 w bytes" % name)
    base = t.data_ptr()
    arr = (fb_frame * n)()
    for k in range(n):
        arr[k] = fb_frame(base + k * sf, sr)
    return arr


def _frames(t: torch.Tensor, name: str, n: int, h: int, w: int):
    """None for a contiguous uint8 [n][h][w][3] GPU tensor, else its fb_frame array."""
    arr = _as_frames(t, name, n, h, w)
    return None if t.is_contiguous() else arr


def _check_pyr(pyr: torch.Tensor, name: str, h: int, w: int, levels: int, patch_radius: int):
    need = load_library().fb_pyramid_bytes(h, w, levels, patch_radius)
    if need == 0 or pyr.numel() < need:
        raise ValueError("%s holds %d bytes, a %d-level pyramid of %dx%d needs %d"
                         % (name, pyr.numel(), levels, h, w, need))


def make_params(patch_radius: int = 2, levels: int = 3, iters: int = 6, seed: int = 0,
                flags: int = 0, alpha16: int = 16, plain_iters: int = 0) -> fb_params:
    """alpha16: the guide weight of the Eq. 3 loss (FB_STYLE_LOSS), alpha = alpha16 / 16.
    plain_iters: with FB_LEARNED_SEED, the iterations per level of the plain run
    a seed is raced against and falls back to (0: 6)."""
    return fb_params(patch_radius, levels, iters, flags, seed & 0xFFFFFFFFFFFFFFFF, alpha16, plain_iters)


def energy_u32(energy: torch.Tensor) -> torch.Tensor:
    """The uint32 energies of the C ABI as int64 values.  The binding returns
    energy tensors as int32 (torch's unsigned 32-bit type lacks most ops); a
    value of 2^31 or more reads negative there, so compare or average this
    view instead."""
    return energy.to(torch.int64) & 0xFFFFFFFF


def level_size(h: int, w: int, level: int):
    return -(-h // (1 << level)), -(-w // (1 << level))


class Context:
    """An ``fb_ctx`` on one device (workspace, plans, graphs, autotuning)."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _check(load_library().fb_create(device, ctypes.byref(h)), "fb_create")
        self.handle = h

    def close(self):
        if self.handle:
            load_library().fb_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- learned proposal network -----------------------------------------
    def fb_unet_load(self, params: torch.Tensor):
        n = load_library().fb_unet_param_count()
        _check(load_library().fb_unet_load(self.handle, _dev(params, "params", torch.float32, (n,)),
                                           _stream(params)), "fb_unet_load")

    def fb_unet_save_state(self):
        """(params, adam_m, adam_v) as fp32 GPU tensors and the Adam step count."""
        n = load_library().fb_unet_param_count()
        out = [torch.empty(n, dtype=torch.float32, device=self.device) for _ in range(3)]
        step = ctypes.c_int64(0)
        _check(load_library().fb_unet_save_state(self.handle, *[_dev(t, "state") for t in out], ctypes.byref(step),
                                                 _stream(out[0])), "fb_unet_save_state")
        return out[0], out[1], out[2], int(step.value)

    def fb_unet_load_state(self, params: torch.Tensor, adam_m: torch.Tensor, adam_v: torch.Tensor, step: int):
        n = load_library().fb_unet_param_count()
        _check(load_library().fb_unet_load_state(
            self.handle, _dev(params, "params", torch.float32, (n,)), _dev(adam_m, "adam_m", torch.float32, (n,)),
            _dev(adam_v, "adam_v", torch.float32, (n,)), int(step), _stream(params)), "fb_unet_load_state")

    def fb_unet_save(self) -> torch.Tensor:
        n = load_library().fb_unet_param_count()
        out = torch.empty(n, dtype=torch.float32, device=self.device)
        _check(load_library().fb_unet_save(self.handle, _dev(out, "params"), _stream(out)), "fb_unet_save")
        return out

    def fb_unet_forward(self, pair6: torch.Tensor) -> torch.Tensor:
        B, h, w = pair6.shape[:3]
        out = torch.empty((B, h, w, 2), dtype=torch.float32, device=pair6.device)
        _check(load_library().fb_unet_forward(self.handle, _dev(pair6, "pair6", torch.float32, (B, h, w, 6)),
                                              B, h, w, _dev(out, "offsets"), _stream(pair6)), "fb_unet_forward")
        return out

    def fb_unet_gradients(self, pair6, target, mask):
        """(flat fp32 gradients, loss) of the masked L1 loss, parameters unchanged."""
        B, h, w = pair6.shape[:3]
        n = load_library().fb_unet_param_count()
        grads = torch.empty(n, dtype=torch.float32, device=pair6.device)
        loss = torch.empty(1, dtype=torch.float32, device=pair6.device)
        _check(load_library().fb_unet_gradients(
            self.handle, _dev(pair6, "pair6", torch.float32, (B, h, w, 6)),
            _dev(target, "target", torch.float32, (B, h, w, 2)), _dev(mask, "mask", torch.float32, (B, h, w)),
            B, h, w, _dev(grads, "grads"), _dev(loss, "loss"), _stream(pair6)), "fb_unet_gradients")
        return grads, loss

    def fb_unet_pair_input(self, src_pyr, tgt_pyr, h: int, w: int, levels: int, patch_radius: int = 2,
                           out: Optional[torch.Tensor] = None) -> torch.Tensor:
        hc, wc = level_size(h, w, levels - 1)
        H8, W8 = -(-hc // 8) * 8, -(-wc // 8) * 8
        _check_pyr(src_pyr, "src_pyr", h, w, levels, patch_radius)
        _check_pyr(tgt_pyr, "tgt_pyr", h, w, levels, patch_radius)
        if out is None:
            out = torch.empty((H8, W8, 6), dtype=torch.float32, device=src_pyr.device)
        _check(load_library().fb_unet_pair_input(
            self.handle, _dev(src_pyr, "src_pyr", torch.uint8), _dev(tgt_pyr, "tgt_pyr", torch.uint8), h, w,
            levels, patch_radius, _dev(out, "pair6", torch.float32, (H8, W8, 6)), _stream(src_pyr)),
            "fb_unet_pair_input")
        return out

    def fb_unet_train_step(self, pair6, target, mask, lr: float) -> torch.Tensor:
        """One Adam step; returns the loss before the update (device scalar)."""
        B, h, w = pair6.shape[:3]
        loss = torch.empty(1, dtype=torch.float32, device=pair6.device)
        _check(load_library().fb_unet_train_step(
            self.handle, _dev(pair6, "pair6", torch.float32, (B, h, w, 6)),
            _dev(target, "target", torch.float32, (B, h, w, 2)), _dev(mask, "mask", torch.float32, (B, h, w)),
            B, h, w, lr, _dev(loss, "loss"), _stream(pair6)), "fb_unet_train_step")
        return loss

    # ---- measurement ----------------------------------------------------
    def fb_profile_enable(self, on: bool = True):
        _check(load_library().fb_profile_enable(self.handle, 1 if on else 0), "fb_profile_enable")

    def fb_profile_read(self, reset: bool = False) -> dict:
        """{kernel kind: (launches, summed milliseconds)} from the HIP events."""
        pr = fb_profile()
        _check(load_library().fb_profile_read(self.handle, ctypes.byref(pr), 1 if reset else 0),
               "fb_profile_read")
        return {k: (int(pr.launches[i]), float(pr.milliseconds[i])) for i, k in enumerate(KERNEL_KINDS)}

    def fb_gather_probe(self, pyr: torch.Tensor, h: int, w: int, divergent: bool, rows_per_lane: int = 256) -> float:
        """Lane-rows per second of 5-pixel row gathers from level 0 of pyr (a
        measurement of the rate that bounds the PatchMatch iteration)."""
        _check_pyr(pyr, "pyr", h, w, 1, 2)
        r = ctypes.c_double(0.0)
        _check(load_library().fb_gather_probe(self.handle, _dev(pyr, "pyr", torch.uint8), h, w, 2, int(divergent),
                                              rows_per_lane, ctypes.byref(r), _stream(pyr)), "fb_gather_probe")
        return r.value

    def fb_guard_read(self, stream_device: int = 0):
        """(seeded, plain) summed coarsest-level energies of every pair of the
        last blend / interpolation / batch call, as an int64 tensor [n][2]
        (zeros for unguarded pairs); pair k's seed was rejected iff
        [k, 0] > [k, 1].  Waits for the current stream."""
        L = load_library()
        n = ctypes.c_int32(0)
        dummy = (ctypes.c_uint64 * 2)()
        stream = ctypes.c_void_p(torch.cuda.current_stream(stream_device).cuda_stream)
        _check(L.fb_guard_read(self.handle, dummy, 0, ctypes.byref(n), stream), "fb_guard_read")
        buf = (ctypes.c_uint64 * max(2 * n.value, 2))()
        _check(L.fb_guard_read(self.handle, buf, n.value, ctypes.byref(n), stream), "fb_guard_read")
        return torch.tensor([int(x) for x in buf[:2 * n.value]], dtype=torch.int64).reshape(n.value, 2)

    # ---- tuning ---------------------------------------------------------
    def tuning_export(self) -> str:
        L = load_library()
        n = L.fb_tuning_export(self.handle, None, 0)
        buf = ctypes.create_string_buffer(n + 1)
        L.fb_tuning_export(self.handle, buf, n + 1)
        return buf.value.decode()

    def tuning_import(self, text: str):
        _check(load_library().fb_tuning_import(self.handle, text.encode()), "fb_tuning_import")

    def tuning_save(self, path: str):
        """The tuned tile shapes as JSON, keyed by batch shape, with the device
        and the library's tile-shape count they hold for."""
        import json
        L = load_library()
        entries = dict(line.rsplit("=", 1) for line in self.tuning_export().splitlines() if line)
        doc = {"format": 1, "device": torch.cuda.get_device_properties(self.device).gcnArchName,
               "tile_configs": int(L.fb_num_tile_configs()), "entries": {k: int(v) for k, v in entries.items()}}
        with open(path, "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)

    def tuning_load(self, path: str) -> bool:
        """Load a file written by tuning_save; False (nothing loaded) if it was
        written for another device or library."""
        import json
        with open(path) as f:
            doc = json.load(f)
        if (doc.get("format") != 1 or doc.get("device") != torch.cuda.get_device_properties(self.device).gcnArchName
                or doc.get("tile_configs") != load_library().fb_num_tile_configs()):
            return False
        self.tuning_import("".join("%s=%d\n" % (k, v) for k, v in doc["entries"].items()))
        return True

    def fb_autotune_runs(self) -> int:
        return int(load_library().fb_autotune_runs(self.handle))

    def fb_graph_fallbacks(self) -> int:
        return int(load_library().fb_graph_fallbacks(self.handle))

    def fb_set_tile_config(self, index: int):
        _check(load_library().fb_set_tile_config(self.handle, index), "fb_set_tile_config")

    # ---- pyramid --------------------------------------------------------
    def fb_build_pyramid(self, rgb: torch.Tensor, levels: int, patch_radius: int = 2) -> torch.Tensor:
        """rgb: uint8 [h][w][3] on the GPU, contiguous or with a row stride."""
        h, w = rgb.shape[:2]
        fr = _frames(rgb.unsqueeze(0), "rgb", 1, h, w)
        nbytes = load_library().fb_pyramid_bytes(h, w, levels, patch_radius)
        if nbytes == 0:
            raise ValueError("invalid pyramid parameters")
        pyr = torch.empty(nbytes, dtype=torch.uint8, device=rgb.device)
        if fr is None:
            _check(load_library().fb_build_pyramid(self.handle, _dev(rgb, "rgb"), h, w, levels, patch_radius,
                                                   _dev(pyr, "pyr"), _stream(rgb)), "fb_build_pyramid")
        else:
            _check(load_library().fb_build_pyramid_strided(self.handle, ctypes.c_void_p(fr[0].rgb), h, w,
                                                           fr[0].row_stride_bytes, levels, patch_radius,
                                                           _dev(pyr, "pyr"), _stream(rgb)), "fb_build_pyramid_strided")
        return pyr

    # ---- per-pair PatchMatch ------------------------------------------------
    def fb_nnf_init(self, src_pyr, tgt_pyr, h: int, w: int, level: int, params: fb_params,
                    pair_id: int, seed_offsets: Optional[torch.Tensor] = None):
        hl, wl = level_size(h, w, level)
        _check_pyr(src_pyr, "src_pyr", h, w, level + 1, params.patch_radius)
        _check_pyr(tgt_pyr, "tgt_pyr", h, w, level + 1, params.patch_radius)
        nnf = torch.empty((hl, wl, 2), dtype=torch.int32, device=src_pyr.device)
        energy = torch.empty((hl, wl), dtype=torch.int32, device=src_pyr.device)
        _check(load_library().fb_nnf_init(
            self.handle, _dev(src_pyr, "src_pyr", torch.uint8), _dev(tgt_pyr, "tgt_pyr", torch.uint8),
            h, w, level, ctypes.byref(params), pair_id,
            _dev(seed_offsets, "seed_offsets", torch.int32, (hl, wl, 2)),
            _dev(nnf, "nnf"), _dev(energy, "energy"), _stream(src_pyr)), "fb_nnf_init")
        return nnf, energy

    def fb_patchmatch_level(self, src_pyr, tgt_pyr, h: int, w: int, level: int, params: fb_params,
                            pair_id: int, nnf: Optional[torch.Tensor] = None,
                            energy: Optional[torch.Tensor] = None,
                            nnf_coarse: Optional[torch.Tensor] = None):
        """Returns (nnf, energy) at ``level``; nnf/energy (int32) are updated in place if given.
        Energies are uint32 values stored in int32 tensors (see ``energy_u32``)."""
        hl, wl = level_size(h, w, level)
        _check_pyr(src_pyr, "src_pyr", h, w, level + 1, params.patch_radius)
        _check_pyr(tgt_pyr, "tgt_pyr", h, w, level + 1, params.patch_radius)
        if nnf is None:
            nnf = torch.empty((hl, wl, 2), dtype=torch.int32, device=src_pyr.device)
            energy = torch.empty((hl, wl), dtype=torch.int32, device=src_pyr.device)
        if nnf_coarse is None and energy is None:
            raise ValueError("need nnf_coarse, or a starting nnf and energy")
        hc, wc = level_size(h, w, level + 1)
        _check(load_library().fb_patchmatch_level(
            self.handle, _dev(src_pyr, "src_pyr", torch.uint8), _dev(tgt_pyr, "tgt_pyr", torch.uint8),
            h, w, level, ctypes.byref(params), pair_id,
            _dev(nnf_coarse, "nnf_coarse", torch.int32, (hc, wc, 2)),
            _dev(nnf, "nnf", torch.int32, (hl, wl, 2)), _dev(energy, "energy", torch.int32, (hl, wl)),
            _stream(src_pyr)), "fb_patchmatch_level")
        return nnf, energy

    def fb_patchmatch_level_noalloc(self, src_pyr, tgt_pyr, h: int, w: int, level: int, params: fb_params,
                                    pair_id: int, nnf: torch.Tensor, energy: torch.Tensor,
                                    nnf_coarse: Optional[torch.Tensor] = None):
        """fb_patchmatch_level without any allocation: the caller passes nnf and
        energy (int32 [h_l][w_l][2] and [h_l][w_l]), updated in place."""
        hl, wl = level_size(h, w, level)
        hc, wc = level_size(h, w, level + 1)
        _check(load_library().fb_patchmatch_level_noalloc(
            self.handle, _dev(src_pyr, "src_pyr", torch.uint8), _dev(tgt_pyr, "tgt_pyr", torch.uint8),
            h, w, level, ctypes.byref(params), pair_id,
            _dev(nnf_coarse, "nnf_coarse", torch.int32, (hc, wc, 2)),
            _dev(nnf, "nnf", torch.int32, (hl, wl, 2)), _dev(energy, "energy", torch.int32, (hl, wl)),
            _stream(src_pyr)), "fb_patchmatch_level_noalloc")
        return nnf, energy

    # ---- remap / blend / interpolate --------------------------------------
    def fb_remap(self, style: torch.Tensor, nnf: torch.Tensor, patch_radius: int = 2) -> torch.Tensor:
        """style: uint8 [h][w][3] on the GPU, contiguous or with a row stride."""
        h, w = style.shape[:2]
        out = torch.empty((h, w, 3), dtype=torch.float32, device=style.device)
        fr = _frames(style.unsqueeze(0), "style", 1, h, w)
        if fr is None:
            _check(load_library().fb_remap(self.handle, _dev(style, "style", torch.uint8, (h, w, 3)),
                                           _dev(nnf, "nnf", torch.int32, (h, w, 2)), h, w, patch_radius,
                                           _dev(out, "out"), _stream(style)), "fb_remap")
        else:
            _check(load_library().fb_remap_strided(self.handle, ctypes.c_void_p(fr[0].rgb), fr[0].row_stride_bytes,
                                                   _dev(nnf, "nnf", torch.int32, (h, w, 2)), h, w, patch_radius,
                                                   _dev(out, "out"), _stream(style)), "fb_remap_strided")
        return out

    def fb_blend_window(self, guides: torch.Tensor, styles: torch.Tensor, radius_M: int,
                        params: fb_params, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """guides, styles: uint8 [N][h][w][3] on the GPU, contiguous or views
        with packed pixels and any row / frame strides (then the fb_frame call)."""
        n, h, w = guides.shape[:3]
        if out is None:
            out = torch.empty((n, h, w, 3), dtype=torch.float32, device=guides.device)
        fg, fs = _frames(guides, "guides", n, h, w), _frames(styles, "styles", n, h, w)
        if fg is None and fs is None:
            _check(load_library().fb_blend_window(
                self.handle, _dev(guides, "guides", torch.uint8, (n, h, w, 3)),
                _dev(styles, "styles", torch.uint8, (n, h, w, 3)), n, h, w, radius_M, ctypes.byref(params),
                _dev(out, "out", torch.float32, (n, h, w, 3)), _stream(guides)), "fb_blend_window")
        else:
            fg = _as_frames(guides, "guides", n, h, w)
            fs = _as_frames(styles, "styles", n, h, w)
            _check(load_library().fb_blend_window_frames(
                self.handle, fg, fs, n, h, w, radius_M, ctypes.byref(params),
                _dev(out, "out", torch.float32, (n, h, w, 3)), _stream(guides)), "fb_blend_window_frames")
        return out

    def fb_interpolate(self, guides: torch.Tensor, key_idx: Sequence[int], key_styles: torch.Tensor,
                       params: fb_params, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        n, h, w = guides.shape[:3]
        nk = len(key_idx)
        keys = (ctypes.c_int32 * nk)(*[int(k) for k in key_idx])
        if out is None:
            out = torch.empty((n, h, w, 3), dtype=torch.float32, device=guides.device)
        fg, fk = _frames(guides, "guides", n, h, w), _frames(key_styles, "key_styles", nk, h, w)
        if fg is None and fk is None:
            _check(load_library().fb_interpolate(
                self.handle, _dev(guides, "guides", torch.uint8, (n, h, w, 3)), n, h, w,
                ctypes.cast(keys, ctypes.c_void_p),
                _dev(key_styles, "key_styles", torch.uint8, (nk, h, w, 3)), nk,
                ctypes.byref(params), _dev(out, "out", torch.float32, (n, h, w, 3)), _stream(guides)),
                "fb_interpolate")
        else:
            fg = _as_frames(guides, "guides", n, h, w)
            fk = _as_frames(key_styles, "key_styles", nk, h, w)
            _check(load_library().fb_interpolate_frames(
                self.handle, fg, n, h, w, ctypes.cast(keys, ctypes.c_void_p), fk, nk, ctypes.byref(params),
                _dev(out, "out", torch.float32, (n, h, w, 3)), _stream(guides)), "fb_interpolate_frames")
        return out

    def fb_patchmatch_batch(self, pairs: Sequence[dict], params: fb_params):
        """pairs: dicts with src_pyr, tgt_pyr, h, w, levels, pair_id[, seed_offsets]
        [, src_style_pyr (FB_STYLE_LOSS)].
        Returns a list of (nnf int32 [h][w][2], energy int32 [h][w]); the energies
        are uint32 values stored in int32 tensors (see ``energy_u32``)."""
        descs = (fb_pair_desc * len(pairs))()
        outs, keep = [], []
        for k, d in enumerate(pairs):
            h, w = d["h"], d["w"]
            dev = d["src_pyr"].device
            _check_pyr(d["src_pyr"], "src_pyr", h, w, d["levels"], params.patch_radius)
            _check_pyr(d["tgt_pyr"], "tgt_pyr", h, w, d["levels"], params.patch_radius)
            nnf = torch.empty((h, w, 2), dtype=torch.int32, device=dev)
            energy = torch.empty((h, w), dtype=torch.int32, device=dev)
            so = d.get("seed_offsets")
            ss = d.get("src_style_pyr")
            if ss is not None:
                _check_pyr(ss, "src_style_pyr", h, w, d["levels"], params.patch_radius)
            hc, wc = level_size(h, w, d["levels"] - 1)
            descs[k] = fb_pair_desc(_dev(d["src_pyr"], "src_pyr", torch.uint8),
                                    _dev(d["tgt_pyr"], "tgt_pyr", torch.uint8), h, w, d["levels"],
                                    d["pair_id"], _dev(so, "seed_offsets", torch.int32, (hc, wc, 2)),
                                    _dev(nnf, "nnf"), _dev(energy, "energy"),
                                    _dev(ss, "src_style_pyr", torch.uint8))
            outs.append((nnf, energy))
            keep.append(so)
        _check(load_library().fb_patchmatch_batch(self.handle, descs, len(pairs), ctypes.byref(params),
                                                   _stream(pairs[0]["src_pyr"])), "fb_patchmatch_batch")
        return outs
