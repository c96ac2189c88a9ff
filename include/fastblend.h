/*
 * fastblend.h -- C ABI of the FastBlend hot path on AMD MI355X (gfx950).
 *
 * FastBlend (Duan et al., arXiv 2311.09265) removes flicker from a stylised
 * video by estimating nearest-neighbour fields (NNFs) between guide frames
 * with PatchMatch (Section 3.2, Algorithm 1), remapping style frames through
 * them (Section 3.3, Algorithm 2) and averaging the remapped frames over a
 * sliding window (Section 3.4, Eq. 2), or combining two remapped keyframes
 * (Section 3.5, Eq. 9).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Images are uint8 RGB, row-major, HWC, contiguous: [h][w][3] (a video is
 *   [n][h][w][3]).  All pixel, field and output pointers are DEVICE pointers
 *   owned by the caller; the library never frees or retains them after the
 *   call's work has run.  Host pointers are marked (host).
 * - An NNF is int32 [h][w][2]: F(r, c) = (row, col) of the source patch
 *   centre matched to target pixel (r, c) (the paper's F(x, y) = (x', y'),
 *   read as row, column).  Energies are uint32 [h][w]: the integer patch
 *   loss of Eq. 1 for each match.
 * - Source and target of one NNF have the same h x w (Section 3.2).
 * - Pyramid level l has size ceil(h / 2^l) x ceil(w / 2^l).
 * - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL = the
 *   null stream) and the call returns without waiting, except where noted.
 * - Every call validates its arguments on the host first and returns
 *   FB_E_INVALID / FB_E_SHAPE / FB_E_UNSUPPORTED without enqueueing anything.
 *   A HIP runtime error returns FB_E_HIP.  After a non-OK status the outputs
 *   are undefined.  fb_last_error() gives a message for the calling thread.
 * - Results are bit-identical for any batch composition, launch shape or
 *   graph replay: the random draws of a pixel depend only on (seed, pair id,
 *   level, iteration, pixel), never on where the pair sits in a batch.
 * - One fb_ctx may be used by one host thread at a time.  A context keeps a
 *   workspace (pyramids, fields, launch tables) that grows on demand; its
 *   calls run on the device in call order whatever their streams (a call on
 *   another stream than the previous one waits on the device for it).  Launch
 *   tables go to the device with stream-ordered copies from a ring of eight
 *   slots; the host waits only when a slot is reused while the work that
 *   last read it is still running, or when the workspace grows.
 */
#ifndef FASTBLEND_H
#define FASTBLEND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FB_OK = 0,
    FB_E_INVALID = -1,     /* null pointer, non-positive size, bad level, ... */
    FB_E_SHAPE = -2,       /* sizes that do not fit together                  */
    FB_E_UNSUPPORTED = -3, /* valid but not implemented (e.g. patch radius)   */
    FB_E_ALLOC = -4,       /* device or host allocation failed                */
    FB_E_HIP = -5          /* HIP runtime error (launch, copy, graph, ...)    */
} fb_status;

/* Flags of fb_params.flags */
#define FB_USE_GRAPH   0x1u  /* replay the batched launch sequence as a HIP graph */
#define FB_NO_AUTOTUNE 0x2u  /* use the default tile shape, skip the autotuner    */
#define FB_LEARNED_SEED 0x4u /* seed the coarsest level with the proposal network */
/* With FB_LEARNED_SEED, a seeded pair of a plain (Eq. 1) pass is raced, at
 * its coarsest level, against the plain random start (see fb_guard_read);
 * FB_NO_GUARD takes every seed as it is. */
#define FB_NO_GUARD 0x100u
/* FB_USE_GRAPH: when capturing the launch sequence fails (begin, end or
 * instantiation of the capture), the call runs the same launches eagerly and
 * returns FB_OK; fb_graph_fallbacks counts such calls.  FB_DEBUG_FAIL_CAPTURE
 * makes the instantiation report failure, to exercise that path. */
#define FB_DEBUG_FAIL_CAPTURE 0x80000000u
/* Guide + style loss, Eq. 3 (Section 3.4): alpha ||G_j[u] - G_i[v]||^2 +
 * ||S_j[u] - S^_i[v]||^2, where S^_i is the source style S_j remapped (Alg. 2)
 * through the current field, refreshed at the start of every iteration (the
 * incumbent is re-scored under it).  S^_i is kept as a uint8 image (each
 * channel's average rounded half up); alpha = alpha16 / 16 and the energies
 * are the loss scaled by 16, alpha16 SSD(G) + 16 SSD(S, S^), exact in
 * uint32.  Needs iters >= 1 and 0 <= alpha16 <= fb_alpha16_max(p): a patch
 * SSD is at most 3 * 255^2 * (2p+1)^2, and (alpha16 + 16) times that must
 * stay below 2^32 (alpha16 <= 512 for p = 1, 2; 433 for p = 3; 255 for
 * p = 4); larger values return FB_E_INVALID.  Taken by
 * fb_blend_window (the styles are the sources' S_j) and fb_patchmatch_batch
 * (each descriptor's src_style_pyr); the per-level calls and
 * fb_interpolate return FB_E_UNSUPPORTED with it. */
#define FB_STYLE_LOSS 0x8u
/* Fast mode of the window blend (Section 3.4, Alg. 3-5, Eq. 4-6): instead of
 * the 2M NNFs of every frame, a remapping table of O(N log N) NNFs, its
 * column prefix sums (the blending table) and a mirrored twin; each frame's
 * window is then a forward and a mirrored interval query, O(log M) further
 * remaps of table entries (Eq. 4-5 approximations), minus the frame itself
 * (Eq. 6).  Taken by fb_blend_window only; not with FB_STYLE_LOSS or
 * FB_ACCURATE_BLEND. */
#define FB_FAST_BLEND 0x10u
/* Accurate mode of the window blend (Section 3.4, Eq. 7-8): the window's
 * styles remapped with the Eq. 1 NNFs are averaged into T^-_i for every
 * target frame (kept as uint8, the exact average rounded half up); every
 * NNF is estimated again under alpha ||G_j[u] - G_i[v]||^2 + ||S_j[u] -
 * T^-_i[v]||^2 (alpha = alpha16 / 16, loss x 16 as for FB_STYLE_LOSS); the
 * output is the window mean of the styles remapped with the new NNFs.
 * Needs iters >= 1 and 0 <= alpha16 <= fb_alpha16_max(p).  Taken by
 * fb_blend_window only; not with FB_STYLE_LOSS or FB_FAST_BLEND. */
#define FB_ACCURATE_BLEND 0x20u
/* Interpolation extras (Section 3.5), taken by fb_interpolate only.  All
 * NNF(G_k, G_i) of the call are estimated together, level by level and
 * iteration by iteration, each reading the previous iteration's fields.
 * FB_TRACKING: NNF(G_k, G_i) also tries the matches of NNF(G_k, G_{i-1}) and
 * NNF(G_k, G_{i+1}) at the same pixel (when those pairs exist), after the
 * propagation candidates.  FB_ALIGN: the two keyframe fields F_l, F_r of a
 * frame between keys minimise the pairwise alignment loss of Eq. 10,
 * alpha ||G_a[u] - G_i[v]||^2 + ||S_a[u] - S_b[F_b(v)]||^2 (a, b the two keys,
 * S the keyframe styles, F_b the partner's previous field), re-scoring the
 * incumbent every iteration; energies are the loss x 16, alpha = alpha16 / 16,
 * 1 <= alpha16 <= fb_alpha16_max(p), iters >= 1; frames with one key keep
 * Eq. 1. */
#define FB_TRACKING 0x40u
#define FB_ALIGN 0x80u

/* PatchMatch parameters (Algorithm 1).  The paper names p, n and the pyramid
 * but gives no values; 2 / 3 / 6 are the values of the 512x512 blending
 * workload. */
typedef struct {
    int32_t patch_radius;  /* p: patches are (2p+1) x (2p+1) x 3; 1 <= p <= 4  */
    int32_t levels;        /* pyramid levels K >= 1                            */
    int32_t iters;         /* iterations n per level, >= 0                     */
    uint32_t flags;        /* FB_USE_GRAPH | FB_NO_AUTOTUNE | FB_LEARNED_SEED | FB_STYLE_LOSS */
    uint64_t seed;         /* key of the Philox4x32-10 draws                   */
    int32_t alpha16;       /* FB_STYLE_LOSS: guide weight alpha = alpha16 / 16 */
    int32_t plain_iters;   /* FB_LEARNED_SEED: iterations per level of the     */
                           /* plain run a rejected seed falls back to; 0       */
                           /* selects 6; 0 <= plain_iters <= 65534             */
} fb_params;

typedef struct fb_ctx fb_ctx;

/* Create a context on HIP device `device`: it owns the workspace, the
 * per-shape launch plans, captured graphs and autotuning results.
 * Returns FB_E_HIP if the device cannot be used. */
fb_status fb_create(int32_t device, fb_ctx **out);
/* Wait for the context's outstanding work and release it.  NULL is a no-op. */
void fb_destroy(fb_ctx *ctx);
/* Message of the last non-OK status on this thread ("" if none). */
const char *fb_last_error(void);
/* Largest alpha16 the scaled losses of FB_STYLE_LOSS (Eq. 3),
 * FB_ACCURATE_BLEND (Eq. 8) and FB_ALIGN (Eq. 10) accept for patch radius p:
 * min(512, floor((2^32 - 1) / (3 * 255^2 * (2p+1)^2)) - 16), so that every
 * loss value fits its uint32 energy.  0 for p outside [1, 4]. */
int32_t fb_alpha16_max(int32_t patch_radius);

/* Tile shapes of the PatchMatch kernels.  By default the first batched call
 * of every batch shape times each shape on the finest-level iteration and
 * later calls use the fastest (the first call waits for the stream while it
 * measures).  fb_set_tile_config(ctx, i) forces shape i in
 * [0, fb_num_tile_configs()) for all later calls; -1 restores autotuning.
 * Results never depend on the tile shape. */
int32_t fb_num_tile_configs(void);
fb_status fb_set_tile_config(fb_ctx *ctx, int32_t index);
/* Autotuning results can be kept across processes.  fb_tuning_export
 * writes the context's tuned shapes as text, one "batch shape key=index"
 * line each (the key names the patch radius and the run of pair sizes of a
 * batch), NUL-terminated into buf (host) when cap exceeds the text's length,
 * and returns that length (-1 for a NULL context).  fb_tuning_import adds the
 * lines of such a text to the context (FB_E_INVALID for a malformed line or
 * an index outside [0, fb_num_tile_configs())); a batch shape it holds is not
 * timed again.  The indices are only meaningful for the same library build
 * and device.  fb_autotune_runs counts the batch shapes the context has timed. */
int64_t fb_tuning_export(fb_ctx *ctx, char *buf, int64_t cap);
fb_status fb_tuning_import(fb_ctx *ctx, const char *text);
int64_t fb_autotune_runs(fb_ctx *ctx);

/* ---------------------------------------------------------------------- */
/* Image pyramid (Algorithm 1, "resize images S, T" for each level).       */
/* 2x2 box filter with round-half-up, ceil sizes, clamped reads.  The      */
/* pyramid is an opaque device buffer of fb_pyramid_bytes(h,w,levels,p)    */
/* bytes allocated by the caller; it holds every level as 4-byte pixels   */
/* with a border of p replicated pixels (p = patch radius), each followed  */
/* by a table of per-block ranges of the (2p+1)^2 patch sums (at most     */
/* 4 KiB) and a plane of every position's quantised patch sums (4 bytes  */
/* per pixel), which let PatchMatch rule candidates out before reading    */
/* them.                                                                  */
/* ---------------------------------------------------------------------- */
size_t fb_pyramid_bytes(int32_t h, int32_t w, int32_t levels, int32_t patch_radius);
fb_status fb_build_pyramid(fb_ctx *ctx, const uint8_t *rgb, int32_t h, int32_t w,
                           int32_t levels, int32_t patch_radius, void *pyr, void *stream);

/* Frames with their own row stride.  Every call that takes a frame as a
 * contiguous uint8 [h][w][3] (or a video as [N][h][w][3]) has a variant for
 * frames whose rows are not packed -- crops of larger images, rows padded for
 * alignment, frames scattered in memory: row r of a frame starts at
 * rgb + r * row_stride_bytes (device pointer), and row_stride_bytes >= 3 w
 * (else FB_E_INVALID).  Results equal those of the contiguous calls on the
 * same pixels. */
typedef struct {
    const uint8_t *rgb;
    int64_t row_stride_bytes;
} fb_frame;
fb_status fb_build_pyramid_strided(fb_ctx *ctx, const uint8_t *rgb, int32_t h, int32_t w, int64_t row_stride_bytes,
                                   int32_t levels, int32_t patch_radius, void *pyr, void *stream);

/* ---------------------------------------------------------------------- */
/* (1) NNF initialisation at pyramid level `level` (Algorithm 1, "randomly  */
/* initialize F"; "initialize error matrix E").  src_pyr / tgt_pyr come     */
/* from fb_build_pyramid with the same (h, w, levels >= level + 1, p).      */
/* seed_offsets == NULL: every F(r,c) is a uniform Philox draw keyed by     */
/* (params->seed, pair_id, level).  Otherwise seed_offsets is an int32      */
/* [h_l][w_l][2] offset field and F(v) = clamp(v + offset(v)).              */
/* Writes nnf int32 [h_l][w_l][2] and energy uint32 [h_l][w_l].             */
/* ---------------------------------------------------------------------- */
fb_status fb_nnf_init(fb_ctx *ctx, const void *src_pyr, const void *tgt_pyr, int32_t h, int32_t w,
                      int32_t level, const fb_params *params, uint32_t pair_id,
                      const int32_t *seed_offsets, int32_t *nnf, uint32_t *energy, void *stream);

/* ---------------------------------------------------------------------- */
/* (2) One pyramid level of PatchMatch (Algorithm 1 body; Section 3.2).     */
/* If nnf_coarse != NULL it is the level+1 field (int32 [h_{l+1}][w_{l+1}]  */
/* [2]); it is upsampled (F = clamp(2 F_c + parity)) and re-energised.      */
/* Otherwise nnf / energy are read as the starting field (e.g. from         */
/* fb_nnf_init): field entries are clamped into the level, energies are    */
/* taken as given (any uint32; a pixel moves only to a candidate whose     */
/* loss is strictly lower).  Then params->iters concurrent iterations     */
/* run: each pixel tries propagation F(v+d)-d for d = (-1,0),(1,0),(0,-1), */
/* (0,1), then                                                              */
/* random search around its running best at radii max(h_l,w_l) >> m, and   */
/* keeps a candidate only if its loss is strictly lower.  Writes nnf and    */
/* energy (int32 [h_l][w_l][2], uint32 [h_l][w_l]) in place.               */
/* ---------------------------------------------------------------------- */
fb_status fb_patchmatch_level(fb_ctx *ctx, const void *src_pyr, const void *tgt_pyr, int32_t h,
                              int32_t w, int32_t level, const fb_params *params, uint32_t pair_id,
                              const int32_t *nnf_coarse, int32_t *nnf, uint32_t *energy,
                              void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * call as fb_patchmatch_level, with the same arguments and bit-identical
 * results, that allocates nothing.  Its working memory (the level's four
 * ping-pong field and energy planes and the launch descriptors, 16 MiB +
 * 1 KiB) is one fixed device array of the library per GPU, set up by
 * fb_create and held until the process ends.  The level must have at most
 * 1,048,576 pixels (h_l * w_l); larger levels return FB_E_UNSUPPORTED.  Every
 * call on one GPU, from any context or stream, uses that GPU's array and
 * leaves its contents behind: calls that overlap on one GPU race, so the
 * caller serialises them.  It always uses the default tile shape (or the
 * one fb_set_tile_config forces). */
fb_status fb_patchmatch_level_noalloc(fb_ctx *ctx, const void *src_pyr, const void *tgt_pyr, int32_t h,
                                      int32_t w, int32_t level, const fb_params *params, uint32_t pair_id,
                                      const int32_t *nnf_coarse, int32_t *nnf, uint32_t *energy,
                                      void *stream);

/* ---------------------------------------------------------------------- */
/* (3) Memory-efficient remapping (Algorithm 2): out(v) = average over      */
/* d in [-p,p]^2 with v+d inside the image of style(F(v+d) - d) / 255,     */
/* source reads clamped.  style uint8 [h][w][3], nnf int32 [h][w][2] (every */
/* entry must lie in [0,h) x [0,w)), out fp32 [h][w][3] in [0, 1].          */
/* ---------------------------------------------------------------------- */
fb_status fb_remap(fb_ctx *ctx, const uint8_t *style, const int32_t *nnf, int32_t h, int32_t w,
                   int32_t patch_radius, float *out, void *stream);
/* The same with the style frame's own row stride (see fb_frame above):     */
/* row r of the style starts at style + r * row_stride_bytes, which must be */
/* at least 3 w (else FB_E_INVALID).                                        */
fb_status fb_remap_strided(fb_ctx *ctx, const uint8_t *style, int64_t row_stride_bytes, const int32_t *nnf,
                           int32_t h, int32_t w, int32_t patch_radius, float *out, void *stream);

/* ---------------------------------------------------------------------- */
/* (4) Sliding-window blending, Eq. 2 (balanced mode, guide loss Eq. 1):    */
/* out_i = mean over j in [max(0,i-M), min(N-1,i+M)] of (S_j -> S_i), where */
/* S_j -> S_i remaps style j with NNF(G_j, G_i) estimated over `levels`     */
/* levels (pair id j*N + i), and the j == i term is S_i / 255.              */
/* guides, styles uint8 [N][h][w][3]; out fp32 [N][h][w][3].  Every pair of */
/* the window runs batched, level by level.                               */
/* ---------------------------------------------------------------------- */
fb_status fb_blend_window(fb_ctx *ctx, const uint8_t *guides, const uint8_t *styles, int32_t n_frames,
                          int32_t h, int32_t w, int32_t radius_M, const fb_params *params,
                          float *out, void *stream);
/* the same with guides and styles as host arrays of n_frames fb_frame */
fb_status fb_blend_window_frames(fb_ctx *ctx, const fb_frame *guides, const fb_frame *styles, int32_t n_frames,
                                 int32_t h, int32_t w, int32_t radius_M, const fb_params *params, float *out,
                                 void *stream);

/* ---------------------------------------------------------------------- */
/* (5) Keyframe interpolation, Eq. 9: keyframes pass through (style / 255); */
/* a frame i between keys l < i < r gets (r-i)/(r-l) (S_l -> S_i) +         */
/* (i-l)/(r-l) (S_r -> S_i); frames before the first or after the last key  */
/* get the single nearest key's remap.  key_idx (host) is sorted, unique,   */
/* in [0, N); key_styles uint8 [n_keys][h][w][3]; out fp32 [N][h][w][3].    */
/* ---------------------------------------------------------------------- */
fb_status fb_interpolate(fb_ctx *ctx, const uint8_t *guides, int32_t n_frames, int32_t h, int32_t w,
                         const int32_t *key_idx, const uint8_t *key_styles, int32_t n_keys,
                         const fb_params *params, float *out, void *stream);
/* the same with guides (n_frames) and key styles (n_keys) as host arrays of fb_frame */
fb_status fb_interpolate_frames(fb_ctx *ctx, const fb_frame *guides, int32_t n_frames, int32_t h, int32_t w,
                                const int32_t *key_idx, const fb_frame *key_styles, int32_t n_keys,
                                const fb_params *params, float *out, void *stream);

/* ---------------------------------------------------------------------- */
/* Batched PatchMatch (Section 3.2, "we store images in batches"): the      */
/* whole pyramid of every pair, pairs of any size mixed, in grouped         */
/* launches (one per level step and iteration, optionally replayed as a    */
/* HIP graph).  Results equal n_pairs separate single-pair runs.            */
/* ---------------------------------------------------------------------- */
typedef struct {
    const void *src_pyr;          /* fb_build_pyramid output, >= levels levels   */
    const void *tgt_pyr;
    int32_t h, w, levels;         /* level-0 size; pyramid levels of this pair   */
    uint32_t pair_id;
    const int32_t *seed_offsets;  /* optional int32 offsets at level levels-1   */
    int32_t *nnf;                 /* out: int32 [h][w][2] level-0 field          */
    uint32_t *energy;             /* out: uint32 [h][w]                          */
    const void *src_style_pyr;    /* FB_STYLE_LOSS: fb_build_pyramid of the      */
                                  /* source's style frame S_j (same h, w, p,     */
                                  /* >= levels levels); else ignored             */
} fb_pair_desc;

/* pairs (host) holds n_pairs descriptors; params->levels is ignored (each
 * pair has its own), the other fields apply to all pairs. */
fb_status fb_patchmatch_batch(fb_ctx *ctx, const fb_pair_desc *pairs, int32_t n_pairs,
                              const fb_params *params, void *stream);

/* ---------------------------------------------------------------------- */
/* Kernel timing (measurement support).  While profiling is on, every      */
/* launch is bracketed by HIP events recorded on the call's stream and the */
/* calls run their launches eagerly (no graph replay).  fb_profile_read    */
/* waits for the recorded events and returns, per kernel kind, the number  */
/* of launches and the summed event-to-event time since profiling began    */
/* (or since the last read with reset != 0).                               */
/* ---------------------------------------------------------------------- */
enum {
    FB_KERNEL_PYRAMID = 0,   /* pack + downsample + norm of a batch of frames */
    FB_KERNEL_PM_START = 1,  /* init / upsample + energy                      */
    FB_KERNEL_PM_ITER = 2,   /* one PatchMatch iteration over a batch         */
    FB_KERNEL_PM_EXPORT = 3, /* packed field -> int32 NNF + energies          */
    FB_KERNEL_REMAP = 4,     /* remap-sum (Alg. 2 + Eq. 2 / Eq. 9)            */
    FB_KERNEL_OTHER = 5,
    FB_KERNEL_UNET = 6,      /* proposal network forward for a group of pairs */
    FB_KERNEL_STYLE = 7,     /* FB_STYLE_LOSS: refresh of the remapped styles  */
    FB_KERNEL_KINDS = 8
};
typedef struct {
    int64_t launches[FB_KERNEL_KINDS];
    double milliseconds[FB_KERNEL_KINDS];
} fb_profile;

int64_t fb_graph_fallbacks(fb_ctx *ctx);
/* Measurement (no part of the method): the gather rate of patch rows that
 * bounds the PatchMatch iteration.  2048 x 256 lanes each fetch rows_per_lane
 * 5-pixel rows (one 16-byte and one 4-byte load, p = 2 only) from level 0 of
 * the pyramid pyr (from fb_build_pyramid with this h, w, p), with every lane
 * at its own random position (divergent != 0, like random-search candidates)
 * or the 64 lanes of a wave at consecutive pixels (like propagation
 * candidates), and fold each row into a v_dot4 sum.  Times one launch after
 * a warm-up with HIP events on `stream` and waits for it; *rows_per_s
 * (host) receives lane-rows per second. */
fb_status fb_gather_probe(fb_ctx *ctx, const void *pyr, int32_t h, int32_t w, int32_t patch_radius, int32_t divergent,
                          int32_t rows_per_lane, double *rows_per_s, void *stream);
fb_status fb_profile_enable(fb_ctx *ctx, int32_t on);
fb_status fb_profile_read(fb_ctx *ctx, fb_profile *out, int32_t reset);

/* ---------------------------------------------------------------------- */
/* Learned proposal (a project addition; the paper's method is model-free, */
/* Section 3.1).  A 4-level U-Net with (32, 48, 96, 192) channels maps a   */
/* frame pair at the coarsest pyramid level (6 channels: source RGB,       */
/* target RGB, in [0, 1], centred to 2x - 1 inside the network) to a       */
/* 2-channel offset field (row, col, in pixels of that level).  bf16       */
/* weights and activations, fp32 accumulation on the                       */
/* matrix cores.  With FB_LEARNED_SEED in fb_params.flags, the blend,      */
/* interpolation and batch calls seed every pair's coarsest level with the */
/* rounded prediction (F = clamp(v + offset)) instead of the random draw;  */
/* the plain random initialisation stays the default and the fallback.     */
/*                                                                         */
/* Parameters are a flat fp32 vector of fb_unet_param_count() values: for */
/* each of the 15 convolutions in order, its weight [cout][cin][3][3] then */
/* its bias [cout].  Tensors below are device pointers, NHWC:              */
/*   pair6 float [B][h][w][6]; offsets / target float [B][h][w][2];        */
/*   mask float [B][h][w] (per-pixel loss weight); h, w multiples of 8.    */
/* Training minimises sum(mask * |pred - target|_1) / max(sum(mask), 1)    */
/* with Adam (beta 0.9 / 0.999, eps 1e-8); `loss` receives the value       */
/* before the update.  Loading parameters resets the Adam state.           */
/* ---------------------------------------------------------------------- */
int64_t fb_unet_param_count(void);
double fb_unet_forward_flops(int32_t B, int32_t h, int32_t w);
fb_status fb_unet_load(fb_ctx *ctx, const float *params, void *stream);
fb_status fb_unet_save(fb_ctx *ctx, float *params, void *stream);
/* Training state, for checkpoint and resume: the parameters and Adam's first
 * and second moments (each fb_unet_param_count() floats, the flat layout of
 * fb_unet_load; device pointers) and Adam's step count (*step, host).
 * fb_unet_save_state writes them (the step at once, the tensors stream-
 * ordered); fb_unet_load_state sets them, so that later training steps equal
 * those of the run that saved them. */
fb_status fb_unet_save_state(fb_ctx *ctx, float *params, float *adam_m, float *adam_v, int64_t *step,
                             void *stream);
fb_status fb_unet_load_state(fb_ctx *ctx, const float *params, const float *adam_m, const float *adam_v,
                             int64_t step, void *stream);
fb_status fb_unet_forward(fb_ctx *ctx, const float *pair6, int32_t B, int32_t h, int32_t w,
                          float *offsets, void *stream);
fb_status fb_unet_gradients(fb_ctx *ctx, const float *pair6, const float *target, const float *mask,
                            int32_t B, int32_t h, int32_t w, float *grads, float *loss, void *stream);
fb_status fb_unet_train_step(fb_ctx *ctx, const float *pair6, const float *target, const float *mask,
                             int32_t B, int32_t h, int32_t w, float lr, float *loss, void *stream);
/* Guard of a seeded run.  With FB_LEARNED_SEED (and not FB_NO_GUARD), every
 * pair of a plain (Eq. 1) pass that starts from offsets -- predicted by the
 * network or given in its descriptor -- is raced at its coarsest level: the
 * seeded start with params->iters iterations against the random start of
 * Alg. 1 with one iteration more, min(iters + 1, plain_iters): a seed must
 * be worth at least an iteration.  If the seeded level's summed energy is
 * the larger, the seed is rejected and the pair's result is the plain run
 * exactly (random start, plain_iters iterations at every level); otherwise
 * the seeded run's.  The launch sequence does not depend on the
 * outcome (graph replay is unaffected).  Passes under FB_STYLE_LOSS,
 * FB_TRACKING or FB_ALIGN, and the Eq. 8 pass of FB_ACCURATE_BLEND, take
 * seeds unguarded.
 * fb_guard_read waits for `stream` and returns, for the pairs of the last
 * fb_blend_window / fb_interpolate / fb_patchmatch_batch call in the order
 * that call planned them (the batch: descriptor order; the blend: target
 * frame i ascending, then source j ascending; interpolation: frame, then
 * left before right key), sums[2k] = the seeded and sums[2k+1] = the plain
 * summed coarsest-level energy of pair k (both 0 for an unguarded pair), for
 * at most max_pairs pairs (host array of 2 * max_pairs); *n_pairs receives
 * the call's pair count.  Pair k's seed was rejected iff
 * sums[2k] > sums[2k+1]. */
fb_status fb_guard_read(fb_ctx *ctx, uint64_t *sums, int32_t max_pairs, int32_t *n_pairs, void *stream);

/* The network input of one pair exactly as FB_LEARNED_SEED builds it: the
 * coarsest level (levels - 1) of both pyramids, padded to multiples of 8 by
 * repeating the last row / column, pair6 float [H8][W8][6] = pixels / 255. */
fb_status fb_unet_pair_input(fb_ctx *ctx, const void *src_pyr, const void *tgt_pyr, int32_t h, int32_t w,
                             int32_t levels, int32_t patch_radius, float *pair6, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FASTBLEND_H */
