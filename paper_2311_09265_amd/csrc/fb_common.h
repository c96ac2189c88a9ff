// Internal declarations of the FastBlend HIP library (gfx950).
//
// Data layout in device memory
// ----------------------------
// * Pyramid of one frame (fb_build_pyramid): for every level l, the image as
//   4-byte (R, G, B, 0) pixels with a replicated border of p pixels on every
//   side (so a patch read never needs clamping), row pitch rounded up to 16
//   pixels.  A (2p+1)-pixel patch row is one 16-byte + one 4-byte aligned
//   load for p = 2.
//   Each level is followed by its bound table: for every block of
//   2^tab_shift x 2^tab_shift patch positions, the range [mn_c, mx_c] of
//   each channel's (2p+1)^2 patch sum over the block, as three arrays of
//   16-bit pairs (lower half first): (mn_R, mn_G), (mn_B, -mx_R),
//   (-mx_G, -mx_B), each tab_w * tab_h words.  The block size is the
//   smallest from 8 x 8 up whose table fits kBoundTabBytes, so one table
//   always fits a workgroup's LDS.
//   The table is followed by the level's patch-sum plane: for every patch
//   position (r, c), at word r * pitch + c of h rows, each channel's
//   (2p+1)^2 patch sum shifted right by psum_shift(p) (10 bits each: R in
//   bits 0-9, G in 10-19, B in 20-29), so a candidate's own sums are known
//   to within 2^psum_shift - 1.
// * Style frames: the same format at full resolution (one aligned 4-byte
//   gather per remapped pixel).
// * NNFs inside the library are one uint32 per pixel: (row << 16) | col.
//   The C ABI converts to / from int32 [h][w][2].
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fb {

constexpr int kMaxLevels = 16;
constexpr int kMaxP = 4;
constexpr int kPitchAlign = 16;  // pixels
constexpr int kBoundTabBytes = 4096;   // largest bound table of one level
constexpr int kBoundTabMinShift = 3;   // smallest bound-table block: 8 x 8 positions
// Patch-sum plane: each channel's (2p+1)^2 patch sum (at most (2p+1)^2 * 255)
// shifted right until it fits 10 bits
inline int psum_shift(int p) {
    int s = 0;
    while ((((2 * p + 1) * (2 * p + 1) * 255) >> s) >= 1024) ++s;
    return s;
}

struct LevelGeom {
    int32_t h, w;        // level size
    int32_t pitch;       // padded row pitch in pixels
    int32_t rows;        // padded rows = h + 2p
    size_t px_off;       // byte offset of the level in the pyramid
    size_t tab_off;      // byte offset of the level's bound table
    int32_t tab_shift;   // bound-table block side = 1 << tab_shift positions
    int32_t tab_w, tab_h;  // bound-table size in blocks
    size_t sum_off;      // byte offset of the level's patch-sum plane
};

struct PyrLayout {
    int32_t levels, p;
    LevelGeom lv[kMaxLevels];
    size_t bytes;
};

// Host: layout of a pyramid of `levels` levels for patch radius p.
PyrLayout pyr_layout(int h, int w, int levels, int p);
// Host: layout of a single padded level-0 image (styles); pitch in pixels.
size_t padded_image_bytes(int h, int w, int p, int32_t *pitch_out);

inline int ceil_half_pow(int x, int l) { return (x + (1 << l) - 1) >> l; }

// One unit of PatchMatch work: one pair at one level, for one launch.
enum StartMode : int32_t {
    kStartRandom = 0,     // Philox draw at every pixel
    kStartOffsets = 1,    // F = clamp(v + aux_off[v])          (aux_off int32 [h][w][2])
    kStartUpsample = 2,   // F = clamp(2 f_in[v/2] + parity)    (f_in packed, coarse)
    kStartUpsampleAbi = 3,// as 2, coarse field from aux_off int32 [hc][wc][2]
    kStartCopyAbi = 4     // F = aux_off[v], E = e_abi[v] (given field and energy)
};

struct PMJob {
    const uint32_t *src_px;    // padded pixels of the source level, at padded (0, 0)
    const uint32_t *tgt_px;    // padded pixels of the target level
    const uint32_t *f_in;      // packed field read by the launch
    const uint32_t *e_in;      // energies read by iterations
    uint32_t *f_out;           // packed field written by the launch
    uint32_t *e_out;
    const int32_t *aux_off;    // ABI int32 field / offsets (start modes 1, 3, 4)
    const uint32_t *e_abi;     // ABI energies (start mode 4)
    int32_t *nnf_abi;          // export destinations
    uint32_t *energy_abi;
    const uint32_t *src_sty;   // Eq. 3 / 8 / 10 losses: padded pixels of the source style level
    uint32_t *sty_hat;         // Eq. 3 loss: the remapped style S^ (Eq. 8: T^-), padded like the level
    const uint32_t *trk_prev;  // tracking: packed fields of the pairs with the same source and the
    const uint32_t *trk_next;  //   previous / next target frame (nullptr: none)
    const uint32_t *pair_f;    // Eq. 10: the partner pair's packed field (nullptr: not aligned)
    const uint32_t *pair_sty;  // Eq. 10: padded pixels of the partner's source style level
    int32_t h, w, pitch;       // level size; row pitch in pixels
    int32_t hc, wc;            // coarse size for upsampling
    uint32_t pair_id;
    int32_t level;
    int32_t mode;
    int32_t tile_base;         // first flat tile of this job in the launch
    int32_t tiles_x;           // tiles along w
    int32_t alpha16;           // Eq. 3 loss: guide weight alpha = alpha16 / 16
    int32_t tab_shift;         // bound table of the source level (see the layout above):
    int32_t tab_w, tab_n;      //   block shift, width in blocks, entries (0: no table)
    const uint32_t *btab;
    const uint32_t *psum;      // the source level's patch-sum plane (with btab)
    const uint32_t *f_prev;    // Eq. 3 refresh: the field the level's previous refresh used
                               //   (nullptr: refresh every pixel)
    // Guard of a seeded pair (its coarsest level raced against the plain
    // random start): guard points at the pair's two summed coarsest-level
    // energies (seeded, plain); the seed is rejected when the first is the
    // larger.  Iteration launches: guard_when 1 runs the job only for a
    // rejected seed, 2 only for a kept one, 0 always.  k_energy_sum: guard
    // is the sum the job's energies e_in are added to.  k_guard_select: for
    // a rejected seed, (f_alt, e_alt) is copied over (f_out, e_out).
    // k_guard_decide: a rejected seed sets *guard_any.
    uint64_t *guard;
    uint64_t *guard_any;       // nonzero once any seed of the call was rejected
    const uint32_t *f_alt;
    const uint32_t *e_alt;
    int32_t guard_when;
    // style-loss iterations: e_in already holds the incumbent's loss under
    // this iteration's target (Eq. 8, whose target T^- is fixed, after the
    // level's first iteration), so the incumbent is not scored again
    int32_t e_valid;
    int32_t psum_shift;        // quantisation shift of the patch-sum plane
};
static_assert(sizeof(PMJob) % 8 == 0, "PMJob is copied as an array");

// Tile shape of the PatchMatch kernels (one thread per target pixel).
struct TileCfg {
    int32_t tw, th;
};
int n_tile_cfgs();
TileCfg tile_cfg(int i);

// One term of a remap sum: weight * (source remapped through f), or with
// f == nullptr weight * the source itself.  kind 0: the source is a style
// frame, padded level-0 (R,G,B,0) uint8 pixels, in [0,1] units (/ 255);
// kind 1: an fp32 image [h][w][4] (x, y, z, unused), unpadded, read with
// clamped coordinates (the fast mode's tables, Eq. 4-5).
enum RemapKind : int32_t { kRemapStyle = 0, kRemapFloat = 1 };
struct RemapTerm {
    const uint32_t *style_px;  // source (kind 0: padded uint8 pixels; kind 1: float4 pixels)
    const uint32_t *f;         // packed field [h][w] or nullptr
    float weight;
    int32_t kind;
};

// Output frame of a remap sum: out = (sum of its terms) / divisor, written as
// fp32 [h][w][3] (out_kind 0) or [h][w][4] with the 4th channel 0 (out_kind 1);
// out_kind 2: the exact mean of its terms (all style terms of weight 1; the
// divisor is ignored) rounded half up, as uint8 [h][w][3].
struct RemapFrame {
    float *out;
    int32_t term_base, n_terms;
    float divisor;
    int32_t out_kind;
};

// One uint8 RGB input frame: row r starts at rgb + r * row_stride bytes.
struct FrameRef {
    const uint8_t *rgb;
    int64_t row_stride;
};

// ---- launchers (stream-ordered, no synchronisation) ----
// frame f of the n packed is frames[f] (a device table), or `single` when
// frames is nullptr (n = 1)
hipError_t launch_pack_rgbx(const FrameRef *frames, FrameRef single, int n, int h, int w, int p,
                            uint8_t *dst, size_t dst_stride, size_t px_off, int pitch,
                            hipStream_t s);
hipError_t launch_downsample(const uint8_t *base, size_t stride, int n, const LevelGeom &in,
                             const LevelGeom &out, int p, hipStream_t s);
// bound tables of every level of n pyramids at base + f * stride (after the levels are built)
hipError_t launch_bound_tables(uint8_t *base, size_t stride, int n, const PyrLayout &L, hipStream_t s);

hipError_t launch_pm_start(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                           TileCfg cfg, int p, uint64_t seed, hipStream_t s);
// mode bit kIterStyle: the guide + style loss (Eq. 3 / 8 against sty_hat, or
// Eq. 10 against the partner's patch when pair_f is set), which re-scores the
// incumbent instead of reading e_in; bit kIterTrack: tracking candidates
enum IterMode : int { kIterPlain = 0, kIterStyle = 1, kIterTrack = 2 };
// tab_bytes: LDS for the largest bound table among the jobs (12 * max tab_n)
// guarded: every job runs only for one outcome of the guard of seeded pairs
// (guard_when != 0, plain mode): a fixed grid that skips the tiles of jobs
// that do not run
hipError_t launch_pm_iter(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                          TileCfg cfg, int p, int iter, uint64_t seed, int mode, int tab_bytes,
                          hipStream_t s, bool guarded = false);
// S^ = Alg. 2 remap of src_sty through f_in, rounded, into sty_hat (border replicated)
hipError_t launch_style_refresh(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                                TileCfg cfg, int p, hipStream_t s);
hipError_t launch_pm_export(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                            TileCfg cfg, hipStream_t s);
// guard of seeded pairs: sum of each job's energies e_in into *guard; copy
// of (f_alt, e_alt) over (f_out, e_out) for the jobs whose seed was rejected
hipError_t launch_energy_sum(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                             TileCfg cfg, hipStream_t s);
hipError_t launch_guard_select(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                               TileCfg cfg, hipStream_t s);
// one thread per raced pair: sets *guard_any when the pair's seed is rejected
hipError_t launch_guard_decide(const PMJob *jobs, int n_jobs, hipStream_t s);

hipError_t launch_remap_sum(const RemapFrame *frames, int n_frames, const RemapTerm *terms,
                            int h, int w, int pitch, int p, hipStream_t s);

hipError_t launch_field_to_packed(const int32_t *abi, uint32_t *packed, int h, int w, hipStream_t s);
// measurement: blocks x 256 lanes each gather `rows` 5-pixel rows of the
// padded image img (h x w positions, row pitch in pixels >= w + 4)
hipError_t launch_gather_probe(const uint32_t *img, int h, int w, int pitch, bool divergent, int blocks, int rows,
                               uint32_t *out, hipStream_t s);

// ---- learned proposal network (unet.hip, unet_net.hip) ----
// one pair's coarsest pyramid level as network input
struct UNetPairIn {
    const uint32_t *src, *tgt;  // padded pixels of the level
    int32_t h, w, pitch, pad;
};

// Input of a 3x3 convolution: channels [0, ca) from a ([H][W][ca], or
// [H/2][W/2][ca] upsampled 2x nearest when a_half), channels [ca, cin) from
// b ([H][W][cin - ca]); all channel counts multiples of 16.
struct ConvIn {
    const uint16_t *a;
    const uint16_t *b;
    int32_t ca;
    int32_t a_half;
};
constexpr int kConvTile = 256;     // output pixels per workgroup of the LDS kernel
constexpr int kConvHaloMax = 1024; // input pixels (with border) one workgroup may stage
// whether the LDS kernel takes images of this shape (else a single-tensor
// input goes to the direct kernel and a split input is refused)
bool conv_lds_fits(int B, int H, int W);
// out: [px][ostride], channels [0, ostride) of the cout computed ones;
// pool_out (optional, bf16 output only, ostride == cout): also the 2x2
// average pooling of out, [H/2][W/2][cout]
hipError_t launch_conv3x3_in(const ConvIn &X, int B, int H, int W, int cin, const uint16_t *wt,
                             const float *bias, void *out, int cout, int ostride, bool relu, bool out_f32,
                             hipStream_t s, uint16_t *pool_out = nullptr);
hipError_t launch_conv3x3(const uint16_t *in, int B, int H, int W, int cin, const uint16_t *wt,
                          const float *bias, void *out, int cout, int ostride, bool relu, bool out_f32,
                          hipStream_t s);
// the offset head: 32 channels -> fp32 [px][2] (weights [9][cout_pad][32])
hipError_t launch_head3x3(const uint16_t *in, int B, int H, int W, int cin, const uint16_t *wt, int cout_pad,
                          const float *bias, float *out, hipStream_t s);
hipError_t launch_conv_wgrad(const uint16_t *in, const uint16_t *g, int B, int H, int W, int cin, int cout,
                             int chunk_px, float *partial, float *bias_partial, hipStream_t s);
hipError_t launch_reduce_chunks(const float *partial, int n_chunks, long n, float *out, hipStream_t s);
hipError_t launch_pool2(const uint16_t *in, int B, int H, int W, int C, uint16_t *out, hipStream_t s);
hipError_t launch_pool2_bwd_add(const uint16_t *gout, int B, int H, int W, int C, uint16_t *gin, hipStream_t s);
hipError_t launch_upcat(const uint16_t *deep, const uint16_t *skip, int B, int H, int W, int C1, int C2,
                        uint16_t *out, hipStream_t s);
hipError_t launch_upcat_bwd(const uint16_t *gcat, int B, int H, int W, int C1, int C2, uint16_t *gdeep,
                            uint16_t *gskip, hipStream_t s);
hipError_t launch_relu_mask(uint16_t *g, const uint16_t *y, long n, hipStream_t s);
hipError_t launch_input_from_f32(const float *x6, long n_px, uint16_t *out, hipStream_t s);
hipError_t launch_input_from_pyramids(const UNetPairIn *pairs, int n, int H8, int W8, uint16_t *out,
                                      hipStream_t s);
hipError_t launch_pred_to_seed(const float *pred, int H8, int W8, const UNetPairIn *pairs, int32_t *const *seeds,
                               int n, hipStream_t s);
hipError_t launch_pred_extract(const float *pred, long n_px, float *out, hipStream_t s);
hipError_t launch_input_f32_from_pyramid(const UNetPairIn &pair, int H8, int W8, float *out, hipStream_t s);
hipError_t launch_loss(const float *pred, const float *target, const float *mask, long n_px, float *partial,
                       float *totals, uint16_t *grad, hipStream_t s);
hipError_t launch_adam(float *w, const float *g, float *m, float *v, long n_w, long n_total, int cout, int cin,
                       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t *w16, uint16_t *wt16,
                       hipStream_t s);
hipError_t launch_weights_to_bf16(const float *w, long n_w, int cout, int cin, uint16_t *w16, uint16_t *wt16,
                                  hipStream_t s);
hipError_t launch_param_layout(float *flat, float *padded, int cout_r, int cin_r, int cout, int cin, bool to_padded,
                               hipStream_t s);
hipError_t launch_fill_zero(float *p, long n, hipStream_t s);

struct UNet;
UNet *unet_create();
void unet_destroy(UNet *u);
int64_t unet_param_count();
bool unet_loaded(const UNet *u);
hipError_t unet_load(UNet *u, const float *flat, hipStream_t s);
hipError_t unet_save(UNet *u, float *flat, hipStream_t s);
hipError_t unet_save_state(UNet *u, float *flat, float *m, float *v, int64_t *step, hipStream_t s);
hipError_t unet_load_state(UNet *u, const float *flat, const float *m, const float *v, int64_t step, hipStream_t s);
hipError_t unet_grads_flat(UNet *u, float *flat, hipStream_t s);
// reserve: allocate (if needed) and bind the workspace for this shape;
// shape: bind a shape that fits the reserved workspace, never allocating
hipError_t unet_reserve(UNet *u, int B, int H, int W, bool training);
hipError_t unet_shape(UNet *u, int B, int H, int W, bool training);
uint16_t *unet_input_buffer(UNet *u);
float *unet_pred_buffer(UNet *u);
float *unet_loss_buffer(UNet *u);
hipError_t unet_input_from_f32(UNet *u, const float *x6, hipStream_t s);
// keep_cat: also materialise the decoder's concatenated inputs (needed by a
// following backward pass; the forward convolutions read them in place)
hipError_t unet_forward(UNet *u, hipStream_t s, bool keep_cat);
hipError_t unet_loss_backward(UNet *u, const float *target, const float *mask, bool backward, hipStream_t s);
hipError_t unet_adam(UNet *u, float lr, hipStream_t s);
double unet_forward_flops(int B, int H, int W);

}  // namespace fb
