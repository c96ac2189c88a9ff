// PatchMatch kernels (Algorithm 1 and Section 3.2 of arXiv 2311.09265).
//
// One thread per target pixel; a workgroup is a TW x TH tile of one pair at
// one level, and one launch covers every tile of every pair in the batch
// (a flat tile list, see PMJob).  Three kernels:
//
//  k_pm_start   the first field of a level: a Philox draw at the coarsest
//               level ("randomly initialize F"), an offset-field seed, or the
//               upsampled field of the level above ("upsample F"), followed
//               by its loss ("initialize error matrix E").
//  k_pm_iter    one iteration of the concurrent update: every pixel reads the
//               previous field only (its own value and its 4 neighbours), so
//               launches are the only synchronisation (Jacobi double buffer).
//               Candidates, in this fixed order, each against the running
//               best with strict '<':
//                 propagation F(v+d) - d, d = (-1,0), (1,0), (0,-1), (0,1);
//                 random search best + delta, delta uniform on [-rho, rho]^2,
//                 rho = R >> m, m = 0, 1, ... while rho >= 1, R = max(h, w).
//               A candidate equal to the running best is skipped: its loss
//               equals the best loss and could never pass '<'.
//  k_pm_export  packed field -> int32 [h][w][2] and energies for the C ABI.
//
// Loss (Eq. 1) of a candidate u for target v, exact in uint32, row by row:
//   sum s^2 + sum t^2 - 2 sum s t   over each (2p+1)-pixel patch row,
// all as v_dot4_u32_u8 on (R,G,B,0) pixels.  The target patch and its row
// sums t^2 stay in registers for the whole iteration; a source patch row is
// one 16-byte + one 4-byte load from the padded image (no clamping needed).
// Random-search candidates are divergent gathers, so the iteration kernel
// first tests a candidate against the bound table of its source block (no
// pixel read), then fetches its patch row by row and drops it as soon as the
// rows fetched already reach the running best (exact: every pixel's loss is
// >= 0).
//
// Random draws: Philox4x32-10 (Salmon et al., SC'11), key = seed, counter =
// (pixel index r*w + c, pair id, level << 16 | iteration, m >> 2); word m & 3
// gives the row offset from its low 16 bits and the column offset from its
// high 16 bits, a 16-bit draw u mapping to [0, n) as (u * n) >> 16.  The
// initial draw uses iteration 0xFFFF and word 0.  Draws never depend on the
// position of a pair in a batch or on the tile shape.
#include <type_traits>

#include "fb_common.h"

namespace fb {

namespace {

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return min(max(x, lo), hi); }

// Philox4x32-10 block function, from its published definition.
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, x.x), lo0 = 0xD2511F53u * x.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, x.z), lo1 = 0xCD9E8D57u * x.z;
        x = make_uint4(hi1 ^ x.y ^ k0, lo1, hi0 ^ x.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

__device__ __forceinline__ int u16_to_range(uint32_t u16, uint32_t n) {
    return (int)((u16 * n) >> 16);
}

// Consecutive workgroups are dispatched round-robin over the 8 XCDs; give
// each XCD one contiguous range of tiles so a pair's neighbouring tiles (and
// its source image) share that XCD's L2.  A bijection on [0, total).
__device__ __forceinline__ int xcd_tile(int b, int total) {
    const int q = total >> 3, r = total & 7;
    const int x = b & 7, s = b >> 3;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

__device__ __forceinline__ int find_job(const PMJob *__restrict__ jobs, int n, int uniform, int t) {
    if (uniform > 0) return t / uniform;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Device data is read through global (address space 1) pointers: the job
// table only holds generic pointers, and generic loads would compile to flat
// instructions, which wait on both memory counters.  Offsets from the
// wave-uniform image base stay 32-bit.
template <class T>
using gptr = const __attribute__((address_space(1))) T *;
template <class T>
using gptr_mut = __attribute__((address_space(1))) T *;

// (a C-style cast is the one that may change the address space)
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

template <class T>
__device__ __forceinline__ T gload(const void *base, uint32_t byte_off) {
    return *(gptr<T>)((gptr<char>)base + byte_off);
}
template <class T>
__device__ __forceinline__ void gstore(void *base, uint32_t byte_off, T v) {
    *(gptr_mut<T>)((gptr_mut<char>)base + byte_off) = v;
}

// N aligned 4-byte (R,G,B,0) pixels: one 16-byte and one 4-byte load for N = 5.
template <int N>
struct PixRow {
    uint32_t v[N];
};

template <int N>
__device__ __forceinline__ PixRow<N> load_pixrow(const void *base, uint32_t byte_off) {
    gptr<uint32_t> p = (gptr<uint32_t>)((gptr<char>)base + byte_off);
    PixRow<N> r;
#pragma unroll
    for (int j = 0; j < N; ++j) r.v[j] = p[j];
    return r;
}

template <int P>
struct TargetPatch {
    static constexpr int K = 2 * P + 1;
    uint32_t px[K][K];
    uint32_t cum_tt[K];  // sum t^2 of rows 0..i; cum_tt[K - 1] is the patch's
    __device__ __forceinline__ uint32_t pix(int i, int j) const { return px[i][j]; }
};

// A target patch that stays in its LDS-staged tile (row stride SW): only the
// row sums are held in registers, and every use reads the pixel from LDS again
// (the volatile access keeps the compiler from caching the 25 pixels in
// registers), which leaves room for a second patch at a higher occupancy.
template <int P, int SW>
struct LdsPatch {
    static constexpr int K = 2 * P + 1;
    const volatile __attribute__((address_space(3))) uint32_t *s;  // the patch's top-left padded pixel
    uint32_t cum_tt[K];
    __device__ __forceinline__ uint32_t pix(int i, int j) const { return s[i * SW + j]; }
};

template <int P, int SW>
__device__ __forceinline__ void load_target_patch_lds(const uint32_t *s, int base, LdsPatch<P, SW> &t) {
    constexpr int K = 2 * P + 1;
    t.s = (const volatile __attribute__((address_space(3))) uint32_t *)(s + base);
    uint32_t tt = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t x = t.pix(i, j);
            acc = __builtin_amdgcn_udot4(x, x, acc, false);
        }
        tt += acc;
        t.cum_tt[i] = tt;
    }
}

// the patch whose top-left padded pixel is element base of a tile staged in
// LDS with row stride SW
template <int P, int SW>
__device__ __forceinline__ void load_target_patch_lds(const uint32_t *s, int base, TargetPatch<P> &t) {
    constexpr int K = 2 * P + 1;
    uint32_t tt = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            t.px[i][j] = s[base + i * SW + j];
            acc = __builtin_amdgcn_udot4(t.px[i][j], t.px[i][j], acc, false);
        }
        tt += acc;
        t.cum_tt[i] = tt;
    }
}

template <int P>
__device__ __forceinline__ void load_target_patch(const uint32_t *tp, uint32_t off, uint32_t pitch_b,
                                                  TargetPatch<P> &t) {
    constexpr int K = 2 * P + 1;
    uint32_t tt = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const PixRow<K> row = load_pixrow<K>(tp, off + (uint32_t)i * pitch_b);
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            t.px[i][j] = row.v[j];
            acc = __builtin_amdgcn_udot4(row.v[j], row.v[j], acc, false);
        }
        tt += acc;
        t.cum_tt[i] = tt;
    }
}

// sum s^2 - 2 sum s t over pixels [J0, J0 + N) of patch row i
template <int J0, int N, class TP>
__device__ __forceinline__ uint32_t seg_loss(const uint32_t *sp, uint32_t off, const TP &t, int i) {
    const PixRow<N> row = load_pixrow<N>(sp, off);
    uint32_t st = 0, ss = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        st = __builtin_amdgcn_udot4(row.v[j], t.pix(i, J0 + j), st, false);
        ss = __builtin_amdgcn_udot4(row.v[j], row.v[j], ss, false);
    }
    return ss - 2u * st;
}

// Eq. 1 for the source patch whose top-left padded pixel is at byte offset off
template <class TP>
__device__ __forceinline__ uint32_t patch_loss(const uint32_t *sp, uint32_t off, uint32_t pitch_b, const TP &t) {
    constexpr int K = TP::K;
    uint32_t e = t.cum_tt[K - 1];
#pragma unroll
    for (int i = 0; i < K; ++i) e += seg_loss<0, K>(sp, off + (uint32_t)i * pitch_b, t, i);
    return e;
}

struct TileCoord {
    int job, r, c;
    bool active;
};

// flat tile t of a launch: its job, and this thread's pixel in it
template <int TW, int TH>
__device__ __forceinline__ TileCoord locate_tile(const PMJob *__restrict__ jobs, int n_jobs, int uniform_tiles,
                                                 int t) {
    const int j = find_job(jobs, n_jobs, uniform_tiles, t);
    const int lt = t - jobs[j].tile_base;
    const int tx_n = jobs[j].tiles_x;
    const int ty = lt / tx_n, tx = lt - ty * tx_n;
    TileCoord tc;
    tc.job = j;
    tc.r = ty * TH + (int)threadIdx.y;
    tc.c = tx * TW + (int)threadIdx.x;
    tc.active = tc.r < jobs[j].h && tc.c < jobs[j].w;
    return tc;
}

template <int TW, int TH>
__device__ __forceinline__ TileCoord locate(const PMJob *__restrict__ jobs, int n_jobs,
                                            int total_tiles, int uniform_tiles) {
    return locate_tile<TW, TH>(jobs, n_jobs, uniform_tiles, xcd_tile((int)blockIdx.x, total_tiles));
}

// The tile's padded target pixels with their patch border, (TH + 2P) rows of
// TW + 2P, into LDS with coalesced loads; reads past the image are clamped
// into it (those entries are never used).
template <int P, int TW, int TH>
__device__ __forceinline__ void stage_target_tile(uint32_t *s_tgt, const PMJob &J, const TileCoord &tc) {
    constexpr int SW = TW + 2 * P, SH = TH + 2 * P;
    const int tid = (int)(threadIdx.y * TW + threadIdx.x);
    const int rt = tc.r - (int)threadIdx.y, ct = tc.c - (int)threadIdx.x;  // tile origin
    gptr<uint32_t> tp = (gptr<uint32_t>)J.tgt_px;
    for (int i = tid; i < SH * SW; i += TW * TH) {
        const int yy = min(rt + i / SW, J.h + 2 * P - 1), xx = min(ct + i % SW, J.w + 2 * P - 1);
        s_tgt[i] = tp[yy * J.pitch + xx];
    }
}

template <int P, int TW, int TH>
__global__ void __launch_bounds__(TW *TH)
k_pm_start(const PMJob *__restrict__ jobs, int n_jobs, int total_tiles, int uniform_tiles,
           uint32_t k0, uint32_t k1) {
    constexpr int SW = TW + 2 * P, SH = TH + 2 * P;
    __shared__ uint32_t s_tgt[SH * SW];
    const TileCoord tc = locate<TW, TH>(jobs, n_jobs, total_tiles, uniform_tiles);
    const PMJob &J = jobs[tc.job];
    if (J.mode != kStartCopyAbi) {  // the same for the whole workgroup
        stage_target_tile<P, TW, TH>(s_tgt, J, tc);
        __syncthreads();
    }
    if (!tc.active) return;
    const int h = J.h, w = J.w, r = tc.r, c = tc.c;
    const int v = r * w + c;
    int fr, fc;
    switch (J.mode) {
    case kStartRandom: {
        const uint4 x = philox4x32_10(make_uint4((uint32_t)v, J.pair_id,
                                                 ((uint32_t)J.level << 16) | 0xFFFFu, 0u), k0, k1);
        fr = u16_to_range(x.x & 0xFFFFu, (uint32_t)h);
        fc = u16_to_range(x.x >> 16, (uint32_t)w);
        break;
    }
    case kStartOffsets:
        // offsets limited to +-size first, so the sum cannot overflow
        fr = clampi(r + clampi(J.aux_off[2 * v], -h, h), 0, h - 1);
        fc = clampi(c + clampi(J.aux_off[2 * v + 1], -w, w), 0, w - 1);
        break;
    case kStartUpsample: {
        const uint32_t q = J.f_in[(r >> 1) * J.wc + (c >> 1)];
        fr = clampi(2 * (int)(q >> 16) + (r & 1), 0, h - 1);
        fc = clampi(2 * (int)(q & 0xFFFFu) + (c & 1), 0, w - 1);
        break;
    }
    case kStartUpsampleAbi: {
        const int qi = (r >> 1) * J.wc + (c >> 1);
        fr = clampi(2 * clampi(J.aux_off[2 * qi], 0, J.hc - 1) + (r & 1), 0, h - 1);
        fc = clampi(2 * clampi(J.aux_off[2 * qi + 1], 0, J.wc - 1) + (c & 1), 0, w - 1);
        break;
    }
    default: {  // kStartCopyAbi: the given field and energies (entries clamped into range)
        fr = clampi(J.aux_off[2 * v], 0, h - 1);
        fc = clampi(J.aux_off[2 * v + 1], 0, w - 1);
        J.f_out[v] = ((uint32_t)fr << 16) | (uint32_t)fc;
        J.e_out[v] = J.e_abi[v];
        return;
    }
    }
    const uint32_t pitch_b = 4u * (uint32_t)J.pitch;
    TargetPatch<P> t;
    load_target_patch_lds<P, SW>(s_tgt, (int)threadIdx.y * SW + (int)threadIdx.x, t);
    gstore<uint32_t>(J.f_out, 4u * v, ((uint32_t)fr << 16) | (uint32_t)fc);
    gstore<uint32_t>(J.e_out, 4u * v, patch_loss(J.src_px, 4u * (uint32_t)(fr * J.pitch + fc), pitch_b, t));
}

// MODE & kIterStyle: a guide + style loss scaled by 16 to stay an integer,
//   alpha16 SSD(G_j[u], G_i[v]) + 16 SSD(S_j[u], X),
// where X is the patch of sty_hat at v (Eq. 3: the remapped style S^,
// refreshed by k_style_refresh before every iteration launch; Eq. 8: the
// fixed average T^-), or, when pair_f is set, the partner's source-style
// patch at the partner's current match (Eq. 10, the pairwise patch error).
// The incumbent is re-scored under X instead of taking e_in.
// MODE & kIterTrack: after propagation, the matches of the pairs with the
// same source and the neighbouring target frames are candidates too.
// Every launch stages in LDS, with coalesced loads: the tile's target pixels
// with their patch border, the tile's old field with a 1-entry border (the
// incumbent and the propagation neighbours), and the source level's bound
// table (the per-block ranges of the candidates' per-channel patch sums,
// built with the pyramid), by which a candidate whose Cauchy-Schwarz bound
// already reaches the running best is ruled out before any of its pixels is
// fetched.
// With a style loss, a random-search candidate that passes the table is also
// tested against its own quantised patch sums (the source level's patch-sum
// plane) before any row is fetched; the guide patch is read from the LDS tile
// at every use (only the target patch of the style term stays in registers),
// and for p <= 2 the kernel is held to 6 waves per SIMD (at most 80 VGPRs, no
// spills); larger patches keep the compiler's choice.
// One tile (flat index `tile`) of an iteration launch, staged in the workgroup's
// LDS arrays; every thread of the workgroup calls it with the same t.
template <int P, int TW, int TH, int MODE>
__device__ __forceinline__ void pm_iter_tile(const PMJob *__restrict__ jobs, int n_jobs, int uniform_tiles,
                                             int tile, int iter, uint32_t k0, uint32_t k1, uint32_t *s_tgt, uint32_t *s_f,
                                             u32x4 *s_btab4) {
    constexpr bool STYLE = (MODE & kIterStyle) != 0, TRACK = (MODE & kIterTrack) != 0;
    constexpr int K = 2 * P + 1;
    constexpr int FW = TW + 2, FH = TH + 2;          // field tile with a 1-entry border
    constexpr int SW = TW + 2 * P;                   // target tile row with its patch border
    const uint32_t *s_btab = reinterpret_cast<const uint32_t *>(s_btab4);
    const TileCoord tc = locate_tile<TW, TH>(jobs, n_jobs, uniform_tiles, tile);
    const PMJob &J = jobs[tc.job];
    if (J.guard_when != 0) {  // the same for the whole workgroup
        const bool rejected = J.guard[0] > J.guard[1];
        if (rejected != (J.guard_when == 1)) return;
    }
    const int h = J.h, w = J.w, pitch = J.pitch, r = tc.r, c = tc.c;
    const int tab_n = J.tab_n;  // the same for the whole workgroup
    stage_target_tile<P, TW, TH>(s_tgt, J, tc);
    {
        const int tid = (int)(threadIdx.y * TW + threadIdx.x);
        const int rt = r - (int)threadIdx.y, ct = c - (int)threadIdx.x;  // tile origin
        gptr<uint32_t> fp = (gptr<uint32_t>)J.f_in;
        for (int i = tid; i < FH * FW; i += TW * TH) {
            const int yy = rt - 1 + i / FW, xx = ct - 1 + i % FW;
            s_f[i] = (yy >= 0 && yy < h && xx >= 0 && xx < w) ? fp[yy * w + xx] : 0u;
        }
        if (tab_n > 0) {
            // 16-byte loads; the table's region is padded to 256 bytes, so the
            // last load stays inside it
            gptr<u32x4> bt = (gptr<u32x4>)J.btab;
            for (int i = tid; i < (3 * tab_n + 3) / 4; i += TW * TH) s_btab4[i] = bt[i];
        }
    }
    __syncthreads();
    if (!tc.active) return;
    const int v = r * w + c;
    const uint32_t pitch_b = 4u * (uint32_t)pitch;
    const uint32_t *src_px = J.src_px;
    const int fc0 = ((int)threadIdx.y + 1) * FW + (int)threadIdx.x + 1;  // this pixel in s_f

    // the guide patch; with the style loss it is read from LDS at every use
    std::conditional_t<STYLE, LdsPatch<P, SW>, TargetPatch<P>> t;
    TargetPatch<P> ts;  // the patch of S^ or of the partner (style losses only)
    load_target_patch_lds<P, SW>(s_tgt, (int)threadIdx.y * SW + (int)threadIdx.x, t);
    const uint32_t *src_sty = J.src_sty;
    const uint32_t a16 = STYLE ? (uint32_t)J.alpha16 : 1u;
    if constexpr (STYLE) {
        if (J.pair_f) {
            const uint32_t q = gload<uint32_t>(J.pair_f, 4u * v);
            load_target_patch<P>(J.pair_sty, 4u * (uint32_t)((int)(q >> 16) * pitch + (int)(q & 0xFFFFu)), pitch_b, ts);
        } else {
            load_target_patch<P>(J.sty_hat, 4u * (uint32_t)(r * pitch + c), pitch_b, ts);
        }
    }

    // the target patch's per-channel sums T_c, for the bound-table test
    int ts0 = 0, ts1 = 0, ts2 = 0;
    if (tab_n > 0) {
        uint32_t a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const uint32_t x = t.pix(i, j);
                a0 = __builtin_amdgcn_udot4(x, 0x00000001u, a0, false);
                a1 = __builtin_amdgcn_udot4(x, 0x00000100u, a1, false);
                a2 = __builtin_amdgcn_udot4(x, 0x00010000u, a2, false);
            }
        ts0 = (int)a0;
        ts1 = (int)a1;
        ts2 = (int)a2;
    }
    const int tab_shift = J.tab_shift, tab_w = J.tab_w;
    const int qs = J.psum_shift;
    const short nqw = (short)(1 - (1 << qs));  // minus the width of a quantisation step
    // added to the table's pairs (mn_R, mn_G), (mn_B, -mx_R), (-mx_G, -mx_B):
    // the six differences whose positive parts are the distances to the ranges
    const s16x2 u0 = {(short)-ts0, (short)-ts1}, u1 = {(short)-ts2, (short)ts0}, u2 = {(short)ts1, (short)ts2};
    // sum_c dist(T_c, [lo_c, hi_c])^2 for ranges given as those three pairs
    auto range_lb = [&](s16x2 p0, s16x2 p1, s16x2 p2) {
        const s16x2 z = {0, 0};
        const s16x2 d0 = __builtin_elementwise_max(p0 + u0, z);
        const s16x2 d1 = __builtin_elementwise_max(p1 + u1, z);
        const s16x2 d2 = __builtin_elementwise_max(p2 + u2, z);
        uint32_t lb = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, d0), __builtin_bit_cast(u16x2, d0), 0u, false);
        lb = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, d1), __builtin_bit_cast(u16x2, d1), lb, false);
        return __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2, d2), __builtin_bit_cast(u16x2, d2), lb, false);
    };

    const uint32_t f0 = s_f[fc0];
    int br = (int)(f0 >> 16), bc = (int)(f0 & 0xFFFFu);
    uint32_t be;
    if (STYLE && !J.e_valid) {
        const uint32_t off = 4u * (uint32_t)(br * pitch + bc);
        be = a16 * patch_loss(src_px, off, pitch_b, t) + 16u * patch_loss(src_sty, off, pitch_b, ts);
    } else {
        be = gload<uint32_t>(J.e_in, 4u * v);
    }

    // Every pixel's share of the loss is a square, so any part of the patch
    // whose loss alone reaches the running best rules the candidate out of
    // '<'.  A random-search candidate first meets the table bound (no memory
    // read); then the patch is tested after every complete row, so a row is
    // fetched only by lanes still in the race.  The sum of s^2 - 2 s t wraps
    // in uint32, but with the t^2 sums added back every partial loss is the
    // exact nonnegative value.  (Eq. 3: both terms are sums of squares, so the
    // weighted partial sums are lower bounds in the same way; the host admits
    // only alpha16 with (alpha16 + 16) * 3 * 255^2 * (2p+1)^2 < 2^32, so the
    // weighted total, and every partial sum below it, never wraps.)
    // (2p+1)^2 * be, saturated: a bound lb (< 2^32) at or above it rules the
    // candidate out (plain loss; be may be any energy a caller passed in)
    auto bound_threshold = [&]() {
        const uint64_t x = (uint64_t)(K * K) * be;
        return x > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)x;
    };
    uint32_t thr = 0;
    auto consider = [&](int cr, int cc, auto use_bound) {
        if (cr == br && cc == bc) return;
        if (decltype(use_bound)::value && tab_n > 0) {
            // sum_c dist(T_c, [mn_c, mx_c])^2 <= (2p+1)^2 * SSD(G); at most one
            // of each channel's two differences is positive
            const int e = (cr >> tab_shift) * tab_w + (cc >> tab_shift);
            const uint32_t lb = range_lb(__builtin_bit_cast(s16x2, s_btab[e]), __builtin_bit_cast(s16x2, s_btab[tab_n + e]),
                                         __builtin_bit_cast(s16x2, s_btab[2 * tab_n + e]));
            if constexpr (STYLE) {
                if ((uint64_t)a16 * lb >= (uint64_t)(K * K) * be) return;
            } else {
                if (lb >= thr) return;
            }
        }
        const uint32_t off = 4u * (uint32_t)(cr * pitch + cc);
        if (STYLE && decltype(use_bound)::value && tab_n > 0) {
            // the same bound from the candidate's own patch sums, known to
            // within 2^qs - 1 from the plane (only with a style loss, where a
            // candidate that gets this far costs two patches per row; in the
            // guide-only kernel the extra load per candidate costs more than
            // the rows it saves)
            const uint32_t q = gload<uint32_t>(J.psum, off);
            const s16x2 lo01 = __builtin_bit_cast(s16x2, ((q & 0x3FFu) | ((q << 6) & 0x3FF0000u)) << qs);
            const short lo2 = (short)((q >> 20) << qs);
            // the pairs (lo_R, lo_G), (lo_B, -hi_R), (-hi_G, -hi_B), as in the table
            const s16x2 p1 = {lo2, (short)(nqw - lo01.x)}, p2 = {(short)(nqw - lo01.y), (short)(nqw - lo2)};
            const uint32_t lb = range_lb(lo01, p1, p2);
            if constexpr (STYLE) {
                if ((uint64_t)a16 * lb >= (uint64_t)(K * K) * be) return;
            } else {
                if (lb >= thr) return;
            }
        }
        uint32_t acc = 0, accs = 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            acc += seg_loss<0, K>(src_px, off + (uint32_t)i * pitch_b, t, i);
            if constexpr (STYLE) accs += seg_loss<0, K>(src_sty, off + (uint32_t)i * pitch_b, ts, i);
            if (i < K - 1) {
                if constexpr (STYLE) {
                    if (a16 * (t.cum_tt[i] + acc) + 16u * (ts.cum_tt[i] + accs) >= be) return;
                } else {
                    if (t.cum_tt[i] + acc >= be) return;
                }
            }
        }
        uint32_t e;
        if constexpr (STYLE) e = a16 * (t.cum_tt[K - 1] + acc) + 16u * (ts.cum_tt[K - 1] + accs);
        else e = t.cum_tt[K - 1] + acc;
        if (e < be) {
            br = cr;
            bc = cc;
            be = e;
            if constexpr (!STYLE) thr = bound_threshold();
        }
    };
    if constexpr (!STYLE) thr = bound_threshold();
    constexpr std::false_type kNoBound{};
    constexpr std::true_type kBound{};

    // propagation: F(v + d) - d for d = (-1,0), (1,0), (0,-1), (0,1)
    if (r > 0) {
        const uint32_t q = s_f[fc0 - FW];
        consider(min((int)(q >> 16) + 1, h - 1), (int)(q & 0xFFFFu), kNoBound);
    }
    if (r < h - 1) {
        const uint32_t q = s_f[fc0 + FW];
        consider(max((int)(q >> 16) - 1, 0), (int)(q & 0xFFFFu), kNoBound);
    }
    if (c > 0) {
        const uint32_t q = s_f[fc0 - 1];
        consider((int)(q >> 16), min((int)(q & 0xFFFFu) + 1, w - 1), kNoBound);
    }
    if (c < w - 1) {
        const uint32_t q = s_f[fc0 + 1];
        consider((int)(q >> 16), max((int)(q & 0xFFFFu) - 1, 0), kNoBound);
    }
    if constexpr (TRACK) {
        if (J.trk_prev) {
            const uint32_t q = gload<uint32_t>(J.trk_prev, 4u * v);
            consider((int)(q >> 16), (int)(q & 0xFFFFu), kNoBound);
        }
        if (J.trk_next) {
            const uint32_t q = gload<uint32_t>(J.trk_next, 4u * v);
            consider((int)(q >> 16), (int)(q & 0xFFFFu), kNoBound);
        }
    }

    // random search around the running best, radius halving from max(h, w)
    const int R = max(h, w);
    const uint32_t ctr2 = ((uint32_t)J.level << 16) | (uint32_t)iter;
    uint4 x = make_uint4(0, 0, 0, 0);
#pragma unroll 4  // the Philox word of radius m is then picked at compile time
    for (int m = 0; (R >> m) > 0; ++m) {
        if ((m & 3) == 0) x = philox4x32_10(make_uint4((uint32_t)v, J.pair_id, ctr2, (uint32_t)(m >> 2)), k0, k1);
        const int s = m & 3;
        const uint32_t word = s == 0 ? x.x : (s == 1 ? x.y : (s == 2 ? x.z : x.w));
        const int rho = R >> m;
        const uint32_t n = 2u * (uint32_t)rho + 1u;
        const int dr = u16_to_range(word & 0xFFFFu, n) - rho;
        const int dc = u16_to_range(word >> 16, n) - rho;
        consider(clampi(br + dr, 0, h - 1), clampi(bc + dc, 0, w - 1), kBound);
    }
    gstore<uint32_t>(J.f_out, 4u * v, ((uint32_t)br << 16) | (uint32_t)bc);
    gstore<uint32_t>(J.e_out, 4u * v, be);
}

template <int P, int TW, int TH, int MODE>
__global__ void __launch_bounds__(TW *TH, ((MODE & kIterStyle) && P <= 2) ? 6 : 1)
k_pm_iter(const PMJob *__restrict__ jobs, int n_jobs, int total_tiles, int uniform_tiles, int iter,
          uint32_t k0, uint32_t k1) {
    __shared__ uint32_t s_tgt[(TH + 2 * P) * (TW + 2 * P)];  // target tile with its patch border
    __shared__ uint32_t s_f[(TH + 2) * (TW + 2)];            // field tile with a 1-entry border
    extern __shared__ u32x4 s_btab4[];  // the three 16-bit-pair arrays of the bound table
    pm_iter_tile<P, TW, TH, MODE>(jobs, n_jobs, uniform_tiles, xcd_tile((int)blockIdx.x, total_tiles), iter, k0,
                                  k1, s_tgt, s_f, s_btab4);
}

// An iteration launch whose jobs all run only for some outcome of the guard
// of seeded pairs (guard_when != 0): a fixed grid walks the flat tiles and
// skips the tiles of jobs that do not run, at the cost of a few scalar loads;
// when the jobs run only for rejected seeds and no seed of the call was
// rejected, every workgroup returns after one load.
template <int P, int TW, int TH>
__global__ void __launch_bounds__(TW *TH)
k_pm_iter_guarded(const PMJob *__restrict__ jobs, int n_jobs, int total_tiles, int uniform_tiles, int iter,
                  uint32_t k0, uint32_t k1) {
    __shared__ uint32_t s_tgt[(TH + 2 * P) * (TW + 2 * P)];
    __shared__ uint32_t s_f[(TH + 2) * (TW + 2)];
    extern __shared__ u32x4 s_btab4[];
    // the launch's jobs all run only for a rejected seed: none was rejected
    // (the word is set by k_guard_decide before any such launch)
    if (jobs[0].guard_when == 1 && *jobs[0].guard_any == 0) return;
    for (int t = (int)blockIdx.x; t < total_tiles; t += (int)gridDim.x) {
        const PMJob &J = jobs[find_job(jobs, n_jobs, uniform_tiles, t)];
        if (J.guard_when != 0 && (J.guard[0] > J.guard[1]) != (J.guard_when == 1)) continue;
        __syncthreads();  // the previous tile's LDS contents have been read
        pm_iter_tile<P, TW, TH, kIterPlain>(jobs, n_jobs, uniform_tiles, t, iter, k0, k1, s_tgt, s_f, s_btab4);
    }
}

// S^ of Eq. 3 for one iteration: the Alg. 2 remap of the source style level
// through the field f_in, each channel's average rounded half up
// ((2 sum + count) / (2 count)), as (R,G,B,0) pixels written into the padded
// sty_hat together with its replicated border, so the loss never clamps.
// The tile's field entries with a P-pixel border are staged in LDS once.
// After a level's first iteration (f_prev set) only the waves whose field
// neighbourhood changed since the previous refresh recompute their pixels.
template <int P, int TW, int TH>
__global__ void __launch_bounds__(TW *TH)
k_style_refresh(const PMJob *__restrict__ jobs, int n_jobs, int total_tiles, int uniform_tiles) {
    constexpr int SW = TW + 2 * P, SH = TH + 2 * P;
    constexpr int WROWS = TW < 64 ? 64 / TW : 1;  // tile rows of one wave
    __shared__ uint32_t sf[SH * SW];
    __shared__ uint32_t s_rowch[SH];  // staged row holds an entry that differs from f_prev
    const TileCoord tc = locate<TW, TH>(jobs, n_jobs, total_tiles, uniform_tiles);
    const PMJob &J = jobs[tc.job];
    const int h = J.h, w = J.w, pitch = J.pitch, r = tc.r, c = tc.c;
    const int rt = r - (int)threadIdx.y, ct = c - (int)threadIdx.x;  // tile origin
    const int tid = (int)(threadIdx.y * TW + threadIdx.x);
    const bool incr = J.f_prev != nullptr;  // the same for the whole workgroup
    if (incr) {
        for (int i = tid; i < SH; i += TW * TH) s_rowch[i] = 0u;
        __syncthreads();
    }
    for (int i = tid; i < SH * SW; i += TW * TH) {
        const int yy = rt - P + i / SW, xx = ct - P + i % SW;
        const bool in = yy >= 0 && yy < h && xx >= 0 && xx < w;
        const uint32_t q = in ? gload<uint32_t>(J.f_in, 4u * (uint32_t)(yy * w + xx)) : 0u;
        sf[i] = q;
        if (incr && in && q != gload<uint32_t>(J.f_prev, 4u * (uint32_t)(yy * w + xx))) s_rowch[i / SW] = 1u;
    }
    __syncthreads();
    if (!tc.active) return;
    if (incr) {
        // S^ at a pixel depends only on the field entries within P of it: a wave
        // whose pixels saw no change keeps the previous refresh's values (and
        // border copies) in sty_hat
        const int wr0 = (tid >> 6) * WROWS;
        bool changed = false;
        for (int y = wr0; y < wr0 + WROWS + 2 * P; ++y) changed |= s_rowch[y] != 0u;
        if (!changed) return;
    }
    uint32_t rb = 0, g = 0, cnt = 0;  // R and B sums in 16-bit halves; G alone
    // A wave whose whole staged neighbourhood (its rows with the P-row border)
    // holds one translation F(u) - u at every in-image entry has
    // F(v + d) - d = F(v) for every pixel and in-image d: every term is
    // S(F(v)), gathered once (packed (row << 16) + col differences are equal
    // exactly when the translations are, sides being below 2^15).  Waves with
    // pixels outside the image take the general sum.
    const uint32_t q0 = sf[((int)threadIdx.y + P) * SW + (int)threadIdx.x + P];
    bool coherent = __ballot(1) == ~0ull;
    if (coherent) {
        constexpr int RN = (WROWS + 2 * P) * SW;
        const int wy0 = (tid >> 6) * WROWS;
        const uint32_t ref = (uint32_t)__shfl((int)(q0 - (((uint32_t)r << 16) + (uint32_t)c)), 0);
        bool ok = true;
#pragma unroll
        for (int e = tid & 63; e < RN; e += 64) {
            const int ry = wy0 + e / SW, rx = e - (e / SW) * SW;
            const int yy = rt - P + ry, xx = ct - P + rx;
            if (yy >= 0 && yy < h && xx >= 0 && xx < w)
                ok &= sf[ry * SW + rx] - (((uint32_t)yy << 16) + (uint32_t)xx) == ref;
        }
        coherent = __all(ok);
    }
    if (coherent) {
        const uint32_t px = gload<uint32_t>(J.src_sty, 4u * (uint32_t)(((int)(q0 >> 16) + P) * pitch + (int)(q0 & 0xFFFFu) + P));
        cnt = (uint32_t)((min(P, h - 1 - r) + min(P, r) + 1) * (min(P, w - 1 - c) + min(P, c) + 1));
        rb = cnt * (px & 0x00FF00FFu);
        g = cnt * ((px >> 8) & 0xFFu);
    } else {
#pragma unroll
    for (int dr = -P; dr <= P; ++dr) {
        if (r + dr < 0 || r + dr >= h) continue;
#pragma unroll
        for (int dc = -P; dc <= P; ++dc) {
            if (c + dc < 0 || c + dc >= w) continue;
            const uint32_t q = sf[((int)threadIdx.y + P + dr) * SW + (int)threadIdx.x + P + dc];
            // source pixel clamp(F(v + d) - d), read from the padded style level
            const int sr = (int)(q >> 16) - dr + P, sc = (int)(q & 0xFFFFu) - dc + P;
            const uint32_t px = gload<uint32_t>(J.src_sty, 4u * (uint32_t)(sr * pitch + sc));
            rb += px & 0x00FF00FFu;
            g += (px >> 8) & 0xFFu;
            ++cnt;
        }
    }
    }
    const uint32_t vr = (2u * (rb & 0xFFFFu) + cnt) / (2u * cnt);
    const uint32_t vg = (2u * g + cnt) / (2u * cnt);
    const uint32_t vb = (2u * (rb >> 16) + cnt) / (2u * cnt);
    const uint32_t px = vr | (vg << 8) | (vb << 16);
    // this pixel, and the border copies it stands for at the image edges
    const int r0 = r == 0 ? -P : 0, r1 = r == h - 1 ? P : 0;
    const int c0 = c == 0 ? -P : 0, c1 = c == w - 1 ? P : 0;
    for (int a = r0; a <= r1; ++a)
        for (int b = c0; b <= c1; ++b)
            gstore<uint32_t>(J.sty_hat, 4u * (uint32_t)((r + P + a) * pitch + (c + P + b)), px);
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW *TH)
k_pm_export(const PMJob *__restrict__ jobs, int n_jobs, int total_tiles, int uniform_tiles) {
    const TileCoord tc = locate<TW, TH>(jobs, n_jobs, total_tiles, uniform_tiles);
    if (!tc.active) return;
    const PMJob &J = jobs[tc.job];
    const int v = tc.r * J.w + tc.c;
    const uint32_t f = J.f_in[v];
    reinterpret_cast<int2 *>(J.nnf_abi)[v] = make_int2((int)(f >> 16), (int)(f & 0xFFFFu));
    J.energy_abi[v] = J.e_in[v];
}

// Sum of the tile's energies e_in, added to *J.guard (64-bit, so the order of
// the additions cannot change the result).
template <int TW, int TH>
__global__ void __launch_bounds__(TW *TH)
k_energy_sum(const PMJob *__restrict__ jobs, int n_jobs, int total_tiles, int uniform_tiles) {
    __shared__ unsigned long long s_sum[TW * TH];
    const TileCoord tc = locate<TW, TH>(jobs, n_jobs, total_tiles, uniform_tiles);
    const PMJob &J = jobs[tc.job];
    const int tid = (int)(threadIdx.y * TW + threadIdx.x);
    s_sum[tid] = tc.active ? (unsigned long long)J.e_in[tc.r * J.w + tc.c] : 0ull;
    __syncthreads();
    for (int k = TW * TH / 2; k > 0; k >>= 1) {
        if (tid < k) s_sum[tid] += s_sum[tid + k];
        __syncthreads();
    }
    if (tid == 0) atomicAdd(reinterpret_cast<unsigned long long *>(J.guard), s_sum[0]);
}

// For a rejected seed, the plain run's field and energies replace the seeded
// run's.
template <int TW, int TH>
__global__ void __launch_bounds__(TW *TH)
k_guard_select(const PMJob *__restrict__ jobs, int n_jobs, int total_tiles, int uniform_tiles) {
    const TileCoord tc = locate<TW, TH>(jobs, n_jobs, total_tiles, uniform_tiles);
    if (!tc.active) return;
    const PMJob &J = jobs[tc.job];
    if (!(J.guard[0] > J.guard[1])) return;
    const int v = tc.r * J.w + tc.c;
    J.f_out[v] = J.f_alt[v];
    J.e_out[v] = J.e_alt[v];
}

// The race's outcome of every raced pair: a rejected seed sets the call's
// any-rejected word (launches that only rejected seeds need skip at once
// while it is 0).
__global__ void __launch_bounds__(64) k_guard_decide(const PMJob *__restrict__ jobs, int n) {
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const PMJob &J = jobs[k];
    if (J.guard[0] > J.guard[1]) *J.guard_any = 1;
}

// int32 [h][w][2] field -> packed; entries are clamped into the image so a
// malformed field can never steer a later gather outside the padded image.
__global__ void __launch_bounds__(256)
k_field_to_packed(const int32_t *__restrict__ abi, uint32_t *__restrict__ packed, int h, int w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= h * w) return;
    const int2 f = reinterpret_cast<const int2 *>(abi)[i];
    packed[i] = ((uint32_t)clampi(f.x, 0, h - 1) << 16) | (uint32_t)clampi(f.y, 0, w - 1);
}

constexpr TileCfg kTileCfgs[] = {{64, 4}, {32, 8}, {16, 16}, {64, 2}};
constexpr int kGuardedGrid = 2048;  // workgroups of a guarded iteration launch (8 per CU)

}  // namespace

int n_tile_cfgs() { return (int)(sizeof(kTileCfgs) / sizeof(kTileCfgs[0])); }
TileCfg tile_cfg(int i) { return kTileCfgs[i]; }

#define FB_TILE_SWITCH(CFG, MACRO)                                            \
    if ((CFG).tw == 64 && (CFG).th == 4) { MACRO(64, 4); }                    \
    else if ((CFG).tw == 32 && (CFG).th == 8) { MACRO(32, 8); }               \
    else if ((CFG).tw == 16 && (CFG).th == 16) { MACRO(16, 16); }             \
    else if ((CFG).tw == 64 && (CFG).th == 2) { MACRO(64, 2); }               \
    else return hipErrorInvalidValue;

#define FB_P_SWITCH(P_, MACRO2, TW, TH)                                       \
    switch (P_) {                                                             \
    case 1: MACRO2(1, TW, TH); break;                                         \
    case 2: MACRO2(2, TW, TH); break;                                         \
    case 3: MACRO2(3, TW, TH); break;                                         \
    case 4: MACRO2(4, TW, TH); break;                                         \
    default: return hipErrorInvalidValue;                                     \
    }

hipError_t launch_pm_start(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                           TileCfg cfg, int p, uint64_t seed, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#define FB_START2(P_, TW, TH)                                                                 \
    hipLaunchKernelGGL((k_pm_start<P_, TW, TH>), dim3(total_tiles), dim3(TW, TH), 0, s, jobs, \
                       n_jobs, total_tiles, uniform_tiles, k0, k1)
#define FB_START(TW, TH) FB_P_SWITCH(p, FB_START2, TW, TH)
    FB_TILE_SWITCH(cfg, FB_START)
#undef FB_START
#undef FB_START2
    return hipGetLastError();
}

hipError_t launch_pm_iter(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                          TileCfg cfg, int p, int iter, uint64_t seed, int mode, int tab_bytes,
                          hipStream_t s, bool guarded) {
    if (total_tiles <= 0) return hipSuccess;
    if (mode < 0 || mode > 3 || tab_bytes < 0 || tab_bytes > kBoundTabBytes) return hipErrorInvalidValue;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (guarded) {
        if (mode != kIterPlain) return hipErrorInvalidValue;
        const int grid = total_tiles < kGuardedGrid ? total_tiles : kGuardedGrid;
#define FB_GITER2(P_, TW, TH)                                                                           \
    hipLaunchKernelGGL((k_pm_iter_guarded<P_, TW, TH>), dim3(grid), dim3(TW, TH), (size_t)tab_bytes, s, \
                       jobs, n_jobs, total_tiles, uniform_tiles, iter, k0, k1)
#define FB_GITER(TW, TH) FB_P_SWITCH(p, FB_GITER2, TW, TH)
        FB_TILE_SWITCH(cfg, FB_GITER)
#undef FB_GITER
#undef FB_GITER2
        return hipGetLastError();
    }
#define FB_ITER3(P_, TW, TH, M_)                                                                   \
    hipLaunchKernelGGL((k_pm_iter<P_, TW, TH, M_>), dim3(total_tiles), dim3(TW, TH), (size_t)tab_bytes, \
                       s, jobs, n_jobs, total_tiles, uniform_tiles, iter, k0, k1)
#define FB_ITER2(P_, TW, TH)                                                   \
    if (mode == 0) FB_ITER3(P_, TW, TH, 0);                                    \
    else if (mode == 1) FB_ITER3(P_, TW, TH, 1);                               \
    else if (mode == 2) FB_ITER3(P_, TW, TH, 2);                               \
    else FB_ITER3(P_, TW, TH, 3)
#define FB_ITER(TW, TH) FB_P_SWITCH(p, FB_ITER2, TW, TH)
    FB_TILE_SWITCH(cfg, FB_ITER)
#undef FB_ITER
#undef FB_ITER2
#undef FB_ITER3
    return hipGetLastError();
}

hipError_t launch_style_refresh(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                                TileCfg cfg, int p, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
#define FB_REFRESH2(P_, TW, TH)                                                                      \
    hipLaunchKernelGGL((k_style_refresh<P_, TW, TH>), dim3(total_tiles), dim3(TW, TH), 0, s, jobs, \
                       n_jobs, total_tiles, uniform_tiles)
#define FB_REFRESH(TW, TH) FB_P_SWITCH(p, FB_REFRESH2, TW, TH)
    FB_TILE_SWITCH(cfg, FB_REFRESH)
#undef FB_REFRESH
#undef FB_REFRESH2
    return hipGetLastError();
}

hipError_t launch_pm_export(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                            TileCfg cfg, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
#define FB_EXPORT(TW, TH)                                                                     \
    hipLaunchKernelGGL((k_pm_export<TW, TH>), dim3(total_tiles), dim3(TW, TH), 0, s, jobs,    \
                       n_jobs, total_tiles, uniform_tiles)
    FB_TILE_SWITCH(cfg, FB_EXPORT)
#undef FB_EXPORT
    return hipGetLastError();
}

hipError_t launch_energy_sum(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                             TileCfg cfg, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
#define FB_ESUM(TW, TH)                                                                       \
    hipLaunchKernelGGL((k_energy_sum<TW, TH>), dim3(total_tiles), dim3(TW, TH), 0, s, jobs,   \
                       n_jobs, total_tiles, uniform_tiles)
    FB_TILE_SWITCH(cfg, FB_ESUM)
#undef FB_ESUM
    return hipGetLastError();
}

hipError_t launch_guard_select(const PMJob *jobs, int n_jobs, int total_tiles, int uniform_tiles,
                               TileCfg cfg, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
#define FB_GSEL(TW, TH)                                                                       \
    hipLaunchKernelGGL((k_guard_select<TW, TH>), dim3(total_tiles), dim3(TW, TH), 0, s, jobs, \
                       n_jobs, total_tiles, uniform_tiles)
    FB_TILE_SWITCH(cfg, FB_GSEL)
#undef FB_GSEL
    return hipGetLastError();
}

hipError_t launch_guard_decide(const PMJob *jobs, int n_jobs, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_guard_decide, dim3((n_jobs + 63) / 64), dim3(64), 0, s, jobs, n_jobs);
    return hipGetLastError();
}

hipError_t launch_field_to_packed(const int32_t *abi, uint32_t *packed, int h, int w, hipStream_t s) {
    const int n = h * w;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_field_to_packed, dim3((n + 255) / 256), dim3(256), 0, s, abi, packed, h, w);
    return hipGetLastError();
}

}  // namespace fb
