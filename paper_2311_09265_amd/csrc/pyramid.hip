// Image pyramid and frame-packing kernels (Algorithm 1, "resize images S, T"
// at every level).
//
// Reading of the paper's unspecified resize: 2x2 box filter with round-half-up,
// ceil(h/2) x ceil(w/2) output, source reads clamped to the image.
//
// Every level, and every style frame, is stored as 4-byte (R, G, B, 0) pixels
// with a replicated border of p pixels on every side, so that the patch and
// remap kernels never clamp and each pixel is one aligned 4-byte word.
//
// All kernels stream through HBM once per frame and level; they are a
// negligible share of a blend (one pyramid per frame, shared by every pair
// that uses the frame).
#include "fb_common.h"

namespace fb {

namespace {
__device__ __forceinline__ int clampi(int x, int lo, int hi) { return min(max(x, lo), hi); }

int padded_pitch(int w, int p) { return (w + 2 * p + kPitchAlign - 1) / kPitchAlign * kPitchAlign; }
}  // namespace

PyrLayout pyr_layout(int h, int w, int levels, int p) {
    PyrLayout L{};
    L.levels = levels;
    L.p = p;
    size_t off = 0;
    for (int l = 0; l < levels; ++l) {
        LevelGeom &g = L.lv[l];
        g.h = ceil_half_pow(h, l);
        g.w = ceil_half_pow(w, l);
        g.rows = g.h + 2 * p;
        g.pitch = padded_pitch(g.w, p);
        g.px_off = off;
        off += (size_t)g.rows * g.pitch * 4;
        off = (off + 255) & ~(size_t)255;
        // the level's bound table follows its pixels, so the first l levels
        // of a deeper pyramid have the layout of an l-level one
        int sh = kBoundTabMinShift;
        while ((size_t)((g.h + (1 << sh) - 1) >> sh) * (size_t)((g.w + (1 << sh) - 1) >> sh) * 12 >
               (size_t)kBoundTabBytes)
            ++sh;
        g.tab_shift = sh;
        g.tab_h = (g.h + (1 << sh) - 1) >> sh;
        g.tab_w = (g.w + (1 << sh) - 1) >> sh;
        g.tab_off = off;
        off += (size_t)g.tab_h * g.tab_w * 12;
        off = (off + 255) & ~(size_t)255;
        g.sum_off = off;
        off += (size_t)g.h * g.pitch * 4;
        off = (off + 255) & ~(size_t)255;
    }
    L.bytes = off;
    return L;
}

size_t padded_image_bytes(int h, int w, int p, int32_t *pitch_out) {
    const int pitch = padded_pitch(w, p);
    if (pitch_out) *pitch_out = pitch;
    return (((size_t)(h + 2 * p) * pitch * 4) + 255) & ~(size_t)255;
}

namespace {

// RGB8 rows of h x w -> padded (R,G,B,0) pixels; one thread per padded pixel.
__global__ void __launch_bounds__(256)
k_pack_rgbx(const FrameRef *__restrict__ frames, FrameRef single, int h, int w, int p,
            uint8_t *__restrict__ dst, size_t dst_stride, size_t px_off, int pitch) {
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    const int R = blockIdx.y;
    const int f = blockIdx.z;
    if (C >= w + 2 * p) return;
    const FrameRef fr = frames ? frames[f] : single;
    const int r = clampi(R - p, 0, h - 1), c = clampi(C - p, 0, w - 1);
    const uint8_t *s = fr.rgb + (size_t)r * (size_t)fr.row_stride + (size_t)c * 3;
    const uint32_t px = (uint32_t)s[0] | ((uint32_t)s[1] << 8) | ((uint32_t)s[2] << 16);
    uint32_t *d = reinterpret_cast<uint32_t *>(dst + (size_t)f * dst_stride + px_off);
    d[(size_t)R * pitch + C] = px;
}

// Padded level l -> padded level l+1 (2x2 box, round half up, clamped reads).
__global__ void __launch_bounds__(256)
k_downsample(uint8_t *__restrict__ base, size_t stride, int hi_, int wi, int pitch_i, size_t off_i,
             int ho, int wo, int pitch_o, size_t off_o, int p) {
    const int C = blockIdx.x * blockDim.x + threadIdx.x;
    const int R = blockIdx.y;
    const int f = blockIdx.z;
    if (C >= wo + 2 * p) return;
    uint8_t *fb = base + (size_t)f * stride;
    const uint32_t *in = reinterpret_cast<const uint32_t *>(fb + off_i);
    uint32_t *out = reinterpret_cast<uint32_t *>(fb + off_o);
    const int r = clampi(R - p, 0, ho - 1), c = clampi(C - p, 0, wo - 1);
    uint32_t rb = 0, g = 0;  // R and B sums in 16-bit halves; G alone
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int rr = min(2 * r + a, hi_ - 1) + p, cc = min(2 * c + b, wi - 1) + p;
            const uint32_t px = in[(size_t)rr * pitch_i + cc];
            rb += px & 0x00FF00FFu;
            g += (px >> 8) & 0xFFu;
        }
    const uint32_t vr = ((rb & 0xFFFFu) + 2) >> 2, vb = ((rb >> 16) + 2) >> 2, vg = (g + 2) >> 2;
    out[(size_t)R * pitch_o + C] = vr | (vg << 8) | (vb << 16);
}

// Bound table of one level: one wave per block of 2^sh x 2^sh patch
// positions.  Every position's (2p+1)^2 per-channel patch sum is taken from
// the padded level (so it sums the clamped patch the loss compares), and the
// block keeps each channel's minimum and maximum.  By Cauchy-Schwarz,
// (sum_k d_k)^2 <= (2p+1)^2 sum_k d_k^2 for the channel differences d_k of
// two patches, so the distance from a target patch's channel sums to these
// ranges bounds Eq. 1 from below for every candidate in the block.  Sums are
// at most 81 * 255, so each value and its negation fit 16 bits.  Every
// position's sums also go, quantised to 10 bits each, into the level's
// patch-sum plane, which gives the same bound per candidate.
__global__ void __launch_bounds__(64)
k_bound_table(uint8_t *__restrict__ base, size_t stride, int h, int w, int pitch, size_t px_off,
              int sh, int tab_w, int tab_n, size_t tab_off, size_t sum_off, int qs, int p) {
    const int f = blockIdx.y;
    const int by = (int)blockIdx.x / tab_w, bx = (int)blockIdx.x - by * tab_w;
    const uint8_t *fb = base + (size_t)f * stride;
    const uint32_t *img = reinterpret_cast<const uint32_t *>(fb + px_off);
    const int side = 1 << sh, k = 2 * p + 1;
    int mn0 = 1 << 30, mn1 = 1 << 30, mn2 = 1 << 30, mx0 = 0, mx1 = 0, mx2 = 0;
    for (int i = (int)threadIdx.x; i < side * side; i += 64) {
        const int r = (by << sh) + (i >> sh), c = (bx << sh) + (i & (side - 1));
        if (r >= h || c >= w) continue;
        uint32_t rb = 0, g = 0;  // R and B sums in 16-bit halves; G alone
        for (int dr = 0; dr < k; ++dr)
            for (int dc = 0; dc < k; ++dc) {
                const uint32_t px = img[(size_t)(r + dr) * pitch + c + dc];
                rb += px & 0x00FF00FFu;
                g += (px >> 8) & 0xFFu;
            }
        const int s0 = (int)(rb & 0xFFFFu), s1 = (int)g, s2 = (int)(rb >> 16);
        reinterpret_cast<uint32_t *>(base + (size_t)f * stride + sum_off)[(size_t)r * pitch + c] =
            (uint32_t)(s0 >> qs) | ((uint32_t)(s1 >> qs) << 10) | ((uint32_t)(s2 >> qs) << 20);
        mn0 = min(mn0, s0); mx0 = max(mx0, s0);
        mn1 = min(mn1, s1); mx1 = max(mx1, s1);
        mn2 = min(mn2, s2); mx2 = max(mx2, s2);
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        mn0 = min(mn0, __shfl_xor(mn0, m)); mx0 = max(mx0, __shfl_xor(mx0, m));
        mn1 = min(mn1, __shfl_xor(mn1, m)); mx1 = max(mx1, __shfl_xor(mx1, m));
        mn2 = min(mn2, __shfl_xor(mn2, m)); mx2 = max(mx2, __shfl_xor(mx2, m));
    }
    if (threadIdx.x == 0) {
        auto pair16 = [](int lo, int hi) { return ((uint32_t)lo & 0xFFFFu) | ((uint32_t)hi << 16); };
        uint32_t *t = reinterpret_cast<uint32_t *>(base + (size_t)f * stride + tab_off);
        t[blockIdx.x] = pair16(mn0, mn1);
        t[tab_n + blockIdx.x] = pair16(mn2, -mx0);
        t[2 * tab_n + blockIdx.x] = pair16(-mx1, -mx2);
    }
}

}  // namespace

hipError_t launch_bound_tables(uint8_t *base, size_t stride, int n, const PyrLayout &L, hipStream_t s) {
    for (int l = 0; l < L.levels; ++l) {
        const LevelGeom &g = L.lv[l];
        hipLaunchKernelGGL(k_bound_table, dim3(g.tab_w * g.tab_h, n), dim3(64), 0, s, base, stride,
                           g.h, g.w, g.pitch, g.px_off, g.tab_shift, g.tab_w, g.tab_w * g.tab_h, g.tab_off,
                           g.sum_off, psum_shift(L.p), L.p);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pack_rgbx(const FrameRef *frames, FrameRef single, int n, int h, int w, int p,
                            uint8_t *dst, size_t dst_stride, size_t px_off, int pitch,
                            hipStream_t s) {
    dim3 grid((w + 2 * p + 255) / 256, h + 2 * p, n);
    hipLaunchKernelGGL(k_pack_rgbx, grid, dim3(256), 0, s, frames, single, h, w, p, dst,
                       dst_stride, px_off, pitch);
    return hipGetLastError();
}

hipError_t launch_downsample(const uint8_t *base, size_t stride, int n, const LevelGeom &in,
                             const LevelGeom &out, int p, hipStream_t s) {
    dim3 grid((out.w + 2 * p + 255) / 256, out.rows, n);
    hipLaunchKernelGGL(k_downsample, grid, dim3(256), 0, s, const_cast<uint8_t *>(base), stride,
                       in.h, in.w, in.pitch, in.px_off, out.h, out.w, out.pitch, out.px_off, p);
    return hipGetLastError();
}

}  // namespace fb
