// Remapping and blending kernel (Algorithm 2, Eq. 2 and Eq. 9 of arXiv 2311.09265).
//
// out(v) = (sum over terms k of weight_k * R_k(v)) / divisor, where a term is
// either a style frame remapped through an NNF F,
//   R(v) = sum_{d in [-p,p]^2, v+d inside} S(F(v+d) - d) / (255 * count_v)
// (Algorithm 2 computed per output pixel, no patch materialisation; at the
// border only the in-image neighbours count, i.e. the patch-overlap average of
// Section 3.3), or the frame itself, R(v) = S(v) / 255.  The window blend of
// Eq. 2 is one output frame with 2M+1 (truncated) unit-weight terms and
// divisor = their count; the keyframe combination of Eq. 9 has two terms
// with weights (r-i)/(r-l), (i-l)/(r-l) and divisor 1.
//
// One thread per output pixel of one output frame; a workgroup is a tile of
// one frame.  Per remapped term the workgroup stages the tile's NNF entries
// with a p-pixel border in LDS (one coalesced pass), so each thread reads its
// (2p+1)^2 field entries from LDS, then gathers as many 4-byte style pixels
// from the padded frame (so F(v+d) - d needs no clamp) through global
// address space with 32-bit offsets.  Channel sums are integers (R and B in
// the two halves of one register, G in another); each term costs one fp32
// division per channel.  HBM traffic per output frame: its fields and style
// frames once (L2-resident gathers) plus 12 B per output pixel.
#include "fb_common.h"

namespace fb {

namespace {

constexpr int kRTW = 32, kRTH = 8;

// 16-byte float pixels are loaded as a vector type (address-space casts do
// not copy structs)
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T gload(const void *base, uint32_t byte_off) {
    return *(const __attribute__((address_space(1))) T *)((const __attribute__((address_space(1))) char *)base +
                                                          byte_off);
}

// a 16-byte float pixel of an h x w image: its byte offset needs 64 bits
// once h * w reaches 2^28 (the 4-byte images stay below 2^31 bytes)
__device__ __forceinline__ f32x4 gload_f4(const void *base, int pixel) {
    return *((const __attribute__((address_space(1))) f32x4 *)base + (size_t)(uint32_t)pixel);
}

template <int P>
__global__ void __launch_bounds__(kRTW *kRTH)
k_remap_sum(const RemapFrame *__restrict__ frames, const RemapTerm *__restrict__ terms, int h,
            int w, int pitch, int tiles_x) {
    constexpr int SW = kRTW + 2 * P, SH = kRTH + 2 * P;
    __shared__ uint32_t sf[SH * SW];  // the tile's field entries with a P-pixel border
    const RemapFrame fr = frames[blockIdx.y];
    const int ty = (int)blockIdx.x / tiles_x, tx = (int)blockIdx.x - ty * tiles_x;
    const int rt = ty * kRTH, ct = tx * kRTW;
    const int r = rt + (int)threadIdx.y, c = ct + (int)threadIdx.x;
    const int tid = (int)threadIdx.y * kRTW + (int)threadIdx.x;
    const bool active = r < h && c < w;  // no early exit: the term loop has barriers
    const int r0 = max(-P, -r), r1 = min(P, h - 1 - r);
    const int c0 = max(-P, -c), c1 = min(P, w - 1 - c);
    const int cnt_v = (r1 - r0 + 1) * (c1 - c0 + 1);
    const float denom = (float)(255 * cnt_v);
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    uint32_t n0 = 0, n1 = 0, n2 = 0;  // out_kind 2: exact integer totals (style terms, weight 1)
    for (int k = 0; k < fr.n_terms; ++k) {
        const RemapTerm T = terms[fr.term_base + k];
        const uint32_t *sp = T.style_px;
        const bool flt = T.kind == kRemapFloat;
        if (T.f == nullptr) {
            if (active) {
                if (flt) {
                    const f32x4 x = gload_f4(sp, r * w + c);
                    a0 += T.weight * x.x;
                    a1 += T.weight * x.y;
                    a2 += T.weight * x.z;
                } else {
                    const uint32_t px = gload<uint32_t>(sp, 4u * (uint32_t)((r + P) * pitch + (c + P)));
                    a0 += T.weight * ((float)(px & 0xFFu) / 255.0f);
                    a1 += T.weight * ((float)((px >> 8) & 0xFFu) / 255.0f);
                    a2 += T.weight * ((float)((px >> 16) & 0xFFu) / 255.0f);
                    n0 += (uint32_t)cnt_v * (px & 0xFFu);
                    n1 += (uint32_t)cnt_v * ((px >> 8) & 0xFFu);
                    n2 += (uint32_t)cnt_v * ((px >> 16) & 0xFFu);
                }
            }
            continue;
        }
        __syncthreads();  // the previous term's field entries have been read
        for (int i = tid; i < SH * SW; i += kRTW * kRTH) {
            const int yy = rt - P + i / SW, xx = ct - P + i % SW;
            sf[i] = (yy >= 0 && yy < h && xx >= 0 && xx < w) ? gload<uint32_t>(T.f, 4u * (uint32_t)(yy * w + xx)) : 0u;
        }
        __syncthreads();
        if (flt) {
            if (!active) continue;
            float x0 = 0.f, x1 = 0.f, x2 = 0.f;
#pragma unroll
            for (int dr = -P; dr <= P; ++dr) {
                if (dr < r0 || dr > r1) continue;
                const uint32_t *srow = sf + ((int)threadIdx.y + P + dr) * SW + (int)threadIdx.x + P;
#pragma unroll
                for (int dc = -P; dc <= P; ++dc) {
                    if (dc < c0 || dc > c1) continue;
                    const uint32_t q = srow[dc];
                    const int sr = min(max((int)(q >> 16) - dr, 0), h - 1);
                    const int sc = min(max((int)(q & 0xFFFFu) - dc, 0), w - 1);
                    const f32x4 x = gload_f4(sp, sr * w + sc);
                    x0 += x.x;
                    x1 += x.y;
                    x2 += x.z;
                }
            }
            const float cnt = (float)((r1 - r0 + 1) * (c1 - c0 + 1));
            a0 += T.weight * (x0 / cnt);
            a1 += T.weight * (x1 / cnt);
            a2 += T.weight * (x2 / cnt);
            continue;
        }
        uint32_t rb = 0, g = 0;
        // Where the field is one translation around v (F(v+d) - d = F(v) for
        // every in-image d), every term of the sum is S(F(v)), so a wave whose
        // pixels all qualify gathers once per pixel instead of (2p+1)^2 times.
        // The wave tests its whole staged neighbourhood at once (its rows with
        // the P-row border): when every in-image entry u there holds the same
        // translation F(u) - u, every pixel of the wave qualifies.  Packed as
        // (row << 16) + col, equal translations give equal differences and,
        // sides being below 2^15, different ones never do.
        const uint32_t q0 = sf[((int)threadIdx.y + P) * SW + (int)threadIdx.x + P];
        bool coherent = true;
        {
            constexpr int WR = 64 / kRTW;          // tile rows of one wave
            constexpr int RN = (WR + 2 * P) * SW;  // its staged neighbourhood
            const int wy0 = (tid >> 6) * WR;
            const uint64_t act = __ballot(active);
            const uint32_t own = q0 - (((uint32_t)r << 16) + (uint32_t)c);
            const uint32_t ref = (uint32_t)__shfl((int)own, act ? __ffsll((unsigned long long)act) - 1 : 0);
#pragma unroll
            for (int e = tid & 63; e < RN; e += 64) {
                const int ry = wy0 + e / SW, rx = e - (e / SW) * SW;
                const int yy = rt - P + ry, xx = ct - P + rx;
                if (yy >= 0 && yy < h && xx >= 0 && xx < w)
                    coherent &= sf[ry * SW + rx] - (((uint32_t)yy << 16) + (uint32_t)xx) == ref;
            }
        }
        const bool wave_coherent = __all(coherent);
        if (!active) continue;
        if (wave_coherent) {
            const int sr = (int)(q0 >> 16) + P, sc = (int)(q0 & 0xFFFFu) + P;
            const uint32_t px = gload<uint32_t>(sp, 4u * (uint32_t)(sr * pitch + sc));
            rb = (uint32_t)cnt_v * (px & 0x00FF00FFu);
            g = (uint32_t)cnt_v * ((px >> 8) & 0xFFu);
        } else {
#pragma unroll
            for (int dr = -P; dr <= P; ++dr) {
                if (dr < r0 || dr > r1) continue;
                const uint32_t *srow = sf + ((int)threadIdx.y + P + dr) * SW + (int)threadIdx.x + P;
#pragma unroll
                for (int dc = -P; dc <= P; ++dc) {
                    if (dc < c0 || dc > c1) continue;
                    const uint32_t q = srow[dc];
                    const int sr = (int)(q >> 16) - dr + P, sc = (int)(q & 0xFFFFu) - dc + P;
                    const uint32_t px = gload<uint32_t>(sp, 4u * (uint32_t)(sr * pitch + sc));
                    rb += px & 0x00FF00FFu;
                    g += (px >> 8) & 0xFFu;
                }
            }
        }
        a0 += T.weight * ((float)(rb & 0xFFFFu) / denom);
        a1 += T.weight * ((float)g / denom);
        a2 += T.weight * ((float)(rb >> 16) / denom);
        n0 += rb & 0xFFFFu;
        n1 += g;
        n2 += rb >> 16;
    }
    if (!active) return;
    if (fr.out_kind == 2) {
        // the exact mean of the terms (every term's remap at this pixel has
        // the same count cnt_v), rounded half up, as uint8 RGB
        const uint32_t den = (uint32_t)cnt_v * (uint32_t)fr.n_terms;
        uint8_t *o = reinterpret_cast<uint8_t *>(fr.out) + ((size_t)r * w + c) * 3;
        o[0] = (uint8_t)((2u * n0 + den) / (2u * den));
        o[1] = (uint8_t)((2u * n1 + den) / (2u * den));
        o[2] = (uint8_t)((2u * n2 + den) / (2u * den));
        return;
    }
    if (fr.out_kind == 1) {
        reinterpret_cast<float4 *>(fr.out)[(size_t)r * w + c] =
            make_float4(a0 / fr.divisor, a1 / fr.divisor, a2 / fr.divisor, 0.f);
        return;
    }
    float *o = fr.out + ((size_t)r * w + c) * 3;
    o[0] = a0 / fr.divisor;
    o[1] = a1 / fr.divisor;
    o[2] = a2 / fr.divisor;
}

}  // namespace

hipError_t launch_remap_sum(const RemapFrame *frames, int n_frames, const RemapTerm *terms, int h,
                            int w, int pitch, int p, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    const int tiles_x = (w + kRTW - 1) / kRTW, tiles_y = (h + kRTH - 1) / kRTH;
    dim3 grid(tiles_x * tiles_y, n_frames);
    dim3 block(kRTW, kRTH);
    switch (p) {
    case 1: hipLaunchKernelGGL(k_remap_sum<1>, grid, block, 0, s, frames, terms, h, w, pitch, tiles_x); break;
    case 2: hipLaunchKernelGGL(k_remap_sum<2>, grid, block, 0, s, frames, terms, h, w, pitch, tiles_x); break;
    case 3: hipLaunchKernelGGL(k_remap_sum<3>, grid, block, 0, s, frames, terms, h, w, pitch, tiles_x); break;
    case 4: hipLaunchKernelGGL(k_remap_sum<4>, grid, block, 0, s, frames, terms, h, w, pitch, tiles_x); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fb
