// Kernels of the learned proposal network (a small U-Net that predicts an
// initial offset field for PatchMatch).  The network is not part of the
// paper: FastBlend is model-free; this proposal only seeds the coarsest
// pyramid level of Algorithm 1, and plain PatchMatch stays the fallback.
//
// Tensors are NHWC with the channel count padded to a multiple of 16;
// activations and activation gradients are bf16, weights are bf16 copies of
// fp32 master weights, all products accumulate in fp32.
//
// 3x3 convolutions (padding 1, stride 1) are implicit GEMMs on the matrix
// cores: v_mfma_f32_16x16x16_bf16 with M = pixels, N = output channels,
// K = 9 taps x input channels in chunks of 16 channels of one tap.  The same
// kernel computes the data gradient with the flipped, transposed weights.
// Weight gradients are a second implicit GEMM with K = pixels, split into
// chunks whose partial sums a reduction kernel adds in a fixed order.
//
// Matrix-core lane layout of the 16x16x16 bf16 instruction (wave64):
//   A (16 x 16, M x K): lane l holds A[l % 16][4 (l / 16) + j], j = 0..3
//   B (16 x 16, K x N): lane l holds B[4 (l / 16) + j][l % 16]
//   D (16 x 16):        lane l holds D[4 (l / 16) + j][l % 16]
#include <algorithm>

#include "fb_common.h"

namespace fb {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// two floats to packed bf16 (low half: a), rounded to nearest even like f32_to_bf16
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    typedef float f32x2_t __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
    const bf16x2_t h = __builtin_convertvector((f32x2_t){a, b}, bf16x2_t);
    return __builtin_bit_cast(uint32_t, h);
}

__device__ __forceinline__ bf16x4 load_bf16x4(const uint16_t *p) {
    const uint2 u = *reinterpret_cast<const uint2 *>(p);
    bf16x4 r;
    r[0] = (short)(u.x & 0xFFFFu);
    r[1] = (short)(u.x >> 16);
    r[2] = (short)(u.y & 0xFFFFu);
    r[3] = (short)(u.y >> 16);
    return r;
}

// ---------------------------------------------------------------------------
// Forward / data-gradient convolution.  The B*H*W output pixels form one flat
// list; a workgroup (4 waves) takes 256 consecutive pixels, each wave 64 of
// them as 4 row blocks of 16 (M), times NB blocks of 16 output channels
// starting at blockIdx.y * 16 NB (N).  Every 16-channel slice of one tap
// (K) costs each wave 4 + NB fragment loads of 8 bytes per lane for 4 NB
// matrix-core instructions.
// ---------------------------------------------------------------------------
template <int NB, bool RELU, bool OUT_F32>
__global__ void __launch_bounds__(256)
k_conv3x3(const uint16_t *__restrict__ in, int B, int H, int W, int cin,
          const uint16_t *__restrict__ wt, const float *__restrict__ bias, void *__restrict__ out,
          int cout, int ostride) {
    constexpr int MB = 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long total = (long)B * H * W;
    const long p_wave = (long)blockIdx.x * 256 + wave * 64;
    const int co0 = blockIdx.y * 16 * NB;
    const int kq = 4 * (lane >> 4);
    // the pixel whose A row this lane loads, per row block
    int py[MB], px[MB];
    long pn[MB];
    bool pv[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const long p = p_wave + mb * 16 + (lane & 15);
        pv[mb] = p < total;
        const long q = pv[mb] ? p : 0;
        px[mb] = (int)(q % W);
        py[mb] = (int)((q / W) % H);
        pn[mb] = q / ((long)W * H);
    }
    f32x4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[mb][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const uint16_t *arow[MB];
        bool ok[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int yy = py[mb] + dy, xx = px[mb] + dx;
            ok[mb] = pv[mb] && yy >= 0 && yy < H && xx >= 0 && xx < W;
            arow[mb] = in + ((pn[mb] * H + (ok[mb] ? yy : 0)) * W + (ok[mb] ? xx : 0)) * cin + kq;
        }
        const uint16_t *wrow = wt + ((size_t)tap * cout + co0 + (lane & 15)) * cin + kq;
        for (int c0 = 0; c0 < cin; c0 += 16) {
            bf16x4 a[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) a[mb] = ok[mb] ? load_bf16x4(arow[mb] + c0) : bf16x4{0, 0, 0, 0};
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const bf16x4 bw = load_bf16x4(wrow + (size_t)16 * b * cin + c0);
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mb], bw, acc[mb][b], 0, 0, 0);
            }
        }
    }
    // epilogue: lane holds D[4 (lane/16) + j][lane % 16]: pixel row, channel column
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int co = co0 + 16 * b + (lane & 15);
        if (co >= ostride) continue;
        const float bv = bias ? bias[co] : 0.f;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const long p = p_wave + mb * 16 + 4 * (lane >> 4) + j;
                if (p >= total) continue;
                float v = acc[mb][b][j] + bv;
                if (RELU) v = fmaxf(v, 0.f);
                const size_t o = (size_t)p * ostride + co;
                if (OUT_F32) reinterpret_cast<float *>(out)[o] = v;
                else reinterpret_cast<uint16_t *>(out)[o] = f32_to_bf16(v);
            }
    }
}

// ---------------------------------------------------------------------------
// Forward / data-gradient convolution on v_mfma_f32_32x32x16_bf16, staged
// through LDS.  A workgroup takes kConvTile consecutive pixels of one image
// (4 waves x 2 blocks of 32 pixels) and 32 NBW output channels; a matrix-core
// instruction multiplies 32 output channels' weights (A, M) by 32 pixels (B,
// N), so each lane ends up with 16 channels of one pixel.
// For every 16-channel slice of the input (K) it stages in LDS the input rows
// the tile touches, with a zero border (the halo), and the slice's weights of
// all 9 taps; every tap then reads its A and B fragments from LDS, so each
// input element is fetched from memory once per slice instead of once per
// tap.  Input channels [0, ca) may come from a half-resolution tensor
// upsampled 2x (nearest): the decoder's upsample-and-concatenate is read in
// place instead of materialised.
//
// LDS holds each staged 16-channel row as two planes of 8 channels (16 B), so
// the 32 lanes that read one fragment half read 32 consecutive 16-byte words
// (no bank conflicts).  The results go back through LDS too: each 32-channel
// block of the tile is written there as bf16 (8 bytes per lane and store) and
// copied out with 16-byte stores; with POOL the same copy also writes the
// tile's 2x2 average pooling (the tile then covers whole row pairs).  Tiles
// are assigned XCD by XCD (xcd_item), so the halo rows two neighbouring tiles
// share are read from memory once.
//
// 32x32x16 bf16 lane layout (wave64):
//   A (32 x 16): lane l holds A[l % 32][8 (l / 32) + j], j = 0..7
//   B (16 x 32): lane l holds B[8 (l / 32) + j][l % 32]
//   D (32 x 32): lane l holds D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32], i = 0..15
// With A = weights [output channel][input channel] and B = pixels [input
// channel][pixel], the two operands are the same 16-byte LDS words a lane
// would load for the pixel-major product, and each output value is the same
// sum of the same products.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 u) {
    union {
        uint4 u;
        bf16x8 b;
    } c;
    c.u = u;
    return c.b;
}

// Consecutive workgroups are dispatched round-robin over the 8 XCDs.  Give
// each XCD one contiguous range of the launch's work items, so tiles that
// share halo rows run on one XCD close in time and the shared rows are read
// from its L2 instead of from memory twice.  A bijection on [0, total).
__device__ __forceinline__ int xcd_item(int b, int total) {
    const int q = total >> 3, r = total & 7;
    const int x = b & 7, s = b >> 3;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

// floor(n / d) for 0 <= n < 2^24 and 0 < d < 2^24: a float estimate from the
// reciprocal, corrected by one step either way (the estimate is within one)
__device__ __forceinline__ int div_small(int n, int d, float rd) {
    int q = (int)((float)n * rd);
    const int r = n - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

// bf16 pixel stride of the output tile in LDS: 16 bytes of padding put the
// two pixels one store instruction writes (4 apart) on different banks
constexpr int kConvOutStride = 32 + 8;

template <int NBW, int HE, bool RELU, bool POOL>
__global__ void __launch_bounds__(256)
k_conv3x3_lds(ConvIn X, int H, int W, int cin, int tiles_per_img, const uint16_t *__restrict__ wt,
              const float *__restrict__ bias, uint16_t *__restrict__ out, int cout,
              uint16_t *__restrict__ pool_out) {
    // HE: halo pixels staged per thread (the halo has at most 256 HE pixels)
    constexpr int NT = 32 * NBW;
    constexpr int WE = (9 * NT + 255) / 256;  // weight rows staged per thread
    extern __shared__ uint4 lds[];
    uint4 *s_w = lds;               // [2][9][NT]: channel halves of one weight row
    uint4 *s_in = lds + 9 * NT * 2; // [2][halo pixels]: channel halves of one pixel
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // work item: tile-major, the output-channel blocks of one tile adjacent
    const int item = xcd_item((int)(blockIdx.y * gridDim.x + blockIdx.x), (int)(gridDim.x * gridDim.y));
    const int tile = item / (int)gridDim.y, cblk0 = item - tile * (int)gridDim.y;
    const int img = tile / tiles_per_img;
    const int HW = H * W, WP = W + 2;
    const int p0 = (tile - img * tiles_per_img) * kConvTile;
    const int p1 = min(p0 + kConvTile, HW);
    const int ya = p0 / W - 1;                           // first halo row
    const int halo = ((p1 - 1) / W + 1 - ya + 1) * WP;  // <= 256 HE (checked by the host)
    const int co0 = cblk0 * NT;
    const int half = lane >> 5;
    const int cb = cin - X.ca;

    // what this thread stages: halo pixels tid + 256 k (source pixel index in
    // a and in b, or -1 for the zero border) and weight rows tid + 256 k
    const float rWP = 1.0f / (float)WP, rW = 1.0f / (float)W;
    int src_a[HE], src_b[HE];
#pragma unroll
    for (int k = 0; k < HE; ++k) {
        const int i = tid + 256 * k;
        src_a[k] = src_b[k] = -1;
        if (i < halo) {
            const int hy = div_small(i, WP, rWP), hx = i - hy * WP;
            const int y = ya + hy, x = hx - 1;
            if (y >= 0 && y < H && x >= 0 && x < W) {
                src_b[k] = (img * H + y) * W + x;
                src_a[k] = X.a_half ? (img * (H >> 1) + (y >> 1)) * (W >> 1) + (x >> 1) : src_b[k];
            }
        }
    }
    int w_row[WE];
#pragma unroll
    for (int k = 0; k < WE; ++k) {
        const int i = tid + 256 * k;
        const int tap = i / NT, co = co0 + (i - tap * NT);
        w_row[k] = (i < 9 * NT && co < cout) ? tap * cout + co : -1;
    }
    uint4 r_in[HE][2], r_w[WE][2];
    auto fetch = [&](int c0) {
        const bool in_a = c0 < X.ca;
        const uint16_t *base = in_a ? X.a + c0 : X.b + (c0 - X.ca);
        const int stride = in_a ? X.ca : cb;
#pragma unroll
        for (int k = 0; k < HE; ++k) {
            const int sp = in_a ? src_a[k] : src_b[k];
            r_in[k][0] = r_in[k][1] = make_uint4(0, 0, 0, 0);
            if (sp >= 0) {
                const uint4 *q = reinterpret_cast<const uint4 *>(base + (size_t)sp * stride);
                r_in[k][0] = q[0];
                r_in[k][1] = q[1];
            }
        }
#pragma unroll
        for (int k = 0; k < WE; ++k) {
            r_w[k][0] = r_w[k][1] = make_uint4(0, 0, 0, 0);
            if (w_row[k] >= 0) {
                const uint4 *q = reinterpret_cast<const uint4 *>(wt + (size_t)w_row[k] * cin + c0);
                r_w[k][0] = q[0];
                r_w[k][1] = q[1];
            }
        }
    };

    int hidx[2];  // halo index of this lane's pixel in each of its row blocks
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        const int p = min(p0 + 64 * wave + 32 * mb + (lane & 31), p1 - 1);
        const int y = div_small(p, W, rW);
        hidx[mb] = (y - ya) * WP + (p - y * W) + 1;
    }
    f32x16 acc[2][NBW];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[mb][nb][i] = 0.f;

    const uint4 *a_plane = s_in + half * halo;
    const uint4 *b_plane = s_w + half * 9 * NT;
    fetch(0);
    for (int c0 = 0; c0 < cin; c0 += 16) {
        __syncthreads();  // the previous slice's fragments have been read
#pragma unroll
        for (int k = 0; k < HE; ++k) {
            const int i = tid + 256 * k;
            if (i < halo) {
                s_in[i] = r_in[k][0];
                s_in[halo + i] = r_in[k][1];
            }
        }
#pragma unroll
        for (int k = 0; k < WE; ++k) {
            const int i = tid + 256 * k;
            if (i < 9 * NT) {
                s_w[i] = r_w[k][0];
                s_w[9 * NT + i] = r_w[k][1];
            }
        }
        __syncthreads();
        if (c0 + 16 < cin) fetch(c0 + 16);  // in flight while the matrix cores work
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int toff = (tap / 3 - 1) * WP + (tap % 3 - 1);
            bf16x8 a[2], b[NBW];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) a[mb] = as_bf16x8(a_plane[hidx[mb] + toff]);
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) b[nb] = as_bf16x8(b_plane[tap * NT + 32 * nb + (lane & 31)]);
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb)
                    acc[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b[nb], a[mb], acc[mb][nb], 0, 0, 0);
        }
    }

    // epilogue, one 32-channel block at a time: bias, ReLU, bf16 into the LDS
    // tile [pixel][kConvOutStride], then 16-byte stores of whole pixels
    uint16_t *s_o = reinterpret_cast<uint16_t *>(lds);
    const int np = p1 - p0;
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
        const int cblk = co0 + 32 * nb;
        if (cblk >= cout) break;  // uniform
        const int nch = min(32, cout - cblk) >> 3;  // 8-channel chunks of the block that exist
        float bb[4][4];  // bias of the 16 channels this lane holds
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int c = cblk + 8 * g + 4 * half;
            const float4 b4 = bias && c < cout ? *reinterpret_cast<const float4 *>(bias + c) : make_float4(0.f, 0.f, 0.f, 0.f);
            bb[g][0] = b4.x;
            bb[g][1] = b4.y;
            bb[g][2] = b4.z;
            bb[g][3] = b4.w;
        }
        __syncthreads();  // the fragments (or the previous block) have been read
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int pl = 64 * wave + 32 * mb + (lane & 31);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                // channels cblk + 8 g + 4 half + j, j = 0..3, of pixel pl
                const int c4 = 8 * g + 4 * half;
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    v[j] = acc[mb][nb][4 * g + j] + bb[g][j];
                    if (RELU) v[j] = fmaxf(v[j], 0.f);
                }
                *reinterpret_cast<uint2 *>(s_o + pl * kConvOutStride + c4) =
                    make_uint2(pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3]));
            }
        }
        __syncthreads();
        // 4 chunks of 8 channels per pixel, the block's 32 channels of 256 pixels
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = tid + 256 * k, pl = c >> 2, part = c & 3;
            if (pl < np && part < nch)
                *reinterpret_cast<uint4 *>(out + ((size_t)img * HW + p0 + pl) * cout + cblk + 8 * part) =
                    *reinterpret_cast<const uint4 *>(s_o + pl * kConvOutStride + 8 * part);
        }
        if (POOL) {
            // the tile is rows [p0 / W, p1 / W) of even count starting even:
            // np / 4 pooled pixels x 4 chunks of 8 channels
            const int Wo = W >> 1;
            const int q = tid >> 2, part = tid & 3;
            if (tid < np && part < nch) {
                const int qy = q / Wo, qx = q - qy * Wo;
                const int l00 = 2 * qy * W + 2 * qx;
                const uint16_t *r0 = s_o + l00 * kConvOutStride + 8 * part;
                const uint16_t *r1 = r0 + W * kConvOutStride;
                const uint4 u00 = *reinterpret_cast<const uint4 *>(r0);
                const uint4 u01 = *reinterpret_cast<const uint4 *>(r0 + kConvOutStride);
                const uint4 u10 = *reinterpret_cast<const uint4 *>(r1);
                const uint4 u11 = *reinterpret_cast<const uint4 *>(r1 + kConvOutStride);
                const uint32_t *w00 = &u00.x, *w01 = &u01.x, *w10 = &u10.x, *w11 = &u11.x;
                uint32_t o[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    uint32_t r = 0;
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int sh = 16 * h2;
                        // the sum in the order of the separate pooling kernel
                        const float sum = bf16_to_f32((uint16_t)(w00[j] >> sh)) + bf16_to_f32((uint16_t)(w01[j] >> sh)) +
                                          bf16_to_f32((uint16_t)(w10[j] >> sh)) + bf16_to_f32((uint16_t)(w11[j] >> sh));
                        r |= (uint32_t)f32_to_bf16(0.25f * sum) << sh;
                    }
                    o[j] = r;
                }
                const int py = p0 / W / 2 + qy;
                *reinterpret_cast<uint4 *>(pool_out + (((size_t)img * (H >> 1) + py) * Wo + qx) * cout + cblk +
                                           8 * part) = make_uint4(o[0], o[1], o[2], o[3]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Offset head: 3x3 convolution from 32 bf16 channels to the 2 offset channels,
// fp32 out [px][2].  v_mfma_f32_16x16x32_bf16 covers all 32 input channels of
// one tap for 16 pixels (M) and 16 output channels (N, the first 2 real), so
// a tap is one matrix-core instruction per 16 pixels.  The tile's input rows
// with a zero border are staged in LDS once (all 32 channels, as four planes
// of 8 channels, so the 16 lanes of one fragment quarter read consecutive
// 16-byte words); the weights of all taps stay in registers.
//
// 16x16x32 bf16 lane layout (wave64):
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + j], j = 0..7
//   B (32 x 16): lane l holds B[8 (l / 16) + j][l % 16]
//   D (16 x 16): lane l holds D[4 (l / 16) + j][l % 16], j = 0..3
// ---------------------------------------------------------------------------
template <int HE>  // halo pixels staged per thread (the halo has at most 256 HE pixels)
__global__ void __launch_bounds__(256)
k_head3x3(const uint16_t *__restrict__ in, int H, int W, int tiles_per_img, const uint16_t *__restrict__ wt,
          int cout_pad, const float *__restrict__ bias, float *__restrict__ out) {
    constexpr int CIN = 32;
    extern __shared__ uint4 lds[];  // [4][halo pixels]: the four 8-channel quarters of a pixel
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = xcd_item((int)blockIdx.x, (int)gridDim.x);
    const int img = tile / tiles_per_img;
    const int HW = H * W, WP = W + 2;
    const int p0 = (tile - img * tiles_per_img) * kConvTile;
    const int p1 = min(p0 + kConvTile, HW);
    const int ya = p0 / W - 1;
    const int halo = ((p1 - 1) / W + 1 - ya + 1) * WP;
    // all loads first, then all LDS stores
    uint4 v[HE][4];
#pragma unroll
    for (int k = 0; k < HE; ++k) {
        const int i = tid + 256 * k;
        const int hy = i / WP, hx = i - hy * WP;
        const int y = ya + hy, x = hx - 1;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[k][j] = make_uint4(0, 0, 0, 0);
        if (i < halo && y >= 0 && y < H && x >= 0 && x < W) {
            const uint4 *q = reinterpret_cast<const uint4 *>(in + (((size_t)img * H + y) * W + x) * CIN);
#pragma unroll
            for (int j = 0; j < 4; ++j) v[k][j] = q[j];
        }
    }
    // B fragments of all taps: output channel lane % 16, input channels 8 (lane / 16) + j
    bf16x8 b[9];
    const int co = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
        b[tap] = as_bf16x8(*reinterpret_cast<const uint4 *>(wt + ((size_t)tap * cout_pad + co) * CIN + 8 * kq));
#pragma unroll
    for (int k = 0; k < HE; ++k) {
        const int i = tid + 256 * k;
        if (i < halo) {
#pragma unroll
            for (int j = 0; j < 4; ++j) lds[j * halo + i] = v[k][j];
        }
    }
    __syncthreads();
    // each wave: 4 blocks of 16 pixels, their tap chains interleaved
    int hc[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        const int pa = min(p0 + 64 * wave + 16 * mb + (lane & 15), p1 - 1);  // this lane's A row
        const int y = pa / W;
        hc[mb] = (y - ya) * WP + (pa - y * W) + 1;
    }
    f32x4 acc[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int toff = (tap / 3 - 1) * WP + (tap % 3 - 1);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(lds[kq * halo + hc[mb] + toff]), b[tap],
                                                              acc[mb], 0, 0, 0);
    }
    if (co < 2) {
        const float bv = bias[co];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = p0 + 64 * wave + 16 * mb + 4 * kq + j;
                if (p < p1) out[((size_t)img * HW + p) * 2 + co] = acc[mb][j] + bv;
            }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: partial[chunk][tap][co][ci] = sum over the chunk's pixels of
// g[p][co] * in[p shifted by the tap][ci].  One wave per (chunk, tap, 16x16
// block of (co, ci)); A = g^T (co x pixels), B = shifted input (pixels x ci).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64)
k_conv_wgrad(const uint16_t *__restrict__ in, const uint16_t *__restrict__ g, int B, int H, int W,
             int cin, int cout, int chunk_px, float *__restrict__ partial) {
    const int lane = threadIdx.x;
    const int chunk = blockIdx.x, tap = blockIdx.y;
    const int ci_blocks = cin / 16;
    const int cb = blockIdx.z % ci_blocks, ob = blockIdx.z / ci_blocks;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const long total = (long)B * H * W;
    const long p0 = (long)chunk * chunk_px;
    const int co = ob * 16 + (lane & 15), ci = cb * 16 + (lane & 15);
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < chunk_px; k0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long p = p0 + k0 + 4 * (lane >> 4) + j;
            short av = 0, bv = 0;
            if (p < total) {
                av = (short)g[p * cout + co];
                const int x = (int)(p % W), yq = (int)((p / W) % H);
                const int yy = yq + dy, xx = x + dx;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W) bv = (short)in[(p + (long)dy * W + dx) * cin + ci];
            }
            a[j] = av;
            b[j] = bv;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    // D[4 (lane/16) + j][lane % 16]: rows = co, columns = ci
    float *dst = partial + (((size_t)chunk * 9 + tap) * cout) * cin;
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[(size_t)(ob * 16 + 4 * (lane >> 4) + j) * cin + ci] = acc[j];
}

// bias gradient partial sums: partial[chunk][co] = sum of g[p][co] over the chunk
__global__ void __launch_bounds__(256)
k_bias_grad(const uint16_t *__restrict__ g, long total, int cout, int chunk_px, float *__restrict__ partial) {
    const int chunk = blockIdx.x;
    for (int co = threadIdx.x; co < cout; co += blockDim.x) {
        float s = 0.f;
        const long p1 = min((long)(chunk + 1) * chunk_px, total);
        for (long p = (long)chunk * chunk_px; p < p1; ++p) s += bf16_to_f32(g[p * cout + co]);
        partial[(size_t)chunk * cout + co] = s;
    }
}

// out[i] = sum over chunks of partial[chunk][i], in chunk order
__global__ void __launch_bounds__(256)
k_reduce_chunks(const float *__restrict__ partial, int n_chunks, long n, float *__restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int c = 0; c < n_chunks; ++c) s += partial[(size_t)c * n + i];
    out[i] = s;
}

// 2x2 average pooling (even sizes), bf16
__global__ void __launch_bounds__(256)
k_pool2(const uint16_t *__restrict__ in, int B, int H, int W, int C, uint16_t *__restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2;
    if (i >= (long)B * Ho * Wo * C) return;
    const int c = (int)(i % C);
    long q = i / C;
    const int x = (int)(q % Wo);
    q /= Wo;
    const int y = (int)(q % Ho);
    const int n = (int)(q / Ho);
    const size_t base = (((size_t)n * H + 2 * y) * W + 2 * x) * C + c;
    const float s = bf16_to_f32(in[base]) + bf16_to_f32(in[base + C]) +
                    bf16_to_f32(in[base + (size_t)W * C]) + bf16_to_f32(in[base + (size_t)W * C + C]);
    out[i] = f32_to_bf16(0.25f * s);
}

// gradient of 2x2 average pooling, added to gin: gin[y][x] += gout[y/2][x/2] / 4
__global__ void __launch_bounds__(256)
k_pool2_bwd_add(const uint16_t *__restrict__ gout, int B, int H, int W, int C, uint16_t *__restrict__ gin) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)B * H * W * C) return;
    const int c = (int)(i % C);
    long q = i / C;
    const int x = (int)(q % W);
    q /= W;
    const int y = (int)(q % H);
    const int n = (int)(q / H);
    const float g = bf16_to_f32(gout[(((size_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c]);
    gin[i] = f32_to_bf16(bf16_to_f32(gin[i]) + 0.25f * g);
}

// concat(nearest 2x upsample of deep [H/2][W/2][C1], skip [H][W][C2]) -> [H][W][C1 + C2]
__global__ void __launch_bounds__(256)
k_upcat(const uint16_t *__restrict__ deep, const uint16_t *__restrict__ skip, int B, int H, int W,
        int C1, int C2, uint16_t *__restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int C = C1 + C2;
    if (i >= (long)B * H * W * C) return;
    const int c = (int)(i % C);
    long q = i / C;
    const int x = (int)(q % W);
    q /= W;
    const int y = (int)(q % H);
    const int n = (int)(q / H);
    out[i] = c < C1 ? deep[(((size_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * C1 + c]
                    : skip[(((size_t)n * H + y) * W + x) * C2 + (c - C1)];
}

// gradient of k_upcat: gdeep = sum of the 2x2 block of the first C1 channels
// (written), gskip = the other C2 channels (written)
__global__ void __launch_bounds__(256)
k_upcat_bwd(const uint16_t *__restrict__ gcat, int B, int H, int W, int C1, int C2,
            uint16_t *__restrict__ gdeep, uint16_t *__restrict__ gskip) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int C = C1 + C2;
    const long n_deep = (long)B * (H / 2) * (W / 2) * C1;
    const long n_skip = (long)B * H * W * C2;
    if (i < n_deep) {
        const int c = (int)(i % C1);
        long q = i / C1;
        const int x = (int)(q % (W / 2));
        q /= (W / 2);
        const int y = (int)(q % (H / 2));
        const int n = (int)(q / (H / 2));
        const size_t base = (((size_t)n * H + 2 * y) * W + 2 * x) * C + c;
        const float s = bf16_to_f32(gcat[base]) + bf16_to_f32(gcat[base + C]) +
                        bf16_to_f32(gcat[base + (size_t)W * C]) + bf16_to_f32(gcat[base + (size_t)W * C + C]);
        gdeep[i] = f32_to_bf16(s);
    } else if (i < n_deep + n_skip) {
        const long k = i - n_deep;
        const int c = (int)(k % C2);
        const long pix = k / C2;
        gskip[k] = gcat[pix * C + C1 + c];
    }
}

// g *= (y > 0): ReLU gradient through the post-activation output y
__global__ void __launch_bounds__(256)
k_relu_mask(uint16_t *__restrict__ g, const uint16_t *__restrict__ y, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!(bf16_to_f32(y[i]) > 0.f)) g[i] = 0;
}

// fp32 [n_px][6] in [0,1] -> bf16 [n_px][16]: 2x - 1 (centred), channels 6..15 zero
__global__ void __launch_bounds__(256)
k_input_from_f32(const float *__restrict__ x6, long n_px, uint16_t *__restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_px * 16) return;
    const int c = (int)(i % 16);
    out[i] = c < 6 ? f32_to_bf16(2.0f * x6[(i / 16) * 6 + c] - 1.0f) : (uint16_t)0;
}

// network input from the coarsest pyramid level of every pair: channels
// (source R,G,B, target R,G,B) / 255 at [H8][W8] (the level padded to a
// multiple of 8 by replicating its last row / column)
__global__ void __launch_bounds__(256)
k_input_from_pyramids(const UNetPairIn *__restrict__ pairs, int H8, int W8, uint16_t *__restrict__ out) {
    const int n = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= H8 * W8) return;
    const UNetPairIn P = pairs[n];
    const int y = min(i / W8, P.h - 1), x = min(i % W8, P.w - 1);
    const uint32_t s = P.src[(size_t)(y + P.pad) * P.pitch + x + P.pad];
    const uint32_t t = P.tgt[(size_t)(y + P.pad) * P.pitch + x + P.pad];
    uint16_t *o = out + ((size_t)n * H8 * W8 + i) * 16;
    // x = pixel / 255 (a correctly rounded fp32 division), centred to 2x - 1,
    // then bf16: the same steps as k_input_from_f32 on that x
    o[0] = f32_to_bf16(2.0f * ((float)(s & 0xFF) / 255.0f) - 1.0f);
    o[1] = f32_to_bf16(2.0f * ((float)((s >> 8) & 0xFF) / 255.0f) - 1.0f);
    o[2] = f32_to_bf16(2.0f * ((float)((s >> 16) & 0xFF) / 255.0f) - 1.0f);
    o[3] = f32_to_bf16(2.0f * ((float)(t & 0xFF) / 255.0f) - 1.0f);
    o[4] = f32_to_bf16(2.0f * ((float)((t >> 8) & 0xFF) / 255.0f) - 1.0f);
    o[5] = f32_to_bf16(2.0f * ((float)((t >> 16) & 0xFF) / 255.0f) - 1.0f);
#pragma unroll
    for (int c = 6; c < 16; ++c) o[c] = 0;
}

// fp32 network input [H8][W8][6] of one pair from its coarsest pyramid level
// (same pixels and padding as k_input_from_pyramids, before bf16 rounding)
__global__ void __launch_bounds__(256)
k_input_f32_from_pyramid(UNetPairIn P, int H8, int W8, float *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= H8 * W8) return;
    const int y = min(i / W8, P.h - 1), x = min(i % W8, P.w - 1);
    const uint32_t s = P.src[(size_t)(y + P.pad) * P.pitch + x + P.pad];
    const uint32_t t = P.tgt[(size_t)(y + P.pad) * P.pitch + x + P.pad];
    float *o = out + (size_t)i * 6;
    o[0] = (float)(s & 0xFF) / 255.0f;
    o[1] = (float)((s >> 8) & 0xFF) / 255.0f;
    o[2] = (float)((s >> 16) & 0xFF) / 255.0f;
    o[3] = (float)(t & 0xFF) / 255.0f;
    o[4] = (float)((t >> 8) & 0xFF) / 255.0f;
    o[5] = (float)((t >> 16) & 0xFF) / 255.0f;
}

// predicted offsets (head output, fp32 [H8][W8][16], channels 0,1) -> int32
// seed offsets [h][w][2] of each pair, rounded half away from zero
__global__ void __launch_bounds__(256)
k_pred_to_seed(const float *__restrict__ pred, int H8, int W8, const UNetPairIn *__restrict__ pairs,
               int32_t *const *__restrict__ seeds) {
    const int n = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const UNetPairIn P = pairs[n];
    if (i >= P.h * P.w) return;
    const int y = i / P.w, x = i % P.w;
    const float *q = pred + (((size_t)n * H8 + y) * W8 + x) * 2;
    seeds[n][2 * i] = (int32_t)roundf(fminf(fmaxf(q[0], -32767.f), 32767.f));
    seeds[n][2 * i + 1] = (int32_t)roundf(fminf(fmaxf(q[1], -32767.f), 32767.f));
}

// masked L1 loss of pred [n_px][2]; per-block partial
// sums of (mask * |pred - target|) and mask
__global__ void __launch_bounds__(256)
k_loss_partial(const float *__restrict__ pred, const float *__restrict__ target, const float *__restrict__ mask,
               long n_px, float *__restrict__ partial) {
    __shared__ float sl[256], sm[256];
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f, m = 0.f;
    if (i < n_px) {
        m = mask[i];
        l = m * (fabsf(pred[2 * i] - target[2 * i]) + fabsf(pred[2 * i + 1] - target[2 * i + 1]));
    }
    sl[threadIdx.x] = l;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sl[threadIdx.x] += sl[threadIdx.x + s];
            sm[threadIdx.x] += sm[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sl[0];
        partial[2 * blockIdx.x + 1] = sm[0];
    }
}

// one block: totals in block order; totals[0] = loss / max(mask sum, 1), totals[1] = max(mask sum, 1)
__global__ void __launch_bounds__(256)
k_loss_total(const float *__restrict__ partial, int n_blocks, float *__restrict__ totals) {
    __shared__ float sl[256], sm[256];
    float l = 0.f, m = 0.f;
    for (int b = threadIdx.x; b < n_blocks; b += 256) {
        l += partial[2 * b];
        m += partial[2 * b + 1];
    }
    sl[threadIdx.x] = l;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sl[threadIdx.x] += sl[threadIdx.x + s];
            sm[threadIdx.x] += sm[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float d = fmaxf(sm[0], 1.f);
        totals[0] = sl[0] / d;
        totals[1] = d;
    }
}

// d loss / d pred = mask * sign(pred - target) / max(mask sum, 1), bf16 [n_px][16]
__global__ void __launch_bounds__(256)
k_loss_grad(const float *__restrict__ pred, const float *__restrict__ target, const float *__restrict__ mask,
            const float *__restrict__ totals, long n_px, uint16_t *__restrict__ g) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_px * 16) return;
    const long p = i / 16;
    const int c = (int)(i % 16);
    float v = 0.f;
    if (c < 2) {
        const float d = pred[2 * p + c] - target[2 * p + c];
        v = mask[p] * (float)((d > 0.f) - (d < 0.f)) / totals[1];
    }
    g[i] = f32_to_bf16(v);
}

// Adam on fp32 master weights of one layer (padded layout [9][cout][cin] + bias
// [cout]); refreshes the bf16 weights [9][cout][cin] and the flipped,
// transposed bf16 weights [9][cin][cout] used for data gradients.
__global__ void __launch_bounds__(256)
k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
       long n_w, long n_total, int cout, int cin, float lr, float b1, float b2, float eps, float c1, float c2,
       uint16_t *__restrict__ w16, uint16_t *__restrict__ wt16) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (i < n_w) {
        const uint16_t h = f32_to_bf16(wi);
        w16[i] = h;
        const int ci = (int)(i % cin);
        const int co = (int)((i / cin) % cout);
        const int tap = (int)(i / ((long)cin * cout));
        wt16[((size_t)(8 - tap) * cin + ci) * cout + co] = h;
    }
}

// bf16 weight copies from fp32 master weights (after loading parameters)
__global__ void __launch_bounds__(256)
k_weights_to_bf16(const float *__restrict__ w, long n_w, int cout, int cin, uint16_t *__restrict__ w16,
                  uint16_t *__restrict__ wt16) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_w) return;
    const uint16_t h = f32_to_bf16(w[i]);
    w16[i] = h;
    const int ci = (int)(i % cin);
    const int co = (int)((i / cin) % cout);
    const int tap = (int)(i / ((long)cin * cout));
    wt16[((size_t)(8 - tap) * cin + ci) * cout + co] = h;
}

// flat parameters (PyTorch layout: weight [cout_r][cin_r][3][3], bias [cout_r])
// <-> padded master layout ([9][cout][cin], bias [cout]); to_padded = 1: flat -> padded
__global__ void __launch_bounds__(256)
k_param_layout(float *__restrict__ flat, float *__restrict__ padded, int cout_r, int cin_r, int cout, int cin,
               int to_padded) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long n_w = 9L * cout * cin;
    if (i >= n_w + cout) return;
    long f = -1;
    if (i < n_w) {
        const int ci = (int)(i % cin);
        const int co = (int)((i / cin) % cout);
        const int tap = (int)(i / ((long)cin * cout));
        if (ci < cin_r && co < cout_r) f = (((long)co * cin_r + ci) * 3 + tap / 3) * 3 + tap % 3;
    } else {
        const int co = (int)(i - n_w);
        if (co < cout_r) f = 9L * cout_r * cin_r + co;
    }
    if (to_padded) padded[i] = f >= 0 ? flat[f] : 0.f;
    else if (f >= 0) flat[f] = padded[i];
}

__global__ void __launch_bounds__(256) k_fill_zero(float *__restrict__ p, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// head output [n_px][2] -> the caller's offsets [n_px][2]
__global__ void __launch_bounds__(256)
k_pred_extract(const float *__restrict__ pred, long n_px, float *__restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_px * 2) return;
    out[i] = pred[i];
}

}  // namespace

static inline dim3 grid1(long n) { return dim3((unsigned)((n + 255) / 256)); }

// largest halo (pixels) of a kConvTile-pixel tile of a W-wide image of HW pixels
static int conv_halo_px(int H, int W) {
    const int HW = H * W;
    int best = 0;
    for (int p0 = 0; p0 < HW; p0 += kConvTile) {
        const int p1 = std::min(p0 + kConvTile, HW);
        best = std::max(best, ((p1 - 1) / W - p0 / W + 3) * (W + 2));
    }
    return best;
}

hipError_t launch_head3x3(const uint16_t *in, int B, int H, int W, int cin, const uint16_t *wt, int cout_pad,
                          const float *bias, float *out, hipStream_t s) {
    const int halo = conv_halo_px(H, W);
    if (cin != 32 || cout_pad < 16 || halo > kConvHaloMax || (long)B * H * W >= (1L << 31))
        return hipErrorInvalidValue;
    const int tiles = (H * W + kConvTile - 1) / kConvTile;
    const int he = std::max(2, (halo + 255) / 256);
    const dim3 grid((unsigned)(B * tiles));
    const size_t lds = (size_t)halo * 4 * sizeof(uint4);
    if (he == 2) hipLaunchKernelGGL(k_head3x3<2>, grid, dim3(256), lds, s, in, H, W, tiles, wt, cout_pad, bias, out);
    else if (he == 3) hipLaunchKernelGGL(k_head3x3<3>, grid, dim3(256), lds, s, in, H, W, tiles, wt, cout_pad, bias, out);
    else hipLaunchKernelGGL(k_head3x3<4>, grid, dim3(256), lds, s, in, H, W, tiles, wt, cout_pad, bias, out);
    return hipGetLastError();
}

bool conv_lds_fits(int B, int H, int W) {
    return conv_halo_px(H, W) <= kConvHaloMax && (long)B * H * W < (1L << 31);
}

hipError_t launch_conv3x3_in(const ConvIn &X, int B, int H, int W, int cin, const uint16_t *wt,
                             const float *bias, void *out, int cout, int ostride, bool relu, bool out_f32,
                             hipStream_t s, uint16_t *pool_out) {
    if (cin % 16 || cout % 16 || ostride < 1 || ostride > cout || X.ca % 16 || X.ca > cin || (X.ca < cin && !X.b) || (X.a_half && (H % 2 || W % 2)))
        return hipErrorInvalidValue;
    if (pool_out && (out_f32 || ostride != cout || H % 2 || W % 2)) return hipErrorInvalidValue;
    const int nbw = cout <= 32 ? 1 : (cout <= 64 ? 2 : 3);
    const int halo = conv_halo_px(H, W);
    // staged fragments, or the epilogue's output tile if that is larger
    const size_t lds = std::max(((size_t)9 * 32 * nbw + halo) * 2 * sizeof(uint4),
                                (size_t)kConvTile * kConvOutStride * sizeof(uint16_t));
    if (!conv_lds_fits(B, H, W) || out_f32 || ostride != cout) {
        // wide images, fp32 output or a partial channel range: the direct
        // kernel, which needs the input in one tensor
        if (X.ca != cin || X.a_half) return hipErrorInvalidValue;
        hipError_t e = launch_conv3x3(X.a, B, H, W, cin, wt, bias, out, cout, ostride, relu, out_f32, s);
        if (e != hipSuccess || !pool_out) return e;
        return launch_pool2(static_cast<const uint16_t *>(out), B, H, W, cout, pool_out, s);
    }
    // the pooling is fused when every tile covers whole row pairs
    const bool fuse_pool = pool_out && kConvTile % (2 * W) == 0;
    const int tiles = (H * W + kConvTile - 1) / kConvTile;
    const int he = std::max(2, (halo + 255) / 256);
    dim3 grid((unsigned)(B * tiles), (unsigned)((cout + 32 * nbw - 1) / (32 * nbw)));
    uint16_t *o = static_cast<uint16_t *>(out);
    uint16_t *po = fuse_pool ? pool_out : nullptr;
#define FB_CONVL(NB, HE, POOL)                                                                                        \
    if (relu) hipLaunchKernelGGL((k_conv3x3_lds<NB, HE, true, POOL>), grid, dim3(256), lds, s, X, H, W, cin, tiles, wt, bias, o, cout, po); \
    else hipLaunchKernelGGL((k_conv3x3_lds<NB, HE, false, POOL>), grid, dim3(256), lds, s, X, H, W, cin, tiles, wt, bias, o, cout, po);
#define FB_CONVL_HE(NB, POOL) \
    if (he == 2) { FB_CONVL(NB, 2, POOL) } else if (he == 3) { FB_CONVL(NB, 3, POOL) } else { FB_CONVL(NB, 4, POOL) }
#define FB_CONVL_NB(POOL) \
    switch (nbw) { \
    case 1: FB_CONVL_HE(1, POOL) break; \
    case 2: FB_CONVL_HE(2, POOL) break; \
    default: FB_CONVL_HE(3, POOL) break; \
    }
    if (fuse_pool) { FB_CONVL_NB(true) } else { FB_CONVL_NB(false) }
#undef FB_CONVL_NB
#undef FB_CONVL_HE
#undef FB_CONVL
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !pool_out || fuse_pool) return e;
    return launch_pool2(o, B, H, W, cout, pool_out, s);
}

hipError_t launch_conv3x3(const uint16_t *in, int B, int H, int W, int cin, const uint16_t *wt,
                          const float *bias, void *out, int cout, int ostride, bool relu, bool out_f32,
                          hipStream_t s) {
    const long total = (long)B * H * W;
    // NB divides cout / 16 so every channel block of a launch is full
    const int blocks = cout / 16;
    const int nb = blocks % 4 == 0 ? 4 : (blocks % 3 == 0 ? 3 : (blocks % 2 == 0 ? 2 : 1));
    dim3 grid((unsigned)((total + 255) / 256), blocks / nb);
#define FB_CONV(NB)                                                                                        \
    if (out_f32) hipLaunchKernelGGL((k_conv3x3<NB, false, true>), grid, dim3(256), 0, s, in, B, H, W, cin, wt, bias, out, cout, ostride); \
    else if (relu) hipLaunchKernelGGL((k_conv3x3<NB, true, false>), grid, dim3(256), 0, s, in, B, H, W, cin, wt, bias, out, cout, ostride); \
    else hipLaunchKernelGGL((k_conv3x3<NB, false, false>), grid, dim3(256), 0, s, in, B, H, W, cin, wt, bias, out, cout, ostride);
    switch (nb) {
    case 1: FB_CONV(1) break;
    case 2: FB_CONV(2) break;
    case 3: FB_CONV(3) break;
    default: FB_CONV(4) break;
    }
#undef FB_CONV
    return hipGetLastError();
}

hipError_t launch_conv_wgrad(const uint16_t *in, const uint16_t *g, int B, int H, int W, int cin, int cout,
                             int chunk_px, float *partial, float *bias_partial, hipStream_t s) {
    const long total = (long)B * H * W;
    const int n_chunks = (int)((total + chunk_px - 1) / chunk_px);
    hipLaunchKernelGGL(k_conv_wgrad, dim3(n_chunks, 9, (cout / 16) * (cin / 16)), dim3(64), 0, s, in, g, B, H,
                       W, cin, cout, chunk_px, partial);
    hipLaunchKernelGGL(k_bias_grad, dim3(n_chunks), dim3(256), 0, s, g, total, cout, chunk_px, bias_partial);
    return hipGetLastError();
}

hipError_t launch_reduce_chunks(const float *partial, int n_chunks, long n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_chunks, grid1(n), dim3(256), 0, s, partial, n_chunks, n, out);
    return hipGetLastError();
}

hipError_t launch_pool2(const uint16_t *in, int B, int H, int W, int C, uint16_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_pool2, grid1((long)B * (H / 2) * (W / 2) * C), dim3(256), 0, s, in, B, H, W, C, out);
    return hipGetLastError();
}

hipError_t launch_pool2_bwd_add(const uint16_t *gout, int B, int H, int W, int C, uint16_t *gin, hipStream_t s) {
    hipLaunchKernelGGL(k_pool2_bwd_add, grid1((long)B * H * W * C), dim3(256), 0, s, gout, B, H, W, C, gin);
    return hipGetLastError();
}

hipError_t launch_upcat(const uint16_t *deep, const uint16_t *skip, int B, int H, int W, int C1, int C2,
                        uint16_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_upcat, grid1((long)B * H * W * (C1 + C2)), dim3(256), 0, s, deep, skip, B, H, W, C1, C2, out);
    return hipGetLastError();
}

hipError_t launch_upcat_bwd(const uint16_t *gcat, int B, int H, int W, int C1, int C2, uint16_t *gdeep,
                            uint16_t *gskip, hipStream_t s) {
    const long n = (long)B * (H / 2) * (W / 2) * C1 + (long)B * H * W * C2;
    hipLaunchKernelGGL(k_upcat_bwd, grid1(n), dim3(256), 0, s, gcat, B, H, W, C1, C2, gdeep, gskip);
    return hipGetLastError();
}

hipError_t launch_relu_mask(uint16_t *g, const uint16_t *y, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_relu_mask, grid1(n), dim3(256), 0, s, g, y, n);
    return hipGetLastError();
}

hipError_t launch_input_from_f32(const float *x6, long n_px, uint16_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_input_from_f32, grid1(n_px * 16), dim3(256), 0, s, x6, n_px, out);
    return hipGetLastError();
}

hipError_t launch_input_from_pyramids(const UNetPairIn *pairs, int n, int H8, int W8, uint16_t *out,
                                      hipStream_t s) {
    hipLaunchKernelGGL(k_input_from_pyramids, dim3((H8 * W8 + 255) / 256, n), dim3(256), 0, s, pairs, H8, W8, out);
    return hipGetLastError();
}

hipError_t launch_input_f32_from_pyramid(const UNetPairIn &pair, int H8, int W8, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_input_f32_from_pyramid, dim3((H8 * W8 + 255) / 256), dim3(256), 0, s, pair, H8, W8, out);
    return hipGetLastError();
}

hipError_t launch_pred_to_seed(const float *pred, int H8, int W8, const UNetPairIn *pairs, int32_t *const *seeds,
                               int n, hipStream_t s) {
    hipLaunchKernelGGL(k_pred_to_seed, dim3((H8 * W8 + 255) / 256, n), dim3(256), 0, s, pred, H8, W8, pairs, seeds);
    return hipGetLastError();
}

hipError_t launch_loss(const float *pred, const float *target, const float *mask, long n_px, float *partial,
                       float *totals, uint16_t *grad, hipStream_t s) {
    const int nb = (int)((n_px + 255) / 256);
    hipLaunchKernelGGL(k_loss_partial, dim3(nb), dim3(256), 0, s, pred, target, mask, n_px, partial);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, partial, nb, totals);
    if (grad) hipLaunchKernelGGL(k_loss_grad, grid1(n_px * 16), dim3(256), 0, s, pred, target, mask, totals, n_px, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float *w, const float *g, float *m, float *v, long n_w, long n_total, int cout, int cin,
                       float lr, float b1, float b2, float eps, float c1, float c2, uint16_t *w16, uint16_t *wt16,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_adam, grid1(n_total), dim3(256), 0, s, w, g, m, v, n_w, n_total, cout, cin, lr, b1, b2,
                       eps, c1, c2, w16, wt16);
    return hipGetLastError();
}

hipError_t launch_weights_to_bf16(const float *w, long n_w, int cout, int cin, uint16_t *w16, uint16_t *wt16,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_weights_to_bf16, grid1(n_w), dim3(256), 0, s, w, n_w, cout, cin, w16, wt16);
    return hipGetLastError();
}

hipError_t launch_fill_zero(float *p, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_zero, grid1(n), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_pred_extract(const float *pred, long n_px, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_pred_extract, grid1(n_px * 2), dim3(256), 0, s, pred, n_px, out);
    return hipGetLastError();
}

hipError_t launch_param_layout(float *flat, float *padded, int cout_r, int cin_r, int cout, int cin, bool to_padded,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_param_layout, grid1(9L * cout * cin + cout), dim3(256), 0, s, flat, padded, cout_r, cin_r,
                       cout, cin, to_padded ? 1 : 0);
    return hipGetLastError();
}

}  // namespace fb
