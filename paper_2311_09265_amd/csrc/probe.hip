// Measurement kernel (no part of the method): the gather rate of patch rows
// that bounds the PatchMatch iteration (fb_gather_probe).
#include "fb_common.h"

namespace fb {

namespace {

// reads through global (address space 1) pointers with a 32-bit offset from a
// uniform base, as the iteration kernel does
template <class T>
using gptr = const __attribute__((address_space(1))) T *;

// Measurement: the rate at which patch rows (5 pixels: one 16-byte and one
// 4-byte load, as the iteration kernel fetches them) can be gathered from one
// padded image, each row folded into a sum with v_dot4 like a candidate row.
// DIVERGENT: every lane at its own random pixel (random-search candidates);
// otherwise the wave's 64 lanes at consecutive pixels of a random row
// (propagation candidates).  Positions come from a per-lane xorshift; the
// sums are written out so nothing is optimised away.
template <bool DIVERGENT>
__global__ void __launch_bounds__(256)
k_gather_probe(const uint32_t *__restrict__ img, int h, int w, int pitch, int rows, uint32_t *__restrict__ out) {
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    uint32_t x = gid * 0x9E3779B9u + 0x7F4A7C15u;
    x ^= x >> 16;
    const uint32_t t = 0x00010101u * (gid & 0xFFu);
    uint32_t acc = 0;
    for (int k = 0; k < rows; ++k) {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        const uint32_t y = DIVERGENT ? x : (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
        const int r = (int)(((y & 0xFFFFu) * (uint32_t)h) >> 16);
        int c = (int)(((y >> 16) * (uint32_t)w) >> 16);
        if (!DIVERGENT) c = min(c + (int)(threadIdx.x & 63u), w - 1);
        const gptr<uint32_t> q = (gptr<uint32_t>)((gptr<char>)img + 4u * (uint32_t)(r * pitch + c));
        uint32_t row[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) row[j] = q[j];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            acc = __builtin_amdgcn_udot4(row[j], t, acc, false);
            acc = __builtin_amdgcn_udot4(row[j], row[j], acc, false);
        }
    }
    out[gid] = acc;
}

}  // namespace

hipError_t launch_gather_probe(const uint32_t *img, int h, int w, int pitch, bool divergent, int blocks, int rows,
                               uint32_t *out, hipStream_t s) {
    if (divergent) hipLaunchKernelGGL(k_gather_probe<true>, dim3(blocks), dim3(256), 0, s, img, h, w, pitch, rows, out);
    else hipLaunchKernelGGL(k_gather_probe<false>, dim3(blocks), dim3(256), 0, s, img, h, w, pitch, rows, out);
    return hipGetLastError();
}

}  // namespace fb
