// The learned proposal network: layer table, workspace and the forward,
// backward and Adam sequences (host side; kernels in unet.hip).
//
// Architecture (a project addition, not from the paper): a 4-level U-Net on
// the coarsest PatchMatch level of a frame pair.  Input: 6 channels (source
// RGB, target RGB, / 255), centred to 2x - 1.  Encoder levels of (32, 48,
// 96, 192) channels, two 3x3 conv + ReLU per level, 2x2 average pooling
// between levels; decoder: nearest 2x upsampling, concatenation with the
// encoder skip, two 3x3 conv + ReLU; head: 3x3 conv to 2 channels = predicted
// (row, col) offset of the match, in pixels of that level.  1,116,226
// parameters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "fb_common.h"

namespace fb {

namespace {

struct LayerDef {
    int cin_r, cout_r, cin, cout;
    bool relu;
};

constexpr LayerDef kLayers[] = {
    {6, 32, 16, 32, true},      // 0  enc1a
    {32, 32, 32, 32, true},     // 1  enc1b  -> e1
    {32, 48, 32, 48, true},     // 2  enc2a
    {48, 48, 48, 48, true},     // 3  enc2b  -> e2
    {48, 96, 48, 96, true},     // 4  enc3a
    {96, 96, 96, 96, true},     // 5  enc3b  -> e3
    {96, 192, 96, 192, true},   // 6  bottom a
    {192, 192, 192, 192, true}, // 7  bottom b
    {288, 96, 288, 96, true},   // 8  dec3a (upsampled bottom ++ e3)
    {96, 96, 96, 96, true},     // 9  dec3b
    {144, 48, 144, 48, true},   // 10 dec2a (upsampled dec3 ++ e2)
    {48, 48, 48, 48, true},     // 11 dec2b
    {80, 32, 80, 32, true},     // 12 dec1a (upsampled dec2 ++ e1)
    {32, 32, 32, 32, true},     // 13 dec1b
    {32, 2, 32, 16, false},     // 14 head
};
constexpr int kNL = sizeof(kLayers) / sizeof(kLayers[0]);

// activation tensors: spatial scale shift (0: H x W, 1: H/2, ...) and channels
enum T {
    X0, A0, E1, P1, A2, E2, P2, A4, E3, P3, A6, BT, C3, A8, D3, C2, A10, D2, C1, A12, D1, GPRED, kNT
};
constexpr int kTShift[kNT] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0, 0};
constexpr int kTCh[kNT] = {16, 32, 32, 32, 48, 48, 48, 96, 96, 96, 192, 192, 288, 96, 96, 144, 48, 48, 80, 32, 32, 16};

// layer i: input tensor, output tensor
constexpr int kLIn[kNL] = {X0, A0, P1, A2, P2, A4, P3, A6, C3, A8, C2, A10, C1, A12, D1};
constexpr int kLOut[kNL] = {A0, E1, A2, E2, A4, E3, A6, BT, A8, D3, A10, D2, A12, D1, -1};

constexpr int kChunkPx = 4096;

}  // namespace

struct UNet {
    size_t w_off[kNL];   // float offset of each layer's padded weights in the parameter buffers
    size_t w16_off[kNL]; // offset of each layer's bf16 weights
    size_t n_pad = 0, n_w16 = 0;
    float *w32 = nullptr, *g32 = nullptr, *m32 = nullptr, *v32 = nullptr;
    uint16_t *w16 = nullptr, *wt16 = nullptr;
    bool loaded = false;
    int adam_t = 0;
    // workspace for one (B, H, W)
    int B = 0, H = 0, W = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    uint16_t *act[kNT] = {};
    uint16_t *grad[kNT] = {};
    float *pred = nullptr, *partial = nullptr, *bias_partial = nullptr, *loss_partial = nullptr,
          *totals = nullptr;
};

UNet *unet_create() {
    UNet *u = new UNet();
    size_t off = 0, off16 = 0;
    for (int i = 0; i < kNL; ++i) {
        u->w_off[i] = off;
        off += 9 * (size_t)kLayers[i].cout * kLayers[i].cin + kLayers[i].cout;
        u->w16_off[i] = off16;
        off16 += 9 * (size_t)kLayers[i].cout * kLayers[i].cin;
    }
    u->n_pad = off;
    u->n_w16 = off16;
    return u;
}

void unet_destroy(UNet *u) {
    if (!u) return;
    for (void *p : {(void *)u->w32, (void *)u->g32, (void *)u->m32, (void *)u->v32, (void *)u->w16,
                    (void *)u->wt16, u->ws})
        if (p) (void)hipFree(p);
    delete u;
}

int64_t unet_param_count() {
    int64_t n = 0;
    for (const LayerDef &l : kLayers) n += 9LL * l.cout_r * l.cin_r + l.cout_r;
    return n;
}

bool unet_loaded(const UNet *u) { return u && u->loaded; }

static hipError_t alloc_params(UNet *u) {
    if (u->w32) return hipSuccess;
    hipError_t e;
    for (float **p : {&u->w32, &u->g32, &u->m32, &u->v32})
        if ((e = hipMalloc(p, u->n_pad * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc(&u->w16, u->n_w16 * 2)) != hipSuccess) return e;
    return hipMalloc(&u->wt16, u->n_w16 * 2);
}

hipError_t unet_load(UNet *u, const float *flat, hipStream_t s) {
    hipError_t e = alloc_params(u);
    if (e != hipSuccess) return e;
    size_t foff = 0;
    for (int i = 0; i < kNL; ++i) {
        const LayerDef &l = kLayers[i];
        if ((e = launch_param_layout(const_cast<float *>(flat) + foff, u->w32 + u->w_off[i], l.cout_r, l.cin_r,
                                     l.cout, l.cin, true, s)) != hipSuccess)
            return e;
        if ((e = launch_weights_to_bf16(u->w32 + u->w_off[i], 9L * l.cout * l.cin, l.cout, l.cin,
                                        u->w16 + u->w16_off[i], u->wt16 + u->w16_off[i], s)) != hipSuccess)
            return e;
        foff += 9 * (size_t)l.cout_r * l.cin_r + l.cout_r;
    }
    if ((e = launch_fill_zero(u->m32, (long)u->n_pad, s)) != hipSuccess) return e;
    if ((e = launch_fill_zero(u->v32, (long)u->n_pad, s)) != hipSuccess) return e;
    u->adam_t = 0;
    u->loaded = true;
    return hipSuccess;
}

static hipError_t to_flat(UNet *u, const float *padded_base, float *flat, hipStream_t s) {
    size_t foff = 0;
    for (int i = 0; i < kNL; ++i) {
        const LayerDef &l = kLayers[i];
        hipError_t e = launch_param_layout(flat + foff, const_cast<float *>(padded_base) + u->w_off[i], l.cout_r,
                                           l.cin_r, l.cout, l.cin, false, s);
        if (e != hipSuccess) return e;
        foff += 9 * (size_t)l.cout_r * l.cin_r + l.cout_r;
    }
    return hipSuccess;
}

hipError_t unet_save(UNet *u, float *flat, hipStream_t s) { return to_flat(u, u->w32, flat, s); }

// training state: parameters, Adam moments (flat layout) and the step count
hipError_t unet_save_state(UNet *u, float *flat, float *m, float *v, int64_t *step, hipStream_t s) {
    hipError_t e;
    if ((e = to_flat(u, u->w32, flat, s)) != hipSuccess || (e = to_flat(u, u->m32, m, s)) != hipSuccess ||
        (e = to_flat(u, u->v32, v, s)) != hipSuccess)
        return e;
    *step = u->adam_t;
    return hipSuccess;
}

hipError_t unet_load_state(UNet *u, const float *flat, const float *m, const float *v, int64_t step, hipStream_t s) {
    hipError_t e = unet_load(u, flat, s);
    if (e != hipSuccess) return e;
    size_t foff = 0;
    for (int i = 0; i < kNL; ++i) {
        const LayerDef &l = kLayers[i];
        if ((e = launch_param_layout(const_cast<float *>(m) + foff, u->m32 + u->w_off[i], l.cout_r, l.cin_r, l.cout,
                                     l.cin, true, s)) != hipSuccess ||
            (e = launch_param_layout(const_cast<float *>(v) + foff, u->v32 + u->w_off[i], l.cout_r, l.cin_r, l.cout,
                                     l.cin, true, s)) != hipSuccess)
            return e;
        foff += 9 * (size_t)l.cout_r * l.cin_r + l.cout_r;
    }
    u->adam_t = (int)step;
    return hipSuccess;
}
hipError_t unet_grads_flat(UNet *u, float *flat, hipStream_t s) { return to_flat(u, u->g32, flat, s); }

// Carve the workspace for batch B at H x W (H and W multiples of 8).  With
// allocate == false nothing is allocated (as inside a captured launch
// sequence) and a workspace smaller than needed is an error.
static hipError_t carve(UNet *u, int B, int H, int W, bool training, bool allocate) {
    auto tensor_elems = [&](int t) { return (size_t)B * (H >> kTShift[t]) * (W >> kTShift[t]) * kTCh[t]; };
    size_t bytes = 0;
    auto take = [&](size_t n) { size_t o = bytes; bytes += (n + 127) & ~(size_t)127; return o; };
    size_t a_off[kNT], g_off[kNT] = {};
    for (int t = 0; t < kNT; ++t) a_off[t] = take(tensor_elems(t) * 2);
    const size_t px = (size_t)B * H * W;
    const size_t pred_off = take(px * 2 * 4);
    size_t part_off = 0, bpart_off = 0, lpart_off = 0, tot_off = 0;
    if (training) {
        for (int t = 0; t < kNT; ++t) g_off[t] = take(tensor_elems(t) * 2);
        size_t part = 0, bpart = 0;
        for (int i = 0; i < kNL; ++i) {
            const int tin = kLIn[i];
            const size_t pxl = (size_t)B * (H >> kTShift[tin]) * (W >> kTShift[tin]);
            const size_t chunks = (pxl + kChunkPx - 1) / kChunkPx;
            part = std::max(part, chunks * 9 * kLayers[i].cout * kLayers[i].cin);
            bpart = std::max(bpart, chunks * kLayers[i].cout);
        }
        part_off = take(part * 4);
        bpart_off = take(bpart * 4);
        lpart_off = take(((px + 255) / 256) * 2 * 4);
        tot_off = take(2 * 4);
    }
    if (bytes > u->ws_bytes) {
        if (!allocate) return hipErrorInvalidValue;
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        if (u->ws) (void)hipFree(u->ws);
        u->ws = nullptr;
        u->ws_bytes = 0;
        if ((e = hipMalloc(&u->ws, bytes)) != hipSuccess) return e;
        u->ws_bytes = bytes;
    }
    char *base = static_cast<char *>(u->ws);
    for (int t = 0; t < kNT; ++t) {
        u->act[t] = reinterpret_cast<uint16_t *>(base + a_off[t]);
        u->grad[t] = training ? reinterpret_cast<uint16_t *>(base + g_off[t]) : nullptr;
    }
    u->pred = reinterpret_cast<float *>(base + pred_off);
    u->partial = training ? reinterpret_cast<float *>(base + part_off) : nullptr;
    u->bias_partial = training ? reinterpret_cast<float *>(base + bpart_off) : nullptr;
    u->loss_partial = training ? reinterpret_cast<float *>(base + lpart_off) : nullptr;
    u->totals = training ? reinterpret_cast<float *>(base + tot_off) : nullptr;
    u->B = B;
    u->H = H;
    u->W = W;
    return hipSuccess;
}

hipError_t unet_reserve(UNet *u, int B, int H, int W, bool training) { return carve(u, B, H, W, training, true); }
hipError_t unet_shape(UNet *u, int B, int H, int W, bool training) { return carve(u, B, H, W, training, false); }

uint16_t *unet_input_buffer(UNet *u) { return u->act[X0]; }
float *unet_pred_buffer(UNet *u) { return u->pred; }
float *unet_loss_buffer(UNet *u) { return u->totals; }

#define FB_TRY(x)                                \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) return e_;         \
    } while (0)

// decoder layers that read [upsampled deeper tensor, skip] in place
static bool upcat_input(int i, int *deep, int *skip) {
    switch (i) {
    case 8: *deep = BT; *skip = E3; return true;
    case 10: *deep = D3; *skip = E2; return true;
    case 12: *deep = D2; *skip = E1; return true;
    default: return false;
    }
}

// keep_cat: the decoder's concatenated input is materialised anyway
// pool: also write the 2x2 average pooling of the output to that tensor
static hipError_t conv_fwd(UNet *u, int i, bool keep_cat, hipStream_t s, int pool = -1) {
    const LayerDef &l = kLayers[i];
    const int sh = kTShift[kLIn[i]], H = u->H >> sh, W = u->W >> sh;
    const float *bias = u->w32 + u->w_off[i] + 9 * (size_t)l.cout * l.cin;
    void *out = kLOut[i] >= 0 ? (void *)u->act[kLOut[i]] : (void *)u->pred;
    int deep, skip;
    ConvIn X{u->act[kLIn[i]], nullptr, l.cin, 0};
    if (upcat_input(i, &deep, &skip)) {
        if (conv_lds_fits(u->B, H, W)) {
            X = ConvIn{u->act[deep], u->act[skip], kTCh[deep], 1};
        } else if (!keep_cat) {
            FB_TRY(launch_upcat(u->act[deep], u->act[skip], u->B, H, W, kTCh[deep], kTCh[skip], u->act[kLIn[i]], s));
        }
    }
    if (kLOut[i] < 0) {  // the offset head: fp32 [px][2]
        if (conv_lds_fits(u->B, H, W))
            return launch_head3x3(X.a, u->B, H, W, l.cin, u->w16 + u->w16_off[i], l.cout, bias, u->pred, s);
        return launch_conv3x3_in(X, u->B, H, W, l.cin, u->w16 + u->w16_off[i], bias, out, l.cout, l.cout_r, false,
                                 true, s);
    }
    return launch_conv3x3_in(X, u->B, H, W, l.cin, u->w16 + u->w16_off[i], bias, out, l.cout, l.cout, l.relu, false,
                             s, pool >= 0 ? u->act[pool] : nullptr);
}

hipError_t unet_forward(UNet *u, hipStream_t s, bool keep_cat) {
    const int B = u->B, H = u->H, W = u->W;
    FB_TRY(conv_fwd(u, 0, keep_cat, s));
    FB_TRY(conv_fwd(u, 1, keep_cat, s, P1));
    FB_TRY(conv_fwd(u, 2, keep_cat, s));
    FB_TRY(conv_fwd(u, 3, keep_cat, s, P2));
    FB_TRY(conv_fwd(u, 4, keep_cat, s));
    FB_TRY(conv_fwd(u, 5, keep_cat, s, P3));
    FB_TRY(conv_fwd(u, 6, keep_cat, s));
    FB_TRY(conv_fwd(u, 7, keep_cat, s));
    if (keep_cat) FB_TRY(launch_upcat(u->act[BT], u->act[E3], B, H / 4, W / 4, 192, 96, u->act[C3], s));
    FB_TRY(conv_fwd(u, 8, keep_cat, s));
    FB_TRY(conv_fwd(u, 9, keep_cat, s));
    if (keep_cat) FB_TRY(launch_upcat(u->act[D3], u->act[E2], B, H / 2, W / 2, 96, 48, u->act[C2], s));
    FB_TRY(conv_fwd(u, 10, keep_cat, s));
    FB_TRY(conv_fwd(u, 11, keep_cat, s));
    if (keep_cat) FB_TRY(launch_upcat(u->act[D2], u->act[E1], B, H, W, 48, 32, u->act[C1], s));
    FB_TRY(conv_fwd(u, 12, keep_cat, s));
    FB_TRY(conv_fwd(u, 13, keep_cat, s));
    return conv_fwd(u, 14, keep_cat, s);
}

// weight and bias gradients of layer i from the gradient g of its output
static hipError_t conv_wgrad(UNet *u, int i, const uint16_t *g, hipStream_t s) {
    const LayerDef &l = kLayers[i];
    const int sh = kTShift[kLIn[i]];
    const int H = u->H >> sh, W = u->W >> sh;
    const long px = (long)u->B * H * W;
    const int chunks = (int)((px + kChunkPx - 1) / kChunkPx);
    FB_TRY(launch_conv_wgrad(u->act[kLIn[i]], g, u->B, H, W, l.cin, l.cout, kChunkPx, u->partial,
                             u->bias_partial, s));
    float *gw = u->g32 + u->w_off[i];
    FB_TRY(launch_reduce_chunks(u->partial, chunks, 9L * l.cout * l.cin, gw, s));
    return launch_reduce_chunks(u->bias_partial, chunks, l.cout, gw + 9 * (size_t)l.cout * l.cin, s);
}

// data gradient of layer i: gradient of its input from the gradient g of its output
static hipError_t conv_dgrad(UNet *u, int i, const uint16_t *g, uint16_t *gin, hipStream_t s) {
    const LayerDef &l = kLayers[i];
    const int sh = kTShift[kLIn[i]];
    return launch_conv3x3_in(ConvIn{g, nullptr, l.cout, 0}, u->B, u->H >> sh, u->W >> sh, l.cout,
                             u->wt16 + u->w16_off[i], nullptr, gin, l.cin, l.cin, false, false, s);
}

static long elems(UNet *u, int t) { return (long)u->B * (u->H >> kTShift[t]) * (u->W >> kTShift[t]) * kTCh[t]; }

// backward through a ReLU conv layer i whose output gradient is in grad[kLOut[i]]
static hipError_t relu_layer_bwd(UNet *u, int i, hipStream_t s) {
    const int to = kLOut[i], ti = kLIn[i];
    FB_TRY(launch_relu_mask(u->grad[to], u->act[to], elems(u, to), s));
    FB_TRY(conv_wgrad(u, i, u->grad[to], s));
    if (i == 0) return hipSuccess;  // no gradient for the network input
    return conv_dgrad(u, i, u->grad[to], u->grad[ti], s);
}

hipError_t unet_loss_backward(UNet *u, const float *target, const float *mask, bool backward, hipStream_t s) {
    const int B = u->B, H = u->H, W = u->W;
    const long px = (long)B * H * W;
    FB_TRY(launch_loss(u->pred, target, mask, px, u->loss_partial, u->totals, backward ? u->grad[GPRED] : nullptr, s));
    if (!backward) return hipSuccess;
    // head
    FB_TRY(conv_wgrad(u, 14, u->grad[GPRED], s));
    FB_TRY(conv_dgrad(u, 14, u->grad[GPRED], u->grad[D1], s));
    FB_TRY(relu_layer_bwd(u, 13, s));
    FB_TRY(relu_layer_bwd(u, 12, s));
    FB_TRY(launch_upcat_bwd(u->grad[C1], B, H, W, 48, 32, u->grad[D2], u->grad[E1], s));
    FB_TRY(relu_layer_bwd(u, 11, s));
    FB_TRY(relu_layer_bwd(u, 10, s));
    FB_TRY(launch_upcat_bwd(u->grad[C2], B, H / 2, W / 2, 96, 48, u->grad[D3], u->grad[E2], s));
    FB_TRY(relu_layer_bwd(u, 9, s));
    FB_TRY(relu_layer_bwd(u, 8, s));
    FB_TRY(launch_upcat_bwd(u->grad[C3], B, H / 4, W / 4, 192, 96, u->grad[BT], u->grad[E3], s));
    FB_TRY(relu_layer_bwd(u, 7, s));
    FB_TRY(relu_layer_bwd(u, 6, s));
    FB_TRY(launch_pool2_bwd_add(u->grad[P3], B, H / 4, W / 4, 96, u->grad[E3], s));
    FB_TRY(relu_layer_bwd(u, 5, s));
    FB_TRY(relu_layer_bwd(u, 4, s));
    FB_TRY(launch_pool2_bwd_add(u->grad[P2], B, H / 2, W / 2, 48, u->grad[E2], s));
    FB_TRY(relu_layer_bwd(u, 3, s));
    FB_TRY(relu_layer_bwd(u, 2, s));
    FB_TRY(launch_pool2_bwd_add(u->grad[P1], B, H, W, 32, u->grad[E1], s));
    FB_TRY(relu_layer_bwd(u, 1, s));
    return relu_layer_bwd(u, 0, s);
}

hipError_t unet_adam(UNet *u, float lr, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    ++u->adam_t;
    const float c1 = 1.f - powf(b1, (float)u->adam_t), c2 = 1.f - powf(b2, (float)u->adam_t);
    for (int i = 0; i < kNL; ++i) {
        const LayerDef &l = kLayers[i];
        const long nw = 9L * l.cout * l.cin;
        FB_TRY(launch_adam(u->w32 + u->w_off[i], u->g32 + u->w_off[i], u->m32 + u->w_off[i], u->v32 + u->w_off[i],
                           nw, nw + l.cout, l.cout, l.cin, lr, b1, b2, eps, c1, c2, u->w16 + u->w16_off[i],
                           u->wt16 + u->w16_off[i], s));
    }
    return hipSuccess;
}

hipError_t unet_input_from_f32(UNet *u, const float *x6, hipStream_t s) {
    return launch_input_from_f32(x6, (long)u->B * u->H * u->W, u->act[X0], s);
}

double unet_forward_flops(int B, int H, int W) {
    double f = 0;
    for (int i = 0; i < kNL; ++i) {
        const int sh = kTShift[kLIn[i]];
        f += 2.0 * 9 * kLayers[i].cin_r * kLayers[i].cout_r * (double)B * (H >> sh) * (W >> sh);
    }
    return f;
}

}  // namespace fb
