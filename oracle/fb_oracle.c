/*
 * FastBlend CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, deliberately unoptimised C implementation of what the
 * FastBlend hot path computes (Duan et al., "FastBlend: a Powerful Model-Free
 * Toolkit Making Video Stylization Easier", arXiv 2311.09265).  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the GPU library.
 *
 * Every function cites the passage of the paper it follows.  Where the paper
 * is silent, the reading taken is stated at the function (and listed with all
 * other readings in the design notes of the repository):
 *
 *   coordinates   F(r,c) = (row, col) of the source patch centre matched to
 *                 target pixel (r,c); the paper's (x,y) is read as (row, col).
 *   sampling      pixels outside an image are read clamp-to-edge.
 *   pyramid       2x2 box filter with round-half-up, ceil(size/2) per level.
 *   upsampling    F_l(r,c) = clamp(2 F_{l+1}(r/2, c/2) + (r&1, c&1)).
 *   update        Jacobi: every pixel reads only the previous iteration's
 *                 field; each pixel tries its candidates in a fixed order
 *                 against its own running best with strict '<'.
 *   random search symmetric integer offsets in [-rho, rho]^2 around the
 *                 running best, rho = R >> m (R = max(h,w)) while rho >= 1,
 *                 drawn from Philox4x32-10 (Salmon et al., SC'11) keyed by
 *                 the seed, counter = (pixel, pair id, level<<16 | iter, m>>2);
 *                 word m&3 gives (row 16 bits low, col 16 bits high); a
 *                 16-bit draw u maps to [0, n) as (u * n) >> 16.
 *   remap border  neighbours outside the image are skipped and the sum is
 *                 divided by the number that remain (the patch-overlap
 *                 average of Section 3.3).
 *   window ends   the blending window is truncated to [0, N-1] and divided by
 *                 its length; the j == i term is the style frame itself.
 *   Eq. (3)       S^ is a uint8 image (the remap average rounded half up),
 *                 alpha = alpha16 / 16, the loss is scaled by 16 to stay an
 *                 integer; S^ is refreshed at the start of every iteration
 *                 and the incumbent's loss recomputed under it.
 *
 * Images are uint8 [h][w][3] row-major; NNFs are int32 [h][w][2] (row, col);
 * energies are uint32 [h][w].  Floating-point outputs are fp64.
 * Within one call the work over rows is spread with OpenMP; every pixel of a
 * Jacobi iteration is independent, so this does not change any result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define FBO_OK 0
#define FBO_E_INVALID -1
#define FBO_E_ALLOC -4

static int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }
static int maxi(int a, int b) { return a > b ? a : b; }

void fbo_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int fbo_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw, */
/* "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11): 10 rounds of       */
/* (x0,x1,x2,x3) -> (hi(M1 x2)^x1^k0, lo(M1 x2), hi(M0 x0)^x3^k1, lo(M0 x0)) */
/* with the key bumped by the Weyl constants between rounds.                 */
/* The paper draws its initial field and search offsets at random (Alg. 1,   */
/* Section 3.2) without naming a generator; this one is counter based so a   */
/* draw depends only on what it is for, never on evaluation order.           */
/* ------------------------------------------------------------------------ */
void fbo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* a 16-bit uniform draw mapped to [0, n), n <= 65536 */
uint32_t fbo_uniform16(uint32_t u16, uint32_t n) { return (u16 * n) >> 16; }

static void draw_words(uint64_t seed, uint32_t pixel, uint32_t pair_id, uint32_t level,
                       uint32_t iter, uint32_t call, uint32_t out[4])
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { pixel, pair_id, (level << 16) | (iter & 0xFFFFu), call };
    fbo_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Image pyramid (Alg. 1, "resize images S, T" per pyramid level).           */
/* Reading: 2x2 box filter, round half up, output ceil(h/2) x ceil(w/2),     */
/* input reads clamped to the image.                                         */
/* ------------------------------------------------------------------------ */
void fbo_downsample(const uint8_t *in, int h, int w, uint8_t *out)
{
    int ho = (h + 1) / 2, wo = (w + 1) / 2;
    for (int r = 0; r < ho; ++r)
        for (int c = 0; c < wo; ++c)
            for (int ch = 0; ch < 3; ++ch) {
                int s = 0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        int rr = clampi(2 * r + a, 0, h - 1), cc = clampi(2 * c + b, 0, w - 1);
                        s += in[(rr * w + cc) * 3 + ch];
                    }
                out[(r * wo + c) * 3 + ch] = (uint8_t)((s + 2) >> 2);
            }
}

/* ------------------------------------------------------------------------ */
/* Base loss, Eq. (1): squared L2 distance between the (2p+1)x(2p+1)x3       */
/* patches S[u] and T[v].  Integer arithmetic on uint8 pixels, so exact.     */
/* ------------------------------------------------------------------------ */
uint32_t fbo_patch_ssd(const uint8_t *S, const uint8_t *T, int h, int w, int p,
                       int ur, int uc, int vr, int vc)
{
    uint32_t acc = 0;
    for (int dr = -p; dr <= p; ++dr)
        for (int dc = -p; dc <= p; ++dc) {
            const uint8_t *s = S + 3 * (clampi(ur + dr, 0, h - 1) * w + clampi(uc + dc, 0, w - 1));
            const uint8_t *t = T + 3 * (clampi(vr + dr, 0, h - 1) * w + clampi(vc + dc, 0, w - 1));
            for (int ch = 0; ch < 3; ++ch) {
                int d = (int)s[ch] - (int)t[ch];
                acc += (uint32_t)(d * d);
            }
        }
    return acc;
}

/* E(v) = L(S, T, F)_v for every target pixel (Alg. 1, "initialize error matrix"). */
void fbo_energy(const uint8_t *S, const uint8_t *T, int h, int w, int p,
                const int32_t *F, uint32_t *E)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            const int32_t *f = F + 2 * (r * w + c);
            E[r * w + c] = fbo_patch_ssd(S, T, h, w, p, f[0], f[1], r, c);
        }
}

/* ------------------------------------------------------------------------ */
/* Random initialisation of F (Alg. 1, first step), taken at the coarsest    */
/* level: F(v) is a uniformly drawn source position; E is its loss.          */
/* ------------------------------------------------------------------------ */
void fbo_nnf_init_random(const uint8_t *S, const uint8_t *T, int h, int w, int p,
                         int level, uint64_t seed, uint32_t pair_id, int32_t *F, uint32_t *E)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            uint32_t x[4];
            draw_words(seed, (uint32_t)(r * w + c), pair_id, (uint32_t)level, 0xFFFFu, 0u, x);
            int fr = (int)fbo_uniform16(x[0] & 0xFFFFu, (uint32_t)h);
            int fc = (int)fbo_uniform16(x[0] >> 16, (uint32_t)w);
            F[2 * (r * w + c)] = fr;
            F[2 * (r * w + c) + 1] = fc;
            E[r * w + c] = fbo_patch_ssd(S, T, h, w, p, fr, fc, r, c);
        }
}

/* Initialisation from a given offset field: F(v) = clamp(v + off(v)). */
void fbo_nnf_init_offsets(const uint8_t *S, const uint8_t *T, int h, int w, int p,
                          const int32_t *off, int32_t *F, uint32_t *E)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            int fr = clampi(r + off[2 * (r * w + c)], 0, h - 1);
            int fc = clampi(c + off[2 * (r * w + c) + 1], 0, w - 1);
            F[2 * (r * w + c)] = fr;
            F[2 * (r * w + c) + 1] = fc;
            E[r * w + c] = fbo_patch_ssd(S, T, h, w, p, fr, fc, r, c);
        }
}

/* ------------------------------------------------------------------------ */
/* Upsampling F to the next finer level (Alg. 1, "upsample F"), followed by  */
/* recomputing E.  Reading: nearest-neighbour on the offsets, i.e. a coarse   */
/* match (R, C) becomes (2R + (r&1), 2C + (c&1)), clamped into the image.    */
/* (hc, wc) = (ceil(h/2), ceil(w/2)) is the coarse size.                     */
/* ------------------------------------------------------------------------ */
void fbo_nnf_upsample(const int32_t *Fc, int hc, int wc, const uint8_t *S, const uint8_t *T,
                      int h, int w, int p, int32_t *F, uint32_t *E)
{
    (void)hc;
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            const int32_t *f = Fc + 2 * ((r >> 1) * wc + (c >> 1));
            int fr = clampi(2 * f[0] + (r & 1), 0, h - 1);
            int fc = clampi(2 * f[1] + (c & 1), 0, w - 1);
            F[2 * (r * w + c)] = fr;
            F[2 * (r * w + c) + 1] = fc;
            E[r * w + c] = fbo_patch_ssd(S, T, h, w, p, fr, fc, r, c);
        }
}

/* ------------------------------------------------------------------------ */
/* One PatchMatch iteration (Alg. 1 inner loop; Section 3.2):                 */
/*  - propagation: F'(v) = F(v + d) - d for d = (-1,0), (1,0), (0,-1), (0,1)  */
/*    in that order, skipped where v + d is outside the image;               */
/*  - random search: F'(v) = best(v) + delta, delta uniform in [-rho, rho]^2, */
/*    rho = R, R/2, ..., 1 (R = max(h, w)), "declining exponentially";        */
/*  - a candidate replaces the running best only if its loss is strictly     */
/*    lower (the F(E' < E) <- F' update).                                    */
/* Every position is updated independently from the previous iteration's     */
/* field (Fo, Eo) -- the concurrent update the paper adopts instead of       */
/* Barnes et al.'s scan order.  Candidates are clamped into the image.       */
/* ------------------------------------------------------------------------ */
void fbo_pm_iteration(const uint8_t *S, const uint8_t *T, int h, int w, int p, int level,
                      int iter, uint64_t seed, uint32_t pair_id,
                      const int32_t *Fo, const uint32_t *Eo, int32_t *Fn, uint32_t *En)
{
    static const int D[4][2] = { { -1, 0 }, { 1, 0 }, { 0, -1 }, { 0, 1 } };
    const int R = maxi(h, w);
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            int br = Fo[2 * (r * w + c)], bc = Fo[2 * (r * w + c) + 1];
            uint32_t be = Eo[r * w + c];
            for (int k = 0; k < 4; ++k) {
                int qr = r + D[k][0], qc = c + D[k][1];
                if (qr < 0 || qr >= h || qc < 0 || qc >= w) continue;
                int cr = clampi(Fo[2 * (qr * w + qc)] - D[k][0], 0, h - 1);
                int cc = clampi(Fo[2 * (qr * w + qc) + 1] - D[k][1], 0, w - 1);
                uint32_t e = fbo_patch_ssd(S, T, h, w, p, cr, cc, r, c);
                if (e < be) { br = cr; bc = cc; be = e; }
            }
            uint32_t x[4] = { 0, 0, 0, 0 };
            for (int m = 0; (R >> m) >= 1; ++m) {
                int rho = R >> m;
                if ((m & 3) == 0)
                    draw_words(seed, (uint32_t)(r * w + c), pair_id, (uint32_t)level,
                               (uint32_t)iter, (uint32_t)(m >> 2), x);
                uint32_t word = x[m & 3];
                int dr = (int)fbo_uniform16(word & 0xFFFFu, (uint32_t)(2 * rho + 1)) - rho;
                int dc = (int)fbo_uniform16(word >> 16, (uint32_t)(2 * rho + 1)) - rho;
                int cr = clampi(br + dr, 0, h - 1), cc = clampi(bc + dc, 0, w - 1);
                uint32_t e = fbo_patch_ssd(S, T, h, w, p, cr, cc, r, c);
                if (e < be) { br = cr; bc = cc; be = e; }
            }
            Fn[2 * (r * w + c)] = br;
            Fn[2 * (r * w + c) + 1] = bc;
            En[r * w + c] = be;
        }
}

/* ------------------------------------------------------------------------ */
/* Whole coarse-to-fine estimation NNF(S, T) (Alg. 1): pyramid of `levels`   */
/* levels, random (or offset-seeded) initialisation at the coarsest level,   */
/* `iters` iterations at every level, upsampling between levels.             */
/* `seed_off` (optional) is an int32 offset field at the coarsest level.     */
/* ------------------------------------------------------------------------ */
static int patchmatch_impl(const uint8_t *S0, const uint8_t *T0, int h, int w, int p, int levels,
                           int iters, uint64_t seed, uint32_t pair_id, const int32_t *seed_off,
                           int32_t *F, uint32_t *E);

int fbo_patchmatch(const uint8_t *S0, const uint8_t *T0, int h, int w, int p, int levels,
                   int iters, uint64_t seed, uint32_t pair_id, const int32_t *seed_off,
                   int32_t *F, uint32_t *E)
{
    return patchmatch_impl(S0, T0, h, w, p, levels, iters, seed, pair_id, seed_off, F, E);
}

/* ------------------------------------------------------------------------ */
/* Guard of a seeded run (a project addition: the learned proposal replaces  */
/* Alg. 1's random initialisation, and Alg. 1 itself has no such rule).  At  */
/* the coarsest level the seeded start followed by `iters` iterations races  */
/* the random start followed by one more iteration, race = min(iters + 1,    */
/* plain_iters) iterations: a seed must be worth at least an iteration.      */
/* sums[0], sums[1] are the two levels' summed energies (64-bit).  If the    */
/* seeded sum is the larger, the seed is rejected and the result is the      */
/* plain run (random start, plain_iters iterations at every level);          */
/* otherwise it is the seeded run (iters iterations at every level).         */
/* *rejected: 1 if plain was taken.                                          */
/* ------------------------------------------------------------------------ */
static uint64_t sum_u32(const uint32_t *E, size_t n)
{
    uint64_t s = 0;
    for (size_t i = 0; i < n; ++i) s += E[i];
    return s;
}

/* the coarsest level's summed energy after `iters` iterations from a seeded */
/* (seed_off) or random (seed_off == NULL) start                             */
static int coarse_energy(const uint8_t *S0, const uint8_t *T0, int h, int w, int p, int levels, int iters,
                         uint64_t seed, uint32_t pair_id, const int32_t *seed_off, uint64_t *sum)
{
    const int l = levels - 1;
    int hl = h, wl = w;
    for (int k = 0; k < l; ++k) { hl = (hl + 1) / 2; wl = (wl + 1) / 2; }
    const size_t n = (size_t)hl * wl;
    const size_t nb = (size_t)h * w * 3;
    uint8_t *S = (uint8_t *)malloc(nb), *T = (uint8_t *)malloc(nb), *tmp = (uint8_t *)malloc(nb);
    int32_t *Fa = (int32_t *)malloc(n * 2 * sizeof(int32_t)), *Fb = (int32_t *)malloc(n * 2 * sizeof(int32_t));
    uint32_t *Ea = (uint32_t *)malloc(n * sizeof(uint32_t)), *Eb = (uint32_t *)malloc(n * sizeof(uint32_t));
    int status = FBO_OK;
    if (!S || !T || !tmp || !Fa || !Fb || !Ea || !Eb) { status = FBO_E_ALLOC; goto out; }
    memcpy(S, S0, nb);
    memcpy(T, T0, nb);
    {
        int hc = h, wc = w;
        for (int k = 0; k < l; ++k) {
            const size_t no = (size_t)((hc + 1) / 2) * ((wc + 1) / 2) * 3;
            fbo_downsample(S, hc, wc, tmp);
            memcpy(S, tmp, no);
            fbo_downsample(T, hc, wc, tmp);
            memcpy(T, tmp, no);
            hc = (hc + 1) / 2;
            wc = (wc + 1) / 2;
        }
    }
    if (seed_off) fbo_nnf_init_offsets(S, T, hl, wl, p, seed_off, Fa, Ea);
    else fbo_nnf_init_random(S, T, hl, wl, p, l, seed, pair_id, Fa, Ea);
    for (int it = 0; it < iters; ++it) {
        fbo_pm_iteration(S, T, hl, wl, p, l, it, seed, pair_id, Fa, Ea, Fb, Eb);
        int32_t *tf = Fa; Fa = Fb; Fb = tf;
        uint32_t *te = Ea; Ea = Eb; Eb = te;
    }
    *sum = sum_u32(Ea, n);
out:
    free(S); free(T); free(tmp); free(Fa); free(Fb); free(Ea); free(Eb);
    return status;
}

int fbo_patchmatch_raced(const uint8_t *S0, const uint8_t *T0, int h, int w, int p, int levels,
                         int iters, int plain_iters, uint64_t seed, uint32_t pair_id, const int32_t *seed_off,
                         int32_t *F, uint32_t *E, uint64_t *sums, int *rejected)
{
    if (!seed_off || iters < 0 || plain_iters < 0 || levels < 1 || levels > 16 || h < 1 || w < 1 || p < 0)
        return FBO_E_INVALID;
    const int race = iters + 1 < plain_iters ? iters + 1 : plain_iters;
    int st = coarse_energy(S0, T0, h, w, p, levels, iters, seed, pair_id, seed_off, &sums[0]);
    if (st == FBO_OK) st = coarse_energy(S0, T0, h, w, p, levels, race, seed, pair_id, NULL, &sums[1]);
    if (st != FBO_OK) return st;
    *rejected = sums[0] > sums[1];
    if (*rejected) return patchmatch_impl(S0, T0, h, w, p, levels, plain_iters, seed, pair_id, NULL, F, E);
    return patchmatch_impl(S0, T0, h, w, p, levels, iters, seed, pair_id, seed_off, F, E);
}

static int patchmatch_impl(const uint8_t *S0, const uint8_t *T0, int h, int w, int p, int levels,
                           int iters, uint64_t seed, uint32_t pair_id, const int32_t *seed_off,
                           int32_t *F, uint32_t *E)
{
    if (levels < 1 || levels > 16 || h < 1 || w < 1 || p < 0) return FBO_E_INVALID;
    int hs[16], ws[16];
    const uint8_t *Sl[16], *Tl[16];
    uint8_t *own[32];
    int n_own = 0;
    hs[0] = h; ws[0] = w; Sl[0] = S0; Tl[0] = T0;
    for (int l = 1; l < levels; ++l) {
        hs[l] = (hs[l - 1] + 1) / 2;
        ws[l] = (ws[l - 1] + 1) / 2;
        uint8_t *s = (uint8_t *)malloc((size_t)hs[l] * ws[l] * 3);
        uint8_t *t = (uint8_t *)malloc((size_t)hs[l] * ws[l] * 3);
        if (!s || !t) { free(s); free(t); for (int i = 0; i < n_own; ++i) free(own[i]); return FBO_E_ALLOC; }
        fbo_downsample(Sl[l - 1], hs[l - 1], ws[l - 1], s);
        fbo_downsample(Tl[l - 1], hs[l - 1], ws[l - 1], t);
        own[n_own++] = s; own[n_own++] = t;
        Sl[l] = s; Tl[l] = t;
    }
    size_t n0 = (size_t)h * w;
    int32_t *Fa = (int32_t *)malloc(n0 * 2 * sizeof(int32_t));
    int32_t *Fb = (int32_t *)malloc(n0 * 2 * sizeof(int32_t));
    uint32_t *Ea = (uint32_t *)malloc(n0 * sizeof(uint32_t));
    uint32_t *Eb = (uint32_t *)malloc(n0 * sizeof(uint32_t));
    int status = FBO_OK;
    if (!Fa || !Fb || !Ea || !Eb) { status = FBO_E_ALLOC; goto done; }
    for (int l = levels - 1; l >= 0; --l) {
        int hl = hs[l], wl = ws[l];
        if (l == levels - 1) {
            if (seed_off) fbo_nnf_init_offsets(Sl[l], Tl[l], hl, wl, p, seed_off, Fa, Ea);
            else fbo_nnf_init_random(Sl[l], Tl[l], hl, wl, p, l, seed, pair_id, Fa, Ea);
        } else {
            /* the previous level's result sits in Fa; upsample into Fb, then swap */
            fbo_nnf_upsample(Fa, hs[l + 1], ws[l + 1], Sl[l], Tl[l], hl, wl, p, Fb, Eb);
            int32_t *tf = Fa; Fa = Fb; Fb = tf;
            uint32_t *te = Ea; Ea = Eb; Eb = te;
        }
        for (int it = 0; it < iters; ++it) {
            fbo_pm_iteration(Sl[l], Tl[l], hl, wl, p, l, it, seed, pair_id, Fa, Ea, Fb, Eb);
            int32_t *tf = Fa; Fa = Fb; Fb = tf;
            uint32_t *te = Ea; Ea = Eb; Eb = te;
        }
    }
    memcpy(F, Fa, n0 * 2 * sizeof(int32_t));
    memcpy(E, Ea, n0 * sizeof(uint32_t));
done:
    free(Fa); free(Fb); free(Ea); free(Eb);
    for (int i = 0; i < n_own; ++i) free(own[i]);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Memory-efficient remapping (Alg. 2): T^(v) is the average, over the       */
/* offsets d in [-p,p]^2, of S(F(v + d) - d).  Reading at the border: terms  */
/* whose v + d lies outside the image are left out and the sum is divided by */
/* how many remain -- the "average at the overlapping parts" definition in   */
/* Section 3.3; source reads are clamped.  Output in [0, 1] (pixels / 255).  */
/* ------------------------------------------------------------------------ */
void fbo_remap(const uint8_t *style, const int32_t *F, int h, int w, int p, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            long sum[3] = { 0, 0, 0 };
            int cnt = 0;
            for (int dr = -p; dr <= p; ++dr)
                for (int dc = -p; dc <= p; ++dc) {
                    int qr = r + dr, qc = c + dc;
                    if (qr < 0 || qr >= h || qc < 0 || qc >= w) continue;
                    int sr = clampi(F[2 * (qr * w + qc)] - dr, 0, h - 1);
                    int sc = clampi(F[2 * (qr * w + qc) + 1] - dc, 0, w - 1);
                    for (int ch = 0; ch < 3; ++ch) sum[ch] += style[(sr * w + sc) * 3 + ch];
                    ++cnt;
                }
            for (int ch = 0; ch < 3; ++ch)
                out[(r * w + c) * 3 + ch] = (double)sum[ch] / (255.0 * (double)cnt);
        }
}

/* ------------------------------------------------------------------------ */
/* Guide + style loss, Eq. (3) (Section 3.4, after Ebsynth).  For the pair   */
/* (source frame j, target frame i) the loss of target patch v matched to    */
/* source patch u is                                                        */
/*     alpha ||G_j[u] - G_i[v]||^2 + ||S_j[u] - S^_i[v]||^2,                 */
/* where S^_i is the source style S_j remapped through the current field     */
/* (Alg. 2) and is refreshed once at the start of every iteration.          */
/* Readings (the paper gives no precision for S^_i or alpha):               */
/*   S^_i     a uint8 image: each channel of the Alg. 2 average rounded      */
/*            half up, (2 sum + count) / (2 count) in integers;            */
/*   alpha    fixed point, alpha = alpha16 / 16 with 0 <= alpha16 <=        */
/*            fbo_alpha16_max(p), and the loss is scaled by 16 so that it   */
/*            stays an exact integer: L = alpha16 SSD(G_j, G_i) + 16        */
/*            SSD(S_j, S^_i), below 2^32 by the bound on alpha16.          */
/* ------------------------------------------------------------------------ */

/* S^ = Alg. 2 remap of `style` through F, as a uint8 image (rounded). */
void fbo_remap_u8(const uint8_t *style, const int32_t *F, int h, int w, int p, uint8_t *out)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            long sum[3] = { 0, 0, 0 };
            long cnt = 0;
            for (int dr = -p; dr <= p; ++dr)
                for (int dc = -p; dc <= p; ++dc) {
                    int qr = r + dr, qc = c + dc;
                    if (qr < 0 || qr >= h || qc < 0 || qc >= w) continue;
                    int sr = clampi(F[2 * (qr * w + qc)] - dr, 0, h - 1);
                    int sc = clampi(F[2 * (qr * w + qc) + 1] - dc, 0, w - 1);
                    for (int ch = 0; ch < 3; ++ch) sum[ch] += style[(sr * w + sc) * 3 + ch];
                    ++cnt;
                }
            for (int ch = 0; ch < 3; ++ch)
                out[(r * w + c) * 3 + ch] = (uint8_t)((2 * sum[ch] + cnt) / (2 * cnt));
        }
}

/* Eq. (3) for one match, scaled by 16 (see above), exact in 64 bits. */
uint64_t fbo_style_loss(const uint8_t *Gs, const uint8_t *Gt, const uint8_t *Ss, const uint8_t *Sh,
                        int h, int w, int p, int alpha16, int ur, int uc, int vr, int vc)
{
    return (uint64_t)alpha16 * fbo_patch_ssd(Gs, Gt, h, w, p, ur, uc, vr, vc) +
           16u * (uint64_t)fbo_patch_ssd(Ss, Sh, h, w, p, ur, uc, vr, vc);
}

/* Largest alpha16 whose scaled losses (Eq. 3, Eq. 8, Eq. 10) all fit the   */
/* uint32 energies: one patch SSD is at most 3 * 255^2 * (2p+1)^2 (every    */
/* channel difference 255), so the loss is at most (alpha16 + 16) times     */
/* that; alpha16 is further limited to 512 (alpha <= 32).                   */
int fbo_alpha16_max(int p)
{
    const uint64_t ssd_max = 3ull * 255 * 255 * (uint64_t)(2 * p + 1) * (uint64_t)(2 * p + 1);
    const uint64_t a = 0xFFFFFFFFull / ssd_max - 16;
    return a < 512 ? (int)a : 512;
}

/* One iteration under the Eq. (3) loss: S^ is refreshed from the previous   */
/* field Fo (written to Sh), every incumbent's loss is recomputed under it,  */
/* then each pixel tries the same candidate sequence as fbo_pm_iteration.    */
void fbo_pm_iteration_style(const uint8_t *Gs, const uint8_t *Gt, const uint8_t *Ss, int h, int w,
                            int p, int alpha16, int level, int iter, uint64_t seed, uint32_t pair_id,
                            const int32_t *Fo, int32_t *Fn, uint32_t *En, uint8_t *Sh)
{
    static const int D[4][2] = { { -1, 0 }, { 1, 0 }, { 0, -1 }, { 0, 1 } };
    const int R = maxi(h, w);
    fbo_remap_u8(Ss, Fo, h, w, p, Sh);
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            int br = Fo[2 * (r * w + c)], bc = Fo[2 * (r * w + c) + 1];
            uint64_t be = fbo_style_loss(Gs, Gt, Ss, Sh, h, w, p, alpha16, br, bc, r, c);
            for (int k = 0; k < 4; ++k) {
                int qr = r + D[k][0], qc = c + D[k][1];
                if (qr < 0 || qr >= h || qc < 0 || qc >= w) continue;
                int cr = clampi(Fo[2 * (qr * w + qc)] - D[k][0], 0, h - 1);
                int cc = clampi(Fo[2 * (qr * w + qc) + 1] - D[k][1], 0, w - 1);
                uint64_t e = fbo_style_loss(Gs, Gt, Ss, Sh, h, w, p, alpha16, cr, cc, r, c);
                if (e < be) { br = cr; bc = cc; be = e; }
            }
            uint32_t x[4] = { 0, 0, 0, 0 };
            for (int m = 0; (R >> m) >= 1; ++m) {
                int rho = R >> m;
                if ((m & 3) == 0)
                    draw_words(seed, (uint32_t)(r * w + c), pair_id, (uint32_t)level,
                               (uint32_t)iter, (uint32_t)(m >> 2), x);
                uint32_t word = x[m & 3];
                int dr = (int)fbo_uniform16(word & 0xFFFFu, (uint32_t)(2 * rho + 1)) - rho;
                int dc = (int)fbo_uniform16(word >> 16, (uint32_t)(2 * rho + 1)) - rho;
                int cr = clampi(br + dr, 0, h - 1), cc = clampi(bc + dc, 0, w - 1);
                uint64_t e = fbo_style_loss(Gs, Gt, Ss, Sh, h, w, p, alpha16, cr, cc, r, c);
                if (e < be) { br = cr; bc = cc; be = e; }
            }
            Fn[2 * (r * w + c)] = br;
            Fn[2 * (r * w + c) + 1] = bc;
            En[r * w + c] = (uint32_t)be;  /* alpha16 <= fbo_alpha16_max(p): exact */
        }
}

/* NNF(G_j, G_i) under the Eq. (3) loss: Alg. 1 with guide and style         */
/* pyramids (the same 2x2 filter), the same initialisation and upsampling,   */
/* and `iters` >= 1 iterations of fbo_pm_iteration_style per level.  E is    */
/* the loss under the S^ of the last refresh; Sh0 (optional) receives the    */
/* last level-0 S^.                                                          */
int fbo_patchmatch_style(const uint8_t *G0s, const uint8_t *G0t, const uint8_t *S0s, int h, int w,
                         int p, int levels, int iters, uint64_t seed, uint32_t pair_id, int alpha16,
                         int32_t *F, uint32_t *E, uint8_t *Sh0)
{
    if (levels < 1 || levels > 16 || h < 1 || w < 1 || p < 0 || iters < 1 || alpha16 < 0 || alpha16 > fbo_alpha16_max(p))
        return FBO_E_INVALID;
    int hs[16], ws[16];
    const uint8_t *Gs[16], *Gt[16], *Ss[16];
    uint8_t *own[48];
    int n_own = 0;
    hs[0] = h; ws[0] = w; Gs[0] = G0s; Gt[0] = G0t; Ss[0] = S0s;
    for (int l = 1; l < levels; ++l) {
        hs[l] = (hs[l - 1] + 1) / 2;
        ws[l] = (ws[l - 1] + 1) / 2;
        const uint8_t *prev[3] = { Gs[l - 1], Gt[l - 1], Ss[l - 1] };
        uint8_t *next[3];
        for (int k = 0; k < 3; ++k) {
            next[k] = (uint8_t *)malloc((size_t)hs[l] * ws[l] * 3);
            if (!next[k]) { for (int q = 0; q < k; ++q) free(next[q]); for (int i = 0; i < n_own; ++i) free(own[i]); return FBO_E_ALLOC; }
            fbo_downsample(prev[k], hs[l - 1], ws[l - 1], next[k]);
        }
        for (int k = 0; k < 3; ++k) own[n_own++] = next[k];
        Gs[l] = next[0]; Gt[l] = next[1]; Ss[l] = next[2];
    }
    size_t n0 = (size_t)h * w;
    int32_t *Fa = (int32_t *)malloc(n0 * 2 * sizeof(int32_t));
    int32_t *Fb = (int32_t *)malloc(n0 * 2 * sizeof(int32_t));
    uint32_t *Ea = (uint32_t *)malloc(n0 * sizeof(uint32_t));
    uint32_t *Eb = (uint32_t *)malloc(n0 * sizeof(uint32_t));
    uint8_t *Sh = (uint8_t *)malloc(n0 * 3);
    int status = FBO_OK;
    if (!Fa || !Fb || !Ea || !Eb || !Sh) { status = FBO_E_ALLOC; goto done; }
    for (int l = levels - 1; l >= 0; --l) {
        int hl = hs[l], wl = ws[l];
        /* the start of the level (its energies are recomputed by the first iteration) */
        if (l == levels - 1) {
            fbo_nnf_init_random(Gs[l], Gt[l], hl, wl, p, l, seed, pair_id, Fa, Ea);
        } else {
            fbo_nnf_upsample(Fa, hs[l + 1], ws[l + 1], Gs[l], Gt[l], hl, wl, p, Fb, Eb);
            int32_t *tf = Fa; Fa = Fb; Fb = tf;
            uint32_t *te = Ea; Ea = Eb; Eb = te;
        }
        for (int it = 0; it < iters; ++it) {
            fbo_pm_iteration_style(Gs[l], Gt[l], Ss[l], hl, wl, p, alpha16, l, it, seed, pair_id, Fa, Fb, Eb, Sh);
            int32_t *tf = Fa; Fa = Fb; Fb = tf;
            uint32_t *te = Ea; Ea = Eb; Eb = te;
        }
    }
    memcpy(F, Fa, n0 * 2 * sizeof(int32_t));
    memcpy(E, Ea, n0 * sizeof(uint32_t));
    if (Sh0) memcpy(Sh0, Sh, n0 * 3);
done:
    free(Fa); free(Fb); free(Ea); free(Eb); free(Sh);
    for (int i = 0; i < n_own; ++i) free(own[i]);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Sliding-window blending, Eq. (2), balanced mode with the guide-only loss  */
/* (alpha16 < 0) or the Eq. (3) loss:                                        */
/* out_i = mean over j in [max(0,i-M), min(N-1,i+M)] of (S_j -> S_i), where  */
/* S_j -> S_i remaps style frame j with NNF(G_j, G_i) (pair id j*N + i) and  */
/* the j == i term is S_i itself.  Sum in ascending j.                       */
/* ------------------------------------------------------------------------ */
static int blend_window(const uint8_t *guides, const uint8_t *styles, int N, int h, int w, int M,
                        int p, int levels, int iters, uint64_t seed, int alpha16, double *out)
{
    size_t fpix = (size_t)h * w;
    int32_t *F = (int32_t *)malloc(fpix * 2 * sizeof(int32_t));
    uint32_t *E = (uint32_t *)malloc(fpix * sizeof(uint32_t));
    double *tmp = (double *)malloc(fpix * 3 * sizeof(double));
    int status = FBO_OK;
    if (!F || !E || !tmp) { status = FBO_E_ALLOC; goto done; }
    for (int i = 0; i < N; ++i) {
        int lo = maxi(0, i - M), hi = (i + M < N - 1) ? i + M : N - 1;
        double *acc = out + (size_t)i * fpix * 3;
        for (size_t k = 0; k < fpix * 3; ++k) acc[k] = 0.0;
        for (int j = lo; j <= hi; ++j) {
            if (j == i) {
                for (size_t k = 0; k < fpix * 3; ++k) acc[k] += styles[(size_t)i * fpix * 3 + k] / 255.0;
                continue;
            }
            if (alpha16 < 0)
                status = fbo_patchmatch(guides + (size_t)j * fpix * 3, guides + (size_t)i * fpix * 3,
                                        h, w, p, levels, iters, seed, (uint32_t)(j * N + i), NULL, F, E);
            else
                status = fbo_patchmatch_style(guides + (size_t)j * fpix * 3, guides + (size_t)i * fpix * 3,
                                              styles + (size_t)j * fpix * 3, h, w, p, levels, iters, seed,
                                              (uint32_t)(j * N + i), alpha16, F, E, NULL);
            if (status) goto done;
            fbo_remap(styles + (size_t)j * fpix * 3, F, h, w, p, tmp);
            for (size_t k = 0; k < fpix * 3; ++k) acc[k] += tmp[k];
        }
        for (size_t k = 0; k < fpix * 3; ++k) acc[k] /= (double)(hi - lo + 1);
    }
done:
    free(F); free(E); free(tmp);
    return status;
}

int fbo_blend_window(const uint8_t *guides, const uint8_t *styles, int N, int h, int w, int M,
                     int p, int levels, int iters, uint64_t seed, double *out)
{
    return blend_window(guides, styles, N, h, w, M, p, levels, iters, seed, -1, out);
}

/* Eq. (2) with every NNF(G_j, G_i) estimated under the Eq. (3) loss (the    */
/* paper's balanced mode with its improved loss).                            */
int fbo_blend_window_style(const uint8_t *guides, const uint8_t *styles, int N, int h, int w, int M,
                           int p, int levels, int iters, uint64_t seed, int alpha16, double *out)
{
    if (alpha16 < 0) return FBO_E_INVALID;
    return blend_window(guides, styles, N, h, w, M, p, levels, iters, seed, alpha16, out);
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 on a floating-point image X [h][w][3] (a sum of remapped frames,   */
/* as the fast mode remaps them again, Eq. 4-5): out(v) = sum over in-image  */
/* v + d of X(clamp(F(v + d) - d)) / count.                                  */
/* ------------------------------------------------------------------------ */
void fbo_remap_f64(const double *X, const int32_t *F, int h, int w, int p, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            double sum[3] = { 0, 0, 0 };
            int cnt = 0;
            for (int dr = -p; dr <= p; ++dr)
                for (int dc = -p; dc <= p; ++dc) {
                    int qr = r + dr, qc = c + dc;
                    if (qr < 0 || qr >= h || qc < 0 || qc >= w) continue;
                    int sr = clampi(F[2 * (qr * w + qc)] - dr, 0, h - 1);
                    int sc = clampi(F[2 * (qr * w + qc) + 1] - dc, 0, w - 1);
                    for (int ch = 0; ch < 3; ++ch) sum[ch] += X[(sr * w + sc) * 3 + ch];
                    ++cnt;
                }
            for (int ch = 0; ch < 3; ++ch) out[(r * w + c) * 3 + ch] = sum[ch] / (double)cnt;
        }
}

/* ------------------------------------------------------------------------ */
/* Fast mode (Section 3.4, "Efficiency Improvement"): the remapping table   */
/* (Alg. 3), the blending table of its column prefix sums (Alg. 4), the     */
/* interval query (Alg. 5) and the sliding window as a forward and a        */
/* mirrored query (Eq. 6).  Readings where the listings are garbled:        */
/*  - the query steps back by the block it used, i <- i - 2^L, and remaps   */
/*    to S_r (the listing never decrements i and writes S_j);               */
/*  - the block ending at r itself is added without a remap (NNF(G_r, G_r)  */
/*    is the identity; R13's j == i convention);                            */
/*  - blending-table columns run to L = ceil(log2 N) inclusive, the widest  */
/*    block the query can ask for;                                          */
/*  - the mirrored ("symmetric") tables index frames as N - 1 - i;          */
/*  - NNF(G_i, G_j) is the whole coarse-to-fine estimation with pair id     */
/*    i N + j, as everywhere else;                                          */
/*  - identity_nnf != 0 replaces every NNF by the identity field (a test    */
/*    hook: the result must then be the exact window mean).                 */
/* Values are fp64 in [0,1] units (styles / 255); the window sum of Eq. 6   */
/* is divided by the truncated window's length.                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    const uint8_t *guides, *styles;
    int N, h, w, p, levels, iters, identity_nnf;
    uint64_t seed;
    int32_t *F;
    uint32_t *E;
} fast_ctx;

static int fast_nnf(fast_ctx *fc, int src, int tgt)
{
    size_t fpix = (size_t)fc->h * fc->w;
    if (fc->identity_nnf) {
        for (int r = 0; r < fc->h; ++r)
            for (int c = 0; c < fc->w; ++c) {
                fc->F[2 * (r * fc->w + c)] = r;
                fc->F[2 * (r * fc->w + c) + 1] = c;
            }
        return FBO_OK;
    }
    return fbo_patchmatch(fc->guides + (size_t)src * fpix * 3, fc->guides + (size_t)tgt * fpix * 3, fc->h, fc->w,
                          fc->p, fc->levels, fc->iters, fc->seed, (uint32_t)(src * fc->N + tgt), NULL, fc->F, fc->E);
}

/* Blending table BT[k][L] (k in table order, frame = map(k)), L = 0..Lmax. */
static int build_blending_table(fast_ctx *fc, int mirrored, int Lmax, double **BT, double *tmp)
{
    const int N = fc->N;
    size_t n3 = (size_t)fc->h * fc->w * 3;
#define FRAME(k) (mirrored ? N - 1 - (k) : (k))
    /* Alg. 3: RemappingTable(j, L + 1) collects (S_i -> S_j); kept in BT[j][L + 1] */
    for (int j = 0; j < N; ++j)
        for (int L = 0; L <= Lmax; ++L) memset(BT[j * (Lmax + 1) + L], 0, n3 * sizeof(double));
    for (int i = 0; i < N; ++i) {
        int j = i;
        for (int L = 0; L < Lmax; ++L) {
            if (i & (1 << L)) continue;
            j |= 1 << L;
            if (j < N) {
                int st = fast_nnf(fc, FRAME(i), FRAME(j));
                if (st) return st;
                fbo_remap(fc->styles + (size_t)FRAME(i) * n3, fc->F, fc->h, fc->w, fc->p, tmp);
                double *dst = BT[j * (Lmax + 1) + L + 1];
                for (size_t q = 0; q < n3; ++q) dst[q] += tmp[q];
            }
        }
    }
    /* Alg. 4: BlendingTable(i, 0) = S_i, BlendingTable(i, L) = BlendingTable(i, L - 1) + RemappingTable(i, L) */
    for (int i = 0; i < N; ++i) {
        double *b0 = BT[i * (Lmax + 1)];
        const uint8_t *s = fc->styles + (size_t)FRAME(i) * n3;
        for (size_t q = 0; q < n3; ++q) b0[q] = s[q] / 255.0;
        for (int L = 1; L <= Lmax; ++L) {
            double *b = BT[i * (Lmax + 1) + L], *prev = BT[i * (Lmax + 1) + L - 1];
            for (size_t q = 0; q < n3; ++q) b[q] += prev[q];
        }
    }
#undef FRAME
    return FBO_OK;
}

/* Alg. 5 without the final division: A = sum_{i=l}^{r} (S_i -> S_r), in table order. */
static int query_blending_table(fast_ctx *fc, int mirrored, int Lmax, double **BT, int l, int r, double *A,
                                double *tmp)
{
    const int N = fc->N;
    size_t n3 = (size_t)fc->h * fc->w * 3;
    for (size_t q = 0; q < n3; ++q) A[q] = 0.0;
    int i = r;
    while (i >= l) {
        int L = 0;
        while ((i & (1 << L)) && i - (1 << (L + 1)) + 1 >= l) ++L;
        const double *X = BT[i * (Lmax + 1) + L];
        if (i == r) {
            for (size_t q = 0; q < n3; ++q) A[q] += X[q];
        } else {
            int src = mirrored ? N - 1 - i : i, tgt = mirrored ? N - 1 - r : r;
            int st = fast_nnf(fc, src, tgt);
            if (st) return st;
            fbo_remap_f64(X, fc->F, fc->h, fc->w, fc->p, tmp);
            for (size_t q = 0; q < n3; ++q) A[q] += tmp[q];
        }
        i -= 1 << L;
    }
    return FBO_OK;
}

int fbo_blend_window_fast(const uint8_t *guides, const uint8_t *styles, int N, int h, int w, int M, int p,
                          int levels, int iters, uint64_t seed, int identity_nnf, double *out)
{
    if (N < 1 || M < 0 || h < 1 || w < 1) return FBO_E_INVALID;
    int Lmax = 0;
    while ((1 << Lmax) < N) ++Lmax;
    size_t fpix = (size_t)h * w, n3 = fpix * 3;
    fast_ctx fc = { guides, styles, N, h, w, p, levels, iters, identity_nnf, seed, NULL, NULL };
    int status = FBO_OK;
    size_t nbt = (size_t)N * (Lmax + 1);
    double **BT[2] = { (double **)calloc(nbt, sizeof(double *)), (double **)calloc(nbt, sizeof(double *)) };
    double *tmp = (double *)malloc(n3 * sizeof(double));
    double *left = (double *)malloc(n3 * sizeof(double));
    double *right = (double *)malloc(n3 * sizeof(double));
    fc.F = (int32_t *)malloc(fpix * 2 * sizeof(int32_t));
    fc.E = (uint32_t *)malloc(fpix * sizeof(uint32_t));
    if (!BT[0] || !BT[1] || !tmp || !left || !right || !fc.F || !fc.E) { status = FBO_E_ALLOC; goto done; }
    for (int d = 0; d < 2; ++d)
        for (size_t k = 0; k < nbt; ++k)
            if (!(BT[d][k] = (double *)malloc(n3 * sizeof(double)))) { status = FBO_E_ALLOC; goto done; }
    for (int d = 0; d < 2; ++d)
        if ((status = build_blending_table(&fc, d, Lmax, BT[d], tmp))) goto done;
    /* Eq. (6): left half on the forward table, right half on the mirrored one */
    for (int i = 0; i < N; ++i) {
        int lo = maxi(0, i - M), hi = (i + M < N - 1) ? i + M : N - 1;
        if ((status = query_blending_table(&fc, 0, Lmax, BT[0], lo, i, left, tmp))) goto done;
        if ((status = query_blending_table(&fc, 1, Lmax, BT[1], N - 1 - hi, N - 1 - i, right, tmp))) goto done;
        double *o = out + (size_t)i * n3;
        const uint8_t *s = styles + (size_t)i * n3;
        for (size_t q = 0; q < n3; ++q) o[q] = (left[q] + right[q] - s[q] / 255.0) / (double)(hi - lo + 1);
    }
done:
    for (int d = 0; d < 2; ++d) {
        if (BT[d]) for (size_t k = 0; k < nbt; ++k) free(BT[d][k]);
        free(BT[d]);
    }
    free(tmp); free(left); free(right); free(fc.F); free(fc.E);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Accurate mode (Section 3.4, "Quality Improvement", Eq. 7-8).  For target */
/* frame i with window W = [max(0,i-M), min(N-1,i+M)]:                      */
/*  1. T^-_i, the average of the window's style frames remapped to frame i  */
/*     (Eq. 7) with the Eq. 1 NNFs (S_i itself for j == i);                 */
/*  2. every NNF(G_j, G_i), j != i, estimated again under Eq. 8:            */
/*       alpha ||G_j[u] - G_i[v]||^2 + ||S_j[u] - T^-_i[v]||^2;             */
/*  3. the window mean of the styles remapped with the new NNFs (Eq. 2).    */
/* Readings: the guide term uses the guides (the NNF is between guide       */
/* frames) and the alignment term the style frames, the images that are     */
/* averaged; T^-_i is fixed during step 2; it is kept as a uint8 image, the  */
/* exact average rounded half up -- every remap at pixel v has the same     */
/* in-image count c_v, so 255 T^- = (sum of the remaps' integer sums +      */
/* c_v S_i(v)) / (c_v |W|); alpha = alpha16 / 16 and the loss is scaled by  */
/* 16 as in Eq. 3; T^- is downsampled with the pyramid filter for the       */
/* coarser levels; step 2 uses the same pair ids (j N + i) and draws.       */
/* ------------------------------------------------------------------------ */

/* T^- (uint8) of target frame i from the NNFs F[k] of the window's other    */
/* frames js[k] (n of them) and the frame's own style.                      */
void fbo_window_mean_u8(const uint8_t *styles, int i, const int *js, const int32_t *const *F, int n, int h,
                        int w, int p, uint8_t *out)
{
    size_t fpix = (size_t)h * w;
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            long num[3] = { 0, 0, 0 };
            long cnt = 0;
            for (int dr = -p; dr <= p; ++dr)
                for (int dc = -p; dc <= p; ++dc)
                    if (r + dr >= 0 && r + dr < h && c + dc >= 0 && c + dc < w) ++cnt;
            for (int k = 0; k < n; ++k) {
                const uint8_t *S = styles + (size_t)js[k] * fpix * 3;
                for (int dr = -p; dr <= p; ++dr)
                    for (int dc = -p; dc <= p; ++dc) {
                        int qr = r + dr, qc = c + dc;
                        if (qr < 0 || qr >= h || qc < 0 || qc >= w) continue;
                        int sr = clampi(F[k][2 * (qr * w + qc)] - dr, 0, h - 1);
                        int sc = clampi(F[k][2 * (qr * w + qc) + 1] - dc, 0, w - 1);
                        for (int ch = 0; ch < 3; ++ch) num[ch] += S[(sr * w + sc) * 3 + ch];
                    }
            }
            const uint8_t *Si = styles + (size_t)i * fpix * 3 + (r * w + c) * 3;
            long den = cnt * (n + 1);
            for (int ch = 0; ch < 3; ++ch) {
                num[ch] += cnt * Si[ch];
                out[(r * w + c) * 3 + ch] = (uint8_t)((2 * num[ch] + den) / (2 * den));
            }
        }
}

/* One iteration under the Eq. 8 loss against the fixed T^- level Tb: the   */
/* same candidate sequence as fbo_pm_iteration, the incumbent scored under  */
/* the loss.                                                                */
void fbo_pm_iteration_target(const uint8_t *Gs, const uint8_t *Gt, const uint8_t *Ss, const uint8_t *Tb, int h,
                             int w, int p, int alpha16, int level, int iter, uint64_t seed, uint32_t pair_id,
                             const int32_t *Fo, int32_t *Fn, uint32_t *En)
{
    static const int D[4][2] = { { -1, 0 }, { 1, 0 }, { 0, -1 }, { 0, 1 } };
    const int R = maxi(h, w);
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            int br = Fo[2 * (r * w + c)], bc = Fo[2 * (r * w + c) + 1];
            uint64_t be = fbo_style_loss(Gs, Gt, Ss, Tb, h, w, p, alpha16, br, bc, r, c);
            for (int k = 0; k < 4; ++k) {
                int qr = r + D[k][0], qc = c + D[k][1];
                if (qr < 0 || qr >= h || qc < 0 || qc >= w) continue;
                int cr = clampi(Fo[2 * (qr * w + qc)] - D[k][0], 0, h - 1);
                int cc = clampi(Fo[2 * (qr * w + qc) + 1] - D[k][1], 0, w - 1);
                uint64_t e = fbo_style_loss(Gs, Gt, Ss, Tb, h, w, p, alpha16, cr, cc, r, c);
                if (e < be) { br = cr; bc = cc; be = e; }
            }
            uint32_t x[4] = { 0, 0, 0, 0 };
            for (int m = 0; (R >> m) >= 1; ++m) {
                int rho = R >> m;
                if ((m & 3) == 0)
                    draw_words(seed, (uint32_t)(r * w + c), pair_id, (uint32_t)level,
                               (uint32_t)iter, (uint32_t)(m >> 2), x);
                uint32_t word = x[m & 3];
                int dr = (int)fbo_uniform16(word & 0xFFFFu, (uint32_t)(2 * rho + 1)) - rho;
                int dc = (int)fbo_uniform16(word >> 16, (uint32_t)(2 * rho + 1)) - rho;
                int cr = clampi(br + dr, 0, h - 1), cc = clampi(bc + dc, 0, w - 1);
                uint64_t e = fbo_style_loss(Gs, Gt, Ss, Tb, h, w, p, alpha16, cr, cc, r, c);
                if (e < be) { br = cr; bc = cc; be = e; }
            }
            Fn[2 * (r * w + c)] = br;
            Fn[2 * (r * w + c) + 1] = bc;
            En[r * w + c] = (uint32_t)be;  /* alpha16 <= fbo_alpha16_max(p): exact */
        }
}

/* NNF(G_j, G_i) under Eq. 8 against T^- (level-0 Tb0), coarse to fine, with */
/* guide, style and T^- pyramids; iters >= 1.                               */
int fbo_patchmatch_target(const uint8_t *G0s, const uint8_t *G0t, const uint8_t *S0s, const uint8_t *Tb0, int h,
                          int w, int p, int levels, int iters, uint64_t seed, uint32_t pair_id, int alpha16,
                          int32_t *F, uint32_t *E)
{
    if (levels < 1 || levels > 16 || h < 1 || w < 1 || p < 0 || iters < 1 || alpha16 < 0 || alpha16 > fbo_alpha16_max(p))
        return FBO_E_INVALID;
    int hs[16], ws[16];
    const uint8_t *Gs[16], *Gt[16], *Ss[16], *Tb[16];
    uint8_t *own[64];
    int n_own = 0;
    hs[0] = h; ws[0] = w; Gs[0] = G0s; Gt[0] = G0t; Ss[0] = S0s; Tb[0] = Tb0;
    for (int l = 1; l < levels; ++l) {
        hs[l] = (hs[l - 1] + 1) / 2;
        ws[l] = (ws[l - 1] + 1) / 2;
        const uint8_t *prev[4] = { Gs[l - 1], Gt[l - 1], Ss[l - 1], Tb[l - 1] };
        uint8_t *next[4];
        for (int k = 0; k < 4; ++k) {
            next[k] = (uint8_t *)malloc((size_t)hs[l] * ws[l] * 3);
            if (!next[k]) { for (int q = 0; q < k; ++q) free(next[q]); for (int i = 0; i < n_own; ++i) free(own[i]); return FBO_E_ALLOC; }
            fbo_downsample(prev[k], hs[l - 1], ws[l - 1], next[k]);
        }
        for (int k = 0; k < 4; ++k) own[n_own++] = next[k];
        Gs[l] = next[0]; Gt[l] = next[1]; Ss[l] = next[2]; Tb[l] = next[3];
    }
    size_t n0 = (size_t)h * w;
    int32_t *Fa = (int32_t *)malloc(n0 * 2 * sizeof(int32_t));
    int32_t *Fb = (int32_t *)malloc(n0 * 2 * sizeof(int32_t));
    uint32_t *Ea = (uint32_t *)malloc(n0 * sizeof(uint32_t));
    uint32_t *Eb = (uint32_t *)malloc(n0 * sizeof(uint32_t));
    int status = FBO_OK;
    if (!Fa || !Fb || !Ea || !Eb) { status = FBO_E_ALLOC; goto done; }
    for (int l = levels - 1; l >= 0; --l) {
        int hl = hs[l], wl = ws[l];
        if (l == levels - 1) {
            fbo_nnf_init_random(Gs[l], Gt[l], hl, wl, p, l, seed, pair_id, Fa, Ea);
        } else {
            fbo_nnf_upsample(Fa, hs[l + 1], ws[l + 1], Gs[l], Gt[l], hl, wl, p, Fb, Eb);
            int32_t *tf = Fa; Fa = Fb; Fb = tf;
            uint32_t *te = Ea; Ea = Eb; Eb = te;
        }
        for (int it = 0; it < iters; ++it) {
            fbo_pm_iteration_target(Gs[l], Gt[l], Ss[l], Tb[l], hl, wl, p, alpha16, l, it, seed, pair_id, Fa, Fb, Eb);
            int32_t *tf = Fa; Fa = Fb; Fb = tf;
            uint32_t *te = Ea; Ea = Eb; Eb = te;
        }
    }
    memcpy(F, Fa, n0 * 2 * sizeof(int32_t));
    memcpy(E, Ea, n0 * sizeof(uint32_t));
done:
    free(Fa); free(Fb); free(Ea); free(Eb);
    for (int i = 0; i < n_own; ++i) free(own[i]);
    return status;
}

int fbo_blend_window_accurate(const uint8_t *guides, const uint8_t *styles, int N, int h, int w, int M, int p,
                              int levels, int iters, uint64_t seed, int alpha16, double *out, uint8_t *tbar_out)
{
    if (N < 1 || M < 0 || iters < 1 || alpha16 < 0 || alpha16 > fbo_alpha16_max(p)) return FBO_E_INVALID;
    size_t fpix = (size_t)h * w, n3 = fpix * 3;
    int wmax = 2 * M + 1 < N ? 2 * M + 1 : N;
    int32_t **F = (int32_t **)calloc((size_t)wmax, sizeof(int32_t *));
    int *js = (int *)malloc((size_t)wmax * sizeof(int));
    uint32_t *E = (uint32_t *)malloc(fpix * sizeof(uint32_t));
    uint8_t *tb = (uint8_t *)malloc(n3);
    double *tmp = (double *)malloc(n3 * sizeof(double));
    int status = FBO_OK;
    if (!F || !js || !E || !tb || !tmp) { status = FBO_E_ALLOC; goto done; }
    for (int k = 0; k < wmax; ++k)
        if (!(F[k] = (int32_t *)malloc(fpix * 2 * sizeof(int32_t)))) { status = FBO_E_ALLOC; goto done; }
    for (int i = 0; i < N; ++i) {
        int lo = maxi(0, i - M), hi = (i + M < N - 1) ? i + M : N - 1, n = 0;
        const uint8_t *Gi = guides + (size_t)i * n3;
        for (int j = lo; j <= hi; ++j) {
            if (j == i) continue;
            status = fbo_patchmatch(guides + (size_t)j * n3, Gi, h, w, p, levels, iters, seed,
                                    (uint32_t)(j * N + i), NULL, F[n], E);
            if (status) goto done;
            js[n++] = j;
        }
        fbo_window_mean_u8(styles, i, js, (const int32_t *const *)F, n, h, w, p, tb);
        if (tbar_out) memcpy(tbar_out + (size_t)i * n3, tb, n3);
        double *o = out + (size_t)i * n3;
        for (size_t q = 0; q < n3; ++q) o[q] = styles[(size_t)i * n3 + q] / 255.0;
        for (int k = 0; k < n; ++k) {
            int j = js[k];
            status = fbo_patchmatch_target(guides + (size_t)j * n3, Gi, styles + (size_t)j * n3, tb, h, w, p,
                                           levels, iters, seed, (uint32_t)(j * N + i), alpha16, F[k], E);
            if (status) goto done;
            fbo_remap(styles + (size_t)j * n3, F[k], h, w, p, tmp);
            for (size_t q = 0; q < n3; ++q) o[q] += tmp[q];
        }
        for (size_t q = 0; q < n3; ++q) o[q] /= (double)(n + 1);
    }
done:
    if (F) for (int k = 0; k < wmax; ++k) free(F[k]);
    free(F); free(js); free(E); free(tb); free(tmp);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Interpolation extras (Section 3.5): tracking and the pairwise alignment  */
/* loss (Eq. 10).  All NNF(G_k, G_i) of an interpolation (k a bracketing     */
/* key of frame i) are estimated together, level by level and iteration by  */
/* iteration, every pair reading only the previous iteration's fields      */
/* (the concurrent update of Section 3.2 applied across pairs).             */
/*  - tracking: NNF(G_k, G_i) also tries F_{k,i-1}(v) and F_{k,i+1}(v), the */
/*    matches of the pairs with the same key and the neighbouring target    */
/*    frames, when those pairs exist; they come after the 4 propagation     */
/*    candidates and before the random search;                             */
/*  - alignment: for a frame with both keys l and r, the pair (a, i) and    */
/*    its partner (b, i) minimise                                          */
/*       alpha ||G_a[u] - G_i[v]||^2 + ||S_a[u] - S_b[F_b(v)]||^2           */
/*    (S the keyframe styles, F_b the partner's previous field; guide term  */
/*    on guides, alignment on styles as in Eq. 8); the incumbent is scored  */
/*    anew every iteration; alpha = alpha16 / 16, loss x 16, alpha16 >= 1;  */
/*    frames with a single key keep the Eq. 1 loss.                         */
/* ------------------------------------------------------------------------ */
#define FBO_TRACK 1
#define FBO_ALIGN 2

/* One iteration of pair q.  Fo[k] / Eo[k]: previous fields and energies of  */
/* all pairs; prev / next / partner: pair indices or -1.  Gs = G_a (source  */
/* key), Gt = G_i, Ss = S_a and Sp = S_b (keyframe styles at this level).   */
void fbo_pm_iteration_ext(const uint8_t *Gs, const uint8_t *Gt, const uint8_t *Ss, const uint8_t *Sp, int h, int w,
                          int p, int alpha16, int flags, int level, int iter, uint64_t seed, uint32_t pair_id,
                          const int32_t *const *Fo, const uint32_t *const *Eo, int q, int prev, int next,
                          int partner, int32_t *Fn, uint32_t *En)
{
    static const int D[4][2] = { { -1, 0 }, { 1, 0 }, { 0, -1 }, { 0, 1 } };
    const int R = maxi(h, w);
    const int aligned = (flags & FBO_ALIGN) && partner >= 0;
    const int32_t *F = Fo[q];
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < h; ++r)
        for (int c = 0; c < w; ++c) {
            const int v = r * w + c;
            int br = F[2 * v], bc = F[2 * v + 1];
            /* the partner's match fixes this iteration's alignment patch */
            const int pr = aligned ? Fo[partner][2 * v] : 0, pc = aligned ? Fo[partner][2 * v + 1] : 0;
#define LOSS(UR, UC) (aligned ? (uint64_t)alpha16 * fbo_patch_ssd(Gs, Gt, h, w, p, UR, UC, r, c) + \
                                    16u * (uint64_t)fbo_patch_ssd(Ss, Sp, h, w, p, UR, UC, pr, pc) \
                              : (uint64_t)fbo_patch_ssd(Gs, Gt, h, w, p, UR, UC, r, c))
            uint64_t be = aligned ? LOSS(br, bc) : Eo[q][v];
            for (int k = 0; k < 4; ++k) {
                int qr = r + D[k][0], qc = c + D[k][1];
                if (qr < 0 || qr >= h || qc < 0 || qc >= w) continue;
                int cr = clampi(F[2 * (qr * w + qc)] - D[k][0], 0, h - 1);
                int cc = clampi(F[2 * (qr * w + qc) + 1] - D[k][1], 0, w - 1);
                uint64_t e = LOSS(cr, cc);
                if (e < be) { br = cr; bc = cc; be = e; }
            }
            if (flags & FBO_TRACK) {
                const int nb[2] = { prev, next };
                for (int k = 0; k < 2; ++k) {
                    if (nb[k] < 0) continue;
                    int cr = Fo[nb[k]][2 * v], cc = Fo[nb[k]][2 * v + 1];
                    uint64_t e = LOSS(cr, cc);
                    if (e < be) { br = cr; bc = cc; be = e; }
                }
            }
            uint32_t x[4] = { 0, 0, 0, 0 };
            for (int m = 0; (R >> m) >= 1; ++m) {
                int rho = R >> m;
                if ((m & 3) == 0)
                    draw_words(seed, (uint32_t)v, pair_id, (uint32_t)level, (uint32_t)iter, (uint32_t)(m >> 2), x);
                uint32_t word = x[m & 3];
                int dr = (int)fbo_uniform16(word & 0xFFFFu, (uint32_t)(2 * rho + 1)) - rho;
                int dc = (int)fbo_uniform16(word >> 16, (uint32_t)(2 * rho + 1)) - rho;
                int cr = clampi(br + dr, 0, h - 1), cc = clampi(bc + dc, 0, w - 1);
                uint64_t e = LOSS(cr, cc);
                if (e < be) { br = cr; bc = cc; be = e; }
            }
#undef LOSS
            Fn[2 * v] = br;
            Fn[2 * v + 1] = bc;
            En[v] = (uint32_t)be;  /* alpha16 <= fbo_alpha16_max(p): exact */
        }
}

/* Eq. (9) with tracking and / or alignment (flags FBO_TRACK | FBO_ALIGN). */
int fbo_interpolate_ext(const uint8_t *guides, int N, int h, int w, const int32_t *keys, const uint8_t *key_styles,
                        int n_keys, int p, int levels, int iters, uint64_t seed, int alpha16, int flags,
                        double *out)
{
    if (N < 1 || n_keys < 1 || levels < 1 || levels > 16 || iters < 0) return FBO_E_INVALID;
    if ((flags & FBO_ALIGN) && (iters < 1 || alpha16 < 1 || alpha16 > fbo_alpha16_max(p))) return FBO_E_INVALID;
    size_t fpix = (size_t)h * w, n3 = fpix * 3;
    int hs[16], ws[16];
    hs[0] = h; ws[0] = w;
    for (int l = 1; l < levels; ++l) { hs[l] = (hs[l - 1] + 1) / 2; ws[l] = (ws[l - 1] + 1) / 2; }
    /* pairs: (key index, frame) with the same order as the plain interpolation */
    int *pk = (int *)malloc(sizeof(int) * 2 * (size_t)N), *pf = (int *)malloc(sizeof(int) * 2 * (size_t)N);
    int *kself = (int *)malloc(sizeof(int) * (size_t)N), *kl = (int *)malloc(sizeof(int) * (size_t)N);
    int *kr = (int *)malloc(sizeof(int) * (size_t)N);
    int np = 0, status = FBO_OK;
    uint8_t **G = (uint8_t **)calloc((size_t)N * levels, sizeof(uint8_t *));
    uint8_t **KS = (uint8_t **)calloc((size_t)n_keys * levels, sizeof(uint8_t *));
    int32_t **Fa = NULL, **Fb = NULL;
    uint32_t **Ea = NULL, **Eb = NULL;
    int *prev = NULL, *next = NULL, *partner = NULL;
    double *tmp = (double *)malloc(n3 * sizeof(double));
    if (!pk || !pf || !kself || !kl || !kr || !G || !KS || !tmp) { status = FBO_E_ALLOC; goto done; }
    for (int i = 0; i < N; ++i) {
        kself[i] = kl[i] = kr[i] = -1;
        for (int k = 0; k < n_keys; ++k) {
            if (keys[k] == i) kself[i] = k;
            if (keys[k] < i) kl[i] = k;
            if (keys[k] > i && kr[i] < 0) kr[i] = k;
        }
        if (kself[i] >= 0) continue;
        if (kl[i] >= 0) { pk[np] = kl[i]; pf[np] = i; ++np; }
        if (kr[i] >= 0) { pk[np] = kr[i]; pf[np] = i; ++np; }
    }
    /* pyramids of every guide frame and every keyframe style */
    for (int i = 0; i < N; ++i) {
        G[(size_t)i * levels] = (uint8_t *)(guides + (size_t)i * n3);
        for (int l = 1; l < levels; ++l) {
            uint8_t *d = (uint8_t *)malloc((size_t)hs[l] * ws[l] * 3);
            if (!d) { status = FBO_E_ALLOC; goto done; }
            fbo_downsample(G[(size_t)i * levels + l - 1], hs[l - 1], ws[l - 1], d);
            G[(size_t)i * levels + l] = d;
        }
    }
    for (int k = 0; k < n_keys; ++k) {
        KS[(size_t)k * levels] = (uint8_t *)(key_styles + (size_t)k * n3);
        for (int l = 1; l < levels; ++l) {
            uint8_t *d = (uint8_t *)malloc((size_t)hs[l] * ws[l] * 3);
            if (!d) { status = FBO_E_ALLOC; goto done; }
            fbo_downsample(KS[(size_t)k * levels + l - 1], hs[l - 1], ws[l - 1], d);
            KS[(size_t)k * levels + l] = d;
        }
    }
    Fa = (int32_t **)calloc((size_t)np + 1, sizeof(int32_t *));
    Fb = (int32_t **)calloc((size_t)np + 1, sizeof(int32_t *));
    Ea = (uint32_t **)calloc((size_t)np + 1, sizeof(uint32_t *));
    Eb = (uint32_t **)calloc((size_t)np + 1, sizeof(uint32_t *));
    prev = (int *)malloc(sizeof(int) * ((size_t)np + 1));
    next = (int *)malloc(sizeof(int) * ((size_t)np + 1));
    partner = (int *)malloc(sizeof(int) * ((size_t)np + 1));
    if (!Fa || !Fb || !Ea || !Eb || !prev || !next || !partner) { status = FBO_E_ALLOC; goto done; }
    for (int q = 0; q < np; ++q) {
        Fa[q] = (int32_t *)malloc(fpix * 2 * sizeof(int32_t));
        Fb[q] = (int32_t *)malloc(fpix * 2 * sizeof(int32_t));
        Ea[q] = (uint32_t *)malloc(fpix * sizeof(uint32_t));
        Eb[q] = (uint32_t *)malloc(fpix * sizeof(uint32_t));
        if (!Fa[q] || !Fb[q] || !Ea[q] || !Eb[q]) { status = FBO_E_ALLOC; goto done; }
        prev[q] = next[q] = partner[q] = -1;
        for (int t = 0; t < np; ++t) {
            if (pk[t] == pk[q] && pf[t] == pf[q] - 1) prev[q] = t;
            if (pk[t] == pk[q] && pf[t] == pf[q] + 1) next[q] = t;
            if (t != q && pf[t] == pf[q]) partner[q] = t;
        }
    }
    for (int l = levels - 1; l >= 0; --l) {
        int hl = hs[l], wl = ws[l];
        for (int q = 0; q < np; ++q) {
            const uint8_t *Gs = G[(size_t)keys[pk[q]] * levels + l], *Gt = G[(size_t)pf[q] * levels + l];
            uint32_t pid = (uint32_t)(keys[pk[q]] * N + pf[q]);
            if (l == levels - 1) {
                fbo_nnf_init_random(Gs, Gt, hl, wl, p, l, seed, pid, Fa[q], Ea[q]);
            } else {
                fbo_nnf_upsample(Fa[q], hs[l + 1], ws[l + 1], Gs, Gt, hl, wl, p, Fb[q], Eb[q]);
                int32_t *tf = Fa[q]; Fa[q] = Fb[q]; Fb[q] = tf;
                uint32_t *te = Ea[q]; Ea[q] = Eb[q]; Eb[q] = te;
            }
        }
        for (int it = 0; it < iters; ++it) {
            for (int q = 0; q < np; ++q) {
                const uint8_t *Gs = G[(size_t)keys[pk[q]] * levels + l], *Gt = G[(size_t)pf[q] * levels + l];
                const uint8_t *Ss = KS[(size_t)pk[q] * levels + l];
                const uint8_t *Sp = partner[q] >= 0 ? KS[(size_t)pk[partner[q]] * levels + l] : Ss;
                fbo_pm_iteration_ext(Gs, Gt, Ss, Sp, hl, wl, p, alpha16, flags, l, it, seed,
                                     (uint32_t)(keys[pk[q]] * N + pf[q]), (const int32_t *const *)Fa,
                                     (const uint32_t *const *)Ea, q, prev[q], next[q], partner[q], Fb[q], Eb[q]);
            }
            for (int q = 0; q < np; ++q) {
                int32_t *tf = Fa[q]; Fa[q] = Fb[q]; Fb[q] = tf;
                uint32_t *te = Ea[q]; Ea[q] = Eb[q]; Eb[q] = te;
            }
        }
    }
    /* Eq. (9) with the final fields */
    for (int i = 0, q = 0; i < N; ++i) {
        double *o = out + (size_t)i * n3;
        if (kself[i] >= 0) {
            for (size_t t = 0; t < n3; ++t) o[t] = key_styles[(size_t)kself[i] * n3 + t] / 255.0;
            continue;
        }
        for (size_t t = 0; t < n3; ++t) o[t] = 0.0;
        const int both = kl[i] >= 0 && kr[i] >= 0;
        for (int side = 0; side < 2; ++side) {
            int k = side == 0 ? kl[i] : kr[i];
            if (k < 0) continue;
            double wgt = 1.0;
            if (both) {
                int lk = keys[kl[i]], rk = keys[kr[i]];
                wgt = side == 0 ? (double)(rk - i) / (double)(rk - lk) : (double)(i - lk) / (double)(rk - lk);
            }
            fbo_remap(key_styles + (size_t)k * n3, Fa[q], h, w, p, tmp);
            for (size_t t = 0; t < n3; ++t) o[t] += wgt * tmp[t];
            ++q;
        }
    }
done:
    if (G) for (int i = 0; i < N; ++i) for (int l = 1; l < levels; ++l) free(G[(size_t)i * levels + l]);
    if (KS) for (int k = 0; k < n_keys; ++k) for (int l = 1; l < levels; ++l) free(KS[(size_t)k * levels + l]);
    if (Fa) for (int q = 0; q < np; ++q) { free(Fa[q]); free(Fb[q]); free(Ea[q]); free(Eb[q]); }
    free(G); free(KS); free(Fa); free(Fb); free(Ea); free(Eb); free(prev); free(next); free(partner);
    free(pk); free(pf); free(kself); free(kl); free(kr); free(tmp);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Keyframe interpolation, Eq. (9): for l < i < r (l, r the bracketing keys) */
/* out_i = (r-i)/(r-l) (S_l -> S_i) + (i-l)/(r-l) (S_r -> S_i); keyframes    */
/* are passed through unchanged (Section 3.5).  Reading for frames before    */
/* the first or after the last key: the single nearest key, weight 1.        */
/* keys: sorted, unique, n_keys >= 1; key_styles[k] belongs to keys[k].      */
/* ------------------------------------------------------------------------ */
int fbo_interpolate(const uint8_t *guides, int N, int h, int w, const int32_t *keys,
                    const uint8_t *key_styles, int n_keys, int p, int levels, int iters,
                    uint64_t seed, double *out)
{
    size_t fpix = (size_t)h * w;
    int32_t *F = (int32_t *)malloc(fpix * 2 * sizeof(int32_t));
    uint32_t *E = (uint32_t *)malloc(fpix * sizeof(uint32_t));
    double *tmp = (double *)malloc(fpix * 3 * sizeof(double));
    int status = FBO_OK;
    if (!F || !E || !tmp) { status = FBO_E_ALLOC; goto done; }
    for (int i = 0; i < N; ++i) {
        double *o = out + (size_t)i * fpix * 3;
        int kl = -1, kr = -1, ki = -1;
        for (int k = 0; k < n_keys; ++k) {
            if (keys[k] == i) ki = k;
            if (keys[k] < i) kl = k;
            if (keys[k] > i && kr < 0) kr = k;
        }
        if (ki >= 0) {
            for (size_t k = 0; k < fpix * 3; ++k) o[k] = key_styles[(size_t)ki * fpix * 3 + k] / 255.0;
            continue;
        }
        for (size_t k = 0; k < fpix * 3; ++k) o[k] = 0.0;
        int sides[2] = { kl, kr };
        for (int s = 0; s < 2; ++s) {
            int k = sides[s];
            if (k < 0) continue;
            double wgt = 1.0;
            if (kl >= 0 && kr >= 0) {
                int l = keys[kl], r = keys[kr];
                wgt = (s == 0) ? (double)(r - i) / (double)(r - l) : (double)(i - l) / (double)(r - l);
            }
            status = fbo_patchmatch(guides + (size_t)keys[k] * fpix * 3, guides + (size_t)i * fpix * 3,
                                    h, w, p, levels, iters, seed, (uint32_t)(keys[k] * N + i), NULL, F, E);
            if (status) goto done;
            fbo_remap(key_styles + (size_t)k * fpix * 3, F, h, w, p, tmp);
            for (size_t q = 0; q < fpix * 3; ++q) o[q] += wgt * tmp[q];
        }
    }
done:
    free(F); free(E); free(tmp);
    return status;
}
