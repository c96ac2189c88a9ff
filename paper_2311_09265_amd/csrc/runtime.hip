// Host runtime of the FastBlend library: the C ABI of include/fastblend.h.
//
// Every call is turned into a Plan: a list of stream-ordered kernel launches
// plus one table of launch descriptors (PMJob / RemapTerm / RemapFrame)
// uploaded to device memory in a single copy.  Batched PatchMatch plans
// group all pairs that sit at the same pyramid level into one launch per
// step (start of level, each iteration), the pairs' tiles forming one flat
// list, so a 290-pair window fills all 256 CUs with ~300k workgroups.
//
// Plans are rebuilt on the host at every call (microseconds); the device
// table is re-uploaded only when its bytes change, and with FB_USE_GRAPH the
// launch list is captured once into a HIP graph and replayed while the plan
// stays the same.  The autotuner times the finest-level iteration launch of
// a batch with every tile shape once per batch shape and keeps the fastest;
// tile shapes never change results.
#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fastblend.h"
#include "fb_common.h"

using namespace fb;

namespace {

thread_local std::string g_err;

fb_status fail(fb_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define FB_HIP(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(FB_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

struct Buf {
    void *p = nullptr;
    size_t n = 0;
};

struct Op {
    int kind;  // FB_KERNEL_*
    std::function<hipError_t(hipStream_t, const uint8_t *)> fn;
};

struct Plan {
    std::vector<uint8_t> table;  // host image of the device tables
    std::vector<Op> ops;
    std::string sig;             // every kernel argument not in the table
    // autotuning: the finest-level iteration launch of a PatchMatch batch
    bool has_tune = false;
    std::vector<PMJob> tune_jobs;
    int tune_iter = 0;
    int tune_mode = kIterPlain;
    std::string tune_key;
};

template <class T>
size_t table_append(Plan &P, const T *data, size_t n) {
    const size_t off = (P.table.size() + 255) & ~(size_t)255;
    P.table.resize(off + n * sizeof(T));
    if (n) std::memcpy(P.table.data() + off, data, n * sizeof(T));
    return off;
}

void sig_add(Plan &P, const char *tag, long long a, long long b = 0, long long c = 0,
             long long d = 0) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s:%lld:%lld:%lld:%lld;", tag, a, b, c, d);
    P.sig += buf;
}

void assign_tiles(std::vector<PMJob> &jobs, TileCfg cfg, int *total, int *uniform) {
    int base = 0, uni = -1;
    for (PMJob &j : jobs) {
        const int tx = (j.w + cfg.tw - 1) / cfg.tw, ty = (j.h + cfg.th - 1) / cfg.th;
        j.tiles_x = tx;
        j.tile_base = base;
        base += tx * ty;
        if (uni == -1) uni = tx * ty;
        else if (uni != tx * ty) uni = 0;
    }
    *total = base;
    *uniform = uni > 0 ? uni : 0;
}

enum LaunchKind { kLaunchStart, kLaunchIter, kLaunchStyleRefresh, kLaunchExport, kLaunchEnergySum,
                  kLaunchGuardSelect };

// LDS an iteration launch stages: the largest source bound table of its jobs
int max_tab_bytes(const std::vector<PMJob> &jobs) {
    int n = 0;
    for (const PMJob &j : jobs) n = std::max(n, j.tab_n);
    return (n * 12 + 15) & ~15;  // staged with 16-byte loads
}

void add_pm_launch(Plan &P, LaunchKind kind, std::vector<PMJob> jobs, TileCfg cfg, int p,
                   uint64_t seed, int iter, int mode = kIterPlain) {
    if (jobs.empty()) return;
    int total = 0, uniform = 0;
    assign_tiles(jobs, cfg, &total, &uniform);
    const size_t off = table_append(P, jobs.data(), jobs.size());
    const int n = (int)jobs.size();
    sig_add(P, "pm", kind * 16 + mode, (long long)off, n, ((long long)iter << 32) | (cfg.tw << 8) | cfg.th);
    switch (kind) {
    case kLaunchStart:
        P.ops.push_back({FB_KERNEL_PM_START, [=](hipStream_t s, const uint8_t *tab) {
            return launch_pm_start(reinterpret_cast<const PMJob *>(tab + off), n, total, uniform,
                                   cfg, p, seed, s);
        }});
        break;
    case kLaunchIter: {
        const int tab_bytes = max_tab_bytes(jobs);
        bool guarded = true;  // every job runs only for one outcome of the guard
        for (const PMJob &j : jobs) guarded &= j.guard_when != 0;
        P.ops.push_back({FB_KERNEL_PM_ITER, [=](hipStream_t s, const uint8_t *tab) {
            return launch_pm_iter(reinterpret_cast<const PMJob *>(tab + off), n, total, uniform,
                                  cfg, p, iter, seed, mode, tab_bytes, s, guarded);
        }});
        break;
    }
    case kLaunchStyleRefresh:
        P.ops.push_back({FB_KERNEL_STYLE, [=](hipStream_t s, const uint8_t *tab) {
            return launch_style_refresh(reinterpret_cast<const PMJob *>(tab + off), n, total, uniform,
                                        cfg, p, s);
        }});
        break;
    case kLaunchExport:
        P.ops.push_back({FB_KERNEL_PM_EXPORT, [=](hipStream_t s, const uint8_t *tab) {
            return launch_pm_export(reinterpret_cast<const PMJob *>(tab + off), n, total, uniform,
                                    cfg, s);
        }});
        break;
    case kLaunchEnergySum:
        P.ops.push_back({FB_KERNEL_OTHER, [=](hipStream_t s, const uint8_t *tab) {
            return launch_energy_sum(reinterpret_cast<const PMJob *>(tab + off), n, total, uniform, cfg, s);
        }});
        break;
    case kLaunchGuardSelect:
        P.ops.push_back({FB_KERNEL_OTHER, [=](hipStream_t s, const uint8_t *tab) {
            return launch_guard_select(reinterpret_cast<const PMJob *>(tab + off), n, total, uniform, cfg, s);
        }});
        break;
    }
}

// The guard's decision: one thread per raced pair sets the call's any-rejected
// word when the pair's seeded sum exceeds its plain sum.
void add_guard_decide(Plan &P, const std::vector<PMJob> &dec) {
    if (dec.empty()) return;
    const size_t off = table_append(P, dec.data(), dec.size());
    const int n = (int)dec.size();
    sig_add(P, "gdec", (long long)off, n);
    P.ops.push_back({FB_KERNEL_OTHER, [=](hipStream_t s, const uint8_t *tab) {
        return launch_guard_decide(reinterpret_cast<const PMJob *>(tab + off), n, s);
    }});
}

// Frames of a call: n uint8 RGB frames, each with its own pointer and row
// stride (the contiguous calls pass [n][h][w][3]).
typedef std::vector<FrameRef> Frames;

Frames contiguous_frames(const uint8_t *base, int n, int h, int w) {
    Frames f((size_t)n);
    for (int k = 0; k < n; ++k) f[k] = FrameRef{base + (size_t)k * h * w * 3, (int64_t)w * 3};
    return f;
}

// Pyramids of the frames into dst[f * stride].  Pyramids whose frames are
// never a PatchMatch source (styles, T^-) skip the bound tables (tables =
// false).
void plan_pyramids(Plan &P, const Frames &frames, int h, int w, const PyrLayout &L,
                   uint8_t *dst, size_t stride, bool tables = true) {
    const int p = L.p, n = (int)frames.size();
    const size_t foff = table_append(P, frames.data(), frames.size());
    sig_add(P, tables ? "pyr" : "pyr-nt", (long long)foff, n, ((long long)h << 32) | w,
            (long long)(uintptr_t)dst + L.levels);
    P.ops.push_back({FB_KERNEL_PYRAMID, [=](hipStream_t s, const uint8_t *tab) {
        hipError_t e = launch_pack_rgbx(reinterpret_cast<const FrameRef *>(tab + foff), FrameRef{}, n, h, w, p, dst,
                                        stride, L.lv[0].px_off, L.lv[0].pitch, s);
        for (int l = 1; l < L.levels && e == hipSuccess; ++l)
            e = launch_downsample(dst, stride, n, L.lv[l - 1], L.lv[l], p, s);
        if (e == hipSuccess && tables) e = launch_bound_tables(dst, stride, n, L, s);
        return e;
    }});
}

// Padded 4-byte pixels of the style frames.
void plan_style_pack(Plan &P, const Frames &frames, int h, int w, int p, uint8_t *dst, size_t stride,
                     int pitch) {
    const int n = (int)frames.size();
    const size_t foff = table_append(P, frames.data(), frames.size());
    sig_add(P, "sty", (long long)foff, n, ((long long)h << 32) | w, (long long)(uintptr_t)dst);
    P.ops.push_back({FB_KERNEL_PYRAMID, [=](hipStream_t s, const uint8_t *tab) {
        return launch_pack_rgbx(reinterpret_cast<const FrameRef *>(tab + foff), FrameRef{}, n, h, w, p, dst, stride,
                                0, pitch, s);
    }});
}

struct PairSpec {
    const uint8_t *src_pyr, *tgt_pyr;
    PyrLayout L;               // L.levels: this pair's pyramid levels
    uint32_t pair_id;
    const int32_t *seed_offsets;
    uint32_t *f[2], *e[2];     // ping-pong buffers (level-0 capacity)
    int32_t *nnf_abi;          // optional export of the final field
    uint32_t *energy_abi;
    const uint8_t *src_sty_pyr;  // Eq. 3 / Eq. 8 loss: pyramid of the source style frame
    uint32_t *sty_hat;         // Eq. 3 loss: padded S^ buffer (level-0 capacity)
    const uint8_t *tbar_pyr;   // Eq. 8 loss: pyramid of the fixed target T^- (instead of S^)
    int trk_prev = -1, trk_next = -1;  // tracking: pairs with the same source, adjacent targets
    int partner = -1;                  // Eq. 10: the pair it is aligned with
    const uint8_t *partner_sty_pyr = nullptr;  // Eq. 10: the partner's source style pyramid
    int final_buf;             // filled by the planner
    // guard of a seeded pair: its index among the call's guarded pairs (-1:
    // none) and the plain run's ping-pong buffers at its coarsest level
    int guard_slot = -1;
    uint32_t *rf[2] = {nullptr, nullptr}, *re[2] = {nullptr, nullptr};
};

// The guard of the seeded pairs of one call: each pair with guard_slot >= 0
// races its seeded coarsest level (iters iterations) against the plain random
// start (min(iters + 1, plain_iters) iterations); sums[2 g], sums[2 g + 1]
// receive the two summed energies of guarded pair g, and sums[2 n] is set
// when any seed is rejected.  A rejected pair continues as the plain run
// (plain_iters iterations at every level).
struct GuardPlan {
    int plain_iters = 0;
    uint64_t *sums = nullptr;
    int n = 0;
};

PMJob job_geom(const PairSpec &ps, int l) {
    PMJob j;
    std::memset(&j, 0, sizeof j);
    const LevelGeom &g = ps.L.lv[l];
    j.src_px = reinterpret_cast<const uint32_t *>(ps.src_pyr + g.px_off);
    j.tgt_px = reinterpret_cast<const uint32_t *>(ps.tgt_pyr + g.px_off);
    j.h = g.h;
    j.w = g.w;
    j.pitch = g.pitch;
    j.pair_id = ps.pair_id;
    j.level = l;
    j.btab = reinterpret_cast<const uint32_t *>(ps.src_pyr + g.tab_off);
    j.tab_shift = g.tab_shift;
    j.tab_w = g.tab_w;
    j.tab_n = g.tab_w * g.tab_h;
    j.psum = reinterpret_cast<const uint32_t *>(ps.src_pyr + g.sum_off);
    j.psum_shift = psum_shift(ps.L.p);
    if (ps.src_sty_pyr) {
        j.src_sty = reinterpret_cast<const uint32_t *>(ps.src_sty_pyr + g.px_off);
        // the iteration only reads sty_hat; T^- is never written
        j.sty_hat = ps.tbar_pyr ? const_cast<uint32_t *>(reinterpret_cast<const uint32_t *>(ps.tbar_pyr + g.px_off))
                                : ps.sty_hat;
    }
    return j;
}

std::string tune_key_of(const std::vector<PairSpec> &pairs, int p) {
    std::string k = "p" + std::to_string(p);
    int run = 0, ph = -1, pw = -1;
    auto flush = [&]() {
        if (run) k += ";" + std::to_string(ph) + "x" + std::to_string(pw) + "*" + std::to_string(run);
    };
    for (const PairSpec &ps : pairs) {
        if (ps.L.lv[0].h != ph || ps.L.lv[0].w != pw) {
            flush();
            ph = ps.L.lv[0].h;
            pw = ps.L.lv[0].w;
            run = 0;
        }
        ++run;
    }
    flush();
    return k;
}

// The whole coarse-to-fine PatchMatch of every pair (Algorithm 1), grouped by
// level: a pair with K levels joins at pass Kmax - K, so at every pass all
// active pairs sit at the same level number.  With the Eq. 3 loss (style),
// every iteration launch is preceded by the refresh of the pairs' S^ from the
// field the iteration starts from.  With the Eq. 8 loss (style and
// fixed_target) the second patch is each pair's fixed T^-: no refresh.
// Tracking (track) and the pairwise alignment loss (align, pairs with a
// partner) read the fields the other pairs start the same iteration from.
// With a guard (plain passes only), every guarded pair also runs the plain
// random start at its coarsest level in its own buffers; once both runs of
// the race are done the two levels' energies are summed; the plain run's
// later iterations there, and plain_iters iterations at the finer levels,
// run only for a rejected seed, which then takes the plain field (launch
// jobs that only run for a rejected or only for a kept seed), so the launch
// sequence is the same whatever the outcome.
void plan_patchmatch(Plan &P, std::vector<PairSpec> &pairs, int iters, int p, uint64_t seed,
                     TileCfg cfg, bool style = false, int alpha16 = 0, bool fixed_target = false,
                     bool track = false, bool align = false, const GuardPlan *guard = nullptr) {
    int kmax = 0;
    for (const PairSpec &ps : pairs) kmax = std::max(kmax, ps.L.levels);
    const bool guarded = guard && guard->n > 0;
    const int plain_iters = guarded ? guard->plain_iters : iters;
    const int it_common = std::min(iters, plain_iters), it_all = std::max(iters, plain_iters);
    // the race: the plain start gets one iteration more than the seed; the
    // decision is taken once both runs of the race are done, and the plain
    // run's remaining coarsest-level iterations run only for a rejected seed
    const int race_iters = std::min(iters + 1, plain_iters), it_dec = std::max(iters, race_iters);
    if (guarded) {
        uint64_t *sums = guard->sums;
        const long n4 = 4L * guard->n + 2;  // two uint64 per pair and the any-rejected word, cleared as floats
        sig_add(P, "gclr", (long long)(uintptr_t)sums, n4);
        P.ops.push_back({FB_KERNEL_OTHER, [=](hipStream_t s, const uint8_t *) {
            return launch_fill_zero(reinterpret_cast<float *>(sums), n4, s);
        }});
    }
    std::vector<int> cur(pairs.size(), 0), rcur(pairs.size(), 0);
    for (int t = 0; t < kmax; ++t) {
        const int l = kmax - 1 - t;
        std::vector<size_t> active;
        bool any_guard = false, any_race = false;
        for (size_t k = 0; k < pairs.size(); ++k)
            if (pairs[k].L.levels > l) {
                active.push_back(k);
                any_guard |= pairs[k].guard_slot >= 0;
                any_race |= pairs[k].guard_slot >= 0 && l == pairs[k].L.levels - 1;
            }
        if (active.empty()) continue;
        auto gsum = [&](const PairSpec &ps) { return guard->sums + 2 * ps.guard_slot; };
        uint64_t *gany = guarded ? guard->sums + 2 * guard->n : nullptr;
        std::vector<PMJob> js;
        for (size_t k : active) {
            PairSpec &ps = pairs[k];
            PMJob j = job_geom(ps, l);
            int dst;
            if (l == ps.L.levels - 1) {
                j.mode = ps.seed_offsets ? kStartOffsets : kStartRandom;
                j.aux_off = ps.seed_offsets;
                dst = 0;
                if (ps.guard_slot >= 0) {  // the plain run it races
                    PMJob r = job_geom(ps, l);
                    r.mode = kStartRandom;
                    r.f_out = ps.rf[0];
                    r.e_out = ps.re[0];
                    rcur[k] = 0;
                    js.push_back(r);
                }
            } else {
                j.mode = kStartUpsample;
                j.f_in = ps.f[cur[k]];
                j.hc = ps.L.lv[l + 1].h;
                j.wc = ps.L.lv[l + 1].w;
                dst = cur[k] ^ 1;
            }
            j.f_out = ps.f[dst];
            j.e_out = ps.e[dst];
            cur[k] = dst;
            rcur[k] = ps.guard_slot >= 0 && l < ps.L.levels - 1 ? dst : rcur[k];
            js.push_back(j);
        }
        add_pm_launch(P, kLaunchStart, js, cfg, p, seed, 0);
        const int its = any_guard ? it_all : iters;
        // the race's outcome for the pairs at their coarsest level: both
        // summed energies, then the any-rejected word
        bool decided = false;
        auto decide = [&]() {
            std::vector<PMJob> sums, dec;
            for (size_t k : active) {
                PairSpec &ps = pairs[k];
                if (ps.guard_slot < 0 || l != ps.L.levels - 1) continue;
                PMJob a = job_geom(ps, l), b = job_geom(ps, l), d = job_geom(ps, l);
                a.e_in = ps.e[cur[k]];
                a.guard = gsum(ps);
                b.e_in = ps.re[rcur[k]];
                b.guard = gsum(ps) + 1;
                d.guard = gsum(ps);
                d.guard_any = gany;
                sums.push_back(a);
                sums.push_back(b);
                dec.push_back(d);
            }
            add_pm_launch(P, kLaunchEnergySum, sums, cfg, p, seed, 0);
            add_guard_decide(P, dec);
            decided = true;
        };
        for (int it = 0; it < its; ++it) {
            if (any_race && it == it_dec) decide();
            if (style && !fixed_target) {
                js.clear();
                for (size_t k : active) {
                    PMJob j = job_geom(pairs[k], l);
                    j.f_in = pairs[k].f[cur[k]];
                    // after the level's first iteration the other buffer still holds
                    // the field the previous refresh used
                    if (it > 0) j.f_prev = pairs[k].f[cur[k] ^ 1];
                    js.push_back(j);
                }
                add_pm_launch(P, kLaunchStyleRefresh, js, cfg, p, seed, it);
            }
            // every pair reads the fields all pairs start this iteration from
            std::vector<const uint32_t *> fin(pairs.size(), nullptr);
            for (size_t k : active) fin[k] = pairs[k].f[cur[k]];
            std::vector<PMJob> js_style, js_plain;
            for (size_t k : active) {
                PairSpec &ps = pairs[k];
                PMJob j = job_geom(ps, l);
                j.alpha16 = alpha16;
                if (ps.guard_slot >= 0) {
                    if (l == ps.L.levels - 1) {
                        // coarsest level: the seeded run and the plain run, side by side
                        if (it < plain_iters) {
                            PMJob r = job_geom(ps, l);
                            r.f_in = ps.rf[rcur[k]];
                            r.e_in = ps.re[rcur[k]];
                            r.f_out = ps.rf[rcur[k] ^ 1];
                            r.e_out = ps.re[rcur[k] ^ 1];
                            if (it >= race_iters) {  // past the race: only a rejected seed needs it
                                r.guard = gsum(ps);
                                r.guard_any = gany;
                                r.guard_when = 1;
                            }
                            rcur[k] ^= 1;
                            js_plain.push_back(r);
                        }
                        if (it >= iters) continue;
                        j.f_in = ps.f[cur[k]];
                        j.e_in = ps.e[cur[k]];
                        j.f_out = ps.f[cur[k] ^ 1];
                        j.e_out = ps.e[cur[k] ^ 1];
                        cur[k] ^= 1;
                    } else if (it < it_common) {
                        j.f_in = ps.f[cur[k]];
                        j.e_in = ps.e[cur[k]];
                        j.f_out = ps.f[cur[k] ^ 1];
                        j.e_out = ps.e[cur[k] ^ 1];
                        cur[k] ^= 1;
                        rcur[k] = cur[k];
                    } else {
                        // the longer of the two runs: rcur follows the plain run
                        const bool plain_longer = plain_iters > iters;
                        int &c = plain_longer ? rcur[k] : cur[k];
                        j.f_in = ps.f[c];
                        j.e_in = ps.e[c];
                        j.f_out = ps.f[c ^ 1];
                        j.e_out = ps.e[c ^ 1];
                        j.guard = gsum(ps);
                        j.guard_any = gany;
                        j.guard_when = plain_longer ? 1 : 2;
                        c ^= 1;
                    }
                    js_plain.push_back(j);
                    continue;
                }
                if (it >= iters) continue;
                j.f_in = fin[k];
                j.e_in = ps.e[cur[k]];
                j.f_out = ps.f[cur[k] ^ 1];
                j.e_out = ps.e[cur[k] ^ 1];
                // Eq. 8: after the level's first iteration the stored energy is
                // already the loss under the fixed target (the level start
                // scores Eq. 1)
                j.e_valid = style && fixed_target && it > 0;
                if (track) {
                    j.trk_prev = ps.trk_prev >= 0 ? fin[ps.trk_prev] : nullptr;
                    j.trk_next = ps.trk_next >= 0 ? fin[ps.trk_next] : nullptr;
                }
                const bool aligned = align && ps.partner >= 0;
                if (aligned) {
                    j.pair_f = fin[ps.partner];
                    j.pair_sty = reinterpret_cast<const uint32_t *>(ps.partner_sty_pyr + ps.L.lv[l].px_off);
                }
                cur[k] ^= 1;
                ((style || aligned) ? js_style : js_plain).push_back(j);
            }
            const int tmode = track ? kIterTrack : kIterPlain;
            // (a guarded plan is not tuned: rerunning one of its launches after
            // the guarded ones could rewrite a field that a rejected or kept
            // run ended in; it takes the shape tuned for its batch shape, if any)
            if (l == 0 && it == its - 1 && !guarded) {
                P.has_tune = true;
                P.tune_jobs = js_style.empty() ? js_plain : js_style;
                P.tune_iter = it;
                P.tune_mode = js_style.empty() ? tmode : (tmode | kIterStyle);
            }
            add_pm_launch(P, kLaunchIter, js_style, cfg, p, seed, it, tmode | kIterStyle);
            add_pm_launch(P, kLaunchIter, js_plain, cfg, p, seed, it, tmode);
        }
        if (!any_guard) continue;
        if (any_race && !decided) decide();
        // a rejected pair's plain field replaces the seeded one wherever the
        // two runs ended in different buffers
        std::vector<PMJob> sel;
        for (size_t k : active) {
            PairSpec &ps = pairs[k];
            if (ps.guard_slot < 0) continue;
            PMJob j = job_geom(ps, l);
            j.guard = gsum(ps);
            j.guard_any = gany;
            if (l == ps.L.levels - 1) {
                j.f_alt = ps.rf[rcur[k]];
                j.e_alt = ps.re[rcur[k]];
            } else {
                if (rcur[k] == cur[k]) continue;
                j.f_alt = ps.f[rcur[k]];
                j.e_alt = ps.e[rcur[k]];
            }
            j.f_out = ps.f[cur[k]];
            j.e_out = ps.e[cur[k]];
            rcur[k] = cur[k];
            sel.push_back(j);
        }
        add_pm_launch(P, kLaunchGuardSelect, sel, cfg, p, seed, 0);
    }
    std::vector<PMJob> ex;
    for (size_t k = 0; k < pairs.size(); ++k) {
        pairs[k].final_buf = cur[k];
        if (!pairs[k].nnf_abi) continue;
        PMJob j = job_geom(pairs[k], 0);
        j.f_in = pairs[k].f[cur[k]];
        j.e_in = pairs[k].e[cur[k]];
        j.nnf_abi = pairs[k].nnf_abi;
        j.energy_abi = pairs[k].energy_abi;
        ex.push_back(j);
    }
    add_pm_launch(P, kLaunchExport, ex, cfg, p, seed, 0);
    if (P.has_tune) P.tune_key = tune_key_of(pairs, p);
}

void add_remap_launch(Plan &P, const std::vector<RemapFrame> &frames,
                      const std::vector<RemapTerm> &terms, int h, int w, int pitch, int p) {
    const size_t toff = table_append(P, terms.data(), terms.size());
    const size_t foff = table_append(P, frames.data(), frames.size());
    const int nf = (int)frames.size();
    sig_add(P, "remap", (long long)toff, (long long)foff, nf, ((long long)h << 32) | w);
    P.ops.push_back({FB_KERNEL_REMAP, [=](hipStream_t s, const uint8_t *tab) {
        return launch_remap_sum(reinterpret_cast<const RemapFrame *>(tab + foff), nf,
                                reinterpret_cast<const RemapTerm *>(tab + toff), h, w, pitch, p, s);
    }});
}

// ---- fast mode (Section 3.4, Alg. 3-5, Eq. 6) ----

// Frame of position k in table d (d = 1: the mirrored table of the
// "symmetric" queries, frames in reverse order).
int fast_frame(int d, int k, int N) { return d ? N - 1 - k : k; }

// Alg. 5's blocks for the interval [l, r] (table positions): (i, L) with
// BlendingTable(i, L) = sum of the 2^L frames ending at i, remapped to i;
// the walk steps back by each block (i <- i - 2^L).
std::vector<std::pair<int, int>> fast_query_blocks(int l, int r) {
    std::vector<std::pair<int, int>> out;
    for (int i = r; i >= l;) {
        int L = 0;
        while (((i >> L) & 1) && i - (1 << (L + 1)) + 1 >= l) ++L;
        out.push_back({i, L});
        i -= 1 << L;
    }
    return out;
}

// BlendingTable(k, L) exists when L == 0 or the low L bits of k are all set.
bool fast_entry_valid(int k, int L) { return L == 0 || (k & ((1 << L) - 1)) == (1 << L) - 1; }

}  // namespace

// A slot of the ring of launch-descriptor tables.  A plan's table is copied
// stream-ordered from the slot's pinned host image into its device buffer;
// `done` is recorded after the plan's launches, so a slot is rewritten only
// once the work that read it has finished (no device-wide synchronisation).
struct TabSlot {
    void *dev = nullptr;      // device copy
    void *pinned = nullptr;   // pinned host staging buffer of the copy
    size_t cap = 0;
    std::vector<uint8_t> host;  // bytes currently in the slot
    uint64_t gen = 0;           // 0: empty
    hipEvent_t done = nullptr;  // recorded after the last launches that read the slot
};
constexpr int kTabRing = 8;

struct fb_ctx {
    int device = 0;
    TabSlot tab[kTabRing];
    int tab_last = 0;           // slot of the last plan
    hipStream_t last_stream = nullptr;  // stream of the last plan
    uint64_t table_gen = 0;
    Buf pyr, style, fe, tune_table, shat, tables, race, gsum, probe;
    std::vector<int> guard_map;  // last call: guard slot of each planned pair (-1: not guarded)
    int guard_n = 0;
    std::map<std::string, int> tuned;
    int64_t autotune_runs = 0;
    int64_t graph_fallbacks = 0;  // captures that failed and ran eagerly instead
    std::string graph_fallback_reason;
    int forced_cfg = -1;
    std::string graph_sig;
    uint64_t graph_gen = ~0ull;
    hipStream_t graph_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // kernel timing: events bracketing each launch, read lazily
    UNet *unet = nullptr;
    Buf seeds, unet_tab;
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    struct Mark { int kind; hipEvent_t a, b; };
    std::vector<Mark> marks;
    fb_profile acc{};
};

namespace {

fb_status ensure(fb_ctx *ctx, Buf &b, size_t n) {
    if (b.n >= n) return FB_OK;
    // buffers may be in use by enqueued work: wait for it before replacing
    FB_HIP(hipDeviceSynchronize());
    if (b.p) FB_HIP(hipFree(b.p));
    b.p = nullptr;
    b.n = 0;
    n = std::max<size_t>(n, 256);
    if (hipMalloc(&b.p, n) != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(FB_E_ALLOC, "device allocation of " + std::to_string(n) + " bytes failed");
    }
    b.n = n;
    // pointers inside uploaded tables may now be stale
    for (TabSlot &t : ctx->tab) t.gen = 0;
    return FB_OK;
}

// The device table of plan P: a slot that already holds these bytes, else
// the next slot of the ring, refilled with a stream-ordered copy once the
// launches that last read it have finished.
fb_status upload_table(fb_ctx *ctx, const Plan &P, hipStream_t s, int *slot) {
    for (int i = 0; i < kTabRing; ++i) {
        const int k = (ctx->tab_last + kTabRing - i) % kTabRing;
        if (ctx->tab[k].gen && ctx->tab[k].host == P.table) {
            // its copy may have been enqueued on another stream
            FB_HIP(hipStreamWaitEvent(s, ctx->tab[k].done, 0));
            *slot = k;
            return FB_OK;
        }
    }
    const int k = (ctx->tab_last + 1) % kTabRing;
    TabSlot &t = ctx->tab[k];
    t.gen = 0;
    if (t.done) FB_HIP(hipEventSynchronize(t.done));
    else FB_HIP(hipEventCreateWithFlags(&t.done, hipEventDisableTiming));
    const size_t n = P.table.size();
    if (t.cap < n) {
        if (t.dev) FB_HIP(hipFree(t.dev));
        if (t.pinned) FB_HIP(hipHostFree(t.pinned));
        t.dev = t.pinned = nullptr;
        t.cap = 0;
        size_t cap = 4096;
        while (cap < n) cap <<= 1;
        if (hipMalloc(&t.dev, cap) != hipSuccess || hipHostMalloc(&t.pinned, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(FB_E_ALLOC, "launch table of " + std::to_string(cap) + " bytes");
        }
        t.cap = cap;
    }
    std::memcpy(t.pinned, P.table.data(), n);
    FB_HIP(hipMemcpyAsync(t.dev, t.pinned, n, hipMemcpyHostToDevice, s));
    t.host = P.table;
    t.gen = ++ctx->table_gen;
    *slot = k;
    return FB_OK;
}

TileCfg choose_cfg(fb_ctx *ctx, const std::string &key, uint32_t flags) {
    if (ctx->forced_cfg >= 0) return tile_cfg(ctx->forced_cfg);
    if (!(flags & FB_NO_AUTOTUNE)) {
        auto it = ctx->tuned.find(key);
        if (it != ctx->tuned.end()) return tile_cfg(it->second);
    }
    return tile_cfg(0);
}

// Re-run the plan's finest-level iteration launch with every tile shape and
// keep the fastest.  That launch reads a buffer nothing later writes and
// rewrites its output with identical values, so the timing runs are harmless.
fb_status autotune(fb_ctx *ctx, Plan &P, hipStream_t s, int p, uint64_t seed) {
    hipEvent_t e0, e1;
    FB_HIP(hipEventCreate(&e0));
    FB_HIP(hipEventCreate(&e1));
    int best = 0;
    float best_ms = 1e30f;
    for (int c = 0; c < n_tile_cfgs(); ++c) {
        std::vector<PMJob> jobs = P.tune_jobs;
        int total = 0, uniform = 0;
        assign_tiles(jobs, tile_cfg(c), &total, &uniform);
        fb_status st = ensure(ctx, ctx->tune_table, jobs.size() * sizeof(PMJob));
        if (st) return st;
        FB_HIP(hipStreamSynchronize(s));
        FB_HIP(hipMemcpy(ctx->tune_table.p, jobs.data(), jobs.size() * sizeof(PMJob),
                         hipMemcpyHostToDevice));
        const PMJob *dj = reinterpret_cast<const PMJob *>(ctx->tune_table.p);
        // reruns of the last iteration read what it read and write what it wrote
        const int tab_bytes = max_tab_bytes(jobs);
        FB_HIP(launch_pm_iter(dj, (int)jobs.size(), total, uniform, tile_cfg(c), p, P.tune_iter, seed,
                              P.tune_mode, tab_bytes, s));
        FB_HIP(hipEventRecord(e0, s));
        for (int rep = 0; rep < 3; ++rep)
            FB_HIP(launch_pm_iter(dj, (int)jobs.size(), total, uniform, tile_cfg(c), p, P.tune_iter, seed,
                                  P.tune_mode, tab_bytes, s));
        FB_HIP(hipEventRecord(e1, s));
        FB_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        FB_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    FB_HIP(hipEventDestroy(e0));
    FB_HIP(hipEventDestroy(e1));
    ctx->tuned[P.tune_key] = best;
    ++ctx->autotune_runs;
    return FB_OK;
}

fb_status run_plan(fb_ctx *ctx, Plan &P, uint32_t flags, hipStream_t s, int p, uint64_t seed) {
    if (P.table.empty()) P.table.resize(256);
    // the context's workspace is shared by its calls: a call on another
    // stream waits on the device for the previous call's launches
    const TabSlot &prev = ctx->tab[ctx->tab_last];
    if (prev.done && s != ctx->last_stream) FB_HIP(hipStreamWaitEvent(s, prev.done, 0));
    ctx->last_stream = s;
    int slot = 0;
    fb_status st = upload_table(ctx, P, s, &slot);
    if (st) return st;
    ctx->tab_last = slot;
    TabSlot &ts = ctx->tab[slot];
    const uint8_t *tab = static_cast<const uint8_t *>(ts.dev);
    const bool tune = P.has_tune && ctx->forced_cfg < 0 && !(flags & FB_NO_AUTOTUNE) &&
                      !ctx->tuned.count(P.tune_key);
    if ((flags & FB_USE_GRAPH) && s != nullptr && !tune && !ctx->profiling) {
        if (!ctx->graph_exec || ctx->graph_gen != ts.gen || ctx->graph_sig != P.sig ||
            ctx->graph_stream != s) {
            if (ctx->graph_exec) FB_HIP(hipGraphExecDestroy(ctx->graph_exec));
            ctx->graph_exec = nullptr;
            // A launch that fails is an error in any mode; a failure of the
            // capture itself (begin, end, instantiate) falls back to running
            // the same launches eagerly.
            const char *stage = "hipStreamBeginCapture";
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                for (Op &op : P.ops) {
                    const hipError_t le = op.fn(s, tab);
                    if (le != hipSuccess) {
                        hipGraph_t dummy = nullptr;
                        (void)hipStreamEndCapture(s, &dummy);
                        if (dummy) (void)hipGraphDestroy(dummy);
                        return fail(FB_E_HIP, std::string("launch during capture: ") + hipGetErrorString(le));
                    }
                }
                hipGraph_t g = nullptr;
                stage = "hipStreamEndCapture";
                e = hipStreamEndCapture(s, &g);
                if (e == hipSuccess) {
                    stage = "hipGraphInstantiate";
                    // FB_DEBUG_FAIL_CAPTURE: report this step as failed (tests of the fallback)
                    e = (flags & FB_DEBUG_FAIL_CAPTURE) ? hipErrorNotSupported
                                                         : hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                }
            }
            if (e != hipSuccess) {
                (void)hipGetLastError();
                ctx->graph_exec = nullptr;
                ++ctx->graph_fallbacks;
                ctx->graph_fallback_reason = std::string(stage) + ": " + hipGetErrorString(e);
            } else {
                ctx->graph_sig = P.sig;
                ctx->graph_gen = ts.gen;
                ctx->graph_stream = s;
            }
        }
        if (ctx->graph_exec) {
            FB_HIP(hipGraphLaunch(ctx->graph_exec, s));
            FB_HIP(hipEventRecord(ts.done, s));
            return FB_OK;
        }
    }
    for (Op &op : P.ops) {
        if (ctx->profiling) {
            fb_ctx::Mark m{op.kind, nullptr, nullptr};
            for (hipEvent_t *e : {&m.a, &m.b}) {
                if (!ctx->ev_pool.empty()) {
                    *e = ctx->ev_pool.back();
                    ctx->ev_pool.pop_back();
                } else {
                    FB_HIP(hipEventCreate(e));
                }
            }
            FB_HIP(hipEventRecord(m.a, s));
            FB_HIP(op.fn(s, tab));
            FB_HIP(hipEventRecord(m.b, s));
            ctx->marks.push_back(m);
        } else {
            FB_HIP(op.fn(s, tab));
        }
    }
    FB_HIP(hipEventRecord(ts.done, s));
    if (tune) return autotune(ctx, P, s, p, seed);
    return FB_OK;
}

fb_status drain_marks(fb_ctx *ctx) {
    for (fb_ctx::Mark &m : ctx->marks) {
        FB_HIP(hipEventSynchronize(m.b));
        float ms = 0.f;
        FB_HIP(hipEventElapsedTime(&ms, m.a, m.b));
        const int k = (m.kind >= 0 && m.kind < FB_KERNEL_KINDS) ? m.kind : FB_KERNEL_OTHER;
        ctx->acc.launches[k] += 1;
        ctx->acc.milliseconds[k] += ms;
        ctx->ev_pool.push_back(m.a);
        ctx->ev_pool.push_back(m.b);
    }
    ctx->marks.clear();
    return FB_OK;
}

bool valid_p(int p) { return p >= 1 && p <= kMaxP; }

constexpr int kUNetChunk = 512;  // pairs per network launch sequence (about 9 MB of activations per pair at 128x128)

// Learned proposal: the network predicts each pair's offset field at its
// coarsest level from the two coarsest pyramid levels; the rounded offsets
// seed the level (kStartOffsets) instead of the random draw.  Pairs that
// already carry seed offsets keep them.  Consecutive pairs with the same
// coarsest size share network launches (up to kUNetChunk pairs).
fb_status plan_learned_seeds(fb_ctx *ctx, Plan &P, std::vector<PairSpec> &pairs) {
    struct Group { size_t first, count; int H8, W8; };
    std::vector<Group> groups;
    size_t seed_elems = 0;
    std::vector<size_t> seed_off(pairs.size(), 0);
    int maxB = 0, maxH8 = 8, maxW8 = 8;
    for (size_t k = 0; k < pairs.size(); ++k) {
        if (pairs[k].seed_offsets) continue;
        const LevelGeom &g = pairs[k].L.lv[pairs[k].L.levels - 1];
        const int H8 = (g.h + 7) / 8 * 8, W8 = (g.w + 7) / 8 * 8;
        if (!groups.empty() && groups.back().first + groups.back().count == k && groups.back().H8 == H8 &&
            groups.back().W8 == W8 && groups.back().count < (size_t)kUNetChunk)
            ++groups.back().count;
        else
            groups.push_back({k, 1, H8, W8});
        seed_off[k] = seed_elems;
        seed_elems += (size_t)g.h * g.w * 2;
    }
    if (groups.empty()) return FB_OK;
    if (!unet_loaded(ctx->unet))
        return fail(FB_E_INVALID, "FB_LEARNED_SEED needs network parameters (fb_unet_load)");
    // the largest group shape bounds the workspace (bound without allocating later)
    size_t best = 0;
    for (const Group &gr : groups) {
        const size_t need = gr.count * (size_t)gr.H8 * gr.W8;
        if (need > best) { best = need; maxB = (int)gr.count; maxH8 = gr.H8; maxW8 = gr.W8; }
    }
    fb_status st;
    if ((st = ensure(ctx, ctx->seeds, std::max<size_t>(seed_elems, 1) * 4))) return st;
    for (const Group &gr : groups) {
        // reserve for every group shape so that binding any of them later fits
        hipError_t e = unet_reserve(ctx->unet, (int)gr.count, gr.H8, gr.W8, false);
        if (e != hipSuccess) return fail(FB_E_ALLOC, std::string("network workspace: ") + hipGetErrorString(e));
    }
    (void)maxB; (void)maxH8; (void)maxW8;
    int32_t *seeds = static_cast<int32_t *>(ctx->seeds.p);
    UNet *u = ctx->unet;
    // captured launches hold workspace addresses: a new workspace is a new plan
    sig_add(P, "unetws", (long long)(uintptr_t)unet_input_buffer(u), (long long)(uintptr_t)seeds);
    for (const Group &gr : groups) {
        std::vector<UNetPairIn> in(gr.count);
        std::vector<int32_t *> dst(gr.count);
        for (size_t q = 0; q < gr.count; ++q) {
            PairSpec &ps = pairs[gr.first + q];
            const LevelGeom &g = ps.L.lv[ps.L.levels - 1];
            in[q] = UNetPairIn{reinterpret_cast<const uint32_t *>(ps.src_pyr + g.px_off),
                               reinterpret_cast<const uint32_t *>(ps.tgt_pyr + g.px_off), g.h, g.w, g.pitch,
                               ps.L.p};
            dst[q] = seeds + seed_off[gr.first + q];
            ps.seed_offsets = dst[q];
        }
        const size_t in_off = table_append(P, in.data(), in.size());
        const size_t dst_off = table_append(P, dst.data(), dst.size());
        const int B = (int)gr.count, H8 = gr.H8, W8 = gr.W8;
        sig_add(P, "unet", (long long)in_off, (long long)dst_off, B, ((long long)H8 << 32) | W8);
        P.ops.push_back({FB_KERNEL_UNET, [=](hipStream_t s, const uint8_t *tab) {
            hipError_t e = unet_shape(u, B, H8, W8, false);
            if (e != hipSuccess) return e;
            const UNetPairIn *pin = reinterpret_cast<const UNetPairIn *>(tab + in_off);
            if ((e = launch_input_from_pyramids(pin, B, H8, W8, unet_input_buffer(u), s)) != hipSuccess) return e;
            if ((e = unet_forward(u, s, false)) != hipSuccess) return e;
            return launch_pred_to_seed(unet_pred_buffer(u), H8, W8, pin,
                                       reinterpret_cast<int32_t *const *>(tab + dst_off), B, s);
        }});
    }
    return FB_OK;
}

// The guard of the seeded pairs of a plain (Eq. 1) pass with FB_LEARNED_SEED
// and without FB_NO_GUARD: every pair that starts from offsets gets a slot,
// the plain run's buffers at its coarsest level and two summed energies.
constexpr int kDefaultPlainIters = 6;

fb_status prepare_guard(fb_ctx *ctx, std::vector<PairSpec> &pairs, const fb_params *prm, bool plain_pass,
                        GuardPlan *g) {
    g->n = 0;
    ctx->guard_map.assign(pairs.size(), -1);
    ctx->guard_n = 0;
    if (!plain_pass || !(prm->flags & FB_LEARNED_SEED) || (prm->flags & FB_NO_GUARD)) return FB_OK;
    size_t race_px = 0;
    int n = 0;
    for (const PairSpec &ps : pairs)
        if (ps.seed_offsets) {
            const LevelGeom &c = ps.L.lv[ps.L.levels - 1];
            race_px += (size_t)c.h * c.w;
            ++n;
        }
    if (!n) return FB_OK;
    fb_status st;
    if ((st = ensure(ctx, ctx->race, race_px * 16)) || (st = ensure(ctx, ctx->gsum, (size_t)n * 16 + 8))) return st;
    uint32_t *base = static_cast<uint32_t *>(ctx->race.p);
    size_t off = 0;
    int slot = 0;
    for (size_t k = 0; k < pairs.size(); ++k) {
        PairSpec &ps = pairs[k];
        if (!ps.seed_offsets) continue;
        const LevelGeom &c = ps.L.lv[ps.L.levels - 1];
        ps.guard_slot = slot;
        ps.rf[0] = base + off;
        ps.rf[1] = base + race_px + off;
        ps.re[0] = base + 2 * race_px + off;
        ps.re[1] = base + 3 * race_px + off;
        off += (size_t)c.h * c.w;
        ctx->guard_map[k] = slot++;
    }
    g->plain_iters = prm->plain_iters ? prm->plain_iters : kDefaultPlainIters;
    g->sums = static_cast<uint64_t *>(ctx->gsum.p);
    g->n = n;
    ctx->guard_n = n;
    return FB_OK;
}

fb_status check_unet_shape(int B, int h, int w) {
    if (B < 1 || h < 8 || w < 8 || h % 8 || w % 8)
        return fail(FB_E_SHAPE, "network input needs B >= 1 and h, w positive multiples of 8");
    if ((long long)B * h * w > (1LL << 28)) return fail(FB_E_UNSUPPORTED, "network batch too large");
    return FB_OK;
}

// Largest alpha16 for which every scaled loss alpha16 SSD(G) + 16 SSD(S, X)
// (Eq. 3, 8, 10) fits in uint32: a patch SSD is at most 3 * 255^2 * (2p+1)^2,
// so (alpha16 + 16) times that must stay below 2^32; and alpha16 <= 512.
int alpha16_max(int p) {
    const uint64_t k = 2u * (uint64_t)p + 1u;
    const uint64_t a = 0xFFFFFFFFull / (3ull * 255u * 255u * k * k) - 16u;
    return (int)std::min<uint64_t>(a, 512u);
}

fb_status check_params(const fb_params *prm, bool need_levels) {
    if (!prm) return fail(FB_E_INVALID, "params is NULL");
    if (!valid_p(prm->patch_radius))
        return fail(FB_E_UNSUPPORTED, "patch_radius must be in [1, 4]");
    if (need_levels && (prm->levels < 1 || prm->levels > kMaxLevels))
        return fail(FB_E_INVALID, "levels must be in [1, 16]");
    if (prm->iters < 0 || prm->iters > 0xFFFE) return fail(FB_E_INVALID, "iters must be in [0, 65534]");
    if (prm->plain_iters < 0 || prm->plain_iters > 0xFFFE)
        return fail(FB_E_INVALID, "plain_iters must be in [0, 65534]");
    if (prm->flags & (FB_STYLE_LOSS | FB_ACCURATE_BLEND | FB_ALIGN)) {
        if (prm->iters < 1) return fail(FB_E_INVALID, "FB_STYLE_LOSS, FB_ACCURATE_BLEND and FB_ALIGN need iters >= 1");
        const int amax = alpha16_max(prm->patch_radius);
        if (prm->alpha16 < 0 || prm->alpha16 > amax)
            return fail(FB_E_INVALID, "alpha16 must be in [0, " + std::to_string(amax) + "] for patch_radius " +
                                          std::to_string(prm->patch_radius) + " (the loss must fit in uint32)");
        if ((prm->flags & FB_ALIGN) && prm->alpha16 < 1) return fail(FB_E_INVALID, "FB_ALIGN needs alpha16 >= 1");
    }
    return FB_OK;
}

fb_status check_size(int h, int w) {
    if (h < 1 || w < 1) return fail(FB_E_INVALID, "image sizes must be positive");
    if (h > 32767 || w > 32767) return fail(FB_E_UNSUPPORTED, "image sides are limited to 32767");
    // kernels address a padded frame with 32-bit byte offsets
    if ((uint64_t)(h + 2 * kMaxP) * (uint64_t)(w + 2 * kMaxP + kPitchAlign) * 4u >= (1ull << 31))
        return fail(FB_E_UNSUPPORTED, "a padded frame must stay below 2 GiB");
    return FB_OK;
}

fb_status begin(fb_ctx *ctx) {
    if (!ctx) return fail(FB_E_INVALID, "ctx is NULL");
    FB_HIP(hipSetDevice(ctx->device));
    return FB_OK;
}

}  // namespace

// Fast-mode window blend: Alg. 3 (remapping table) and Alg. 4 (blending
// table, its column prefix sums) for the forward and the mirrored frame
// order, then every frame's window as the forward query [lo, i] plus the
// mirrored query [i, hi] minus the frame itself (Eq. 6), divided by the
// window's length.  All NNFs the tables and queries use run as one batch;
// table column L is one remap launch (its entries add the column L - 1
// entry and the frames of the new block), the output one more.
fb_status blend_fast(fb_ctx *ctx, const Frames &guides, const Frames &styles, int N, int h, int w, int M,
                     const fb_params *params, float *out, hipStream_t stream) {
    fb_status st;
    const int p = params->patch_radius, K = params->levels;
    if (params->flags & (FB_STYLE_LOSS | FB_ACCURATE_BLEND))
        return fail(FB_E_UNSUPPORTED, "FB_FAST_BLEND takes neither FB_STYLE_LOSS nor FB_ACCURATE_BLEND");
    int Lmax = 0;
    while ((1 << Lmax) < N) ++Lmax;
    const PyrLayout Lp = pyr_layout(h, w, K, p);
    int32_t pitch = 0;
    const size_t sbytes = padded_image_bytes(h, w, p, &pitch);
    const size_t npx = (size_t)h * w;

    // every NNF(G_src, G_tgt) the tables and the queries remap through
    std::map<uint64_t, size_t> need;  // src * N + tgt -> pair index
    std::vector<std::pair<int, int>> need_list;
    auto add = [&](int src, int tgt) {
        const uint64_t key = (uint64_t)src * N + tgt;
        if (need.emplace(key, need_list.size()).second) need_list.push_back({src, tgt});
    };
    for (int d = 0; d < 2; ++d)
        for (int i = 0; i < N; ++i)
            for (int L = 0, j = i; L < Lmax; ++L) {
                if ((i >> L) & 1) continue;
                j |= 1 << L;
                if (j < N) add(fast_frame(d, i, N), fast_frame(d, j, N));
            }
    std::vector<std::vector<std::pair<int, int>>> qblocks[2];
    for (int i = 0; i < N; ++i) {
        const int lo = std::max(0, i - M), hi = std::min(N - 1, i + M);
        qblocks[0].push_back(fast_query_blocks(lo, i));
        qblocks[1].push_back(fast_query_blocks(N - 1 - hi, N - 1 - i));
        for (int d = 0; d < 2; ++d) {
            const int r = d ? N - 1 - i : i;
            for (const auto &b : qblocks[d].back())
                if (b.first != r) add(fast_frame(d, b.first, N), i);
        }
    }
    // table entries (d, k, L) -> slot
    std::vector<int> slot(2 * (size_t)N * (Lmax + 1), -1);
    int n_slots = 0;
    for (int d = 0; d < 2; ++d)
        for (int k = 0; k < N; ++k)
            for (int L = 0; L <= Lmax; ++L)
                if (fast_entry_valid(k, L)) slot[((size_t)d * N + k) * (Lmax + 1) + L] = n_slots++;
    const size_t n_pairs = need_list.size();
    if ((st = ensure(ctx, ctx->pyr, (size_t)N * Lp.bytes)) || (st = ensure(ctx, ctx->style, (size_t)N * sbytes)) ||
        (st = ensure(ctx, ctx->fe, std::max<size_t>(n_pairs, 1) * npx * 16)) ||
        (st = ensure(ctx, ctx->tables, (size_t)n_slots * npx * 16)))
        return st;
    uint8_t *pyr = static_cast<uint8_t *>(ctx->pyr.p);
    uint8_t *sty = static_cast<uint8_t *>(ctx->style.p);
    uint32_t *fe = static_cast<uint32_t *>(ctx->fe.p);
    float *tab = static_cast<float *>(ctx->tables.p);

    Plan P;
    plan_pyramids(P, guides, h, w, Lp, pyr, Lp.bytes);
    plan_style_pack(P, styles, h, w, p, sty, sbytes, pitch);
    std::vector<PairSpec> pairs;
    for (size_t k = 0; k < n_pairs; ++k) {
        PairSpec ps{};
        ps.src_pyr = pyr + (size_t)need_list[k].first * Lp.bytes;
        ps.tgt_pyr = pyr + (size_t)need_list[k].second * Lp.bytes;
        ps.L = Lp;
        ps.pair_id = (uint32_t)need_list[k].first * (uint32_t)N + (uint32_t)need_list[k].second;
        ps.f[0] = fe + k * npx;
        ps.f[1] = fe + (n_pairs + k) * npx;
        ps.e[0] = fe + (2 * n_pairs + k) * npx;
        ps.e[1] = fe + (3 * n_pairs + k) * npx;
        pairs.push_back(ps);
    }
    if (params->flags & FB_LEARNED_SEED)
        if ((st = plan_learned_seeds(ctx, P, pairs))) return st;
    GuardPlan gp;
    if ((st = prepare_guard(ctx, pairs, params, true, &gp))) return st;
    const TileCfg cfg = choose_cfg(ctx, tune_key_of(pairs, p), params->flags);
    if (!pairs.empty()) plan_patchmatch(P, pairs, params->iters, p, params->seed, cfg, false, 0, false, false, false, &gp);

    auto style_px = [&](int f) { return reinterpret_cast<const uint32_t *>(sty + (size_t)f * sbytes); };
    auto field = [&](int src, int tgt) {
        const PairSpec &ps = pairs[need.at((uint64_t)src * N + tgt)];
        return (const uint32_t *)ps.f[ps.final_buf];
    };
    auto entry = [&](int d, int k, int L) { return tab + (size_t)slot[((size_t)d * N + k) * (Lmax + 1) + L] * npx * 4; };
    for (int L = 0; L <= Lmax; ++L) {
        std::vector<RemapTerm> terms;
        std::vector<RemapFrame> frames;
        for (int d = 0; d < 2; ++d)
            for (int k = 0; k < N; ++k) {
                if (!fast_entry_valid(k, L)) continue;
                RemapFrame fr{entry(d, k, L), (int32_t)terms.size(), 0, 1.0f, 1};
                const int fk = fast_frame(d, k, N);
                if (L == 0) {
                    terms.push_back(RemapTerm{style_px(fk), nullptr, 1.0f, kRemapStyle});
                } else {
                    terms.push_back(RemapTerm{reinterpret_cast<const uint32_t *>(entry(d, k, L - 1)), nullptr, 1.0f,
                                              kRemapFloat});
                    for (int i = k - (1 << L) + 1; i <= k - (1 << (L - 1)); ++i) {
                        const int fi = fast_frame(d, i, N);
                        terms.push_back(RemapTerm{style_px(fi), field(fi, fk), 1.0f, kRemapStyle});
                    }
                }
                fr.n_terms = (int32_t)terms.size() - fr.term_base;
                frames.push_back(fr);
            }
        if (!frames.empty()) add_remap_launch(P, frames, terms, h, w, pitch, p);
    }
    std::vector<RemapTerm> terms;
    std::vector<RemapFrame> frames;
    for (int i = 0; i < N; ++i) {
        const int lo = std::max(0, i - M), hi = std::min(N - 1, i + M);
        RemapFrame fr{out + (size_t)i * npx * 3, (int32_t)terms.size(), 0, (float)(hi - lo + 1), 0};
        for (int d = 0; d < 2; ++d) {
            const int r = d ? N - 1 - i : i;
            for (const auto &b : qblocks[d][i]) {
                const int fk = fast_frame(d, b.first, N);
                terms.push_back(RemapTerm{reinterpret_cast<const uint32_t *>(entry(d, b.first, b.second)),
                                          b.first == r ? nullptr : field(fk, i), 1.0f, kRemapFloat});
            }
        }
        terms.push_back(RemapTerm{style_px(i), nullptr, -1.0f, kRemapStyle});
        fr.n_terms = (int32_t)terms.size() - fr.term_base;
        frames.push_back(fr);
    }
    add_remap_launch(P, frames, terms, h, w, pitch, p);
    return run_plan(ctx, P, params->flags, stream, p, params->seed);
}

// Accurate-mode window blend (Eq. 7-8): the window NNFs under Eq. 1; T^- of
// every frame, the exact mean of its window's remapped styles rounded to
// uint8 (one remap launch), and its pyramid; every NNF estimated again under
// Eq. 8 against its target frame's T^- (the style iteration kernel, no
// refresh); the window mean of the styles remapped with the new NNFs.
fb_status blend_accurate(fb_ctx *ctx, const Frames &guides, const Frames &styles, int N, int h, int w, int M,
                         const fb_params *params, float *out, hipStream_t stream) {
    fb_status st;
    const int p = params->patch_radius, K = params->levels;
    if (params->flags & (FB_STYLE_LOSS | FB_FAST_BLEND))
        return fail(FB_E_UNSUPPORTED, "FB_ACCURATE_BLEND takes neither FB_STYLE_LOSS nor FB_FAST_BLEND");
    const PyrLayout L = pyr_layout(h, w, K, p);
    int32_t pitch = 0;
    (void)padded_image_bytes(h, w, p, &pitch);
    const size_t npx = (size_t)h * w;
    size_t n_pairs = 0;
    for (int i = 0; i < N; ++i) n_pairs += (size_t)(std::min(N - 1, i + M) - std::max(0, i - M));
    // style: N style pyramids, then N T^- frames (uint8 RGB) and their pyramids
    const size_t tbar_rgb = ((size_t)N * npx * 3 + 255) & ~(size_t)255;
    if ((st = ensure(ctx, ctx->pyr, (size_t)N * L.bytes)) ||
        (st = ensure(ctx, ctx->style, 2 * (size_t)N * L.bytes + tbar_rgb)) ||
        (st = ensure(ctx, ctx->fe, std::max<size_t>(2 * n_pairs, 1) * npx * 16)))
        return st;
    uint8_t *pyr = static_cast<uint8_t *>(ctx->pyr.p);
    uint8_t *sty = static_cast<uint8_t *>(ctx->style.p);
    uint8_t *tbar = sty + (size_t)N * L.bytes;
    uint8_t *tbar_in = tbar + (size_t)N * L.bytes;
    uint32_t *fe = static_cast<uint32_t *>(ctx->fe.p);

    Plan P;
    plan_pyramids(P, guides, h, w, L, pyr, L.bytes);
    plan_pyramids(P, styles, h, w, L, sty, L.bytes, false);
    // fields and energies of pair k in pass q (0: Eq. 1, 1: Eq. 8), n pairs,
    // in slices of npx entries of fe: f[0] at q n + k, f[1] at 2n + q n + k,
    // e[0] at 4n + q n + k, e[1] at 6n + q n + k
    std::vector<PairSpec> first, second;
    auto bufs = [&](PairSpec &ps, int q, size_t k) {
        ps.f[0] = fe + (q * n_pairs + k) * npx;
        ps.f[1] = fe + (2 * n_pairs + q * n_pairs + k) * npx;
        ps.e[0] = fe + (4 * n_pairs + q * n_pairs + k) * npx;
        ps.e[1] = fe + (6 * n_pairs + q * n_pairs + k) * npx;
    };
    for (int i = 0; i < N; ++i)
        for (int j = std::max(0, i - M); j <= std::min(N - 1, i + M); ++j) {
            if (j == i) continue;
            PairSpec ps{};
            ps.src_pyr = pyr + (size_t)j * L.bytes;
            ps.tgt_pyr = pyr + (size_t)i * L.bytes;
            ps.L = L;
            ps.pair_id = (uint32_t)j * (uint32_t)N + (uint32_t)i;
            const size_t k = first.size();
            bufs(ps, 0, k);
            first.push_back(ps);
            ps.src_sty_pyr = sty + (size_t)j * L.bytes;
            ps.tbar_pyr = tbar + (size_t)i * L.bytes;
            bufs(ps, 1, k);
            second.push_back(ps);
        }
    if (params->flags & FB_LEARNED_SEED) {
        if ((st = plan_learned_seeds(ctx, P, first))) return st;
        for (size_t k = 0; k < first.size(); ++k) second[k].seed_offsets = first[k].seed_offsets;
    }
    GuardPlan gp;  // the Eq. 1 pass is guarded; the Eq. 8 pass starts from the same seeds
    if ((st = prepare_guard(ctx, first, params, true, &gp))) return st;
    const TileCfg cfg = choose_cfg(ctx, tune_key_of(first, p), params->flags);
    if (!first.empty()) plan_patchmatch(P, first, params->iters, p, params->seed, cfg, false, 0, false, false, false, &gp);
    // T^- of every frame, then its pyramid
    auto style_px = [&](int f) { return reinterpret_cast<const uint32_t *>(sty + (size_t)f * L.bytes); };
    std::vector<RemapTerm> terms;
    std::vector<RemapFrame> frames;
    size_t k = 0;
    for (int i = 0; i < N; ++i) {
        const int lo = std::max(0, i - M), hi = std::min(N - 1, i + M);
        RemapFrame fr{reinterpret_cast<float *>(tbar_in + (size_t)i * npx * 3), (int32_t)terms.size(), hi - lo + 1,
                      1.0f, 2};
        for (int j = lo; j <= hi; ++j) {
            if (j == i) terms.push_back(RemapTerm{style_px(i), nullptr, 1.0f, kRemapStyle});
            else { terms.push_back(RemapTerm{style_px(j), first[k].f[first[k].final_buf], 1.0f, kRemapStyle}); ++k; }
        }
        frames.push_back(fr);
    }
    add_remap_launch(P, frames, terms, h, w, pitch, p);
    plan_pyramids(P, contiguous_frames(tbar_in, N, h, w), h, w, L, tbar, L.bytes, false);
    if (!second.empty()) plan_patchmatch(P, second, params->iters, p, params->seed, cfg, true, params->alpha16, true);
    terms.clear();
    frames.clear();
    k = 0;
    for (int i = 0; i < N; ++i) {
        const int lo = std::max(0, i - M), hi = std::min(N - 1, i + M);
        RemapFrame fr{out + (size_t)i * npx * 3, (int32_t)terms.size(), hi - lo + 1, (float)(hi - lo + 1), 0};
        for (int j = lo; j <= hi; ++j) {
            if (j == i) terms.push_back(RemapTerm{style_px(i), nullptr, 1.0f, kRemapStyle});
            else { terms.push_back(RemapTerm{style_px(j), second[k].f[second[k].final_buf], 1.0f, kRemapStyle}); ++k; }
        }
        frames.push_back(fr);
    }
    add_remap_launch(P, frames, terms, h, w, pitch, p);
    return run_plan(ctx, P, params->flags, stream, p, params->seed);
}

// ---- working memory of fb_patchmatch_level_noalloc ----
// A fixed array per GPU, so that entry point never allocates: the four
// ping-pong planes (field and energy, 4 bytes per pixel each) of a level of
// up to kNoAllocPixels pixels, then the launch descriptors.  Host code uses
// the device address hipGetSymbolAddress gives for the current device (the
// name itself is a host-side stand-in).
constexpr size_t kNoAllocPixels = (size_t)1 << 20;
constexpr int kNoAllocJobs = 4;
constexpr size_t kNoAllocFieldBytes = 16 * kNoAllocPixels;
constexpr size_t kNoAllocBytes = kNoAllocFieldBytes + ((kNoAllocJobs * sizeof(PMJob) + 255) & ~(size_t)255);
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device (set up by fb_create)

// once per device, with that device current
fb_status scratch_setup(int device) {
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0 || device >= kMaxDevices) return fail(FB_E_UNSUPPORTED, "device index above 63");
    if (g_scratch_ptr[device]) return FB_OK;
    void *ptr = nullptr;
    FB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = ptr;
    return FB_OK;
}

struct NoAllocJobs {
    PMJob j[kNoAllocJobs];
};

// the launch descriptors, written by a kernel from its argument (no copy from
// host memory, no allocation)
__global__ void __launch_bounds__(64) k_store_jobs(NoAllocJobs jobs, PMJob *dst, int n) {
    const uint64_t *src = reinterpret_cast<const uint64_t *>(&jobs);
    uint64_t *d = reinterpret_cast<uint64_t *>(dst);
    const int words = n * (int)(sizeof(PMJob) / 8);
    for (int i = (int)threadIdx.x; i < words; i += 64) d[i] = src[i];
}

}  // namespace

// ============================== C ABI ==================================

extern "C" {

fb_status fb_create(int32_t device, fb_ctx **out) {
    if (!out) return fail(FB_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    FB_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(FB_E_INVALID, "no such device");
    FB_HIP(hipSetDevice(device));
    fb_status st = scratch_setup(device);
    if (st) return st;
    fb_ctx *c = new fb_ctx();
    c->device = device;
    *out = c;
    return FB_OK;
}

void fb_destroy(fb_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    for (fb_ctx::Mark &m : ctx->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    unet_destroy(ctx->unet);
    for (Buf *b : {&ctx->seeds, &ctx->unet_tab})
        if (b->p) (void)hipFree(b->p);
    for (Buf *b : {&ctx->pyr, &ctx->style, &ctx->fe, &ctx->tune_table, &ctx->shat, &ctx->tables, &ctx->race,
                   &ctx->gsum, &ctx->probe})
        if (b->p) (void)hipFree(b->p);
    for (TabSlot &t : ctx->tab) {
        if (t.dev) (void)hipFree(t.dev);
        if (t.pinned) (void)hipHostFree(t.pinned);
        if (t.done) (void)hipEventDestroy(t.done);
    }
    delete ctx;
}

const char *fb_last_error(void) { return g_err.c_str(); }

int32_t fb_alpha16_max(int32_t patch_radius) { return valid_p(patch_radius) ? alpha16_max(patch_radius) : 0; }

fb_status fb_profile_enable(fb_ctx *ctx, int32_t on) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!on && (st = drain_marks(ctx))) return st;
    ctx->profiling = on != 0;
    return FB_OK;
}

fb_status fb_profile_read(fb_ctx *ctx, fb_profile *out, int32_t reset) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!out) return fail(FB_E_INVALID, "out is NULL");
    if ((st = drain_marks(ctx))) return st;
    *out = ctx->acc;
    if (reset) ctx->acc = fb_profile{};
    return FB_OK;
}

int32_t fb_num_tile_configs(void) { return n_tile_cfgs(); }

fb_status fb_gather_probe(fb_ctx *ctx, const void *pyr, int32_t h, int32_t w, int32_t patch_radius, int32_t divergent,
                          int32_t rows_per_lane, double *rows_per_s, void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!pyr || !rows_per_s) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_size(h, w))) return st;
    if (patch_radius != 2) return fail(FB_E_UNSUPPORTED, "the probe gathers 5-pixel rows: patch_radius 2 only");
    if (rows_per_lane < 1 || rows_per_lane > 4096) return fail(FB_E_INVALID, "rows_per_lane must be in [1, 4096]");
    constexpr int kBlocks = 2048;  // 8 workgroups of 256 lanes per CU
    if ((st = ensure(ctx, ctx->probe, (size_t)kBlocks * 256 * 4))) return st;
    const PyrLayout L = pyr_layout(h, w, 1, patch_radius);
    const uint32_t *img = reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(pyr) + L.lv[0].px_off);
    uint32_t *out = static_cast<uint32_t *>(ctx->probe.p);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    FB_HIP(hipEventCreate(&e0));
    FB_HIP(hipEventCreate(&e1));
    hipError_t e = launch_gather_probe(img, h, w, L.lv[0].pitch, divergent != 0, kBlocks, rows_per_lane, out, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch_gather_probe(img, h, w, L.lv[0].pitch, divergent != 0, kBlocks, rows_per_lane, out, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FB_HIP(e);
    *rows_per_s = ms > 0.f ? (double)kBlocks * 256.0 * rows_per_lane / (ms * 1e-3) : 0.0;
    return FB_OK;
}

int64_t fb_autotune_runs(fb_ctx *ctx) { return ctx ? ctx->autotune_runs : -1; }

int64_t fb_graph_fallbacks(fb_ctx *ctx) { return ctx ? ctx->graph_fallbacks : -1; }

int64_t fb_tuning_export(fb_ctx *ctx, char *buf, int64_t cap) {
    if (!ctx) return -1;
    std::string text;
    for (const auto &kv : ctx->tuned) text += kv.first + "=" + std::to_string(kv.second) + "\n";
    if (buf && cap > (int64_t)text.size()) std::memcpy(buf, text.c_str(), text.size() + 1);
    return (int64_t)text.size();
}

fb_status fb_tuning_import(fb_ctx *ctx, const char *text) {
    if (!ctx || !text) return fail(FB_E_INVALID, "null pointer");
    std::map<std::string, int> got;
    const char *p = text;
    while (*p) {
        const char *eol = std::strchr(p, '\n');
        const std::string line(p, eol ? (size_t)(eol - p) : std::strlen(p));
        p = eol ? eol + 1 : p + line.size();
        if (line.empty()) continue;
        const size_t eq = line.rfind('=');
        if (eq == std::string::npos || eq == 0 || eq + 1 >= line.size())
            return fail(FB_E_INVALID, "tuning line without key=index: " + line);
        int idx = 0;
        for (size_t k = eq + 1; k < line.size(); ++k) {
            if (line[k] < '0' || line[k] > '9' || idx > 1000) return fail(FB_E_INVALID, "bad tile index: " + line);
            idx = idx * 10 + (line[k] - '0');
        }
        if (idx >= n_tile_cfgs()) return fail(FB_E_INVALID, "no such tile config: " + line);
        got[line.substr(0, eq)] = idx;
    }
    for (const auto &kv : got) ctx->tuned[kv.first] = kv.second;
    return FB_OK;
}

fb_status fb_set_tile_config(fb_ctx *ctx, int32_t index) {
    if (!ctx) return fail(FB_E_INVALID, "ctx is NULL");
    if (index < -1 || index >= n_tile_cfgs()) return fail(FB_E_INVALID, "no such tile config");
    ctx->forced_cfg = index;
    return FB_OK;
}

size_t fb_pyramid_bytes(int32_t h, int32_t w, int32_t levels, int32_t patch_radius) {
    if (h < 1 || w < 1 || levels < 1 || levels > kMaxLevels || !valid_p(patch_radius)) return 0;
    return pyr_layout(h, w, levels, patch_radius).bytes;
}

fb_status fb_build_pyramid(fb_ctx *ctx, const uint8_t *rgb, int32_t h, int32_t w, int32_t levels,
                           int32_t patch_radius, void *pyr, void *stream) {
    return fb_build_pyramid_strided(ctx, rgb, h, w, (int64_t)w * 3, levels, patch_radius, pyr, stream);
}

fb_status fb_build_pyramid_strided(fb_ctx *ctx, const uint8_t *rgb, int32_t h, int32_t w, int64_t row_stride_bytes,
                                   int32_t levels, int32_t patch_radius, void *pyr, void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!rgb || !pyr) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_size(h, w))) return st;
    if (row_stride_bytes < (int64_t)w * 3) return fail(FB_E_INVALID, "row_stride_bytes must be at least 3 w");
    if (levels < 1 || levels > kMaxLevels) return fail(FB_E_INVALID, "levels must be in [1, 16]");
    if (!valid_p(patch_radius)) return fail(FB_E_UNSUPPORTED, "patch_radius must be in [1, 4]");
    const PyrLayout L = pyr_layout(h, w, levels, patch_radius);
    hipStream_t s = static_cast<hipStream_t>(stream);
    FB_HIP(launch_pack_rgbx(nullptr, FrameRef{rgb, row_stride_bytes}, 1, h, w, patch_radius,
                            static_cast<uint8_t *>(pyr), 0, L.lv[0].px_off, L.lv[0].pitch, s));
    for (int l = 1; l < levels; ++l)
        FB_HIP(launch_downsample(static_cast<uint8_t *>(pyr), 0, 1, L.lv[l - 1], L.lv[l],
                                 patch_radius, s));
    FB_HIP(launch_bound_tables(static_cast<uint8_t *>(pyr), 0, 1, L, s));
    return FB_OK;
}

fb_status fb_nnf_init(fb_ctx *ctx, const void *src_pyr, const void *tgt_pyr, int32_t h, int32_t w,
                      int32_t level, const fb_params *params, uint32_t pair_id,
                      const int32_t *seed_offsets, int32_t *nnf, uint32_t *energy, void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!src_pyr || !tgt_pyr || !nnf || !energy) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_size(h, w)) || (st = check_params(params, false))) return st;
    if (params->flags & FB_STYLE_LOSS)
        return fail(FB_E_UNSUPPORTED, "FB_STYLE_LOSS is taken by fb_blend_window and fb_patchmatch_batch only");
    if (level < 0 || level >= kMaxLevels) return fail(FB_E_INVALID, "level must be in [0, 15]");
    const int p = params->patch_radius;
    const PyrLayout L = pyr_layout(h, w, level + 1, p);
    const size_t npx = (size_t)L.lv[level].h * L.lv[level].w;
    if ((st = ensure(ctx, ctx->fe, npx * 8))) return st;
    uint32_t *f = static_cast<uint32_t *>(ctx->fe.p), *e = f + npx;
    PairSpec ps{};
    ps.src_pyr = static_cast<const uint8_t *>(src_pyr);
    ps.tgt_pyr = static_cast<const uint8_t *>(tgt_pyr);
    ps.L = L;
    ps.pair_id = pair_id;
    Plan P;
    const TileCfg cfg = choose_cfg(ctx, "", FB_NO_AUTOTUNE);
    PMJob j = job_geom(ps, level);
    j.mode = seed_offsets ? kStartOffsets : kStartRandom;
    j.aux_off = seed_offsets;
    j.f_out = f;
    j.e_out = e;
    add_pm_launch(P, kLaunchStart, {j}, cfg, p, params->seed, 0);
    j = job_geom(ps, level);
    j.f_in = f;
    j.e_in = e;
    j.nnf_abi = nnf;
    j.energy_abi = energy;
    add_pm_launch(P, kLaunchExport, {j}, cfg, p, params->seed, 0);
    return run_plan(ctx, P, params->flags, static_cast<hipStream_t>(stream), p, params->seed);
}

fb_status fb_patchmatch_level(fb_ctx *ctx, const void *src_pyr, const void *tgt_pyr, int32_t h,
                              int32_t w, int32_t level, const fb_params *params, uint32_t pair_id,
                              const int32_t *nnf_coarse, int32_t *nnf, uint32_t *energy,
                              void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!src_pyr || !tgt_pyr || !nnf || !energy) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_size(h, w)) || (st = check_params(params, false))) return st;
    if (params->flags & FB_STYLE_LOSS)
        return fail(FB_E_UNSUPPORTED, "FB_STYLE_LOSS is taken by fb_blend_window and fb_patchmatch_batch only");
    if (level < 0 || level >= kMaxLevels - 1) return fail(FB_E_INVALID, "level must be in [0, 14]");
    const int p = params->patch_radius;
    const PyrLayout L = pyr_layout(h, w, level + 2, p);  // level + 1 for the coarse size only
    const size_t npx = (size_t)L.lv[level].h * L.lv[level].w;
    if ((st = ensure(ctx, ctx->fe, npx * 16))) return st;
    uint32_t *base = static_cast<uint32_t *>(ctx->fe.p);
    PairSpec ps{};
    ps.src_pyr = static_cast<const uint8_t *>(src_pyr);
    ps.tgt_pyr = static_cast<const uint8_t *>(tgt_pyr);
    ps.L = L;
    ps.pair_id = pair_id;
    ps.f[0] = base;
    ps.f[1] = base + npx;
    ps.e[0] = base + 2 * npx;
    ps.e[1] = base + 3 * npx;
    Plan P;
    const TileCfg cfg = choose_cfg(ctx, "", FB_NO_AUTOTUNE);
    PMJob j = job_geom(ps, level);
    if (nnf_coarse) {
        j.mode = kStartUpsampleAbi;
        j.aux_off = nnf_coarse;
        j.hc = L.lv[level + 1].h;
        j.wc = L.lv[level + 1].w;
    } else {
        j.mode = kStartCopyAbi;
        j.aux_off = nnf;
        j.e_abi = energy;
    }
    j.f_out = ps.f[0];
    j.e_out = ps.e[0];
    add_pm_launch(P, kLaunchStart, {j}, cfg, p, params->seed, 0);
    int cur = 0;
    for (int it = 0; it < params->iters; ++it) {
        j = job_geom(ps, level);
        j.f_in = ps.f[cur];
        j.e_in = ps.e[cur];
        j.f_out = ps.f[cur ^ 1];
        j.e_out = ps.e[cur ^ 1];
        cur ^= 1;
        add_pm_launch(P, kLaunchIter, {j}, cfg, p, params->seed, it);
    }
    j = job_geom(ps, level);
    j.f_in = ps.f[cur];
    j.e_in = ps.e[cur];
    j.nnf_abi = nnf;
    j.energy_abi = energy;
    add_pm_launch(P, kLaunchExport, {j}, cfg, p, params->seed, 0);
    return run_plan(ctx, P, params->flags, static_cast<hipStream_t>(stream), p, params->seed);
}

fb_status fb_patchmatch_level_noalloc(fb_ctx *ctx, const void *src_pyr, const void *tgt_pyr, int32_t h,
                                      int32_t w, int32_t level, const fb_params *params, uint32_t pair_id,
                                      const int32_t *nnf_coarse, int32_t *nnf, uint32_t *energy,
                                      void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!src_pyr || !tgt_pyr || !nnf || !energy) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_size(h, w)) || (st = check_params(params, false))) return st;
    if (params->flags & FB_STYLE_LOSS)
        return fail(FB_E_UNSUPPORTED, "FB_STYLE_LOSS is taken by fb_blend_window and fb_patchmatch_batch only");
    if (level < 0 || level >= kMaxLevels - 1) return fail(FB_E_INVALID, "level must be in [0, 14]");
    uint8_t *base = static_cast<uint8_t *>(g_scratch_ptr[ctx->device]);
    if (!base) return fail(FB_E_INVALID, "the context's device has no working array");
    const int p = params->patch_radius;
    const PyrLayout L = pyr_layout(h, w, level + 2, p);  // level + 1 for the coarse size only
    const size_t npx = (size_t)L.lv[level].h * L.lv[level].w;
    if (npx > kNoAllocPixels)
        return fail(FB_E_UNSUPPORTED, "fb_patchmatch_level_noalloc takes levels of at most 1048576 pixels");
    uint32_t *f[2] = {reinterpret_cast<uint32_t *>(base), reinterpret_cast<uint32_t *>(base) + npx};
    uint32_t *e[2] = {reinterpret_cast<uint32_t *>(base) + 2 * npx, reinterpret_cast<uint32_t *>(base) + 3 * npx};
    PMJob *djobs = reinterpret_cast<PMJob *>(base + kNoAllocFieldBytes);
    PairSpec ps{};
    ps.src_pyr = static_cast<const uint8_t *>(src_pyr);
    ps.tgt_pyr = static_cast<const uint8_t *>(tgt_pyr);
    ps.L = L;
    ps.pair_id = pair_id;
    const TileCfg cfg = tile_cfg(ctx->forced_cfg >= 0 ? ctx->forced_cfg : 0);
    const LevelGeom &g = L.lv[level];
    const int tiles_x = (g.w + cfg.tw - 1) / cfg.tw;
    const int total = tiles_x * ((g.h + cfg.th - 1) / cfg.th);
    NoAllocJobs J;
    std::memset(&J, 0, sizeof J);
    // 0: start of the level; 1, 2: even and odd iterations; 3: export
    for (int k = 0; k < kNoAllocJobs; ++k) {
        J.j[k] = job_geom(ps, level);
        J.j[k].tiles_x = tiles_x;
        J.j[k].tile_base = 0;
    }
    if (nnf_coarse) {
        J.j[0].mode = kStartUpsampleAbi;
        J.j[0].aux_off = nnf_coarse;
        J.j[0].hc = L.lv[level + 1].h;
        J.j[0].wc = L.lv[level + 1].w;
    } else {
        J.j[0].mode = kStartCopyAbi;
        J.j[0].aux_off = nnf;
        J.j[0].e_abi = energy;
    }
    J.j[0].f_out = f[0];
    J.j[0].e_out = e[0];
    for (int k = 0; k < 2; ++k) {
        J.j[1 + k].f_in = f[k];
        J.j[1 + k].e_in = e[k];
        J.j[1 + k].f_out = f[k ^ 1];
        J.j[1 + k].e_out = e[k ^ 1];
    }
    const int fin = params->iters & 1;
    J.j[3].f_in = f[fin];
    J.j[3].e_in = e[fin];
    J.j[3].nnf_abi = nnf;
    J.j[3].energy_abi = energy;
    const int tab_bytes = (J.j[1].tab_n * 12 + 15) & ~15;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_store_jobs, dim3(1), dim3(64), 0, s, J, djobs, kNoAllocJobs);
    FB_HIP(hipGetLastError());
    FB_HIP(launch_pm_start(djobs, 1, total, total, cfg, p, params->seed, s));
    for (int it = 0; it < params->iters; ++it)
        FB_HIP(launch_pm_iter(djobs + 1 + (it & 1), 1, total, total, cfg, p, it, params->seed, kIterPlain,
                              tab_bytes, s));
    FB_HIP(launch_pm_export(djobs + 3, 1, total, total, cfg, s));
    return FB_OK;
}

fb_status fb_remap(fb_ctx *ctx, const uint8_t *style, const int32_t *nnf, int32_t h, int32_t w,
                   int32_t patch_radius, float *out, void *stream) {
    return fb_remap_strided(ctx, style, (int64_t)w * 3, nnf, h, w, patch_radius, out, stream);
}

fb_status fb_remap_strided(fb_ctx *ctx, const uint8_t *style, int64_t row_stride_bytes, const int32_t *nnf,
                           int32_t h, int32_t w, int32_t patch_radius, float *out, void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!style || !nnf || !out) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_size(h, w))) return st;
    if (row_stride_bytes < (int64_t)w * 3) return fail(FB_E_INVALID, "row_stride_bytes must be at least 3 w");
    if (!valid_p(patch_radius)) return fail(FB_E_UNSUPPORTED, "patch_radius must be in [1, 4]");
    const int p = patch_radius;
    int32_t pitch = 0;
    const size_t sbytes = padded_image_bytes(h, w, p, &pitch);
    const size_t npx = (size_t)h * w;
    if ((st = ensure(ctx, ctx->style, sbytes)) || (st = ensure(ctx, ctx->fe, npx * 4))) return st;
    uint8_t *sty = static_cast<uint8_t *>(ctx->style.p);
    uint32_t *f = static_cast<uint32_t *>(ctx->fe.p);
    Plan P;
    plan_style_pack(P, Frames{FrameRef{style, row_stride_bytes}}, h, w, p, sty, sbytes, pitch);
    sig_add(P, "f2p", (long long)(uintptr_t)nnf, h, w, (long long)(uintptr_t)f);
    P.ops.push_back({FB_KERNEL_OTHER, [=](hipStream_t s, const uint8_t *) {
        return launch_field_to_packed(nnf, f, h, w, s);
    }});
    RemapTerm t{reinterpret_cast<const uint32_t *>(sty), f, 1.0f, 0};
    RemapFrame fr{out, 0, 1, 1.0f, 0};
    add_remap_launch(P, {fr}, {t}, h, w, pitch, p);
    return run_plan(ctx, P, 0, static_cast<hipStream_t>(stream), p, 0);
}

}  // extern "C"

static fb_status blend_window_impl(fb_ctx *ctx, const Frames &guides, const Frames &styles, int32_t n_frames,
                                   int32_t h, int32_t w, int32_t radius_M, const fb_params *params,
                                   float *out, void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!out) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_size(h, w)) || (st = check_params(params, true))) return st;
    if (n_frames < 1) return fail(FB_E_INVALID, "n_frames must be >= 1");
    if (radius_M < 0) return fail(FB_E_INVALID, "radius_M must be >= 0");
    const int N = n_frames, M = radius_M, p = params->patch_radius, K = params->levels;
    if ((uint64_t)N * (uint64_t)N > 0xFFFFFFFFull) return fail(FB_E_UNSUPPORTED, "pair ids j*N+i must fit in 32 bits");
    if (params->flags & FB_FAST_BLEND)
        return blend_fast(ctx, guides, styles, N, h, w, M, params, out, static_cast<hipStream_t>(stream));
    if (params->flags & FB_ACCURATE_BLEND)
        return blend_accurate(ctx, guides, styles, N, h, w, M, params, out, static_cast<hipStream_t>(stream));
    const PyrLayout L = pyr_layout(h, w, K, p);
    int32_t pitch = 0;
    const size_t pbytes = padded_image_bytes(h, w, p, &pitch);
    // with the Eq. 3 loss the styles get whole pyramids (level 0 of a pyramid
    // is laid out as a padded frame)
    const bool style = params->flags & FB_STYLE_LOSS;
    const size_t sbytes = style ? L.bytes : pbytes;
    const size_t npx = (size_t)h * w;
    size_t n_pairs = 0;
    for (int i = 0; i < N; ++i) n_pairs += (size_t)(std::min(N - 1, i + M) - std::max(0, i - M));
    if ((st = ensure(ctx, ctx->pyr, (size_t)N * L.bytes)) ||
        (st = ensure(ctx, ctx->style, (size_t)N * sbytes)) ||
        (st = ensure(ctx, ctx->fe, std::max<size_t>(n_pairs, 1) * npx * 16)) ||
        (style && (st = ensure(ctx, ctx->shat, std::max<size_t>(n_pairs, 1) * pbytes))))
        return st;
    uint8_t *pyr = static_cast<uint8_t *>(ctx->pyr.p);
    uint8_t *sty = static_cast<uint8_t *>(ctx->style.p);
    uint32_t *fe = static_cast<uint32_t *>(ctx->fe.p);
    uint8_t *shat = static_cast<uint8_t *>(ctx->shat.p);

    Plan P;
    plan_pyramids(P, guides, h, w, L, pyr, L.bytes);
    if (style) plan_pyramids(P, styles, h, w, L, sty, L.bytes, false);
    else plan_style_pack(P, styles, h, w, p, sty, sbytes, pitch);
    std::vector<PairSpec> pairs;
    pairs.reserve(n_pairs);
    for (int i = 0; i < N; ++i)
        for (int j = std::max(0, i - M); j <= std::min(N - 1, i + M); ++j) {
            if (j == i) continue;
            const size_t k = pairs.size();
            PairSpec ps{};
            ps.src_pyr = pyr + (size_t)j * L.bytes;
            ps.tgt_pyr = pyr + (size_t)i * L.bytes;
            ps.L = L;
            ps.pair_id = (uint32_t)j * (uint32_t)N + (uint32_t)i;
            ps.f[0] = fe + k * npx;
            ps.f[1] = fe + (n_pairs + k) * npx;
            ps.e[0] = fe + (2 * n_pairs + k) * npx;
            ps.e[1] = fe + (3 * n_pairs + k) * npx;
            if (style) {
                ps.src_sty_pyr = sty + (size_t)j * sbytes;
                ps.sty_hat = reinterpret_cast<uint32_t *>(shat + k * pbytes);
            }
            pairs.push_back(ps);
        }
    if (params->flags & FB_LEARNED_SEED)
        if ((st = plan_learned_seeds(ctx, P, pairs))) return st;
    GuardPlan gp;
    if ((st = prepare_guard(ctx, pairs, params, !style, &gp))) return st;
    const TileCfg cfg = choose_cfg(ctx, tune_key_of(pairs, p), params->flags);
    plan_patchmatch(P, pairs, params->iters, p, params->seed, cfg, style, params->alpha16, false, false, false, &gp);

    std::vector<RemapTerm> terms;
    std::vector<RemapFrame> frames;
    size_t k = 0;
    for (int i = 0; i < N; ++i) {
        const int lo = std::max(0, i - M), hi = std::min(N - 1, i + M);
        RemapFrame fr{out + (size_t)i * npx * 3, (int32_t)terms.size(), hi - lo + 1,
                      (float)(hi - lo + 1), 0};
        for (int j = lo; j <= hi; ++j) {
            const uint32_t *spx = reinterpret_cast<const uint32_t *>(sty + (size_t)j * sbytes);
            if (j == i) {
                terms.push_back(RemapTerm{spx, nullptr, 1.0f, 0});
            } else {
                terms.push_back(RemapTerm{spx, pairs[k].f[pairs[k].final_buf], 1.0f, 0});
                ++k;
            }
        }
        frames.push_back(fr);
    }
    add_remap_launch(P, frames, terms, h, w, pitch, p);
    return run_plan(ctx, P, params->flags, static_cast<hipStream_t>(stream), p, params->seed);
}

static fb_status interpolate_impl(fb_ctx *ctx, const Frames &guides, int32_t n_frames, int32_t h, int32_t w,
                                  const int32_t *key_idx, const Frames &key_styles, int32_t n_keys,
                                  const fb_params *params, float *out, void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!key_idx || !out) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_size(h, w)) || (st = check_params(params, true))) return st;
    if (params->flags & (FB_STYLE_LOSS | FB_FAST_BLEND | FB_ACCURATE_BLEND))
        return fail(FB_E_UNSUPPORTED, "fb_interpolate takes FB_TRACKING and FB_ALIGN, not the blend's loss or modes");
    if (n_frames < 1 || n_keys < 1) return fail(FB_E_INVALID, "need n_frames >= 1 and n_keys >= 1");
    for (int k = 0; k < n_keys; ++k) {
        if (key_idx[k] < 0 || key_idx[k] >= n_frames) return fail(FB_E_INVALID, "key index out of range");
        if (k && key_idx[k] <= key_idx[k - 1]) return fail(FB_E_INVALID, "key indices must be sorted and unique");
    }
    const int N = n_frames, p = params->patch_radius, K = params->levels;
    if ((uint64_t)N * (uint64_t)N > 0xFFFFFFFFull) return fail(FB_E_UNSUPPORTED, "pair ids key*N+i must fit in 32 bits");
    const PyrLayout L = pyr_layout(h, w, K, p);
    int32_t pitch = 0;
    const size_t sbytes = padded_image_bytes(h, w, p, &pitch);
    const size_t npx = (size_t)h * w;
    // bracketing keys of every frame
    std::vector<int> kl(N, -1), kr(N, -1), kself(N, -1);
    for (int i = 0; i < N; ++i)
        for (int k = 0; k < n_keys; ++k) {
            if (key_idx[k] == i) kself[i] = k;
            if (key_idx[k] < i) kl[i] = k;
            if (key_idx[k] > i && kr[i] < 0) kr[i] = k;
        }
    size_t n_pairs = 0;
    for (int i = 0; i < N; ++i)
        if (kself[i] < 0) n_pairs += (kl[i] >= 0) + (kr[i] >= 0);
    const bool track = params->flags & FB_TRACKING, align = params->flags & FB_ALIGN;
    // with the alignment loss the keyframe styles get whole pyramids (level 0
    // of a pyramid is laid out as a padded frame)
    const size_t kbytes = align ? L.bytes : sbytes;
    if ((st = ensure(ctx, ctx->pyr, (size_t)N * L.bytes)) ||
        (st = ensure(ctx, ctx->style, (size_t)n_keys * kbytes)) ||
        (st = ensure(ctx, ctx->fe, std::max<size_t>(n_pairs, 1) * npx * 16)))
        return st;
    uint8_t *pyr = static_cast<uint8_t *>(ctx->pyr.p);
    uint8_t *sty = static_cast<uint8_t *>(ctx->style.p);
    uint32_t *fe = static_cast<uint32_t *>(ctx->fe.p);

    Plan P;
    plan_pyramids(P, guides, h, w, L, pyr, L.bytes);
    if (align) plan_pyramids(P, key_styles, h, w, L, sty, L.bytes, false);
    else plan_style_pack(P, key_styles, h, w, p, sty, sbytes, pitch);
    std::vector<PairSpec> pairs;
    std::vector<int> pair_key;
    for (int i = 0; i < N; ++i) {
        if (kself[i] >= 0) continue;
        for (int side = 0; side < 2; ++side) {
            const int k = side == 0 ? kl[i] : kr[i];
            if (k < 0) continue;
            const size_t q = pairs.size();
            PairSpec ps{};
            ps.src_pyr = pyr + (size_t)key_idx[k] * L.bytes;
            ps.tgt_pyr = pyr + (size_t)i * L.bytes;
            ps.L = L;
            ps.pair_id = (uint32_t)key_idx[k] * (uint32_t)N + (uint32_t)i;
            ps.f[0] = fe + q * npx;
            ps.f[1] = fe + (n_pairs + q) * npx;
            ps.e[0] = fe + (2 * n_pairs + q) * npx;
            ps.e[1] = fe + (3 * n_pairs + q) * npx;
            if (align) ps.src_sty_pyr = sty + (size_t)k * kbytes;
            pairs.push_back(ps);
            pair_key.push_back(k);
        }
    }
    // tracking neighbours (same key, adjacent target frames) and alignment
    // partners (same target frame, the other key)
    std::vector<int> pair_frame;
    for (int i = 0; i < N; ++i) {
        if (kself[i] >= 0) continue;
        for (int side = 0; side < 2; ++side)
            if ((side == 0 ? kl[i] : kr[i]) >= 0) pair_frame.push_back(i);
    }
    for (size_t a = 0; a < pairs.size(); ++a)
        for (size_t b = 0; b < pairs.size(); ++b) {
            if (pair_key[b] == pair_key[a] && pair_frame[b] == pair_frame[a] - 1) pairs[a].trk_prev = (int)b;
            if (pair_key[b] == pair_key[a] && pair_frame[b] == pair_frame[a] + 1) pairs[a].trk_next = (int)b;
            if (b != a && pair_frame[b] == pair_frame[a]) {
                pairs[a].partner = (int)b;
                if (align) pairs[a].partner_sty_pyr = sty + (size_t)pair_key[b] * kbytes;
            }
        }
    if (params->flags & FB_LEARNED_SEED)
        if ((st = plan_learned_seeds(ctx, P, pairs))) return st;
    GuardPlan gp;
    if ((st = prepare_guard(ctx, pairs, params, !track && !align, &gp))) return st;
    const TileCfg cfg = choose_cfg(ctx, tune_key_of(pairs, p), params->flags);
    plan_patchmatch(P, pairs, params->iters, p, params->seed, cfg, false, params->alpha16, false, track, align, &gp);

    std::vector<RemapTerm> terms;
    std::vector<RemapFrame> frames;
    size_t q = 0;
    for (int i = 0; i < N; ++i) {
        RemapFrame fr{out + (size_t)i * npx * 3, (int32_t)terms.size(), 0, 1.0f, 0};
        if (kself[i] >= 0) {
            terms.push_back(RemapTerm{reinterpret_cast<const uint32_t *>(sty + (size_t)kself[i] * kbytes),
                                      nullptr, 1.0f, 0});
        } else {
            const bool both = kl[i] >= 0 && kr[i] >= 0;
            const int l = both ? key_idx[kl[i]] : 0, r = both ? key_idx[kr[i]] : 0;
            for (int side = 0; side < 2; ++side) {
                const int k = side == 0 ? kl[i] : kr[i];
                if (k < 0) continue;
                float wgt = 1.0f;
                if (both) wgt = side == 0 ? (float)(r - i) / (float)(r - l) : (float)(i - l) / (float)(r - l);
                terms.push_back(RemapTerm{reinterpret_cast<const uint32_t *>(sty + (size_t)pair_key[q] * kbytes),
                                          pairs[q].f[pairs[q].final_buf], wgt, 0});
                ++q;
            }
        }
        fr.n_terms = (int32_t)terms.size() - fr.term_base;
        frames.push_back(fr);
    }
    add_remap_launch(P, frames, terms, h, w, pitch, p);
    return run_plan(ctx, P, params->flags, static_cast<hipStream_t>(stream), p, params->seed);
}

static fb_status frames_of(const fb_frame *in, int32_t n, int32_t w, Frames *out) {
    if (!in) return fail(FB_E_INVALID, "null pointer");
    if (n < 1) return fail(FB_E_INVALID, "need at least one frame");
    out->resize((size_t)n);
    for (int32_t k = 0; k < n; ++k) {
        if (!in[k].rgb) return fail(FB_E_INVALID, "null frame pointer");
        if (in[k].row_stride_bytes < (int64_t)w * 3) return fail(FB_E_INVALID, "row_stride_bytes must be at least 3 w");
        (*out)[k] = FrameRef{in[k].rgb, in[k].row_stride_bytes};
    }
    return FB_OK;
}

extern "C" {

fb_status fb_blend_window(fb_ctx *ctx, const uint8_t *guides, const uint8_t *styles, int32_t n_frames,
                          int32_t h, int32_t w, int32_t radius_M, const fb_params *params,
                          float *out, void *stream) {
    if (!ctx) return fail(FB_E_INVALID, "ctx is NULL");
    if (!guides || !styles) return fail(FB_E_INVALID, "null pointer");
    if (n_frames < 1 || h < 1 || w < 1) return fail(FB_E_INVALID, "n_frames and image sizes must be positive");
    return blend_window_impl(ctx, contiguous_frames(guides, n_frames, h, w), contiguous_frames(styles, n_frames, h, w),
                             n_frames, h, w, radius_M, params, out, stream);
}

fb_status fb_blend_window_frames(fb_ctx *ctx, const fb_frame *guides, const fb_frame *styles, int32_t n_frames,
                                 int32_t h, int32_t w, int32_t radius_M, const fb_params *params, float *out,
                                 void *stream) {
    if (!ctx) return fail(FB_E_INVALID, "ctx is NULL");
    Frames g, s;
    fb_status st;
    if ((st = frames_of(guides, n_frames, w, &g)) || (st = frames_of(styles, n_frames, w, &s))) return st;
    return blend_window_impl(ctx, g, s, n_frames, h, w, radius_M, params, out, stream);
}

fb_status fb_interpolate(fb_ctx *ctx, const uint8_t *guides, int32_t n_frames, int32_t h, int32_t w,
                         const int32_t *key_idx, const uint8_t *key_styles, int32_t n_keys,
                         const fb_params *params, float *out, void *stream) {
    if (!ctx) return fail(FB_E_INVALID, "ctx is NULL");
    if (!guides || !key_styles) return fail(FB_E_INVALID, "null pointer");
    if (n_frames < 1 || n_keys < 1 || h < 1 || w < 1)
        return fail(FB_E_INVALID, "need n_frames >= 1, n_keys >= 1 and positive image sizes");
    return interpolate_impl(ctx, contiguous_frames(guides, n_frames, h, w), n_frames, h, w, key_idx,
                            contiguous_frames(key_styles, n_keys, h, w), n_keys, params, out, stream);
}

fb_status fb_interpolate_frames(fb_ctx *ctx, const fb_frame *guides, int32_t n_frames, int32_t h, int32_t w,
                                const int32_t *key_idx, const fb_frame *key_styles, int32_t n_keys,
                                const fb_params *params, float *out, void *stream) {
    if (!ctx) return fail(FB_E_INVALID, "ctx is NULL");
    Frames g, k;
    fb_status st;
    if ((st = frames_of(guides, n_frames, w, &g)) || (st = frames_of(key_styles, n_keys, w, &k))) return st;
    return interpolate_impl(ctx, g, n_frames, h, w, key_idx, k, n_keys, params, out, stream);
}

fb_status fb_patchmatch_batch(fb_ctx *ctx, const fb_pair_desc *pairs_in, int32_t n_pairs,
                              const fb_params *params, void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!pairs_in || n_pairs < 1) return fail(FB_E_INVALID, "need n_pairs >= 1 descriptors");
    if ((st = check_params(params, false))) return st;
    const int p = params->patch_radius;
    const bool style = params->flags & FB_STYLE_LOSS;
    size_t total_px = 0, shat_bytes = 0;
    for (int k = 0; k < n_pairs; ++k) {
        const fb_pair_desc &d = pairs_in[k];
        if (!d.src_pyr || !d.tgt_pyr || !d.nnf || !d.energy) return fail(FB_E_INVALID, "null pointer in pair descriptor");
        if ((st = check_size(d.h, d.w))) return st;
        if (d.levels < 1 || d.levels > kMaxLevels) return fail(FB_E_INVALID, "levels must be in [1, 16]");
        if (style && !d.src_style_pyr) return fail(FB_E_INVALID, "FB_STYLE_LOSS needs src_style_pyr in every descriptor");
        total_px += (size_t)d.h * d.w;
        if (style) shat_bytes += padded_image_bytes(d.h, d.w, p, nullptr);
    }
    if ((st = ensure(ctx, ctx->fe, total_px * 16)) || (style && (st = ensure(ctx, ctx->shat, shat_bytes))))
        return st;
    uint32_t *fe = static_cast<uint32_t *>(ctx->fe.p);
    uint8_t *shat = static_cast<uint8_t *>(ctx->shat.p);
    size_t shat_off = 0;
    std::vector<PairSpec> pairs;
    size_t off = 0;
    for (int k = 0; k < n_pairs; ++k) {
        const fb_pair_desc &d = pairs_in[k];
        PairSpec ps{};
        ps.src_pyr = static_cast<const uint8_t *>(d.src_pyr);
        ps.tgt_pyr = static_cast<const uint8_t *>(d.tgt_pyr);
        ps.L = pyr_layout(d.h, d.w, d.levels, p);
        ps.pair_id = d.pair_id;
        ps.seed_offsets = d.seed_offsets;
        ps.f[0] = fe + off;
        ps.f[1] = fe + total_px + off;
        ps.e[0] = fe + 2 * total_px + off;
        ps.e[1] = fe + 3 * total_px + off;
        ps.nnf_abi = d.nnf;
        ps.energy_abi = d.energy;
        if (style) {
            ps.src_sty_pyr = static_cast<const uint8_t *>(d.src_style_pyr);
            ps.sty_hat = reinterpret_cast<uint32_t *>(shat + shat_off);
            shat_off += padded_image_bytes(d.h, d.w, p, nullptr);
        }
        off += (size_t)d.h * d.w;
        pairs.push_back(ps);
    }
    Plan P;
    if (params->flags & FB_LEARNED_SEED)
        if ((st = plan_learned_seeds(ctx, P, pairs))) return st;
    GuardPlan gp;
    if ((st = prepare_guard(ctx, pairs, params, !style, &gp))) return st;
    const TileCfg cfg = choose_cfg(ctx, tune_key_of(pairs, p), params->flags);
    plan_patchmatch(P, pairs, params->iters, p, params->seed, cfg, style, params->alpha16, false, false, false, &gp);
    return run_plan(ctx, P, params->flags, static_cast<hipStream_t>(stream), p, params->seed);
}

fb_status fb_guard_read(fb_ctx *ctx, uint64_t *sums, int32_t max_pairs, int32_t *n_pairs, void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!sums || !n_pairs || max_pairs < 0) return fail(FB_E_INVALID, "null pointer or negative size");
    const int n = (int)std::min<size_t>(ctx->guard_map.size(), (size_t)max_pairs);
    std::vector<uint64_t> dev(2 * (size_t)ctx->guard_n);
    if (ctx->guard_n) {
        hipStream_t s = static_cast<hipStream_t>(stream);
        FB_HIP(hipMemcpyAsync(dev.data(), ctx->gsum.p, dev.size() * 8, hipMemcpyDeviceToHost, s));
        FB_HIP(hipStreamSynchronize(s));
    }
    for (int k = 0; k < n; ++k) {
        const int g = ctx->guard_map[k];
        sums[2 * k] = g >= 0 ? dev[2 * g] : 0;
        sums[2 * k + 1] = g >= 0 ? dev[2 * g + 1] : 0;
    }
    *n_pairs = (int32_t)ctx->guard_map.size();
    return FB_OK;
}

int64_t fb_unet_param_count(void) { return unet_param_count(); }

static fb_status unet_ctx(fb_ctx *ctx) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!ctx->unet) ctx->unet = unet_create();
    return FB_OK;
}

fb_status fb_unet_load(fb_ctx *ctx, const float *params, void *stream) {
    fb_status st = unet_ctx(ctx);
    if (st) return st;
    if (!params) return fail(FB_E_INVALID, "params is NULL");
    FB_HIP(unet_load(ctx->unet, params, static_cast<hipStream_t>(stream)));
    return FB_OK;
}

fb_status fb_unet_save(fb_ctx *ctx, float *params, void *stream) {
    fb_status st = unet_ctx(ctx);
    if (st) return st;
    if (!params) return fail(FB_E_INVALID, "params is NULL");
    if (!unet_loaded(ctx->unet)) return fail(FB_E_INVALID, "no network parameters loaded");
    FB_HIP(unet_save(ctx->unet, params, static_cast<hipStream_t>(stream)));
    return FB_OK;
}

fb_status fb_unet_save_state(fb_ctx *ctx, float *params, float *adam_m, float *adam_v, int64_t *step,
                             void *stream) {
    fb_status st = unet_ctx(ctx);
    if (st) return st;
    if (!params || !adam_m || !adam_v || !step) return fail(FB_E_INVALID, "null pointer");
    if (!unet_loaded(ctx->unet)) return fail(FB_E_INVALID, "no network parameters loaded");
    FB_HIP(unet_save_state(ctx->unet, params, adam_m, adam_v, step, static_cast<hipStream_t>(stream)));
    return FB_OK;
}

fb_status fb_unet_load_state(fb_ctx *ctx, const float *params, const float *adam_m, const float *adam_v,
                             int64_t step, void *stream) {
    fb_status st = unet_ctx(ctx);
    if (st) return st;
    if (!params || !adam_m || !adam_v) return fail(FB_E_INVALID, "null pointer");
    if (step < 0 || step > 0x7FFFFFFF) return fail(FB_E_INVALID, "step must be in [0, 2^31 - 1]");
    FB_HIP(unet_load_state(ctx->unet, params, adam_m, adam_v, step, static_cast<hipStream_t>(stream)));
    return FB_OK;
}

fb_status fb_unet_forward(fb_ctx *ctx, const float *pair6, int32_t B, int32_t h, int32_t w, float *offsets,
                          void *stream) {
    fb_status st = unet_ctx(ctx);
    if (st) return st;
    if (!pair6 || !offsets) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_unet_shape(B, h, w))) return st;
    if (!unet_loaded(ctx->unet)) return fail(FB_E_INVALID, "no network parameters loaded");
    hipStream_t s = static_cast<hipStream_t>(stream);
    UNet *u = ctx->unet;
    FB_HIP(unet_reserve(u, B, h, w, false));
    FB_HIP(unet_input_from_f32(u, pair6, s));
    FB_HIP(unet_forward(u, s, false));
    FB_HIP(launch_pred_extract(unet_pred_buffer(u), (long)B * h * w, offsets, s));
    return FB_OK;
}

static fb_status unet_backward_common(fb_ctx *ctx, const float *pair6, const float *target, const float *mask,
                                      int32_t B, int32_t h, int32_t w, float *loss, hipStream_t s) {
    fb_status st = unet_ctx(ctx);
    if (st) return st;
    if (!pair6 || !target || !mask) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_unet_shape(B, h, w))) return st;
    if (!unet_loaded(ctx->unet)) return fail(FB_E_INVALID, "no network parameters loaded");
    UNet *u = ctx->unet;
    FB_HIP(unet_reserve(u, B, h, w, true));
    FB_HIP(unet_input_from_f32(u, pair6, s));
    FB_HIP(unet_forward(u, s, true));
    FB_HIP(unet_loss_backward(u, target, mask, true, s));
    if (loss) FB_HIP(hipMemcpyAsync(loss, unet_loss_buffer(u), sizeof(float), hipMemcpyDeviceToDevice, s));
    return FB_OK;
}

fb_status fb_unet_gradients(fb_ctx *ctx, const float *pair6, const float *target, const float *mask, int32_t B,
                            int32_t h, int32_t w, float *grads, float *loss, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!grads) return fail(FB_E_INVALID, "grads is NULL");
    fb_status st = unet_backward_common(ctx, pair6, target, mask, B, h, w, loss, s);
    if (st) return st;
    FB_HIP(unet_grads_flat(ctx->unet, grads, s));
    return FB_OK;
}

fb_status fb_unet_train_step(fb_ctx *ctx, const float *pair6, const float *target, const float *mask, int32_t B,
                             int32_t h, int32_t w, float lr, float *loss, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!(lr > 0.f)) return fail(FB_E_INVALID, "lr must be positive");
    fb_status st = unet_backward_common(ctx, pair6, target, mask, B, h, w, loss, s);
    if (st) return st;
    FB_HIP(unet_adam(ctx->unet, lr, s));
    return FB_OK;
}

double fb_unet_forward_flops(int32_t B, int32_t h, int32_t w) { return unet_forward_flops(B, h, w); }

fb_status fb_unet_pair_input(fb_ctx *ctx, const void *src_pyr, const void *tgt_pyr, int32_t h, int32_t w,
                             int32_t levels, int32_t patch_radius, float *pair6, void *stream) {
    fb_status st = begin(ctx);
    if (st) return st;
    if (!src_pyr || !tgt_pyr || !pair6) return fail(FB_E_INVALID, "null pointer");
    if ((st = check_size(h, w))) return st;
    if (levels < 1 || levels > kMaxLevels) return fail(FB_E_INVALID, "levels must be in [1, 16]");
    if (!valid_p(patch_radius)) return fail(FB_E_UNSUPPORTED, "patch_radius must be in [1, 4]");
    const PyrLayout L = pyr_layout(h, w, levels, patch_radius);
    const LevelGeom &g = L.lv[levels - 1];
    const UNetPairIn in{reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(src_pyr) + g.px_off),
                        reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(tgt_pyr) + g.px_off),
                        g.h, g.w, g.pitch, patch_radius};
    FB_HIP(launch_input_f32_from_pyramid(in, (g.h + 7) / 8 * 8, (g.w + 7) / 8 * 8, pair6,
                                         static_cast<hipStream_t>(stream)));
    return FB_OK;
}

}  // extern "C"
