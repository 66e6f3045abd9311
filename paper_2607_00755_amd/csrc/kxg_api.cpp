// C ABI of libkxg (declared in include/kxg.h): argument checks, handles,
// device memory, and the order of kernel launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "kxg_plan.h"
#include "kxg_step.h"

namespace kxg {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

static int div_up(long a, long b) { return (int)((a + b - 1) / b); }

// Process-wide gain-kernel profile: pairs of timing events.
struct Profile {
    bool on = false;
    std::vector<hipEvent_t> a, b;
    int used = 0;
};
static Profile g_prof;

void profile_mark_begin(hipStream_t s)
{
    if (g_prof.on && g_prof.used < (int)g_prof.a.size()) (void)hipEventRecord(g_prof.a[g_prof.used], s);
}

void profile_mark_end(hipStream_t s)
{
    if (g_prof.on && g_prof.used < (int)g_prof.a.size()) {
        (void)hipEventRecord(g_prof.b[g_prof.used], s);
        ++g_prof.used;
    }
}

static void profile_clear()
{
    for (auto e : g_prof.a) (void)hipEventDestroy(e);
    for (auto e : g_prof.b) (void)hipEventDestroy(e);
    g_prof = Profile{};
}

template <typename T>
static kxg_status dalloc(T **ptr, size_t count)
{
    if (hipMalloc((void **)ptr, count * sizeof(T)) != hipSuccess) {
        *ptr = nullptr;
        set_error("device allocation of %zu bytes failed", count * sizeof(T));
        return KXG_ENOMEM;
    }
    return KXG_OK;
}

static void release(kxg_kernel *k)
{
    if (!k) return;
    void *ptrs[] = {k->d_p, k->d_dp, k->d_E, k->d_K, k->d_h, k->d_A64, k->d_RT, k->d_R,
                    k->d_G32, k->d_Gbf, k->d_Gh, k->d_hrow, k->d_pairs, k->d_invdK,
                    k->d_AX64, k->d_AX32, k->d_JX, k->d_xpairs, k->d_xib,
                    k->d_pairs_c, k->d_cib, k->d_units, k->d_pairs16, k->d_cit16,
                    k->d_units16, k->d_act16, k->d_P64, k->d_P32, k->d_pairs64, k->d_ib64};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    free_workspace(k->ws);
    delete k;
}

}  // namespace kxg

using namespace kxg;

struct kxg_stepper {
    const kxg_kernel *k = nullptr;
    kxg_stepper_params prm{};
    SlotDev *d_slots = nullptr;
    double *d_x = nullptr, *d_fb = nullptr, *d_acc = nullptr, *d_xs = nullptr;
    double *d_dt = nullptr;
    Workspace ws;
    std::vector<char> used;
    int b_hi = 0;
    // captured iterations (HIP graphs) per batch bucket of 16 slots: one,
    // and kGraphIters in a row (fewer graph launches on long advances), and
    // the stream they were captured on; a bucket is captured on its first
    // use and kept, so that a batch moving between buckets (slots retired
    // and refilled) replays instead of capturing again
    struct Graphs {
        hipGraphExec_t one = nullptr, many = nullptr;
        hipStream_t stream = nullptr;
    };
    std::vector<Graphs> graphs;
    // staging of slot records for kxg_stepper_set_many: pinned host buffer,
    // its device copy, and an event that marks the end of the last copy
    SlotDev *h_init = nullptr;
    SlotDev *d_init = nullptr;
    hipEvent_t init_evt = nullptr;
};

template <typename T>
static hipError_t h2d(T *dst, const std::vector<T> &src)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Slot counts of the i-blocks, packed for the epilogue (16 bits each).
static SlotCounts pack_slot_counts(const std::vector<int> &per_ib)
{
    SlotCounts c;
    c.per_block = 1;
    for (size_t ib = 0; ib < per_ib.size() && ib < 32; ++ib)
        c.w[ib / 4] |= (uint64_t)(per_ib[ib] & 0xFFFF) << (16 * (ib % 4));
    return c;
}

static kxg_status build_compact(kxg_kernel *k, int b_cap, bool want64, bool want32, bool wantbf, bool wanth,
                                bool wantx64, bool wantx32, hipStream_t s)
{
    const Geometry &g = k->geo;
    const size_t nflags = (size_t)g.nib * g.npairs;
    unsigned char *d_flags = nullptr;
    unsigned int *d_nnz = nullptr;
    kxg_status st = dalloc(&d_flags, nflags);
    if (st == KXG_OK) st = dalloc(&d_nnz, nflags);
    if (st != KXG_OK) {
        if (d_flags) (void)hipFree(d_flags);
        return st;
    }
    std::vector<unsigned char> flags(nflags);
    std::vector<unsigned int> nnz(nflags);
    hipError_t e = launch_block_nz(*k, d_flags, d_nnz, s);
    if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), d_flags, nflags, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(nnz.data(), d_nnz, nflags * sizeof(unsigned int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_flags);
    (void)hipFree(d_nnz);
    if (e != hipSuccess) { set_error("kxg_kernel_build: %s", hipGetErrorString(e)); return KXG_EHIP; }
    k->nnz_packed = 0;
    for (unsigned int c : nnz) k->nnz_packed += c;
    // kept pairs of a group of i-blocks [ib0, ib0 + w), with the mask of
    // the group's non-zero i-blocks in each
    auto compact = [&](int w, std::vector<int> &pairs_c, std::vector<int> &cgrp, std::vector<int> &cnt,
                       std::vector<int> &first, std::vector<int> &mask) {
        const int ng = div_up(g.nib, w);
        cnt.assign(ng, 0);
        first.assign(ng, 0);
        for (int q = 0; q < ng; ++q) {
            first[q] = (int)cgrp.size();
            int pr = 0;
            for (int kb = 0; kb < g.nb; ++kb)
                for (int mb = kb; mb < g.nb; ++mb, ++pr) {
                    int bits = 0;
                    for (int ib = q * w; ib < std::min(g.nib, (q + 1) * w); ++ib)
                        if (flags[(size_t)ib * g.npairs + pr]) bits |= 1 << (ib - q * w);
                    if (!bits) continue;
                    pairs_c.push_back(kb);
                    pairs_c.push_back(mb);
                    cgrp.push_back(q);
                    mask.push_back(bits);
                    ++cnt[q];
                }
        }
    };
    const bool wantp32 = want32 && b_cap <= 4;
    if (want64 || wantp32) {
        // the plain evaluations (FP64; FP32 on single-distribution handles)
        // stream the kept blocks row by row; a workgroup takes one chunk of
        // one row (whole 16-byte load steps of 256 threads, at most one
        // round of loads per thread), sized so that one launch has about
        // KXG_PSTREAM_ROWS_TARGET non-empty workgroups
        std::vector<int> pairs_c, cib, cnt, first, mask;
        compact(1, pairs_c, cib, cnt, first, mask);
        k->ncomp64 = (long)cib.size();
        std::vector<int> tab(pairs_c);
        tab.insert(tab.end(), cib.begin(), cib.end());
        std::vector<int> ibt(2 * (size_t)g.nib);
        int maxcnt = 0;
        long total = 0;
        for (int ib = 0; ib < g.nib; ++ib) {
            ibt[2 * ib] = first[ib];
            ibt[2 * ib + 1] = cnt[ib];
            maxcnt = std::max(maxcnt, cnt[ib]);
            total += (long)cnt[ib] * std::min(kIBlk, k->n - ib * kIBlk) * 256;
        }
        auto split = [&](int bytes, int &chunk_out, int &nsplit_out) {
            const long step = 256 * (16 / bytes);
            long chunk = div_up(std::max<long>(1, total), KXG_PSTREAM_ROWS_TARGET);
            chunk = std::min<long>(std::max<long>(div_up(chunk, step) * step, 4 * step), pstream_chunk(bytes));
            chunk_out = (int)chunk;
            nsplit_out = std::max(1, div_up((long)maxcnt * 256, chunk));
        };
        const size_t vals = (size_t)std::max<long>(1, k->ncomp64) * kIBlk * 256;
        if (want64) {
            split(8, k->chunk64, k->nsplit64);
            st = dalloc(&k->d_P64, vals);
        }
        if (st == KXG_OK && wantp32) {
            split(4, k->chunk32, k->nsplit32);
            st = dalloc(&k->d_P32, vals);
        }
        if (st == KXG_OK) st = dalloc(&k->d_pairs64, std::max<size_t>(3, tab.size()));
        if (st == KXG_OK) st = dalloc(&k->d_ib64, ibt.size());
        if (st != KXG_OK) return st;
        e = h2d(k->d_pairs64, tab);
        if (e == hipSuccess) e = h2d(k->d_ib64, ibt);
        if (e == hipSuccess) e = launch_pack_rows(*k, s);
    }
    if (e == hipSuccess && (wantx64 || wantx32)) {
        // the exact forms stream A and the brackets over the blocks, in both
        // (kb, mb) orders, of every pair with a structural weight in the
        // i-block (a superset of the non-zero entries of A); a workgroup takes
        // whole load steps of one row, sized like the plain streams
        std::vector<int> xp, xc, xib(2 * (size_t)g.nib);
        int maxcnt = 0;
        long total = 0;
        for (int ib = 0; ib < g.nib; ++ib) {
            xib[2 * ib] = (int)xc.size();
            int pr = 0;
            for (int kb = 0; kb < g.nb; ++kb)
                for (int mb = kb; mb < g.nb; ++mb, ++pr) {
                    if (!nnz[(size_t)ib * g.npairs + pr]) continue;
                    xp.push_back(kb);
                    xp.push_back(mb);
                    xc.push_back(ib);
                    if (kb != mb) {
                        xp.push_back(mb);
                        xp.push_back(kb);
                        xc.push_back(ib);
                    }
                }
            xib[2 * ib + 1] = (int)xc.size() - xib[2 * ib];
            maxcnt = std::max(maxcnt, xib[2 * ib + 1]);
            total += (long)xib[2 * ib + 1] * std::min(kIBlk, k->n - ib * kIBlk) * 256;
        }
        k->nx = (long)xc.size();
        auto split = [&](int bytes, int &chunk_out, int &nsplit_out) {
            const long step = 256 * (16 / bytes);
            long chunk = div_up(std::max<long>(1, total), KXG_PSTREAM_ROWS_TARGET);
            chunk = std::max<long>(div_up(chunk, step) * step, 4 * step);
            chunk = std::min<long>(chunk, (long)kPStreamPairs / 2 * 256);   // (a multiple of both steps)
            chunk_out = (int)chunk;
            nsplit_out = std::max(1, div_up((long)maxcnt * 256, chunk));
        };
        xp.insert(xp.end(), xc.begin(), xc.end());
        const size_t vals = (size_t)std::max<long>(1, k->nx) * kIBlk * 256;
        if (wantx64) {
            split(8, k->chunkx64, k->nsplitx64);
            st = dalloc(&k->d_AX64, vals);
        }
        if (st == KXG_OK && wantx32) {
            split(4, k->chunkx32, k->nsplitx32);
            st = dalloc(&k->d_AX32, vals);
        }
        if (st == KXG_OK) st = dalloc(&k->d_JX, vals);
        if (st == KXG_OK) st = dalloc(&k->d_xpairs, std::max<size_t>(3, xp.size()));
        if (st == KXG_OK) st = dalloc(&k->d_xib, xib.size());
        if (st != KXG_OK) return st;
        e = h2d(k->d_xpairs, xp);
        if (e == hipSuccess) e = h2d(k->d_xib, xib);
        if (e == hipSuccess) e = launch_pack_exact(*k, s);
    }
    if (e == hipSuccess && want32) {
        std::vector<int> pairs_c, cib, cnt, first, mask;
        compact(1, pairs_c, cib, cnt, first, mask);
        k->ncomp = (long)cib.size();
        const int bbw = b_cap <= 32 ? 1 : (b_cap <= 64 ? 2 : 4);
        const Units U = make_units(cnt, first, kBlk / kF32SS, div_up(b_cap, 32 * bbw), KXG_GEMM_WG_TARGET);
        k->nunits = (int)(U.units.size() / 4);
        k->maxslots = U.maxslots;
        st = dalloc(&k->d_G32, (size_t)std::max<long>(1, k->ncomp) * kBlk * 512);
        if (st == KXG_OK) st = dalloc(&k->d_pairs_c, std::max<size_t>(2, pairs_c.size()));
        if (st == KXG_OK) st = dalloc(&k->d_cib, std::max<size_t>(1, cib.size()));
        if (st == KXG_OK) st = dalloc(&k->d_units, std::max<size_t>(4, U.units.size()));
        if (st != KXG_OK) return st;
        e = h2d(k->d_pairs_c, pairs_c);
        if (e == hipSuccess) e = h2d(k->d_cib, cib);
        if (e == hipSuccess) e = h2d(k->d_units, U.units);
        k->nslot = pack_slot_counts(U.nslot);
        if (e == hipSuccess) e = launch_pack_f32(*k, s);
    }
    if (e == hipSuccess && (wantbf || wanth)) {
        constexpr int w = KXG_LDS_IBW;
        std::vector<int> pairs_c, cit, cnt, first, mask;
        compact(w, pairs_c, cit, cnt, first, mask);
        k->ncomp16 = (long)cit.size();
        // The non-zero i-blocks of a kept pair are, but for a handful, the
        // first few of its group (the kinematic cuts empty the blocks of
        // large i first).  Each pair gets the count of i-blocks up to its
        // last non-zero one, the GEMM multiplies only those, and the pairs of
        // a group are reordered by that count (descending, stable) so that
        // work units can run with a fixed count each.
        std::vector<int> act(mask.size());
        for (size_t c = 0; c < mask.size(); ++c) act[c] = 32 - __builtin_clz((unsigned)mask[c]);
        k->mult16 = 0;
        for (size_t q = 0; q < cnt.size(); ++q) {
            const int f = first[q];
            std::vector<int> ord(cnt[q]);
            for (int j = 0; j < cnt[q]; ++j) ord[j] = f + j;
            std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return act[x] > act[y]; });
            std::vector<int> pc(2 * cnt[q]), ac(cnt[q]);
            for (int j = 0; j < cnt[q]; ++j) {
                pc[2 * j] = pairs_c[2 * ord[j]];
                pc[2 * j + 1] = pairs_c[2 * ord[j] + 1];
                ac[j] = act[ord[j]];
            }
            std::copy(pc.begin(), pc.end(), pairs_c.begin() + 2 * f);
            std::copy(ac.begin(), ac.end(), act.begin() + f);
            for (int j = f; j < f + cnt[q]; ++j) k->mult16 += act[j];
        }
        // A unit runs with the count of its first (largest) pair; a
        // super-step costs the staging and the F2 split (KXG_LDS_STEP_COST
        // blocks' worth of MFMA time) plus one per block multiplied.
        std::vector<double> wcost(act.size());
        for (size_t c = 0; c < act.size(); ++c) wcost[c] = KXG_LDS_STEP_COST + act[c];
        const Units U = make_units_cost(cnt, first, wcost, kBlk / KXG_LDS_SS,
                                        div_up(b_cap, 4 * KXG_LDS_BBW * 32), KXG_LDS_WG_TARGET);
        k->nunits16 = (int)(U.units.size() / 4);
        k->maxslots16 = U.maxslots;
        std::vector<int> nslot_ib(g.nib, 0);
        for (int ib = 0; ib < g.nib; ++ib) nslot_ib[ib] = U.nslot[ib / w];
        const size_t gsz = (size_t)std::max<long>(1, k->ncomp16) * w * kBlk * 1024;
        if (wantbf) st = dalloc(&k->d_Gbf, gsz);
        if (st == KXG_OK && wanth) st = dalloc(&k->d_Gh, gsz);
        if (st == KXG_OK) st = dalloc(&k->d_pairs16, std::max<size_t>(2, pairs_c.size()));
        if (st == KXG_OK) st = dalloc(&k->d_cit16, std::max<size_t>(1, cit.size()));
        if (st == KXG_OK) st = dalloc(&k->d_units16, std::max<size_t>(4, U.units.size()));
        if (st == KXG_OK) st = dalloc(&k->d_act16, std::max<size_t>(1, act.size()));
        if (st != KXG_OK) return st;
        e = h2d(k->d_pairs16, pairs_c);
        if (e == hipSuccess) e = h2d(k->d_act16, act);
        if (e == hipSuccess) e = h2d(k->d_cit16, cit);
        if (e == hipSuccess) e = h2d(k->d_units16, U.units);
        k->nslot16 = pack_slot_counts(nslot_ib);
        if (e == hipSuccess) e = launch_pack_16(*k, w, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_error("kxg_kernel_build: %s", hipGetErrorString(e)); return KXG_EHIP; }
    return KXG_OK;
}

extern "C" {

const char *kxg_last_error(void) { return g_err; }

kxg_status kxg_profile_begin(int32_t capacity)
{
    g_err[0] = 0;
    if (capacity < 1 || capacity > (1 << 20)) { set_error("kxg_profile_begin: bad capacity"); return KXG_EINVAL; }
    profile_clear();
    g_prof.a.resize(capacity);
    g_prof.b.resize(capacity);
    for (int i = 0; i < capacity; ++i) {
        if (hipEventCreate(&g_prof.a[i]) != hipSuccess || hipEventCreate(&g_prof.b[i]) != hipSuccess) {
            g_prof.a.resize(i);
            g_prof.b.resize(i);
            profile_clear();
            set_error("kxg_profile_begin: hipEventCreate failed");
            return KXG_EHIP;
        }
    }
    g_prof.on = true;
    return KXG_OK;
}

kxg_status kxg_profile_end(double *total_ms, int32_t *launches)
{
    g_err[0] = 0;
    if (!total_ms || !launches) { set_error("kxg_profile_end: null output"); return KXG_EINVAL; }
    double tot = 0.0;
    for (int i = 0; i < g_prof.used; ++i) {
        float ms = 0.0f;
        if (hipEventSynchronize(g_prof.b[i]) != hipSuccess ||
            hipEventElapsedTime(&ms, g_prof.a[i], g_prof.b[i]) != hipSuccess) {
            profile_clear();
            set_error("kxg_profile_end: event query failed");
            return KXG_EHIP;
        }
        tot += ms;
    }
    *total_ms = tot;
    *launches = g_prof.used;
    profile_clear();
    return KXG_OK;
}

kxg_status kxg_peak_probe(double *out, void *stream)
{
    // out[0..3]: FP32 and BF16 MFMA TFLOP/s, read and copy GB/s
    g_err[0] = 0;
    if (!out) { set_error("kxg_peak_probe: null output"); return KXG_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    constexpr int kWg = 1024, kIters = 4096;          // four waves per SIMD on 256 CUs
    constexpr int kReadWg = 8192;                      // 128 KiB of the 1 GiB read each
    constexpr long kVec = (512L << 20) / 16;           // 512 MiB in 16-byte vectors
    float *sink = nullptr;
    char *buf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    kxg_status rs = dalloc(&sink, (size_t)kReadWg * 256);
    if (rs == KXG_OK) rs = dalloc(&buf, (size_t)2 * kVec * 16);
    if (rs != KXG_OK) {
        if (sink) (void)hipFree(sink);
        return rs;
    }
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // best of three timed launches after one untimed one
    auto best_ms = [&](auto &&launch) {
        float best = 0.0f;
        for (int r = 0; r < 4 && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = launch();
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (r > 0 && (best == 0.0f || ms < best)) best = ms;
        }
        return (double)best;
    };
    const double waves = (double)kWg * 4 * kIters * 4;  // MFMAs per launch
    const double f32 = best_ms([&] { return launch_peak_mfma(0, kWg, kIters, sink, st); });
    const double b16 = best_ms([&] { return launch_peak_mfma(1, kWg, kIters, sink, st); });
    const double cp = best_ms([&] { return launch_copy16(buf, buf + kVec * 16, kVec, st); });
    const double rd = best_ms([&] { return launch_read16(buf, 2 * kVec, sink, kReadWg, st); });
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    (void)hipFree(buf);
    if (e != hipSuccess || f32 <= 0.0 || b16 <= 0.0 || cp <= 0.0 || rd <= 0.0) {
        set_error("kxg_peak_probe: %s", hipGetErrorString(e));
        return KXG_EHIP;
    }
    out[0] = waves * 4096.0 / (f32 * 1e-3) / 1e12;
    out[1] = waves * 32768.0 / (b16 * 1e-3) / 1e12;
    out[2] = 2.0 * kVec * 16 / (rd * 1e-3) / 1e9;
    out[3] = 2.0 * kVec * 16 / (cp * 1e-3) / 1e9;
    return KXG_OK;
}

kxg_status kxg_gauss_legendre(int32_t n, double *x, double *w)
{
    g_err[0] = 0;
    if (n < 1 || n > 100000 || !x || !w) {
        set_error("kxg_gauss_legendre: need n >= 1 and output arrays");
        return KXG_EINVAL;
    }
    gauss_legendre(n, x, w);
    return KXG_OK;
}


kxg_status kxg_kernel_build(const kxg_grid *grid, uint32_t prec_mask, int32_t b_cap,
                            void *stream, kxg_kernel **out)
{
    g_err[0] = 0;
    if (!grid || !out) { set_error("kxg_kernel_build: null grid or out"); return KXG_EINVAL; }
    *out = nullptr;
    const int n = grid->n;
    if (n < 4 || n > kMaxN) { set_error("kxg_kernel_build: n=%d outside [4, %d]", n, kMaxN); return KXG_EINVAL; }
    if (!grid->p) { set_error("kxg_kernel_build: p is NULL"); return KXG_EINVAL; }
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(grid->p[i]) || grid->p[i] <= 0.0) { set_error("kxg_kernel_build: p[%d] not finite and > 0", i); return KXG_EINVAL; }
        if (i > 0 && !(grid->p[i] > grid->p[i - 1])) { set_error("kxg_kernel_build: p not strictly increasing at %d", i); return KXG_EINVAL; }
        if (grid->dp && !(std::isfinite(grid->dp[i]) && grid->dp[i] > 0.0)) { set_error("kxg_kernel_build: dp[%d] not finite and > 0", i); return KXG_EINVAL; }
    }
    if (!(grid->mass > 0.0) || !(grid->g_dof > 0.0) || !(grid->m2 > 0.0) ||
        !std::isfinite(grid->mass) || !std::isfinite(grid->g_dof) || !std::isfinite(grid->m2)) {
        set_error("kxg_kernel_build: mass, g_dof and m2 must be finite and > 0");
        return KXG_EINVAL;
    }
    if (grid->quad != KXG_QUAD_GL && grid->quad != KXG_QUAD_EXACT) { set_error("kxg_kernel_build: bad quad %d", grid->quad); return KXG_EINVAL; }
    if (grid->quad == KXG_QUAD_GL && (grid->n_mu < 1 || grid->n_mu > 4096)) { set_error("kxg_kernel_build: n_mu=%d outside [1, 4096]", grid->n_mu); return KXG_EINVAL; }
    if (b_cap < 1 || b_cap > (1 << 20)) { set_error("kxg_kernel_build: b_cap=%d outside [1, 2^20]", b_cap); return KXG_EINVAL; }
    if (prec_mask & ~(0x1Fu | KXG_WITH_BRACKETS | KXG_LEAN)) { set_error("kxg_kernel_build: unknown precision bits 0x%x", prec_mask); return KXG_EINVAL; }
    hipStream_t s = static_cast<hipStream_t>(stream);

    kxg_kernel *k = new (std::nothrow) kxg_kernel;
    if (!k) { set_error("host allocation failed"); return KXG_ENOMEM; }
    k->n = n;
    k->mass = grid->mass;
    k->gdof = grid->g_dof;
    k->m2 = grid->m2;
    k->quad = grid->quad;
    k->nmu = grid->quad == KXG_QUAD_GL ? grid->n_mu : 0;
    k->b_cap = b_cap;
    const bool want_jl = (prec_mask & KXG_WITH_BRACKETS) != 0;
    // lean handles keep the dense FP64 tensor only when FP64 evaluations are
    // asked for, and the dense FP32 copy only where an evaluation streams it
    const bool lean = (prec_mask & KXG_LEAN) != 0;
    const bool keep64 = !lean || (prec_mask & KXG_PREC_BIT(KXG_F64));
    k->prec_mask = (prec_mask & 0x1Fu) | (keep64 ? KXG_PREC_BIT(KXG_F64) : 0u);
    k->p.assign(grid->p, grid->p + n);
    k->dp.resize(n);
    k->E.resize(n);
    k->K.resize(n);
    k->h.resize(n);
    // Energies, kinetic energies (K = p^2/(E+m), no cancellation), widths
    // (trapezoid in ln p unless given) and moment weights h = p^2 dp.
    for (int i = 0; i < n; ++i) {
        const double p = k->p[i];
        k->E[i] = std::sqrt(p * p + k->mass * k->mass);
        k->K[i] = (p * p) / (k->E[i] + k->mass);
    }
    for (int i = 0; i < n; ++i) {
        if (grid->dp) {
            k->dp[i] = grid->dp[i];
        } else {
            const double left = std::log(k->p[i > 0 ? i - 1 : i]);
            const double right = std::log(k->p[i < n - 1 ? i + 1 : i]);
            k->dp[i] = k->p[i] * (right - left) / 2.0;
        }
        k->h[i] = k->p[i] * k->p[i] * k->dp[i];
    }
    Geometry &g = k->geo;
    g.nb = div_up(n, kBlk);
    g.npairs = g.nb * (g.nb + 1) / 2;
    g.nib = div_up(n, kIBlk);
    g.ipad = g.nib * kIBlk;
    g.dksteps = (long)g.npairs * kBlk;

    const size_t n3 = (size_t)n * n * n, n2 = (size_t)n * n;
    const bool want32 = prec_mask & KXG_PREC_BIT(KXG_F32);
    const bool wantbf = prec_mask & KXG_PREC_BIT(KXG_BF16X3);
    // FP16 x3 and x2 share one operand (hi and lo of A; x2 reads the hi)
    const bool wanth = prec_mask & (KXG_PREC_BIT(KXG_F16X3) | KXG_PREC_BIT(KXG_F16X2));
    kxg_status st = KXG_OK;
#define KXG_ALLOC(ptr, cnt) \
    if (st == KXG_OK) st = dalloc(&(ptr), (cnt))
    KXG_ALLOC(k->d_p, n);
    KXG_ALLOC(k->d_dp, n);
    KXG_ALLOC(k->d_E, n);
    KXG_ALLOC(k->d_K, n);
    KXG_ALLOC(k->d_h, n);
    KXG_ALLOC(k->d_A64, n3);
    KXG_ALLOC(k->d_RT, n2);
    KXG_ALLOC(k->d_R, n2);
    KXG_ALLOC(k->d_pairs, 2 * (size_t)g.npairs);
    if (wanth) { KXG_ALLOC(k->d_hrow, (size_t)g.ipad); }
    if (want_jl) { KXG_ALLOC(k->d_invdK, (size_t)n); }
    double *d_xmu = nullptr, *d_wmu = nullptr;
    if (k->nmu > 0) { KXG_ALLOC(d_xmu, (size_t)k->nmu); KXG_ALLOC(d_wmu, (size_t)k->nmu); }
#undef KXG_ALLOC
    if (st != KXG_OK) {
        if (d_xmu) (void)hipFree(d_xmu);
        if (d_wmu) (void)hipFree(d_wmu);
        release(k);
        return st;
    }
    std::vector<int> pairs(2 * (size_t)g.npairs);
    {
        int q = 0;
        for (int kb = 0; kb < g.nb; ++kb)
            for (int mb = kb; mb < g.nb; ++mb) {
                pairs[2 * q] = kb;
                pairs[2 * q + 1] = mb;
                ++q;
            }
    }
    std::vector<double> xmu(k->nmu), wmu(k->nmu);
    if (k->nmu > 0) gauss_legendre(k->nmu, xmu.data(), wmu.data());
    hipError_t e = hipSuccess;
#define KXG_H2D(dst, src, bytes) \
    if (e == hipSuccess) e = hipMemcpy((dst), (src), (bytes), hipMemcpyHostToDevice)
    KXG_H2D(k->d_p, k->p.data(), n * sizeof(double));
    KXG_H2D(k->d_dp, k->dp.data(), n * sizeof(double));
    KXG_H2D(k->d_E, k->E.data(), n * sizeof(double));
    KXG_H2D(k->d_K, k->K.data(), n * sizeof(double));
    KXG_H2D(k->d_h, k->h.data(), n * sizeof(double));
    KXG_H2D(k->d_pairs, pairs.data(), pairs.size() * sizeof(int));
    if (k->nmu > 0) {
        KXG_H2D(d_xmu, xmu.data(), k->nmu * sizeof(double));
        KXG_H2D(d_wmu, wmu.data(), k->nmu * sizeof(double));
    }
    if (want_jl) {
        std::vector<double> inv(n, 0.0);
        for (int j = 0; j + 1 < n; ++j) inv[j] = 1.0 / (k->K[j + 1] - k->K[j]);
        KXG_H2D(k->d_invdK, inv.data(), n * sizeof(double));
    }
#undef KXG_H2D
    if (e == hipSuccess) e = launch_build_A(*k, d_xmu, d_wmu, s);
    if (e == hipSuccess) e = launch_build_R(*k, s);
    if (e == hipSuccess) e = launch_derive(*k, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (d_xmu) (void)hipFree(d_xmu);
    if (d_wmu) (void)hipFree(d_wmu);
    if (e != hipSuccess) {
        set_error("kxg_kernel_build: %s", hipGetErrorString(e));
        release(k);
        return KXG_EHIP;
    }
    if (keep64 || want32 || wantbf || wanth) {
        st = build_compact(k, b_cap, keep64, want32, wantbf, wanth, want_jl && keep64, want_jl && want32, s);
        if (st != KXG_OK) { release(k); return st; }
    }
    if (!keep64) {
        (void)hipFree(k->d_A64);
        k->d_A64 = nullptr;
    }
    st = alloc_workspace(*k, b_cap, k->ws);
    if (st != KXG_OK) { release(k); return st; }
    // tensors an evaluation at each precision reads
    // (plain evaluations: the packed kept blocks and R; the exact forms: A
    // and the brackets over their blocks)
    const size_t packed64 = k->d_P64 ? (size_t)k->ncomp64 * kIBlk * 256 : 0;
    const size_t packed32 = k->d_P32 ? (size_t)k->ncomp64 * kIBlk * 256 : 0;
    const size_t xvals = (size_t)k->nx * kIBlk * 256;
    const size_t jl = k->d_JX ? xvals * sizeof(uint16_t) : 0;
    const size_t ax64 = k->d_AX64 ? xvals * sizeof(double) : 0, ax32 = k->d_AX32 ? xvals * sizeof(float) : 0;
    if (keep64) k->bytes[KXG_F64] = (packed64 + n2) * sizeof(double) + (ax64 ? ax64 + jl : 0);
    if (want32)
        k->bytes[KXG_F32] = (packed32 + (size_t)k->ncomp * kBlk * 512) * sizeof(float) + n2 * sizeof(double) +
                            (ax32 ? ax32 + jl : 0);
    const size_t packed16 = (size_t)k->ncomp16 * KXG_LDS_IBW * kBlk * 1024;   // hi + lo values
    if (wantbf) k->bytes[KXG_BF16X3] = packed16 * sizeof(uint16_t) + n2 * sizeof(double);
    if (prec_mask & KXG_PREC_BIT(KXG_F16X3)) k->bytes[KXG_F16X3] = packed16 * sizeof(uint16_t) + n2 * sizeof(double);
    // (FP16 x2 reads the hi halves only)
    if (prec_mask & KXG_PREC_BIT(KXG_F16X2)) k->bytes[KXG_F16X2] = packed16 / 2 * sizeof(uint16_t) + n2 * sizeof(double);
    // everything the handle holds on the device
    const size_t fbytes = (size_t)k->geo.nb * k->ws.bpad_cap * kBlk * sizeof(float);
    k->held = 5 * (size_t)n * sizeof(double) + 2 * n2 * sizeof(double) + 2 * (size_t)g.npairs * sizeof(int) +
              (k->d_A64 ? n3 * sizeof(double) : 0) + ax64 + ax32 + jl +
              (k->d_xpairs ? (3 * (size_t)k->nx + 2 * (size_t)g.nib) * sizeof(int) : 0) +
              (want_jl ? (size_t)n * sizeof(double) : 0) +
              (size_t)k->ncomp * kBlk * 512 * sizeof(float) + (wantbf ? packed16 * sizeof(uint16_t) : 0) +
              packed64 * sizeof(double) + packed32 * sizeof(float) +
              (k->ncomp64 || packed64 || packed32 ? (3 * (size_t)k->ncomp64 + 2 * (size_t)g.nib) * sizeof(int) : 0) +
              (wanth ? packed16 * sizeof(uint16_t) + (size_t)g.ipad * sizeof(float) : 0) +
              k->ws.part_bytes + 2 * fbytes + (size_t)k->ws.bpad_cap * sizeof(float);
    *out = k;
    return KXG_OK;
}

void kxg_kernel_free(kxg_kernel *k) { release(k); }

int32_t kxg_kernel_n(const kxg_kernel *k) { return k ? k->n : 0; }

size_t kxg_kernel_bytes(const kxg_kernel *k, int32_t prec)
{
    if (!k) return 0;
    if (prec >= 0 && prec < 5) return k->bytes[prec];
    return k->held;
}

kxg_status kxg_kernel_stats(const kxg_kernel *k, kxg_kernel_info *out)
{
    g_err[0] = 0;
    if (!k || !out) { set_error("kxg_kernel_stats: null argument"); return KXG_EINVAL; }
    out->n = k->n;
    out->packed_blocks = (int64_t)k->geo.nib * k->geo.npairs;
    out->nonzero_blocks = k->d_G32 ? k->ncomp : 0;
    out->gemm_units = k->nunits;
    out->max_slots = k->maxslots;
    out->blocks16 = (k->d_Gbf || k->d_Gh) ? k->mult16 : 0;
    out->staged16 = (k->d_Gbf || k->d_Gh) ? k->ncomp16 * KXG_LDS_IBW : 0;
    out->blocks64 = (k->d_P64 || k->d_P32) ? k->ncomp64 : 0;
    out->blocks_exact = k->d_JX ? k->nx : 0;
    out->nnz_packed = (k->d_G32 || k->d_Gbf || k->d_Gh) ? k->nnz_packed : 0;
    return KXG_OK;
}

kxg_status kxg_kernel_export(const kxg_kernel *k, double *A_host, double *R_host)
{
    g_err[0] = 0;
    if (!k) { set_error("kxg_kernel_export: null handle"); return KXG_EINVAL; }
    const size_t n = k->n;
    if (A_host && !k->d_A64) { set_error("kxg_kernel_export: lean handle without the FP64 tensor"); return KXG_EUNSUPPORTED; }
    if (A_host) KXG_TRY_HIP(hipMemcpy(A_host, k->d_A64, n * n * n * sizeof(double), hipMemcpyDeviceToHost));
    if (R_host) {
        std::vector<double> rt(n * n);
        KXG_TRY_HIP(hipMemcpy(rt.data(), k->d_RT, n * n * sizeof(double), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < n; ++i)
            for (size_t j = 0; j < n; ++j) R_host[i * n + j] = rt[j * n + i];
    }
    return KXG_OK;
}

kxg_status kxg_kernel_grid(const kxg_kernel *k, double *dp, double *E, double *K, double *h)
{
    g_err[0] = 0;
    if (!k) { set_error("kxg_kernel_grid: null handle"); return KXG_EINVAL; }
    const size_t b = k->n * sizeof(double);
    if (dp) std::memcpy(dp, k->dp.data(), b);
    if (E) std::memcpy(E, k->E.data(), b);
    if (K) std::memcpy(K, k->K.data(), b);
    if (h) std::memcpy(h, k->h.data(), b);
    return KXG_OK;
}

static kxg_status check_prec(const kxg_kernel *k, int32_t prec)
{
    if (prec < 0 || prec > 4) { set_error("unknown precision %d", prec); return KXG_EINVAL; }
    if (!(k->prec_mask & KXG_PREC_BIT(prec))) {
        set_error("precision %d was not built into this kernel handle", prec);
        return KXG_EUNSUPPORTED;
    }
    return KXG_OK;
}

// Argument checks shared by kxg_eval and kxg_eval_noalloc.
static kxg_status check_eval(const kxg_kernel *k, int32_t prec, const double *f_dev, int32_t B,
                             double *C_dev, uint32_t flags)
{
    if (!k || !f_dev || !C_dev) { set_error("kxg_eval: null handle or buffer"); return KXG_EINVAL; }
    if (B < 1 || B > k->b_cap) { set_error("kxg_eval: B=%d outside [1, b_cap=%d]", B, k->b_cap); return KXG_EINVAL; }
    if (flags & ~(KXG_PROJECT | KXG_INTERP_LOG | KXG_STAT_BOSE | KXG_STAT_FERMI | KXG_SPLIT_F_ONLY | KXG_SPLIT_NONE)) { set_error("kxg_eval: unknown flags 0x%x", flags); return KXG_EINVAL; }
    if ((flags & KXG_SPLIT_F_ONLY) && (flags & KXG_SPLIT_NONE)) { set_error("kxg_eval: two split ablations together"); return KXG_EINVAL; }
    if ((flags & (KXG_SPLIT_F_ONLY | KXG_SPLIT_NONE)) && prec != KXG_BF16X3 && prec != KXG_F16X3) { set_error("kxg_eval: split ablations apply to the three-product 16-bit precisions only"); return KXG_EINVAL; }
    if ((flags & KXG_STAT_BOSE) && (flags & KXG_STAT_FERMI)) { set_error("kxg_eval: Bose and Fermi statistics together"); return KXG_EINVAL; }
    kxg_status st = check_prec(k, prec);
    if (st != KXG_OK) return st;
    if (flags & (KXG_INTERP_LOG | KXG_STAT_BOSE | KXG_STAT_FERMI)) {
        if (!k->d_JX) { set_error("kxg_eval: exact-form evaluation needs a handle built with KXG_WITH_BRACKETS"); return KXG_EUNSUPPORTED; }
        if (prec != KXG_F64 && prec != KXG_F32) { set_error("kxg_eval: exact-form evaluation runs in FP64 or FP32 only"); return KXG_EUNSUPPORTED; }
        if (prec == KXG_F32 && !k->d_AX32) { set_error("kxg_eval: FP32 exact-form operand not built"); return KXG_EUNSUPPORTED; }
        if (prec == KXG_F64 && !k->d_AX64) { set_error("kxg_eval: FP64 exact-form operand not built"); return KXG_EUNSUPPORTED; }
    }
    return KXG_OK;
}

kxg_status kxg_eval(const kxg_kernel *k, int32_t prec, const double *f_dev, int32_t B,
                    double *C_dev, uint32_t flags, double *diag_dev, void *stream)
{
    g_err[0] = 0;
    const kxg_status st = check_eval(k, prec, f_dev, B, C_dev, flags);
    if (st != KXG_OK) return st;
    return eval_impl(*k, k->ws, prec, f_dev, B, C_dev, flags, diag_dev,
                     static_cast<hipStream_t>(stream));
}

kxg_status kxg_eval_noalloc(const kxg_kernel *k, int32_t prec, const double *f_dev, int32_t B,
                            double *C_dev, uint32_t flags, double *diag_dev, void *stream)
{
    g_err[0] = 0;
    const kxg_status st = check_eval(k, prec, f_dev, B, C_dev, flags);
    if (st != KXG_OK) return st;
    return eval_noalloc_impl(*k, prec, f_dev, B, C_dev, flags, diag_dev,
                             static_cast<hipStream_t>(stream));
}

kxg_status kxg_moments(const kxg_kernel *k, const double *f_dev, int32_t B, double *out_dev,
                       void *stream)
{
    g_err[0] = 0;
    if (!k || !f_dev || !out_dev || B < 1) { set_error("kxg_moments: bad arguments"); return KXG_EINVAL; }
    KXG_TRY_HIP(launch_moments(*k, f_dev, B, out_dev, static_cast<hipStream_t>(stream)));
    return KXG_OK;
}

// ------------------------------------------------------------------ steppers

kxg_status kxg_stepper_create(const kxg_kernel *k, const kxg_stepper_params *prm,
                              kxg_stepper **out)
{
    g_err[0] = 0;
    if (!k || !prm || !out) { set_error("kxg_stepper_create: null argument"); return KXG_EINVAL; }
    *out = nullptr;
    if (prm->kind != KXG_RK4 && prm->kind != KXG_HEUN) { set_error("kxg_stepper_create: bad kind"); return KXG_EINVAL; }
    if (prm->expansion != KXG_EXP_NONE && prm->expansion != KXG_EXP_RADIATION) { set_error("kxg_stepper_create: bad expansion"); return KXG_EINVAL; }
    if (prm->expansion == KXG_EXP_RADIATION && prm->kind != KXG_HEUN) { set_error("kxg_stepper_create: expansion needs the Heun stepper"); return KXG_EINVAL; }
    if (prm->b_cap < 1 || prm->b_cap > (1 << 20)) { set_error("kxg_stepper_create: bad b_cap"); return KXG_EINVAL; }
    if (prm->freeze_in != 0 && (prm->kind != KXG_HEUN || prm->expansion != KXG_EXP_RADIATION)) {
        set_error("kxg_stepper_create: freeze-in sources need the Heun stepper with expansion");
        return KXG_EINVAL;
    }
    if (prm->kind == KXG_HEUN && prm->adapt &&
        !(prm->rtol > 0 && prm->safety > 0 && prm->fac_min > 0 && prm->fac_max >= prm->fac_min)) {
        set_error("kxg_stepper_create: bad Heun controller parameters");
        return KXG_EINVAL;
    }
    kxg_status st = check_prec(k, prm->prec);
    if (st != KXG_OK) return st;
    kxg_stepper *s = new (std::nothrow) kxg_stepper;
    if (!s) { set_error("host allocation failed"); return KXG_ENOMEM; }
    s->k = k;
    s->prm = *prm;
    const size_t rows = (size_t)prm->b_cap * k->n;
    if (st == KXG_OK) st = dalloc(&s->d_slots, (size_t)prm->b_cap);
    if (st == KXG_OK) st = dalloc(&s->d_x, rows);
    if (st == KXG_OK) st = dalloc(&s->d_fb, rows);
    if (st == KXG_OK) st = dalloc(&s->d_acc, rows);
    if (st == KXG_OK) st = dalloc(&s->d_xs, rows);
    if (st == KXG_OK) st = dalloc(&s->d_dt, (size_t)prm->b_cap);
    if (st == KXG_OK) st = dalloc(&s->d_init, (size_t)prm->b_cap);
    if (st == KXG_OK && hipHostMalloc((void **)&s->h_init, (size_t)prm->b_cap * sizeof(SlotDev)) != hipSuccess) {
        s->h_init = nullptr;
        set_error("kxg_stepper_create: pinned host allocation failed");
        st = KXG_ENOMEM;
    }
    if (st == KXG_OK && hipEventCreateWithFlags(&s->init_evt, hipEventDisableTiming) != hipSuccess) {
        s->init_evt = nullptr;
        set_error("kxg_stepper_create: hipEventCreate failed");
        st = KXG_EHIP;
    }
    if (st == KXG_OK) st = alloc_workspace(*k, prm->b_cap, s->ws);
    if (st == KXG_OK) {
        std::vector<SlotDev> init(prm->b_cap);
        for (auto &q : init) {
            std::memset(&q, 0, sizeof q);
            q.status = -3;
        }
        if (hipMemcpy(s->d_slots, init.data(), init.size() * sizeof(SlotDev), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(s->d_x, 0, rows * sizeof(double)) != hipSuccess ||
            hipMemset(s->d_fb, 0, rows * sizeof(double)) != hipSuccess) {
            set_error("kxg_stepper_create: initialisation failed");
            st = KXG_EHIP;
        }
    }
    if (st != KXG_OK) {
        kxg_stepper_free(s);
        return st;
    }
    s->used.assign(prm->b_cap, 0);
    *out = s;
    return KXG_OK;
}

void kxg_stepper_free(kxg_stepper *s)
{
    if (!s) return;
    for (kxg_stepper::Graphs &g : s->graphs) {
        if (g.one) (void)hipGraphExecDestroy(g.one);
        if (g.many) (void)hipGraphExecDestroy(g.many);
    }
    if (s->init_evt) {
        (void)hipEventSynchronize(s->init_evt);
        (void)hipEventDestroy(s->init_evt);
    }
    if (s->h_init) (void)hipHostFree(s->h_init);
    void *ptrs[] = {s->d_slots, s->d_x, s->d_fb, s->d_acc, s->d_xs, s->d_dt, s->d_init};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    free_workspace(s->ws);
    delete s;
}

static void update_hi(kxg_stepper *s)
{
    int hi = 0;
    for (int b = 0; b < (int)s->used.size(); ++b)
        if (s->used[b]) hi = b + 1;
    s->b_hi = hi;
}

static bool solve_params_ok(const kxg_solve_params *sp)
{
    return std::isfinite(sp->lambda) && sp->lambda >= 0.0 && std::isfinite(sp->t_end) &&
           sp->t_end > 0.0 && std::isfinite(sp->dt) && std::isfinite(sp->h_i);
}

static bool has_freeze_in(const kxg_solve_params *sp)
{
    return sp->src_n0 != 0.0 || sp->src_kappa != 0.0 || sp->du_src > 0.0;
}

// Freeze-in fields of a solve (Sec. 3, Sec. 4.2); "" if they are valid for
// this stepper, else what is wrong.
static const char *freeze_in_error(const kxg_stepper *s, const kxg_solve_params *sp)
{
    if (!has_freeze_in(sp)) return "";
    if (!s->prm.freeze_in) return "freeze-in fields on a stepper created without freeze_in";
    const double fin[] = {sp->src_n0, sp->src_gamma, sp->src_p0, sp->src_kappa, sp->src_mh,
                          sp->src_ti, sp->du_src, sp->eps_switch};
    for (double v : fin)
        if (!std::isfinite(v)) return "non-finite freeze-in field";
    if (!(sp->h_i > 0.0)) return "a freeze-in solve needs h_i > 0 (H at u = 0)";
    if (sp->src_n0 < 0.0 || sp->src_gamma < 0.0 || sp->src_kappa < 0.0) return "negative source";
    if (sp->src_n0 > 0.0) {
        const kxg_kernel &k = *s->k;
        const double m = k.mass, K0 = sp->src_p0 * sp->src_p0 / (std::sqrt(sp->src_p0 * sp->src_p0 + m * m) + m);
        if (!(sp->src_p0 > 0.0) || !(K0 >= k.K[0] && K0 <= k.K[k.n - 1]))
            return "condensate momentum src_p0 outside the grid";
    }
    if (sp->src_kappa > 0.0 && !(sp->src_mh > 2.0 * s->k->mass && sp->src_ti > 0.0))
        return "Higgs source needs src_mh > 2 m and src_ti > 0";
    return "";
}

static SlotDev slot_record(const kxg_stepper *s, const kxg_solve_params *sp)
{
    SlotDev init;
    std::memset(&init, 0, sizeof init);
    init.lam = sp->lambda;
    init.hi_scale = sp->h_i;
    init.dt = sp->dt;
    init.t = 0.0;
    init.tend = sp->t_end;
    init.maxsteps = sp->max_steps;
    init.status = 0;
    init.phase = 1;
    init.jdep = -1;
    if (s->prm.freeze_in && has_freeze_in(sp)) {
        const kxg_kernel &k = *s->k;
        const double m = k.mass;
        init.src_n0 = sp->src_n0;
        init.src_gamma = sp->src_gamma;
        init.src_kappa = sp->src_kappa;
        init.src_mh = sp->src_mh;
        init.src_kh = sp->src_kappa > 0.0 ? std::sqrt(sp->src_mh * sp->src_mh - 4.0 * m * m) : 0.0;
        init.src_ti = sp->src_ti;
        init.du_src = sp->du_src;
        init.eps_switch = sp->eps_switch;
        init.phase = sp->du_src > 0.0 ? 0 : 1;
        if (sp->src_n0 > 0.0) {
            // the two grid points that bracket p0 in kinetic energy, with the
            // energy-linear weights (App. B eq. app_interp_weights), over h
            const double p0 = sp->src_p0;
            const double K0 = p0 * p0 / (std::sqrt(p0 * p0 + m * m) + m);
            int j = 0;
            for (int q = 0; q < k.n - 1; ++q)
                if (k.K[q] <= K0) j = q;
            const double wr = (K0 - k.K[j]) / (k.K[j + 1] - k.K[j]);
            init.jdep = j;
            init.wl_h = (1.0 - wr) / k.h[j];
            init.wr_h = wr / k.h[j + 1];
        }
    }
    return init;
}

kxg_status kxg_stepper_set(kxg_stepper *s, int32_t slot, const double *f0_dev,
                           const kxg_solve_params *sp, void *stream)
{
    g_err[0] = 0;
    if (!s || !f0_dev || !sp) { set_error("kxg_stepper_set: null argument"); return KXG_EINVAL; }
    if (slot < 0 || slot >= s->prm.b_cap) { set_error("kxg_stepper_set: slot %d out of range", slot); return KXG_EINVAL; }
    if (!solve_params_ok(sp)) {
        set_error("kxg_stepper_set: lambda >= 0, finite dt/h_i and t_end > 0 required");
        return KXG_EINVAL;
    }
    const char *fe = freeze_in_error(s, sp);
    if (*fe) { set_error("kxg_stepper_set: %s", fe); return KXG_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const SlotDev init = slot_record(s, sp);
    KXG_TRY_HIP(launch_slot_init(slot, init, s->d_slots, st));
    KXG_TRY_HIP(launch_slot_set(s->k->n, s->prm.kind, s->prm.expansion, s->prm.atol_rel, slot,
                                s->d_slots, f0_dev, s->k->d_p, s->k->d_RT, s->d_x, s->d_fb, st));
    s->used[slot] = 1;
    update_hi(s);
    return KXG_OK;
}

kxg_status kxg_stepper_set_many(kxg_stepper *s, int32_t slot0, int32_t count,
                                const double *f0_dev, const kxg_solve_params *sp_host,
                                void *stream)
{
    g_err[0] = 0;
    if (!s || !f0_dev || !sp_host) { set_error("kxg_stepper_set_many: null argument"); return KXG_EINVAL; }
    if (count < 1 || slot0 < 0 || slot0 > s->prm.b_cap - count) {
        set_error("kxg_stepper_set_many: slots [%d, %d) outside [0, %d)", slot0, slot0 + count, s->prm.b_cap);
        return KXG_EINVAL;
    }
    for (int j = 0; j < count; ++j) {
        if (!solve_params_ok(&sp_host[j])) {
            set_error("kxg_stepper_set_many: solve %d: lambda >= 0, finite dt/h_i and t_end > 0 required", j);
            return KXG_EINVAL;
        }
        const char *fe = freeze_in_error(s, &sp_host[j]);
        if (*fe) { set_error("kxg_stepper_set_many: solve %d: %s", j, fe); return KXG_EINVAL; }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the staging buffer is reused: wait until the previous copy out of it is done
    KXG_TRY_HIP(hipEventSynchronize(s->init_evt));
    for (int j = 0; j < count; ++j) s->h_init[j] = slot_record(s, &sp_host[j]);
    KXG_TRY_HIP(hipMemcpyAsync(s->d_init, s->h_init, (size_t)count * sizeof(SlotDev), hipMemcpyHostToDevice, st));
    KXG_TRY_HIP(hipEventRecord(s->init_evt, st));
    KXG_TRY_HIP(launch_slot_set_many(s->k->n, s->prm.kind, s->prm.expansion, s->prm.atol_rel, slot0, count,
                                     s->d_init, s->d_slots, f0_dev, s->k->d_p, s->k->d_RT, s->d_x, s->d_fb, st));
    for (int j = 0; j < count; ++j) s->used[slot0 + j] = 1;
    update_hi(s);
    return KXG_OK;
}

size_t kxg_stepper_bytes(const kxg_stepper *s)
{
    if (!s) return 0;
    const size_t b = (size_t)s->prm.b_cap, n = (size_t)s->k->n;
    const size_t fbytes = (size_t)s->k->geo.nb * s->ws.bpad_cap * kBlk * sizeof(float);
    return b * (2 * sizeof(SlotDev) + sizeof(double)) + 4 * b * n * sizeof(double) + s->ws.part_bytes +
           2 * fbytes + (size_t)s->ws.bpad_cap * sizeof(float);
}

kxg_status kxg_stepper_release(kxg_stepper *s, int32_t slot, void *stream)
{
    g_err[0] = 0;
    if (!s || slot < 0 || slot >= s->prm.b_cap) { set_error("kxg_stepper_release: bad slot"); return KXG_EINVAL; }
    KXG_TRY_HIP(launch_slot_clear(s->k->n, slot, s->d_slots, s->d_x, s->d_fb,
                                  static_cast<hipStream_t>(stream)));
    s->used[slot] = 0;
    update_hi(s);
    return KXG_OK;
}

// One iteration of the stepper over the first B slots: RK4 = 4 x (operator
// call + stage update); Heun = operator call, predictor, operator call,
// corrector with control.
static kxg_status enqueue_iteration(kxg_stepper *s, int B, hipStream_t st)
{
    const kxg_kernel &k = *s->k;
    const kxg_stepper_params &P = s->prm;
    const uint32_t flags = P.project ? KXG_PROJECT : 0u;
    StepArgs a{};
    a.sl = s->d_slots;
    a.x = s->d_x;
    a.acc = s->d_acc;
    a.xs = s->d_xs;
    a.fb = s->d_fb;
    a.p = k.d_p;
    a.dp = k.d_dp;
    a.expansion = P.expansion;
    a.adapt = P.adapt;
    a.rtol = P.rtol;
    a.safety = P.safety;
    a.fac_lo = P.fac_min;
    a.fac_hi = P.fac_max;
    a.dt_min = P.dt_min;
    a.freeze_in = P.freeze_in;
    a.atol_rel = P.atol_rel;
    a.mass = k.mass;
    // every operator call of the iteration takes its GEMM operand from the
    // epilogue of the call before (the first from kxg_stepper_advance)
    a.write_op = 1;
    a.op_ready = 1;
    if (P.kind == KXG_RK4) {
        a.mode = kStepRK4;
        for (int stage = 1; stage <= 4; ++stage) {
            a.stage = stage;
            kxg_status r = eval_impl(k, s->ws, P.prec, s->d_fb, B, nullptr, flags, nullptr, st, &a);
            if (r != KXG_OK) return r;
        }
        return KXG_OK;
    }
    a.mode = kStepHeunPred;
    kxg_status r = eval_impl(k, s->ws, P.prec, s->d_fb, B, nullptr, flags, nullptr, st, &a);
    if (r != KXG_OK) return r;
    a.mode = kStepHeunCorr;
    return eval_impl(k, s->ws, P.prec, s->d_fb, B, nullptr, flags, nullptr, st, &a);
}

// Iterations per replay of the long graph; the remainder of an advance call
// replays the one-iteration graph.  Both are captured per batch bucket, on
// the bucket's first use, and again only when it is replayed on another
// stream.
constexpr int kGraphIters = 8;

// Capture `iters` iterations of the stepper on `st` into an executable graph
// (null if capture or instantiation fails).
static hipGraphExec_t capture_iterations(kxg_stepper *s, int batch, int iters, hipStream_t st)
{
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    kxg_status r = KXG_OK;
    for (int it = 0; it < iters && r == KXG_OK; ++it) r = enqueue_iteration(s, batch, st);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (r != KXG_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess || !exec) {
        (void)hipGetLastError();
        return nullptr;
    }
    return exec;
}

// The graphs of a batch bucket (batch = a multiple of 16 up to b_cap, or
// b_cap), captured on `st` if they are not held for it yet; null if the
// capture fails.
static const kxg_stepper::Graphs *ensure_graph(kxg_stepper *s, int batch, hipStream_t st)
{
    const size_t slot = (size_t)((batch + 15) / 16 - 1);
    if (s->graphs.size() <= slot) s->graphs.resize(slot + 1);
    kxg_stepper::Graphs &g = s->graphs[slot];
    if (g.one && g.stream == st) return &g;
    if (g.one) (void)hipGraphExecDestroy(g.one);
    if (g.many) (void)hipGraphExecDestroy(g.many);
    g = kxg_stepper::Graphs{};
    g.one = capture_iterations(s, batch, 1, st);
    if (!g.one) return nullptr;
    g.many = capture_iterations(s, batch, kGraphIters, st);   // optional
    g.stream = st;
    return &g;
}

kxg_status kxg_stepper_advance(kxg_stepper *s, int32_t n_iter, void *stream)
{
    g_err[0] = 0;
    if (!s || n_iter < 0) { set_error("kxg_stepper_advance: bad arguments"); return KXG_EINVAL; }
    const int B = s->b_hi;
    if (B == 0 || n_iter == 0) return KXG_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // Launch-bound iterations replay a captured graph on a non-default stream
    // (batch rounded up to a multiple of 16 slots; free slots are skipped by
    // the kernels).  Direct launches while a profile is open or on the
    // default stream.
    const int bucket = std::min(s->prm.b_cap, (B + 15) / 16 * 16);
    const kxg_stepper::Graphs *g = (st != nullptr && !g_prof.on) ? ensure_graph(s, bucket, st) : nullptr;
    if (g) {
        kxg_status r = prep_operands(*s->k, s->ws, s->prm.prec, s->d_fb, bucket, st);
        if (r != KXG_OK) return r;
        int it = 0;
        if (g->many)
            for (; it + kGraphIters <= n_iter; it += kGraphIters) KXG_TRY_HIP(hipGraphLaunch(g->many, st));
        for (; it < n_iter; ++it) KXG_TRY_HIP(hipGraphLaunch(g->one, st));
        return KXG_OK;
    }
    kxg_status r0 = prep_operands(*s->k, s->ws, s->prm.prec, s->d_fb, B, st);
    if (r0 != KXG_OK) return r0;
    for (int it = 0; it < n_iter; ++it) {
        kxg_status r = enqueue_iteration(s, B, st);
        if (r != KXG_OK) return r;
    }
    return KXG_OK;
}

kxg_status kxg_stepper_set_dt(kxg_stepper *s, const double *dt_host, void *stream)
{
    g_err[0] = 0;
    if (!s || !dt_host) { set_error("kxg_stepper_set_dt: null argument"); return KXG_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    KXG_TRY_HIP(hipMemcpyAsync(s->d_dt, dt_host, s->prm.b_cap * sizeof(double), hipMemcpyHostToDevice, st));
    KXG_TRY_HIP(launch_set_dt(s->prm.b_cap, s->d_dt, s->d_slots, st));
    KXG_TRY_HIP(hipStreamSynchronize(st));
    return KXG_OK;
}

kxg_status kxg_stepper_query(kxg_stepper *s, kxg_slot_state *out, void *stream)
{
    g_err[0] = 0;
    if (!s || !out) { set_error("kxg_stepper_query: null argument"); return KXG_EINVAL; }
    std::vector<SlotDev> h(s->prm.b_cap);
    hipStream_t st = static_cast<hipStream_t>(stream);
    KXG_TRY_HIP(hipMemcpyAsync(h.data(), s->d_slots, h.size() * sizeof(SlotDev), hipMemcpyDeviceToHost, st));
    KXG_TRY_HIP(hipStreamSynchronize(st));
    for (size_t b = 0; b < h.size(); ++b) {
        out[b].t = h[b].t;
        out[b].dt = h[b].dt;
        out[b].outflow = h[b].outflow;
        out[b].h_i = h[b].hi_scale;
        out[b].steps = h[b].steps;
        out[b].rejected = h[b].rejected;
        out[b].status = s->used[b] ? h[b].status : -3;
        out[b].phase = h[b].phase;
        out[b].u_switch = h[b].u_switch;
        out[b].n_src = h[b].nsrc;
        out[b].pad = 0;
    }
    return KXG_OK;
}

kxg_status kxg_stepper_get(kxg_stepper *s, int32_t slot, double *f_dev, void *stream)
{
    g_err[0] = 0;
    if (!s || !f_dev || slot < 0 || slot >= s->prm.b_cap) { set_error("kxg_stepper_get: bad arguments"); return KXG_EINVAL; }
    KXG_TRY_HIP(launch_slot_get(s->k->n, s->prm.expansion, slot, s->d_slots, s->k->d_p, s->d_x,
                                f_dev, static_cast<hipStream_t>(stream)));
    return KXG_OK;
}

static const uint32_t kMagic = 0x4b584731u;   // "KXG1"

kxg_status kxg_stepper_save(kxg_stepper *s, int32_t slot, void *buf, size_t *len, void *stream)
{
    g_err[0] = 0;
    if (!s || !len || slot < 0 || slot >= s->prm.b_cap) { set_error("kxg_stepper_save: bad arguments"); return KXG_EINVAL; }
    const int n = s->k->n;
    const size_t need = 4 * sizeof(uint32_t) + sizeof(SlotDev) + n * sizeof(double);
    if (!buf) { *len = need; return KXG_OK; }
    if (*len < need) { set_error("kxg_stepper_save: buffer of %zu bytes, need %zu", *len, need); return KXG_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *c = static_cast<char *>(buf);
    const uint32_t hdr[4] = {kMagic, (uint32_t)n, (uint32_t)s->prm.kind, (uint32_t)s->prm.expansion};
    std::memcpy(c, hdr, sizeof hdr);
    KXG_TRY_HIP(hipMemcpyAsync(c + sizeof hdr, s->d_slots + slot, sizeof(SlotDev), hipMemcpyDeviceToHost, st));
    KXG_TRY_HIP(hipMemcpyAsync(c + sizeof hdr + sizeof(SlotDev), s->d_x + (size_t)slot * n,
                               n * sizeof(double), hipMemcpyDeviceToHost, st));
    KXG_TRY_HIP(hipStreamSynchronize(st));
    *len = need;
    return KXG_OK;
}

kxg_status kxg_stepper_load(kxg_stepper *s, int32_t slot, const void *buf, size_t len, void *stream)
{
    g_err[0] = 0;
    if (!s || !buf || slot < 0 || slot >= s->prm.b_cap) { set_error("kxg_stepper_load: bad arguments"); return KXG_EINVAL; }
    const int n = s->k->n;
    const size_t need = 4 * sizeof(uint32_t) + sizeof(SlotDev) + n * sizeof(double);
    uint32_t hdr[4];
    if (len < need) { set_error("kxg_stepper_load: %zu bytes, need %zu", len, need); return KXG_EINVAL; }
    std::memcpy(hdr, buf, sizeof hdr);
    if (hdr[0] != kMagic || hdr[1] != (uint32_t)n || hdr[2] != (uint32_t)s->prm.kind ||
        hdr[3] != (uint32_t)s->prm.expansion) {
        set_error("kxg_stepper_load: checkpoint does not match this stepper");
        return KXG_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *c = static_cast<const char *>(buf);
    SlotDev sd;
    std::memcpy(&sd, c + sizeof hdr, sizeof sd);
    KXG_TRY_HIP(launch_slot_init(slot, sd, s->d_slots, st));
    KXG_TRY_HIP(hipMemcpyAsync(s->d_x + (size_t)slot * n, c + sizeof hdr + sizeof(SlotDev),
                               n * sizeof(double), hipMemcpyHostToDevice, st));
    KXG_TRY_HIP(launch_slot_refresh(n, s->prm.expansion, slot, s->d_slots, s->k->d_p, s->d_x, s->d_fb, st));
    KXG_TRY_HIP(hipStreamSynchronize(st));
    s->used[slot] = 1;
    update_hi(s);
    return KXG_OK;
}

}  // extern "C"
