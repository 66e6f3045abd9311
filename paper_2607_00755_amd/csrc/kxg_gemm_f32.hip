// Batched gain on the FP32 matrix cores (Sec. 4.1, eq.
// discrete_collision_operator as a GEMM over K = (k, m) with the loss term
// folded into the packed operand): gain - loss for a tile of distributions
// and one i-block, K split into work units; the partials are reduced by the
// FP64 epilogue.
#include "kxg_device.h"

#ifndef KXG_F32_NST
#define KXG_F32_NST 2        // register stages of the FP32 GEMM
#endif

namespace kxg {
namespace {

// FP32 GEMM on v_mfma_f32_32x32x2f32 over the non-zero blocks of the packed
// operand.  Workgroup = (batch tile of BBW*32 distributions, work unit =
// i-block of 32 rows and a range of its blocks); its 4 waves take 4
// consecutive sub-ranges of the unit's dk steps.  Per dk step (one row k of a
// (kb, mb) block, 16 K values) a wave issues 8*BBW MFMAs; the A operand
// (F2 = f_k f_m) is one multiply per MFMA, the B operand (packed tensor)
// comes straight from memory in MFMA order.
//
// The loop runs over super-steps of SS dk steps with NST register stages
// (packed tensor, f_k and f_m of one super-step) used in rotation, so that
// the loads of the next NST-1 super-steps are in flight during the MFMAs of
// the current one without any register copy or branch around them (either
// would make the compiler wait for them early); a prefetch past the end of
// the range re-reads the last super-step.  The wave index is made uniform so
// that the pair table is read through scalar loads.
template <int BBW, int SS>
struct F32Stage {
    float4 g[2 * SS];          // packed tensor, two 16-byte vectors per dk step
    float fk[BBW][SS];         // f_k of each batch sub-tile, per dk step
    float4 fm[BBW][2];         // f_m of the (kb, mb) block in parity order
};

template <int BBW, int SS = kF32SS, int NST = 2>
__global__ __launch_bounds__(256, 2) void k_gemm_f32(
    const float *__restrict__ G, const float *__restrict__ fop, const float *__restrict__ fpar,
    const int *__restrict__ pairs, const int *__restrict__ units, int bpad, int ipad, int nbt,
    float *__restrict__ part)
{
    static_assert(SS == 2 || SS == 4, "super-step of 2 or 4 dk steps");
    static_assert(NST == 2 || NST == 3, "2 or 3 register stages");
    typedef float fkvec __attribute__((ext_vector_type(SS)));
    constexpr int PPS = kBlk / SS;                 // super-steps per (kb, mb) pair
    __shared__ __align__(16) float lds[4 * BBW * 16 * 64];
    static_assert(SS == kF32SS, "work units are counted in super-steps of kF32SS dk steps");
    const int L = xcd_logical(blockIdx.x, gridDim.x);
    const int bt = L % nbt, u = L / nbt;
    // work unit: i-block, K slot and range of (compacted) super-steps
    const int ib = units[4 * u], sp = units[4 * u + 1];
    const long ub = units[4 * u + 2], ue = units[4 * u + 3];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int r = lane & 31, hb = lane >> 5;
    const long s0 = ub + (ue - ub) * wave / kWaves, s1 = ub + (ue - ub) * (wave + 1) / kWaves;
    const int brow0 = bt * BBW * 32;
    const float *Gi = G;
    const float *fkb = fop + (long)(brow0 + r) * kBlk;
    const float *fmb = fpar + ((long)(brow0 + r) * 2 + hb) * 8;
    const long bstride = (long)bpad * kBlk;        // one 16-block of the grid, all rows

    floatx16 acc[BBW];
#pragma unroll
    for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[bb][e] = 0.0f;

    F32Stage<BBW, SS> st[NST];

    // (kb, mb) of the next stage to load, read one stage ahead so that the
    // scalar load is not waited for right before the vector loads it feeds
    const int2 *pairs2 = reinterpret_cast<const int2 *>(pairs);
    auto pair_of = [&](long s) { return pairs2[(s < s1 ? s : s1 - 1) / PPS]; };
    int2 pnext = pair_of(s0);
    auto load_stage = [&](long s, F32Stage<BBW, SS> &x) {
        s = s < s1 ? s : s1 - 1;
        const int kb = pnext.x, mb = pnext.y;
        pnext = pair_of(s + 1);
        const float4 *gp = reinterpret_cast<const float4 *>(Gi + s * (SS * 512));
#pragma unroll
        for (int d = 0; d < SS; ++d) {
            x.g[2 * d] = gp[d * 128 + lane];
            x.g[2 * d + 1] = gp[d * 128 + 64 + lane];
        }
        const int dk = (int)(s % PPS) * SS;
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb) {
            const fkvec v = *reinterpret_cast<const fkvec *>(fkb + kb * bstride + bb * 32 * kBlk + dk);
#pragma unroll
            for (int d = 0; d < SS; ++d) x.fk[bb][d] = v[d];
            const float4 *src = reinterpret_cast<const float4 *>(fmb + mb * bstride + bb * 32 * kBlk);
            x.fm[bb][0] = src[0];
            x.fm[bb][1] = src[1];
        }
    };
    // F2 operand of step q = 8 d + t of a stage: f_k (dk step d) times f_m
    // (t-th value of this lane's half of the block)
    auto f2 = [&](const F32Stage<BBW, SS> &x, int q, int bb) {
        const int d = q >> 3, t = q & 7;
        return x.fk[bb][d] * x.fm[bb][t >> 2][t & 3];
    };
    // The products of step q + 1 are formed before the MFMAs of step q (the
    // scheduler may not move them across), so a product never takes the
    // register that an MFMA in flight is reading.
    auto compute = [&](const F32Stage<BBW, SS> &x) {
        float pv[2][BBW];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb) pv[0][bb] = f2(x, 0, bb);
#pragma unroll
        for (int q = 0; q < SS * 8; ++q) {
            const int d = q >> 3, t = q & 7;
            const float4 gv = x.g[2 * d + (t >> 2)];
            const float bv = (t & 3) == 0 ? gv.x : (t & 3) == 1 ? gv.y : (t & 3) == 2 ? gv.z : gv.w;
            if (q + 1 < SS * 8) {
#pragma unroll
                for (int bb = 0; bb < BBW; ++bb) pv[(q + 1) & 1][bb] = f2(x, q + 1, bb);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int bb = 0; bb < BBW; ++bb)
                acc[bb] = __builtin_amdgcn_mfma_f32_32x32x2f32(pv[q & 1][bb], bv, acc[bb], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    // Rounds of NST super-steps with no exit between them (a conditional exit
    // would let the compiler sink the prefetch below it); at the start of a
    // round st[j] holds super-step s + j for j < NST - 1, and the last
    // s1 - s < NST super-steps are done after the loop from those stages.
    if (s0 < s1) {
#pragma unroll
        for (int j = 0; j < NST - 1; ++j) load_stage(s0 + j, st[j]);
    }
    long s = s0;
    for (; s + NST <= s1; s += NST) {
#pragma unroll
        for (int j = 0; j < NST; ++j) {
            load_stage(s + j + NST - 1, st[(j + NST - 1) % NST]);
            __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
            compute(st[j]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int j = 0; j < NST - 1; ++j)
        if (s + j < s1) compute(st[j]);
    store_tile<BBW>(acc, lds, part, sp, bpad, ipad, brow0, ib * kIBlk);
}

}  // namespace

hipError_t launch_gemm_f32(int bbw, int nwg, const float *G, const float *fop, const float *fpar,
                           const int *pairs, const int *units, int bpad, int ipad, int nbt, float *part,
                           hipStream_t s)
{
#define KXG_GEMM_F32(W)                                                                              \
    hipLaunchKernelGGL((k_gemm_f32<W, kF32SS, KXG_F32_NST>), dim3(nwg), dim3(256), 0, s, G, fop, fpar, \
                       pairs, units, bpad, ipad, nbt, part)
    if (bbw == 1) KXG_GEMM_F32(1);
    else if (bbw == 2) KXG_GEMM_F32(2);
    else KXG_GEMM_F32(4);
#undef KXG_GEMM_F32
    return hipGetLastError();
}

}  // namespace kxg
