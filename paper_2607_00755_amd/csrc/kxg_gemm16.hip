// Batched gain minus loss on the 16-bit matrix cores (Sec. 4.1, eq.
// discrete_collision_operator as a GEMM over K = (k, m) with the loss term
// folded into the packed operand): BF16 or FP16 32x32x16 MFMAs with a hi+lo
// split of the operand and of F2 = f_k f_m (three products, or two: A hi
// only), for a tile of distributions and a group of i-blocks, K split into
// work units; the partials are reduced by the FP64 epilogue.
#include "kxg_device.h"
#include "kxg_internal.h"

#include <type_traits>

namespace kxg {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x8 __attribute__((ext_vector_type(8)));

// 16-bit split GEMM, the packed tensor shared through LDS.
// A workgroup's 4 waves work on the same K split and the same IBW i-blocks;
// wave w takes the BBW b-blocks [w*BBW, (w+1)*BBW) of the workgroup's
// 4*BBW*32-row batch tile.  The K range runs in super-steps of SS dk steps:
// the workgroup stages the hi/lo fragments of its i-blocks for one
// super-step (IBW*SS*2 KB) into one of two LDS slots, each thread carrying
// IBW*SS/2 16-byte vectors through registers.  Two register stages (the
// vectors in transit and f_k of the super-step) alternate without copies:
// the global loads of super-step s+1 are in flight while the MFMAs of
// super-step s run, and are written to the other LDS slot after them; one
// barrier per super-step.  f_m is the same for the kBlk/SS super-steps of a
// (kb, mb) pair: it is loaded once per pair, a pair ahead, and kept in one
// of two wave-private LDS sets chosen by the pair's parity (registers can't
// be chosen at run time without copies).  Every wave forms and splits its F2
// operand once per (b-block, dk) and feeds it to SPLIT*IBA MFMAs.  The kept
// pairs of a unit all have their non-zero blocks in the group's first IBA
// i-blocks (IBA of its first pair, the pairs of a group being ordered by
// that count): only those are staged and multiplied, the others' partials
// are written as zeros.  Partials: one per K split.
template <int BBW, int SS, int NQ>
struct X3Stage {
    u32x4 gv[NQ];              // packed-tensor vectors in transit to LDS
    float fk[BBW][SS];         // f_k per b-block and dk step
};

template <int IBW, int SS, int SPLIT>
struct X3Shape {
    static constexpr int VPS = SS * 128;           // 16-byte vectors per i-block and super-step
    static constexpr int NV = IBW * VPS;           // per super-step
    // SPLIT < 3 never reads the lo halves of the tensor: only the hi vectors
    // (64 of each step's 128) are loaded and staged.
    static constexpr int HALF = SPLIT == 3 ? 1 : 2;
    static constexpr int NQ = NV / HALF / 256;     // loaded vectors per thread
    static constexpr int PPS = kBlk / SS;          // super-steps per (kb, mb) pair
};

template <int BBW, int IBW, int SS, bool F16, int SPLIT, int IBA>
__device__ __forceinline__ void x3_run(
    const uint16_t *G, const float *__restrict__ fop, const int *__restrict__ pairs, int it, int sp,
    long s0, long s1, int bt, int nib, int bpad, int ipad, float *__restrict__ part,
    u32x4 (&sA)[2][X3Shape<IBW, SS, SPLIT>::NV], floatx4 (&sF)[2][4][BBW][2][64])
{
    typedef typename std::conditional<F16, halfx8, bf16x8>::type opx8;
    typedef float fkvec __attribute__((ext_vector_type(SS)));
    typedef X3Shape<IBW, SS, SPLIT> Sh;
    constexpr int VPS = Sh::VPS, NV = Sh::NV, HALF = Sh::HALF, NQ = Sh::NQ, PPS = Sh::PPS;
    static_assert(NV % (256 * HALF) == 0, "a super-step must split evenly over 256 threads");
    static_assert(PPS >= 2, "f_m is prefetched on the second super-step of a pair");
    static_assert(IBA >= 1 && IBA <= IBW, "active i-blocks");
    typedef X3Stage<BBW, SS, NQ> Stage;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int r = lane & 31, hb = lane >> 5;
    const int brow0 = bt * (4 * BBW * 32) + wave * (BBW * 32);
    const int ib0 = it * IBW;
    const long bstride = (long)bpad * kBlk;
    const float *fkb = fop + (long)(brow0 + r) * kBlk;
    const float *fmb = fop + (long)(brow0 + r) * kBlk + 8 * hb;
    // loader role: vector q = threadIdx.x + 256 c of a super-step belongs to
    // i-block q / VPS of the group (q / (VPS / 2) when only hi vectors are
    // loaded: step (q / 64) of the i-block's super-step, lane q % 64); block
    // c of the compacted operand holds IBW * 16 * 128 vectors.  A wave's 64
    // vectors are consecutive, so everything but the lane is uniform: qoff
    // and qlds are the wave's offsets into the stage's tensor block and into
    // an LDS slot, qact whether they belong to one of the IBA multiplied
    // i-blocks.
    static_assert((VPS / HALF) % 64 == 0, "a wave's vectors lie in one i-block");
    const int wv = wave & 3;
    int qoff[NQ], qlds[NQ];
    bool qact[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
        const int qw = wv * 64 + 256 * c;
        const int w = HALF == 1 ? qw % VPS : (qw % (VPS / 2)) / 64 * 128;
        const int ib = qw / (VPS / HALF);
        qoff[c] = ib * kBlk * 128 + w;
        qlds[c] = ib * VPS + w;
        qact[c] = ib < IBA;
    }

    floatx16 acc[BBW][IBW];
#pragma unroll
    for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
        for (int ib = 0; ib < IBW; ++ib)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[bb][ib][e] = 0.0f;

    Stage sa, sb;
    // f_m of pair pr (this lane's K half of each b-block's m values)
    auto load_fm = [&](int pr, floatx4 (&dst)[BBW][2]) {
        const int mb = pairs[2 * pr + 1];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb) {
            const floatx4 *src = reinterpret_cast<const floatx4 *>(fmb + mb * bstride + bb * 32 * kBlk);
            dst[bb][0] = src[0];
            dst[bb][1] = src[1];
        }
    };
    auto put_fm = [&](int set, const floatx4 (&v)[BBW][2]) {
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
            for (int j = 0; j < 2; ++j) sF[set][wave][bb][j][lane] = v[bb][j];
    };
    // f_m of the pair after that of super-step t is due when t is the second
    // super-step of a pair past the unit's first: loaded with t's stage,
    // written to the LDS set of its parity after the MFMAs of t - 1 (the
    // first super-step of t's pair, which reads the other set); the set it
    // overwrites was last read by the pair before t's.  The first two pairs
    // of the unit are loaded before the loop.
    auto fm_due = [&](long t) {
        return t % PPS == 1 && t / PPS > s0 / PPS && (t / PPS + 1) * PPS < s1;
    };
    floatx4 fmt[BBW][2];
    auto load_stage = [&](long s, Stage &x) {
        s = s < s1 ? s : s1 - 1;
        const long cb = s / PPS, d0 = (s % PPS) * SS;   // block, first dk step
        const u32x4 *Gs = reinterpret_cast<const u32x4 *>(G) + (cb * IBW * kBlk + d0) * 128;
#pragma unroll
        for (int c = 0; c < NQ; ++c)
            if (qact[c]) x.gv[c] = Gs[qoff[c] + lane];
        const int pr = (int)(s / PPS);
        const int kb = pairs[2 * pr];
        const int dk = (int)(s % PPS) * SS;
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb) {
            const fkvec v = *reinterpret_cast<const fkvec *>(fkb + kb * bstride + bb * 32 * kBlk + dk);
#pragma unroll
            for (int d = 0; d < SS; ++d) x.fk[bb][d] = v[d];
        }
    };
    auto stash = [&](int slot, const Stage &x) {
#pragma unroll
        for (int c = 0; c < NQ; ++c)
            if (qact[c]) sA[slot][qlds[c] + lane] = x.gv[c];
    };
    auto compute_fm = [&](int slot, const Stage &x, const floatx4 (&fmr)[BBW][2]) {
#pragma unroll
        for (int d = 0; d < SS; ++d) {
            opx8 Ah[IBA], Al[IBA];
#pragma unroll
            for (int ib = 0; ib < IBA; ++ib) {
                Ah[ib] = __builtin_bit_cast(opx8, sA[slot][ib * VPS + d * 128 + lane]);
                Al[ib] = __builtin_bit_cast(opx8, sA[slot][ib * VPS + d * 128 + 64 + lane]);
            }
#pragma unroll
            for (int bb = 0; bb < BBW; ++bb) {
                // F2 = f_k f_m for this lane's 8 K values, split hi + lo as
                // whole vectors (conversions two values per instruction).
                // BF16: hi is the product with its low 16 bits cleared (exact
                // in BF16, no conversion), lo = product - hi is exact in FP32
                // and rounded to BF16; FP16: hi rounded, lo = product - hi.
                // (FP16 results straight from fused multiply-adds take fewer
                // instructions but ran slower: each writes half a register.)
                const floatx4 m0 = fmr[bb][0], m1 = fmr[bb][1];
                const floatx8 fmv = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
                const floatx8 pv = x.fk[bb][d] * fmv;
                opx8 ph, pl;
                if constexpr (F16) {
                    ph = __builtin_convertvector(pv, opx8);
                    pl = __builtin_convertvector(pv - __builtin_convertvector(ph, floatx8), opx8);
                } else {
                    const u32x8 bits = __builtin_bit_cast(u32x8, pv);
                    const u32x8 hb = bits & 0xFFFF0000u;
                    u32x4 hw;
#pragma unroll
                    for (int j = 0; j < 4; ++j) hw[j] = (bits[2 * j] >> 16) | hb[2 * j + 1];
                    ph = __builtin_bit_cast(opx8, hw);
                    pl = __builtin_convertvector(pv - __builtin_bit_cast(floatx8, hb), opx8);
                }
                // three products, smallest first (SPLIT = 2: lo*hi, hi*hi
                // only, A not split; SPLIT = 1: hi*hi alone)
#pragma unroll
                for (int t = 0; t < 3; ++t)
#pragma unroll
                    for (int ib = 0; ib < IBA; ++ib) {
                        if constexpr (SPLIT == 1) {
                            if (t != 2) continue;
                        } else if constexpr (SPLIT == 2) {
                            if (t == 1) continue;
                        }
                        const opx8 &av = t == 0 ? pl : ph;
                        const opx8 &bv = t == 1 ? Al[ib] : Ah[ib];
                        if constexpr (F16)
                            acc[bb][ib] = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, acc[bb][ib], 0, 0, 0);
                        else
                            acc[bb][ib] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[bb][ib], 0, 0, 0);
                    }
            }
        }
    };

    // super-step s with the f_m set of its pair
    auto compute = [&](int slot, const Stage &x, long s) {
        const int set = (int)((s / PPS) & 1);
        floatx4 cur[BBW][2];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
            for (int j = 0; j < 2; ++j) cur[bb][j] = sF[set][wave][bb][j][lane];
        compute_fm(slot, x, cur);
    };

    // One super-step of the pipeline: the loads of super-step t = cs + 1 go
    // out into stage ld, super-step cs is computed from stage cx and LDS slot
    // cslot, then stage sx (super-step cs + 1) goes to the other slot; one
    // barrier.
    auto step = [&](long t, Stage &ld, int cslot, const Stage &cx, long cs, int sslot, const Stage &sx) {
        // (f_m first: its wait before put_fm then leaves stage t's loads in flight)
        const bool f = fm_due(t);
        if (f) load_fm((int)(t / PPS) + 1, fmt);
        load_stage(t, ld);
        __builtin_amdgcn_sched_barrier(0);      // keep the prefetch ahead of the MFMAs
        compute(cslot, cx, cs);
        __builtin_amdgcn_sched_barrier(0);
        stash(sslot, sx);
        if (f) put_fm((int)((t / PPS + 1) & 1), fmt);
        __syncthreads();
    };

    if (s0 < s1) {
        const int p0 = (int)(s0 / PPS);
        load_stage(s0, sa);
        load_fm(p0, fmt);
        put_fm(p0 & 1, fmt);
        if ((long)(p0 + 1) * PPS < s1) {
            load_fm(p0 + 1, fmt);
            put_fm((p0 + 1) & 1, fmt);
        }
        stash(0, sa);
    }
    __syncthreads();
    long s = s0;
    // Pairs of super-steps with no exit between them (a conditional exit
    // would let the compiler sink the prefetch below it); an odd last one is
    // done after the loop from stage a and slot 0, which then hold it.  (The
    // tensor pointer is not restrict-qualified: loads through it are then not
    // moved down to their use in stash.)
    for (; s + 1 < s1; s += 2) {
        step(s + 1, sb, 0, sa, s, 1, sb);
        step(s + 2, sa, 1, sb, s + 1, 0, sa);
    }
    if (s < s1) compute(0, sa, s);
    float *dst = part + (long)sp * bpad * ipad;
#pragma unroll
    for (int ib = 0; ib < IBW; ++ib) {
        if (ib0 + ib >= nib) continue;
        const int col = (ib0 + ib) * kIBlk + r;
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = brow0 + bb * 32 + 8 * (e >> 2) + 4 * hb + (e & 3);
                dst[(long)row * ipad + col] = acc[bb][ib][e];
            }
    }
}

// The launch: work unit u = (group of IBW i-blocks, K slot, range of
// compacted super-steps) with its count of multiplied i-blocks, one copy of
// the pipeline per count.
template <int BBW, int IBW, int SS, bool F16, int SPLIT = 3>
__global__ __launch_bounds__(256, 2) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_gemm_x3_lds(
    const uint16_t *G, const float *__restrict__ fop, const int *__restrict__ pairs,
    const int *__restrict__ act, const int *__restrict__ units, int nib, int bpad, int ipad, int nbt,
    float *__restrict__ part)
{
    static_assert(IBW == 4, "one pipeline per count of multiplied i-blocks, 1 to 4");
    typedef X3Shape<IBW, SS, SPLIT> Sh;
    __shared__ u32x4 sA[2][Sh::NV];
    __shared__ floatx4 sF[2][4][BBW][2][64];        // f_m: parity set, wave, b-block, half, lane
    const int L = xcd_logical(blockIdx.x, gridDim.x);
    const int bt = L % nbt, u = L / nbt;
    const int it = units[4 * u], sp = units[4 * u + 1];
    const long s0 = units[4 * u + 2], s1 = units[4 * u + 3];
    // (the first pair of a unit has the largest count of its pairs)
    const int na = s0 < s1 ? act[s0 / Sh::PPS] : IBW;
#define KXG_X3_RUN(A) \
    x3_run<BBW, IBW, SS, F16, SPLIT, A>(G, fop, pairs, it, sp, s0, s1, bt, nib, bpad, ipad, part, sA, sF)
    if (na == 1)
        KXG_X3_RUN(1);
    else if (na == 2)
        KXG_X3_RUN(2);
    else if (na == 3)
        KXG_X3_RUN(3);
    else
        KXG_X3_RUN(4);
#undef KXG_X3_RUN
}

}  // namespace

hipError_t launch_gemm16(bool f16, int split, int nwg, const uint16_t *G, const float *fop, const int *pairs,
                         const int *act, const int *units, int nib, int bpad, int ipad, int nbt, float *part,
                         hipStream_t s)
{
    constexpr int BBW = KXG_LDS_BBW, IBW = KXG_LDS_IBW;
#define KXG_X3(F, S)                                                                                   \
    hipLaunchKernelGGL((k_gemm_x3_lds<BBW, IBW, KXG_LDS_SS, F, S>), dim3(nwg), dim3(256), 0, s, G, fop, \
                       pairs, act, units, nib, bpad, ipad, nbt, part)
    if (f16) {
        if (split == 3) KXG_X3(true, 3); else if (split == 2) KXG_X3(true, 2); else KXG_X3(true, 1);
    } else {
        if (split == 3) KXG_X3(false, 3); else if (split == 2) KXG_X3(false, 2); else KXG_X3(false, 1);
    }
#undef KXG_X3
    return hipGetLastError();
}

}  // namespace kxg
