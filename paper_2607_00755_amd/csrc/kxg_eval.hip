// Evaluation of C[f] = gain - loss for a batch of distributions
// (Sec. 4.1 eq. discrete_collision_operator of arXiv 2607.00755, linear
// interpolation form), with the FP64 epilogue: loss term, two-moment
// projection (App. C) and diagnostics.
//
// gain paths
//   * stream: one pass over the dense tensor A[i][k][m] per group of up to
//     4 distributions, f staged in LDS; HBM-bound (single distribution).
//   * GEMM: gain[b][i] = sum_K F2[b][K] A'[i][K] with K = (k,m) over the
//     block-packed (k <= m) tensor, F2[b][(k,m)] = f_bk f_bm formed in
//     registers, on the MFMA units (FP32 32x32x2, or BF16/FP16 32x32x16 with a
//     hi+lo split of A' and of F2: hi*hi + hi*lo + lo*hi).  K is split over
//     workgroups (and over the 4 waves of each); partials are reduced in FP64
//     by the epilogue in a fixed order, independent of the batch size.
#include "kxg_step.h"

#include <type_traits>

namespace kxg {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

inline int div_up(long a, long b) { return (int)((a + b - 1) / b); }

#ifndef KXG_STREAM_UNROLL
#define KXG_STREAM_UNROLL 8
#endif
#ifndef KXG_STREAM_NT
#define KXG_STREAM_NT 1
#endif
// shape of the LDS-shared 16-bit GEMM: b-blocks and i-blocks per wave
#ifndef KXG_LDS_BBW
#define KXG_LDS_BBW 4
#endif
#ifndef KXG_LDS_IBW
#define KXG_LDS_IBW 2
#endif

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap so that consecutive logical indices share an XCD: workgroups
// that read the same slice of A (same i-block and K split, different batch
// tiles) then hit the same L2.
__device__ inline int xcd_logical(int bid, int nwg)
{
    if (nwg % 8 != 0) return bid;
    return (bid % 8) * (nwg / 8) + bid / 8;
}

// ---------------------------------------------------------------------------
// Stream gain: grid (split, i, group of BT distributions).  Each workgroup
// reads a contiguous chunk of row i of the dense tensor once and forms
// sum A[i][k][m] f_k f_m for its BT distributions, f taken from LDS; the
// (k, m) position of each element is tracked incrementally.
template <typename T, int VEC, int BT>
__global__ __launch_bounds__(256) void k_stream(const T *__restrict__ A,
                                                const double *__restrict__ f, int n, int B,
                                                int chunk, double *__restrict__ part)
{
    extern __shared__ double smem_d[];
    T *fs = reinterpret_cast<T *>(smem_d);
    __shared__ double red[4][BT];
    const int split = blockIdx.x, i = blockIdx.y, b0 = blockIdx.z * BT;
    for (int q = threadIdx.x; q < BT * n; q += 256) {
        const int bb = q / n, m = q - bb * n;
        fs[q] = (b0 + bb < B) ? (T)f[(long)(b0 + bb) * n + m] : (T)0;
    }
    __syncthreads();
    const long n2 = (long)n * n;
    const T *row = A + (long)i * n2;
    const long e_beg = (long)split * chunk;
    const long e_end = e_beg + chunk < n2 ? e_beg + chunk : n2;
    long e = e_beg + (long)threadIdx.x * VEC;
    int k = (int)(e / n), m = (int)(e - (long)k * n);
    constexpr int step = 256 * VEC;
    const int sk = step / n, sm = step - (step / n) * n;
    T acc[BT];
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) acc[bb] = (T)0;
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    // KXG_STREAM_UNROLL loads in flight per thread; A is read once per call,
    // so the loads are marked non-temporal
    constexpr int UN = KXG_STREAM_UNROLL;
    for (; e + (UN - 1) * step < e_end; e += UN * step) {
        vec_t a[UN];
        int kk[UN], mm[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
#if KXG_STREAM_NT
            a[u] = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(row + e + (long)u * step));
#else
            a[u] = *reinterpret_cast<const vec_t *>(row + e + (long)u * step);
#endif
            kk[u] = k;
            mm[u] = m;
            m += sm;
            k += sk;
            if (m >= n) { m -= n; ++k; }
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
#pragma unroll
            for (int bb = 0; bb < BT; ++bb) {
                const T *fb = fs + bb * n;
                T s = (T)0;
#pragma unroll
                for (int v = 0; v < VEC; ++v) s += a[u][v] * fb[mm[u] + v];
                acc[bb] += fb[kk[u]] * s;
            }
        }
    }
    for (; e < e_end; e += step) {
        const vec_t a = *reinterpret_cast<const vec_t *>(row + e);
#pragma unroll
        for (int bb = 0; bb < BT; ++bb) {
            const T *fb = fs + bb * n;
            T s = (T)0;
#pragma unroll
            for (int v = 0; v < VEC; ++v) s += a[v] * fb[m + v];
            acc[bb] += fb[k] * s;
        }
        m += sm;
        k += sk;
        if (m >= n) { m -= n; ++k; }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) {
        double v = (double)acc[bb];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][bb] = v;
    }
    __syncthreads();
    if (threadIdx.x < BT && b0 + (int)threadIdx.x < B) {
        const int bb = threadIdx.x;
        const double v = ((red[0][bb] + red[1][bb]) + red[2][bb]) + red[3][bb];
        part[((long)split * B + b0 + bb) * n + i] = v;
    }
}

// ---------------------------------------------------------------------------
// Exact-form stream (eq. app_dense_collision with the statistical factor of
// eq. Lambda_quantum): one pass over the dense weights and the bracket table;
// per (i, n, m) the fourth-momentum value f~ is interpolated with the
// energy-linear weights omega_R = (K~ - K_jL) / (K_jL+1 - K_jL), linearly in
// f or (LOGI) in ln max(f, 1e-300), and four sums are accumulated per
// distribution: gain = sum W f_n f_m, S0 = sum W f~, S1 = sum W f~ (f_n + f_m),
// T1 = sum W f~ f_n f_m (the last two only with quantum statistics).  The
// epilogue forms C = (1 + eta f_i)(gain + eta T1) - f_i (S0 + eta S1 + eta^2 T1).
template <typename T, int VEC, int BT, bool LOGI, bool QUANT>
__global__ __launch_bounds__(256) void k_stream_x(const T *__restrict__ A,
                                                  const uint16_t *__restrict__ JL,
                                                  const double *__restrict__ f,
                                                  const double *__restrict__ K,
                                                  const double *__restrict__ invdK, int n, int B,
                                                  int chunk, double *__restrict__ part)
{
    constexpr int NA = QUANT ? 4 : 2;
    extern __shared__ double smem_d[];
    double *Ks = smem_d;                       // [n]
    double *iK = Ks + n;                       // [n]
    T *fs = reinterpret_cast<T *>(iK + n);     // [BT][n]
    T *ls = fs + BT * n;                       // [BT][n] ln max(f, floor) (LOGI)
    __shared__ double red[4][BT][NA];
    const int split = blockIdx.x, i = blockIdx.y, b0 = blockIdx.z * BT;
    for (int q = threadIdx.x; q < n; q += 256) {
        Ks[q] = K[q];
        iK[q] = invdK[q];
    }
    for (int q = threadIdx.x; q < BT * n; q += 256) {
        const int bb = q / n, m = q - bb * n;
        const double v = (b0 + bb < B) ? f[(long)(b0 + bb) * n + m] : 0.0;
        fs[q] = (T)v;
        if (LOGI) ls[q] = (T)log(v > 1e-300 ? v : 1e-300);
    }
    __syncthreads();
    const long n2 = (long)n * n;
    const T *row = A + (long)i * n2;
    const uint16_t *jrow = JL + (long)i * n2;
    const double ki = Ks[i];
    const long e_beg = (long)split * chunk;
    const long e_end = e_beg + chunk < n2 ? e_beg + chunk : n2;
    long e = e_beg + (long)threadIdx.x * VEC;
    int k = (int)(e / n), m = (int)(e - (long)k * n);
    constexpr int step = 256 * VEC;
    const int sk = step / n, sm = step - (step / n) * n;
    T acc[BT][NA];
#pragma unroll
    for (int bb = 0; bb < BT; ++bb)
#pragma unroll
        for (int c = 0; c < NA; ++c) acc[bb][c] = (T)0;
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    for (; e < e_end; e += step) {
        const vec_t a = *reinterpret_cast<const vec_t *>(row + e);
        const double kk = Ks[k];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int mv = m + v;
            const int jl = jrow[e + v];
            if (jl == 0xFFFF) continue;
            const double kt = (kk + Ks[mv]) - ki;
            const T wr = (T)((kt - Ks[jl]) * iK[jl]);
            const T wl = (T)1 - wr;
            const T w = a[v];
#pragma unroll
            for (int bb = 0; bb < BT; ++bb) {
                const T *fb = fs + bb * n;
                const T fn = fb[k], fm = fb[mv];
                T ft;
                if (LOGI) {
                    const T *lb = ls + bb * n;
                    ft = (T)exp(wl * lb[jl] + wr * lb[jl + 1]);
                } else {
                    ft = wl * fb[jl] + wr * fb[jl + 1];
                }
                const T wf = w * ft;
                acc[bb][0] += w * fn * fm;
                acc[bb][1] += wf;
                if constexpr (QUANT) {
                    acc[bb][2] += wf * (fn + fm);
                    acc[bb][3] += wf * fn * fm;
                }
            }
        }
        m += sm;
        k += sk;
        if (m >= n) { m -= n; ++k; }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int bb = 0; bb < BT; ++bb)
#pragma unroll
        for (int c = 0; c < NA; ++c) {
            double v = (double)acc[bb][c];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[wave][bb][c] = v;
        }
    __syncthreads();
    if ((int)threadIdx.x < BT * 4) {
        // all four sums are written (zeros for the quantum ones in the dilute form)
        const int bb = threadIdx.x / 4, c = threadIdx.x % 4;
        if (b0 + bb < B) {
            const double v = c < NA ? ((red[0][bb][c] + red[1][bb][c]) + red[2][bb][c]) + red[3][bb][c]
                                    : 0.0;
            part[(((long)split * B + b0 + bb) * 4 + c) * n + i] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// MFMA operand of the distributions: per 16-wide block of the grid, FP32
// values in natural order [nb][bpad][16] and in parity order
// [nb][bpad][2][8] (the 32x32x2 MFMA pairs K indices 2t and 2t+1).
// For FP16 each distribution is scaled by a power of two so that
// max f <= 2^7 (F2 <= 2^14).  One workgroup per (padded) distribution.
__global__ __launch_bounds__(256) void k_prep(const double *__restrict__ f, int B, int n,
                                              int nb, int bpad, int scale16,
                                              float *__restrict__ fop,
                                              float *__restrict__ fpar,
                                              float *__restrict__ fscale)
{
    __shared__ double red[256];
    const int b = blockIdx.x;
    float sc = 1.0f;
    if (scale16) {
        double mx = 0.0;
        if (b < B)
            for (int q = threadIdx.x; q < n; q += 256) mx = fmax(mx, fabs(f[(long)b * n + q]));
        red[threadIdx.x] = mx;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        mx = red[0];
        if (mx > 0.0 && isfinite(mx)) sc = (float)ldexp(1.0, 7 - (int)ceil(log2(mx)));
        if (threadIdx.x == 0) fscale[b] = sc;
    }
    for (int q = threadIdx.x; q < nb * kBlk; q += 256) {
        const double v = (b < B && q < n) ? f[(long)b * n + q] : 0.0;
        const float x = (float)v * sc;
        const int blk = q / kBlk, d = q % kBlk;
        fop[((long)blk * bpad + b) * kBlk + d] = x;
        fpar[(((long)blk * bpad + b) * 2 + (d & 1)) * 8 + (d >> 1)] = x;
    }
}

// Reduce the 4 waves' accumulators of a workgroup (fixed order 0+1+2+3) and
// store the FP32 partial of this K split.  32x32 MFMA result layout: register
// e of lane l holds row 8*(e/4) + 4*(l/32) + e%4, column l%32.
template <int BBW>
__device__ void store_tile(floatx16 (&acc)[BBW], float *lds, float *__restrict__ part, int sp,
                           int bpad, int ipad, int brow0, int icol0)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave > 0) {
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                lds[(((wave - 1) * BBW + bb) * 16 + e) * 64 + lane] = acc[bb][e];
    }
    __syncthreads();
    if (wave == 0) {
        float *dst = part + (long)sp * bpad * ipad;
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                float v = acc[bb][e];
                v += lds[((0 * BBW + bb) * 16 + e) * 64 + lane];
                v += lds[((1 * BBW + bb) * 16 + e) * 64 + lane];
                v += lds[((2 * BBW + bb) * 16 + e) * 64 + lane];
                const int row = brow0 + bb * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                dst[(long)row * ipad + icol0 + (lane & 31)] = v;
            }
    }
}

// FP32 GEMM on v_mfma_f32_32x32x2f32.  Workgroup = (batch tile of BBW*32
// distributions, i-block of 32 rows, K split); its 4 waves take 4
// consecutive sub-ranges of the split's dk steps.  Per dk step (one row k of a
// (kb, mb) block, 16 K values) a wave issues 8*BBW MFMAs; the A operand
// (F2 = f_k f_m) is one multiply per MFMA, the B operand (packed tensor)
// comes straight from memory in MFMA order, prefetched one step ahead.
template <int BBW>
__global__ __launch_bounds__(256, 2) void k_gemm_f32(
    const float *__restrict__ G, const float *__restrict__ fop, const float *__restrict__ fpar,
    const int *__restrict__ pairs, int npairs, int bpad, int ipad, int nbt, int splits,
    long dksteps, float *__restrict__ part)
{
    __shared__ float lds[3 * BBW * 16 * 64];
    int L = xcd_logical(blockIdx.x, gridDim.x);
    const int bt = L % nbt;
    L /= nbt;
    const int sp = L % splits;
    const int ib = L / splits;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 31, hb = lane >> 5;
    const long w = (long)sp * kWaves + wave, nw = (long)splits * kWaves;
    const long u0 = w * dksteps / nw, u1 = (w + 1) * dksteps / nw;
    const int brow0 = bt * BBW * 32;
    const float *Gi = G + (long)ib * npairs * kBlk * 512;

    floatx16 acc[BBW];
#pragma unroll
    for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[bb][e] = 0.0f;

    float fm[BBW][8];
    int cur_pair = -1;
    float4 nb0 = make_float4(0, 0, 0, 0), nb1 = nb0;
    float nfk[BBW];
    if (u0 < u1) {
        const int pr = (int)(u0 >> 4), dk = (int)(u0 & 15);
        const float *gp = Gi + u0 * 512;
        nb0 = reinterpret_cast<const float4 *>(gp)[lane];
        nb1 = reinterpret_cast<const float4 *>(gp + 256)[lane];
        const int kb = pairs[2 * pr];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb)
            nfk[bb] = fop[((long)kb * bpad + brow0 + bb * 32 + r) * kBlk + dk];
    }
    for (long u = u0; u < u1; ++u) {
        const int pr = (int)(u >> 4);
        if (pr != cur_pair) {
            cur_pair = pr;
            const int mb = pairs[2 * pr + 1];
#pragma unroll
            for (int bb = 0; bb < BBW; ++bb) {
                const float4 *src = reinterpret_cast<const float4 *>(
                    fpar + (((long)mb * bpad + brow0 + bb * 32 + r) * 2 + hb) * 8);
                const float4 x0 = src[0], x1 = src[1];
                fm[bb][0] = x0.x; fm[bb][1] = x0.y; fm[bb][2] = x0.z; fm[bb][3] = x0.w;
                fm[bb][4] = x1.x; fm[bb][5] = x1.y; fm[bb][6] = x1.z; fm[bb][7] = x1.w;
            }
        }
        const float4 b0 = nb0, b1 = nb1;
        float fk[BBW];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb) fk[bb] = nfk[bb];
        if (u + 1 < u1) {
            const long un = u + 1;
            const int prn = (int)(un >> 4), dkn = (int)(un & 15);
            const float *gp = Gi + un * 512;
            nb0 = reinterpret_cast<const float4 *>(gp)[lane];
            nb1 = reinterpret_cast<const float4 *>(gp + 256)[lane];
            const int kbn = pairs[2 * prn];
#pragma unroll
            for (int bb = 0; bb < BBW; ++bb)
                nfk[bb] = fop[((long)kbn * bpad + brow0 + bb * 32 + r) * kBlk + dkn];
        }
        const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int bb = 0; bb < BBW; ++bb)
                acc[bb] = __builtin_amdgcn_mfma_f32_32x32x2f32(fk[bb] * fm[bb][t], bv[t],
                                                               acc[bb], 0, 0, 0);
    }
    store_tile<BBW>(acc, lds, part, sp, bpad, ipad, brow0, ib * kIBlk);
}

// 16-bit x3 GEMM on v_mfma_f32_32x32x16_{bf16,f16}: per dk step one MFMA
// K-step of 16; F2 is formed in FP32 and split into hi + lo; the packed
// tensor arrives pre-split.  gain ~ A_hi F2_hi + A_hi F2_lo + A_lo F2_hi.
template <int BBW, bool F16>
__global__ __launch_bounds__(256, 2) void k_gemm_x3(
    const uint16_t *__restrict__ G, const float *__restrict__ fop, const int *__restrict__ pairs,
    int npairs, int bpad, int ipad, int nbt, int splits, long dksteps,
    float *__restrict__ part)
{
    typedef typename std::conditional<F16, halfx8, bf16x8>::type opx8;
    typedef typename std::conditional<F16, _Float16, __bf16>::type op_t;
    __shared__ float lds[3 * BBW * 16 * 64];
    int L = xcd_logical(blockIdx.x, gridDim.x);
    const int bt = L % nbt;
    L /= nbt;
    const int sp = L % splits;
    const int ib = L / splits;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 31, hb = lane >> 5;
    const long w = (long)sp * kWaves + wave, nw = (long)splits * kWaves;
    const long u0 = w * dksteps / nw, u1 = (w + 1) * dksteps / nw;
    const int brow0 = bt * BBW * 32;
    const uint16_t *Gi = G + (long)ib * npairs * kBlk * 1024;

    floatx16 acc[BBW];
#pragma unroll
    for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[bb][e] = 0.0f;

    float fm[BBW][8];
    int cur_pair = -1;
    uint4 nh = make_uint4(0, 0, 0, 0), nl = nh;
    float nfk[BBW];
    if (u0 < u1) {
        const int pr = (int)(u0 >> 4), dk = (int)(u0 & 15);
        const uint16_t *gp = Gi + u0 * 1024;
        nh = reinterpret_cast<const uint4 *>(gp)[lane];
        nl = reinterpret_cast<const uint4 *>(gp + 512)[lane];
        const int kb = pairs[2 * pr];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb)
            nfk[bb] = fop[((long)kb * bpad + brow0 + bb * 32 + r) * kBlk + dk];
    }
    for (long u = u0; u < u1; ++u) {
        const int pr = (int)(u >> 4);
        if (pr != cur_pair) {
            cur_pair = pr;
            const int mb = pairs[2 * pr + 1];
#pragma unroll
            for (int bb = 0; bb < BBW; ++bb) {
                const float4 *src = reinterpret_cast<const float4 *>(
                    fop + ((long)mb * bpad + brow0 + bb * 32 + r) * kBlk + 8 * hb);
                const float4 x0 = src[0], x1 = src[1];
                fm[bb][0] = x0.x; fm[bb][1] = x0.y; fm[bb][2] = x0.z; fm[bb][3] = x0.w;
                fm[bb][4] = x1.x; fm[bb][5] = x1.y; fm[bb][6] = x1.z; fm[bb][7] = x1.w;
            }
        }
        const uint4 ah = nh, al = nl;
        float fk[BBW];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb) fk[bb] = nfk[bb];
        if (u + 1 < u1) {
            const long un = u + 1;
            const int prn = (int)(un >> 4), dkn = (int)(un & 15);
            const uint16_t *gp = Gi + un * 1024;
            nh = reinterpret_cast<const uint4 *>(gp)[lane];
            nl = reinterpret_cast<const uint4 *>(gp + 512)[lane];
            const int kbn = pairs[2 * prn];
#pragma unroll
            for (int bb = 0; bb < BBW; ++bb)
                nfk[bb] = fop[((long)kbn * bpad + brow0 + bb * 32 + r) * kBlk + dkn];
        }
        const opx8 Ah = __builtin_bit_cast(opx8, ah);
        const opx8 Al = __builtin_bit_cast(opx8, al);
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb) {
            opx8 ph, pl;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float pv = fk[bb] * fm[bb][j];
                const op_t h = (op_t)pv;
                ph[j] = h;
                pl[j] = (op_t)(pv - (float)h);
            }
            if constexpr (F16) {
                acc[bb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(pl, Ah, acc[bb], 0, 0, 0);
                acc[bb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ph, Al, acc[bb], 0, 0, 0);
                acc[bb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ph, Ah, acc[bb], 0, 0, 0);
            } else {
                acc[bb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl, Ah, acc[bb], 0, 0, 0);
                acc[bb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, Al, acc[bb], 0, 0, 0);
                acc[bb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, Ah, acc[bb], 0, 0, 0);
            }
        }
    }
    store_tile<BBW>(acc, lds, part, sp, bpad, ipad, brow0, ib * kIBlk);
}

// 16-bit x3 GEMM for large batches, A operand shared through LDS.  A
// workgroup's 4 waves work on the same K chunk (split) and the same IBW
// i-blocks; wave w takes the BBW b-blocks [w*BBW, (w+1)*BBW) of the
// workgroup's 4*BBW*32-row batch tile.  Per dk step the workgroup stages the
// hi/lo A fragments of its i-blocks (2 KB each) once into a 3-deep LDS ring
// (global loads issued two steps ahead); every wave forms and splits its F2
// operand once per b-block and feeds it to 3*IBW MFMAs.  One barrier per dk
// step.  Partials: one per K split.
template <int BBW, int IBW, bool F16>
__global__ __launch_bounds__(256, 2) void k_gemm_x3_lds(
    const uint16_t *__restrict__ G, const float *__restrict__ fop, const int *__restrict__ pairs,
    int npairs, int nib, int bpad, int ipad, int nbt, int nit, int splits, long dksteps,
    float *__restrict__ part)
{
    typedef typename std::conditional<F16, halfx8, bf16x8>::type opx8;
    typedef typename std::conditional<F16, _Float16, __bf16>::type op_t;
    constexpr int NV = IBW * 2 * 64;               // 16-byte vectors per dk step
    constexpr int PT = (NV + 255) / 256;           // vectors per thread
    __shared__ uint4 sA[3][NV];
    int L = xcd_logical(blockIdx.x, gridDim.x);
    const int bt = L % nbt;
    L /= nbt;
    const int sp = L % splits;
    const int it = L / splits;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 31, hb = lane >> 5;
    const long u0 = (long)sp * dksteps / splits, u1 = (long)(sp + 1) * dksteps / splits;
    const int brow0 = bt * (4 * BBW * 32) + wave * (BBW * 32);
    const int ib0 = it * IBW;
    // loader role: vectors q = threadIdx.x + 256 c of each dk step; a dk step
    // of one i-block is 1024 16-bit values = 128 vectors ([hi|lo][lane][8])
    const uint4 *qsrc[PT];
    bool qload[PT];
#pragma unroll
    for (int c = 0; c < PT; ++c) {
        const int q = threadIdx.x + 256 * c;
        const int qib = q / 128;
        qload[c] = q < NV && ib0 + qib < nib;
        qsrc[c] = reinterpret_cast<const uint4 *>(
                      G + (long)(ib0 + (qload[c] ? qib : 0)) * npairs * kBlk * 1024) + (q % 128);
    }
    const uint4 zero4 = make_uint4(0, 0, 0, 0);
    auto fetch = [&](long u, uint4 (&dst)[PT]) {
#pragma unroll
        for (int c = 0; c < PT; ++c) dst[c] = (qload[c] && u < u1) ? qsrc[c][u * 128] : zero4;
    };
    auto stash = [&](int slot, const uint4 (&src)[PT]) {
#pragma unroll
        for (int c = 0; c < PT; ++c) {
            const int q = threadIdx.x + 256 * c;
            if (q < NV) sA[slot][q] = src[c];
        }
    };
    auto load_fk = [&](long u, float (&dst)[BBW]) {
        if (u >= u1) return;
        const int pr = (int)(u >> 4), dk = (int)(u & 15);
        const int kb = pairs[2 * pr];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb)
            dst[bb] = fop[((long)kb * bpad + brow0 + bb * 32 + r) * kBlk + dk];
    };

    floatx16 acc[BBW][IBW];
#pragma unroll
    for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
        for (int ib = 0; ib < IBW; ++ib)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[bb][ib][e] = 0.0f;

    uint4 ra[PT], rb[PT];
    float fk1[BBW], fk2[BBW], fm[BBW][8];
    if (u0 < u1) {
        uint4 r0[PT];
        fetch(u0, r0);
        stash(0, r0);
    }
    fetch(u0 + 1, ra);
    fetch(u0 + 2, rb);
    load_fk(u0, fk1);
    load_fk(u0 + 1, fk2);
    int cur_pair = -1;
    __syncthreads();
    for (long u = u0; u < u1; ++u) {
        const int idx = (int)(u - u0);
        const int slot = idx % 3;
        stash((idx + 1) % 3, ra);         // data of step u+1, read after the next barrier
#pragma unroll
        for (int c = 0; c < PT; ++c) ra[c] = rb[c];
        fetch(u + 3, rb);
        float fk[BBW];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb) { fk[bb] = fk1[bb]; fk1[bb] = fk2[bb]; }
        load_fk(u + 2, fk2);
        const int pr = (int)(u >> 4);
        if (pr != cur_pair) {
            cur_pair = pr;
            const int mb = pairs[2 * pr + 1];
#pragma unroll
            for (int bb = 0; bb < BBW; ++bb) {
                const float4 *src = reinterpret_cast<const float4 *>(
                    fop + ((long)mb * bpad + brow0 + bb * 32 + r) * kBlk + 8 * hb);
                const float4 x0 = src[0], x1 = src[1];
                fm[bb][0] = x0.x; fm[bb][1] = x0.y; fm[bb][2] = x0.z; fm[bb][3] = x0.w;
                fm[bb][4] = x1.x; fm[bb][5] = x1.y; fm[bb][6] = x1.z; fm[bb][7] = x1.w;
            }
        }
        opx8 ph[BBW], pl[BBW];
#pragma unroll
        for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float pv = fk[bb] * fm[bb][j];
                const op_t h = (op_t)pv;
                ph[bb][j] = h;
                pl[bb][j] = (op_t)(pv - (float)h);
            }
        opx8 Ah[IBW], Al[IBW];
#pragma unroll
        for (int ib = 0; ib < IBW; ++ib) {
            Ah[ib] = __builtin_bit_cast(opx8, sA[slot][ib * 128 + lane]);
            Al[ib] = __builtin_bit_cast(opx8, sA[slot][ib * 128 + 64 + lane]);
        }
        // three products, smallest first; consecutive MFMAs hit different
        // accumulators
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int bb = 0; bb < BBW; ++bb)
#pragma unroll
                for (int ib = 0; ib < IBW; ++ib) {
                    const opx8 &a = t == 0 ? pl[bb] : ph[bb];
                    const opx8 &bm = t == 1 ? Al[ib] : Ah[ib];
                    if constexpr (F16)
                        acc[bb][ib] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, bm, acc[bb][ib], 0, 0, 0);
                    else
                        acc[bb][ib] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bm, acc[bb][ib], 0, 0, 0);
                }
        __syncthreads();
    }
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

// ---------------------------------------------------------------------------
// Loss rates rate[b][i] = sum_j R[i][j] f_bj in FP64 on v_mfma_f64_16x16x4f64.
// Workgroup = one 16 (b) x 16 (i) output tile; its 4 waves take 4
// consecutive j ranges and their accumulators are added in the fixed order
// 0+1+2+3.  Operand/result layout of the instruction: A[row][k] at lane
// row + 16k, B[k][col] at lane col + 16k, D[row][col] at lane
// col + 16 (row % 4), register row / 4.
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int kRateT = 16;
__global__ __launch_bounds__(256) void k_rate(const double *__restrict__ RT,
                                              const double *__restrict__ f, int n, int B,
                                              double *__restrict__ rate)
{
    __shared__ double red[3][4][64];
    const int b0 = blockIdx.x * kRateT, i0 = blockIdx.y * kRateT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int nsteps = (n + 3) / 4;                         // K steps of 4
    const int per = (nsteps + 3) / 4;
    const int s0 = wave * per, s1 = min(nsteps, s0 + per);
    const int b = b0 + lr, i = i0 + lr;
    const double *frow = f + (long)(b < B ? b : 0) * n;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    int st = s0;
    for (; st + 4 <= s1; st += 4) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = 4 * (st + u) + lk;
            av[u] = (b < B && j < n) ? frow[j] : 0.0;
            bv[u] = (i < n && j < n) ? RT[(long)j * n + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    for (; st < s1; ++st) {
        const int j = 4 * st + lk;
        const double av = (b < B && j < n) ? frow[j] : 0.0;
        const double bv = (i < n && j < n) ? RT[(long)j * n + i] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    if (wave > 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave - 1][r][lane] = acc[r];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double v = ((acc[r] + red[0][r][lane]) + red[1][r][lane]) + red[2][r][lane];
            const int bo = b0 + lk + 4 * r, io = i0 + lr;
            if (bo < B && io < n) rate[(long)bo * n + io] = v;
        }
    }
}

// Wave-wide (64-lane) butterfly reductions; every lane ends with the same
// value, since each pairwise step adds the same two operands.
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// Deterministic block sums over 256 threads (4 waves), used by k_moments.
template <int NV>
__device__ void block_sum(double (&v)[NV], double *lds)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) lds[wave * NV + j] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = ((lds[j] + lds[NV + j]) + lds[2 * NV + j]) + lds[3 * NV + j];
    __syncthreads();
}

// FP64 epilogue, one wave per distribution (4 per workgroup), PER grid
// points per lane (App. C):
//   gain = sum of the split partials (fixed order; FP16 scales undone),
//   C_raw = gain - f * rate,
//   xi_i = |f_i|/f_max above 1e-12, and the 2x2 system for the correction
//   xi (alpha' + beta' K) written in kinetic energy K = E - m (the span of
//   {xi, xi E} equals that of {xi, xi K}; alpha = alpha' - beta' m,
//   beta = beta' in the paper's E-form), C_proj = C_raw - xi (alpha' + beta' K),
//   and the diagnostics of eqs. app_epsilon_definition and
//   app_projection_relative_correction.
template <int PER>
__device__ void step_update(const StepArgs &A, int b, int n, const double (&out)[PER], int lane);

template <typename PT, int PER>
__global__ __launch_bounds__(256) void k_epilogue(
    const PT *__restrict__ part, int nsplit, long split_stride, int ld_b,
    const float *__restrict__ fscale, const float *__restrict__ rscale,
    const double *__restrict__ rate, const double *__restrict__ f,
    const double *__restrict__ h, const double *__restrict__ K, const double *__restrict__ E,
    double mass, int n, int B, int project, double *__restrict__ C, double *__restrict__ diag,
    StepArgs step, const double *__restrict__ ext, double eta)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B) return;                      // whole wave; no block barriers below
    const double *fb = f + (long)b * n;
    double fv[PER], craw[PER], xi[PER];
    double fmaxv = 0.0, rmax = 0.0, gmax = 0.0, flag = 0.0;
    double inv_s2 = 1.0;
    if (fscale) {
        const double sc = fscale[b];
        inv_s2 = 1.0 / (sc * sc);
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = lane + 64 * q;
        fv[q] = 0.0;
        craw[q] = 0.0;
        if (i < n) {
            const double x = fb[i];
            fv[q] = x;
            if (!isfinite(x)) flag = fmax(flag, 1.0);
            else if (x < 0.0) flag = fmax(flag, 0.5);
            fmaxv = fmax(fmaxv, fabs(x));
            if (ext) {
                // exact form: four split sums per row, layout [split][B][4][n]
                double a4[4] = {0.0, 0.0, 0.0, 0.0};
                for (int sp = 0; sp < nsplit; ++sp)
#pragma unroll
                    for (int c = 0; c < 4; ++c) a4[c] += ext[(((long)sp * B + b) * 4 + c) * n + i];
                const double gq = (1.0 + eta * x) * (a4[0] + eta * a4[3]);
                const double lq = x * (a4[1] + eta * a4[2] + eta * eta * a4[3]);
                rmax = fmax(rmax, a4[1]);
                gmax = fmax(gmax, fabs(gq));
                craw[q] = gq - lq;
            } else {
                // split partials: loads issued 8 at a time, added in split order
                const PT *pp = part + (long)b * ld_b + i;
                double g = 0.0;
                int sp = 0;
                for (; sp + 8 <= nsplit; sp += 8) {
                    double v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = (double)pp[(sp + u) * split_stride];
#pragma unroll
                    for (int u = 0; u < 8; ++u) g += v[u];
                }
                for (; sp < nsplit; ++sp) g += (double)pp[sp * split_stride];
                if (fscale) g *= inv_s2 / (double)rscale[i];
                const double rt = rate[(long)b * n + i];
                rmax = fmax(rmax, rt);
                gmax = fmax(gmax, fabs(g));
                craw[q] = g - x * rt;
            }
        }
    }
    fmaxv = wave_max(fmaxv);
    rmax = wave_max(rmax);
    gmax = wave_max(gmax);
    flag = wave_max(flag);
    double s0 = 0, s1 = 0, b00 = 0, b01 = 0, b11 = 0, an = 0, ae = 0, se = 0, num = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = lane + 64 * q;
        xi[q] = 0.0;
        if (i < n) {
            const double hi = h[i], ki = K[i], ei = E[i];
            const double r = fmaxv > 0.0 ? fabs(fv[q]) / fmaxv : 0.0;
            xi[q] = r > 1e-12 ? r : 0.0;
            s0 += hi * craw[q];
            s1 += hi * ki * craw[q];
            b00 += hi * xi[q];
            b01 += hi * ki * xi[q];
            b11 += hi * ki * ki * xi[q];
            an += hi * fabs(craw[q]);
            ae += hi * ei * fabs(craw[q]);
            se += hi * ei * craw[q];
            num += hi * fv[q];
        }
    }
    s0 = wave_sum(s0); s1 = wave_sum(s1);
    b00 = wave_sum(b00); b01 = wave_sum(b01); b11 = wave_sum(b11);
    an = wave_sum(an); ae = wave_sum(ae); se = wave_sum(se); num = wave_sum(num);
    double al = 0.0, be = 0.0;
    const double det = b00 * b11 - b01 * b01;
    if (project && det != 0.0 && isfinite(det)) {
        al = (s0 * b11 - s1 * b01) / det;
        be = (s1 * b00 - s0 * b01) / det;
    }
    double t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0, t5 = 0, bad = 0.0;
    double out[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = lane + 64 * q;
        out[q] = 0.0;
        if (i < n) {
            const double hi = h[i], ei = E[i];
            const double cp = craw[q] - xi[q] * (al + be * K[i]);
            const double d = fabs(cp - craw[q]);
            t0 += hi * cp;
            t1 += hi * ei * cp;
            t2 += hi * fabs(cp);
            t3 += hi * ei * fabs(cp);
            t4 += hi * d;
            t5 += hi * ei * d;
            out[q] = project ? cp : craw[q];
            if (!isfinite(out[q])) bad = 1.0;
        }
    }
    if (step.mode != kStepNone) {
        step_update<PER>(step, b, n, out, lane);
        return;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = lane + 64 * q;
        if (i < n) C[(long)b * n + i] = out[q];
    }
    if (diag) {
        t0 = wave_sum(t0); t1 = wave_sum(t1); t2 = wave_sum(t2);
        t3 = wave_sum(t3); t4 = wave_sum(t4); t5 = wave_sum(t5);
        bad = wave_max(bad);
        if (lane == 0) {
            double *d = diag + (long)b * KXG_NDIAG;
            d[0] = al - be * mass;
            d[1] = be;
            d[2] = an > 0.0 ? s0 / an : 0.0;
            d[3] = ae > 0.0 ? se / ae : 0.0;
            d[4] = t2 > 0.0 ? t0 / t2 : 0.0;
            d[5] = t3 > 0.0 ? t1 / t3 : 0.0;
            d[6] = an > 0.0 ? t4 / an : 0.0;
            d[7] = ae > 0.0 ? t5 / ae : 0.0;
            d[8] = rmax;
            d[9] = gmax;
            double st = 0.0;
            if (flag >= 1.0) st += 1.0;
            else if (flag > 0.0) st += 2.0;
            if (bad > 0.0) st += 4.0;
            d[10] = st;
            d[11] = num;
        }
    }
}


// Stepper update of slot b from the operator output `out` (lane-strided,
// element i = lane + 64 q), Sec. 4.2: RK4 stage, or Heun predictor
// x* = x + dt k1, or Heun corrector x_new = x + dt (k1 + k2)/2 with the
// predictor-corrector error err = max |x_new - x*| / (atol + rtol
// max(|x|, |x_new|)), acceptance err <= 1 (always in replay mode) and
// dt *= clamp(safety err^-1/2, fac_lo, fac_hi), clipped to end at t_end.
// Every lane reaches the same decision (butterfly reductions); lane 0
// writes the slot record.
template <int PER>
__device__ void step_update(const StepArgs &A, int b, int n, const double (&out)[PER], int lane)
{
    SlotDev &S = A.sl[b];
    const int running = S.status == 0;
    const long row = (long)b * n;
    const double dt = S.dt, u = S.t;
    if (A.mode == kStepRK4) {
        const double lam = S.lam / S.hi_scale;
        double bad = 0.0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = lane + 64 * q;
            if (i >= n) continue;
            const double xv = A.x[row + i];
            if (!running) { A.fb[row + i] = xv; continue; }
            const double k = lam * out[q];
            if (A.stage == 1) { A.acc[row + i] = k; A.fb[row + i] = xv + 0.5 * dt * k; }
            else if (A.stage == 2) { A.acc[row + i] += 2.0 * k; A.fb[row + i] = xv + 0.5 * dt * k; }
            else if (A.stage == 3) { A.acc[row + i] += 2.0 * k; A.fb[row + i] = xv + dt * k; }
            else {
                const double xn = xv + dt / 6.0 * (A.acc[row + i] + k);
                A.x[row + i] = xn;
                A.fb[row + i] = xn;
                if (!isfinite(xn)) bad = 1.0;
            }
        }
        if (A.stage == 4) {
            bad = wave_max(bad);
            if (lane == 0 && running) {
                S.t = u + dt;
                S.steps += 1;
                if (bad > 0.0) S.status = -1;
                else if (S.t >= S.tend * (1.0 - 1e-14) || (S.maxsteps > 0 && S.steps >= S.maxsteps))
                    S.status = 1;
                else if (S.t + dt > S.tend) S.dt = S.tend - S.t;
            }
        }
        return;
    }
    if (A.mode == kStepHeunPred) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = lane + 64 * q;
            if (i >= n) continue;
            const double xv = A.x[row + i];
            if (!running) { A.xs[row + i] = xv; continue; }
            const double nx = (i + 1 < n) ? A.x[row + i + 1] : 0.0;
            const double k = rhs_u(A.expansion, xv, nx, out[q], A.p[i], A.dp[i], S.lam, S.hi_scale, u);
            A.acc[row + i] = k;
            const double v = xv + dt * k;
            A.xs[row + i] = v;
            A.fb[row + i] = A.expansion ? g_to_f(v, A.p[i], u + dt) : v;
        }
        return;
    }
    // Heun corrector and control
    double xn[PER];
    double err = 0.0, nonfin = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = lane + 64 * q;
        xn[q] = 0.0;
        if (i >= n || !running) continue;
        const double xsv = A.xs[row + i];
        const double nx = (i + 1 < n) ? A.xs[row + i + 1] : 0.0;
        const double k2 = rhs_u(A.expansion, xsv, nx, out[q], A.p[i], A.dp[i], S.lam, S.hi_scale, u + dt);
        const double x0 = A.x[row + i];
        const double v = x0 + 0.5 * dt * (A.acc[row + i] + k2);
        xn[q] = v;
        const double sc = S.atol + A.rtol * fmax(fabs(x0), fabs(v));
        const double e = fabs(v - xsv) / sc;
        if (!isfinite(v)) nonfin = 1.0;
        err = fmax(err, isfinite(e) ? e : 1e300);
    }
    err = wave_max(err);
    nonfin = wave_max(nonfin);
    int accept = 0, status = S.status, steps = S.steps, rej = S.rejected;
    double tnew = u, dtnew = dt, outflow = S.outflow;
    if (running) {
        if (nonfin > 0.0) {
            status = -1;
        } else {
            accept = (!A.adapt) || err <= 1.0;
            if (accept) {
                if (A.expansion) outflow += 0.5 * dt * (A.x[row] + A.xs[row]);
                tnew = u + dt;
                steps += 1;
            } else {
                rej += 1;
            }
            if (A.adapt) {
                double fac = err > 0.0 ? A.safety / sqrt(err) : A.fac_hi;
                fac = fmin(A.fac_hi, fmax(A.fac_lo, fac));
                dtnew = dt * fac;
            }
            if (accept && (tnew >= S.tend * (1.0 - 1e-14) || (S.maxsteps > 0 && steps >= S.maxsteps))) {
                status = 1;
            } else {
                if (tnew + dtnew > S.tend) dtnew = S.tend - tnew;
                if (A.adapt && dtnew < A.dt_min) status = -2;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = lane + 64 * q;
        if (i >= n) continue;
        double v = A.x[row + i];
        if (accept) {
            v = xn[q];
            A.x[row + i] = v;
        }
        A.fb[row + i] = A.expansion ? g_to_f(v, A.p[i], tnew) : v;
    }
    if (lane == 0 && running) {
        S.t = tnew;
        S.dt = dtnew;
        S.steps = steps;
        S.rejected = rej;
        S.status = status;
        S.outflow = outflow;
    }
}

template <typename PT>
hipError_t launch_epilogue(const PT *part, int nsplit, long split_stride, int ld_b,
                           const float *fscale, const float *rscale, const double *rate,
                           const double *f, const kxg_kernel &k, int B, int project, double *C,
                           double *diag, const StepArgs *step, hipStream_t s,
                           const double *ext = nullptr, double eta = 0.0)
{
    const int n = k.n;
    const dim3 grid((B + 3) / 4), blk(256);
    StepArgs sa{};
    if (step) sa = *step;
    else sa.mode = kStepNone;
#define KXG_EPI(P)                                                                             \
    hipLaunchKernelGGL((k_epilogue<PT, P>), grid, blk, 0, s, part, nsplit, split_stride, ld_b, \
                       fscale, rscale, rate, f, k.d_h, k.d_K, k.d_E, k.mass, n, B, project, C, \
                       diag, sa, ext, eta)
    if (n <= 64) KXG_EPI(1);
    else if (n <= 128) KXG_EPI(2);
    else if (n <= 256) KXG_EPI(4);
    else if (n <= 512) KXG_EPI(8);
    else KXG_EPI(16);
#undef KXG_EPI
    return hipGetLastError();
}

hipError_t launch_rate(const kxg_kernel &k, const double *f, int B, double *rate, hipStream_t s)
{
    const dim3 grid((B + kRateT - 1) / kRateT, (k.n + kRateT - 1) / kRateT);
    hipLaunchKernelGGL(k_rate, grid, dim3(256), 0, s, k.d_RT, f, k.n, B, rate);
    return hipGetLastError();
}

// Moments sum h f, sum h E f, -sum_{f>0} h f (ln f - 1); one workgroup per row.
__global__ __launch_bounds__(256) void k_moments(const double *__restrict__ f, int n,
                                                 const double *__restrict__ h,
                                                 const double *__restrict__ E,
                                                 double *__restrict__ out)
{
    __shared__ double lds[4 * 3];
    const int b = blockIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += 256) {
        const double x = f[(long)b * n + i];
        v[0] += h[i] * x;
        v[1] += h[i] * E[i] * x;
        if (x > 0.0) v[2] -= h[i] * x * (log(x) - 1.0);
    }
    block_sum<3>(v, lds);
    if (threadIdx.x == 0) {
        out[3 * b + 0] = v[0];
        out[3 * b + 1] = v[1];
        out[3 * b + 2] = v[2];
    }
}

int stream_splits(int n)
{
    const long n2 = (long)n * n;
    int s = div_up(2048, n);
    const int cap = (int)(n2 / 2048);           // keep chunks >= 2048 elements
    if (s > cap) s = cap;
    if (s < 1) s = 1;
    return s;
}

int gemm_bbw(int B) { return B <= 32 ? 1 : (B <= 64 ? 2 : 4); }

}  // namespace

// ---------------------------------------------------------------------------
kxg_status alloc_workspace(const kxg_kernel &k, int b_cap, Workspace &ws)
{
    const int n = k.n;
    const int bpad = div_up(b_cap, 128) * 128;
    size_t need = (size_t)stream_splits(n) * b_cap * n * sizeof(double);
    if (k.d_JL) need = (size_t)stream_splits(n) * b_cap * 4 * n * sizeof(double);
    if (k.d_G32 || k.d_Gbf || k.d_Gh) {
        const size_t g = (size_t)k.gemm_splits * bpad * k.geo.ipad * sizeof(float);
        if (g > need) need = g;
    }
    if ((k.d_Gbf || k.d_Gh) && b_cap >= kLdsMinB) {
        const size_t bl = (size_t)div_up(b_cap, 512) * 512;
        const size_t g = (size_t)k.lds_splits * bl * k.geo.ipad * sizeof(float);
        if (g > need) need = g;
    }
    need += (size_t)b_cap * n * sizeof(double);      // loss rates
    ws.part_bytes = need;
    ws.bpad_cap = bpad;
    ws.b_cap = b_cap;
    if (hipMalloc(&ws.part, need) != hipSuccess) { set_error("workspace: out of memory"); return KXG_ENOMEM; }
    const int bpad_l = div_up(b_cap, 512) * 512;
    const size_t fb = (size_t)k.geo.nb * (bpad_l > bpad ? bpad_l : bpad) * kBlk * sizeof(float);
    if (hipMalloc((void **)&ws.fop, fb) != hipSuccess || hipMalloc((void **)&ws.fpar, fb) != hipSuccess ||
        hipMalloc((void **)&ws.fscale, (bpad_l > bpad ? bpad_l : bpad) * sizeof(float)) != hipSuccess) {
        set_error("workspace: out of memory");
        return KXG_ENOMEM;
    }
    return KXG_OK;
}

void free_workspace(Workspace &ws)
{
    if (ws.part) (void)hipFree(ws.part);
    if (ws.fop) (void)hipFree(ws.fop);
    if (ws.fpar) (void)hipFree(ws.fpar);
    if (ws.fscale) (void)hipFree(ws.fscale);
    ws = Workspace{};
}

kxg_status eval_impl(const kxg_kernel &k, const Workspace &ws, int prec, const double *f,
                     int B, double *C, uint32_t flags, double *diag, hipStream_t s,
                     const StepArgs *step)
{
    const int n = k.n;
    const Geometry &g = k.geo;
    // the loss-rate buffer [b_cap][n] sits at the end of the workspace
    double *rate = reinterpret_cast<double *>(static_cast<char *>(ws.part) + ws.part_bytes) -
                   (size_t)ws.b_cap * n;
    // FP32 takes the stream kernel only on handles built for tiny batches, so
    // that on any one handle the path (and the rounding) of a row does not
    // depend on how many rows share the call.
    const bool exact = (flags & (KXG_INTERP_LOG | KXG_STAT_BOSE | KXG_STAT_FERMI)) != 0;
    if (exact) {
        const bool logi = (flags & KXG_INTERP_LOG) != 0;
        const bool quant = (flags & (KXG_STAT_BOSE | KXG_STAT_FERMI)) != 0;
        const double eta = (flags & KXG_STAT_BOSE) ? 1.0 : ((flags & KXG_STAT_FERMI) ? -1.0 : 0.0);
        const int ns = stream_splits(n);
        const long n2 = (long)n * n;
        const bool dbl = prec == KXG_F64;
        const int vec = (n % 2 == 0) ? 2 : 1;
        int chunk = div_up(n2, ns);
        chunk = div_up(chunk, 256 * vec) * (256 * vec);
        const int nsplit = (int)((n2 + chunk - 1) / chunk);
        constexpr int BT = 2;
        const dim3 grid(nsplit, n, div_up(B, BT));
        const size_t shm = 2 * n * sizeof(double) + 2 * (size_t)BT * n * (dbl ? sizeof(double) : sizeof(float));
        double *ext = static_cast<double *>(ws.part);
#define KXG_SX(T, V, L, Q)                                                                        \
    hipLaunchKernelGGL((k_stream_x<T, V, BT, L, Q>), grid, dim3(256), shm, s,                     \
                       reinterpret_cast<const T *>(dbl ? (const void *)k.d_A64 : (const void *)k.d_A32), \
                       k.d_JL, f, k.d_K, k.d_invdK, n, B, chunk, ext)
#define KXG_SX2(T, V)                                                                             \
    if (logi && quant) KXG_SX(T, V, true, true);                                                  \
    else if (logi) KXG_SX(T, V, true, false);                                                     \
    else KXG_SX(T, V, false, true)
        profile_mark_begin(s);
        if (dbl) {
            if (vec == 2) { KXG_SX2(double, 2); } else { KXG_SX2(double, 1); }
        } else {
            if (vec == 2) { KXG_SX2(float, 2); } else { KXG_SX2(float, 1); }
        }
#undef KXG_SX2
#undef KXG_SX
        profile_mark_end(s);
        KXG_TRY_HIP(hipGetLastError());
        KXG_TRY_HIP(launch_epilogue<double>(ext, nsplit, 0, 0, nullptr, nullptr, rate, f, k, B,
                                            (flags & KXG_PROJECT) ? 1 : 0, C, diag, step, s, ext,
                                            eta));
        return KXG_OK;
    }
    const bool use_stream = prec == KXG_F64 || (prec == KXG_F32 && B <= 4 && k.b_cap <= 4 && k.d_A32);
    const int project = (flags & KXG_PROJECT) ? 1 : 0;
    if (use_stream) {
        const int ns = stream_splits(n);
        const long n2 = (long)n * n;
        const bool dbl = prec == KXG_F64;
        const int vec = dbl ? ((n % 2 == 0) ? 2 : 1) : ((n % 4 == 0) ? 4 : ((n % 2 == 0) ? 2 : 1));
        int chunk = div_up(n2, ns);
        chunk = div_up(chunk, 256 * vec) * (256 * vec);
        const int nsplit = (int)((n2 + chunk - 1) / chunk);
        // distributions per pass: one for a single distribution (no idle
        // lanes of work), four otherwise
        const int BT = B == 1 ? 1 : (B == 2 ? 2 : 4);
        const dim3 grid(nsplit, n, div_up(B, BT));
        const size_t shm = (size_t)BT * n * (dbl ? sizeof(double) : sizeof(float));
        double *part = static_cast<double *>(ws.part);
        profile_mark_begin(s);
#define KXG_ST(T, V, BTV) \
    hipLaunchKernelGGL((k_stream<T, V, BTV>), grid, dim3(256), shm, s, \
                       reinterpret_cast<const T *>(dbl ? (const void *)k.d_A64 : (const void *)k.d_A32), f, n, B, chunk, part)
#define KXG_ST2(T, V) \
    if (BT == 1) KXG_ST(T, V, 1); else if (BT == 2) KXG_ST(T, V, 2); else KXG_ST(T, V, 4)
        if (dbl) {
            if (vec == 2) { KXG_ST2(double, 2); } else { KXG_ST2(double, 1); }
        } else {
            if (vec == 4) { KXG_ST2(float, 4); } else if (vec == 2) { KXG_ST2(float, 2); } else { KXG_ST2(float, 1); }
        }
#undef KXG_ST2
#undef KXG_ST
        profile_mark_end(s);
        KXG_TRY_HIP(hipGetLastError());
        KXG_TRY_HIP(launch_rate(k, f, B, rate, s));
        KXG_TRY_HIP(launch_epilogue<double>(part, nsplit, (long)B * n, n, nullptr, nullptr, rate,
                                            f, k, B, project, C, diag, step, s));
        return KXG_OK;
    }
    const bool f16 = prec == KXG_F16X3;
    if ((prec == KXG_BF16X3 || prec == KXG_F16X3) && B >= kLdsMinB) {
        // large batch: 16-bit GEMM with the A operand shared through LDS
        constexpr int BBW = KXG_LDS_BBW, IBW = KXG_LDS_IBW, TILE = 4 * BBW * 32;
        const int bpad = div_up(B, TILE) * TILE;
        const int nbt = bpad / TILE, nit = div_up(g.nib, IBW);
        const int splits = k.lds_splits;
        hipLaunchKernelGGL(k_prep, dim3(bpad), dim3(256), 0, s, f, B, n, g.nb, bpad, f16 ? 1 : 0,
                           ws.fop, ws.fpar, ws.fscale);
        float *part = static_cast<float *>(ws.part);
        profile_mark_begin(s);
        if (f16)
            hipLaunchKernelGGL((k_gemm_x3_lds<BBW, IBW, true>), dim3(nbt * nit * splits), dim3(256), 0, s,
                               k.d_Gh, ws.fop, k.d_pairs, g.npairs, g.nib, bpad, g.ipad, nbt, nit,
                               splits, g.dksteps, part);
        else
            hipLaunchKernelGGL((k_gemm_x3_lds<BBW, IBW, false>), dim3(nbt * nit * splits), dim3(256), 0, s,
                               k.d_Gbf, ws.fop, k.d_pairs, g.npairs, g.nib, bpad, g.ipad, nbt, nit,
                               splits, g.dksteps, part);
        profile_mark_end(s);
        KXG_TRY_HIP(hipGetLastError());
        KXG_TRY_HIP(launch_rate(k, f, B, rate, s));
        KXG_TRY_HIP(launch_epilogue<float>(part, splits, (long)bpad * g.ipad, g.ipad,
                                           f16 ? ws.fscale : nullptr, f16 ? k.d_hrow : nullptr, rate,
                                           f, k, B, project, C, diag, step, s));
        return KXG_OK;
    }
    // GEMM path
    const int bbw = gemm_bbw(B);
    const int tile = 32 * bbw;
    const int bpad = div_up(B, tile) * tile;
    const int nbt = bpad / tile;
    const int splits = k.gemm_splits;
    const int nwg = nbt * g.nib * splits;
    hipLaunchKernelGGL(k_prep, dim3(bpad), dim3(256), 0, s, f, B, n, g.nb, bpad, f16 ? 1 : 0,
                       ws.fop, ws.fpar, ws.fscale);
    float *part = static_cast<float *>(ws.part);
    profile_mark_begin(s);
#define KXG_GEMM_F32(W)                                                                  \
    hipLaunchKernelGGL(k_gemm_f32<W>, dim3(nwg), dim3(256), 0, s, k.d_G32, ws.fop, ws.fpar, \
                       k.d_pairs, g.npairs, bpad, g.ipad, nbt, splits, g.dksteps, part)
#define KXG_GEMM_X3(W, H, GP)                                                              \
    hipLaunchKernelGGL((k_gemm_x3<W, H>), dim3(nwg), dim3(256), 0, s, GP, ws.fop, k.d_pairs, \
                       g.npairs, bpad, g.ipad, nbt, splits, g.dksteps, part)
    if (prec == KXG_F32) {
        if (bbw == 1) KXG_GEMM_F32(1); else if (bbw == 2) KXG_GEMM_F32(2); else KXG_GEMM_F32(4);
    } else if (prec == KXG_BF16X3) {
        if (bbw == 1) KXG_GEMM_X3(1, false, k.d_Gbf);
        else if (bbw == 2) KXG_GEMM_X3(2, false, k.d_Gbf);
        else KXG_GEMM_X3(4, false, k.d_Gbf);
    } else {
        if (bbw == 1) KXG_GEMM_X3(1, true, k.d_Gh);
        else if (bbw == 2) KXG_GEMM_X3(2, true, k.d_Gh);
        else KXG_GEMM_X3(4, true, k.d_Gh);
    }
#undef KXG_GEMM_F32
#undef KXG_GEMM_X3
    profile_mark_end(s);
    KXG_TRY_HIP(hipGetLastError());
    KXG_TRY_HIP(launch_rate(k, f, B, rate, s));
    KXG_TRY_HIP(launch_epilogue<float>(part, splits, (long)bpad * g.ipad, g.ipad,
                                       f16 ? ws.fscale : nullptr, f16 ? k.d_hrow : nullptr, rate, f,
                                       k, B, project, C, diag, step, s));
    return KXG_OK;
}

hipError_t launch_moments(const kxg_kernel &k, const double *f, int B, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments, dim3(B), dim3(256), 0, s, f, k.n, k.d_h, k.d_E, out);
    return hipGetLastError();
}

}  // namespace kxg
