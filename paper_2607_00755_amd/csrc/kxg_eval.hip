// Evaluation of C[f] = gain - loss for a batch of distributions
// (Sec. 4.1 eq. discrete_collision_operator of arXiv 2607.00755, linear
// interpolation form), with the FP64 epilogue: split-K reduction, two-moment
// projection (App. C), diagnostics and the stepper's stage update.
//
// contraction paths (each yields gain - loss in its partials)
//   * stream: one pass over the dense tensor A[i][k][m] per group of up to
//     4 distributions, f staged in LDS, the loss row f_i sum_m R_im f_m added
//     by the first K split of each row; HBM-bound (single distribution).
//   * GEMM: C[b][i] = sum_K F2[b][K] A'[i][K] with K = (k,m) over the
//     block-packed (k <= m) tensor with the loss folded in
//     (A' = A - delta_ik R_im), F2[b][(k,m)] = f_bk f_bm formed in registers,
//     on the MFMA units (FP32 32x32x2 in kxg_gemm_f32.hip, or BF16/FP16
//     32x32x16 in kxg_gemm16.hip with a hi+lo split of A' and of F2:
//     hi*hi + hi*lo + lo*hi).  K is split over workgroups (and over the 4 waves of each);
//     partials are reduced in FP64 by the epilogue in a fixed order,
//     independent of the batch size.
//   * exact forms (log interpolation, quantum statistics): k_stream_x.
// The loss rates R f (k_rate) are computed only for the diagnostics.
#include "kxg_device.h"
#include "kxg_internal.h"
#include "kxg_step.h"

#include <algorithm>
#include <mutex>
#include <type_traits>

namespace kxg {
namespace {

inline int div_up(long a, long b) { return (int)((a + b - 1) / b); }

#ifndef KXG_STREAMX_VEC32
#define KXG_STREAMX_VEC32 2   // FP32 weights per load in the exact-form stream (2 or 4)
#endif
#ifndef KXG_STREAMX_UNROLL
#define KXG_STREAMX_UNROLL 4   // element groups in flight per thread in the exact-form stream
#endif
#ifndef KXG_EPI_WAVE_BCAP
#define KXG_EPI_WAVE_BCAP 2048   // handles from this b_cap get a wave per distribution in the epilogue
#endif
#ifndef KXG_EPI_U
#define KXG_EPI_U 32         // FP32 split partials in flight per thread in the epilogue
#endif
#ifndef KXG_EPI_MINB
#define KXG_EPI_MINB 1       // epilogue workgroups per CU the register budget must allow
#endif

// ---------------------------------------------------------------------------
// Plain evaluation over the packed operand (FP64, or FP32 on
// single-distribution handles): grid (split, i, group of BT distributions).
// Row i holds, for each kept (kb, mb) pair of its i-block, the 16 x 16 block
// of A'[i,k,m] + A'[i,m,k] (A' = A with the loss folded in, kb < mb) or of
// A'[i,k,m] (kb = mb), [dk][dm]; each workgroup reads `chunk` consecutive
// values of the row once (16-byte non-temporal loads of VEC values of one
// block row) and forms sum P f_k f_m for its BT distributions, f zero-padded
// to whole blocks in LDS; per-thread sums in T, the workgroup's reduction
// in FP64.  The (kb, mb) of the pairs its chunk spans are staged in LDS.
// Split s of a row shorter than s * chunk writes a zero partial, so every
// row has `gridDim.x` partials (gain minus loss) in split order.
template <typename T, int BT>
__global__ __launch_bounds__(256) void k_stream_p(const T *__restrict__ P,
                                                  const int *__restrict__ pairs,
                                                  const int *__restrict__ ib64,
                                                  const double *__restrict__ f, int n, int nbf, int B,
                                                  int chunk, double *__restrict__ part)
{
    extern __shared__ double smem_d[];
    T *fs = reinterpret_cast<T *>(smem_d);          // [BT][nbf]
    __shared__ int2 spair[kPStreamPairs];           // (16 kb, 16 mb)
    __shared__ double red[4][BT];
    constexpr int VEC = 16 / sizeof(T);
    typedef T vt __attribute__((ext_vector_type(VEC)));
    constexpr int UN = KXG_PSTREAM_UNROLL, STEP = 256 * VEC;
    const int split = blockIdx.x, i = blockIdx.y, b0 = blockIdx.z * BT;
    const int ib = i / kIBlk;
    const int first = ib64[2 * ib], cnt = ib64[2 * ib + 1];
    const long len = (long)cnt * 256;
    const long e_beg = (long)split * chunk;
    if (e_beg >= len) {
        if ((int)threadIdx.x < BT && b0 + (int)threadIdx.x < B)
            part[((long)split * B + b0 + threadIdx.x) * n + i] = 0.0;
        return;
    }
    const long e_end = e_beg + chunk < len ? e_beg + chunk : len;
    const T *row = P + ((long)first * kIBlk + (long)(i % kIBlk) * cnt) * 256;
    // the first UN loads of every thread go out before f and the pair
    // table are staged, so that their latencies overlap (a chunk is one
    // such round unless the host chose a longer one)
    auto load_round = [&](long e, vt (&a)[UN]) {
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const long eu = e + (long)u * STEP;
            a[u] = eu < e_end ? __builtin_nontemporal_load(reinterpret_cast<const vt *>(row + eu)) : vt{};
        }
    };
    long e = e_beg + VEC * (long)threadIdx.x;
    vt a[UN];
    load_round(e, a);
    const int c0 = (int)(e_beg >> 8), nc = (int)((e_end - 1) >> 8) - c0 + 1;
    for (int q = threadIdx.x; q < BT * nbf; q += 256) {
        const int bb = q / nbf, m = q - bb * nbf;
        fs[q] = (b0 + bb < B && m < n) ? (T)f[(long)(b0 + bb) * n + m] : (T)0;
    }
    for (int c = threadIdx.x; c < nc; c += 256)
        spair[c] = make_int2(pairs[2 * (first + c0 + c)] * kBlk, pairs[2 * (first + c0 + c) + 1] * kBlk);
    __syncthreads();
    T acc[BT];
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) acc[bb] = (T)0;
    while (e < e_end) {
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const long eu = e + (long)u * STEP;
            if (eu < e_end) {
                const int w = (int)(eu & 255);
                const int2 pr = spair[(int)(eu >> 8) - c0];
                const int kk = pr.x + (w >> 4), mm = pr.y + (w & 15);
#pragma unroll
                for (int bb = 0; bb < BT; ++bb) {
                    const T *fb = fs + bb * nbf;
                    T sv = (T)0;
#pragma unroll
                    for (int v = 0; v < VEC; ++v) sv += a[u][v] * fb[mm + v];
                    acc[bb] += fb[kk] * sv;
                }
            }
        }
        e += (long)UN * STEP;
        if (e < e_end) load_round(e, a);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int bb = 0; bb < BT; ++bb) {
        double v = (double)acc[bb];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][bb] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < BT && b0 + (int)threadIdx.x < B) {
        const int bb = threadIdx.x;
        part[((long)split * B + b0 + bb) * n + i] = ((red[0][bb] + red[1][bb]) + red[2][bb]) + red[3][bb];
    }
}

// e^x for the FP64 log interpolation, whose exponents lie in
// [ln 1e-300, ln f_max] (no overflow, no subnormal results, no special
// cases), by Tang's table-driven method (ACM TOMS 15, 1989): x = (32 m + j)
// ln2/32 + r with ln2/32 = L1 + L2 (L1 of 38 significant bits, so N L1 is
// exact for |N| < 2^15), |r| <= ln2/64; e^x = 2^m 2^(j/32) (1 + p(r)) with p
// the Taylor polynomial of e^r - 1 to degree 5 (truncation below 3e-15
// relative) and 2^(j/32) from a 32-entry table in LDS.  Relative error a few
// 1e-15 (the path's tolerance is 1e-10); a fifth of the kernel's time less
// than the library exp at n = 384.  FP32 keeps the library's expf (no gain).
__device__ inline double exp_interp(double x, const double *t32)
{
    const double nd = __builtin_rint(x * 46.16624130844683);           // 32 / ln 2
    double r = fma(-nd, 0.021660849392446835, x);                      // L1
    r = fma(-nd, 5.145609244655338e-14, r);                            // L2
    double p = 1.0 / 120.0;
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p *= r;                                                            // e^r - 1
    const int n = (int)nd;
    const double tj = t32[n & 31];
    return ldexp(fma(tj, p, tj), n >> 5);
}

__device__ inline float exp_interp(float x, const float *) { return expf(x); }

// ---------------------------------------------------------------------------
// Exact-form stream (eq. app_dense_collision with the statistical factor of
// eq. Lambda_quantum): one pass over the weights A[i,n,m] and the bracket
// table of the blocks that hold a weight (row i: its i-block's (kb, mb)
// blocks in both orders, [dk][dm]; the pairs' (kb, mb) staged in LDS);
// per (i, n, m) the fourth-momentum value f~ is interpolated with the
// energy-linear weights omega_R = (K~ - K_jL) / (K_jL+1 - K_jL), linearly in
// f or (LOGI) in ln max(f, 1e-300), and four sums are accumulated per
// distribution: gain = sum W f_n f_m, S0 = sum W f~, S1 = sum W f~ (f_n + f_m),
// T1 = sum W f~ f_n f_m (the last two only with quantum statistics).  The
// epilogue forms C = (1 + eta f_i)(gain + eta T1) - f_i (S0 + eta S1 + eta^2 T1).
// Grid (split, i, group of BT distributions); split s of a row shorter than
// s * chunk writes zero partials.
template <typename T, int BT, bool LOGI, bool QUANT>
__global__ __launch_bounds__(256) void k_stream_x(const T *__restrict__ A,
                                                  const uint16_t *__restrict__ JL,
                                                  const int *__restrict__ xpairs,
                                                  const int *__restrict__ xib,
                                                  const double *__restrict__ f,
                                                  const double *__restrict__ K,
                                                  const double *__restrict__ invdK, int n, int nbf, int B,
                                                  int chunk, double *__restrict__ part)
{
    // 16-byte weight loads in FP32 (four values), 16 in FP64 (two); the
    // brackets of the same values alongside
    constexpr int NA = QUANT ? 4 : 2, VEC = 16 / sizeof(T) < 4 ? 16 / sizeof(T) : KXG_STREAMX_VEC32;
    extern __shared__ double smem_d[];
    double *Ks = smem_d;                       // [nbf]
    double *iK = Ks + nbf;                     // [nbf]
    T *fs = reinterpret_cast<T *>(iK + nbf);   // [BT][nbf]
    T *ls = fs + BT * nbf;                     // [BT][nbf] ln max(f, floor) (LOGI)
    __shared__ double red[4][BT][NA];
    __shared__ T t32[32];                      // 2^(j/32) for the FP64 exponential
    __shared__ int2 spair[kPStreamPairs];      // (16 kb, 16 mb)
    const int split = blockIdx.x, i = blockIdx.y, b0 = blockIdx.z * BT;
    const int ib = i / kIBlk;
    const int first = xib[2 * ib], cnt = xib[2 * ib + 1];
    const long len = (long)cnt * 256;
    const long e_beg = (long)split * chunk;
    if (e_beg >= len) {
        if ((int)threadIdx.x < BT * 4 && b0 + (int)threadIdx.x / 4 < B)
            part[(((long)split * B + b0 + threadIdx.x / 4) * 4 + threadIdx.x % 4) * n + i] = 0.0;
        return;
    }
    const long e_end = e_beg + chunk < len ? e_beg + chunk : len;
    const int c0 = (int)(e_beg >> 8), nc = (int)((e_end - 1) >> 8) - c0 + 1;
    for (int q = threadIdx.x; q < nbf; q += 256) {
        Ks[q] = q < n ? K[q] : 0.0;
        iK[q] = q < n ? invdK[q] : 0.0;
    }
    if (LOGI && sizeof(T) == 8 && threadIdx.x < 32) t32[threadIdx.x] = (T)exp2((double)threadIdx.x / 32.0);
    for (int q = threadIdx.x; q < BT * nbf; q += 256) {
        const int bb = q / nbf, m = q - bb * nbf;
        const double v = (b0 + bb < B && m < n) ? f[(long)(b0 + bb) * n + m] : 0.0;
        fs[q] = (T)v;
        if (LOGI) ls[q] = (T)log(v > 1e-300 ? v : 1e-300);
    }
    for (int c = threadIdx.x; c < nc; c += 256)
        spair[c] = make_int2(xpairs[2 * (first + c0 + c)] * kBlk, xpairs[2 * (first + c0 + c) + 1] * kBlk);
    __syncthreads();
    const long roff = ((long)first * kIBlk + (long)(i % kIBlk) * cnt) * 256;
    const T *row = A + roff;
    const uint16_t *jrow = JL + roff;
    const double ki = Ks[i];
    T acc[BT][NA];
#pragma unroll
    for (int bb = 0; bb < BT; ++bb)
#pragma unroll
        for (int c = 0; c < NA; ++c) acc[bb][c] = (T)0;
    typedef T vec_t __attribute__((ext_vector_type(VEC)));
    typedef uint16_t jvec_t __attribute__((ext_vector_type(VEC)));
    // one element group (VEC weights of block row k, columns m .. m + VEC - 1)
    auto body = [&](const vec_t &a, const jvec_t &jv, int kq, int mq) {
        const double kk = Ks[kq];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int mv = mq + v;
            const int jl = jv[v];
            if (jl == 0xFFFF) continue;
            const double kt = (kk + Ks[mv]) - ki;
            const T wr = (T)((kt - Ks[jl]) * iK[jl]);
            const T wl = (T)1 - wr;
            const T w = a[v];
#pragma unroll
            for (int bb = 0; bb < BT; ++bb) {
                const T *fb = fs + bb * nbf;
                const T fn = fb[kq], fm = fb[mv];
                T ft;
                if (LOGI) {
                    const T *lb = ls + bb * nbf;
                    ft = exp_interp(wl * lb[jl] + wr * lb[jl + 1], t32);
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
    };
    // KXG_STREAMX_UNROLL groups of loads in flight per thread (weights and
    // brackets), non-temporal: both tables are read once per call
    constexpr int UN = KXG_STREAMX_UNROLL, STEP = 256 * VEC;
    for (long e = e_beg + (long)threadIdx.x * VEC; e < e_end; e += (long)UN * STEP) {
        vec_t a[UN];
        jvec_t jv[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const long eu = e + (long)u * STEP;
            const bool in = eu < e_end;
            a[u] = in ? __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(row + eu)) : vec_t{};
            jv[u] = in ? __builtin_nontemporal_load(reinterpret_cast<const jvec_t *>(jrow + eu))
                       : jvec_t(0xFFFF);
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const long eu = e + (long)u * STEP;
            const int w = (int)(eu & 255);
            const int2 pr = spair[eu < e_end ? (int)(eu >> 8) - c0 : 0];
            body(a[u], jv[u], pr.x + (w >> 4), pr.y + (w & 15));
        }
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

// ---------------------------------------------------------------------------
// Loss rates rate[b][i] = sum_j R[i][j] f_bj in FP64 on v_mfma_f64_16x16x4f64.
// One 16 (b) x 16 (i) output tile per call by a whole workgroup: its 4 waves
// take 4 consecutive j ranges (all loads of a wave in flight at once at
// n = 256) and their accumulators are added in the fixed order 0+1+2+3, so a
// row's rates do not depend on B.  Operand/result layout of the
// instruction: A[row][k] at lane row + 16k, B[k][col] at lane col + 16k,
// D[row][col] at lane col + 16 (row % 4), register row / 4.
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int kRateT = 16;
struct RateArgs {
    const double *RT;     // R transposed [n][n]
    const double *f;      // [B][n]
    int n, B;
    double *rate;         // [B][n]
    int tiles_b;          // ceil(B / 16)
};
// `red`: 3*4*64 doubles of LDS; ends with a barrier, so the caller may reuse it.
__device__ void rate_tile(const RateArgs &ra, int tile, double *red)
{
    const int n = ra.n, B = ra.B;
    const int b0 = (tile % ra.tiles_b) * kRateT, i0 = (tile / ra.tiles_b) * kRateT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int nsteps = (n + 3) / 4;                         // K steps of 4
    const int per = (nsteps + 3) / 4;
    const int s0 = wave * per, s1 = min(nsteps, s0 + per);
    const int b = b0 + lr, i = i0 + lr;
    const double *frow = ra.f + (long)(b < B ? b : 0) * n;
    const double *RT = ra.RT;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
    int st = s0;
    for (; st + 16 <= s1; st += 16) {
        double av[16], bv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int j = 4 * (st + u) + lk;
            av[u] = (b < B && j < n) ? frow[j] : 0.0;
            bv[u] = (i < n && j < n) ? RT[(long)j * n + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
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
        for (int r = 0; r < 4; ++r) red[((wave - 1) * 4 + r) * 64 + lane] = acc[r];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double v = ((acc[r] + red[(0 * 4 + r) * 64 + lane]) + red[(1 * 4 + r) * 64 + lane]) +
                             red[(2 * 4 + r) * 64 + lane];
            const int bo = b0 + lk + 4 * r, io = i0 + lr;
            if (bo < B && io < n) ra.rate[(long)bo * n + io] = v;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_rate(RateArgs ra)
{
    __shared__ double red[3 * 4 * 64];
    rate_tile(ra, blockIdx.x, red);
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

template <int NV>
__device__ void block_max(double (&v)[NV], double *lds)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_max(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) lds[wave * NV + j] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j)
        v[j] = fmax(fmax(fmax(lds[j], lds[NV + j]), lds[2 * NV + j]), lds[3 * NV + j]);
    __syncthreads();
}

// Reductions over the threads of one distribution in the epilogue: a wave
// (TPB = 64) or the whole workgroup (TPB = 256, through `lds`).
template <int NV, int TPB>
__device__ void grp_sum(double (&v)[NV], double *lds)
{
    if constexpr (TPB == 64) {
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    } else {
        block_sum<NV>(v, lds);
    }
}

template <int NV, int TPB>
__device__ void grp_max(double (&v)[NV], double *lds)
{
    if constexpr (TPB == 64) {
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = wave_max(v[j]);
    } else {
        block_max<NV>(v, lds);
    }
}

template <int TPB>
__device__ inline int epi_tl() { return (int)threadIdx.x % TPB; }

// Stepper inputs of one slot, loaded at the start of the epilogue so that
// their latency overlaps that of the split partials.
// K slots of i-block ib (wave-uniform) from the packed counts; 0 past 32.
// The words pass through readfirstlane so that the selection stays among
// scalar registers (an indexed load of the argument block would be a
// memory access the partial loads must wait behind).
__device__ inline int slot_count(const SlotCounts &c, int ib)
{
    const int j = ib >> 2;
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const uint32_t l = __builtin_amdgcn_readfirstlane((uint32_t)c.w[t]);
        const uint32_t h = __builtin_amdgcn_readfirstlane((uint32_t)(c.w[t] >> 32));
        lo = j == t ? l : lo;
        hi = j == t ? h : hi;
    }
    const uint64_t w = ((uint64_t)hi << 32) | lo;
    return ib < 32 ? (int)((w >> (16 * (ib & 3))) & 0xFFFF) : 0;
}

template <int PER>
struct StepIn {
    double x[PER], acc[PER], xs[PER], nx[PER];
    double lam, hi, dt, t;      // the slot's control values (stepper modes only)
    int status, phase;
};

template <int PER, int TPB>
__device__ void load_step_inputs(const StepArgs &A, int b, int n, StepIn<PER> &in)
{
    const long row = (long)b * n;
    if (A.mode != kStepNone) {
        const SlotDev &S = A.sl[b];
        in.lam = S.lam;
        in.hi = S.hi_scale;
        in.dt = S.dt;
        in.t = S.t;
        in.status = S.status;
        in.phase = S.phase;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        in.x[q] = in.acc[q] = in.xs[q] = in.nx[q] = 0.0;
        if (i >= n) continue;
        if (A.mode == kStepRK4) {
            in.x[q] = A.x[row + i];
            if (A.stage > 1) in.acc[q] = A.acc[row + i];
        } else if (A.mode == kStepHeunPred) {
            in.x[q] = A.x[row + i];
            in.nx[q] = (i + 1 < n) ? A.x[row + i + 1] : 0.0;
        } else if (A.mode == kStepHeunCorr) {
            in.xs[q] = A.xs[row + i];
            in.nx[q] = (i + 1 < n) ? A.xs[row + i + 1] : 0.0;
            in.x[q] = A.x[row + i];
            in.acc[q] = A.acc[row + i];
        }
    }
}

// Grid quantities and operator input of one distribution as the epilogue
// holds them (element i = t + TPB q), and its loss rates R f (or null).
template <int PER>
struct EpiRow {
    const double (&h)[PER], (&e)[PER], (&f)[PER];
    const double *rate;
};

template <int PER, int TPB>
__device__ void step_update(const StepArgs &A, int b, int n, const double (&out)[PER],
                            const StepIn<PER> &in, double *lds, const EpiRow<PER> &row);

// FP64 epilogue, TPB threads per distribution (a wave, or the whole 256-thread
// workgroup), PER grid points per thread (element i = t + TPB q), App. C:
//   gain = sum of the split partials (fixed order; FP16 scales undone),
//   C_raw = gain - f * rate,
//   xi_i = |f_i|/f_max above 1e-12, and the 2x2 system for the correction
//   xi (alpha' + beta' K) written in kinetic energy K = E - m (the span of
//   {xi, xi E} equals that of {xi, xi K}; alpha = alpha' - beta' m,
//   beta = beta' in the paper's E-form), C_proj = C_raw - xi (alpha' + beta' K),
//   and the diagnostics of eqs. app_epsilon_definition and
//   app_projection_relative_correction.
// All loads of a thread (partials, rates, stepper state) are issued before
// the first reduction; the reductions add in a fixed order, so the result
// of a distribution does not depend on B.
template <typename PT, int PER, bool EXT, int TPB>
__global__ __launch_bounds__(256, KXG_EPI_MINB) void k_epilogue(
    const PT *__restrict__ part, int nsplit, SlotCounts nsc, long split_stride, int ld_b,
    const float *__restrict__ fscale, const float *__restrict__ rscale,
    const double *__restrict__ rate, const double *__restrict__ f,
    const double *__restrict__ h, const double *__restrict__ K, const double *__restrict__ E,
    double mass, int n, int B, int project, double *__restrict__ C, double *__restrict__ diag,
    StepArgs step, const double *__restrict__ ext, double eta, int folded)
{
    __shared__ double red[4 * 12];
    // one distribution per workgroup (TPB = 256) or per wave (TPB = 64)
    const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * (256 / TPB) + (int)threadIdx.x / TPB);
    if constexpr (TPB == 64) {
        if (b >= B) return;                    // whole wave; no barriers with TPB = 64
    }
    const double *fb = f + (long)b * n;
    StepIn<PER> in;
    load_step_inputs<PER, TPB>(step, b, n, in);
    // Every load of a thread (grid constants, f, the split partials below)
    // is issued before the first of them is used: rows past n read row 0
    // and drop the value, so no load sits behind a branch and a wait.
    double hv[PER], kv[PER], ev[PER], fv[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        const int ic = i < n ? i : 0;
        const double hx = h[ic], kx = K[ic], ex = E[ic], fx = fb[ic];
        hv[q] = i < n ? hx : 0.0;
        kv[q] = i < n ? kx : 0.0;
        ev[q] = i < n ? ex : 0.0;
        fv[q] = i < n ? fx : 0.0;
    }
    double craw[PER], xi[PER];
    double mx[4] = {0.0, 0.0, 0.0, 0.0};      // f_max, largest rate, largest |gain|, input flag
    double g[PER] = {};
    if constexpr (!EXT) {
        // split partials: up to 32 (FP32) or 16 (FP64) loads per thread in
        // flight over all its grid points, each row's added in split order.
        // With `folded` the partials already hold gain - loss (the loss term
        // is part of the GEMM operand) and the loss rates, when given, only
        // feed the diagnostics.
        // Slots up to nsplit (the largest count) are read for every row,
        // unconditionally: past the row's own count its last slot again (a
        // cache hit, no memory traffic), dropped in the sum.
        constexpr int U = (sizeof(PT) == 4 ? KXG_EPI_U : 16) / PER > 0 ? (sizeof(PT) == 4 ? KXG_EPI_U : 16) / PER : 1;
        int ns[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = epi_tl<TPB>() + TPB * q;
            // K slots of this row: the 64 rows of a wave span the i-block of
            // its first row and the next one
            int nq = nsplit;
            if (nsc.per_block) {
                const int ib0 = __builtin_amdgcn_readfirstlane((epi_tl<TPB>() + TPB * q) / kIBlk);
                const int c0 = __builtin_amdgcn_readfirstlane(slot_count(nsc, ib0));
                const int c1 = __builtin_amdgcn_readfirstlane(slot_count(nsc, ib0 + 1));
                nq = i / kIBlk == ib0 ? c0 : c1;
            }
            ns[q] = i < n ? nq : 0;
        }
        for (int sp0 = 0; sp0 < nsplit; sp0 += U) {
            PT v[PER][U];
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int i = epi_tl<TPB>() + TPB * q;
                const PT *pp = part + (long)b * ld_b + (i < n ? i : 0);
                const int last = ns[q] > 0 ? ns[q] - 1 : 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int sp = sp0 + u < last ? sp0 + u : last;   // no branch
                    v[q][u] = pp[(long)sp * split_stride];
                }
            }
            // the row counts are used only below, so that no wait for them
            // is placed ahead of the loads
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < PER; ++q)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (sp0 + u < ns[q]) g[q] += (double)v[q][u];
        }
    }
    double inv_s2 = 1.0;
    if (fscale) {
        const double sc = fscale[b];
        inv_s2 = 1.0 / (sc * sc);
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        craw[q] = 0.0;
        if (i < n) {
            const double x = fv[q];
            if (!isfinite(x)) mx[3] = fmax(mx[3], 1.0);
            else if (x < 0.0) mx[3] = fmax(mx[3], 0.5);
            mx[0] = fmax(mx[0], fabs(x));
            if constexpr (EXT) {
                // exact form: four split sums per row, layout [split][B][4][n]
                double a4[4] = {0.0, 0.0, 0.0, 0.0};
                for (int sp0 = 0; sp0 < nsplit; sp0 += 4) {
                    double v[4][4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            v[u][c] = (sp0 + u < nsplit)
                                          ? ext[(((long)(sp0 + u) * B + b) * 4 + c) * n + i] : 0.0;
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int c = 0; c < 4; ++c) a4[c] += v[u][c];
                }
                const double gq = (1.0 + eta * x) * (a4[0] + eta * a4[3]);
                const double lq = x * (a4[1] + eta * a4[2] + eta * eta * a4[3]);
                mx[1] = fmax(mx[1], a4[1]);
                mx[2] = fmax(mx[2], fabs(gq));
                craw[q] = gq - lq;
            }
        }
    }
    if constexpr (!EXT) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = epi_tl<TPB>() + TPB * q;
            if (i >= n) continue;
            double gq = g[q];
            if (fscale) gq *= inv_s2 / (double)rscale[i];
            const double rt = rate ? rate[(long)b * n + i] : 0.0;
            const double x = fv[q];
            mx[1] = fmax(mx[1], rt);
            if (folded) {
                mx[2] = fmax(mx[2], fabs(gq + x * rt));
                craw[q] = gq;
            } else {
                mx[2] = fmax(mx[2], fabs(gq));
                craw[q] = gq - x * rt;
            }
        }
    }
    // without diagnostics only f_max and the five projection sums are
    // reduced (the reductions of single values are the same either way)
    const bool lean = diag == nullptr;
    if (lean) {
        double m1[1] = {mx[0]};
        grp_max<1, TPB>(m1, red);
        mx[0] = m1[0];
    } else {
        grp_max<4, TPB>(mx, red);
    }
    const double fmaxv = mx[0];
    // s0, s1, b00, b01, b11, sum h|C|, sum hE|C|, sum hEC, number
    double sm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        xi[q] = 0.0;
        if (i < n) {
            const double hi = hv[q], ki = kv[q], ei = ev[q];
            const double r = fmaxv > 0.0 ? fabs(fv[q]) / fmaxv : 0.0;
            xi[q] = r > 1e-12 ? r : 0.0;
            sm[0] += hi * craw[q];
            sm[1] += hi * ki * craw[q];
            sm[2] += hi * xi[q];
            sm[3] += hi * ki * xi[q];
            sm[4] += hi * ki * ki * xi[q];
            sm[5] += hi * fabs(craw[q]);
            sm[6] += hi * ei * fabs(craw[q]);
            sm[7] += hi * ei * craw[q];
            sm[8] += hi * fv[q];
        }
    }
    if (lean) {
        double s5[5] = {sm[0], sm[1], sm[2], sm[3], sm[4]};
        grp_sum<5, TPB>(s5, red);
#pragma unroll
        for (int j = 0; j < 5; ++j) sm[j] = s5[j];
    } else {
        grp_sum<9, TPB>(sm, red);
    }
    const double s0 = sm[0], s1 = sm[1], b00 = sm[2], b01 = sm[3], b11 = sm[4];
    const double an = sm[5], ae = sm[6], se = sm[7], num = sm[8];
    double al = 0.0, be = 0.0;
    const double det = b00 * b11 - b01 * b01;
    if (project && det != 0.0 && isfinite(det)) {
        al = (s0 * b11 - s1 * b01) / det;
        be = (s1 * b00 - s0 * b01) / det;
    }
    double tt[6] = {0, 0, 0, 0, 0, 0};
    double bad[1] = {0.0};
    double out[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        out[q] = 0.0;
        if (i < n) {
            const double hi = hv[q], ei = ev[q];
            const double cp = craw[q] - xi[q] * (al + be * kv[q]);
            const double d = fabs(cp - craw[q]);
            tt[0] += hi * cp;
            tt[1] += hi * ei * cp;
            tt[2] += hi * fabs(cp);
            tt[3] += hi * ei * fabs(cp);
            tt[4] += hi * d;
            tt[5] += hi * ei * d;
            out[q] = project ? cp : craw[q];
            if (!isfinite(out[q])) bad[0] = 1.0;
        }
    }
    if (step.mode != kStepNone) {
        const EpiRow<PER> er{hv, ev, fv, rate ? rate + (long)b * n : nullptr};
        step_update<PER, TPB>(step, b, n, out, in, red, er);
        return;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        if (i < n) C[(long)b * n + i] = out[q];
    }
    if (diag) {
        grp_sum<6, TPB>(tt, red);
        grp_max<1, TPB>(bad, red);
        if (epi_tl<TPB>() == 0) {
            double *d = diag + (long)b * KXG_NDIAG;
            d[0] = al - be * mass;
            d[1] = be;
            d[2] = an > 0.0 ? s0 / an : 0.0;
            d[3] = ae > 0.0 ? se / ae : 0.0;
            d[4] = tt[2] > 0.0 ? tt[0] / tt[2] : 0.0;
            d[5] = tt[3] > 0.0 ? tt[1] / tt[3] : 0.0;
            d[6] = an > 0.0 ? tt[4] / an : 0.0;
            d[7] = ae > 0.0 ? tt[5] / ae : 0.0;
            d[8] = mx[1];
            d[9] = mx[2];
            double st = 0.0;
            if (mx[3] >= 1.0) st += 1.0;
            else if (mx[3] > 0.0) st += 2.0;
            if (bad[0] > 0.0) st += 4.0;
            d[10] = st;
            d[11] = num;
        }
    }
}


// GEMM operand of the next operator call from the new f of slot b (element
// i = thread + 256 q), in the layouts and with the FP16 scaling of k_prep;
// the padding (grid points n.. and rows beyond the batch) keeps the zeros
// written by k_prep at the start of the run.
template <int PER, int TPB>
__device__ void write_operand(const StepArgs &A, int b, int n, const double (&nf)[PER],
                              double *lds)
{
    float sc = 1.0f;
    if (A.scale16) {
        double m[1] = {0.0};
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if ((int)epi_tl<TPB>() + TPB * q < n) m[0] = fmax(m[0], fabs(nf[q]));
        grp_max<1, TPB>(m, lds);
        if (m[0] > 0.0 && isfinite(m[0])) sc = (float)ldexp(1.0, 7 - (int)ceil(log2(m[0])));
        if (epi_tl<TPB>() == 0) A.fscale[b] = sc;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        if (i >= n) continue;
        const float x = (float)nf[q] * sc;
        const int blk = i / kBlk, d = i % kBlk;
        A.fop[((long)blk * A.bpad + b) * kBlk + d] = x;
        A.fpar[(((long)blk * A.bpad + b) * 2 + (d & 1)) * 8 + (d >> 1)] = x;
    }
}

// Values at element i + 1 of a distribution held as element i = t + TPB q
// (0 beyond n): from the next lane within a wave (lane 0 of the next q for
// the last lane), through LDS across the four waves of a workgroup.
template <int PER, int TPB>
__device__ void next_elems(const double (&v)[PER], double (&nx)[PER], int n)
{
    if constexpr (TPB == 64) {
        const int lane = (int)threadIdx.x & 63;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const double a = __shfl(v[q], (lane + 1) & 63);
            const double c = __shfl(v[q + 1 < PER ? q + 1 : q], 0);
            nx[q] = lane < 63 ? a : (q + 1 < PER ? c : 0.0);
            if (lane + 64 * q + 1 >= n) nx[q] = 0.0;
        }
    } else {
        __shared__ double xch[PER * TPB];
        __syncthreads();                       // earlier readers of xch are done
#pragma unroll
        for (int q = 0; q < PER; ++q) xch[threadIdx.x + TPB * q] = v[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = threadIdx.x + TPB * q;
            nx[q] = i + 1 < n ? xch[i + 1] : 0.0;
        }
    }
}

// One classical RK4 step of size du in u of the source-only regime of a
// freeze-in slot (Sec. 4.2: elastic operator off, drift and sources only),
// x -> xn; returns (on every thread) the step's outflow through p_min with
// the RK4 weights of the stage states' g_0, and a non-finite flag.
template <int PER, int TPB>
__device__ void source_rk4(const StepArgs &A, const SlotDev &S, int n, const StepIn<PER> &in,
                           const EpiRow<PER> &row, double u, double du, double (&xn)[PER],
                           double (&flow_bad)[2], double *lds)
{
    double y[PER], nx[PER], acc[PER];
    double o = 0.0;
    auto rhs = [&](const double (&st)[PER], const double (&nxt)[PER], double uu, int q) {
        const int i = epi_tl<TPB>() + TPB * q;
        const double src = freeze_in_source(S, i, A.p[i], row.e[q], A.mass, uu);
        return rhs_u(1, st[q], nxt[q], 0.0, A.p[i], A.dp[i], in.lam, in.hi, uu, src);
    };
    // stage 1 from the state and its stored neighbours
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        y[q] = in.x[q];
        nx[q] = in.nx[q];
    }
    o = y[0];
    const double cst[3] = {0.5, 0.5, 1.0}, wst[3] = {2.0, 2.0, 1.0};
    double k[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        k[q] = i < n ? rhs(y, nx, u, q) : 0.0;
        acc[q] = k[q];
    }
    for (int st = 0; st < 3; ++st) {
#pragma unroll
        for (int q = 0; q < PER; ++q) y[q] = in.x[q] + cst[st] * du * k[q];
        next_elems<PER, TPB>(y, nx, n);
        o += wst[st] * y[0];
        const double us = u + cst[st] * du;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = epi_tl<TPB>() + TPB * q;
            k[q] = i < n ? rhs(y, nx, us, q) : 0.0;
            acc[q] += wst[st] * k[q];
        }
    }
    double bad[1] = {0.0};
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        xn[q] = i < n ? in.x[q] + du / 6.0 * acc[q] : 0.0;
        if (i < n && !isfinite(xn[q])) bad[0] = 1.0;
    }
    grp_max<1, TPB>(bad, lds);
    flow_bad[0] = du / 6.0 * o;                // meaningful on the thread holding i = 0
    flow_bad[1] = bad[0];
}

// Stepper update of slot b from the operator output `out` (element
// i = thread + 256 q), Sec. 4.2: RK4 stage, or Heun predictor
// x* = x + dt k1, or Heun corrector x_new = x + dt (k1 + k2)/2 with the
// predictor-corrector error err = max |x_new - x*| / (atol + rtol
// max(|x|, |x_new|)), acceptance err <= 1 (always in replay mode) and
// dt *= clamp(safety err^-1/2, fac_lo, fac_hi), clipped to end at t_end.
// Every thread reaches the same decision (block reductions); thread 0
// writes the slot record.
template <int PER, int TPB>
__device__ void step_update(const StepArgs &A, int b, int n, const double (&out)[PER],
                            const StepIn<PER> &in, double *lds, const EpiRow<PER> &er)
{
    SlotDev &S = A.sl[b];
    const int running = in.status == 0;
    const long row = (long)b * n;
    const double u = in.t;
    double dt = in.dt;
    double nf[PER];                            // the next operator input
    if (A.mode == kStepRK4) {
        const double lam = in.lam / in.hi;
        double bad[1] = {0.0};
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = epi_tl<TPB>() + TPB * q;
            nf[q] = 0.0;
            if (i >= n) continue;
            const double xv = in.x[q];
            double v = xv;
            if (running) {
                const double k = lam * out[q];
                if (A.stage == 1) { A.acc[row + i] = k; v = xv + 0.5 * dt * k; }
                else if (A.stage == 2) { A.acc[row + i] = in.acc[q] + 2.0 * k; v = xv + 0.5 * dt * k; }
                else if (A.stage == 3) { A.acc[row + i] = in.acc[q] + 2.0 * k; v = xv + dt * k; }
                else {
                    v = xv + dt / 6.0 * (in.acc[q] + k);
                    A.x[row + i] = v;
                    if (!isfinite(v)) bad[0] = 1.0;
                }
            }
            A.fb[row + i] = v;
            nf[q] = v;
        }
        if (A.write_op) write_operand<PER, TPB>(A, b, n, nf, lds);
        if (A.stage == 4) {
            grp_max<1, TPB>(bad, lds);
            if (epi_tl<TPB>() == 0 && running) {
                S.t = u + dt;
                S.steps += 1;
                if (bad[0] > 0.0) S.status = -1;
                else if (S.t >= S.tend * (1.0 - 1e-14)) S.status = 1;
                else if (S.maxsteps > 0 && S.steps >= S.maxsteps) S.status = 2;
                else if (S.t + dt > S.tend) S.dt = S.tend - S.t;
            }
        }
        return;
    }
    if (A.mode == kStepHeunPred) {
        if (A.freeze_in && running && in.phase == 0) {
            // Source-only regime: test Gamma_22 / H of the current state
            // (Gamma_22 = lambda sum h f (R f) / sum h f); over eps_switch the
            // elastic operator comes on and this attempt is the first Heun
            // predictor, otherwise one RK4 step of drift and sources.
            double r2[2] = {0.0, 0.0};
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int i = epi_tl<TPB>() + TPB * q;
                if (i >= n) continue;
                r2[0] += er.h[q] * er.f[q] * er.rate[i];
                r2[1] += er.h[q] * er.f[q];
            }
            grp_sum<2, TPB>(r2, lds);
            const double g22 = r2[1] > 0.0 ? in.lam * r2[0] / r2[1] : 0.0;
            if (g22 / (in.hi * exp(-2.0 * u)) > S.eps_switch) {
                double mx[1] = {0.0};
#pragma unroll
                for (int q = 0; q < PER; ++q)
                    if (epi_tl<TPB>() + TPB * q < n) mx[0] = fmax(mx[0], fabs(in.x[q]));
                grp_max<1, TPB>(mx, lds);
                if (A.adapt && u + dt > S.tend) dt = S.tend - u;
                if (epi_tl<TPB>() == 0) {
                    const double at = A.atol_rel * mx[0];
                    S.phase = 1;
                    S.u_switch = u;
                    S.atol = at > 0.0 ? at : 1e-300;
                    S.dt = dt;
                }
            } else {
                const double du = u + S.du_src > S.tend ? S.tend - u : S.du_src;
                double xn[PER], fb2[2];
                source_rk4<PER, TPB>(A, S, n, in, er, u, du, xn, fb2, lds);
                const double un = u + du;
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int i = epi_tl<TPB>() + TPB * q;
                    nf[q] = 0.0;
                    if (i >= n) continue;
                    A.x[row + i] = xn[q];
                    A.xs[row + i] = xn[q];
                    nf[q] = g_to_f(xn[q], A.p[i], un);
                    A.fb[row + i] = nf[q];
                }
                if (A.write_op) write_operand<PER, TPB>(A, b, n, nf, lds);
                if (epi_tl<TPB>() == 0) {
                    S.t = un;
                    S.steps += 1;
                    S.nsrc += 1;
                    S.outflow += fb2[0];
                    if (fb2[1] > 0.0) S.status = -1;
                    else if (un >= S.tend * (1.0 - 1e-14)) S.status = 1;
                    else if (S.maxsteps > 0 && S.steps >= S.maxsteps) S.status = 2;
                }
                return;
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = epi_tl<TPB>() + TPB * q;
            nf[q] = 0.0;
            if (i >= n) continue;
            const double xv = in.x[q];
            if (!running) {
                // f of a stopped slot is left as it is (f of x at its last t)
                A.xs[row + i] = xv;
                nf[q] = A.expansion ? g_to_f(xv, A.p[i], u) : xv;
                continue;
            }
            const double src = A.freeze_in ? freeze_in_source(S, i, A.p[i], er.e[q], A.mass, u) : 0.0;
            const double k = rhs_u(A.expansion, xv, in.nx[q], out[q], A.p[i], A.dp[i], in.lam, in.hi, u, src);
            A.acc[row + i] = k;
            const double v = xv + dt * k;
            A.xs[row + i] = v;
            nf[q] = A.expansion ? g_to_f(v, A.p[i], u + dt) : v;
            A.fb[row + i] = nf[q];
        }
        if (A.write_op) write_operand<PER, TPB>(A, b, n, nf, lds);
        return;
    }
    // Heun corrector and control (a freeze-in slot still in the source-only
    // regime took its step in the predictor's epilogue and is left alone)
    const int heun = running && !(A.freeze_in && in.phase == 0);
    double xn[PER];
    double ev[2] = {0.0, 0.0};              // err, non-finite flag
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        xn[q] = 0.0;
        if (i >= n || !heun) continue;
        const double xsv = in.xs[q];
        const double src = A.freeze_in ? freeze_in_source(S, i, A.p[i], er.e[q], A.mass, u + dt) : 0.0;
        const double k2 = rhs_u(A.expansion, xsv, in.nx[q], out[q], A.p[i], A.dp[i], in.lam, in.hi, u + dt, src);
        const double x0 = in.x[q];
        const double v = x0 + 0.5 * dt * (in.acc[q] + k2);
        xn[q] = v;
        const double sc = S.atol + A.rtol * fmax(fabs(x0), fabs(v));
        const double e = fabs(v - xsv) / sc;
        if (!isfinite(v)) ev[1] = 1.0;
        ev[0] = fmax(ev[0], isfinite(e) ? e : 1e300);
    }
    grp_max<2, TPB>(ev, lds);
    const double err = ev[0], nonfin = ev[1];
    int accept = 0, status = S.status, steps = S.steps, rej = S.rejected;
    double tnew = u, dtnew = dt, outflow = S.outflow;
    if (heun) {
        if (nonfin > 0.0) {
            status = -1;
        } else {
            accept = (!A.adapt) || err <= 1.0;
            if (accept) {
                // g_0 of the state and of the predictor, held by thread 0
                if (A.expansion) outflow += 0.5 * dt * (in.x[0] + in.xs[0]);
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
            if (accept && tnew >= S.tend * (1.0 - 1e-14)) {
                status = 1;
            } else if (accept && S.maxsteps > 0 && steps >= S.maxsteps) {
                status = 2;                         // step cap before t_end
            } else {
                if (tnew + dtnew > S.tend) dtnew = S.tend - tnew;
                if (A.adapt && dtnew < A.dt_min) status = -2;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = epi_tl<TPB>() + TPB * q;
        nf[q] = 0.0;
        if (i >= n) continue;
        double v = in.x[q];
        if (accept) {
            v = xn[q];
            A.x[row + i] = v;
        }
        nf[q] = A.expansion ? g_to_f(v, A.p[i], tnew) : v;
        A.fb[row + i] = nf[q];
    }
    if (A.write_op) write_operand<PER, TPB>(A, b, n, nf, lds);
    if (epi_tl<TPB>() == 0 && heun) {
        S.t = tnew;
        S.dt = dtnew;
        S.steps = steps;
        S.rejected = rej;
        S.status = status;
        S.outflow = outflow;
    }
}

template <typename PT>
hipError_t launch_epilogue(const PT *part, int nsplit, const SlotCounts &nsc, long split_stride, int ld_b,
                           const float *fscale, const float *rscale, const double *rate,
                           const double *f, const kxg_kernel &k, int B, int project, double *C,
                           double *diag, const StepArgs *step, hipStream_t s,
                           const double *ext = nullptr, double eta = 0.0, int folded = 0)
{
    const int n = k.n;
    // threads per distribution: a wave for handles built for large batches
    // (more distributions in flight), else the whole workgroup; fixed per
    // handle, so a row's reduction order does not depend on B
    const int tpb = k.b_cap >= KXG_EPI_WAVE_BCAP ? 64 : 256;
    const dim3 grid(tpb == 64 ? (B + 3) / 4 : B), blk(256);
    StepArgs sa{};
    if (step) sa = *step;
    else sa.mode = kStepNone;
#define KXG_EPI1(P, X, T)                                                                      \
    hipLaunchKernelGGL((k_epilogue<PT, P, X, T>), grid, blk, 0, s, part, nsplit, nsc, split_stride, ld_b, \
                       fscale, rscale, rate, f, k.d_h, k.d_K, k.d_E, k.mass, n, B, project, C, \
                       diag, sa, ext, eta, folded)
#define KXG_EPI(P, T) if (ext) KXG_EPI1(P, true, T); else KXG_EPI1(P, false, T)
    if (tpb == 256) {
        if (n <= 256) KXG_EPI(1, 256);
        else if (n <= 512) KXG_EPI(2, 256);
        else KXG_EPI(4, 256);
    } else {
        if (n <= 256) KXG_EPI(4, 64);
        else if (n <= 512) KXG_EPI(8, 64);
        else KXG_EPI(16, 64);
    }
#undef KXG_EPI1
#undef KXG_EPI
    return hipGetLastError();
}

RateArgs rate_args(const kxg_kernel &k, const double *f, int B, double *rate)
{
    return RateArgs{k.d_RT, f, k.n, B, rate, (B + kRateT - 1) / kRateT};
}

int rate_tiles(const kxg_kernel &k, int B)
{
    return ((B + kRateT - 1) / kRateT) * ((k.n + kRateT - 1) / kRateT);
}

hipError_t launch_rate(const kxg_kernel &k, const double *f, int B, double *rate, hipStream_t s)
{
    hipLaunchKernelGGL(k_rate, dim3(rate_tiles(k, B)), dim3(256), 0, s, rate_args(k, f, B, rate));
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

// 32-row batch blocks per wave of the FP32 GEMM for a call of B rows: the
// width that minimises width x (workgroups per CU), the MFMA time of the
// busiest CU.  On a tie a narrower tile wins while the launch stays within
// two workgroups per CU (two waves per SIMD hide each other's latencies),
// else the wider one (more MFMAs per operand load).  The work units are
// fixed per handle and a row's partials do not depend on the width, so
// neither does any result.
int gemm_bbw(int nunits, int B)
{
    int best = 4;
    long tbest = -1;
    for (int w = 4; w >= 1; w >>= 1) {
        const long wgs = (long)nunits * div_up(B, 32 * w);
        const long t = w * ((wgs + 255) / 256);
        if (tbest < 0 || t < tbest || (t == tbest && wgs <= 512)) {
            tbest = t;
            best = w;
        }
    }
    return best;
}

}  // namespace

// ---------------------------------------------------------------------------
kxg_status alloc_workspace(const kxg_kernel &k, int b_cap, Workspace &ws)
{
    const int n = k.n;
    // rows of the GEMM operands: a multiple of both batch tilings
    constexpr int tile16 = 4 * KXG_LDS_BBW * 32;
    const int bpad = div_up(div_up(b_cap, 128) * 128, tile16) * tile16;
    size_t need = (size_t)std::max({1, k.nsplit64, k.nsplit32}) * b_cap * n * sizeof(double);
    if (k.d_JX) need = std::max(need, (size_t)std::max(k.nsplitx64, k.nsplitx32) * b_cap * 4 * n * sizeof(double));
    const size_t slots = (size_t)std::max(k.d_G32 ? k.maxslots : 0, (k.d_Gbf || k.d_Gh) ? k.maxslots16 : 0);
    need = std::max(need, slots * bpad * k.geo.ipad * sizeof(float));
    need += (size_t)b_cap * n * sizeof(double);      // loss rates
    ws.part_bytes = need;
    ws.bpad_cap = bpad;
    ws.b_cap = b_cap;
    if (hipMalloc(&ws.part, need) != hipSuccess) { set_error("workspace: out of memory"); return KXG_ENOMEM; }
    const size_t fb = (size_t)k.geo.nb * bpad * kBlk * sizeof(float);
    if (hipMalloc((void **)&ws.fop, fb) != hipSuccess || hipMalloc((void **)&ws.fpar, fb) != hipSuccess ||
        hipMalloc((void **)&ws.fscale, bpad * sizeof(float)) != hipSuccess) {
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

// Which contraction a call takes: the HBM stream (FP64; FP32 on handles
// built for tiny batches, so that on one handle the path and the rounding
// of a row do not depend on how many rows share the call), the LDS-shared
// 16-bit GEMM for large batches, or the register GEMM.  bpad = rows of the
// GEMM operand (0 for the stream).
struct Path {
    bool stream, lds;
    int bpad;
};
static Path path_of(const kxg_kernel &k, int prec, int B)
{
    Path p{false, false, 0};
    if (prec == KXG_F64 || (prec == KXG_F32 && B <= 4 && k.b_cap <= 4 && k.d_P32)) {
        p.stream = true;
        return p;
    }
    if (prec == KXG_BF16X3 || prec == KXG_F16X3 || prec == KXG_F16X2) {
        constexpr int TILE = 4 * KXG_LDS_BBW * 32;
        p.lds = true;
        p.bpad = div_up(B, TILE) * TILE;
        return p;
    }
    const int tile = 32 * gemm_bbw(k.nunits, B);
    p.bpad = div_up(B, tile) * tile;
    return p;
}

// GEMM operand of f for the path of (prec, B); a no-op for the stream path.
kxg_status prep_operands(const kxg_kernel &k, const Workspace &ws, int prec, const double *f,
                         int B, hipStream_t s)
{
    const Path P = path_of(k, prec, B);
    if (P.stream) return KXG_OK;
    hipLaunchKernelGGL(k_prep, dim3(P.bpad), dim3(256), 0, s, f, B, k.n, k.geo.nb, P.bpad,
                       (prec == KXG_F16X3 || prec == KXG_F16X2) ? 1 : 0, ws.fop, ws.fpar, ws.fscale);
    KXG_TRY_HIP(hipGetLastError());
    return KXG_OK;
}

kxg_status eval_impl(const kxg_kernel &k, const Workspace &ws, int prec, const double *f,
                     int B, double *C, uint32_t flags, double *diag, hipStream_t s,
                     const StepArgs *step_in)
{
    const int n = k.n;
    const Geometry &g = k.geo;
    // Operand hand-over between stepper calls applies to the GEMM paths only;
    // they re-enable it below with the layout of their operand.
    StepArgs sa{};
    const StepArgs *step = nullptr;
    if (step_in) {
        sa = *step_in;
        sa.write_op = 0;
        step = &sa;
    }
    const bool op_ready = step_in && step_in->op_ready;
    auto hand_over = [&](int bpad, int f16) {
        if (!step_in || !step_in->write_op) return;
        sa.write_op = 1;
        sa.fop = ws.fop;
        sa.fpar = ws.fpar;
        sa.fscale = ws.fscale;
        sa.nb = g.nb;
        sa.bpad = bpad;
        sa.scale16 = f16;
    };
    // the loss-rate buffer [b_cap][n] sits at the end of the workspace
    double *rate = reinterpret_cast<double *>(static_cast<char *>(ws.part) + ws.part_bytes) -
                   (size_t)ws.b_cap * n;
    const bool exact = (flags & (KXG_INTERP_LOG | KXG_STAT_BOSE | KXG_STAT_FERMI)) != 0;
    if (exact) {
        const bool logi = (flags & KXG_INTERP_LOG) != 0;
        const bool quant = (flags & (KXG_STAT_BOSE | KXG_STAT_FERMI)) != 0;
        const double eta = (flags & KXG_STAT_BOSE) ? 1.0 : ((flags & KXG_STAT_FERMI) ? -1.0 : 0.0);
        const bool dbl = prec == KXG_F64;
        const int nsplit = dbl ? k.nsplitx64 : k.nsplitx32;
        const int chunk = dbl ? k.chunkx64 : k.chunkx32;
        const int nbf = k.geo.nb * kBlk;
        // distributions per pass: one for a single distribution (no idle
        // arithmetic on an empty slot), two otherwise
        const int BT = B == 1 ? 1 : 2;
        const dim3 grid(nsplit, n, div_up(B, BT));
        const size_t shm = 2 * nbf * sizeof(double) + 2 * (size_t)BT * nbf * (dbl ? sizeof(double) : sizeof(float));
        double *ext = static_cast<double *>(ws.part);
#define KXG_SX1(T, AX, BTV, L, Q)                                                                    \
    hipLaunchKernelGGL((k_stream_x<T, BTV, L, Q>), grid, dim3(256), shm, s, AX, k.d_JX, k.d_xpairs, k.d_xib, f, \
                       k.d_K, k.d_invdK, n, nbf, B, chunk, ext)
#define KXG_SX(T, AX, L, Q) if (BT == 1) KXG_SX1(T, AX, 1, L, Q); else KXG_SX1(T, AX, 2, L, Q)
#define KXG_SX2(T, AX)                                                                              \
    if (logi && quant) KXG_SX(T, AX, true, true);                                                   \
    else if (logi) KXG_SX(T, AX, true, false);                                                      \
    else KXG_SX(T, AX, false, true)
        profile_mark_begin(s);
        if (dbl) { KXG_SX2(double, k.d_AX64); } else { KXG_SX2(float, k.d_AX32); }
#undef KXG_SX2
#undef KXG_SX
#undef KXG_SX1
        profile_mark_end(s);
        KXG_TRY_HIP(hipGetLastError());
        KXG_TRY_HIP(launch_epilogue<double>(ext, nsplit, SlotCounts{}, 0, 0, nullptr, nullptr, rate, f, k, B,
                                            (flags & KXG_PROJECT) ? 1 : 0, C, diag, step, s, ext,
                                            eta));
        return KXG_OK;
    }
    const Path P = path_of(k, prec, B);
    const int project = (flags & KXG_PROJECT) ? 1 : 0;
    // loss rates: for the diagnostics, and for the regime switch of
    // freeze-in slots, which is tested on the predictor's input only
    const bool want_rate = diag != nullptr ||
                           (step_in && step_in->freeze_in && step_in->mode == kStepHeunPred);
    if (P.stream) {
        // plain evaluation over the packed kept blocks (FP64; FP32 on
        // single-distribution handles), the loss folded in; loss rates only
        // for diagnostics and the regime switch of freeze-in steppers
        const bool dbl = prec == KXG_F64;
        if (dbl ? !k.d_P64 : !k.d_P32) {
            set_error("kxg_eval: packed stream operand not built");
            return KXG_EUNSUPPORTED;
        }
        const int BT = B == 1 ? 1 : (B == 2 ? 2 : 4);
        const int nbf = k.geo.nb * kBlk;
        const int nsplit = dbl ? k.nsplit64 : k.nsplit32;
        const dim3 grid(nsplit, n, div_up(B, BT));
        const size_t shm = (size_t)BT * nbf * (dbl ? sizeof(double) : sizeof(float));
        double *part = static_cast<double *>(ws.part);
        profile_mark_begin(s);
#define KXG_SP(T, P, CH, BTV) \
    hipLaunchKernelGGL((k_stream_p<T, BTV>), grid, dim3(256), shm, s, P, k.d_pairs64, k.d_ib64, f, n, nbf, B, CH, part)
#define KXG_SP2(T, P, CH) \
    if (BT == 1) KXG_SP(T, P, CH, 1); else if (BT == 2) KXG_SP(T, P, CH, 2); else KXG_SP(T, P, CH, 4)
        if (dbl) { KXG_SP2(double, k.d_P64, k.chunk64); } else { KXG_SP2(float, k.d_P32, k.chunk32); }
#undef KXG_SP2
#undef KXG_SP
        profile_mark_end(s);
        KXG_TRY_HIP(hipGetLastError());
        if (want_rate) KXG_TRY_HIP(launch_rate(k, f, B, rate, s));
        KXG_TRY_HIP(launch_epilogue<double>(part, nsplit, SlotCounts{}, (long)B * n, n, nullptr, nullptr,
                                            want_rate ? rate : nullptr, f, k, B, project, C, diag, step, s,
                                            nullptr, 0.0, 1));
        return KXG_OK;
    }
    const bool f16 = prec == KXG_F16X3 || prec == KXG_F16X2;
    if (P.lds) {
        // 16-bit GEMM, the packed tensor shared through LDS
        constexpr int TILE = 4 * KXG_LDS_BBW * 32;
        const int bpad = P.bpad;
        const int nbt = bpad / TILE;
        if (!op_ready)
            hipLaunchKernelGGL(k_prep, dim3(bpad), dim3(256), 0, s, f, B, n, g.nb, bpad, f16 ? 1 : 0,
                               ws.fop, ws.fpar, ws.fscale);
        hand_over(bpad, f16 ? 1 : 0);
        float *part = static_cast<float *>(ws.part);
        const dim3 grid(nbt * k.nunits16);
        // products of the hi+lo split: 3 (x3), 2 (FP16 x2: A unsplit, f_n f_m
        // split; also the F2-only ablation of x3) or 1 (ablation)
        const int split = prec == KXG_F16X2 ? 2
                          : ((flags & KXG_SPLIT_NONE) ? 1 : ((flags & KXG_SPLIT_F_ONLY) ? 2 : 3));
        profile_mark_begin(s);
        KXG_TRY_HIP(launch_gemm16(f16, split, (int)grid.x, f16 ? k.d_Gh : k.d_Gbf, ws.fop, k.d_pairs16,
                                  k.d_act16, k.d_units16, g.nib, bpad, g.ipad, nbt, part, s));
        profile_mark_end(s);
        KXG_TRY_HIP(hipGetLastError());
        // the loss term is folded into the operand; loss rates only for
        // diagnostics and the regime switch
        if (want_rate) KXG_TRY_HIP(launch_rate(k, f, B, rate, s));
        KXG_TRY_HIP(launch_epilogue<float>(part, k.maxslots16, k.nslot16, (long)bpad * g.ipad, g.ipad,
                                           f16 ? ws.fscale : nullptr, f16 ? k.d_hrow : nullptr,
                                           want_rate ? rate : nullptr, f, k, B, project, C, diag, step, s,
                                           nullptr, 0.0, 1));
        return KXG_OK;
    }
    // FP32 GEMM
    const int bbw = gemm_bbw(k.nunits, B);
    const int bpad = P.bpad;
    const int nbt = bpad / (32 * bbw);
    if (!op_ready)
        hipLaunchKernelGGL(k_prep, dim3(bpad), dim3(256), 0, s, f, B, n, g.nb, bpad, 0,
                           ws.fop, ws.fpar, ws.fscale);
    hand_over(bpad, 0);
    float *part = static_cast<float *>(ws.part);
    profile_mark_begin(s);
    KXG_TRY_HIP(launch_gemm_f32(bbw, nbt * k.nunits, k.d_G32, ws.fop, ws.fpar, k.d_pairs_c, k.d_units, bpad,
                                g.ipad, nbt, part, s));
    profile_mark_end(s);
    KXG_TRY_HIP(hipGetLastError());
    // the loss term is folded into the operand; loss rates only for
    // diagnostics and the regime switch
    if (want_rate) KXG_TRY_HIP(launch_rate(k, f, B, rate, s));
    KXG_TRY_HIP(launch_epilogue<float>(part, k.maxslots, k.nslot, (long)bpad * g.ipad, g.ipad,
                                       nullptr, nullptr, want_rate ? rate : nullptr, f, k, B, project, C,
                                       diag, step, s, nullptr, 0.0, 1));
    return KXG_OK;
}

// ---------------------------------------------------------------------------
// Evaluation without allocation: the workspace of one call (split partials,
// loss rates, GEMM operands and FP16 scales) is carved out of a file-scope
// device array instead of the handle's workspace.  Each device holds its own
// copy of the array for the life of the process; host code never passes the
// array's name to a kernel (that is a host-side stand-in, not a device
// address) but the address hipGetSymbolAddress returns for the current
// device, looked up once per device.  Calls that overlap on one device share
// the array and race.
static __device__ __align__(256) unsigned char scratch[KXG_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices] = {};

static kxg_status scratch_of_current_device(unsigned char **out)
{
    int dev = 0;
    KXG_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("kxg_eval_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
        return KXG_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("kxg_eval_noalloc: hipGetSymbolAddress of the scratch array failed: %s",
                      hipGetErrorString(e));
            return KXG_EHIP;
        }
        g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return KXG_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Bytes of workspace one call of (prec, B, flags) needs, laid out as
// [partials | loss rates [B][n]] [operand, natural order] [operand, parity
// order] [FP16 scales]; fills ws with addresses inside `base` (if given).
static size_t call_workspace(const kxg_kernel &k, int prec, int B, uint32_t flags,
                             unsigned char *base, Workspace &ws)
{
    const int n = k.n;
    const bool exact = (flags & (KXG_INTERP_LOG | KXG_STAT_BOSE | KXG_STAT_FERMI)) != 0;
    const Path P = path_of(k, prec, B);
    size_t part;
    int bpad = 0;
    if (exact) {
        part = (size_t)std::max(k.nsplitx64, k.nsplitx32) * B * 4 * n * sizeof(double);
    } else if (P.stream) {
        part = (size_t)std::max({1, k.nsplit64, k.nsplit32}) * B * n * sizeof(double);
    } else {
        bpad = P.bpad;
        const int slots = P.lds ? k.maxslots16 : k.maxslots;
        part = (size_t)slots * bpad * k.geo.ipad * sizeof(float);
    }
    const size_t rate = (size_t)B * n * sizeof(double);
    const size_t fb = (size_t)k.geo.nb * bpad * kBlk * sizeof(float);
    const size_t o_part = 0, o_fop = align256(part + rate), o_fpar = o_fop + align256(fb),
                 o_fsc = o_fpar + align256(fb), total = o_fsc + align256((size_t)bpad * sizeof(float));
    ws = Workspace{};
    ws.part_bytes = part + rate;
    ws.b_cap = B;
    ws.bpad_cap = bpad;
    if (base) {
        ws.part = base + o_part;
        ws.fop = bpad ? reinterpret_cast<float *>(base + o_fop) : nullptr;
        ws.fpar = bpad ? reinterpret_cast<float *>(base + o_fpar) : nullptr;
        ws.fscale = bpad ? reinterpret_cast<float *>(base + o_fsc) : nullptr;
    }
    return total;
}

kxg_status eval_noalloc_impl(const kxg_kernel &k, int prec, const double *f, int B, double *C,
                             uint32_t flags, double *diag, hipStream_t s)
{
    Workspace ws;
    const size_t need = call_workspace(k, prec, B, flags, nullptr, ws);
    if (need > (size_t)KXG_NOALLOC_SCRATCH_BYTES) {
        set_error("kxg_eval_noalloc: this call needs %zu bytes of scratch, the static array holds %zu "
                  "(fewer distributions per call, or kxg_eval)", need, (size_t)KXG_NOALLOC_SCRATCH_BYTES);
        return KXG_EINVAL;
    }
    unsigned char *base = nullptr;
    const kxg_status st = scratch_of_current_device(&base);
    if (st != KXG_OK) return st;
    call_workspace(k, prec, B, flags, base, ws);
    return eval_impl(k, ws, prec, f, B, C, flags, diag, s);
}

hipError_t launch_moments(const kxg_kernel &k, const double *f, int B, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments, dim3(B), dim3(256), 0, s, f, k.n, k.d_h, k.d_E, out);
    return hipGetLastError();
}

}  // namespace kxg
