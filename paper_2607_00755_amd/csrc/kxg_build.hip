// Kernel-tensor build on the device (App. B of arXiv 2607.00755).
//
// Compiled with -ffp-contract=off: the kinematic cut and the interpolation
// bracket of every (i,n,m) are decided on K~ = (K_n + K_m) - K_i with plain
// IEEE double adds, from host-computed K, so that the decisions do not depend
// on FMA contraction.
#include "kxg_internal.h"

#include <cmath>

namespace kxg {
namespace {

constexpr double kPi = 3.14159265358979323846;

// Angular factor of the reduced kernel by the paper's route (App. B,
// eqs. app_cosphi to app_F_1d): Gauss-Legendre in mu; for each node the
// quadratic a nu^2 + b nu + c >= 0 that encodes |cos phi| <= 1, its roots
// clipped to [-1,1], and the analytic nu integral
// I(mu) = [asin((2a nu_- + b)/sqrt(D)) - asin((2a nu_+ + b)/sqrt(D))]/sqrt(-a).
// Returns p_n p_m sum_q w_q I(mu_q), i.e. the double integral over (mu, nu).
__device__ double phi_gauss(double pi, double pn, double pm, double ki, double kn,
                            double km, int nmu, const double *__restrict__ xmu,
                            const double *__restrict__ wmu)
{
    // m^2 + E_n E_m - E_n E_i - E_m E_i == (K_n - K_i)(K_m - K_i) - p_i^2
    const double base = (kn - ki) * (km - ki) - pi * pi;
    const double pnpm = pn * pm;
    double total = 0.0;
    for (int q = 0; q < nmu; ++q) {
        const double mu = xmu[q];
        const double a0 = base + pi * pn * mu;
        const double a1 = pi * pm - pnpm * mu;
        const double kk = pnpm * pnpm * (1.0 - mu * mu);
        const double qa = -(kk + a1 * a1);
        const double qb = -2.0 * a0 * a1;
        // b^2 - 4ac (c = K^2 - A0^2) through the exact identity
        // 4 K^2 (K^2 + A1^2 - A0^2): no cancellation in the sign decision
        const double disc = 4.0 * kk * ((kk + a1 * a1) - a0 * a0);
        if (!(disc > 0.0) || !(qa < 0.0)) continue;
        const double sq = sqrt(disc);
        const double ra = (-qb + sq) / (2.0 * qa);
        const double rb = (-qb - sq) / (2.0 * qa);
        const double rlo = fmin(ra, rb), rhi = fmax(ra, rb);
        const double nlo = fmax(rlo, -1.0);
        const double nhi = fmin(rhi, 1.0);
        if (!(nlo < nhi)) continue;
        // the arcsine argument is exactly +1 / -1 at an unclipped smaller /
        // larger root (qa < 0); only clipped limits are evaluated
        const double ulo = rlo < -1.0 ? fmin(fmax((2.0 * qa * nlo + qb) / sq, -1.0), 1.0) : 1.0;
        const double uhi = rhi > 1.0 ? fmin(fmax((2.0 * qa * nhi + qb) / sq, -1.0), 1.0) : -1.0;
        total += wmu[q] * ((asin(ulo) - asin(uhi)) / sqrt(-qa));
    }
    return pnpm * total;
}

// Closed form of the same double integral for a constant matrix element:
// pi S / (2 p1) with S the signed sum of |p1 +- p2 +- p3 +- p4| (momentum
// delta written as a Fourier integral, solid angles done analytically).
__device__ double phi_closed(double p1, double p2, double p3, double p4)
{
    const double pos = fabs(p1 - p2 - p3 - p4) + fabs(p1 - p2 + p3 + p4) +
                       fabs(p1 + p2 - p3 + p4) + fabs(p1 + p2 + p3 - p4);
    const double neg = fabs(p1 - p2 - p3 + p4) + fabs(p1 - p2 + p3 - p4) +
                       fabs(p1 + p2 - p3 - p4) + (p1 + p2 + p3 + p4);
    return kPi * (pos - neg) / (2.0 * p1);
}

// One thread per (i, n, m): the fourth momentum from energy conservation
// (eq. app_fourth_momentum, in kinetic energy), the cuts E~ >= m and
// q_min <= q~ <= q_max (K_0 <= K~ <= K_{N-1}), and
// W_inm = dp_n dp_m F_inm / (2 E_i g) (eq. discrete_weight) with
// F_inm = |M|^2 / (4 (2 pi)^4) (p_n p_m / (E_n E_m)) Phi_inm; the factor
// p_n p_m/(E_n E_m) is the phase-space measure 1/(2E) of the two outgoing
// legs that the reduction of eq. C22_general leaves behind.
__global__ __launch_bounds__(256) void k_build_A(
    int n, const double *__restrict__ p, const double *__restrict__ dp,
    const double *__restrict__ E, const double *__restrict__ K, double mass, double gdof,
    double m2, int quad, int nmu, const double *__restrict__ xmu,
    const double *__restrict__ wmu, double *__restrict__ A)
{
    const long total = (long)n * n * n;
    const double pref = m2 / (4.0 * (2.0 * kPi) * (2.0 * kPi) * (2.0 * kPi) * (2.0 * kPi));
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        const int m = (int)(idx % n);
        const long r = idx / n;
        const int a = (int)(r % n);
        const int i = (int)(r / n);
        const double kt = (K[a] + K[m]) - K[i];
        double w = 0.0;
        if (kt >= K[0] && kt <= K[n - 1]) {
            double phi;
            if (quad == KXG_QUAD_EXACT) {
                const double pt = sqrt(kt * (kt + 2.0 * mass));
                phi = phi_closed(p[i], pt, p[a], p[m]);
            } else {
                phi = phi_gauss(p[i], p[a], p[m], K[i], K[a], K[m], nmu, xmu, wmu);
            }
            const double jac = (p[a] * p[m]) / (E[a] * E[m]);
            w = (dp[a] * dp[m]) * (pref * jac * phi) / (2.0 * E[i] * gdof);
        }
        A[idx] = w;
    }
}

// First m in [0, n) whose K~ = (K_a + K_m) - K_i is >= x (strict: > x).
__device__ int first_at_least(const double *__restrict__ K, int n, double ka, double ki,
                              double x, bool strict)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const double kt = (ka + K[mid]) - ki;
        const bool up = strict ? (kt > x) : (kt >= x);
        if (up) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// One thread per (i, j): R[i][j] = sum over (n,m) of W_inm times the
// energy-linear interpolation weight (eq. app_interp_weights) that the
// fourth momentum puts on bin j.  The bracket is j_L = the largest
// j <= N-2 with K_j <= K~; for fixed (i, n), K~ grows with m, so the m with
// j_L = j form one contiguous range, found by bisection on the same K~
// expression the weight kernel uses.  Summation order: n ascending, m
// ascending.  Writes RT[j][i].
__global__ __launch_bounds__(256) void k_build_R(int n, const double *__restrict__ K,
                                                 const double *__restrict__ A,
                                                 double *__restrict__ RT)
{
    const long total = (long)n * n;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        const int i = (int)(idx / n);
        const int j = (int)(idx % n);
        const double ki = K[i];
        double acc = 0.0;
        for (int a = 0; a < n; ++a) {
            const double ka = K[a];
            const double *row = A + ((long)i * n + a) * n;
            for (int side = 0; side < 2; ++side) {
                // side 0: bracket j_L = j-1 (weight omega_R on j),
                // side 1: bracket j_L = j   (weight omega_L on j)
                const int jl = side == 0 ? j - 1 : j;
                if (jl < 0 || jl > n - 2) continue;
                const int lo = first_at_least(K, n, ka, ki, K[jl], false);
                const int hi = (jl < n - 2) ? first_at_least(K, n, ka, ki, K[jl + 1], false)
                                            : first_at_least(K, n, ka, ki, K[n - 1], true);
                const double kl = K[jl], kr = K[jl + 1];
                for (int m = lo; m < hi; ++m) {
                    const double kt = (ka + K[m]) - ki;
                    const double wr = (kt - kl) / (kr - kl);
                    acc += side == 0 ? row[m] * wr : row[m] * (1.0 - wr);
                }
            }
        }
        RT[(long)j * n + i] = acc;
    }
}

// Interpolation bracket of entry (i, k, m) for the exact-form evaluations
// (eq. app_interp_weights): the largest j <= N-2 with K_j <= K~ for
// K~ = K_k + K_m - K_i (the same K~ expression and comparisons as the weight
// kernel), 0xFFFF where the entry is cut (K~ outside the grid) or an index
// lies past the grid (padding).  Bisection over the grid.
__device__ uint16_t bracket_of(int n, const double *__restrict__ K, int i, int k, int m)
{
    if (i >= n || k >= n || m >= n) return 0xFFFF;
    const double kt = (K[k] + K[m]) - K[i];
    if (!(kt >= K[0] && kt <= K[n - 1])) return 0xFFFF;
    int lo = 0, hi = n - 2;                 // invariant: K[lo] <= kt
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (K[mid] <= kt) lo = mid; else hi = mid - 1;
    }
    return (uint16_t)lo;
}

// Value of the block-packed operand for output row i and pair (kb <= mb),
// block-local (dk, dm): off-diagonal blocks carry both orderings of (k,m).
// The loss term is folded in: f_i sum_m R_im f_m = sum_{k,m} delta_ik R_im
// f_k f_m, so the operand holds A'_ikm = A_ikm - delta_ik R_im and the GEMM
// yields gain - loss directly (eq. discrete_collision_operator).
__device__ double packed_value(const double *__restrict__ A, const double *__restrict__ RT, int n,
                               int i, int kb, int mb, int dk, int dm)
{
    const int k = kb * kBlk + dk, m = mb * kBlk + dm;
    if (i >= n || k >= n || m >= n) return 0.0;
    const long row = (long)i * n * n;
    double v = A[row + (long)k * n + m];
    if (k == i) v -= RT[(long)m * n + i];
    if (kb != mb) {
        v += A[row + (long)m * n + k];
        if (m == i) v -= RT[(long)k * n + i];
    }
    return v;
}

// Whether entry (k, m) of the symmetric packing has any contributing term:
// A[i,k,m], A[i,m,k] or a loss weight R[i,.] on the diagonal k = i or m = i.
// Counting these instead of the non-zero values keeps the count free of
// accidental cancellations (A - R rounding to exactly zero in one evaluation
// order and not in another); it depends only on the kinematic cuts.
__device__ int packed_structural(const double *__restrict__ A, const double *__restrict__ RT,
                                 int n, int i, int k, int m)
{
    if (i >= n || k >= n || m >= n) return 0;
    const long row = (long)i * n * n;
    int s = A[row + (long)k * n + m] != 0.0 || A[row + (long)m * n + k] != 0.0;
    if (k == i) s |= RT[(long)m * n + i] != 0.0;
    if (m == i) s |= RT[(long)k * n + i] != 0.0;
    return s;
}

// Non-zero flag of every (i-block, pair) block of the packed operand: 32
// rows i x the 16 x 16 (k, m) block and its transpose.  Also the number of
// entries of the symmetric packing restricted to k <= m (inside a diagonal
// block only dk <= dm) that carry a weight: the contraction's own work, 2
// flops per entry and distribution.  Grid (pair, i-block).
__global__ __launch_bounds__(256) void k_block_nz(int n, int npairs, const int *__restrict__ pairs,
                                                  const double *__restrict__ A,
                                                  const double *__restrict__ RT,
                                                  unsigned char *__restrict__ flags,
                                                  unsigned int *__restrict__ nnz)
{
    __shared__ int cnt[4];
    const int pr = blockIdx.x, ib = blockIdx.y;
    const int kb = pairs[2 * pr], mb = pairs[2 * pr + 1];
    int any = 0, c = 0;
    for (int e = threadIdx.x; e < kIBlk * kBlk * kBlk; e += 256) {
        const int i = ib * kIBlk + e / (kBlk * kBlk);
        const int dk = (e / kBlk) % kBlk, dm = e % kBlk;
        const double v = packed_value(A, RT, n, i, kb, mb, dk, dm);
        if (v != 0.0) any = 1;
        // entries (k <= m) with a contributing term (inside a diagonal
        // block only dk <= dm)
        if (kb != mb || dk <= dm) c += packed_structural(A, RT, n, i, kb * kBlk + dk, mb * kBlk + dm);
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = c;
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) {
        flags[(long)ib * npairs + pr] = (unsigned char)(any != 0);
        nnz[(long)ib * npairs + pr] = (unsigned int)(cnt[0] + cnt[1] + cnt[2] + cnt[3]);
    }
}

// FP32 GEMM operand, ordered as the 32x32x2 MFMA consumes it, over the
// compacted blocks: [block c][dk][half][lane][4]; block c is pair
// (kb, mb) = pairs_c[c] of i-block cib[c]; lane l holds row
// i = cib*32 + l%32 and K index 2t + l/32 of row dk of the block,
// t = 4*half + r.
__global__ void k_pack_f32(int n, long ncomp, const int *__restrict__ pairs_c,
                           const int *__restrict__ cib, const double *__restrict__ A,
                           const double *__restrict__ RT, float *__restrict__ G)
{
    const long total = ncomp * kBlk * 2 * 64 * 4;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        long t = idx;
        const int r = (int)(t % 4); t /= 4;
        const int lane = (int)(t % 64); t /= 64;
        const int half = (int)(t % 2); t /= 2;
        const int dk = (int)(t % kBlk);
        const long c = t / kBlk;
        const int i = cib[c] * kIBlk + (lane & 31);
        const int dm = 2 * (4 * half + r) + (lane >> 5);
        G[idx] = (float)packed_value(A, RT, n, i, pairs_c[2 * c], pairs_c[2 * c + 1], dk, dm);
    }
}

// Operand of the plain evaluation over the kept blocks (FP64 or FP32), row
// by row: row i of i-block ib = i / 32 starts at (first_ib * 32 + (i % 32)
// cnt_ib) blocks of 256 values and holds the blocks of the i-block's kept
// pairs in order, each [dk][dm] (m fastest).  Work item = (kept block c, row
// of the i-block, value).
template <typename T>
__global__ void k_pack_rows(int n, long ncomp, const int *__restrict__ pairs,
                            const int *__restrict__ ib64, const int *__restrict__ cib,
                            const double *__restrict__ A, const double *__restrict__ RT,
                            T *__restrict__ P)
{
    const long total = ncomp * kIBlk * 256;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        const int w = (int)(idx % 256);
        const long t = idx / 256;
        const int r = (int)(t % kIBlk);
        const long c = t / kIBlk;
        const int ib = cib[c];
        const int first = ib64[2 * ib], cnt = ib64[2 * ib + 1];
        const long dst = ((long)first * kIBlk + (long)r * cnt + (c - first)) * 256 + w;
        P[dst] = (T)packed_value(A, RT, n, ib * kIBlk + r, pairs[2 * c], pairs[2 * c + 1], w / kBlk, w % kBlk);
    }
}

// Operands of the exact forms over the ordered kept blocks, row by row:
// row i of i-block ib starts at (first_ib * 32 + (i % 32) cnt_ib) blocks of
// 256 values and holds A[i,k,m] (as is: no symmetrisation, no loss) of its
// i-block's blocks (kb, mb) in order, each [dk][dm], and (if JX is given)
// the brackets j_L of the same entries.  Work item = (block c, row, value).
template <typename T>
__global__ void k_pack_exact(int n, long nx, const int *__restrict__ xpairs, const int *__restrict__ xib,
                             const int *__restrict__ cib, const double *__restrict__ A,
                             const double *__restrict__ K, T *__restrict__ AX, uint16_t *__restrict__ JX)
{
    const long total = nx * kIBlk * 256;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        const int w = (int)(idx % 256);
        const long t = idx / 256;
        const int r = (int)(t % kIBlk);
        const long c = t / kIBlk;
        const int ib = cib[c];
        const int first = xib[2 * ib], cnt = xib[2 * ib + 1];
        const long dst = ((long)first * kIBlk + (long)r * cnt + (c - first)) * 256 + w;
        const int i = ib * kIBlk + r;
        const int k = xpairs[2 * c] * kBlk + w / kBlk, m = xpairs[2 * c + 1] * kBlk + w % kBlk;
        const bool in = i < n && k < n && m < n;
        AX[dst] = in ? (T)A[((long)i * n + k) * n + m] : (T)0;
        if (JX) JX[dst] = bracket_of(n, K, i, k, m);
    }
}

__device__ inline uint16_t bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf/nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// 16-bit hi/lo operands for the 32x32x16 MFMA over the kept blocks of a
// group of ibw i-blocks: [block c][i-block of the group][dk][hi|lo][lane][8];
// block c is pair pairs16[c] of group cit[c]; lane l holds row
// i = (cit*ibw + g)*32 + l%32 and the 8 consecutive K indices 8*(l/32) + j
// of row dk of the block.  BF16: hi = bf16(v), lo = bf16(v - hi); FP16 (row
// scale rs): the same of v * rs[i] in FP16.
template <bool F16>
__global__ void k_pack_16(int n, long ncomp, int ibw, const int *__restrict__ pairs16,
                          const int *__restrict__ cit, const double *__restrict__ A,
                          const double *__restrict__ RT, const float *__restrict__ rs,
                          uint16_t *__restrict__ G)
{
    const long total = ncomp * ibw * kBlk * 64 * 8;          // hi/lo written together
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        long t = idx;
        const int j = (int)(t % 8); t /= 8;
        const int lane = (int)(t % 64); t /= 64;
        const int dk = (int)(t % kBlk); t /= kBlk;
        const int gi = (int)(t % ibw);
        const long c = t / ibw;
        const int i = (cit[c] * ibw + gi) * kIBlk + (lane & 31);
        const int dm = 8 * (lane >> 5) + j;
        const double v = packed_value(A, RT, n, i, pairs16[2 * c], pairs16[2 * c + 1], dk, dm);
        uint16_t hi, lo;
        if constexpr (F16) {
            const double vs = i < n ? v * (double)rs[i] : 0.0;
            const _Float16 h = (_Float16)(float)vs;
            const _Float16 l = (_Float16)(float)(vs - (double)(float)h);
            hi = __builtin_bit_cast(uint16_t, h);
            lo = __builtin_bit_cast(uint16_t, l);
        } else {
            hi = bf16_rne((float)v);
            lo = bf16_rne((float)(v - (double)bf16_to_f32(hi)));
        }
        const long base = (((c * ibw + gi) * kBlk + dk) * 2) * 64 * 8;
        G[base + (long)lane * 8 + j] = hi;
        G[base + 64 * 8 + (long)lane * 8 + j] = lo;
    }
}

// Power-of-two scale per output row for the FP16 operand: the largest
// packed entry of row i (bounded by twice the row maximum of A plus twice
// that of R, which is folded into the operand) lands in [2^13, 2^14].  One
// workgroup per row.
__global__ __launch_bounds__(256) void k_row_scale(int n, int ipad, const double *__restrict__ A,
                                                   const double *__restrict__ RT,
                                                   float *__restrict__ scale)
{
    __shared__ double red[2][256];
    const int i = blockIdx.x;
    double ma = 0.0, mr = 0.0;
    if (i < n) {
        const double *row = A + (long)i * n * n;
        for (long e = threadIdx.x; e < (long)n * n; e += blockDim.x) ma = fmax(ma, fabs(row[e]));
        for (int j = threadIdx.x; j < n; j += blockDim.x) mr = fmax(mr, fabs(RT[(long)j * n + i]));
    }
    red[0][threadIdx.x] = ma;
    red[1][threadIdx.x] = mr;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double top = 2.0 * (red[0][0] + red[1][0]);
        float sc = 1.0f;
        if (top > 0.0) {
            const int e = 14 - (int)ceil(log2(top));
            sc = (float)ldexp(1.0, e);
        }
        scale[i] = sc;
    }
}

inline int grid_for(long work, int block = 256, int cap = 1 << 20)
{
    long g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

// R in row order (R[i][j]) from its transpose, for the row-wise loss of the
// single-distribution stream.
__global__ __launch_bounds__(256) void k_transpose(int n, const double *__restrict__ RT,
                                                   double *__restrict__ R)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)n * n) return;
    const int i = (int)(t / n), j = (int)(t % n);
    R[t] = RT[(long)j * n + i];
}

hipError_t launch_build_A(const kxg_kernel &k, const double *d_xmu, const double *d_wmu,
                          hipStream_t s)
{
    const long total = (long)k.n * k.n * k.n;
    hipLaunchKernelGGL(k_build_A, dim3(grid_for(total)), dim3(256), 0, s, k.n, k.d_p, k.d_dp,
                       k.d_E, k.d_K, k.mass, k.gdof, k.m2, k.quad, k.nmu, d_xmu, d_wmu,
                       k.d_A64);
    return hipGetLastError();
}

hipError_t launch_build_R(const kxg_kernel &k, hipStream_t s)
{
    const long total = (long)k.n * k.n;
    hipLaunchKernelGGL(k_build_R, dim3(grid_for(total, 64)), dim3(64), 0, s, k.n, k.d_K,
                       k.d_A64, k.d_RT);
    hipLaunchKernelGGL(k_transpose, dim3(grid_for(total)), dim3(256), 0, s, k.n, k.d_RT, k.d_R);
    return hipGetLastError();
}

hipError_t launch_pack_exact(const kxg_kernel &k, hipStream_t s)
{
    const long tot = k.nx * kIBlk * 256;
    if (tot <= 0) return hipSuccess;
    const int *cib = k.d_xpairs + 2 * k.nx;
    if (k.d_AX64)
        hipLaunchKernelGGL(k_pack_exact<double>, dim3(grid_for(tot)), dim3(256), 0, s, k.n, k.nx, k.d_xpairs,
                           k.d_xib, cib, k.d_A64, k.d_K, k.d_AX64, k.d_JX);
    if (k.d_AX32)
        hipLaunchKernelGGL(k_pack_exact<float>, dim3(grid_for(tot)), dim3(256), 0, s, k.n, k.nx, k.d_xpairs,
                           k.d_xib, cib, k.d_A64, k.d_K, k.d_AX32, k.d_AX64 ? nullptr : k.d_JX);
    return hipGetLastError();
}

hipError_t launch_block_nz(const kxg_kernel &k, unsigned char *flags, unsigned int *nnz,
                           hipStream_t s)
{
    const Geometry &g = k.geo;
    hipLaunchKernelGGL(k_block_nz, dim3(g.npairs, g.nib), dim3(256), 0, s, k.n, g.npairs,
                       k.d_pairs, k.d_A64, k.d_RT, flags, nnz);
    return hipGetLastError();
}

hipError_t launch_pack_f32(const kxg_kernel &k, hipStream_t s)
{
    const long tot = k.ncomp * kBlk * 2 * 64 * 4;
    if (tot > 0)
        hipLaunchKernelGGL(k_pack_f32, dim3(grid_for(tot)), dim3(256), 0, s, k.n, k.ncomp,
                           k.d_pairs_c, k.d_cib, k.d_A64, k.d_RT, k.d_G32);
    return hipGetLastError();
}

hipError_t launch_pack_rows(const kxg_kernel &k, hipStream_t s)
{
    const long tot = k.ncomp64 * kIBlk * 256;
    if (tot > 0 && k.d_P64)
        hipLaunchKernelGGL(k_pack_rows<double>, dim3(grid_for(tot)), dim3(256), 0, s, k.n, k.ncomp64,
                           k.d_pairs64, k.d_ib64, k.d_pairs64 + 2 * k.ncomp64, k.d_A64, k.d_RT, k.d_P64);
    if (tot > 0 && k.d_P32)
        hipLaunchKernelGGL(k_pack_rows<float>, dim3(grid_for(tot)), dim3(256), 0, s, k.n, k.ncomp64,
                           k.d_pairs64, k.d_ib64, k.d_pairs64 + 2 * k.ncomp64, k.d_A64, k.d_RT, k.d_P32);
    return hipGetLastError();
}

hipError_t launch_pack_16(const kxg_kernel &k, int ibw, hipStream_t s)
{
    const long tot = k.ncomp16 * ibw * kBlk * 64 * 8;
    if (tot <= 0) return hipSuccess;
    if (k.d_Gbf)
        hipLaunchKernelGGL(k_pack_16<false>, dim3(grid_for(tot)), dim3(256), 0, s, k.n, k.ncomp16,
                           ibw, k.d_pairs16, k.d_cit16, k.d_A64, k.d_RT, k.d_hrow, k.d_Gbf);
    if (k.d_Gh)
        hipLaunchKernelGGL(k_pack_16<true>, dim3(grid_for(tot)), dim3(256), 0, s, k.n, k.ncomp16,
                           ibw, k.d_pairs16, k.d_cit16, k.d_A64, k.d_RT, k.d_hrow, k.d_Gh);
    return hipGetLastError();
}

hipError_t launch_derive(kxg_kernel &k, hipStream_t s)
{
    const Geometry &g = k.geo;
    if (k.d_hrow)
        hipLaunchKernelGGL(k_row_scale, dim3(g.ipad), dim3(256), 0, s, k.n, g.ipad, k.d_A64,
                           k.d_RT, k.d_hrow);
    return hipGetLastError();
}

}  // namespace kxg
