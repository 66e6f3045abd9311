// Slot management of the on-device FP64 steppers (Sec. 4.2 of arXiv
// 2607.00755): loading, reading back, clearing and restoring slots.  The
// stage updates themselves (RK4 stages, Heun predictor and corrector with
// per-slot step control) run inside the evaluation epilogue (kxg_eval.hip).
#include "kxg_step.h"

namespace kxg {
namespace {

template <int NV>
__device__ void bmax(double (&v)[NV], double *lds)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        for (int off = 32; off > 0; off >>= 1) v[j] = fmax(v[j], __shfl_xor(v[j], off));
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) lds[wave * NV + j] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j)
        v[j] = fmax(fmax(lds[j], lds[NV + j]), fmax(lds[2 * NV + j], lds[3 * NV + j]));
    __syncthreads();
}

// Slot load: x from f0 (g = p^3 f at u = 0 when expanding), operator input,
// h_i from the largest initial loss rate when not given, default dt and atol.
// The slot record already holds the solve parameters.
__device__ void slot_set(int n, int kind, int expansion, double atol_rel, int slot,
                         SlotDev *__restrict__ sl, const double *__restrict__ f0,
                         const double *__restrict__ p, const double *__restrict__ RT,
                         double *__restrict__ x, double *__restrict__ fb)
{
    __shared__ double frow[kMaxN];
    __shared__ double lds[8];
    SlotDev &S = sl[slot];
    for (int i = threadIdx.x; i < n; i += 256) frow[i] = f0[i];
    __syncthreads();
    double red[2] = {0.0, 0.0};     // rate max, |x| max
    for (int i = threadIdx.x; i < n; i += 256) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += RT[(long)j * n + i] * frow[j];
        red[0] = fmax(red[0], r);
        const double xv = expansion ? frow[i] * (p[i] * p[i] * p[i]) : frow[i];
        red[1] = fmax(red[1], fabs(xv));
        x[(long)slot * n + i] = xv;
        fb[(long)slot * n + i] = frow[i];
    }
    bmax<2>(red, lds);
    if (threadIdx.x == 0) {
        S.rate0 = red[0];
        if (!(S.hi_scale > 0.0)) S.hi_scale = red[0] > 0.0 ? red[0] : 1.0;
        if (!(S.dt > 0.0)) {
            if (kind == KXG_RK4) {
                const double rate = S.lam * S.rate0 / S.hi_scale;
                S.dt = rate > 0.0 ? 0.1 / rate : 1.0;
            } else {
                S.dt = 1e-3;
            }
        }
        if (S.t + S.dt > S.tend) S.dt = S.tend - S.t;
        S.atol = atol_rel * red[1];
        if (!(S.atol > 0.0)) S.atol = 1e-300;
        S.status = 0;
    }
}

__global__ __launch_bounds__(256) void k_slot_set(int n, int kind, int expansion, double atol_rel,
                                                  int slot, SlotDev *__restrict__ sl,
                                                  const double *__restrict__ f0,
                                                  const double *__restrict__ p,
                                                  const double *__restrict__ RT,
                                                  double *__restrict__ x, double *__restrict__ fb)
{
    slot_set(n, kind, expansion, atol_rel, slot, sl, f0, p, RT, x, fb);
}

// Many slots at once: workgroup j copies record init[j] into slot slot0 + j,
// then loads that slot from row j of f0 [count][n].
__global__ __launch_bounds__(256) void k_slot_set_many(int n, int kind, int expansion,
                                                       double atol_rel, int slot0,
                                                       const SlotDev *__restrict__ init,
                                                       SlotDev *__restrict__ sl,
                                                       const double *__restrict__ f0,
                                                       const double *__restrict__ p,
                                                       const double *__restrict__ RT,
                                                       double *__restrict__ x,
                                                       double *__restrict__ fb)
{
    const int j = blockIdx.x;
    if (threadIdx.x == 0) sl[slot0 + j] = init[j];
    __syncthreads();
    slot_set(n, kind, expansion, atol_rel, slot0 + j, sl, f0 + (long)j * n, p, RT, x, fb);
}

__global__ void k_slot_get(int n, int expansion, int slot, const SlotDev *__restrict__ sl,
                           const double *__restrict__ p, const double *__restrict__ x,
                           double *__restrict__ out)
{
    const double u = sl[slot].t;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = x[(long)slot * n + i];
        out[i] = expansion ? g_to_f(v, p[i], u) : v;
    }
}

__global__ void k_slot_refresh(int n, int expansion, int slot, const SlotDev *__restrict__ sl,
                               const double *__restrict__ p, const double *__restrict__ x,
                               double *__restrict__ fb)
{
    const double u = sl[slot].t;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = x[(long)slot * n + i];
        fb[(long)slot * n + i] = expansion ? g_to_f(v, p[i], u) : v;
    }
}

__global__ void k_slot_clear(int n, int slot, SlotDev *__restrict__ sl, double *__restrict__ x,
                             double *__restrict__ fb)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        x[(long)slot * n + i] = 0.0;
        fb[(long)slot * n + i] = 0.0;
    }
    if (threadIdx.x == 0) sl[slot].status = -3;
}

__global__ void k_set_dt(int B, const double *__restrict__ dt, SlotDev *__restrict__ sl)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) sl[b].dt = dt[b];
}

__global__ void k_slot_init(int slot, SlotDev init, SlotDev *__restrict__ sl) { sl[slot] = init; }

}  // namespace

hipError_t launch_slot_clear(int n, int slot, SlotDev *sl, double *x, double *fb, hipStream_t s)
{
    hipLaunchKernelGGL(k_slot_clear, dim3(1), dim3(256), 0, s, n, slot, sl, x, fb);
    return hipGetLastError();
}

hipError_t launch_set_dt(int B, const double *dt, SlotDev *sl, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_dt, dim3((B + 255) / 256), dim3(256), 0, s, B, dt, sl);
    return hipGetLastError();
}

hipError_t launch_slot_init(int slot, const SlotDev &init, SlotDev *sl, hipStream_t s)
{
    hipLaunchKernelGGL(k_slot_init, dim3(1), dim3(1), 0, s, slot, init, sl);
    return hipGetLastError();
}

hipError_t launch_slot_set(int n, int kind, int expansion, double atol_rel, int slot,
                           SlotDev *sl, const double *f0, const double *p, const double *RT,
                           double *x, double *fb, hipStream_t s)
{
    hipLaunchKernelGGL(k_slot_set, dim3(1), dim3(256), 0, s, n, kind, expansion, atol_rel, slot,
                       sl, f0, p, RT, x, fb);
    return hipGetLastError();
}

hipError_t launch_slot_set_many(int n, int kind, int expansion, double atol_rel, int slot0,
                                int count, const SlotDev *init, SlotDev *sl, const double *f0,
                                const double *p, const double *RT, double *x, double *fb,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_slot_set_many, dim3(count), dim3(256), 0, s, n, kind, expansion, atol_rel,
                       slot0, init, sl, f0, p, RT, x, fb);
    return hipGetLastError();
}

hipError_t launch_slot_get(int n, int expansion, int slot, const SlotDev *sl, const double *p,
                           const double *x, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_slot_get, dim3(1), dim3(256), 0, s, n, expansion, slot, sl, p, x, out);
    return hipGetLastError();
}

hipError_t launch_slot_refresh(int n, int expansion, int slot, const SlotDev *sl,
                               const double *p, const double *x, double *fb, hipStream_t s)
{
    hipLaunchKernelGGL(k_slot_refresh, dim3(1), dim3(256), 0, s, n, expansion, slot, sl, p, x,
                       fb);
    return hipGetLastError();
}

}  // namespace kxg
