// On-device FP64 steppers (Sec. 4.2 of arXiv 2607.00755): fixed RK4 on
// df/dt = lambda C[f], and adaptive Heun in u = ln a on the expanding-universe
// equation (eq. numerical_evolution_loga) with the Hubble drift of eq. fbe.
// One workgroup per slot; per-slot control (accept/reject, dt, end of solve)
// is decided on the device, so advancing never waits for the host.
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

// f on the physical grid from the comoving state g = a^3 p^3 f at u = ln a.
__device__ inline double g_to_f(double g, double p, double u)
{
    return g / (exp(3.0 * u) * (p * p * p));
}

// RK4 stage s (1..4) after C[y_s] is in Cb: k = lambda C; accumulate
// k1 + 2 k2 + 2 k3 + k4; write the next stage input (or the new state) to fb.
__global__ __launch_bounds__(256) void k_rk4_stage(int stage, int n, SlotDev *__restrict__ sl,
                                                   double *__restrict__ x,
                                                   double *__restrict__ acc,
                                                   const double *__restrict__ Cb,
                                                   double *__restrict__ fb)
{
    const int b = blockIdx.x;
    SlotDev &S = sl[b];
    const int running = S.status == 0;
    const double lam = S.lam / S.hi_scale, dt = S.dt;
    double *xb = x + (long)b * n, *ab = acc + (long)b * n, *fbb = fb + (long)b * n;
    const double *cb = Cb + (long)b * n;
    int bad = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        if (!running) { fbb[i] = xb[i]; continue; }
        const double k = lam * cb[i];
        if (stage == 1) { ab[i] = k; fbb[i] = xb[i] + 0.5 * dt * k; }
        else if (stage == 2) { ab[i] += 2.0 * k; fbb[i] = xb[i] + 0.5 * dt * k; }
        else if (stage == 3) { ab[i] += 2.0 * k; fbb[i] = xb[i] + dt * k; }
        else {
            const double xn = xb[i] + dt / 6.0 * (ab[i] + k);
            xb[i] = xn;
            fbb[i] = xn;
            if (!isfinite(xn)) bad = 1;
        }
    }
    if (stage == 4) {
        bad = __syncthreads_or(bad);
        if (threadIdx.x == 0 && running) {
            S.t += dt;
            S.steps += 1;
            if (bad) S.status = -1;
            else if (S.t >= S.tend * (1.0 - 1e-14) || (S.maxsteps > 0 && S.steps >= S.maxsteps))
                S.status = 1;
            else if (S.t + dt > S.tend) S.dt = S.tend - S.t;
        }
    }
}

// Right-hand side in u: drift (conservative upwind on g, cell sizes
// V_i = dp_i/p_i, nothing enters at p_max) plus the collision term
// a^3 p^3 lambda C / H with H = h_i e^{-2u}; without expansion lambda C / h_i.
__device__ inline double rhs_u(int expansion, int i, int n, const double *xs, double c,
                               const double *__restrict__ p, const double *__restrict__ dp,
                               double lam, double hsc, double u)
{
    if (!expansion) return lam * c / hsc;
    const double next = (i + 1 < n) ? xs[i + 1] : 0.0;
    const double V = dp[i] / p[i];
    const double drift = (next - xs[i]) / V;
    const double pi3 = p[i] * p[i] * p[i];
    return drift + exp(5.0 * u) * pi3 * lam * c / hsc;
}

// Heun predictor: k1 = rhs(u, x) with C[f(x)] in Cb; x* = x + dt k1; next
// operator input f(x*, u + dt).
__global__ __launch_bounds__(256) void k_heun_pred(int n, int expansion, SlotDev *__restrict__ sl,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ dp,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ k1,
                                                   double *__restrict__ xs,
                                                   const double *__restrict__ Cb,
                                                   double *__restrict__ fb)
{
    __shared__ double xrow[kMaxN];
    const int b = blockIdx.x;
    const SlotDev &S = sl[b];
    const int running = S.status == 0;
    const double *xb = x + (long)b * n;
    for (int i = threadIdx.x; i < n; i += 256) xrow[i] = xb[i];
    __syncthreads();
    const double dt = S.dt, u = S.t;
    for (int i = threadIdx.x; i < n; i += 256) {
        if (!running) { xs[(long)b * n + i] = xrow[i]; continue; }
        const double k = rhs_u(expansion, i, n, xrow, Cb[(long)b * n + i], p, dp, S.lam,
                               S.hi_scale, u);
        k1[(long)b * n + i] = k;
        const double v = xrow[i] + dt * k;
        xs[(long)b * n + i] = v;
        fb[(long)b * n + i] = expansion ? g_to_f(v, p[i], u + dt) : v;
    }
}

// Heun corrector and control: k2 = rhs(u + dt, x*), x_new = x + dt (k1+k2)/2,
// err = max |x_new - x*| / (atol + rtol max(|x|, |x_new|)); accept if
// err <= 1 (always in replay mode), then dt *= clamp(safety err^-1/2,
// fac_min, fac_max), clipped so that the solve ends exactly at t_end.
// Writes the next operator input f(x, u).
__global__ __launch_bounds__(256) void k_heun_corr(int n, int expansion, int adapt, double rtol,
                                                   double safety, double fac_lo, double fac_hi,
                                                   double dt_min, SlotDev *__restrict__ sl,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ dp,
                                                   double *__restrict__ x,
                                                   const double *__restrict__ k1,
                                                   const double *__restrict__ xs,
                                                   const double *__restrict__ Cb,
                                                   double *__restrict__ fb)
{
    __shared__ double srow[kMaxN];
    __shared__ double lds[8];
    __shared__ int accept_s;
    const int b = blockIdx.x;
    SlotDev &S = sl[b];
    const int running = S.status == 0;
    const double *xsb = xs + (long)b * n;
    for (int i = threadIdx.x; i < n; i += 256) srow[i] = xsb[i];
    __syncthreads();
    const double dt = S.dt, u = S.t;
    constexpr int kPer = kMaxN / 256;
    double xn[kPer];
    double red[2] = {0.0, 0.0};    // error norm, non-finite flag
    for (int q = 0; q < kPer; ++q) {
        const int i = threadIdx.x + 256 * q;
        xn[q] = 0.0;
        if (i < n && running) {
            const double k2 = rhs_u(expansion, i, n, srow, Cb[(long)b * n + i], p, dp, S.lam,
                                    S.hi_scale, u + dt);
            const double x0 = x[(long)b * n + i];
            const double v = x0 + 0.5 * dt * (k1[(long)b * n + i] + k2);
            xn[q] = v;
            const double sc = S.atol + rtol * fmax(fabs(x0), fabs(v));
            const double e = fabs(v - srow[i]) / sc;
            if (!isfinite(v)) red[1] = 1.0;
            red[0] = fmax(red[0], isfinite(e) ? e : 1e300);
        }
    }
    bmax<2>(red, lds);
    if (threadIdx.x == 0) {
        int acc = 0;
        if (running) {
            const double err = red[0];
            if (red[1] > 0.0) {
                S.status = -1;
            } else {
                acc = (!adapt) || err <= 1.0;
                if (acc) {
                    S.outflow += expansion ? 0.5 * dt * (x[(long)b * n] + srow[0]) : 0.0;
                    S.t = u + dt;
                    S.steps += 1;
                } else {
                    S.rejected += 1;
                }
                if (adapt) {
                    double fac = err > 0.0 ? safety / sqrt(err) : fac_hi;
                    fac = fmin(fac_hi, fmax(fac_lo, fac));
                    S.dt = dt * fac;
                }
                if (acc && (S.t >= S.tend * (1.0 - 1e-14) ||
                            (S.maxsteps > 0 && S.steps >= S.maxsteps))) {
                    S.status = 1;
                } else {
                    if (S.t + S.dt > S.tend) S.dt = S.tend - S.t;
                    if (adapt && S.dt < dt_min) S.status = -2;
                }
            }
        }
        accept_s = acc;
    }
    __syncthreads();
    const int acc = accept_s;
    const double unew = S.t;
    for (int q = 0; q < kPer; ++q) {
        const int i = threadIdx.x + 256 * q;
        if (i >= n) continue;
        double v = x[(long)b * n + i];
        if (acc) {
            v = xn[q];
            x[(long)b * n + i] = v;
        }
        fb[(long)b * n + i] = expansion ? g_to_f(v, p[i], unew) : v;
    }
}

// Slot load: x from f0 (g = p^3 f at u = 0 when expanding), operator input,
// h_i from the largest initial loss rate when not given, default dt and atol.
__global__ __launch_bounds__(256) void k_slot_set(int n, int kind, int expansion, double atol_rel,
                                                  int slot, SlotDev *__restrict__ sl,
                                                  const double *__restrict__ f0,
                                                  const double *__restrict__ p,
                                                  const double *__restrict__ RT,
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

hipError_t launch_rk4_stage(int stage, int n, int B, SlotDev *sl, double *x, double *acc,
                            const double *C, double *fb, hipStream_t s)
{
    hipLaunchKernelGGL(k_rk4_stage, dim3(B), dim3(256), 0, s, stage, n, sl, x, acc, C, fb);
    return hipGetLastError();
}

hipError_t launch_heun_pred(int n, int B, int expansion, SlotDev *sl, const double *p,
                            const double *dp, const double *x, double *k1, double *xs,
                            const double *C, double *fb, hipStream_t s)
{
    hipLaunchKernelGGL(k_heun_pred, dim3(B), dim3(256), 0, s, n, expansion, sl, p, dp, x, k1,
                       xs, C, fb);
    return hipGetLastError();
}

hipError_t launch_heun_corr(int n, int B, int expansion, int adapt, double rtol, double safety,
                            double fmin, double fmaxf, double dt_min, SlotDev *sl,
                            const double *p, const double *dp, double *x, const double *k1,
                            const double *xs, const double *C, double *fb, hipStream_t s)
{
    hipLaunchKernelGGL(k_heun_corr, dim3(B), dim3(256), 0, s, n, expansion, adapt, rtol, safety,
                       fmin, fmaxf, dt_min, sl, p, dp, x, k1, xs, C, fb);
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
