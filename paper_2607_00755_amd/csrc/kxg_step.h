// Internal declarations of the on-device steppers.
#pragma once

#include "kxg_internal.h"

namespace kxg {

// Per-slot solve state kept on the device.
struct SlotDev {
    double lam;        // rate prefactor lambda
    double hi_scale;   // H_i (expansion) or time unit (none)
    double dt;         // next step
    double t;          // t (RK4) or u = ln a (Heun)
    double tend;       // end of t or u
    double atol;       // absolute tolerance of the Heun controller
    double outflow;    // comoving number drifted out below p_0
    double rate0;      // largest initial loss rate
    int steps, rejected, status, maxsteps;
};

// Stepper update applied by the evaluation epilogue to the operator output
// of every slot (one workgroup per slot), instead of writing C.
enum StepMode { kStepNone = 0, kStepRK4 = 1, kStepHeunPred = 2, kStepHeunCorr = 3 };
struct StepArgs {
    SlotDev *sl;
    double *x;        // state [B][n]
    double *acc;      // RK4 stage accumulator / Heun k1 [B][n]
    double *xs;       // Heun predictor state [B][n]
    double *fb;       // next operator input f [B][n]
    const double *p, *dp;
    int mode, stage, expansion, adapt;
    double rtol, safety, fac_lo, fac_hi, dt_min;
    // GEMM operand of the next operator call, written by the epilogue from
    // the new f (write_op) instead of by a separate pass; op_ready: the
    // operand of this call was written that way (or by an explicit pass).
    float *fop, *fpar, *fscale;
    int nb, bpad, scale16, write_op, op_ready;
};

// f on the physical grid from the comoving state g = a^3 p^3 f at u = ln a.
__device__ inline double g_to_f(double g, double p, double u)
{
    return g / (exp(3.0 * u) * (p * p * p));
}

// Right-hand side in u: drift (conservative upwind on g, cell sizes
// V_i = dp_i/p_i, nothing enters at p_max) plus the collision term
// a^3 p^3 lambda C / H with H = h_i e^{-2u}; without expansion lambda C / h_i.
// `next` is the state at i+1 (0 beyond the grid).
__device__ inline double rhs_u(int expansion, double xi, double next, double c, double p,
                               double dp, double lam, double hsc, double u)
{
    if (!expansion) return lam * c / hsc;
    const double drift = (next - xi) / (dp / p);
    return drift + exp(5.0 * u) * (p * p * p) * lam * c / hsc;
}
hipError_t launch_slot_set(int n, int kind, int expansion, double atol_rel, int slot,
                           SlotDev *sl, const double *f0, const double *p, const double *RT,
                           double *x, double *fb, hipStream_t s);
hipError_t launch_slot_set_many(int n, int kind, int expansion, double atol_rel, int slot0,
                                int count, const SlotDev *init, SlotDev *sl, const double *f0,
                                const double *p, const double *RT, double *x, double *fb,
                                hipStream_t s);
hipError_t launch_slot_get(int n, int expansion, int slot, const SlotDev *sl, const double *p,
                           const double *x, double *out, hipStream_t s);
hipError_t launch_slot_refresh(int n, int expansion, int slot, const SlotDev *sl,
                               const double *p, const double *x, double *fb, hipStream_t s);

hipError_t launch_slot_clear(int n, int slot, SlotDev *sl, double *x, double *fb, hipStream_t s);
hipError_t launch_set_dt(int B, const double *dt, SlotDev *sl, hipStream_t s);
hipError_t launch_slot_init(int slot, const SlotDev &init, SlotDev *sl, hipStream_t s);

}  // namespace kxg
