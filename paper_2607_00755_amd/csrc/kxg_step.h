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

hipError_t launch_rk4_stage(int stage, int n, int B, SlotDev *sl, double *x, double *acc,
                            const double *C, double *fb, hipStream_t s);
hipError_t launch_heun_pred(int n, int B, int expansion, SlotDev *sl, const double *p,
                            const double *dp, const double *x, double *k1, double *xs,
                            const double *C, double *fb, hipStream_t s);
hipError_t launch_heun_corr(int n, int B, int expansion, int adapt, double rtol, double safety,
                            double fmin, double fmaxf, double dt_min, SlotDev *sl,
                            const double *p, const double *dp, double *x, const double *k1,
                            const double *xs, const double *C, double *fb, hipStream_t s);
hipError_t launch_slot_set(int n, int kind, int expansion, double atol_rel, int slot,
                           SlotDev *sl, const double *f0, const double *p, const double *RT,
                           double *x, double *fb, hipStream_t s);
hipError_t launch_slot_get(int n, int expansion, int slot, const SlotDev *sl, const double *p,
                           const double *x, double *out, hipStream_t s);
hipError_t launch_slot_refresh(int n, int expansion, int slot, const SlotDev *sl,
                               const double *p, const double *x, double *fb, hipStream_t s);

hipError_t launch_slot_clear(int n, int slot, SlotDev *sl, double *x, double *fb, hipStream_t s);
hipError_t launch_set_dt(int B, const double *dt, SlotDev *sl, hipStream_t s);
hipError_t launch_slot_init(int slot, const SlotDev &init, SlotDev *sl, hipStream_t s);

}  // namespace kxg
