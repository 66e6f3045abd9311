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
    // freeze-in sources (Sec. 3) and the regimes of Sec. 4.2
    double src_n0;     // a^3 nu_Phi at u = 0 (0: no condensate)
    double src_gamma;  // condensate decay rate
    double src_kappa;  // Higgs-decay amplitude (0: none)
    double src_mh;     // Higgs mass / particle mass
    double src_kh;     // sqrt(m_h^2 - 4 m^2)
    double src_ti;     // bath temperature at u = 0
    double wl_h, wr_h; // condensate deposit weights over h at jdep, jdep + 1
    double du_src;     // step of the source-only regime
    double eps_switch; // Gamma_22 / H threshold
    double u_switch;   // u at the switch
    int steps, rejected, status, maxsteps;
    int jdep;          // deposit node of the condensate (-1: none)
    int phase;         // 0 source-only regime, 1 elastic operator on
    int nsrc;          // steps taken in the source-only regime
    int pad;
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
    // freeze-in steppers: sources, the source-only regime and its switch;
    // every operator call then also forms the loss rates R f
    int freeze_in;
    double atol_rel, mass;
};

// f on the physical grid from the comoving state g = a^3 p^3 f at u = ln a.
__device__ inline double g_to_f(double g, double p, double u)
{
    return g / (exp(3.0 * u) * (p * p * p));
}

// Right-hand side in u: drift (conservative upwind on g, cell sizes
// V_i = dp_i/p_i, nothing enters at p_max) plus the collision and source
// terms a^3 p^3 (lambda C + S) / H with H = h_i e^{-2u}; without expansion
// lambda C / h_i.  `next` is the state at i+1 (0 beyond the grid).
__device__ inline double rhs_u(int expansion, double xi, double next, double c, double p,
                               double dp, double lam, double hsc, double u, double src = 0.0)
{
    if (!expansion) return lam * c / hsc;
    const double drift = (next - xi) / (dp / p);
    return drift + exp(5.0 * u) * (p * p * p) * (lam * c + src) / hsc;
}

// Freeze-in source of slot S at grid point i (momentum p, energy E) and
// u = ln a, in the units of C (Sec. 3): the Higgs decay in the bath,
// kappa (T / E p) e^{-E_-/T} (1 - e^{-(E_+ - E_-)/T}) with T = T_i e^{-u},
// E_+- = (m_h^2 E +- m_h p k_h) / (2 m^2); and the condensate's
// 2 Gamma nu_Phi injection shared by the grid points jdep, jdep + 1, with
// a^3 nu_Phi = n0 exp(-(Gamma / 2 h_i)(e^{2u} - 1)).
__device__ inline double freeze_in_source(const SlotDev &S, int i, double p, double E,
                                          double mass, double u)
{
    double s = 0.0;
    if (S.src_kappa > 0.0) {
        const double T = S.src_ti * exp(-u);
        const double m2x2 = 2.0 * mass * mass;
        const double em = (S.src_mh * S.src_mh * E - S.src_mh * p * S.src_kh) / m2x2;
        const double de = 2.0 * S.src_mh * p * S.src_kh / m2x2;
        s += S.src_kappa * (T / (E * p)) * exp(-em / T) * (-expm1(-de / T));
    }
    if (S.src_n0 > 0.0 && (i == S.jdep || i == S.jdep + 1)) {
        const double nu = exp(-3.0 * u) * (S.src_n0 * exp(-(S.src_gamma / (2.0 * S.hi_scale)) *
                                                          (exp(2.0 * u) - 1.0)));
        s += 2.0 * S.src_gamma * nu * (i == S.jdep ? S.wl_h : S.wr_h);
    }
    return s;
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
