/*
 * kxg.h -- C ABI of libkxg: the discretised, isotropic, elastic 2->2
 * self-collision operator of arXiv 2607.00755 on one MI355X (gfx950).
 *
 * The library evaluates, for a batch of distributions f_b on a fixed
 * momentum grid,
 *
 *     C_i[f] = sum_{n,m} A[i,n,m] f_n f_m  -  f_i sum_j R[i,j] f_j
 *
 * (gain minus loss, Sec. 4.1 eq. discrete_collision_operator with the
 * energy-linear interpolation weights of App. B eq. app_interp_weights
 * applied to f), optionally followed by the two-moment conservation
 * projection of App. C (eqs. app_self_projection, app_projection_system),
 * and integrates df/dt = lambda C[f] (fixed RK4) or the expanding-universe
 * equation of Sec. 4.2 (eq. numerical_evolution_loga, adaptive Heun in
 * u = ln a, with the Hubble drift of eq. fbe) on the device.
 *
 * Conventions for every entry point:
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory on the current device; "stream" is a hipStream_t passed as void*
 *    (NULL = the default stream).
 *  - Distributions and results are FP64, row-major [B][n] (distribution b
 *    at offset b*n), whatever precision the contraction runs in.
 *  - Caller-owned buffers stay caller-owned; handles own everything they
 *    allocate and release it in the matching *_free call.
 *  - Entry points return a kxg_status and never throw; on error nothing has
 *    been enqueued and kxg_last_error() gives a message (thread-local).
 *  - Work is enqueued asynchronously on the stream; device faults surface as
 *    KXG_EHIP on a later call that synchronises.
 *  - The library orders nothing across streams: calls on one handle that are
 *    issued on different streams (say kxg_stepper_set on the default stream,
 *    then kxg_stepper_advance on a non-blocking one) race unless the caller
 *    orders them (a synchronisation or an event wait in between).
 */
#ifndef KXG_H
#define KXG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KXG_OK = 0,
    KXG_EINVAL = 1,        /* bad argument (message says which) */
    KXG_ENOMEM = 2,        /* device or host allocation failed */
    KXG_EHIP = 3,          /* a HIP runtime call failed */
    KXG_EUNSUPPORTED = 4,  /* precision not built into this kernel handle */
    KXG_ESTEP = 5,         /* step size underflow in the adaptive stepper */
    KXG_ENUMERIC = 6       /* non-finite values met */
} kxg_status;

/* Precision of the contraction sum_{n,m} A f f.  The projection, the
 * reduction of the split partials and all state updates are FP64 in every
 * case; the loss term f_i sum_j R_ij f_j is folded into the packed operand
 * of the GEMM paths and of the plain streams (so it takes the contraction's
 * precision there) and is summed in FP64 on the exact-form streams. */
typedef enum {
    KXG_F64 = 0,     /* FP64 stream over the kept blocks of the packed
                        A' (the exact forms: A and its brackets on the
                        kept blocks, both orders)                          */
    KXG_F32 = 1,     /* FP32: stream over the packed kept blocks if
                        b_cap <= 4, else MFMA GEMM                        */
    KXG_BF16X3 = 2,  /* BF16 MFMA, hi+lo split of A and of f_n f_m,
                        3 products, FP32 accumulation                     */
    KXG_F16X3 = 3,   /* FP16 MFMA, hi+lo split with power-of-two scaling  */
    KXG_F16X2 = 4    /* FP16 MFMA, A in one FP16 value (power-of-two row
                        scaling), hi+lo split of f_n f_m: 2 products       */
} kxg_prec;
#define KXG_PREC_BIT(p) (1u << (p))
/* Extra bit of kxg_kernel_build's prec_mask: also build the operands the
 * exact-form evaluations (KXG_INTERP_LOG, KXG_STAT_BOSE, KXG_STAT_FERMI)
 * stream: the weights A[i,n,m] (FP64 and/or FP32, as the handle's
 * precisions ask) and the interpolation brackets j_L (2 bytes each) on the
 * blocks that hold a weight. */
#define KXG_WITH_BRACKETS (1u << 8)
/* Extra bit of kxg_kernel_build's prec_mask: a lean handle keeps only the
 * tensors its evaluations read.  The dense FP64 tensor is released after
 * the build unless KXG_F64 is in the mask (FP64 evaluations and
 * kxg_kernel_export of A then return KXG_EUNSUPPORTED).  Meant for callers
 * that admit work by memory footprint. */
#define KXG_LEAN (1u << 9)

/* Angular integral of the reduced kernel (App. B). */
typedef enum {
    KXG_QUAD_GL = 0,    /* Gauss-Legendre in mu, analytic nu (eq. app_I_mu) */
    KXG_QUAD_EXACT = 1  /* closed form of the same double integral          */
} kxg_quad;

/* Momentum grid and model (Sec. 4.1 and App. B).  All host memory, read
 * only during kxg_kernel_build. */
typedef struct {
    int32_t n;          /* grid points, 4 <= n <= 1024                        */
    const double *p;    /* [n] physical momenta, > 0, strictly increasing     */
    const double *dp;   /* [n] widths Delta p_i, or NULL for the trapezoid in
                           ln p (interior p_i (ln p_{i+1} - ln p_{i-1})/2,
                           half that at the two ends)                          */
    double mass;        /* particle mass m > 0                                 */
    double g_dof;       /* internal degrees of freedom g_chi > 0               */
    double m2;          /* constant |M|^2 > 0 (contact interaction)            */
    int32_t n_mu;       /* Gauss-Legendre nodes in mu (the paper uses 18)      */
    int32_t quad;       /* kxg_quad                                            */
} kxg_grid;

typedef struct kxg_kernel kxg_kernel;

/* Build the kernel tensors of a grid (App. B eqs. app_fourth_momentum to
 * app_interp_weights, Sec. 4.1 eq. discrete_weight): on the device, for every
 * (i,n,m) the fourth momentum from energy conservation, the kinematic cuts,
 * the angular integral and the weight W_inm = A[i,n,m]; then R[i,j] from the
 * interpolation bracket of the fourth momentum.  The FP64 tensors are always
 * built; prec_mask (bits KXG_PREC_BIT(p)) selects the extra device copies.
 * b_cap is the largest batch any later kxg_eval on this handle will pass
 * (sizes its workspace).  Blocks until the build has finished.
 * Errors: KXG_EINVAL (grid fields out of range, p not increasing, b_cap < 1),
 * KXG_ENOMEM, KXG_EHIP. */
kxg_status kxg_kernel_build(const kxg_grid *grid, uint32_t prec_mask,
                            int32_t b_cap, void *stream, kxg_kernel **out);

/* Release a kernel handle and all its device memory (NULL is a no-op).
 * Free every stepper created on the handle first.  The release waits for
 * the device (hipFree), so work already enqueued with it completes. */
void kxg_kernel_free(kxg_kernel *k);

/* Grid size n of a handle. */
int32_t kxg_kernel_n(const kxg_kernel *k);

/* Device bytes of the tensors an evaluation at precision prec reads (0 if
 * the precision was not built), or, for prec < 0, every device byte the
 * handle holds (tensors, tables and workspace).  Used for admission by
 * memory footprint. */
size_t kxg_kernel_bytes(const kxg_kernel *k, int32_t prec);

/* Shape of the contraction a handle runs (for reporting work and bytes).
 * The block-packed operand of the batched FP32 path has pair blocks of
 * 32 rows i x 16 x 16 (k, m) (off-diagonal ones carrying both orderings);
 * the blocks that the kinematic cuts (App. B) leave all zero are dropped. */
typedef struct {
    int32_t n;
    int64_t packed_blocks;    /* (i-block, pair) blocks of the full packing   */
    int64_t nonzero_blocks;   /* blocks kept in the FP32 operand (0 if no FP32) */
    int32_t gemm_units;       /* FP32 GEMM work units (K ranges) per batch tile */
    int32_t max_slots;        /* most K partials of an i-block                  */
    int64_t blocks16;         /* (i-block, pair) blocks the 16-bit GEMM multiplies:
                                 the non-zero blocks of the pairs it keeps for
                                 each group of i-blocks a workgroup covers (the
                                 group's all-zero blocks are skipped; 0 if no
                                 16-bit) */
    int64_t nnz_packed;       /* entries (i, k <= m) of the symmetric packing of
                                 A'[i,k,m] = A[i,k,m] - delta_ik R[i,m]
                                 (A'_ikm + A'_imk for k < m) that carry a weight
                                 (A[i,k,m], A[i,m,k], or R on k = i or m = i;
                                 counted by structure, so exact cancellations do
                                 not move it): the contraction's own work is 2
                                 flops per entry and distribution (0 on handles
                                 without a GEMM precision) */
    int64_t staged16;         /* (i-block, pair) blocks of the 16-bit operand:
                                 every i-block of the group for each pair kept
                                 (the union over the group); they are streamed
                                 through LDS whether multiplied or not */
    int64_t blocks64;         /* (i-block, pair) blocks of the packed operand
                                 the plain evaluations stream (the same blocks
                                 as the FP32 GEMM operand; each 32 rows of
                                 16 x 16 values: 64 KiB in FP64, 32 KiB in
                                 FP32 on single-distribution handles; 0 on
                                 handles with neither) */
    int64_t blocks_exact;     /* (i-block, kb, mb) blocks, both (kb, mb) orders,
                                 the exact-form evaluations stream: those of
                                 every pair with a structural weight; each 32
                                 rows of 16 x 16 weights and brackets (64 KiB
                                 of FP64 or 32 KiB of FP32 weights, 16 KiB of
                                 brackets; 0 on handles without brackets) */
} kxg_kernel_info;

/* Fill *out for handle k.  Errors: KXG_EINVAL (null argument). */
kxg_status kxg_kernel_stats(const kxg_kernel *k, kxg_kernel_info *out);

/* Copy the FP64 tensors to host memory: A_host [n][n][n] (m fastest),
 * R_host [n][n].  Either may be NULL.  Synchronous. */
kxg_status kxg_kernel_export(const kxg_kernel *k, double *A_host, double *R_host);

/* Host copies of the grid quantities the library uses: widths dp, energies
 * E = sqrt(p^2+m^2), kinetic energies K = E - m, moment weights h = p^2 dp
 * (App. B).  Any may be NULL. */
kxg_status kxg_kernel_grid(const kxg_kernel *k, double *dp, double *E,
                           double *K, double *h);

/* Evaluation flags. */
#define KXG_PROJECT 1u     /* apply the two-moment projection of App. C      */
#define KXG_INTERP_LOG 2u  /* f at the fourth momentum by the paper's log
                              interpolation (App. B eq. app_log_interp, floor
                              1e-300) instead of linear interpolation of f    */
#define KXG_STAT_BOSE 4u   /* Bose-Einstein factors (eq. Lambda_quantum, eta=+1) */
#define KXG_STAT_FERMI 8u  /* Fermi-Dirac factors (eq. Lambda_quantum, eta=-1)   */
#define KXG_SPLIT_F_ONLY 16u /* ablation, 16-bit precisions: A not split, only
                                F2 split (products hi*hi + lo*hi)              */
#define KXG_SPLIT_NONE 32u   /* ablation, 16-bit precisions: no split at all
                                (the product hi*hi alone)                      */
#define KXG_NDIAG 12       /* diagnostics per distribution, see kxg_eval     */

/* Evaluate C[f] for B distributions (Sec. 4.1 eq. discrete_collision_
 * operator; projection of App. C when flags has KXG_PROJECT).
 * Without KXG_INTERP_LOG / KXG_STAT_* the operator is the precomputed
 * linear-interpolation form gain - f R f (any precision).  With them it is
 * eq. app_dense_collision with the statistical factor of eq. Lambda_quantum
 * (eta = +1, -1, or 0 for the dilute limit) and f at the fourth momentum
 * interpolated linearly or in log f; this exact form streams A and its
 * interpolation brackets (on the blocks that hold a weight) once per group
 * of distributions (precisions KXG_F64 and KXG_F32 only; the handle must be
 * built with KXG_WITH_BRACKETS).
 *  f_dev   device [B][n] FP64 input distributions
 *  C_dev   device [B][n] FP64 output (raw or projected)
 *  diag_dev device [B][KXG_NDIAG] FP64 or NULL:
 *          0 alpha, 1 beta (App. C, E-form: correction xi (alpha + beta E)),
 *          2 eps_N raw, 3 eps_E raw, 4 eps_N projected, 5 eps_E projected
 *          (eq. app_epsilon_definition), 6 R_N, 7 R_E
 *          (eq. app_projection_relative_correction), 8 max_i sum_j R_ij f_j
 *          (largest loss rate), 9 max_i |gain_i|, 10 status bits
 *          (1 non-finite input, 2 negative input, 4 non-finite output),
 *          11 number moment sum_i h_i f_i.
 *  1 <= B <= b_cap of the handle.  Calls on one handle share its workspace:
 *  serialise them on one stream.  Asynchronous.
 * KXG_SPLIT_F_ONLY / KXG_SPLIT_NONE drop products of the hi+lo split of the
 * 16-bit contraction (accuracy ablations; 16-bit precisions only).
 * Errors: KXG_EINVAL (bad flags, both statistics, both ablations, an
 * ablation at FP64/FP32), KXG_EUNSUPPORTED (precision or exact-form operands
 * not built, exact form at 16-bit), KXG_EHIP. */
kxg_status kxg_eval(const kxg_kernel *k, int32_t prec, const double *f_dev,
                    int32_t B, double *C_dev, uint32_t flags, double *diag_dev,
                    void *stream);

/* Size of the library's static device scratch array (64 MiB per device),
 * the workspace of kxg_eval_noalloc. */
#define KXG_NOALLOC_SCRATCH_BYTES (64u << 20)

/* kxg_eval that allocates nothing: for callers that cannot call hipMalloc
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * device allocation).  Same arguments, results and errors as kxg_eval, bit
 * for bit; the call's workspace (split partials, loss rates, GEMM operands,
 * FP16 scales) lives in a static device array of KXG_NOALLOC_SCRATCH_BYTES
 * that every device the library runs on holds until the process ends,
 * instead of in the handle's workspace.  The first call on a device looks up
 * that device's copy of the array (no allocation).  Every call on a device
 * shares its array: calls that overlap on one device (on several streams,
 * or from several threads without ordering) race; calls on one stream are
 * ordered.  The array keeps the last call's contents; nothing in it needs
 * to start at zero.  Additional error: KXG_EINVAL when the call needs more
 * scratch than the array holds (the message gives both sizes). */
kxg_status kxg_eval_noalloc(const kxg_kernel *k, int32_t prec, const double *f_dev,
                            int32_t B, double *C_dev, uint32_t flags, double *diag_dev,
                            void *stream);

/* Discrete moments of B distributions (App. B): out_dev [B][3] =
 * { sum h f, sum h E f, -sum_{f>0} h f (ln f - 1) }.  Asynchronous. */
kxg_status kxg_moments(const kxg_kernel *k, const double *f_dev, int32_t B,
                       double *out_dev, void *stream);

/* Gauss-Legendre nodes (ascending) and weights on [-1,1] as the library
 * computes them (Golub-Welsch), host memory, n >= 1. */
kxg_status kxg_gauss_legendre(int32_t n, double *x, double *w);

/* ---------------- on-device steppers (Sec. 4.2) -------------------------- */

typedef enum { KXG_RK4 = 0, KXG_HEUN = 1 } kxg_stepper_kind;
typedef enum { KXG_EXP_NONE = 0, KXG_EXP_RADIATION = 1 } kxg_expansion;

typedef struct {
    int32_t kind;       /* KXG_RK4: fixed classical RK4 in t on df/dt = lambda C.
                           KXG_HEUN: adaptive Heun (Euler predictor, trapezoid
                           corrector, their difference as error estimate)      */
    int32_t prec;       /* kxg_prec of the contraction                          */
    int32_t expansion;  /* KXG_EXP_RADIATION (Heun only): state g = a^3 p^3 f in
                           u = ln a, H = h_i e^{-2u}, conservative upwind drift;
                           KXG_EXP_NONE: state f                               */
    int32_t project;    /* 1: evolve with the projected operator (App. C)       */
    int32_t adapt;      /* Heun: 1 adapt dt, 0 take dt as set (replay)          */
    int32_t b_cap;      /* number of slots                                      */
    double rtol;        /* Heun controller: err = max |x_new - x*| /
                           (atol + rtol max(|x|,|x_new|)), accept if err <= 1   */
    double atol_rel;    /* atol = atol_rel * max |x(0)| per slot                */
    double safety;      /* dt *= clamp(safety err^-1/2, fac_min, fac_max)       */
    double fac_min, fac_max;
    double dt_min;      /* Heun: a slot whose dt falls below this fails         */
    int32_t freeze_in;  /* 1: the slots may carry freeze-in sources and start in
                           the source-only regime (kxg_solve_params src_*,
                           du_src, eps_switch; Heun with KXG_EXP_RADIATION only).
                           Every operator call then also forms the FP64 loss
                           rates R f that the regime switch tests.             */
    int32_t pad_;
} kxg_stepper_params;

typedef struct {
    double lambda;      /* rate prefactor lambda of df/dt = lambda C             */
    double h_i;         /* H at u = 0 (expansion) or 1 (none); <= 0 selects the
                           largest initial loss rate max_i sum_j R_ij f_j(0)     */
    double dt;          /* RK4: step in t; Heun: first step (u or t);
                           <= 0 selects 0.1 / (lambda * rate0) for RK4, 1e-3 Heun */
    double t_end;       /* end of t (RK4) or u (Heun)                            */
    int32_t max_steps;  /* accepted-step cap (<= 0: none), both regimes together */
    int32_t pad_;
    /* Freeze-in sources of Sec. 3 (steppers with freeze_in = 1; all zero for
     * none), in the code's units: densities as nu = (2 pi^2 / g) n, so that
     * sum_i h_i f_i is the chi density; time in units of 1/h_i (H = h_i e^{-2u},
     * so h_i must be given, > 0).  Condensate (eq. C_condensate_decay):
     * 2 Gamma nu_Phi particles per unit time at momentum p0, shared between
     * the two grid points that bracket p0 in kinetic energy with the
     * energy-linear weights of eq. app_interp_weights (number and energy
     * injected exactly), a^3 nu_Phi = src_n0 exp(-(Gamma / 2 h_i)(e^{2u} - 1)).
     * Higgs decay (eq. C_higgs_decay): kappa (T / E p)(e^{-E_-/T} - e^{-E_+/T}),
     * E_+- = (m_h^2 E +- m_h p sqrt(m_h^2 - 4 m^2)) / (2 m^2), T = T_i e^{-u}. */
    double src_n0;      /* a^3 nu_Phi at u = 0 (0: no condensate)                */
    double src_gamma;   /* condensate decay rate Gamma_Phi                       */
    double src_p0;      /* momentum of the decay products (inside the grid)      */
    double src_kappa;   /* Higgs-decay amplitude kappa (0: no Higgs source)      */
    double src_mh;      /* Higgs mass / particle mass (> 2)                      */
    double src_ti;      /* bath temperature at u = 0 / particle mass (> 0)       */
    /* Regimes of Sec. 4.2: du_src > 0 starts the slot in the source-only
     * regime (elastic operator off, one classical RK4 step of size du_src in u
     * per iteration); before each such step the slot tests
     * Gamma_22 / H > eps_switch, with Gamma_22 = lambda sum h f (R f) / sum h f
     * the mean per-particle loss rate of the current f, and from the first
     * state over it on runs the adaptive Heun with the elastic operator and
     * the sources (first step dt, atol = atol_rel max |x| at the switch).
     * du_src <= 0: the elastic operator is on from the start. */
    double du_src;
    double eps_switch;  /* the paper uses 1e-2                                   */
} kxg_solve_params;

typedef struct {
    double t;           /* time (RK4) or u = ln a (Heun)                        */
    double dt;          /* next step                                           */
    double outflow;     /* comoving number drifted out below p_0 (expansion)   */
    double h_i;         /* the H_i (or rate0) in use                           */
    int32_t steps;      /* accepted steps                                      */
    int32_t rejected;   /* rejected Heun attempts                              */
    int32_t status;     /* 0 running, 1 reached t_end, 2 stopped at max_steps
                           before t_end, -1 non-finite, -2 dt underflow (Heun:
                           the next step would be below dt_min), -3 free slot */
    int32_t phase;      /* 0 source-only regime, 1 elastic operator on          */
    double u_switch;    /* u at the switch (0 if it started with collisions on) */
    int32_t n_src;      /* steps taken in the source-only regime (in steps too) */
    int32_t pad;
} kxg_slot_state;

typedef struct kxg_stepper kxg_stepper;

/* Create a stepper with b_cap slots over a kernel handle (which must outlive
 * it and have params->prec built).  Allocates its own state and workspace.
 * Errors: KXG_EINVAL, KXG_EUNSUPPORTED, KXG_ENOMEM, KXG_EHIP. */
kxg_status kxg_stepper_create(const kxg_kernel *k, const kxg_stepper_params *params,
                              kxg_stepper **out);
/* Release a stepper, its captured graphs and its device memory (NULL is a
 * no-op); waits for the device like kxg_kernel_free. */
void kxg_stepper_free(kxg_stepper *s);

/* Load slot `slot` with the distribution f0_dev (device [n] FP64) and its
 * solve parameters; the slot becomes active.  Asynchronous on stream. */
kxg_status kxg_stepper_set(kxg_stepper *s, int32_t slot, const double *f0_dev,
                           const kxg_solve_params *sp, void *stream);

/* Load `count` consecutive slots [slot0, slot0 + count) at once, slot
 * slot0 + j from row j of f0_dev (device [count][n] FP64) with the solve
 * parameters sp_host[j] (host [count], read before the call returns); one
 * launch for all of them.  The records travel through a pinned staging
 * buffer of the stepper: a call waits until the copy of the previous call
 * has left it.  Errors: KXG_EINVAL (null argument, slots out of range, bad
 * parameters of any solve; nothing is enqueued then), KXG_EHIP.
 * Asynchronous on stream. */
kxg_status kxg_stepper_set_many(kxg_stepper *s, int32_t slot0, int32_t count,
                                const double *f0_dev, const kxg_solve_params *sp_host,
                                void *stream);

/* Device bytes the stepper holds (slot records, state vectors, workspace),
 * for admission by memory footprint; 0 for NULL. */
size_t kxg_stepper_bytes(const kxg_stepper *s);

/* Free a slot: it stops being advanced, its state is zeroed and it counts
 * as empty.  Asynchronous on stream. */
kxg_status kxg_stepper_release(kxg_stepper *s, int32_t slot, void *stream);

/* Advance every running slot by n_iter iterations (RK4: steps; Heun:
 * attempted steps, two operator calls each).  Slots that reach t_end,
 * max_steps or fail stop by themselves on the device.  On a non-default
 * stream the iterations replay HIP graphs captured on first use (eight
 * iterations per replay, then single ones for the rest), one pair per batch
 * bucket of 16 slots, kept for the stepper's lifetime and captured again
 * only when that bucket is replayed on another stream; on the default stream, or while a
 * profile is open, they are launched directly.  Same results either way.
 * Asynchronous. */
kxg_status kxg_stepper_advance(kxg_stepper *s, int32_t n_iter, void *stream);

/* Set the next dt of every slot from host memory dt_host [b_cap] (replay of
 * a given step sequence with adapt = 0).  Asynchronous (copies first). */
kxg_status kxg_stepper_set_dt(kxg_stepper *s, const double *dt_host, void *stream);

/* Copy all slot states to host memory out [b_cap].  Synchronises stream. */
kxg_status kxg_stepper_query(kxg_stepper *s, kxg_slot_state *out, void *stream);

/* Copy a slot's distribution f (converted from g = a^3 p^3 f when expanding)
 * into device memory f_dev [n].  Asynchronous. */
kxg_status kxg_stepper_get(kxg_stepper *s, int32_t slot, double *f_dev, void *stream);

/* Checkpoint of one slot (state vector, t, dt, counters, controller state)
 * to host bytes: with buf == NULL sets *len to the size needed; otherwise
 * writes *len bytes.  kxg_stepper_load restores it into a slot.  Both
 * synchronise the stream. */
kxg_status kxg_stepper_save(kxg_stepper *s, int32_t slot, void *buf, size_t *len,
                            void *stream);
kxg_status kxg_stepper_load(kxg_stepper *s, int32_t slot, const void *buf, size_t len,
                            void *stream);

/* ---------------- profiling -------------------------------------------------
 * While a profile is open, every launch of a gain kernel (the MFMA GEMM or
 * the single-distribution stream kernel, inside kxg_eval and the steppers)
 * is bracketed by two HIP events on the stream it is launched on, for up to
 * `capacity` launches (process-wide; not for concurrent use from several
 * threads).  kxg_profile_end waits for the events and returns the summed
 * kernel time in milliseconds and the number of launches measured. */
kxg_status kxg_profile_begin(int32_t capacity);
kxg_status kxg_profile_end(double *total_ms, int32_t *launches);

/* Device self-calibration, for reporting roofline fractions against what
 * this chip sustains beside its datasheet peaks (not an operation of the
 * method).  out [4] (host): out[0] FP32 matrix-core rate in TFLOP/s, from a
 * loop of independent v_mfma_f32_32x32x2f32 on every SIMD; out[1] the same
 * for v_mfma_f32_32x32x16_bf16; out[2] device-memory read bandwidth in GB/s
 * (a 16-byte-vector read of 1 GiB, the access pattern of the stream
 * kernels); out[3] copy bandwidth in GB/s (512 MiB copied, bytes read plus
 * bytes written).  Each is the best of three timed launches (HIP events on
 * `stream`) after one untimed launch.  Allocates and frees 1 GiB plus 8 MiB
 * of device memory; synchronises the stream.  Errors: KXG_EINVAL (null
 * out), KXG_ENOMEM, KXG_EHIP. */
kxg_status kxg_peak_probe(double *out, void *stream);

/* Thread-local message of the last error ("" if none). */
const char *kxg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KXG_H */
