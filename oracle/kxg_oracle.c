/*
 * kxg_oracle.c -- plain, slow FP64 CPU oracle for the discretised, isotropic,
 * elastic 2->2 self-collision operator of arXiv 2607.00755 ("KineticXGPU").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline of the benchmark load it (through oracle/__init__.py).  It shares
 * no source with the GPU library.
 *
 * Every routine follows the paper's own steps and notation, in FP64, with
 * plain loops.  Readings of points the paper leaves open (weights, the
 * Jacobian of the reduced kernel, linear vs. log interpolation, the drift
 * discretisation) are stated at the routine that takes them.
 *
 * Parity pins: every routine here is checked by the CPU tests
 * (tests/test_oracle_pins.py, tests/test_golden_cpu.py) against the paper's
 * printed numbers, closed forms, invariants, brute force or an independent
 * integration.  The adaptive Heun controller is pinned by its accuracy
 * against a fine fixed-step RK4 solution (error within rtol and falling in
 * proportion to it, step count growing as rtol^-1/2, rejections until the
 * estimate falls to one), the Hubble factor of the expanding-universe
 * right-hand side by the a^-1 scaling of its collision increment.  Its
 * step-size law (safety 0.9, exponent 1/2, clamps [0.2, 5]) is a reading
 * the paper leaves open; the tests check it only against its own statement.
 * The freeze-in part (Sec. 3, Sec. 4.2) is pinned by the injection moments
 * of the condensate (number and energy, exactly), the decay law of the
 * condensate against a numerical solution, the Higgs-decay rate against
 * its Bessel-function closed form, Gamma_22 against n sigma <v_rel> of a
 * non-relativistic Maxwell-Boltzmann gas, conservation of chi number plus
 * twice the condensate's (fourth order in the source-only step), the switch
 * at the first state over the threshold, and the second regime against the
 * pinned Heun of the expanding run.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Grid (App. B, "physical momenta p_i, energies E_i, widths Delta p_i,      */
/* moment weights h_i = p_i^2 Delta p_i").                                   */
/* Reading of the unspecified widths: grid points are quadrature nodes,      */
/* endpoints included; Delta p_i = p_i * (trapezoid width in ln p), i.e.     */
/* p_i (ln p_{i+1} - ln p_{i-1})/2 inside and one-sided halves at the ends.  */
/* A caller may override the widths.                                         */
/* Kinetic energy K_i = E_i - m is formed as p^2/(E+m) so that the           */
/* energy-conservation cut can be decided without cancellation.              */
/* ------------------------------------------------------------------------ */
void or_grid(int n, const double *p, double mass, const double *dp_override,
             double *dp, double *E, double *K, double *h)
{
    for (int i = 0; i < n; ++i) {
        E[i] = sqrt(p[i] * p[i] + mass * mass);
        K[i] = (p[i] * p[i]) / (E[i] + mass);
    }
    for (int i = 0; i < n; ++i) {
        if (dp_override) {
            dp[i] = dp_override[i];
        } else {
            double lo = (i > 0) ? log(p[i - 1]) : log(p[i]);
            double hi = (i < n - 1) ? log(p[i + 1]) : log(p[i]);
            dp[i] = p[i] * (hi - lo) / 2.0;
        }
        h[i] = p[i] * p[i] * dp[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes and weights on [-1,1] (App. B: "the remaining mu    */
/* integral is evaluated with Gauss-Legendre quadrature").  Newton's method */
/* on the Legendre polynomial P_n, three-term recurrence.  Nodes ascending. */
/* ------------------------------------------------------------------------ */
void or_gauss_legendre(int n, double *x, double *w)
{
    for (int k = 0; k < n; ++k) {
        /* k-th root counted from +1 downwards */
        double z = cos(M_PI * (k + 0.75) / (n + 0.5));
        double pn = 0.0, pnm1 = 0.0, dpn = 1.0;
        for (int it = 0; it < 200; ++it) {
            double a = 1.0, b = 0.0;            /* P_j, P_{j-1} */
            for (int j = 1; j <= n; ++j) {
                double c = b;
                b = a;
                a = ((2.0 * j - 1.0) * z * b - (j - 1.0) * c) / j;
            }
            pn = a;
            pnm1 = b;
            dpn = n * (z * pn - pnm1) / (z * z - 1.0);
            double dz = pn / dpn;
            z -= dz;
            if (fabs(dz) <= 1e-16 * fabs(z) + 1e-300)
                break;
        }
        {
            double a = 1.0, b = 0.0;
            for (int j = 1; j <= n; ++j) {
                double c = b;
                b = a;
                a = ((2.0 * j - 1.0) * z * b - (j - 1.0) * c) / j;
            }
            dpn = n * (z * a - b) / (z * z - 1.0);
        }
        x[n - 1 - k] = z;
        w[n - 1 - k] = 2.0 / ((1.0 - z * z) * dpn * dpn);
    }
}

/* ------------------------------------------------------------------------ */
/* Angular factor Phi_inm = int dmu dnu / (sqrt(1-mu^2) sqrt(1-nu^2)        */
/*                                        sqrt(1-cos^2 phi))               */
/* by the paper's route (App. B, eqs. app_cosphi, app_measure_rewrite,      */
/* app_I_mu, app_F_1d): for each Gauss-Legendre node mu, the coefficients   */
/* A0, A1, K^2, the quadratic a nu^2 + b nu + c, its discriminant, roots    */
/* clipped to [-1,1] and the analytic nu integral I(mu) via arcsin; then    */
/* Phi = p_n p_m sum_q w_q I(mu_q).                                         */
/* A0 is written as (K_n-K_i)(K_m-K_i) - p_i^2 + p_i p_n mu, which equals   */
/* m^2 + E_n E_m - E_n E_i - E_m E_i + p_i p_n mu exactly.                  */
/* ------------------------------------------------------------------------ */
double or_angular_gl(double pi, double pn, double pm, double Ki, double Kn,
                     double Km, int nmu, const double *xmu, const double *wmu)
{
    double a0c = (Kn - Ki) * (Km - Ki) - pi * pi;
    double sum = 0.0;
    for (int q = 0; q < nmu; ++q) {
        double mu = xmu[q];
        double A0 = a0c + pi * pn * mu;
        double A1 = pi * pm - pn * pm * mu;
        double K2 = pn * pn * pm * pm * (1.0 - mu * mu);
        double a = -(K2 + A1 * A1);
        double b = -2.0 * A0 * A1;
        /* discriminant b^2 - 4ac with c = K^2 - A0^2, written through the
         * identity b^2 - 4ac = 4 K^2 (K^2 + A1^2 - A0^2): the same number,
         * without the cancellation of the two O(A0^2 A1^2) terms that would
         * otherwise decide its sign near zero */
        double disc = 4.0 * K2 * ((K2 + A1 * A1) - A0 * A0);
        if (!(disc > 0.0) || !(a < 0.0))
            continue;                        /* no allowed nu interval */
        double sd = sqrt(disc);
        double r1 = (-b + sd) / (2.0 * a);
        double r2 = (-b - sd) / (2.0 * a);
        double lo = r1 < r2 ? r1 : r2;
        double hi = r1 < r2 ? r2 : r1;
        int lo_clip = lo < -1.0, hi_clip = hi > 1.0;
        if (lo_clip) lo = -1.0;
        if (hi_clip) hi = 1.0;
        if (!(lo < hi))
            continue;                        /* interval misses [-1,1] */
        /* at an unclipped root (2a r + b)/sqrt(D) is exactly +1 (smaller
         * root, a < 0) or -1 (larger root); only clipped limits are computed */
        double s_lo = lo_clip ? (2.0 * a * lo + b) / sd : 1.0;
        double s_hi = hi_clip ? (2.0 * a * hi + b) / sd : -1.0;
        if (s_lo > 1.0) s_lo = 1.0;
        if (s_lo < -1.0) s_lo = -1.0;
        if (s_hi > 1.0) s_hi = 1.0;
        if (s_hi < -1.0) s_hi = -1.0;
        double I = (asin(s_lo) - asin(s_hi)) / sqrt(-a);
        sum += wmu[q] * I;
    }
    return pn * pm * sum;
}

/* ------------------------------------------------------------------------ */
/* Closed form of the same angular factor for a constant matrix element,    */
/* used as an independent pin of the Gauss-Legendre route:                  */
/*   Phi = pi * S(p1,p2,p3,p4) / (2 p1),                                    */
/* S = |p1-p2-p3-p4| + |p1-p2+p3+p4| + |p1+p2-p3+p4| + |p1+p2+p3-p4|        */
/*   - |p1-p2-p3+p4| - |p1-p2+p3-p4| - |p1+p2-p3-p4| - (p1+p2+p3+p4),       */
/* with p1 = p_i, p2 = p_j~ (the fourth momentum), p3 = p_n, p4 = p_m.      */
/* It follows from writing the momentum delta function of eq. C22_general   */
/* as a Fourier integral and doing the three solid-angle integrals.         */
/* ------------------------------------------------------------------------ */
double or_angular_exact(double p1, double p2, double p3, double p4)
{
    double s = fabs(p1 - p2 - p3 - p4) + fabs(p1 - p2 + p3 + p4)
             + fabs(p1 + p2 - p3 + p4) + fabs(p1 + p2 + p3 - p4)
             - fabs(p1 - p2 - p3 + p4) - fabs(p1 - p2 + p3 - p4)
             - fabs(p1 + p2 - p3 - p4) - (p1 + p2 + p3 + p4);
    return M_PI * s / (2.0 * p1);
}

/* ------------------------------------------------------------------------ */
/* One kernel entry (i,n,m): the fourth momentum from energy conservation   */
/* (eq. app_fourth_momentum, in kinetic energy K = E - m), the kinematic    */
/* cuts (E_j~ >= m and q_min <= q_j~ <= q_max, App. B), the discrete weight  */
/* (eq. discrete_weight) and the energy-linear interpolation bracket        */
/* (eq. app_interp_weights).                                                */
/*                                                                          */
/* Reading of the reduced kernel: the reduction of eq. C22_general carries  */
/* the phase-space factors 1/(2E_3) 1/(2E_4) of the two integrated legs, so */
/*   F_inm = |M|^2/(4 (2 pi)^4) * (p_n p_m/(E_n E_m)) * Phi_inm,             */
/* which is the printed eq. app_F_1d times p_n p_m/(E_n E_m).  The MC pin   */
/* of the full 9-D definition decides between the two (tests).              */
/*                                                                          */
/* Cuts in K: keep iff K_0 <= K~ <= K_{N-1} (equivalent to E~ >= m and the  */
/* grid range cut on a grid with p_0 > 0).  Bracket: jL = the largest       */
/* j <= N-2 with K_j <= K~, omega_R = (K~ - K_jL)/(K_jL+1 - K_jL), which is */
/* the paper's energy-linear weight since E - K is constant.                */
/* Returns W (0 when cut) and writes jL, omega_R.                           */
/* ------------------------------------------------------------------------ */
double or_weight(int n, const double *p, const double *dp, const double *E,
                 const double *K, double mass, double gdof, double m2,
                 int quad, int nmu, const double *xmu, const double *wmu,
                 int i, int a, int b, int *jl_out, double *wr_out)
{
    double kt = (K[a] + K[b]) - K[i];
    *jl_out = -1;
    *wr_out = 0.0;
    if (!(kt >= K[0] && kt <= K[n - 1]))
        return 0.0;
    int jl = 0;
    for (int j = 0; j <= n - 2; ++j)
        if (K[j] <= kt)
            jl = j;
    double wr = (kt - K[jl]) / (K[jl + 1] - K[jl]);
    double phi;
    if (quad == 1) {
        double pt = sqrt(kt * (kt + 2.0 * mass));
        phi = or_angular_exact(p[i], pt, p[a], p[b]);
    } else {
        phi = or_angular_gl(p[i], p[a], p[b], K[i], K[a], K[b], nmu, xmu, wmu);
    }
    double F = m2 / (4.0 * pow(2.0 * M_PI, 4.0)) * (p[a] * p[b] / (E[a] * E[b])) * phi;
    double W = dp[a] * dp[b] * F / (2.0 * E[i] * gdof);
    *jl_out = jl;
    *wr_out = wr;
    return W;
}

/* ------------------------------------------------------------------------ */
/* Kernel tensors of the linear-interpolation form of eq. app_dense_collision:
 *   A[i][n][m] = W_inm (0 if cut),
 *   R[i][j]    = sum_{n,m} W_inm (omega_L delta_{j,jL} + omega_R delta_{j,jL+1}),
 * so that C_i = sum_{n,m} A_inm f_n f_m - f_i sum_j R_ij f_j.
 * Optionally the per-entry bracket (jL, omega_R) for the direct evaluation.
 * quad: 0 = Gauss-Legendre in mu with analytic nu (the paper's), 1 = closed form.
 * ------------------------------------------------------------------------ */
void or_kernel_build(int n, const double *p, const double *dp_override,
                     double mass, double gdof, double m2, int quad, int nmu,
                     double *A, double *R, int *jl_all, double *wr_all)
{
    double *dp = malloc(sizeof(double) * n), *E = malloc(sizeof(double) * n);
    double *K = malloc(sizeof(double) * n), *h = malloc(sizeof(double) * n);
    double *xmu = malloc(sizeof(double) * (nmu > 0 ? nmu : 1));
    double *wmu = malloc(sizeof(double) * (nmu > 0 ? nmu : 1));
    or_grid(n, p, mass, dp_override, dp, E, K, h);
    if (nmu > 0)
        or_gauss_legendre(nmu, xmu, wmu);
    memset(R, 0, sizeof(double) * (size_t)n * n);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < n; ++a) {
            for (int b = 0; b < n; ++b) {
                int jl;
                double wr;
                double W = or_weight(n, p, dp, E, K, mass, gdof, m2, quad, nmu,
                                     xmu, wmu, i, a, b, &jl, &wr);
                size_t idx = ((size_t)i * n + a) * n + b;
                A[idx] = W;
                if (jl_all) jl_all[idx] = jl;
                if (wr_all) wr_all[idx] = wr;
                if (jl >= 0) {
                    R[(size_t)i * n + jl] += W * (1.0 - wr);
                    R[(size_t)i * n + jl + 1] += W * wr;
                }
            }
        }
    }
    free(dp); free(E); free(K); free(h); free(xmu); free(wmu);
}

/* ------------------------------------------------------------------------ */
/* Direct evaluation of eq. app_dense_collision: for every (i,n,m) recompute */
/* W_inm, the fourth momentum and the interpolated f_j~, then sum           */
/* W Lambda.  interp = 0: energy-linear interpolation of f (the form that   */
/* the precomputed A/R tensors represent); interp = 1: the paper's log      */
/* interpolation (eq. app_log_interp) with an absolute floor of 1e-300     */
/* under the logarithm.  eta = 0: dilute limit, Lambda = f_n f_m - f_i f_j~;*/
/* eta = +1 / -1: Bose-Einstein / Fermi-Dirac factors of eq.                */
/* Lambda_quantum with particles 1 = i, 2 = j~, 3 = n, 4 = m:               */
/*   Lambda = f_n f_m (1 + eta f_i)(1 + eta f_j~)                           */
/*          - f_i f_j~ (1 + eta f_n)(1 + eta f_m).                          */
/* Outputs gain (first product), loss (second) and C = gain - loss.         */
/* ------------------------------------------------------------------------ */
void or_collision_direct_q(int n, const double *p, const double *dp_override,
                           double mass, double gdof, double m2, int quad, int nmu,
                           int interp, int eta, const double *f, double *gain,
                           double *loss, double *C);

void or_collision_direct(int n, const double *p, const double *dp_override,
                         double mass, double gdof, double m2, int quad, int nmu,
                         int interp, const double *f, double *gain,
                         double *loss, double *C)
{
    or_collision_direct_q(n, p, dp_override, mass, gdof, m2, quad, nmu, interp, 0, f,
                          gain, loss, C);
}

void or_collision_direct_q(int n, const double *p, const double *dp_override,
                           double mass, double gdof, double m2, int quad, int nmu,
                           int interp, int eta, const double *f, double *gain,
                           double *loss, double *C)
{
    const double floor_ = 1e-300;
    double *dp = malloc(sizeof(double) * n), *E = malloc(sizeof(double) * n);
    double *K = malloc(sizeof(double) * n), *h = malloc(sizeof(double) * n);
    double *xmu = malloc(sizeof(double) * (nmu > 0 ? nmu : 1));
    double *wmu = malloc(sizeof(double) * (nmu > 0 ? nmu : 1));
    or_grid(n, p, mass, dp_override, dp, E, K, h);
    if (nmu > 0)
        or_gauss_legendre(nmu, xmu, wmu);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n; ++i) {
        double g = 0.0, l = 0.0;
        for (int a = 0; a < n; ++a) {
            for (int b = 0; b < n; ++b) {
                int jl;
                double wr;
                double W = or_weight(n, p, dp, E, K, mass, gdof, m2, quad, nmu,
                                     xmu, wmu, i, a, b, &jl, &wr);
                if (jl < 0)
                    continue;
                double ft;
                if (interp == 0) {
                    ft = (1.0 - wr) * f[jl] + wr * f[jl + 1];
                } else {
                    double fl = f[jl] > floor_ ? f[jl] : floor_;
                    double fr = f[jl + 1] > floor_ ? f[jl + 1] : floor_;
                    ft = exp((1.0 - wr) * log(fl) + wr * log(fr));
                }
                g += W * f[a] * f[b] * (1.0 + eta * f[i]) * (1.0 + eta * ft);
                l += W * f[i] * ft * (1.0 + eta * f[a]) * (1.0 + eta * f[b]);
            }
        }
        gain[i] = g;
        loss[i] = l;
        C[i] = g - l;
    }
    free(dp); free(E); free(K); free(h); free(xmu); free(wmu);
}

/* ------------------------------------------------------------------------ */
/* The same operator from the precomputed tensors (linear interpolation):   */
/* gain_i = sum_{n,m} A_inm f_n f_m, loss_i = f_i sum_j R_ij f_j.           */
/* f holds nb distributions of length n, row-major.                         */
/* ------------------------------------------------------------------------ */
void or_collision_ar(int n, int nb, const double *A, const double *R,
                     const double *f, double *gain, double *loss, double *C)
{
    for (int bb = 0; bb < nb; ++bb) {
        const double *fb = f + (size_t)bb * n;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            double g = 0.0;
            for (int a = 0; a < n; ++a) {
                const double *row = A + ((size_t)i * n + a) * n;
                double s = 0.0;
                for (int b = 0; b < n; ++b)
                    s += row[b] * fb[b];
                g += fb[a] * s;
            }
            double r = 0.0;
            for (int j = 0; j < n; ++j)
                r += R[(size_t)i * n + j] * fb[j];
            double l = fb[i] * r;
            if (gain) gain[(size_t)bb * n + i] = g;
            if (loss) loss[(size_t)bb * n + i] = l;
            C[(size_t)bb * n + i] = g - l;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Two-moment projection (App. C, eqs. app_self_projection and              */
/* app_projection_system): support weights xi_i = |f_i|/f_max above        */
/* eps_supp, the 2x2 system in (alpha, beta) with A00, A01, A11 and the raw */
/* residuals R0, R1, and C_proj = C_raw - xi (alpha + beta E).              */
/* Diagnostics (eqs. app_epsilon_definition, app_projection_relative_       */
/* correction): diag = {alpha, beta, eps_N_raw, eps_E_raw, eps_N_proj,      */
/* eps_E_proj, R_N, R_E}.  One distribution.                                */
/* ------------------------------------------------------------------------ */
void or_project(int n, const double *h, const double *E, const double *f,
                const double *craw, double eps_supp, double *cproj,
                double *diag)
{
    double fmax = 0.0;
    for (int i = 0; i < n; ++i)
        if (fabs(f[i]) > fmax)
            fmax = fabs(f[i]);
    double A00 = 0, A01 = 0, A11 = 0, R0 = 0, R1 = 0;
    double *xi = malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) {
        double r = fmax > 0.0 ? fabs(f[i]) / fmax : 0.0;
        xi[i] = r > eps_supp ? r : 0.0;
        A00 += h[i] * xi[i];
        A01 += h[i] * E[i] * xi[i];
        A11 += h[i] * E[i] * E[i] * xi[i];
        R0 += h[i] * craw[i];
        R1 += h[i] * E[i] * craw[i];
    }
    double det = A00 * A11 - A01 * A01;
    double alpha = 0.0, beta = 0.0;
    if (det != 0.0) {
        alpha = (R0 * A11 - R1 * A01) / det;
        beta = (R1 * A00 - R0 * A01) / det;
    }
    double nr = 0, dr = 0, ner = 0, der = 0, np_ = 0, nep = 0, cn = 0, ce = 0;
    for (int i = 0; i < n; ++i) {
        cproj[i] = craw[i] - xi[i] * (alpha + beta * E[i]);
        nr += h[i] * craw[i];
        dr += h[i] * fabs(craw[i]);
        ner += h[i] * E[i] * craw[i];
        der += h[i] * E[i] * fabs(craw[i]);
        np_ += h[i] * cproj[i];
        nep += h[i] * E[i] * cproj[i];
        cn += h[i] * fabs(cproj[i] - craw[i]);
        ce += h[i] * E[i] * fabs(cproj[i] - craw[i]);
    }
    double dp_ = 0, dep = 0;
    for (int i = 0; i < n; ++i) {
        dp_ += h[i] * fabs(cproj[i]);
        dep += h[i] * E[i] * fabs(cproj[i]);
    }
    if (diag) {
        diag[0] = alpha;
        diag[1] = beta;
        diag[2] = dr > 0 ? nr / dr : 0.0;
        diag[3] = der > 0 ? ner / der : 0.0;
        diag[4] = dp_ > 0 ? np_ / dp_ : 0.0;
        diag[5] = dep > 0 ? nep / dep : 0.0;
        diag[6] = dr > 0 ? cn / dr : 0.0;
        diag[7] = der > 0 ? ce / der : 0.0;
    }
    free(xi);
}

/* ------------------------------------------------------------------------ */
/* Discrete moments (App. B): number sum h f, energy sum h E f, and the     */
/* Boltzmann entropy S = -sum h f (ln f - 1) over bins with f > 0.          */
/* ------------------------------------------------------------------------ */
void or_moments(int n, const double *h, const double *E, const double *f,
                double *out3)
{
    double N = 0, En = 0, S = 0;
    for (int i = 0; i < n; ++i) {
        N += h[i] * f[i];
        En += h[i] * E[i] * f[i];
        if (f[i] > 0.0)
            S -= h[i] * f[i] * (log(f[i]) - 1.0);
    }
    out3[0] = N;
    out3[1] = En;
    out3[2] = S;
}

/* Right-hand side lambda * C[f] of df/dt = lambda C (projected or raw). */
static void rhs_static(int n, const double *A, const double *R, const double *h,
                       const double *E, const double *f, double lambda,
                       int project, double *out, double *tmp)
{
    or_collision_ar(n, 1, A, R, f, NULL, NULL, tmp);
    if (project)
        or_project(n, h, E, f, tmp, 1e-12, out, NULL);
    else
        memcpy(out, tmp, sizeof(double) * n);
    for (int i = 0; i < n; ++i)
        out[i] *= lambda;
}

/* ------------------------------------------------------------------------ */
/* Fixed-step classical RK4 (Sec. 4.2) on df/dt = lambda C_proj[f] without  */
/* expansion; f is advanced in place by nsteps steps of size dt.  If traj   */
/* is given, it receives f after every step ((nsteps) x n).                 */
/* ------------------------------------------------------------------------ */
void or_rk4(int n, const double *A, const double *R, const double *h,
            const double *E, double *f, double lambda, double dt, int nsteps,
            int project, double *traj)
{
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *k3 = malloc(sizeof(double) * n), *k4 = malloc(sizeof(double) * n);
    double *y = malloc(sizeof(double) * n), *tmp = malloc(sizeof(double) * n);
    for (int s = 0; s < nsteps; ++s) {
        rhs_static(n, A, R, h, E, f, lambda, project, k1, tmp);
        for (int i = 0; i < n; ++i) y[i] = f[i] + 0.5 * dt * k1[i];
        rhs_static(n, A, R, h, E, y, lambda, project, k2, tmp);
        for (int i = 0; i < n; ++i) y[i] = f[i] + 0.5 * dt * k2[i];
        rhs_static(n, A, R, h, E, y, lambda, project, k3, tmp);
        for (int i = 0; i < n; ++i) y[i] = f[i] + dt * k3[i];
        rhs_static(n, A, R, h, E, y, lambda, project, k4, tmp);
        for (int i = 0; i < n; ++i)
            f[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        if (traj)
            memcpy(traj + (size_t)s * n, f, sizeof(double) * n);
    }
    free(k1); free(k2); free(k3); free(k4); free(y); free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Hubble drift of the fBE (eq. fbe) on a fixed physical grid.  In          */
/* u = ln a the redshift term is d_u f = d_{ln p} f; it is discretised in   */
/* conservative upwind form on g_i = a^3 p_i^3 f_i (comoving number per     */
/* unit ln p), with cell sizes V_i = Delta p_i / p_i (the same measure as   */
/* the moment weights h_i, so that drift and collisions conserve the same   */
/* sum_i V_i g_i):                                                          */
/*   V_i dg_i/du = g_{i+1} - g_i  (i < N-1),   V_{N-1} dg/du = -g_{N-1},    */
/* nothing enters through p_max, and g_0 per unit u leaves through p_min.   */
/* Writes dg/du into out; returns the outflow rate g_0.                     */
/* ------------------------------------------------------------------------ */
double or_drift(int n, const double *p, const double *dp, const double *g,
                double *out)
{
    for (int i = 0; i < n; ++i) {
        double V = dp[i] / p[i];
        double next = (i + 1 < n) ? g[i + 1] : 0.0;
        out[i] = (next - g[i]) / V;
    }
    return g[0];
}

/* Right-hand side in u = ln a (eq. numerical_evolution_loga) for the state
 * x: with expansion, x = g = a^3 p^3 f and
 *   dg/du = drift + a^3 p^3 lambda C[f] / H(u),  H = H_i e^{-2u} (radiation),
 * without expansion x = f and dx/du = lambda C[f] / H_i (u is then t H_i). */
static double rhs_u(int n, const double *A, const double *R, const double *p,
                    const double *dp, const double *h, const double *E,
                    const double *x, double u, double lambda, double Hi,
                    int expansion, int project, double *out, double *f,
                    double *c, double *tmp)
{
    if (!expansion) {
        rhs_static(n, A, R, h, E, x, lambda / Hi, project, out, tmp);
        return 0.0;
    }
    double a3 = exp(3.0 * u);
    for (int i = 0; i < n; ++i)
        f[i] = x[i] / (a3 * p[i] * p[i] * p[i]);
    rhs_static(n, A, R, h, E, f, lambda, project, c, tmp);
    double outflow = or_drift(n, p, dp, x, out);
    double H = Hi * exp(-2.0 * u);
    for (int i = 0; i < n; ++i)
        out[i] += a3 * p[i] * p[i] * p[i] * c[i] / H;
    return outflow;
}

/* ------------------------------------------------------------------------ */
/* Adaptive Heun in u (Sec. 4.2): Euler predictor x* = x + dt k1, trapezoid */
/* corrector x_new = x + dt (k1 + k2)/2 with k2 = rhs(u+dt, x*), and the    */
/* predictor-corrector difference as the local error estimate:             */
/*   err = max_i |x_new - x*| / (atol + rtol max(|x_i|, |x_new_i|)),        */
/* accept iff err <= 1; next dt = dt * clamp(safety err^{-1/2}, fmin, fmax). */
/* The step is clipped to end exactly at u_end.  Two operator calls per     */
/* attempted step.  With nreplay > 0 the steps are not adapted: dt_k is     */
/* taken from replay_dt and always accepted.  Records accepted (u_k, dt_k). */
/* Returns the number of accepted steps; *outflow accumulates the drift     */
/* outflow (trapezoid in u, consistent with the Heun update).  With att_dt  */
/* given, the first att_cap attempts are logged (dt, err, accepted) and    */
/* *n_att receives the number of attempts made.                            */
/* ------------------------------------------------------------------------ */
int or_heun(int n, const double *A, const double *R, const double *p,
            const double *dp_override, double mass, double *x, int expansion,
            int project, double lambda, double Hi, double u0, double u_end,
            double dt0, double rtol, double atol, double safety, double fmin,
            double fmax, int max_steps, int nreplay, const double *replay_dt,
            double *acc_u, double *acc_dt, double *outflow, int *nrejected,
            int att_cap, double *att_dt, double *att_err, int *att_ok, int *n_att)
{
    double *dp = malloc(sizeof(double) * n), *E = malloc(sizeof(double) * n);
    double *K = malloc(sizeof(double) * n), *h = malloc(sizeof(double) * n);
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *xs = malloc(sizeof(double) * n), *xn = malloc(sizeof(double) * n);
    double *f = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n);
    double *tmp = malloc(sizeof(double) * n);
    or_grid(n, p, mass, dp_override, dp, E, K, h);
    double u = u0, dt = dt0;
    int acc = 0, rej = 0, natt = 0;
    double out = 0.0;
    int limit = nreplay > 0 ? nreplay : max_steps;
    while (acc < limit) {
        if (nreplay > 0) {
            dt = replay_dt[acc];
        } else {
            if (!(u < u_end))
                break;
            if (u + dt > u_end)
                dt = u_end - u;
        }
        double o1 = rhs_u(n, A, R, p, dp, h, E, x, u, lambda, Hi, expansion,
                          project, k1, f, c, tmp);
        for (int i = 0; i < n; ++i)
            xs[i] = x[i] + dt * k1[i];
        double o2 = rhs_u(n, A, R, p, dp, h, E, xs, u + dt, lambda, Hi,
                          expansion, project, k2, f, c, tmp);
        double err = 0.0;
        for (int i = 0; i < n; ++i) {
            xn[i] = x[i] + 0.5 * dt * (k1[i] + k2[i]);
            double sc = atol + rtol * (fabs(x[i]) > fabs(xn[i]) ? fabs(x[i]) : fabs(xn[i]));
            double e = fabs(xn[i] - xs[i]) / sc;
            if (e > err)
                err = e;
        }
        if (att_dt && natt < att_cap) {
            att_dt[natt] = dt;
            att_err[natt] = err;
            att_ok[natt] = (nreplay > 0 || err <= 1.0);
        }
        ++natt;
        if (nreplay > 0 || err <= 1.0) {
            if (acc_u) acc_u[acc] = u;
            if (acc_dt) acc_dt[acc] = dt;
            out += 0.5 * dt * (o1 + o2);
            u += dt;
            memcpy(x, xn, sizeof(double) * n);
            ++acc;
        } else {
            ++rej;
        }
        if (nreplay == 0) {
            double fac = err > 0.0 ? safety / sqrt(err) : fmax;
            if (fac < fmin) fac = fmin;
            if (fac > fmax) fac = fmax;
            dt *= fac;
        }
    }
    if (outflow) *outflow = out;
    if (nrejected) *nrejected = rej;
    if (n_att) *n_att = natt;
    free(dp); free(E); free(K); free(h); free(k1); free(k2); free(xs);
    free(xn); free(f); free(c); free(tmp);
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Freeze-in sources of the two-source scenario (Sec. 3), in the code's     */
/* units: f as in the moments sum_i h_i f_i = (2 pi^2 / g) n, so a number   */
/* density n enters as nu = (2 pi^2 / g) n, and time in units where H at    */
/* u = ln a = 0 is H_i (radiation era, H = H_i e^{-2u}, t = e^{2u}/(2H_i)). */
/*                                                                          */
/* Cold condensate, eq. C_condensate_decay: C = (2 pi^2/g) 2 Gamma n_Phi    */
/* delta(p - p0)/p0^2, i.e. 2 Gamma nu_Phi particles per unit time and      */
/* volume at momentum p0.  nu_Phi follows d(nu a^3)/dt = -Gamma nu a^3 (the */
/* decay law of the condensate, dn/dt + 3Hn = -Gamma n), whose solution in  */
/* the radiation era is                                                      */
/*   a^3 nu_Phi(u) = N0 exp(-(Gamma / (2 H_i)) (e^{2u} - 1)),               */
/* N0 = a^3 nu_Phi at u = 0.                                                 */
/* Reading of the delta on the grid: the injection is shared between the    */
/* two nodes that bracket p0 in kinetic energy, with the energy-linear      */
/* weights of eq. app_interp_weights, w_{j+1} = (K0 - K_j)/(K_{j+1} - K_j), */
/* w_j = 1 - w_{j+1}, each divided by h_j: then sum_i h_i C_i = 2 Gamma nu  */
/* and sum_i h_i E_i C_i = E0 2 Gamma nu exactly (E0 = sqrt(p0^2+m^2) =     */
/* m_Phi/2 for Phi -> chi chi), the two injection moments of Sec. 3.        */
/* Returns j (or -1 when p0 lies outside the grid) and the two weights.     */
/* ------------------------------------------------------------------------ */
int or_deposit(int n, const double *p, double mass, double p0, double *wl,
               double *wr)
{
    double K0 = p0 * p0 / (sqrt(p0 * p0 + mass * mass) + mass);
    double Kf = p[0] * p[0] / (sqrt(p[0] * p[0] + mass * mass) + mass);
    double Kl = p[n - 1] * p[n - 1] / (sqrt(p[n - 1] * p[n - 1] + mass * mass) + mass);
    if (!(K0 >= Kf && K0 <= Kl))
        return -1;
    int j = 0;
    for (int q = 0; q < n - 1; ++q) {
        double Kq = p[q] * p[q] / (sqrt(p[q] * p[q] + mass * mass) + mass);
        if (Kq <= K0)
            j = q;
    }
    double Kj = p[j] * p[j] / (sqrt(p[j] * p[j] + mass * mass) + mass);
    double Kj1 = p[j + 1] * p[j + 1] / (sqrt(p[j + 1] * p[j + 1] + mass * mass) + mass);
    *wr = (K0 - Kj) / (Kj1 - Kj);
    *wl = 1.0 - *wr;
    return j;
}

double or_condensate_a3nu(double N0, double Gamma, double Hi, double u)
{
    return N0 * exp(-(Gamma / (2.0 * Hi)) * (exp(2.0 * u) - 1.0));
}

/* Higgs decay h -> chi chi in the thermal bath, eq. C_higgs_decay:         */
/*   C(p) = kappa (T / (E p)) (exp(-E_-/T) - exp(-E_+/T)),                  */
/*   E_+- = (m_h^2 E +- m_h p sqrt(m_h^2 - 4 m^2)) / (2 m^2),               */
/* kappa = (lambda_Hchi v)^2 / (8 pi g) in the code's units.  Reading of    */
/* the bath temperature (the paper does not print T(a)): T = T_i e^{-u},    */
/* the radiation era with a constant number of relativistic species, the    */
/* same era as H = H_i e^{-2u}.  The difference of exponentials is taken as */
/* exp(-E_-/T) (1 - exp(-(E_+ - E_-)/T)) with the second factor by expm1.   */
static double higgs_source(double p, double E, double mass, double kappa,
                           double mh, double T)
{
    double kh = sqrt(mh * mh - 4.0 * mass * mass);
    double m2x2 = 2.0 * mass * mass;
    double Em = (mh * mh * E - mh * p * kh) / m2x2;
    double dE = 2.0 * mh * p * kh / m2x2;                  /* E_+ - E_- */
    return kappa * (T / (E * p)) * exp(-Em / T) * (-expm1(-dE / T));
}

/* Source vector S_i(u) (both channels) in the units of C. */
void or_sources(int n, const double *p, const double *h, const double *E,
                double mass, double u, double Hi, double N0, double Gamma,
                int jdep, double wl, double wr, double kappa, double mh,
                double Ti, double *S)
{
    for (int i = 0; i < n; ++i)
        S[i] = 0.0;
    if (kappa > 0.0) {
        double T = Ti * exp(-u);
        for (int i = 0; i < n; ++i)
            S[i] += higgs_source(p[i], E[i], mass, kappa, mh, T);
    }
    if (N0 > 0.0 && jdep >= 0) {
        double nu = exp(-3.0 * u) * or_condensate_a3nu(N0, Gamma, Hi, u);
        S[jdep] += 2.0 * Gamma * nu * wl / h[jdep];
        S[jdep + 1] += 2.0 * Gamma * nu * wr / h[jdep + 1];
    }
}

/* Effective self-scattering rate Gamma_22 = n <sigma v> (Sec. 4.2): the    */
/* per-particle loss rate lambda sum_j R_ij f_j averaged over the particles */
/* of f, lambda sum_i h_i f_i (R f)_i / sum_i h_i f_i (0 for f = 0).        */
double or_gamma22(int n, const double *R, const double *h, const double *f,
                  double lambda)
{
    double num = 0.0, den = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = 0.0;
        for (int j = 0; j < n; ++j)
            r += R[(size_t)i * n + j] * f[j];
        num += h[i] * f[i] * r;
        den += h[i] * f[i];
    }
    return den > 0.0 ? lambda * num / den : 0.0;
}

/* Right-hand side of the freeze-in run in u for g = a^3 p^3 f:            */
/*   dg/du = drift + a^3 p^3 (coll lambda C[f] + S(u)) / H(u),              */
/* C projected if asked; coll = 0 in the source-only regime.  Returns the   */
/* outflow rate g_0 of the drift.                                           */
static double rhs_fi(int n, const double *A, const double *R, const double *p,
                     const double *dp, const double *h, const double *E,
                     double mass, const double *x, double u, double lambda,
                     double Hi, int coll, int project, double N0, double Gamma,
                     int jdep, double wl, double wr, double kappa, double mh,
                     double Ti, double *out, double *f, double *c, double *S,
                     double *tmp)
{
    double a3 = exp(3.0 * u);
    for (int i = 0; i < n; ++i)
        f[i] = x[i] / (a3 * p[i] * p[i] * p[i]);
    if (coll)
        rhs_static(n, A, R, h, E, f, lambda, project, c, tmp);
    else
        for (int i = 0; i < n; ++i)
            c[i] = 0.0;
    or_sources(n, p, h, E, mass, u, Hi, N0, Gamma, jdep, wl, wr, kappa, mh, Ti, S);
    double outflow = or_drift(n, p, dp, x, out);
    double H = Hi * exp(-2.0 * u);
    for (int i = 0; i < n; ++i)
        out[i] += a3 * p[i] * p[i] * p[i] * (c[i] + S[i]) / H;
    return outflow;
}

/* ------------------------------------------------------------------------ */
/* The two regimes of Sec. 4.2 for a freeze-in run, from u0 to u_end:       */
/*  1. source-only: elastic operator off, classical RK4 on fixed steps du   */
/*     in u (the sources are smooth); before each step the effective rate   */
/*     Gamma_22 of the current f is compared with H(u);                     */
/*  2. from the first state with Gamma_22 / H > eps_switch on: the elastic  */
/*     operator is on and the adaptive Heun of or_heun advances the state   */
/*     (first step dt0; in replay mode the dt list of this regime), with    */
/*     atol = atol_rel max_i |x_i| of the state at the switch (a run that   */
/*     starts from f = 0 has no scale before the sources act).               */
/* The source-only step is clipped to end at u_end.  Counts: *n_src steps  */
/* in regime 1, u_switch (u_end if never switched), the accepted regime-2  */
/* steps (returned; their (u, dt) in acc_u/acc_dt), rejections, outflow    */
/* (RK4 weights in regime 1, trapezoid in regime 2).  max_steps caps the   */
/* accepted steps of both regimes together.                                */
/* ------------------------------------------------------------------------ */
int or_freeze_in(int n, const double *A, const double *R, const double *p,
                 const double *dp_override, double mass, double *x, int project,
                 double lambda, double Hi, double u0, double u_end, double du,
                 double eps_switch, double N0, double Gamma, double p0,
                 double kappa, double mh, double Ti, double dt0, double rtol,
                 double atol_rel, double safety, double fmin, double fmax,
                 int max_steps, int nreplay, const double *replay_dt,
                 double *acc_u, double *acc_dt, int *n_src, double *u_switch,
                 double *outflow, int *nrejected)
{
    double *dp = malloc(sizeof(double) * n), *E = malloc(sizeof(double) * n);
    double *K = malloc(sizeof(double) * n), *h = malloc(sizeof(double) * n);
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *k3 = malloc(sizeof(double) * n), *k4 = malloc(sizeof(double) * n);
    double *y = malloc(sizeof(double) * n), *xn = malloc(sizeof(double) * n);
    double *f = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n);
    double *S = malloc(sizeof(double) * n), *tmp = malloc(sizeof(double) * n);
    or_grid(n, p, mass, dp_override, dp, E, K, h);
    double wl = 0.0, wr = 0.0;
    int jdep = N0 > 0.0 ? or_deposit(n, p, mass, p0, &wl, &wr) : -1;
    double u = u0, out = 0.0;
    int steps = 0, nsrc = 0, rej = 0, acc = 0, coll = 0;
    *u_switch = u_end;
#define RHS(xx, uu, kk, cc) rhs_fi(n, A, R, p, dp, h, E, mass, xx, uu, lambda, Hi, cc, \
                                   project, N0, Gamma, jdep, wl, wr, kappa, mh, Ti, kk, \
                                   f, c, S, tmp)
    /* regime 1 */
    while (u < u_end && (max_steps <= 0 || steps < max_steps)) {
        double a3 = exp(3.0 * u);
        for (int i = 0; i < n; ++i)
            f[i] = x[i] / (a3 * p[i] * p[i] * p[i]);
        double H = Hi * exp(-2.0 * u);
        if (or_gamma22(n, R, h, f, lambda) / H > eps_switch) {
            coll = 1;
            *u_switch = u;
            break;
        }
        double d = u + du > u_end ? u_end - u : du;
        double o1 = RHS(x, u, k1, 0);
        for (int i = 0; i < n; ++i) y[i] = x[i] + 0.5 * d * k1[i];
        double o2 = RHS(y, u + 0.5 * d, k2, 0);
        for (int i = 0; i < n; ++i) y[i] = x[i] + 0.5 * d * k2[i];
        double o3 = RHS(y, u + 0.5 * d, k3, 0);
        for (int i = 0; i < n; ++i) y[i] = x[i] + d * k3[i];
        double o4 = RHS(y, u + d, k4, 0);
        for (int i = 0; i < n; ++i)
            x[i] += d / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        out += d / 6.0 * (o1 + 2.0 * o2 + 2.0 * o3 + o4);
        u += d;
        ++steps;
        ++nsrc;
    }
    /* regime 2: adaptive (or replayed) Heun with the elastic operator */
    double dt = dt0, atol = 0.0;
    for (int i = 0; i < n; ++i)
        if (fabs(x[i]) > atol)
            atol = fabs(x[i]);
    atol *= atol_rel;
    if (!(atol > 0.0))
        atol = 1e-300;
    int limit = nreplay > 0 ? nreplay : (max_steps > 0 ? max_steps - steps : 0x7fffffff);
    while (coll && acc < limit) {
        if (nreplay > 0) {
            dt = replay_dt[acc];
        } else {
            if (!(u < u_end))
                break;
            if (u + dt > u_end)
                dt = u_end - u;
        }
        double o1 = RHS(x, u, k1, 1);
        for (int i = 0; i < n; ++i) y[i] = x[i] + dt * k1[i];
        double o2 = RHS(y, u + dt, k2, 1);
        double err = 0.0;
        for (int i = 0; i < n; ++i) {
            xn[i] = x[i] + 0.5 * dt * (k1[i] + k2[i]);
            double sc = atol + rtol * (fabs(x[i]) > fabs(xn[i]) ? fabs(x[i]) : fabs(xn[i]));
            double e = fabs(xn[i] - y[i]) / sc;
            if (e > err)
                err = e;
        }
        if (nreplay > 0 || err <= 1.0) {
            if (acc_u) acc_u[acc] = u;
            if (acc_dt) acc_dt[acc] = dt;
            out += 0.5 * dt * (o1 + o2);
            u += dt;
            memcpy(x, xn, sizeof(double) * n);
            ++acc;
        } else {
            ++rej;
        }
        if (nreplay == 0) {
            double fac = err > 0.0 ? safety / sqrt(err) : fmax;
            if (fac < fmin) fac = fmin;
            if (fac > fmax) fac = fmax;
            dt *= fac;
        }
    }
#undef RHS
    *n_src = nsrc;
    if (outflow) *outflow = out;
    if (nrejected) *nrejected = rej;
    free(dp); free(E); free(K); free(h); free(k1); free(k2); free(k3); free(k4);
    free(y); free(xn); free(f); free(c); free(S); free(tmp);
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Comoving grid (Sec. 4.1): the distribution lives on fixed comoving      */
/* momenta q_i (p = q / a); at scale factor a = e^u the operator is the     */
/* one of the physical grid p_i = q_i / a with widths dp_i = dq_i / a (the  */
/* trapezoid-in-ln rule gives exactly that), so the kernel tensors depend   */
/* on a.  Two readings of how a time integrator obtains them:               */
/*  - exact: the tensors of the grid q / a, rebuilt at every a;             */
/*  - tabulated: the tensors at J nodes u_j = u_min + j du of ln a, and     */
/*    at u in [u_j, u_j+1] the operator of the linear mix                   */
/*    (1 - w) {A, R}(u_j) + w {A, R}(u_j+1), w = (u - u_j) / du, which is   */
/*    (1 - w) C_j[f] + w C_j+1[f] since C is linear in A and R.             */
/* The projection (App. C) always uses h and E of the grid q / a at u      */
/* itself.  ntab = 0 selects the exact reading.                             */
/* ------------------------------------------------------------------------ */
void or_comoving_tensors(int n, const double *q, double u, double mass, double gdof,
                         double m2, int quad, int nmu, double *A, double *R)
{
    double *p = malloc(sizeof(double) * n);
    double a = exp(u);
    for (int i = 0; i < n; ++i)
        p[i] = q[i] / a;
    or_kernel_build(n, p, NULL, mass, gdof, m2, quad, nmu, A, R, NULL, NULL);
    free(p);
}

/* Raw comoving operator C_raw[f] at u (exact or tabulated, see above);   */
/* tabA [ntab][n][n][n], tabR [ntab][n][n] hold the node tensors.          */
static void comoving_raw(int n, const double *q, double u, double mass, double gdof,
                         double m2, int quad, int nmu, int ntab, double umin, double du,
                         const double *tabA, const double *tabR, const double *f,
                         double *C, double *A, double *R, double *tmp)
{
    size_t n3 = (size_t)n * n * n, n2 = (size_t)n * n;
    if (ntab <= 0) {
        or_comoving_tensors(n, q, u, mass, gdof, m2, quad, nmu, A, R);
        or_collision_ar(n, 1, A, R, f, NULL, NULL, C);
        return;
    }
    double s = (u - umin) / du;
    int j = (int)floor(s);
    if (j < 0) j = 0;
    if (j > ntab - 2) j = ntab - 2;
    double w = s - j;
    or_collision_ar(n, 1, tabA + (size_t)j * n3, tabR + (size_t)j * n2, f, NULL, NULL, C);
    or_collision_ar(n, 1, tabA + (size_t)(j + 1) * n3, tabR + (size_t)(j + 1) * n2, f, NULL, NULL, tmp);
    for (int i = 0; i < n; ++i)
        C[i] = (1.0 - w) * C[i] + w * tmp[i];
}

/* Projected comoving operator at u: C_raw, then the projection with the  */
/* moment weights h and energies E of the grid q / a.                       */
void or_comoving_collision(int n, const double *q, double u, double mass, double gdof,
                           double m2, int quad, int nmu, int ntab, double umin, double du,
                           const double *tabA, const double *tabR, const double *f,
                           int project, double *C)
{
    size_t n3 = (size_t)n * n * n;
    double *A = ntab <= 0 ? malloc(sizeof(double) * n3) : NULL;
    double *R = ntab <= 0 ? malloc(sizeof(double) * n * n) : NULL;
    double *tmp = malloc(sizeof(double) * n), *raw = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *dp = malloc(sizeof(double) * n);
    double *E = malloc(sizeof(double) * n), *K = malloc(sizeof(double) * n);
    double *h = malloc(sizeof(double) * n);
    comoving_raw(n, q, u, mass, gdof, m2, quad, nmu, ntab, umin, du, tabA, tabR, f, raw, A, R, tmp);
    if (project) {
        double a = exp(u);
        for (int i = 0; i < n; ++i)
            p[i] = q[i] / a;
        or_grid(n, p, mass, NULL, dp, E, K, h);
        or_project(n, h, E, f, raw, 1e-12, C, NULL);
    } else {
        memcpy(C, raw, sizeof(double) * n);
    }
    free(A); free(R); free(tmp); free(raw); free(p); free(dp); free(E); free(K); free(h);
}

/* Adaptive (or replayed) Heun in u = ln a on the comoving grid, the state */
/* f itself (no drift term: q is fixed), dx/du = lambda C[f](u) / H(u),    */
/* H = H_i e^{-2u}; the controller of or_heun.  Returns the accepted steps, */
/* their (u, dt) in acc_u / acc_dt, rejections in *nrejected.               */
int or_heun_comoving(int n, const double *q, double mass, double gdof, double m2,
                     int quad, int nmu, int ntab, double umin, double du,
                     const double *tabA, const double *tabR, double *x, int project,
                     double lambda, double Hi, double u0, double u_end, double dt0,
                     double rtol, double atol, double safety, double fmin, double fmax,
                     int max_steps, int nreplay, const double *replay_dt, double *acc_u,
                     double *acc_dt, int *nrejected)
{
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *xs = malloc(sizeof(double) * n), *xn = malloc(sizeof(double) * n);
    double u = u0, dt = dt0;
    int acc = 0, rej = 0;
    int limit = nreplay > 0 ? nreplay : max_steps;
    while (acc < limit) {
        if (nreplay > 0) {
            dt = replay_dt[acc];
        } else {
            if (!(u < u_end))
                break;
            if (u + dt > u_end)
                dt = u_end - u;
        }
        or_comoving_collision(n, q, u, mass, gdof, m2, quad, nmu, ntab, umin, du, tabA, tabR,
                              x, project, k1);
        double H = Hi * exp(-2.0 * u);
        for (int i = 0; i < n; ++i) {
            k1[i] *= lambda / H;
            xs[i] = x[i] + dt * k1[i];
        }
        or_comoving_collision(n, q, u + dt, mass, gdof, m2, quad, nmu, ntab, umin, du, tabA,
                              tabR, xs, project, k2);
        double H2 = Hi * exp(-2.0 * (u + dt));
        double err = 0.0;
        for (int i = 0; i < n; ++i) {
            k2[i] *= lambda / H2;
            xn[i] = x[i] + 0.5 * dt * (k1[i] + k2[i]);
            double sc = atol + rtol * (fabs(x[i]) > fabs(xn[i]) ? fabs(x[i]) : fabs(xn[i]));
            double e = fabs(xn[i] - xs[i]) / sc;
            if (e > err)
                err = e;
        }
        if (nreplay > 0 || err <= 1.0) {
            if (acc_u) acc_u[acc] = u;
            if (acc_dt) acc_dt[acc] = dt;
            u += dt;
            memcpy(x, xn, sizeof(double) * n);
            ++acc;
        } else {
            ++rej;
        }
        if (nreplay == 0) {
            double fac = err > 0.0 ? safety / sqrt(err) : fmax;
            if (fac < fmin) fac = fmin;
            if (fac > fmax) fac = fmax;
            dt *= fac;
        }
    }
    if (nrejected) *nrejected = rej;
    free(k1); free(k2); free(xs); free(xn);
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Thread count of the OpenMP loops (timing of the oracle only).            */
/* ------------------------------------------------------------------------ */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int or_max_threads(void) { return omp_get_max_threads(); }
