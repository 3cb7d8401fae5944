/*
 * helios_ref.c -- plain FP64 CPU oracle of the HELIOS radiative-equilibrium
 * hot path (Malik et al. 2017, "HELIOS: an open-source, GPU-accelerated
 * radiative transfer code for self-consistent exoplanetary atmospheres").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library; the two
 * meet only in the seeded input arrays.
 *
 * Everything is double precision, cgs units, one atmosphere per call, in the
 * order and notation of the paper:
 *   grid ............ Sec. 2.2.1 (staggered non-isothermal grid, Fig. 2)
 *   sources / BCs ... Sec. 2.2.2 (stellar TOA flux, internal BOA flux)
 *   opacity ......... Sec. 2.3, eq:kappa_gauss, eq:mixing, table footnote
 *   two-stream ...... Sec. 2.1.3, eq:trans, eq:cap, eq:isoscat,
 *                     eq:nonisoscat, eq:purescat
 *   scattering iter.  Sec. 2.2.3 (Gauss-Seidel passes, warm start)
 *   g / lambda sums . Sec. 2.3 (Gauss-Legendre rule, eq:trans_gen)
 *   RE step ......... Sec. 2.2.3 eq:step, Sec. 2.2.4 (adaptive timestep,
 *                     oscillation control, eq:condition)
 *   exact solution .. Sec. 2.1.2 eq:isodirect, eq:nonisodirect,
 *                     eq:direct_trans, eq:diff (check mode only)
 *   isothermal grid . Sec. 2.2.1 (n isothermal layers, n + 1 interfaces)
 *   Rayleigh ........ Sec. 2.1.4 (H2 cross-section, scattering albedo)
 *
 * Where the paper leaves a point open, the reading taken is stated at the
 * place it applies.
 *
 * Parity unpinned: the oscillation-control window semantics and the
 * temperature floor (nothing in the paper fixes the trajectory), see the RE
 * step below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- constants
 * CODATA 2018 exact values in cgs.  The Stefan-Boltzmann constant is derived
 * from them (sigma = 2 pi^5 k^4 / (15 h^3 c^2)). */
#define REF_PI 3.14159265358979323846
static const double REF_H = 6.62607015e-27;  /* erg s   */
static const double REF_C = 2.99792458e10;   /* cm s^-1 */
static const double REF_K = 1.380649e-16;    /* erg K^-1 */

double ref_sigma_sb(void) {
    double k4 = REF_K * REF_K * REF_K * REF_K;
    return 2.0 * pow(REF_PI, 5) * k4 / (15.0 * REF_H * REF_H * REF_H * REF_C * REF_C);
}

/* ------------------------------------------------------- Gauss-Legendre rule
 * Sec. 2.3: the g-integral over [0,1] is (1/2) sum_g w_g psi((1+y_g)/2) with
 * y_g the roots of P_n and w_g = 2 / ((1-y_g^2) P_n'(y_g)^2).  Roots found by
 * Newton's method on the three-term Legendre recurrence.  Output: nodes on
 * [0,1] in ascending order and the halved weights (they sum to 1). */
int ref_gauss_legendre(int n, double* g_node, double* g_weight) {
    if (n < 1 || n > 256) return -1;
    for (int i = 0; i < n; ++i) {
        /* i-th root counted from +1 downwards */
        double y = cos(REF_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = y;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * y * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = y; p0 = 1.0; }
            /* P_n = p1, P_{n-1} = p0; derivative from the standard identity */
            dp = n * (y * p1 - p0) / (y * y - 1.0);
            double dy = p1 / dp;
            y -= dy;
            if (fabs(dy) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = y;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * y * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = y; p0 = 1.0; }
            dp = n * (y * p1 - p0) / (y * y - 1.0);
        }
        double w = 2.0 / ((1.0 - y * y) * dp * dp);
        /* descending y over i; store ascending */
        g_node[n - 1 - i] = 0.5 * (1.0 + y);
        g_weight[n - 1 - i] = 0.5 * w;
    }
    return 0;
}

/* ---------------------------------------------------------------- the grid
 * Sec. 2.2.1 and Fig. 2.  n layers with centre pressures P_c[0] (bottom) ..
 * P_c[n-1] (top).  Interfaces sit at the geometric mean of neighbouring
 * centres; the outer two are half a log-step beyond the outermost centres.
 * Points are interleaved bottom to top: point 2i is interface i, point 2i+1
 * is the centre of layer i; 2n+1 points, 2n sublayers. */
void ref_grid(int n, const double* P_c, double* P_pt) {
    for (int i = 0; i < n; ++i) P_pt[2 * i + 1] = P_c[i];
    for (int i = 1; i < n; ++i) P_pt[2 * i] = sqrt(P_c[i - 1] * P_c[i]);
    P_pt[0] = P_c[0] * sqrt(P_c[0] / P_c[1]);
    P_pt[2 * n] = P_c[n - 1] * sqrt(P_c[n - 1] / P_c[n - 2]);
}

/* Sec. 2.2.1: temperatures at the interfaces are interpolated from the layer
 * centres, here linearly in ln P; the outer interfaces take the adjacent
 * centre temperature. */
void ref_profile(int n, const double* P_pt, const double* T_c, double* T_pt) {
    for (int i = 0; i < n; ++i) T_pt[2 * i + 1] = T_c[i];
    for (int i = 1; i < n; ++i) {
        double x0 = log(P_pt[2 * i - 1]), x1 = log(P_pt[2 * i + 1]);
        double x = log(P_pt[2 * i]);
        double f = (x - x0) / (x1 - x0);
        T_pt[2 * i] = T_c[i - 1] + f * (T_c[i] - T_c[i - 1]);
    }
    T_pt[0] = T_c[0];
    T_pt[2 * n] = T_c[n - 1];
}

/* --------------------------------------------------------------- sources
 * Planck function per unit wavelength and solid angle, erg s^-1 cm^-2 sr^-1
 * cm^-1, evaluated at the bin's centre wavelength (Sec. 2.6 evaluates it at
 * the model's wavelength values). */
double ref_planck(double lambda, double T) {
    if (!(T > 0.0)) return 0.0;
    double x = REF_H * REF_C / (lambda * REF_K * T);
    return 2.0 * REF_H * REF_C * REF_C / pow(lambda, 5) / expm1(x);
}

/* Planck values of nb bins at npt temperatures: out[l * npt + p]. */
void ref_planck_table(int nb, int npt, const double* lambda, const double* T, double* out) {
    for (int l = 0; l < nb; ++l)
        for (int p = 0; p < npt; ++p) out[(size_t)l * npt + p] = ref_planck(lambda[l], T[p]);
}

/* Sec. 2.2.2.  TOA: F_down,n = f (R_star/a)^2 pi B_star(lambda); the workloads give the
 * irradiation temperature T_irr with sigma T_irr^4 = f (R_star/a)^2 sigma T_star^4, so
 * f (R_star/a)^2 = (T_irr/T_star)^4.  BOA: the internal flux pi B_int has the shape of
 * a blackbody at T_int and is scaled so that its integral over the model's
 * bins is sigma T_int^4 (the band does not cover all wavelengths). */
void ref_boundary(int nb, const double* lambda_c, const double* dlambda,
                  double T_star, double T_irr, double T_int,
                  double* F_top, double* F_int) {
    double dil = (T_star > 0.0) ? pow(T_irr / T_star, 4) : 0.0;
    double sum = 0.0;
    for (int l = 0; l < nb; ++l) {
        F_top[l] = dil * REF_PI * ref_planck(lambda_c[l], T_star);
        F_int[l] = REF_PI * ref_planck(lambda_c[l], T_int);
        sum += F_int[l] * dlambda[l];
    }
    double s = (sum > 0.0) ? ref_sigma_sb() * pow(T_int, 4) / sum : 0.0;
    for (int l = 0; l < nb; ++l) F_int[l] *= s;
}

/* --------------------------------------------------------------- opacity
 * eq:kappa_gauss with eq:mixing: kappa = sum_j X_j m_j / mbar * k_j(T, P).
 * Table mode: k_j is linear in T and in log10 P between table nodes
 * (bilinear on the linear k values); outside the table the nearest node
 * value is used (table footnote: coordinates are clamped).
 * k: [nsp][nT][nP][nbt][ng] float32; vmr: [nsp][npt]; kappa: [nb][ng][npt]. */
void ref_mix_table(int npt, const double* T_pt, const double* P_pt,
                   int nsp, const double* vmr, const double* mass, double mmw,
                   int nT, int nP, double T0, double dT, double lP0, double dlP,
                   int nbt, int ng, const float* k,
                   int nb, const int32_t* bin_index, double* kappa) {
    for (int p = 0; p < npt; ++p) {
        double x = (T_pt[p] - T0) / dT;
        double y = (log10(P_pt[p]) - lP0) / dlP;
        if (x < 0.0) x = 0.0;
        if (x > nT - 1) x = nT - 1;
        if (y < 0.0) y = 0.0;
        if (y > nP - 1) y = nP - 1;
        int iT = (int)floor(x), iP = (int)floor(y);
        if (iT > nT - 2) iT = nT - 2;
        if (iP > nP - 2) iP = nP - 2;
        double fT = x - iT, fP = y - iP;
        for (int l = 0; l < nb; ++l) {
            int bt = bin_index[l];
            for (int g = 0; g < ng; ++g) {
                double sum = 0.0;
                for (int j = 0; j < nsp; ++j) {
                    double X = vmr[(size_t)j * npt + p] * mass[j] / mmw; /* eq:mixing */
                    size_t base = (size_t)j * nT * nP;
                    double k00 = k[(((base + (size_t)iT * nP + iP) * nbt) + bt) * ng + g];
                    double k01 = k[(((base + (size_t)iT * nP + iP + 1) * nbt) + bt) * ng + g];
                    double k10 = k[(((base + (size_t)(iT + 1) * nP + iP) * nbt) + bt) * ng + g];
                    double k11 = k[(((base + (size_t)(iT + 1) * nP + iP + 1) * nbt) + bt) * ng + g];
                    double kj = (1 - fT) * (1 - fP) * k00 + (1 - fT) * fP * k01
                              + fT * (1 - fP) * k10 + fT * fP * k11;
                    sum += X * kj;
                }
                kappa[((size_t)l * ng + g) * npt + p] = sum;
            }
        }
    }
}

/* Power-law opacity of the plain workload: k_j = k0_j (P/P_ref)^a (T/T_ref)^b,
 * mixed the same way.  k0: [nsp][nbt][ng]. */
void ref_mix_powerlaw(int npt, const double* T_pt, const double* P_pt,
                      int nsp, const double* vmr, const double* mass, double mmw,
                      int nbt, int ng, const double* k0,
                      double p_exp, double t_exp, double P_ref, double T_ref,
                      int nb, const int32_t* bin_index, double* kappa) {
    for (int p = 0; p < npt; ++p) {
        double scale = pow(P_pt[p] / P_ref, p_exp) * pow(T_pt[p] / T_ref, t_exp);
        for (int l = 0; l < nb; ++l) {
            int bt = bin_index[l];
            for (int g = 0; g < ng; ++g) {
                double sum = 0.0;
                for (int j = 0; j < nsp; ++j) {
                    double X = vmr[(size_t)j * npt + p] * mass[j] / mmw;
                    sum += X * k0[((size_t)j * nbt + bt) * ng + g] * scale;
                }
                kappa[((size_t)l * ng + g) * npt + p] = sum;
            }
        }
    }
}

/* ----------------------------------------------- two-stream, one sublayer
 * A sublayer joins a lower end ("d", point s) and an upper end ("u", point
 * s+1).  F_up_d, F_dn_u are the incoming fluxes; the functions return the
 * outgoing upward flux at the upper end and downward flux at the lower end.
 *
 * eq:trans  T   = exp(-D sqrt((1-w0 g0)(1-w0)) dtau)
 * zeta_pm = (1 +- sqrt((1-w0)/(1-w0 g0)))/2
 * eq:cap    alpha = zm^2 T^2 - zp^2, beta = zp zm (1-T^2),
 *           xi = (zm^2 - zp^2) T,    ups = (zm^2 T + zp^2)(1-T)
 *
 * Branches (Sec. 2.1.4 and Sec. 2.2.1):
 *   (1 - w0) < 1e-6 ......... eq:purescat (tau0 = dtau)
 *   dtau < 1e-4 ............. eq:isoscat with the mean of the two end B
 *   otherwise ............... eq:nonisoscat
 * eq:nonisoscat is used with two readings (both established by direct
 * integration of the two-stream equations, see the tests): the Planck value
 * paired with the outgoing upward flux is that of the sublayer's upper end
 * and B' = (B_lower - B_upper)/dtau is the gradient in optical depth measured
 * downward; the factor multiplying B' is eps/(1 - w0 g0). */
typedef struct {
    double T, zp, zm, alpha, beta, xi, ups;
} ref_coeff;

static void ref_coeffs(double dtau, double w0, double g0, double D, ref_coeff* c) {
    c->T = exp(-D * sqrt((1.0 - w0 * g0) * (1.0 - w0)) * dtau);
    double r = sqrt((1.0 - w0) / (1.0 - w0 * g0));
    c->zp = 0.5 * (1.0 + r);
    c->zm = 0.5 * (1.0 - r);
    double T = c->T, zp = c->zp, zm = c->zm;
    c->alpha = zm * zm * T * T - zp * zp;
    c->beta = zp * zm * (1.0 - T * T);
    c->xi = (zm * zm - zp * zp) * T;
    c->ups = (zm * zm * T + zp * zp) * (1.0 - T);
}

enum { REF_BR_PURESCAT = 0, REF_BR_ISO = 1, REF_BR_NONISO = 2 };

int ref_branch(double dtau, double w0) {
    if (1.0 - w0 < 1e-6) return REF_BR_PURESCAT;
    if (dtau < 1e-4) return REF_BR_ISO;
    return REF_BR_NONISO;
}

double ref_sub_up(double dtau, double w0, double g0, double D,
                  double B_u, double B_d, double F_up_d, double F_dn_u) {
    double eps = 1.0 / D;
    int br = ref_branch(dtau, w0);
    if (br == REF_BR_PURESCAT) {
        double q = D * (1.0 - g0) * dtau;
        return F_up_d - q * (F_up_d - F_dn_u) / (2.0 + q);
    }
    ref_coeff c;
    ref_coeffs(dtau, w0, g0, D, &c);
    if (br == REF_BR_ISO) {
        double B = 0.5 * (B_u + B_d);
        return (c.xi * F_up_d - c.beta * F_dn_u + 2.0 * REF_PI * eps * B * (c.beta - c.ups)) / c.alpha;
    }
    double Bp = (B_d - B_u) / dtau;
    double f = eps / (1.0 - w0 * g0);
    return (c.xi * F_up_d - c.beta * F_dn_u
            + 2.0 * REF_PI * eps * (B_u * (c.alpha + c.beta) - B_d * c.xi
                                    + f * Bp * (c.alpha - c.xi - c.beta))) / c.alpha;
}

double ref_sub_down(double dtau, double w0, double g0, double D,
                    double B_u, double B_d, double F_up_d, double F_dn_u) {
    double eps = 1.0 / D;
    int br = ref_branch(dtau, w0);
    if (br == REF_BR_PURESCAT) {
        double q = D * (1.0 - g0) * dtau;
        return F_dn_u + q * (F_up_d - F_dn_u) / (2.0 + q);
    }
    ref_coeff c;
    ref_coeffs(dtau, w0, g0, D, &c);
    if (br == REF_BR_ISO) {
        double B = 0.5 * (B_u + B_d);
        return (c.xi * F_dn_u - c.beta * F_up_d + 2.0 * REF_PI * eps * B * (c.beta - c.ups)) / c.alpha;
    }
    double Bp = (B_d - B_u) / dtau;
    double f = eps / (1.0 - w0 * g0);
    return (c.xi * F_dn_u - c.beta * F_up_d
            + 2.0 * REF_PI * eps * (B_d * (c.alpha + c.beta) - B_u * c.xi
                                    + f * Bp * (c.xi - c.alpha + c.beta))) / c.alpha;
}

/* Transmission of one sublayer (eq:trans), exported for the tests. */
double ref_sub_trans(double dtau, double w0, double g0, double D) {
    ref_coeff c;
    ref_coeffs(dtau, w0, g0, D, &c);
    return c.T;
}

/* ------------------------------------------------------------- flux solve
 * One atmosphere: n layers, nb bins, ng g-points.
 * Inputs: P_pt, T_pt [npt]; kappa [nb][ng][npt] at the points; w0, g0
 * [nb][n] per layer and bin (shared by both sublayers and all g); bins'
 * centre wavelengths and widths; g weights (sum 1).
 * Sublayer s joins points s and s+1; its opacity is the mean of the two
 * point opacities (Sec. 2.3) and dtau = kappa_sub (P_s - P_{s+1}) / grav
 * (eq:layertau).
 * Scattering iterations (Sec. 2.2.3): 1 + n_scat Gauss-Seidel passes, each a
 * downward sweep from the TOA boundary followed by the BOA condition and an
 * upward sweep.  F_up holds the warm start on entry (zeros on the first
 * temperature step) and the final upward fluxes on exit; the downward sweep
 * only reads upward fluxes, so no downward warm start exists.
 * Outputs: F_dn [nb][ng][npt] (optional), per-bin g-quadrature F_up_bin,
 * F_dn_bin [nb][npt] (Sec. 2.3: the Gaussian sum is taken at the end of the
 * propagation), bolometric F_bol [npt][3] = (up, down, up - down) summed over
 * bins with their widths (Sec. 2.2.3).  Sums are Neumaier-compensated in a
 * fixed order. */
typedef struct { double s, c; } ref_acc;
static void ref_acc_add(ref_acc* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}


/* Gaussian sum at the end of the propagation, then the bin sum. */
static void ref_sums(int npt, int nb, int ng, const double* dlambda, const double* g_weight,
                     const double* F_up, const double* F_dn,
                     double* F_up_bin, double* F_dn_bin, double* F_bol) {
    for (int l = 0; l < nb; ++l) {
        for (int p = 0; p < npt; ++p) {
            ref_acc au = {0.0, 0.0}, ad = {0.0, 0.0};
            for (int g = 0; g < ng; ++g) {
                size_t idx = ((size_t)l * ng + g) * npt + p;
                ref_acc_add(&au, g_weight[g] * F_up[idx]);
                ref_acc_add(&ad, g_weight[g] * F_dn[idx]);
            }
            F_up_bin[(size_t)l * npt + p] = au.s + au.c;
            F_dn_bin[(size_t)l * npt + p] = ad.s + ad.c;
        }
    }
    for (int p = 0; p < npt; ++p) {
        ref_acc au = {0.0, 0.0}, ad = {0.0, 0.0};
        for (int l = 0; l < nb; ++l) {
            ref_acc_add(&au, dlambda[l] * F_up_bin[(size_t)l * npt + p]);
            ref_acc_add(&ad, dlambda[l] * F_dn_bin[(size_t)l * npt + p]);
        }
        F_bol[3 * p + 0] = au.s + au.c;
        F_bol[3 * p + 1] = ad.s + ad.c;
        F_bol[3 * p + 2] = F_bol[3 * p + 0] - F_bol[3 * p + 1];
    }
}

/* Optical depth, single-scattering albedo and asymmetry of sublayer s of
 * column (l, g).  Without Rayleigh scattering (kappa_R == NULL): the mean of
 * the two point opacities, and the layer's w0 and g0.  With it (Sec. 2.1.4):
 * the H2 scattering opacity kappa_R[l] is added to that mean, and the
 * sublayer scatters the fraction kappa_R / (total) of its extinction,
 * isotropically (g0 = 0); the given w0, g0 do not enter. */
static void ref_sub_optics(const double* kap, int s, double dm_s, const double* w0l, const double* g0l,
                           const double* kappa_R, int l, double* dtau, double* w0, double* g0) {
    double k_abs = 0.5 * (kap[s] + kap[s + 1]);
    if (!kappa_R) {
        *dtau = k_abs * dm_s;
        *w0 = w0l[s / 2];
        *g0 = g0l[s / 2];
        return;
    }
    double k_tot = k_abs + kappa_R[l];
    *dtau = k_tot * dm_s;
    *w0 = kappa_R[l] / k_tot;
    *g0 = 0.0;
}

static int ref_flux_core(int n, int nb, int ng,
                         const double* P_pt, double grav, const double* T_pt,
                         const double* lambda_c, const double* dlambda, const double* g_weight,
                         double T_star, double T_irr, double T_int,
                         const double* kappa, const double* w0, const double* g0, const double* kappa_R,
                         int n_scat, double D,
                         double* F_up, double* F_dn,
                         double* F_up_bin, double* F_dn_bin, double* F_bol,
                         int n_threads) {
    const int npt = 2 * n + 1;
    const size_t ncell = (size_t)nb * ng * npt;
    double* F_top = (double*)malloc(sizeof(double) * nb);
    double* F_int = (double*)malloc(sizeof(double) * nb);
    double* B = (double*)malloc(sizeof(double) * (size_t)nb * npt);
    double* dm = (double*)malloc(sizeof(double) * 2 * n);
    double* dn_all = F_dn ? F_dn : (double*)malloc(sizeof(double) * ncell);
    if (!F_top || !F_int || !B || !dm || !dn_all) {
        free(F_top); free(F_int); free(B); free(dm);
        if (!F_dn) free(dn_all);
        return -1;
    }
    ref_boundary(nb, lambda_c, dlambda, T_star, T_irr, T_int, F_top, F_int);
    for (int l = 0; l < nb; ++l)
        for (int p = 0; p < npt; ++p) B[(size_t)l * npt + p] = ref_planck(lambda_c[l], T_pt[p]);
    for (int s = 0; s < 2 * n; ++s) dm[s] = (P_pt[s] - P_pt[s + 1]) / grav; /* eq:layertau */
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int col = 0; col < nb * ng; ++col) {
        const int l = col / ng;
        const double* kap = kappa + (size_t)col * npt;
        const double* Bl = B + (size_t)l * npt;
        const double* w0l = w0 ? w0 + (size_t)l * n : NULL;
        const double* g0l = g0 ? g0 + (size_t)l * n : NULL;
        double* up = F_up + (size_t)col * npt;
        double* dn = dn_all + (size_t)col * npt;
        for (int pass = 0; pass <= n_scat; ++pass) {
            dn[2 * n] = F_top[l]; /* TOA boundary condition */
            for (int s = 2 * n - 1; s >= 0; --s) {
                double dtau, ws, gs;
                ref_sub_optics(kap, s, dm[s], w0l, g0l, kappa_R, l, &dtau, &ws, &gs);
                dn[s] = ref_sub_down(dtau, ws, gs, D, Bl[s + 1], Bl[s], up[s], dn[s + 1]);
            }
            up[0] = dn[0] + F_int[l]; /* BOA: pi B_int = F_up,0 - F_dn,0 */
            for (int s = 0; s < 2 * n; ++s) {
                double dtau, ws, gs;
                ref_sub_optics(kap, s, dm[s], w0l, g0l, kappa_R, l, &dtau, &ws, &gs);
                up[s + 1] = ref_sub_up(dtau, ws, gs, D, Bl[s + 1], Bl[s], up[s], dn[s + 1]);
            }
        }
    }
    ref_sums(npt, nb, ng, dlambda, g_weight, F_up, dn_all, F_up_bin, F_dn_bin, F_bol);
    free(F_top); free(F_int); free(B); free(dm);
    if (!F_dn) free(dn_all);
    return 0;
}

int ref_flux(int n, int nb, int ng,
             const double* P_pt, double grav, const double* T_pt,
             const double* lambda_c, const double* dlambda, const double* g_weight,
             double T_star, double T_irr, double T_int,
             const double* kappa, const double* w0, const double* g0,
             int n_scat, double D,
             double* F_up, double* F_dn,
             double* F_up_bin, double* F_dn_bin, double* F_bol,
             int n_threads) {
    return ref_flux_core(n, nb, ng, P_pt, grav, T_pt, lambda_c, dlambda, g_weight, T_star, T_irr, T_int,
                         kappa, w0, g0, NULL, n_scat, D, F_up, F_dn, F_up_bin, F_dn_bin, F_bol, n_threads);
}

/* ------------------------------------------- Rayleigh scattering by H2
 * Sec. 2.1.4.  Cross-section per molecule
 *   sigma = 24 pi^3 / (n_ref^2 lambda^4) ((n^2 - 1) / (n^2 + 2))^2 K
 * with, for H2, n_ref = 2.68678e19 cm^-3, King factor K = 1 and refractive
 * index n = 13.58e-5 (1 + 7.52e-11 cm^2 / lambda^2) + 1 (lambda in cm). */
double ref_rayleigh_h2(double lambda) {
    const double n_ref = 2.68678e19, K = 1.0;
    double nl = 13.58e-5 * (1.0 + 7.52e-11 / (lambda * lambda)) + 1.0;
    double f = (nl * nl - 1.0) / (nl * nl + 2.0);
    double l2 = lambda * lambda;
    return 24.0 * REF_PI * REF_PI * REF_PI / (n_ref * n_ref * l2 * l2) * f * f * K;
}

/* The flux solve of ref_flux with Rayleigh scattering by H2 added to the
 * given (absorption) opacities: kappa_R = sigma(lambda_c) / mbar per bin
 * (mbar in g), scattering albedo of each sublayer and g-point from the
 * ratio of scattering to total opacity, isotropic scattering (Sec. 2.1.4);
 * the pure-scattering form applies where (1 - w0) < 1e-6. */
int ref_flux_rayleigh(int n, int nb, int ng,
                      const double* P_pt, double grav, const double* T_pt,
                      const double* lambda_c, const double* dlambda, const double* g_weight,
                      double T_star, double T_irr, double T_int,
                      const double* kappa, double mbar,
                      int n_scat, double D,
                      double* F_up, double* F_dn,
                      double* F_up_bin, double* F_dn_bin, double* F_bol,
                      int n_threads) {
    double* kR = (double*)malloc(sizeof(double) * nb);
    if (!kR) return -1;
    for (int l = 0; l < nb; ++l) kR[l] = ref_rayleigh_h2(lambda_c[l]) / mbar;
    int rc = ref_flux_core(n, nb, ng, P_pt, grav, T_pt, lambda_c, dlambda, g_weight, T_star, T_irr, T_int,
                           kappa, NULL, NULL, kR, n_scat, D, F_up, F_dn, F_up_bin, F_dn_bin, F_bol, n_threads);
    free(kR);
    return rc;
}

/* ---------------------------------------------------------------- RE step
 * Sec. 2.2.3-2.2.4 for one atmosphere.  Layer i is bounded by interfaces at
 * points 2i (below) and 2i+2 (above); the centre fluxes are intermediate
 * (starred in Fig. 2) and do not enter.
 *
 *   dF_i   = F_net(2i+2) - F_net(2i)                  net-flux difference
 *   rho_i  = P_i mbar / (k T_i),  c_p = (2 + 5) k / (2 mbar)
 *   dz_i   = k T_i ln(P_int,i / P_int,i+1) / (mbar g)
 *   t_rad  = c_p P_i / (sigma g T_i^3)
 *   f_pre  = 1e5 / |dF_i|^0.9,   dt_i = m_i f_pre t_rad
 *   dT_i   = - dF_i dt_i / (rho_i c_p dz_i)
 *
 * Sign: with F_net = up - down and dz > 0, a layer whose net upward flux
 * grows across it loses energy and must cool, hence the minus sign (the
 * printed eq:step heats it; the tests show the printed sign diverges).
 * m_i is the per-layer timestep multiplier (Sec. 2.2.4): after each step the
 * sign of dT_i is pushed into a history of the last `window` signs.  Once the
 * history is full it is examined every step: if all signs agree (monotonic
 * change) m_i grows by `grow`; if the temperature oscillated over the whole
 * window (the sign alternated at every step) m_i shrinks by `shrink`; any
 * other pattern leaves m_i alone.  osc_any != 0 selects the alternative
 * reading in which any sign change in the window counts as oscillation.
 * Convergence (eq:condition) is tested first, on the fluxes handed in:
 * resid = max_i |dF_i| / norm_i with norm_i = sigma T_i^4 (paper) or
 * sigma T_int^4; if resid < tol nothing is updated and 1 is returned.
 * T is floored at T_floor.  Returns 0 after an update, 1 when converged, -5 on
 * a non-finite flux or temperature (nothing updated).
 *
 * hist[i] encodes the history: bits 0..15 hold the signs (bit 0 = most recent,
 * 1 = positive dT), bits 16.. hold how many signs were recorded (<= window). */
int ref_radeq(int n, const double* P_pt, const double* F_bol, double grav, double mmw_g,
              double T_int, double* T_c, double* m, int32_t* hist,
              double tol, int norm_sigma_tint, double T_floor, int window, int osc_any,
              double shrink, double grow, double fpre_c, double fpre_p, int deadband,
              double* resid) {
    if (window < 2 || window > 16) return -1;
    /* the grid of Sec. 2.2.1 runs from the bottom (highest pressure) to the
       top: a point pressure that is not positive, finite and below the one
       beneath it is no such grid, and the step refuses it */
    for (int p = 0; p < 2 * n + 1; ++p)
        if (!(P_pt[p] > 0.0) || !isfinite(P_pt[p]) || (p > 0 && !(P_pt[p] < P_pt[p - 1]))) {
            *resid = NAN;
            return -2;
        }
    const double sigma = ref_sigma_sb();
    double worst = 0.0;
    for (int i = 0; i < n; ++i) {
        double dF = F_bol[3 * (2 * i + 2) + 2] - F_bol[3 * (2 * i) + 2];
        if (!isfinite(dF) || !isfinite(T_c[i])) { *resid = NAN; return -5; }
        double norm = norm_sigma_tint ? sigma * pow(T_int, 4) : sigma * pow(T_c[i], 4);
        double r = fabs(dF) / norm;
        if (r > worst) worst = r;
    }
    *resid = worst;
    if (worst < tol) return 1;
    const double cp = (2.0 + 5.0) * REF_K / (2.0 * mmw_g);
    for (int i = 0; i < n; ++i) {
        double dF = F_bol[3 * (2 * i + 2) + 2] - F_bol[3 * (2 * i) + 2];
        double T = T_c[i], P = P_pt[2 * i + 1];
        /* optional dead band: a layer already within the tolerance is left
           as it is (temperature, step multiplier and sign history) */
        if (deadband) {
            double norm = norm_sigma_tint ? sigma * pow(T_int, 4) : sigma * pow(T, 4);
            if (fabs(dF) / norm < tol) continue;
        }
        double dT = 0.0;
        if (dF != 0.0) {
            double rho = P * mmw_g / (REF_K * T);
            double dz = REF_K * T * log(P_pt[2 * i] / P_pt[2 * i + 2]) / (mmw_g * grav);
            double t_rad = cp * P / (sigma * grav * T * T * T);
            double f_pre = fpre_c / pow(fabs(dF), fpre_p);
            double dt = m[i] * f_pre * t_rad;
            dT = -dF * dt / (rho * cp * dz);
        }
        int32_t bits = hist[i] & 0xFFFF, cnt = (hist[i] >> 16) & 0xFFFF;
        int sgn = (dT > 0.0) ? 1 : (dT < 0.0) ? 0 : (cnt > 0 ? (bits & 1) : 1);
        int32_t mask = (int32_t)((1u << window) - 1u);
        bits = ((bits << 1) | sgn) & mask;
        if (cnt < window) cnt += 1;
        if (cnt >= window) {
            int alternating = 1;
            for (int k = 0; k + 1 < window; ++k)
                if (((bits >> k) & 1) == ((bits >> (k + 1)) & 1)) alternating = 0;
            if (bits == 0 || bits == mask) m[i] *= grow;
            else if (osc_any || alternating) m[i] *= shrink;
        }
        hist[i] = (cnt << 16) | bits;
        double Tn = T + dT;
        T_c[i] = (Tn > T_floor) ? Tn : T_floor;
    }
    return 0;
}

/* ------------------------------------------------ exact pure absorption
 * Sec. 2.1.2.  Check mode: used by the tests and the diffusivity study, not by
 * the two-stream path.  E1 from its power series for x <= 1 and from its
 * continued fraction (evaluated with the modified Lentz method) for x > 1
 * (Abramowitz & Stegun 5.1.11 and 5.1.22). */
double ref_E1(double x) {
    if (!(x > 0.0)) return INFINITY;
    if (x <= 1.0) {
        const double euler_gamma = 0.57721566490153286061;
        double sum = 0.0, term = 1.0;
        for (int k = 1; k < 200; ++k) {
            term *= -x / k;              /* (-x)^k / k! */
            double add = -term / k;      /* - (-x)^k / (k k!) */
            sum += add;
            if (fabs(add) < 1e-18 * fabs(sum)) break;
        }
        return -euler_gamma - log(x) + sum;
    }
    /* E1(x) = e^-x / (x + 1 - 1^2/(x + 3 - 2^2/(x + 5 - ...))) */
    const double tiny = 1e-300;
    double b = x + 1.0;
    double f = b, C = b, Dd = 0.0;
    for (int k = 1; k < 500; ++k) {
        double a = -(double)k * k;
        b += 2.0;
        Dd = b + a * Dd;
        if (fabs(Dd) < tiny) Dd = tiny;
        C = b + a / C;
        if (fabs(C) < tiny) C = tiny;
        Dd = 1.0 / Dd;
        double delta = C * Dd;
        f *= delta;
        if (fabs(delta - 1.0) < 1e-16) break;
    }
    return exp(-x) / f;
}

/* eq:direct_trans; at dtau = 0 its limit 1 (dtau^2 E1(dtau) -> 0) */
double ref_exact_trans(double dtau) {
    if (dtau == 0.0) return 1.0;
    return (1.0 - dtau) * exp(-dtau) + dtau * dtau * ref_E1(dtau);
}

/* eq:diff */
double ref_exact_diffusivity(double dtau) {
    return -log(ref_exact_trans(dtau)) / dtau;
}

/* eq:isodirect and eq:nonisodirect with their own labels: interface 1 is the
 * lower, 2 the upper; B_1, B_2 are the Planck values there, dtau > 0 the
 * layer's optical thickness and B' = (B_1 - B_2)/dtau (positive when the
 * layer is hotter below).  iso != 0 selects eq:isodirect (B_1 throughout). */
double ref_exact_up(double dtau, double B1, double B2, double F1_up, int iso) {
    double T = ref_exact_trans(dtau);
    if (iso) return T * F1_up + REF_PI * B1 * (1.0 - T);
    double Bp = (B1 - B2) / dtau;
    return T * F1_up + REF_PI * B1 * (1.0 - T)
         + REF_PI * Bp * (2.0 / 3.0 * (1.0 - exp(-dtau)) - dtau * (1.0 - T / 3.0));
}

double ref_exact_down(double dtau, double B1, double B2, double F2_dn, int iso) {
    double T = ref_exact_trans(dtau);
    if (iso) return T * F2_dn + REF_PI * B1 * (1.0 - T);
    double Bp = (B1 - B2) / dtau;
    return T * F2_dn + REF_PI * B2 * (1.0 - T)
         + REF_PI * Bp * (-2.0 / 3.0 * (1.0 - exp(-dtau)) + dtau * (1.0 - T / 3.0));
}

/* Pure-absorption column solve with the exact layer relations (Sec. 2.1.2,
 * eq:direct_trans, eq:isodirect, eq:nonisodirect), the check mode against
 * which the diffusivity approximation is judged.  Same grid, boundary fluxes,
 * opacities and sums as ref_flux; w0 and g0 do not enter and a single
 * downward and upward sweep is exact (no scattering couples the streams).
 * Sublayer s joins points s (lower, interface 1) and s+1 (upper, interface
 * 2); a sublayer with dtau < 1e-4 uses eq:isodirect with the mean of its two
 * Planck values (as the two-stream path does), others eq:nonisodirect. */
int ref_flux_exact(int n, int nb, int ng,
                   const double* P_pt, double grav, const double* T_pt,
                   const double* lambda_c, const double* dlambda, const double* g_weight,
                   double T_star, double T_irr, double T_int, const double* kappa,
                   double* F_up, double* F_dn, double* F_up_bin, double* F_dn_bin, double* F_bol,
                   int n_threads) {
    const int npt = 2 * n + 1;
    double* F_top = (double*)malloc(sizeof(double) * nb);
    double* F_int = (double*)malloc(sizeof(double) * nb);
    double* B = (double*)malloc(sizeof(double) * (size_t)nb * npt);
    double* dm = (double*)malloc(sizeof(double) * 2 * n);
    if (!F_top || !F_int || !B || !dm) {
        free(F_top); free(F_int); free(B); free(dm);
        return -1;
    }
    ref_boundary(nb, lambda_c, dlambda, T_star, T_irr, T_int, F_top, F_int);
    for (int l = 0; l < nb; ++l)
        for (int p = 0; p < npt; ++p) B[(size_t)l * npt + p] = ref_planck(lambda_c[l], T_pt[p]);
    for (int s = 0; s < 2 * n; ++s) dm[s] = (P_pt[s] - P_pt[s + 1]) / grav;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int col = 0; col < nb * ng; ++col) {
        const int l = col / ng;
        const double* kap = kappa + (size_t)col * npt;
        const double* Bl = B + (size_t)l * npt;
        double* up = F_up + (size_t)col * npt;
        double* dn = F_dn + (size_t)col * npt;
        dn[2 * n] = F_top[l];
        for (int s = 2 * n - 1; s >= 0; --s) {
            double dtau = 0.5 * (kap[s] + kap[s + 1]) * dm[s];
            if (dtau < 1e-4) {
                double Bm = 0.5 * (Bl[s] + Bl[s + 1]);
                dn[s] = ref_exact_down(dtau, Bm, Bm, dn[s + 1], 1);
            } else {
                dn[s] = ref_exact_down(dtau, Bl[s], Bl[s + 1], dn[s + 1], 0);
            }
        }
        up[0] = dn[0] + F_int[l];
        for (int s = 0; s < 2 * n; ++s) {
            double dtau = 0.5 * (kap[s] + kap[s + 1]) * dm[s];
            if (dtau < 1e-4) {
                double Bm = 0.5 * (Bl[s] + Bl[s + 1]);
                up[s + 1] = ref_exact_up(dtau, Bm, Bm, up[s], 1);
            } else {
                up[s + 1] = ref_exact_up(dtau, Bl[s], Bl[s + 1], up[s], 0);
            }
        }
    }
    ref_sums(npt, nb, ng, dlambda, g_weight, F_up, F_dn, F_up_bin, F_dn_bin, F_bol);
    free(F_top); free(F_int); free(B); free(dm);
    return 0;
}

/* ------------------------------------------------ isothermal-layer grid
 * Sec. 2.2.1, first grid: n isothermal layers between n + 1 interfaces.
 * Layer i lies between interface i (below) and interface i + 1 (above); it
 * has one temperature and one opacity (those of its centre) and its optical
 * thickness is dtau_i = kappa_i (P_int,i - P_int,i+1) / grav (eq:layertau).
 * Fluxes live on the interfaces only.  Each layer is propagated with
 * eq:isoscat and the Planck value of its own temperature, for every dtau (no
 * gradient form exists on this grid), or with eq:purescat when
 * (1 - w0) < 1e-6 (the same switch as on the sublayered grid).  Boundary
 * conditions, scattering passes and sums are those of ref_flux.
 *
 * Inputs: P_int [n+1] interface pressures, T_lay [n] layer temperatures,
 * kappa [nb][ng][n] layer opacities, w0, g0 [nb][n].  F_up [nb][ng][n+1] is
 * the warm start on entry and the result on exit; F_dn [nb][ng][n+1]
 * (optional), F_up_bin, F_dn_bin [nb][n+1] and F_bol [n+1][3] as in ref_flux
 * with interfaces in place of points. */
/* One layer in either direction (eq:isoscat and eq:purescat are symmetric
 * under exchanging the streams).  Upward: F_in = F_up at the lower interface,
 * F_other = F_dn at the upper one, result F_up at the upper interface.
 * Downward: F_in = F_dn at the upper interface, F_other = F_up at the lower
 * one, result F_dn at the lower interface. */
static double ref_iso_layer(double dtau, double w0, double g0, double D, double B,
                            double F_in, double F_other) {
    if (ref_branch(dtau, w0) == REF_BR_PURESCAT) {
        double q = D * (1.0 - g0) * dtau;
        return F_in - q * (F_in - F_other) / (2.0 + q);
    }
    ref_coeff c;
    ref_coeffs(dtau, w0, g0, D, &c);
    double eps = 1.0 / D;
    return (c.xi * F_in - c.beta * F_other + 2.0 * REF_PI * eps * B * (c.beta - c.ups)) / c.alpha;
}

int ref_flux_iso(int n, int nb, int ng,
                 const double* P_int, double grav, const double* T_lay,
                 const double* lambda_c, const double* dlambda, const double* g_weight,
                 double T_star, double T_irr, double T_int,
                 const double* kappa, const double* w0, const double* g0,
                 int n_scat, double D,
                 double* F_up, double* F_dn,
                 double* F_up_bin, double* F_dn_bin, double* F_bol,
                 int n_threads) {
    const int nif = n + 1;
    const size_t ncell = (size_t)nb * ng * nif;
    double* F_top = (double*)malloc(sizeof(double) * nb);
    double* F_int = (double*)malloc(sizeof(double) * nb);
    double* B = (double*)malloc(sizeof(double) * (size_t)nb * n);
    double* dm = (double*)malloc(sizeof(double) * n);
    double* dn_all = F_dn ? F_dn : (double*)malloc(sizeof(double) * ncell);
    if (!F_top || !F_int || !B || !dm || !dn_all) {
        free(F_top); free(F_int); free(B); free(dm);
        if (!F_dn) free(dn_all);
        return -1;
    }
    ref_boundary(nb, lambda_c, dlambda, T_star, T_irr, T_int, F_top, F_int);
    for (int l = 0; l < nb; ++l)
        for (int i = 0; i < n; ++i) B[(size_t)l * n + i] = ref_planck(lambda_c[l], T_lay[i]);
    for (int i = 0; i < n; ++i) dm[i] = (P_int[i] - P_int[i + 1]) / grav; /* eq:layertau */
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int col = 0; col < nb * ng; ++col) {
        const int l = col / ng;
        const double* kap = kappa + (size_t)col * n;
        const double* Bl = B + (size_t)l * n;
        const double* w0l = w0 + (size_t)l * n;
        const double* g0l = g0 + (size_t)l * n;
        double* up = F_up + (size_t)col * nif;
        double* dn = dn_all + (size_t)col * nif;
        for (int pass = 0; pass <= n_scat; ++pass) {
            dn[n] = F_top[l];
            for (int i = n - 1; i >= 0; --i)
                dn[i] = ref_iso_layer(kap[i] * dm[i], w0l[i], g0l[i], D, Bl[i], dn[i + 1], up[i]);
            up[0] = dn[0] + F_int[l];
            for (int i = 0; i < n; ++i)
                up[i + 1] = ref_iso_layer(kap[i] * dm[i], w0l[i], g0l[i], D, Bl[i], up[i], dn[i + 1]);
        }
    }
    ref_sums(nif, nb, ng, dlambda, g_weight, F_up, dn_all, F_up_bin, F_dn_bin, F_bol);
    free(F_top); free(F_int); free(B); free(dm);
    if (!F_dn) free(dn_all);
    return 0;
}
