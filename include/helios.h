/*
 * helios.h -- C ABI of the MI355X (gfx950) radiative-equilibrium hot path of
 * HELIOS (Malik et al. 2017, Sec. 2): the two-stream flux solve that each
 * temperature iteration runs, and the temperature update it drives.
 *
 * Conventions for every call
 * --------------------------
 *  * Array arguments are DEVICE pointers unless marked [host].
 *  * The caller owns all memory, including the flux workspace sized by
 *    helios_workspace_bytes().  The library keeps no pointer after a call's
 *    stream-ordered work and allocates no device memory.
 *  * Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL
 *    is the default stream).  Errors found before anything is enqueued are
 *    returned synchronously as negative codes; nothing was enqueued then.
 *  * helios_last_error() returns a thread-local message for the last error.
 *    No call throws, aborts or prints.
 *  * Units are cgs: K, dyn cm^-2, cm, erg s^-1 cm^-2 (fluxes per unit
 *    wavelength: erg s^-1 cm^-3), cm^2 g^-1, cm s^-2.
 *  * A single atmosphere is a batch of one; all calls take a batch.
 *
 * Per-atmosphere data are concatenated in atmosphere order.  With n layers,
 * npt = 2n+1 points (point 2i = interface i, point 2i+1 = centre of layer i,
 * bottom to top), nb bins and ng Gauss points, the layouts are
 *    layer arrays   [n]            offset lay_off[a]
 *    point arrays   [npt]          offset pt_off[a]
 *    bin arrays     [nb]           offset bin_off[a]
 *    bin x layer    [nb][n]        offset lb_off[a]
 *    bin x point    [nb][npt]      offset pb_off[a]
 *    cell arrays    [nb][ng][cs]   offset cell_off[a]   (one column per (bin, g))
 * where each *_off is the exclusive prefix sum of the per-atmosphere sizes,
 * with n_atm+1 entries, and cs = npt rounded up to a multiple of
 * HELIOS_CELL_ALIGN: a column's points start on a 128-byte boundary.  The
 * cs - npt padding entries of a column are ignored on input and unspecified
 * on output.
 */
#ifndef HELIOS_H
#define HELIOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define HELIOS_OK 0
#define HELIOS_NOT_CONVERGED 1
#define HELIOS_EINVAL (-1)     /* null pointer, non-positive size, unknown enum */
#define HELIOS_ESHAPE (-2)     /* inconsistent sizes / offsets / table shape, bin index outside the table */
#define HELIOS_EDEVICE (-3)    /* a HIP call failed */
#define HELIOS_EWORKSPACE (-4) /* workspace smaller than helios_workspace_bytes() */
#define HELIOS_ENUMERIC (-5)   /* non-finite flux or temperature (per-atmosphere status) */

/* per-atmosphere status words written by helios_radeq */
#define HELIOS_ATM_RUNNING 0
#define HELIOS_ATM_CONVERGED 1
#define HELIOS_ATM_BADGRID (-2)  /* point pressures not positive, finite and strictly decreasing upward */
#define HELIOS_ATM_NUMERIC (-5)

#define HELIOS_MAX_SPECIES 8
#define HELIOS_MAX_NG 32
#define HELIOS_MAX_LAYERS 1024
#define HELIOS_CELL_ALIGN 32

typedef enum { HELIOS_FP64 = 0, HELIOS_MIXED = 1 } helios_prec;

/* Convention of the per-g flux arrays (F_up_g, F_dn_g) of the flux calls,
 * OR'ed into their `prec` argument:
 *   HELIOS_STATE_DEVIATION (default): each value is the deviation
 *     G = F - (2 pi / D) B(lambda_bin, T_point) of the flux from the
 *     isothermal solution at the bin centre and the point's temperature (for
 *     helios_flux_exact: from pi B).  The sweeps carry exactly this
 *     quantity; in FP32 it keeps the net flux resolved at depth, where F_up
 *     and F_dn both approach pi B and differ by ~1e-6 of it.  A zero array is
 *     the isothermal start.
 *   HELIOS_STATE_FLUX: each value is the flux F itself (Sec. 2.2.3: the
 *     scattering iteration starts from zero fluxes, and later temperature
 *     steps start from the previous step's fluxes).  A zero array is the
 *     paper's cold start.  The sweep still carries deviations: it takes
 *     (2 pi / D) B off the warm start as it reads it and adds it back to the
 *     per-g values it stores, in the precision of the per-g arrays (meant
 *     for HELIOS_FP64).
 * helios_state_convert() converts an array between the two. */
#define HELIOS_STATE_DEVIATION 0x000
#define HELIOS_STATE_FLUX 0x100
/* OR'ed into the prec argument of helios_autotune and helios_sweep_shapes:
 * the shapes of helios_flux_iso's sweep (one slot per layer) instead of
 * helios_flux's (one per sublayer). */
#define HELIOS_GRID_ISOTHERMAL 0x200
typedef enum { HELIOS_KTAB_TABLE = 0, HELIOS_KTAB_POWERLAW = 1 } helios_ktab_mode;
typedef enum { HELIOS_NORM_SIGMA_T4 = 0, HELIOS_NORM_SIGMA_TINT4 = 1 } helios_norm;

/* Batch descriptor.  Host mirrors are read for validation and launch shapes;
 * the device arrays must hold the same values. */
typedef struct helios_atm {
    int32_t n_atm;               /* atmospheres in the batch, >= 1 */
    int32_t n_g;                 /* Gauss points per bin, 1..HELIOS_MAX_NG */
    const int32_t* n_layer_h;    /* [host][n_atm] layers, 2..HELIOS_MAX_LAYERS */
    const int32_t* n_bin_h;      /* [host][n_atm] bins, >= 1 */
    const int32_t* n_layer;      /* [n_atm] */
    const int32_t* n_bin;        /* [n_atm] */
    const int64_t* lay_off;      /* [n_atm+1] */
    const int64_t* pt_off;       /* [n_atm+1] */
    const int64_t* bin_off;      /* [n_atm+1] */
    const int64_t* lb_off;       /* [n_atm+1] */
    const int64_t* pb_off;       /* [n_atm+1] */
    const int64_t* cell_off;     /* [n_atm+1] */
    const int32_t* bin_index;    /* [sum nb] k-table bin of each model bin */
    const int32_t* bin_index_h;  /* [host][sum nb] the same values (validated against the table) */
    const double* lambda_c;      /* [sum nb] bin centre wavelength, cm */
    const double* dlambda;       /* [sum nb] bin width, cm */
    const double* P_c;           /* [sum n] layer-centre pressure, bottom -> top */
    double* P_pt;                /* [sum npt] point pressures, written by helios_grid */
    const double* grav;          /* [n_atm] surface gravity */
    const double* T_star;        /* [n_atm] stellar blackbody temperature */
    const double* T_irr;         /* [n_atm] irradiation temperature: TOA flux is (T_irr/T_star)^4 pi B(T_star) */
    const double* T_int;         /* [n_atm] internal temperature of the BOA flux */
    const int32_t* status;       /* [n_atm] optional (NULL: all active): atmospheres whose
                                    status is not HELIOS_ATM_RUNNING are skipped by
                                    helios_mix_opacity and helios_flux, their outputs left
                                    unchanged (a batch's active set shrinks on the device,
                                    without a new descriptor) */
} helios_atm;

/* Opacity source (Sec. 2.3).  TABLE: k-coefficients on a uniform
 * T x log10 P grid, interpolated bilinearly and clamped at the table edges.
 * POWERLAW: k = k0 (P/P_ref)^p_exp (T/T_ref)^t_exp. */
typedef struct helios_ktab {
    int32_t mode;                /* helios_ktab_mode */
    int32_t n_species;           /* 1..HELIOS_MAX_SPECIES */
    int32_t n_T, n_P;            /* TABLE: nodes per axis, >= 2 */
    int32_t n_bin_table;         /* bins in the table (bin_index < n_bin_table) */
    int32_t n_g;                 /* must equal helios_atm.n_g */
    double T_min, T_step;        /* TABLE: T axis, K */
    double logP_min, logP_step;  /* TABLE: log10 P axis, P in dyn cm^-2 */
    const float* k;              /* TABLE: [n_species][n_T][n_P][n_bin_table][n_g] */
    const double* k0;            /* POWERLAW: [n_species][n_bin_table][n_g] */
    double p_exp, t_exp, P_ref, T_ref;
    const double* species_mass;  /* [host][n_species] molecular mass, proton masses */
    double mmw;                  /* mean molecular mass, proton masses (2.4) */
} helios_ktab;

/* Options of the temperature update (Sec. 2.2.3-2.2.4). */
typedef struct helios_re_opts {
    double tol;       /* convergence threshold on max_i |dF_i| / norm_i */
    int32_t norm;     /* helios_norm: sigma T_i^4 (paper) or sigma T_int^4 */
    int32_t window;   /* oscillation-control window, 2..16 (paper: 6) */
    int32_t osc_any;  /* 0: oscillation = sign alternated over the whole window;
                         1: any sign change in the window counts */
    int32_t deadband; /* 0: every layer steps (paper); 1: a layer with |dF_i| / norm_i < tol
                         keeps its temperature, step multiplier and sign history */
    double T_floor;   /* lower temperature bound, K */
    double shrink;    /* multiplier on oscillation (paper: reduce by 33% -> 0.67) */
    double grow;      /* multiplier when monotonic (paper: +10% -> 1.1) */
    double fpre_c;    /* f_pre = fpre_c / |dF|^fpre_p (paper: 1e5, 0.9) */
    double fpre_p;
} helios_re_opts;

/* Per-layer RE state, owned by the caller, initialised to m = 1, hist = 0.
 * hist bits 0..15: signs of the most recent dT (bit 0 newest, 1 = warming);
 * bits 16..31: number of signs recorded (saturates at the window). */
typedef struct helios_re_state {
    double* m;        /* [sum n] timestep multipliers */
    int32_t* hist;    /* [sum n] sign histories */
    int32_t* iter;    /* [n_atm] temperature updates taken (may be NULL) */
} helios_re_state;

/* Fills atm->P_pt (Sec. 2.2.1, Fig. 2): centres copied to odd points,
 * interfaces at the geometric mean of neighbouring centres, the outermost
 * half a log-step beyond the outermost centres. */
int helios_grid(const helios_atm* atm, void* stream);

/* Interface temperatures (Sec. 2.2.1): T_pt[odd] = T_c; inner interfaces
 * linear in ln P between the neighbouring centres; outer interfaces copy the
 * adjacent centre.  T_c [sum n] -> T_pt [sum npt].  Needs atm->P_pt. */
int helios_profile(const helios_atm* atm, const double* T_c, double* T_pt, void* stream);

/* Opacity at the points (eq:kappa_gauss, eq:mixing, Sec. 2.3):
 * kappa[cell] = sum_j X_j m_j/mbar k_j(T_pt, P_pt, bin_index, g).
 * vmr: [n_species][sum npt] volume mixing ratios.  kappa: cell array, double
 * (HELIOS_FP64) or float (HELIOS_MIXED).
 * Errors: -2 (nothing enqueued) if a bin_index_h entry lies outside
 * 0 .. n_bin_table - 1 or the table's n_g differs from the batch's. */
int helios_mix_opacity(const helios_atm* atm, const helios_ktab* kt, const double* T_pt,
                       const double* vmr, void* kappa, helios_prec prec, void* stream);

/* Sublayer coefficients (eq:trans, eq:cap, eq:isoscat, eq:nonisoscat,
 * eq:purescat; the branch switches of Sec. 2.1.4 and 2.2.1), for inspection:
 * for every (bin, g, sublayer s) five doubles {Trans, a, c, S_up, S_dn} with
 *   F_up(s+1) = a F_up(s) + c F_dn(s+1) + S_up
 *   F_dn(s)   = a F_dn(s+1) + c F_up(s) + S_dn
 * out: [sum over atmospheres nb*ng*2n][5] in (atmosphere, bin, g, sublayer)
 * order (offset 2*ng*lb_off[a]).  The flux sweep computes the same values in
 * registers. */
int helios_transmission(const helios_atm* atm, const void* kappa, const double* T_pt,
                        const double* w0, const double* g0, double D, double* out,
                        helios_prec prec, void* stream);

/* Workspace bytes needed by helios_flux for this batch and precision. */
size_t helios_workspace_bytes(const helios_atm* atm, helios_prec prec);

/* One two-stream flux solve (Sec. 2.1.3, 2.2.2, 2.2.3, 2.3):
 * Planck sources at the points, TOA/BOA boundary fluxes, sublayer
 * coefficients, 1 + n_scat scattering passes (down sweep, BOA condition, up
 * sweep) per (bin, g) column, Gauss sum over g and width-weighted sum over
 * bins.
 *   kappa     cell array (double or float by prec) from helios_mix_opacity
 *   T_pt      [sum npt]
 *   w0, g0    [bin x layer] single-scattering albedo and asymmetry
 *   n_scat    additional scattering passes (paper: 4 in the RE loop, 80 post)
 *   D         diffusivity factor (paper: 2)
 *   F_up_g    cell array, in: warm start, out: upward fluxes of the last pass
 *             (zeros on the first call of an RE iteration with
 *             HELIOS_STATE_FLUX: the paper's start)
 *   F_dn_g    cell array, out: downward fluxes of the last pass (may be NULL)
 *   F_up_bin, F_dn_bin  [bin x point] double, Gauss-summed fluxes; either may
 *             be NULL (not written: the iteration itself needs only F_bol)
 *   F_bol     [sum npt][3] double: bolometric up, down, and net = up - down
 *             (the net flux is summed from the deviations below, in which
 *             the Planck term cancels, not by subtracting the two totals)
 *   prec      HELIOS_FP64 or HELIOS_MIXED (element type of kappa and the
 *             per-g arrays), OR'ed with the per-g convention
 *             HELIOS_STATE_DEVIATION (default) or HELIOS_STATE_FLUX.  With
 *             deviations, F = value + (2 pi / D) B(lambda_bin, T_point) and a
 *             zero array is the isothermal start; across temperature steps
 *             the warm start then keeps each column's deviation from its local
 *             Planck flux.  With fluxes the warm start is the previous fluxes
 *             themselves (Sec. 2.2.3).  helios_state_convert() converts.
 *   ws        workspace of at least helios_workspace_bytes(atm, prec) bytes
 * Downward fluxes carry no state between calls: each pass recomputes them
 * from the TOA condition and the previous upward fluxes.
 * Errors: -2 (nothing enqueued) also for an atmosphere of more than 832
 * layers (the deepest sweep shape holds 1664 sublayers). */
int helios_flux(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0,
                const double* g0, int32_t n_scat, double D, void* F_up_g, void* F_dn_g,
                double* F_up_bin, double* F_dn_bin, double* F_bol, void* ws, size_t ws_bytes,
                helios_prec prec, void* stream);

/* helios_flux for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, arguments and results, without the ws / ws_bytes pair.
 * The workspace is a static device array of HELIOS_NOALLOC_WS_BYTES inside
 * the library, one copy per device, kept until the process ends; its device
 * address is looked up on the first call on each device.  The call itself
 * allocates nothing.  Errors: HELIOS_EWORKSPACE (nothing enqueued) if the
 * batch needs more than HELIOS_NOALLOC_WS_BYTES of workspace
 * (helios_workspace_bytes tells), otherwise as helios_flux.  Every call on
 * one device uses the same array: calls that can overlap on a device (on
 * different streams, or from several threads without ordering) race and
 * must be serialised by the caller; each call rewrites all the workspace it
 * reads, so no clearing is needed between calls. */
#define HELIOS_NOALLOC_WS_BYTES ((size_t)64 << 20)
int helios_flux_noalloc(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0,
                        const double* g0, int32_t n_scat, double D, void* F_up_g, void* F_dn_g,
                        double* F_up_bin, double* F_dn_bin, double* F_bol, helios_prec prec, void* stream);

/* The same two-stream solve on the isothermal-layer grid (Sec. 2.2.1): the
 * atmosphere is n isothermal layers between the n + 1 interfaces at the even
 * points (P_pt[2i]); layer i has the temperature and opacity of its centre
 * (T_pt[2i+1] and the kappa values at point 2i+1), optical thickness
 * kappa (P_pt[2i] - P_pt[2i+2]) / g (eq:layertau), and is propagated with
 * eq:isoscat and B(T_i) at every optical thickness (eq:purescat where
 * (1 - w0) < 1e-6).  Boundary conditions, scattering passes, precision and
 * sums as helios_flux.  Only the centre values of T_pt and kappa are used.
 *   F_up_g, F_dn_g  cell arrays in the point layout: at point 2i the fluxes at
 *                   interface i, at point 2i+1 those at interface i+1 (the top
 *                   of layer i), stored as deviations from (2 pi / D) B(T_i)
 *                   at points 2i and 2i+1 and from (2 pi / D) B(T_{n-1}) at the
 *                   TOA point; a zero array is the isothermal start
 *   F_up_bin, F_dn_bin, F_bol  at the points as for helios_flux; even points
 *                   are the interfaces and point 2i+1 repeats interface i+1,
 *                   so helios_radeq takes F_bol unchanged
 * A layer is one slot of the sweep, so this grid takes up to
 * HELIOS_MAX_LAYERS layers (helios_flux up to 832: two slots per layer).
 * Errors: as helios_flux. */
int helios_flux_iso(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0,
                    const double* g0, int32_t n_scat, double D, void* F_up_g, void* F_dn_g,
                    double* F_up_bin, double* F_dn_bin, double* F_bol, void* ws, size_t ws_bytes,
                    helios_prec prec, void* stream);

/* helios_flux with Rayleigh scattering by H2 (Sec. 2.1.4).  kappa holds
 * the absorption opacities; the library adds the scattering opacity
 * sigma(lambda_c) / mbar of each bin, with the H2 cross-section
 * sigma = 24 pi^3 / (n_ref^2 lambda^4) ((n^2 - 1)/(n^2 + 2))^2 (n_ref =
 * 2.68678e19 cm^-3, King factor 1, n - 1 = 13.58e-5 (1 + 7.52e-11 cm^2 /
 * lambda^2)), to every sublayer, and each sublayer and g-point scatters the
 * scattering share of its extinction isotropically: w0 = kappa_scat /
 * (kappa_abs + kappa_scat), g0 = 0 (eq:purescat where 1 - w0 < 1e-6).  No
 * w0 or g0 array is read.
 *   mbar      mean molecular mass in g (2.4 m_p for the paper's hydrogen
 *             atmospheres), > 0
 * Everything else, including the warm-start convention and the outputs, as
 * helios_flux.  Errors: as helios_flux; -1 if mbar <= 0. */
int helios_flux_rayleigh(const helios_atm* atm, const void* kappa, const double* T_pt, double mbar,
                         int32_t n_scat, double D, void* F_up_g, void* F_dn_g, double* F_up_bin,
                         double* F_dn_bin, double* F_bol, void* ws, size_t ws_bytes, helios_prec prec,
                         void* stream);

/* Pure-absorption flux solve with the exact layer relations (Sec. 2.1.2:
 * transmission eq:direct_trans = 2 E3(dtau), sources eq:nonisodirect, and
 * eq:isodirect with the mean of the sublayer's two Planck values where
 * dtau < 1e-4), the check against which the two-stream diffusivity factor D
 * is judged.  FP64 only.  Same grid, opacities (double cell array), Planck
 * values, boundary fluxes and sums as helios_flux; single-scattering albedo,
 * asymmetry and D do not enter, and one downward and one upward sweep per
 * (bin, g) column are exact (no scattering couples the streams).
 *   F_up_g, F_dn_g  cell arrays, out: deviations from pi B at the points
 *                   (pi B is the isothermal solution of this mode), or the
 *                   fluxes with HELIOS_STATE_FLUX in `state`; no warm start is
 *                   read
 *   F_up_bin, F_dn_bin, F_bol  as for helios_flux (the per-bin arrays may be
 *                   NULL)
 *   ws        workspace of at least helios_workspace_bytes(atm, HELIOS_FP64)
 * Errors: as helios_flux. */
int helios_flux_exact(const helios_atm* atm, const double* kappa, const double* T_pt, double* F_up_g,
                      double* F_dn_g, double* F_up_bin, double* F_dn_bin, double* F_bol, void* ws,
                      size_t ws_bytes, int32_t state, void* stream);

/* Conversion of a per-g cell array between the two conventions of the flux
 * calls, with the reference (2 pi / D) B(lambda_bin, T_point) formed on the
 * device from T_pt (the Planck function at the bin centre, as in the flux
 * solve):
 *   HELIOS_CONVERT_TO_DEVIATION  F_g <- F_g - (2 pi / D) B
 *   HELIOS_CONVERT_TO_FLUX       F_g <- F_g + (2 pi / D) B
 *   HELIOS_CONVERT_ZERO_FLUX     F_g <- -(2 pi / D) B: the zero-flux start of
 *                                the scattering iteration (Sec. 2.2.3) in
 *                                deviation form; the input is not read
 *   layers    HELIOS_LAYERS_SUBLAYERED (helios_flux, helios_flux_rayleigh) or
 *             HELIOS_LAYERS_ISOTHERMAL (helios_flux_iso: reference B(T_i) at
 *             points 2i and 2i+1, B(T_{n-1}) at the TOA point).  The exact
 *             mode's reference pi B is the sublayered one with D = 2.
 *   prec      element type of F_g (double for HELIOS_FP64, float for
 *             HELIOS_MIXED); values are formed in FP64 and rounded once.
 * Atmospheres whose status is not RUNNING are left unchanged.
 * Errors: -1 for a NULL pointer, an unknown mode, layers or prec, D <= 0. */
#define HELIOS_CONVERT_TO_DEVIATION 0
#define HELIOS_CONVERT_TO_FLUX 1
#define HELIOS_CONVERT_ZERO_FLUX 2
#define HELIOS_LAYERS_SUBLAYERED 0
#define HELIOS_LAYERS_ISOTHERMAL 1
int helios_state_convert(const helios_atm* atm, const double* T_pt, double D, void* F_g, int32_t mode,
                         int32_t layers, helios_prec prec, void* stream);

/* Temperature update (Sec. 2.2.3 eq:step, Sec. 2.2.4, eq:condition), always
 * FP64.  For each atmosphere whose status is not CONVERGED: resid = max over
 * layers of |dF_i| / norm_i with dF_i the net-flux difference across layer i
 * (interfaces 2i and 2i+2 of F_bol); if resid < tol the status becomes
 * CONVERGED and nothing moves; otherwise every layer takes
 * dT_i = -sgn(dF_i) |dF_i|^(1-fpre_p) fpre_c m_i / (sigma T_i^3 ln(P_2i/P_2i+2)),
 * T is floored, the step multipliers are adapted and T_pt is re-interpolated.
 * Non-finite input sets the status to NUMERIC, point pressures that are not
 * positive, finite and strictly decreasing from the bottom up (Sec. 2.2.1)
 * set it to BADGRID; nothing moves then, and both are kept by later calls.
 *   status [n_atm] in/out, resid [n_atm] out (may be NULL). */
int helios_radeq(const helios_atm* atm, const double* F_bol, double* T_c, double* T_pt,
                 const helios_re_state* st, const helios_re_opts* opt, int32_t* status,
                 double* resid, void* stream);

/* Autotuner of the flux sweep (a batching aid; the paper runs one
 * atmosphere at a time).  helios_flux groups atmospheres into size classes by
 * layer count (n <= 32, 64, 112, 208, 400, 1024) and sweeps each class with
 * one launch of its own shape (sublayers per lane x lanes per column).  For
 * each class present in the batch, every compiled shape that holds the
 * class's deepest atmosphere (the 64-lane long-column shape only where no
 * other one does), with one or more waves per bin (more than one only for
 * batches of at most 65536 bins), is timed here on up to 4096 bins of that atmosphere
 * (same arguments as helios_flux, status ignored), and the fastest is used
 * by later helios_flux calls of this process with the same precision and
 * n_g.  Synchronous: returns after the timing.  F_up_g is restored to its
 * input values; the workspace must be at least helios_workspace_bytes(atm,
 * prec) bytes.  Atmospheres of a class that are adjacent in the batch share
 * one contiguous launch range; ordering a batch by layer count keeps every
 * class's range free of other classes' bins.  With HELIOS_GRID_ISOTHERMAL
 * OR'ed into prec the shapes are tuned (and kept) for helios_flux_iso. */
int helios_autotune(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0,
                    const double* g0, int32_t n_scat, double D, void* F_up_g, void* ws, size_t ws_bytes,
                    helios_prec prec, void* stream);

/* Forgets every shape helios_autotune chose in this process: later flux
 * calls use the default shapes until the autotuner runs again.  Host only;
 * never fails. */
int helios_autotune_reset(void);

/* The sweep shapes helios_flux would use for this batch: for each of the 6
 * size classes (out holds 3 x max_classes int32, max_classes >= 6) the
 * class's upper layer-count bound, then K (sublayers per lane) and L (lanes
 * per column), both 0 for a class with no member (helios_flux_iso's with
 * HELIOS_GRID_ISOTHERMAL OR'ed into prec).  Returns the number of classes
 * (> 0) or an error code. */
int helios_sweep_shapes(const helios_atm* atm, helios_prec prec, int32_t* out, int32_t max_classes);

/* ------------------------------------------------------------------
 * Learned warm start (an addition to the method: the paper starts every
 * atmosphere from a fixed profile).  A multilayer perceptron maps six
 * atmosphere parameters -- irradiation temperature [K], internal temperature
 * [K], log10 gravity [m s^-2], metallicity [M/H], C/O, log10 opacity scale --
 * to temperatures at n_out fixed pressures:
 *   n_in -> n_hidden (n_hidden_layers times, GELU z Phi(z) after each) -> n_out
 * (linear).  Weights, inputs, hidden activations and back-propagated errors
 * are BF16 on the matrix cores with FP32 accumulation; biases, master
 * parameters, Adam moments, pre-activations and outputs are FP32.
 * Inputs are normalised as (x - in_shift) * in_scale; the network's outputs
 * y are normalised temperatures, T = out_shift + out_scale * y.
 * Flat parameter layout (param_count entries): for each layer in order,
 * W [out][in] row-major, then b [out].
 * Limits: 1 <= n_in <= 64, 1 <= n_hidden <= 1024, 1 <= n_hidden_layers <= 8,
 * 1 <= n_out <= 1024, 1 <= batch <= 2^22. */
typedef struct {
    int32_t n_in, n_hidden, n_hidden_layers, n_out;
    float* params;               /* [param_count] FP32 master parameters */
    uint16_t* params_bf16;       /* [param_count] BF16 copy read by the products (bit pattern) */
    float* adam_m;               /* [param_count] first moments (training only, else NULL) */
    float* adam_v;               /* [param_count] second moments (training only, else NULL) */
    const float* in_shift;       /* [n_in] */
    const float* in_scale;       /* [n_in] */
    const float* out_shift;      /* [n_out] */
    const float* out_scale;      /* [n_out] */
} helios_mlp;

/* Number of parameters (0 if the dimensions are invalid). */
size_t helios_mlp_param_count(const helios_mlp* net);

/* Workspace bytes for a batch of `batch` rows (0 if invalid); also the
 * workspace of helios_warm_start with batch = n_atm. */
size_t helios_mlp_workspace_bytes(const helios_mlp* net, int32_t batch);

/* params_bf16 <- bf16(params), after the master parameters were written. */
int helios_mlp_sync(const helios_mlp* net, void* stream);

/* Inference: T [batch][n_out] (FP32, kelvin) from x [batch][n_in] (FP32). */
int helios_mlp_forward(const helios_mlp* net, const float* x, int32_t batch, float* T, void* ws,
                       size_t ws_bytes, void* stream);

/* Loss and gradient: loss (one float on the device) = mean over batch and
 * outputs of (y - (T_target - out_shift)/out_scale)^2, and grad
 * [param_count] (FP32, flat layout) its gradient by back-propagation.  The
 * output error 2 (y - t)/(batch n_out) and the back-propagated errors are
 * rounded to BF16 before each product; bias gradients sum those BF16 values. */
int helios_mlp_backward(const helios_mlp* net, const float* x, const float* T_target, int32_t batch,
                        float* loss, float* grad, void* ws, size_t ws_bytes, void* stream);

/* One Adam step (Kingma & Ba 2015, with bias correction; step counts from 1)
 * on params, adam_m, adam_v from grad; refreshes params_bf16. */
int helios_mlp_adam(const helios_mlp* net, const float* grad, int32_t step, float lr, float beta1,
                    float beta2, float eps, void* stream);

/* Initial profiles for a batch: the network's temperatures for each
 * atmosphere's parameters x [n_atm][n_in], given at log10 pressures
 * logP_net [n_out] (device, dyn cm^-2, strictly monotone), interpolated
 * linearly in log10 P onto the atmosphere's layer centres atm->P_c (end
 * values held outside).  An atmosphere whose network profile has a value
 * that is not finite or outside [T_lo, T_hi] gets T_iso in every layer and
 * fallback[a] = 1 (else 0).  T_c [sum n] out; workspace of at least
 * helios_mlp_workspace_bytes(net, n_atm) bytes. */
int helios_warm_start(const helios_atm* atm, const helios_mlp* net, const float* x, const double* logP_net,
                      double T_iso, double T_lo, double T_hi, double* T_c, int32_t* fallback, void* ws,
                      size_t ws_bytes, void* stream);

/* Diagnostics for measurement: when `before` and `after` are non-NULL
 * hipEvent_t handles (passed as void*), the calling thread's next
 * helios_flux calls record `before` on their stream just before the flux
 * sweep launches (one per size class present) are enqueued and `after` just
 * after them, so the sweep's own
 * duration can be read with hipEventElapsedTime.  NULL, NULL turns it off.
 * The setting is thread-local; the events are owned by the caller. */
int helios_set_sweep_events(void* before, void* after);

/* Thread-local description of the last error ("" if none). */
const char* helios_last_error(void);

/* ABI version of this library. */
int32_t helios_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HELIOS_H */
