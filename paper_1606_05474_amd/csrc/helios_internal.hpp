// helios_internal.hpp -- types, constants and device helpers shared by the
// HIP translation units of libhelios (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/helios.h"

namespace helios {

// CODATA 2018 exact constants, cgs.
constexpr double kPi = 3.14159265358979323846;
constexpr double kH = 6.62607015e-27;   // erg s
constexpr double kC = 2.99792458e10;    // cm s^-1
constexpr double kKB = 1.380649e-16;    // erg K^-1
// sigma = 2 pi^5 k^4 / (15 h^3 c^2)
__host__ __device__ inline double sigma_sb() {
    const double k2 = kKB * kKB;
    const double pi2 = kPi * kPi;
    return 2.0 * pi2 * pi2 * kPi * k2 * k2 / (15.0 * kH * kH * kH * kC * kC);
}

// Column stride of the cell arrays: 2n+1 points rounded up to HELIOS_CELL_ALIGN.
__host__ __device__ inline int col_stride(int n) {
    return ((2 * n + 1) + HELIOS_CELL_ALIGN - 1) & ~(HELIOS_CELL_ALIGN - 1);
}

// True when the batch marks atmosphere a as no longer running (converged or
// failed): opacity mixing and the flux solve skip it.
__device__ inline bool frozen(const int32_t* status, int a) {
    return status != nullptr && status[a] != HELIOS_ATM_RUNNING;
}

// Index of the atmosphere owning global element idx: the largest a with
// off[a] <= idx (off has n_atm+1 non-decreasing entries).
__device__ inline int find_atm(const int64_t* __restrict__ off, int n_atm, int64_t idx) {
    int lo = 0, hi = n_atm;  // invariant: off[lo] <= idx < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= idx) lo = mid; else hi = mid;
    }
    return lo;
}

// e = exp(-x) and om = 1 - exp(-x) for x >= 0 in FP64.  Cody-Waite
// reduction x = n ln2 + s' with |s'| <= ln2/2 (ln2 carried in two parts), the
// Taylor series of expm1 to degree 13 on the reduced argument (truncation
// below 5e-18) and scaling by 2^-n.  For n = 0 the polynomial gives om
// directly, so om keeps full relative accuracy for small x; for n >= 1,
// e <= 0.71 and 1 - e is free of cancellation.  Arguments beyond 1000 (e = 0
// in FP64) are clamped, which keeps n in integer range.
__device__ inline void exp_neg_om(double x, double& e, double& om) {
    constexpr double ln2_hi = 0.6931471805599453;      // ln 2 rounded to double
    constexpr double ln2_lo = 2.3190468138462996e-17;  // ln 2 - ln2_hi
    constexpr double inv_ln2 = 1.4426950408889634;
    x = fmin(x, 1000.0);
    const double n = rint(x * inv_ln2);
    double r = fma(-n, ln2_hi, x);
    r = fma(-n, ln2_lo, r);
    const double s = -r;  // exp(-x) = 2^-n exp(s)
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = fma(p, s, 1.0 / 479001600.0);
    p = fma(p, s, 1.0 / 39916800.0);
    p = fma(p, s, 1.0 / 3628800.0);
    p = fma(p, s, 1.0 / 362880.0);
    p = fma(p, s, 1.0 / 40320.0);
    p = fma(p, s, 1.0 / 5040.0);
    p = fma(p, s, 1.0 / 720.0);
    p = fma(p, s, 1.0 / 120.0);
    p = fma(p, s, 1.0 / 24.0);
    p = fma(p, s, 1.0 / 6.0);
    p = fma(p, s, 0.5);
    p = fma(p, s, 1.0);
    const double q = p * s;  // expm1(s)
    e = ldexp(1.0 + q, -(int)n);
    om = (n == 0.0) ? -q : 1.0 - e;
}

// H2 Rayleigh cross-section per molecule (cm^2) at wavelength lambda (cm),
// Sec. 2.1.4: 24 pi^3 / (n_ref^2 lambda^4) ((n^2 - 1)/(n^2 + 2))^2 K with
// n_ref = 2.68678e19 cm^-3, K = 1 and n - 1 = 13.58e-5 (1 + 7.52e-11 cm^2 /
// lambda^2); n^2 - 1 is formed as (n - 1)(n + 1), free of cancellation.
__host__ __device__ inline double rayleigh_h2(double lambda) {
    const double l2 = lambda * lambda;
    const double nm1 = 13.58e-5 * (1.0 + 7.52e-11 / l2);
    const double n = 1.0 + nm1;
    const double f = nm1 * (n + 1.0) / (n * n + 2.0);
    const double nr = 2.68678e19;
    return 24.0 * kPi * kPi * kPi / (nr * nr * l2 * l2) * f * f;
}

// Planck function per unit wavelength and steradian at the bin centre:
// 2 h c^2 / lambda^5 / (exp(x) - 1) = 2 h c^2 / lambda^5 * exp(-x) / (1 - exp(-x)),
// x = h c / (lambda k T).
__device__ inline double planck_d(double lambda, double T) {
    if (!(T > 0.0)) return 0.0;
    const double c1 = 2.0 * kH * kC * kC;
    const double x = kH * kC / (lambda * kKB * T);
    const double l2 = lambda * lambda;
    double e, om;
    exp_neg_om(x, e, om);
    return c1 / (l2 * l2 * lambda) * (e / om);
}

// ----------------------------------------------------------- launch args
struct SweepArgs {
    const int32_t* n_layer;
    const int64_t* pt_off;
    const int64_t* bin_off;
    const int64_t* lb_off;
    const int64_t* pb_off;
    const int64_t* cell_off;
    const double* P_pt;
    const double* grav;
    const void* kappa;    // cell array, R
    const void* B;        // [bin x point], R (workspace)
    const double* F_top;  // [sum nb] (workspace)
    const double* F_int;  // [sum nb] (workspace)
    const double* w0;
    const double* g0;
    void* F_up_g;         // cell array, R, in/out
    void* F_dn_g;         // cell array, R, out, may be null
    void* part_up;        // [bin x wave-of-bin x point] Gauss partial sums (workspace)
    void* part_dn;
    const double* gw;     // [n_g] Gauss weights on [0,1] (workspace)
    const double* bnd_part;  // [n_atm][bnd_maxch] chunk sums of pi B(T_int) dlambda (workspace)
    const double* T_int;     // [n_atm]
    const int32_t* status;   // optional: converged atmospheres are skipped
    const int32_t* bin_atm;  // [sum nb] owning atmosphere of each bin (workspace)
    int64_t w_begin, w_end;  // global (bin, part) range covered by the launch
    int32_t n_atm, n_g;
    int32_t wpb;          // groups of 64/L columns per bin (this launch's shape)
    int32_t parts;        // waves per bin in this launch (each a contiguous share of the groups)
    int32_t wpb_stride;   // partials per (bin, point) the workspace holds (>= parts)
    int32_t n_lo, n_hi;   // this launch serves atmospheres with n_lo <= n <= n_hi
    int32_t n_scat;
    int32_t npt_max;      // largest 2n+1 of the batch (LDS staging size)
    int32_t bnd_maxch;    // boundary chunks per atmosphere in bnd_part
    int32_t iso_grid;     // 1: isothermal-layer grid (layer i = sublayer slot 2i, slot 2i+1 the identity)
    int32_t flux_state;   // 1 if F_up_g / F_dn_g hold fluxes, 0 for deviations (from (2 pi / D) B in the
                          // two-stream sweep, which carries deviations either way; from pi B in exact mode)
    double D;
    const double* lambda_c;  // [sum nb] bin centres (Rayleigh scattering)
    double inv_mbar;         // > 0: add H2 Rayleigh scattering with this 1/mbar (g^-1); w0, g0 unused
};

constexpr int kMaxClasses = 8;

struct GaussTable {
    double w[HELIOS_MAX_NG];  // weights on [0,1] (sum 1), ascending nodes
};

struct BolArgs {
    helios_atm atm;
    const void* part_up;  // per-wave Gauss partials from the sweep (double, or float in mixed precision)
    const void* part_dn;
    double* F_up_bin;
    double* F_dn_bin;
    double* chunk;        // [n_chunk][6][sum npt] Neumaier pairs of bin-chunk sums (workspace)
    int64_t total_pt;
    double* F_bol;
    const double* B;      // [bin x point] Planck values (workspace)
    const double* gw;     // [n_g] Gauss weights (workspace)
    double tpe;           // 2 pi eps = 2 pi / D: the sweep's partials are deviations from tpe B
    double tw;            // tpe times the sum of the Gauss weights (in g order), formed on the host
    int32_t wpb_stride, n_chunk, mixed;
    int32_t chunk_bins;              // bins per chunk (bol_chunk_bins of the batch)
    int32_t n_cls;                   // size classes: atmosphere with n <= cls_nhi[k] (first k)
    int32_t cls_nhi[kMaxClasses];    // uses cls_wpb[k] waves per bin
    int32_t cls_wpb[kMaxClasses];
};

// Waves per bin of an atmosphere with n layers under the class table.
__device__ inline int class_wpb(const BolArgs& A, int n) {
    for (int k = 0; k < A.n_cls; ++k)
        if (n <= A.cls_nhi[k]) return A.cls_wpb[k];
    return A.cls_wpb[A.n_cls - 1];
}

// Host-side launchers (defined in the .hip files).
// ------------------------------------------------------ warm-start network
// C = A B^T: A(m, k) = A[m sam + k sak], B(n, k) = B[n sbn + k sbk], BF16.
struct GemmArgs {
    const uint16_t* A;
    int64_t sam, sak;
    const uint16_t* B;
    int64_t sbn, sbk;
    int M, N, K;
    const float* bias;     // [N] (kEpiGelu, kEpiLinear)
    float* out_f;          // FP32 output (pre-activation, output, or weight gradient)
    int64_t ld_f;
    uint16_t* out_b;       // BF16 output (activation or back-propagated error)
    int64_t ld_b;
    const float* zin;      // pre-activation read by kEpiDGelu
    int64_t ld_z;
    const float* oshift;   // optional output scaling (kEpiLinear): y -> oshift + oscale y
    const float* oscale;
};
enum { kEpiGelu = 0, kEpiLinear = 1, kEpiDGelu = 2, kEpiStore = 3 };
constexpr int kMaxNetOut = 1024;  // largest network output (warm start stages it in LDS)

hipError_t launch_gemm(const GemmArgs& g, int epi, hipStream_t s);
hipError_t launch_mlp_input(const float* x, int64_t count, int n_in, const float* shift, const float* scale,
                            uint16_t* X0, hipStream_t s);
hipError_t launch_mlp_loss(const float* Y, const float* T, int64_t count, int n_out, const float* shift,
                           const float* scale, uint16_t* dY, double* partial, int nblk, float* loss,
                           hipStream_t s);
hipError_t launch_mlp_bias_grad(const uint16_t* D, int64_t rows, int N, float* gb, hipStream_t s);
hipError_t launch_mlp_adam(float* p, uint16_t* pb, float* m, float* v, const float* grad, int64_t count, float lr,
                           float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t launch_mlp_sync(const float* p, uint16_t* pb, int64_t count, hipStream_t s);
hipError_t launch_warm_start(const helios_atm* atm, const float* T_net, int n_out, const double* logP_net,
                             double T_iso, double T_lo, double T_hi, double* T_c, int32_t* fallback,
                             hipStream_t s);

hipError_t launch_grid(const helios_atm* atm, int64_t total_pt, hipStream_t s);
hipError_t launch_profile(const helios_atm* atm, int64_t total_pt, const double* T_c, double* T_pt,
                          hipStream_t s);
// Boundary fluxes (F_int unscaled: the sweep applies sigma T_int^4 / sum of
// bnd_part), Gauss weights and the bin -> atmosphere map, then the Planck
// values at the points.
struct SourceArgs {
    double* B;
    double* F_top;
    double* F_int;
    double* gw;
    int32_t* bin_atm;
    double* bnd_part;
    int32_t bnd_maxch, nb_max, npt_max;
    int32_t iso_grid;  // 1: Planck values of the isothermal-layer grid (see planck_kernel)
    int64_t total_bin;
    double* chunk;     // bolometric workspace [n_chunk][kBolQ][total_pt]: the Planck kernel fills quantities 6, 7
    int64_t total_pt;
    int32_t chunk_bins;  // bins per chunk (bol_chunk_bins of the batch)
};
hipError_t launch_planck(const helios_atm* atm, const double* T_pt, const SourceArgs& sa, const GaussTable& gt,
                         hipStream_t s);
hipError_t launch_mix(const helios_atm* atm, const helios_ktab* kt, const double* T_pt, const double* vmr,
                      void* kappa, bool mixed, int64_t total_pt, const int32_t* n_layer_h,
                      const int32_t* n_bin_h, hipStream_t s);
hipError_t launch_state(const helios_atm* atm, const double* T_pt, double tpe, void* F, int mode, int iso_grid,
                        bool mixed, int64_t total_bin, hipStream_t s);
hipError_t launch_sweep(const SweepArgs& a, int K, int L, bool mixed, int grid, hipStream_t s);  // Rayleigh if a.inv_mbar > 0
hipError_t launch_exact(const SweepArgs& a, int64_t n_bins, hipStream_t s);
hipError_t launch_transmission(const helios_atm* atm, const void* kappa, const double* T_pt,
                               const double* w0, const double* g0, double D, double* out,
                               int64_t total_sub, bool mixed, hipStream_t s);
hipError_t launch_bolometric(const BolArgs& a, int npt_max, int nb_max, int64_t total_pt, hipStream_t s);
hipError_t launch_radeq(const helios_atm* atm, const double* F_bol, double* T_c, double* T_pt,
                        const helios_re_state* st, const helios_re_opts& o, int32_t* status,
                        double* resid, int n_max, hipStream_t s);

// Sweep instantiations available (sublayers per lane).
constexpr int kSweepK[] = {4, 8, 14, 26};
constexpr int kLongK = 26;  // the only K instantiated with L = 64 (columns of up to 1664 sublayers)
// bins per bolometric chunk: 64 keeps enough workgroups in flight for a few
// atmospheres; batches of at least kBolLargeBins bins take 256 (more loads in
// flight per thread, a quarter of the chunk sums)
constexpr int kBolChunkSmall = 64, kBolChunkLarge = 256;
constexpr int64_t kBolLargeBins = 65536;
inline int bol_chunk_bins(int64_t total_bin) { return total_bin >= kBolLargeBins ? kBolChunkLarge : kBolChunkSmall; }
// quantities per (bin chunk, point) in the bolometric workspace: Neumaier
// pairs (sum, compensation) of the up, down and net deviation sums and of
// the width-weighted Planck values
constexpr int kBolQ = 8;
constexpr int kBndChunk = 256;  // bins per boundary-flux workgroup
constexpr int kNumSweepK = 4;

}  // namespace helios
