// k_exact.hip -- pure-absorption flux solve with the exact layer relations
// (Sec. 2.1.2: eq:direct_trans, eq:isodirect, eq:nonisodirect), the check
// against which the two-stream diffusivity approximation (Sec. 2.1.1, D) is
// judged.  Without scattering the two streams do not couple, so one downward
// and one upward sweep per (bin, g) column are exact; w0, g0 and D do not
// enter.
//
// The sweeps carry deviations from the isothermal flux, G = F - pi B(point),
// like the two-stream sweep (pi B is the fixed point of an isothermal layer
// here too).  For a sublayer with transmission T = 2 E3(dtau), 1 - e^-dtau =
// om and Planck difference dB = B_lower - B_upper, eq:nonisodirect becomes
//   up:   G_up(upper)   = T G_up(lower)   + sig
//   down: G_dn(lower)   = T G_dn(upper)   - sig,
//   sig = pi (dB/dtau) (2 om/3 + dtau T/3),
// and eq:isodirect with the mean Planck value (dtau < 1e-4) gives
// sig = pi dB (1 + T)/2.  The boundary values are G_dn(TOA) = F_top - pi
// B(TOA) and G_up(BOA) = G_dn(BOA) + F_int.
#include "helios_internal.hpp"

namespace helios {

// 1/v for the continued fraction's tails (v > x + 1 > 2.5: no scaling
// needed): the hardware estimate refined by two Newton steps, a few ulp.
__device__ inline double rcp_nr(double v) {
    double r = __builtin_amdgcn_rcp(v);
    double e = fma(-v, r, 1.0);
    r = fma(r, e, r);
    e = fma(-v, r, 1.0);
    return fma(r, e, r);
}

// Exponential integral E1(x) for x > 0: its power series
// -gamma - ln x - sum_k (-x)^k / (k k!) (34 terms) for x <= 1.5, else the
// continued fraction e^-x / (x + 1 - 1/(x + 3 - 4/(x + 5 - ...))) evaluated
// from depth 60 back to the front (Abramowitz & Stegun 5.1.11, 5.1.22), each
// tail's reciprocal by Newton-refined hardware estimate.
// Relative error below 3e-15 against scipy with exact divisions (checked
// on the host); the Newton reciprocals add a few ulp.
__device__ inline double e1_d(double x) {
    if (x <= 1.5) {
        constexpr double euler_gamma = 0.57721566490153286061;
        double term = 1.0, sum = 0.0;
#pragma unroll
        for (int k = 1; k <= 34; ++k) {
            const double ik = 1.0 / (double)k;  // a compile-time constant per term
            term *= -x * ik;
            sum -= term * ik;
        }
        return -euler_gamma - log(x) + sum;
    }
    double t = x + 121.0;
    for (int k = 60; k >= 1; --k) t = x + (double)(2 * k - 1) - (double)(k * k) * rcp_nr(t);
    double e, om;
    exp_neg_om(x, e, om);
    return e / t;
}

// eq:direct_trans: T = (1 - x) e^-x + x^2 E1(x) = 2 E3(x), limit 1 at x = 0;
// also returns om = 1 - e^-x.
__device__ inline double exact_trans_d(double x, double& om) {
    double e;
    exp_neg_om(x, e, om);
    if (x == 0.0) return 1.0;
    return (1.0 - x) * e + x * x * e1_d(x);
}

// deviation-form source of one sublayer
__device__ inline double exact_sig(double dtau, double T, double om, double dB) {
    if (dtau < 1e-4) return 0.5 * kPi * dB * (1.0 + T);
    return kPi * (dB / dtau) * (2.0 * om / 3.0 + dtau * T / 3.0);
}

// Workgroup = 64 / n_g bins side by side (a grid-stride loop over groups of
// bins of the launch): lane t walks column t % n_g of bin slot t / n_g down
// and up, storing its deviations in the per-g arrays; the workgroup then
// forms the Gauss partials of each of its bins' points in g order (one
// partial per (bin, point)).  The bins of a workgroup may belong to
// different atmospheres, so everything per bin is per lane; the barriers
// and the partial loops are uniform.
__device__ inline int exact_bins_per_wave(int n_g) { return 64 / n_g; }

__global__ void __launch_bounds__(64) exact_kernel(const SweepArgs A) {
    const double* __restrict__ kap_all = static_cast<const double*>(A.kappa);
    const double* __restrict__ B_all = static_cast<const double*>(A.B);
    double* __restrict__ Fu = static_cast<double*>(A.F_up_g);
    double* __restrict__ Fd = static_cast<double*>(A.F_dn_g);
    double* __restrict__ part_up = static_cast<double*>(A.part_up);
    double* __restrict__ part_dn = static_cast<double*>(A.part_dn);
    const int bpw = exact_bins_per_wave(A.n_g);
    const int slot = threadIdx.x / A.n_g, g = threadIdx.x - slot * A.n_g;
    for (int64_t base = A.w_begin + (int64_t)blockIdx.x * bpw; base < A.w_end; base += (int64_t)gridDim.x * bpw) {
        const int64_t gb = base + slot;
        if (slot < bpw && gb < A.w_end) {
            const int at = A.bin_atm[gb];
            if (!frozen(A.status, at)) {
                const int l = (int)(gb - A.bin_off[at]);
                const int n = A.n_layer[at];
                const int nsub = 2 * n, npt = nsub + 1;
                const int cs = col_stride(n);
                const int64_t pb = A.pb_off[at] + (int64_t)l * npt;
                const double* __restrict__ P = A.P_pt + A.pt_off[at];
                const double* __restrict__ B = B_all + pb;
                const double igrav = 1.0 / A.grav[at];
                const int64_t bin = A.bin_off[at] + l;
                const int64_t cell0 = A.cell_off[at] + (int64_t)l * A.n_g * cs;
                // BOA flux scale: sigma T_int^4 over the atmosphere's in-band sum (chunk sums in order)
                double sum = 0.0;
                const int nbch = (int)((A.bin_off[at + 1] - A.bin_off[at] + kBndChunk - 1) / kBndChunk);
                for (int c = 0; c < nbch; ++c) sum += A.bnd_part[(int64_t)at * A.bnd_maxch + c];
                const double t2 = A.T_int[at] * A.T_int[at];
                const double Fint = A.F_int[bin] * ((sum > 0.0) ? sigma_sb() * t2 * t2 / sum : 0.0);
                const double* kap = kap_all + cell0 + (int64_t)g * cs;
                double* up = Fu + cell0 + (int64_t)g * cs;
                double* dn = Fd + cell0 + (int64_t)g * cs;
                double G = A.F_top[bin] - kPi * B[nsub];
                dn[nsub] = G;
                for (int s = nsub - 1; s >= 0; --s) {
                    const double dtau = 0.5 * (kap[s] + kap[s + 1]) * (P[s] - P[s + 1]) * igrav;
                    double om;
                    const double T = exact_trans_d(dtau, om);
                    G = T * G - exact_sig(dtau, T, om, B[s] - B[s + 1]);
                    dn[s] = G;
                    up[s + 1] = T;  // kept for the upward sweep, which overwrites it after use
                }
                G += Fint;
                up[0] = G;
                for (int s = 0; s < nsub; ++s) {
                    const double dtau = 0.5 * (kap[s] + kap[s + 1]) * (P[s] - P[s + 1]) * igrav;
                    double e, om;
                    exp_neg_om(dtau, e, om);
                    const double T = up[s + 1];
                    G = T * G + exact_sig(dtau, T, om, B[s] - B[s + 1]);
                    up[s + 1] = G;
                }
            }
        }
        __syncthreads();
        for (int k = 0; k < bpw; ++k) {  // uniform: the bins of this group in turn
            const int64_t gk = base + k;
            if (gk >= A.w_end) break;
            const int at = A.bin_atm[gk];
            if (frozen(A.status, at)) continue;
            const int l = (int)(gk - A.bin_off[at]);
            const int n = A.n_layer[at];
            const int npt = 2 * n + 1;
            const int cs = col_stride(n);
            const int64_t pb = A.pb_off[at] + (int64_t)l * npt;
            const int64_t cell0 = A.cell_off[at] + (int64_t)l * A.n_g * cs;
            const double* __restrict__ B = static_cast<const double*>(A.B) + pb;
            for (int p = threadIdx.x; p < npt; p += blockDim.x) {
                double su = 0.0, sd = 0.0;
                const double piB = kPi * B[p];
                for (int c = 0; c < A.n_g; ++c) {
                    const int64_t cell = cell0 + (int64_t)c * cs + p;
                    const double u = Fu[cell], d = Fd[cell];
                    su += A.gw[c] * u;
                    sd += A.gw[c] * d;
                    if (A.flux_state) {  // the caller keeps fluxes, not deviations from pi B
                        Fu[cell] = u + piB;
                        Fd[cell] = d + piB;
                    }
                }
                part_up[pb * A.wpb_stride + p] = su;
                part_dn[pb * A.wpb_stride + p] = sd;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_exact(const SweepArgs& a, int64_t n_bins, hipStream_t s) {
    const int bpw = 64 / a.n_g;
    const int64_t groups = (n_bins + bpw - 1) / bpw;
    const int64_t grid = groups < 0x7fffffff ? groups : 0x7fffffff;
    hipLaunchKernelGGL(exact_kernel, dim3((unsigned)grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace helios
