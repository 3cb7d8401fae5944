// k_mix.hip -- opacity at the points (Sec. 2.3, eq:kappa_gauss, eq:mixing):
//   kappa[bin][g][pt] = sum_j X_j m_j / mbar * k_j(T_pt, P_pt; bin_index[bin], g)
// with k_j bilinear in (T, log10 P) on a uniform table grid, coordinates
// clamped to the table, or a power law in P and T.
//
// Work decomposition: a workgroup owns 16 consecutive points of the
// concatenated point axis (possibly straddling two atmospheres) and 256
// consecutive (bin, g) columns.  Per point, the interpolation weights and
// mass mixing ratios are computed once and kept in LDS.  For a fixed point,
// the 256 threads read consecutive (bin, g) entries of each table corner row
// (coalesced, contiguous when bin_index is), and neighbouring points of one
// workgroup reuse the same corner rows through the caches.  Results go
// through an LDS tile so that each column's 16 points are written as one
// contiguous run in the [bin][g][pt] output.
#include "helios_internal.hpp"

namespace helios {

constexpr int kMixPts = 32;
constexpr int kMixCols = 128;

struct MixArgs {
    helios_atm atm;
    const float* k;
    const double* k0;
    const double* T_pt;
    const double* vmr;  // [n_species][total_pt]
    void* kappa;
    int64_t total_pt;
    int32_t mode, n_species, nT, nP, nbt, ng;
    double T_min, T_step, logP_min, logP_step;
    double p_exp, t_exp, P_ref, T_ref;
    double mratio[HELIOS_MAX_SPECIES];  // m_j / mbar
};

// A workgroup owns kMixPts consecutive points of the concatenated point axis
// (possibly straddling atmospheres) and kMixCols consecutive (bin, g)
// columns.  Per point the table cell, corner weights and mass mixing ratios
// are computed once (LDS).  Consecutive points usually fall in the same
// (T, log P) cell; a thread keeps the cell's corner values of its column in
// registers and reloads them only when the cell changes (a workgroup-uniform
// decision).
template <typename R>
__global__ void __launch_bounds__(kMixCols) mix_kernel(const MixArgs A) {
    __shared__ int s_atm[kMixPts], s_p[kMixPts], s_npt[kMixPts], s_ncol[kMixPts], s_cell[kMixPts];
    __shared__ R s_w[kMixPts][4];                   // bilinear corner weights or power-law scale
    __shared__ R s_x[kMixPts][HELIOS_MAX_SPECIES];  // mass mixing ratios
    __shared__ R tile[kMixPts][kMixCols + 1];

    const int t = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * kMixPts;
    const int c0 = blockIdx.y * kMixCols;
    if (t < kMixPts) {
        const int64_t gp = p0 + t;
        if (gp < A.total_pt) {
            const int a = find_atm(A.atm.pt_off, A.atm.n_atm, gp);
            const int n = A.atm.n_layer[a];
            s_atm[t] = a;
            s_p[t] = (int)(gp - A.atm.pt_off[a]);
            s_npt[t] = 2 * n + 1;
            s_ncol[t] = (int)(A.atm.bin_off[a + 1] - A.atm.bin_off[a]) * A.ng;
            const double T = A.T_pt[gp], P = A.atm.P_pt[gp];
            for (int j = 0; j < A.n_species; ++j)
                s_x[t][j] = (R)(A.vmr[(int64_t)j * A.total_pt + gp] * A.mratio[j]);
            if (A.mode == HELIOS_KTAB_TABLE) {
                double x = (T - A.T_min) / A.T_step;
                double y = (log10(P) - A.logP_min) / A.logP_step;
                x = fmin(fmax(x, 0.0), (double)(A.nT - 1));
                y = fmin(fmax(y, 0.0), (double)(A.nP - 1));
                const int iT = min((int)floor(x), A.nT - 2);
                const int iP = min((int)floor(y), A.nP - 2);
                const double fT = x - iT, fP = y - iP;
                s_cell[t] = (a * A.nT + iT) * A.nP + iP;
                s_w[t][0] = (R)((1.0 - fT) * (1.0 - fP));
                s_w[t][1] = (R)((1.0 - fT) * fP);
                s_w[t][2] = (R)(fT * (1.0 - fP));
                s_w[t][3] = (R)(fT * fP);
            } else {
                s_cell[t] = a;
                s_w[t][0] = (R)(pow(P / A.P_ref, A.p_exp) * pow(T / A.T_ref, A.t_exp));
            }
        } else {
            s_atm[t] = -1;
            s_ncol[t] = 0;
            s_cell[t] = -1;
        }
    }
    __syncthreads();

    const int c = c0 + t;
    const size_t row = (size_t)A.nbt * A.ng;  // one (species, T, P) corner row
    R kc[HELIOS_MAX_SPECIES][4];
#pragma unroll
    for (int sp = 0; sp < HELIOS_MAX_SPECIES; ++sp)
        kc[sp][0] = kc[sp][1] = kc[sp][2] = kc[sp][3] = (R)0;
    int cur = -2;
    for (int j = 0; j < kMixPts; ++j) {
        R acc = (R)0;
        const int a = s_atm[j];
        if (a >= 0 && s_cell[j] != cur) {  // uniform: load the new cell's corners
            cur = s_cell[j];
            if (c < s_ncol[j]) {
                const int l = c / A.ng, g = c - l * A.ng;
                // a bad caller index must not read outside the table
                const int bt = min(max(A.atm.bin_index[A.atm.bin_off[a] + l], 0), A.nbt - 1);
                const size_t off = (size_t)bt * A.ng + g;
                if (A.mode == HELIOS_KTAB_TABLE) {
                    const int cell = cur - a * A.nT * A.nP;  // iT * nP + iP
#pragma unroll
                    for (int sp = 0; sp < HELIOS_MAX_SPECIES; ++sp) {
                        if (sp < A.n_species) {
                            const float* kb = A.k + ((size_t)sp * A.nT * A.nP + cell) * row + off;
                            kc[sp][0] = (R)kb[0];
                            kc[sp][1] = (R)kb[row];
                            kc[sp][2] = (R)kb[(size_t)A.nP * row];
                            kc[sp][3] = (R)kb[(size_t)(A.nP + 1) * row];
                        }
                    }
                } else {
#pragma unroll
                    for (int sp = 0; sp < HELIOS_MAX_SPECIES; ++sp)
                        if (sp < A.n_species) kc[sp][0] = (R)A.k0[(size_t)sp * row + off];
                }
            }
        }
        if (a >= 0 && c < s_ncol[j]) {
            if (A.mode == HELIOS_KTAB_TABLE) {
                const R w00 = s_w[j][0], w01 = s_w[j][1], w10 = s_w[j][2], w11 = s_w[j][3];
#pragma unroll
                for (int sp = 0; sp < HELIOS_MAX_SPECIES; ++sp)
                    if (sp < A.n_species)
                        acc += s_x[j][sp] * (w00 * kc[sp][0] + w01 * kc[sp][1] + w10 * kc[sp][2] + w11 * kc[sp][3]);
            } else {
#pragma unroll
                for (int sp = 0; sp < HELIOS_MAX_SPECIES; ++sp)
                    if (sp < A.n_species) acc += s_x[j][sp] * kc[sp][0];
                acc *= s_w[j][0];
            }
        }
        tile[j][t] = acc;
    }
    __syncthreads();

    R* out = (R*)A.kappa;
    for (int e = t; e < kMixPts * kMixCols; e += kMixCols) {
        const int cl = e / kMixPts, j = e - cl * kMixPts;
        const int cc = c0 + cl;
        if (s_atm[j] >= 0 && cc < s_ncol[j]) {
            const int a = s_atm[j];
            out[A.atm.cell_off[a] + (int64_t)cc * s_npt[j] + s_p[j]] = tile[j][cl];
        }
    }
}

hipError_t launch_mix(const helios_atm* atm, const helios_ktab* kt, const double* T_pt, const double* vmr,
                      void* kappa, bool mixed, int64_t total_pt, const int32_t* /*n_layer_h*/,
                      const int32_t* n_bin_h, hipStream_t s) {
    MixArgs A;
    A.atm = *atm;
    A.k = kt->k;
    A.k0 = kt->k0;
    A.T_pt = T_pt;
    A.vmr = vmr;
    A.kappa = kappa;
    A.total_pt = total_pt;
    A.mode = kt->mode;
    A.n_species = kt->n_species;
    A.nT = kt->n_T;
    A.nP = kt->n_P;
    A.nbt = kt->n_bin_table;
    A.ng = kt->n_g;
    A.T_min = kt->T_min;
    A.T_step = kt->T_step;
    A.logP_min = kt->logP_min;
    A.logP_step = kt->logP_step;
    A.p_exp = kt->p_exp;
    A.t_exp = kt->t_exp;
    A.P_ref = kt->P_ref;
    A.T_ref = kt->T_ref;
    for (int j = 0; j < HELIOS_MAX_SPECIES; ++j)
        A.mratio[j] = (j < kt->n_species) ? kt->species_mass[j] / kt->mmw : 0.0;
    int max_cols = 0;
    for (int a = 0; a < atm->n_atm; ++a) max_cols = max(max_cols, n_bin_h[a] * kt->n_g);
    dim3 grid((unsigned)((total_pt + kMixPts - 1) / kMixPts), (unsigned)((max_cols + kMixCols - 1) / kMixCols));
    if (mixed)
        hipLaunchKernelGGL(mix_kernel<float>, grid, dim3(kMixCols), 0, s, A);
    else
        hipLaunchKernelGGL(mix_kernel<double>, grid, dim3(kMixCols), 0, s, A);
    return hipGetLastError();
}

}  // namespace helios
