// k_mix.hip -- opacity at the points (Sec. 2.3, eq:kappa_gauss, eq:mixing):
//   kappa[bin][g][pt] = sum_j X_j m_j / mbar * k_j(T_pt, P_pt; bin_index[bin], g)
// with k_j bilinear in (T, log10 P) on a uniform table grid, coordinates
// clamped to the table, or a power law in P and T.
//
// Work decomposition: a workgroup owns one aligned chunk of kMixPts points of
// one atmosphere and kMixCols consecutive (bin, g) columns; each thread is
// one column.  Per point the table cell, corner weights and mass mixing
// ratios are computed once (LDS).  Consecutive points usually fall in the
// same (T, log P) cell: a thread keeps the cell's corner values of its column
// in registers and reloads them only when the cell changes (a
// workgroup-uniform decision), and it issues the loads of the next cell's
// corners as soon as a cell is entered, so they are in flight while the
// current cell's points are computed.  For a fixed point the threads read
// consecutive (bin, g) entries of each corner row (coalesced).  A thread's
// kMixPts results (32 in FP32, 16 in FP64) are an aligned 128-byte piece of
// its column (the column stride is padded to a multiple of 32 points); the
// workgroup passes them through LDS so that consecutive lanes store
// consecutive 16-byte vectors of one piece (whole cache lines per store),
// up to the last valid point.
#include "helios_internal.hpp"

namespace helios {

// points per workgroup (a divisor of the column stride's 32-point alignment;
// 16 keeps a thread's results in few registers and gives many workgroups)
template <typename R>
constexpr int mix_pts() { return sizeof(R) == 4 ? 32 : 16; }
constexpr int kMixCols = 256;

struct MixArgs {
    helios_atm atm;
    const float* k;
    const double* k0;
    const double* T_pt;
    const double* vmr;  // [n_species][total_pt]
    void* kappa;
    int64_t total_pt;
    int32_t mode, n_species, nT, nP, nbt, ng;
    int32_t max_chunks;  // chunks of mix_pts<R>() points per atmosphere (largest)
    double T_min, T_step, logP_min, logP_step;
    double p_exp, t_exp, P_ref, T_ref;
    double mratio[HELIOS_MAX_SPECIES];  // m_j / mbar
};

template <typename R>
struct Vec2;
template <>
struct Vec2<float> {
    using type = float4;
    static constexpr int per = 4;
};
template <>
struct Vec2<double> {
    using type = double2;
    static constexpr int per = 2;
};

template <typename R, int NSP>
__global__ void __launch_bounds__(kMixCols) mix_kernel(const MixArgs A) {
    constexpr int kMixPts = mix_pts<R>();
    __shared__ int s_cell[kMixPts];
    __shared__ int s_next[kMixPts];  // at the first point of a run of equal cells: the next run's cell, or -1
    __shared__ R s_w[kMixPts][4];    // bilinear corner weights or power-law scale
    __shared__ R s_x[kMixPts][NSP];  // mass mixing ratios
    __shared__ R s_out[kMixCols][kMixPts + 1];  // the workgroup's results, re-read for coalesced stores

    const int t = threadIdx.x;
    const int a = blockIdx.x / A.max_chunks;
    const int ch = blockIdx.x - a * A.max_chunks;
    const int n = A.atm.n_layer[a];
    const int npt = 2 * n + 1;
    const int p0 = ch * kMixPts;
    if (p0 >= npt || frozen(A.atm.status, a)) return;  // uniform: past the points, or converged
    const int ncol = (int)(A.atm.bin_off[a + 1] - A.atm.bin_off[a]) * A.ng;
    const int c = blockIdx.y * kMixCols + t;
    if ((int)blockIdx.y * kMixCols >= ncol) return;  // uniform: past this atmosphere's columns
    const int npts = min(kMixPts, npt - p0);        // valid points of the chunk
    if (t < npts) {
        const int64_t gp = A.atm.pt_off[a] + p0 + t;
        const double T = A.T_pt[gp], P = A.atm.P_pt[gp];
        for (int j = 0; j < NSP; ++j)
            s_x[t][j] = (j < A.n_species) ? (R)(A.vmr[(int64_t)j * A.total_pt + gp] * A.mratio[j]) : (R)0;
        if (A.mode == HELIOS_KTAB_TABLE) {
            double x = (T - A.T_min) / A.T_step;
            double y = (log10(P) - A.logP_min) / A.logP_step;
            x = fmin(fmax(x, 0.0), (double)(A.nT - 1));
            y = fmin(fmax(y, 0.0), (double)(A.nP - 1));
            const int iT = min((int)floor(x), A.nT - 2);
            const int iP = min((int)floor(y), A.nP - 2);
            const double fT = x - iT, fP = y - iP;
            s_cell[t] = iT * A.nP + iP;
            s_w[t][0] = (R)((1.0 - fT) * (1.0 - fP));
            s_w[t][1] = (R)((1.0 - fT) * fP);
            s_w[t][2] = (R)(fT * (1.0 - fP));
            s_w[t][3] = (R)(fT * fP);
        } else {
            s_cell[t] = 0;
            s_w[t][0] = (R)(pow(P / A.P_ref, A.p_exp) * pow(T / A.T_ref, A.t_exp));
        }
    }
    __syncthreads();
    if (t < 64) {  // runs of equal cells along the chunk: where each starts, and what follows it (one wave)
        const bool start = (t < npts) && (t == 0 || s_cell[t] != s_cell[t - 1]);
        const unsigned long long starts = __ballot(start);
        if (t < npts) {
            const unsigned long long later = (t + 1 < 64) ? (starts >> (t + 1)) : 0ull;
            const int nx = later ? t + 1 + __builtin_ctzll(later) : -1;  // the next run's first point
            s_next[t] = start ? (nx >= 0 ? s_cell[nx] : -1) : -2;
        }
    }
    __syncthreads();
    const bool colv = c < ncol;  // threads past the columns still take part in the barrier below
    const int cq = colv ? c : ncol - 1;

    const int l = cq / A.ng, g = cq - l * A.ng;
    // a bad caller index must not read outside the table
    const int bt = min(max(A.atm.bin_index[A.atm.bin_off[a] + l], 0), A.nbt - 1);
    const size_t row = (size_t)A.nbt * A.ng;  // one (species, T, P) corner row
    const size_t off = (size_t)bt * A.ng + g;
    float kc[NSP][4], kn[NSP][4];  // corners of the current cell and of the next one (in flight)
    R kr[sizeof(R) == 8 ? NSP : 1][4];  // FP64: the current cell's corners converted once per run
    auto load_cell = [&](float (&dst)[NSP][4], int cell) {
#pragma unroll
        for (int sp = 0; sp < NSP; ++sp) {
            const float* kb = A.k + ((size_t)sp * A.nT * A.nP + cell) * row + off;
            const bool ok = sp < A.n_species;
            dst[sp][0] = ok ? kb[0] : 0.0f;
            dst[sp][1] = ok ? kb[row] : 0.0f;
            dst[sp][2] = ok ? kb[(size_t)A.nP * row] : 0.0f;
            dst[sp][3] = ok ? kb[(size_t)(A.nP + 1) * row] : 0.0f;
        }
    };
    R kp[NSP];  // power-law coefficients
    R vals[kMixPts];
    int cur = -1;
#pragma unroll
    for (int j = 0; j < kMixPts; ++j) {
        R acc = (R)0;
        if (j < npts) {
            if (A.mode == HELIOS_KTAB_TABLE) {
                const int nx = s_next[j];
                if (nx != -2) {  // uniform: a new run of equal cells starts here
                    if (j == 0) load_cell(kc, s_cell[0]);
                    else {
#pragma unroll
                        for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
                            for (int q = 0; q < 4; ++q) kc[sp][q] = kn[sp][q];
                    }
                    if constexpr (sizeof(R) == 8) {
#pragma unroll
                        for (int sp = 0; sp < NSP; ++sp)
#pragma unroll
                            for (int q = 0; q < 4; ++q) kr[sp][q] = (R)kc[sp][q];  // once per run
                    }
                    if (nx >= 0) load_cell(kn, nx);  // the following run's corners
                }
                const R w00 = s_w[j][0], w01 = s_w[j][1], w10 = s_w[j][2], w11 = s_w[j][3];
                if constexpr (sizeof(R) == 8) {
#pragma unroll
                    for (int sp = 0; sp < NSP; ++sp)
                        acc += s_x[j][sp] * (w00 * kr[sp][0] + w01 * kr[sp][1] + w10 * kr[sp][2] + w11 * kr[sp][3]);
                } else {
#pragma unroll
                    for (int sp = 0; sp < NSP; ++sp)
                        acc += s_x[j][sp] * (w00 * kc[sp][0] + w01 * kc[sp][1] + w10 * kc[sp][2] + w11 * kc[sp][3]);
                }
            } else {
                if (cur < 0) {
                    cur = 0;
#pragma unroll
                    for (int sp = 0; sp < NSP; ++sp)
                        kp[sp] = (sp < A.n_species) ? (R)A.k0[(size_t)sp * row + off] : (R)0;
                }
#pragma unroll
                for (int sp = 0; sp < NSP; ++sp) acc += s_x[j][sp] * kp[sp];
                acc *= s_w[j][0];
            }
        }
        vals[j] = acc;
    }
    // stores through LDS: each column's piece of the chunk (kMixPts points,
    // 128 bytes) is written by kMixPts/per consecutive lanes, so a wave's
    // vector store covers whole 128-byte lines instead of one 16-byte piece
    // of 64 different lines
#pragma unroll
    for (int j = 0; j < kMixPts; ++j) s_out[t][j] = vals[j];
    __syncthreads();
    using V = typename Vec2<R>::type;
    constexpr int per = Vec2<R>::per;
    constexpr int vpc = kMixPts / per;  // vectors per column piece
    const int cs = col_stride(n);
    R* __restrict__ kap = static_cast<R*>(A.kappa) + A.atm.cell_off[a] + (int64_t)blockIdx.y * kMixCols * cs + p0;
#pragma unroll
    for (int r = 0; r < vpc; ++r) {
        const int q = r * kMixCols + t;
        const int cc = q / vpc, v = q - cc * vpc;
        // whole vectors covering the valid points (column padding past them is not written)
        if ((int)blockIdx.y * kMixCols + cc < ncol && per * v < npts) {
            V w;
            if constexpr (per == 4)
                w = V{s_out[cc][4 * v], s_out[cc][4 * v + 1], s_out[cc][4 * v + 2], s_out[cc][4 * v + 3]};
            else
                w = V{s_out[cc][2 * v], s_out[cc][2 * v + 1]};
            using NV = R __attribute__((ext_vector_type(per)));
            NV nv;
            if constexpr (per == 4) nv = NV{w.x, w.y, w.z, w.w};
            else nv = NV{w.x, w.y};
            // streamed past the caches: the array is far larger than they are
            __builtin_nontemporal_store(nv, reinterpret_cast<NV*>(kap + (int64_t)cc * cs + per * v));
        }
    }
}

hipError_t launch_mix(const helios_atm* atm, const helios_ktab* kt, const double* T_pt, const double* vmr,
                      void* kappa, bool mixed, int64_t total_pt, const int32_t* n_layer_h,
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
    int max_cols = 0, max_chunks = 1;
    for (int a = 0; a < atm->n_atm; ++a) {
        max_cols = max(max_cols, n_bin_h[a] * kt->n_g);
        max_chunks = max(max_chunks, col_stride(n_layer_h[a]) / (mixed ? mix_pts<float>() : mix_pts<double>()));
    }
    A.max_chunks = max_chunks;
    dim3 grid((unsigned)(atm->n_atm * max_chunks), (unsigned)((max_cols + kMixCols - 1) / kMixCols));
    const bool few = kt->n_species <= 4;
    if (mixed) {
        if (few) hipLaunchKernelGGL((mix_kernel<float, 4>), grid, dim3(kMixCols), 0, s, A);
        else hipLaunchKernelGGL((mix_kernel<float, HELIOS_MAX_SPECIES>), grid, dim3(kMixCols), 0, s, A);
    } else {
        if (few) hipLaunchKernelGGL((mix_kernel<double, 4>), grid, dim3(kMixCols), 0, s, A);
        else hipLaunchKernelGGL((mix_kernel<double, HELIOS_MAX_SPECIES>), grid, dim3(kMixCols), 0, s, A);
    }
    return hipGetLastError();
}

}  // namespace helios
