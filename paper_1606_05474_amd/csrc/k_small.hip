// k_small.hip -- the light kernels of the hot path: point grid and interface
// temperatures (Sec. 2.2.1), Planck sources and boundary fluxes (Sec. 2.2.2),
// the width-weighted bin sum to bolometric fluxes (Sec. 2.2.3) and the FP64
// temperature update (Sec. 2.2.3-2.2.4).
#include "helios_internal.hpp"

namespace helios {

// ------------------------------------------------------------------ grid
// One thread per point.  Centres are copied to odd points; interface i sits
// at the geometric mean of centres i-1 and i; the outer interfaces are half a
// log-step beyond the outermost centres.
__global__ void grid_kernel(helios_atm atm, int64_t total_pt) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total_pt) return;
    int a = find_atm(atm.pt_off, atm.n_atm, idx);
    int p = (int)(idx - atm.pt_off[a]);
    int n = atm.n_layer[a];
    const double* Pc = atm.P_c + atm.lay_off[a];
    int i = p >> 1;
    double P;
    if (p & 1) P = Pc[i];
    else if (i == 0) P = Pc[0] * sqrt(Pc[0] / Pc[1]);
    else if (i == n) P = Pc[n - 1] * sqrt(Pc[n - 1] / Pc[n - 2]);
    else P = sqrt(Pc[i - 1] * Pc[i]);
    atm.P_pt[idx] = P;
}

hipError_t launch_grid(const helios_atm* atm, int64_t total_pt, hipStream_t s) {
    int block = 256;
    int64_t grid = (total_pt + block - 1) / block;
    hipLaunchKernelGGL(grid_kernel, dim3((unsigned)grid), dim3(block), 0, s, *atm, total_pt);
    return hipGetLastError();
}

// Interface temperature of point p of one atmosphere from its centres.
__device__ inline double interface_T(const double* __restrict__ P, const double* __restrict__ Tc, int n,
                                     int p) {
    int i = p >> 1;
    if (p & 1) return Tc[i];
    if (i == 0) return Tc[0];
    if (i == n) return Tc[n - 1];
    double x0 = log(P[p - 1]), x1 = log(P[p + 1]), x = log(P[p]);
    double f = (x - x0) / (x1 - x0);
    return Tc[i - 1] + f * (Tc[i] - Tc[i - 1]);
}

__global__ void profile_kernel(helios_atm atm, int64_t total_pt, const double* __restrict__ T_c,
                               double* __restrict__ T_pt) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total_pt) return;
    int a = find_atm(atm.pt_off, atm.n_atm, idx);
    int p = (int)(idx - atm.pt_off[a]);
    T_pt[idx] = interface_T(atm.P_pt + atm.pt_off[a], T_c + atm.lay_off[a], atm.n_layer[a], p);
}

hipError_t launch_profile(const helios_atm* atm, int64_t total_pt, const double* T_c, double* T_pt,
                          hipStream_t s) {
    int block = 256;
    int64_t grid = (total_pt + block - 1) / block;
    hipLaunchKernelGGL(profile_kernel, dim3((unsigned)grid), dim3(block), 0, s, *atm, total_pt, T_c, T_pt);
    return hipGetLastError();
}

// --------------------------------------------------------------- sources
// Neumaier summation (a compensated sum: the pair (s, c) carries the rounding
// errors of the running sum s in c).
struct nacc {
    double s, c;
};
__device__ inline void nadd(nacc& a, double v) {
    double t = a.s + v;
    if (fabs(a.s) >= fabs(v)) a.c += (a.s - t) + v;
    else a.c += (v - t) + a.s;
    a.s = t;
}

// B[bin][pt] at the bin centres, and per (chunk of cb bins, point)
// the width-weighted sum of the chunk's Planck values, which the bolometric
// up and down fluxes take from here (times 2 pi eps and the Gauss-weight
// sum) instead of re-reading B.  Workgroup = (atmosphere, 64-point tile,
// chunk of cb bins), 1024 threads = 64 points x 16 groups of cb/16 bins
// (cb = 64 or 256, by batch size), as the bin sum; the group sums are combined in a fixed
// order.
//
// On the isothermal-layer grid (Sec. 2.2.1) layer i has the single
// temperature of its centre (point 2i+1), and the sweep's reference values
// are B(T_i) at points 2i and 2i+1 and B(T_{n-1}) at the TOA point 2n.
__global__ void __launch_bounds__(1024) planck_kernel(helios_atm atm, const double* __restrict__ T_pt,
                                                      double* __restrict__ B, double* __restrict__ chunk,
                                                      int64_t total_pt, int iso_grid, int cb) {
    __shared__ double red[16][64][2];
    const int a = blockIdx.x;
    const int tile = blockIdx.y, ch = blockIdx.z;
    const int pl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int npt = 2 * atm.n_layer[a] + 1;
    const int nb = (int)(atm.bin_off[a + 1] - atm.bin_off[a]);
    if (tile * 64 >= npt || ch * cb >= nb || frozen(atm.status, a)) return;  // uniform
    const int p = tile * 64 + pl;
    const int per = cb / 16;
    const int l0 = ch * cb + q * per;
    nacc acc = {0.0, 0.0};
    if (p < npt) {
        const int pt = (!iso_grid || (p & 1)) ? p : (p + 1 < npt ? p + 1 : p - 1);
        const double T = T_pt[atm.pt_off[a] + pt];
        const int64_t b0 = atm.bin_off[a];
        double* __restrict__ Ba = B + atm.pb_off[a];
#pragma unroll 4
        for (int i = 0; i < per; ++i) {
            const int l = l0 + i;
            if (l < nb) {
                const double v = planck_d(atm.lambda_c[b0 + l], T);
                __builtin_nontemporal_store(v, Ba + (int64_t)l * npt + p);
                nadd(acc, atm.dlambda[b0 + l] * v);
            }
        }
    }
    red[q][pl][0] = acc.s;
    red[q][pl][1] = acc.c;
    __syncthreads();
    if (q == 0 && p < npt) {
        nacc t = {0.0, 0.0};
        double cc = 0.0;
        for (int k = 0; k < 16; ++k) {
            nadd(t, red[k][pl][0]);
            cc += red[k][pl][1];
        }
        const int64_t gpt = atm.pt_off[a] + p;
        chunk[((int64_t)ch * kBolQ + 6) * total_pt + gpt] = t.s;
        chunk[((int64_t)ch * kBolQ + 7) * total_pt + gpt] = t.c + cc;
    }
}

// Boundary fluxes (Sec. 2.2.2), workgroup = (atmosphere, chunk of kBndChunk
// bins): TOA (T_irr/T_star)^4 pi B(T_star); BOA pi B(T_int), left unscaled,
// with the chunk's sum of pi B(T_int) dlambda (a fixed-order tree in LDS) in
// bnd_part.  The sweep scales the BOA flux so that its width-weighted sum over
// the atmosphere's bins is sigma T_int^4.  The same workgroups write the
// Gauss weights and the bin -> atmosphere map.
__global__ void __launch_bounds__(kBndChunk) boundary_kernel(helios_atm atm, SourceArgs sa, GaussTable gt) {
    __shared__ double red[kBndChunk];
    const int a = blockIdx.x, ch = blockIdx.y;
    const int t = threadIdx.x;
    if (a == 0 && ch == 0 && t < atm.n_g) sa.gw[t] = gt.w[t];
    const int nb = (int)(atm.bin_off[a + 1] - atm.bin_off[a]);
    if (ch * kBndChunk >= nb) return;  // uniform
    const int64_t b0 = atm.bin_off[a];
    const int l = ch * kBndChunk + t;
    if (l < nb) sa.bin_atm[b0 + l] = a;
    if (frozen(atm.status, a)) return;  // uniform
    const double Ts = atm.T_star[a], Ti = atm.T_int[a];
    const double r = (Ts > 0.0) ? atm.T_irr[a] / Ts : 0.0;
    const double dil = r * r * r * r;
    double part = 0.0;
    if (l < nb) {
        const double lam = atm.lambda_c[b0 + l];
        sa.F_top[b0 + l] = dil * kPi * planck_d(lam, Ts);
        const double fi = kPi * planck_d(lam, Ti);
        sa.F_int[b0 + l] = fi;
        part = fi * atm.dlambda[b0 + l];
    }
    red[t] = part;
    __syncthreads();
    for (int st = kBndChunk / 2; st > 0; st >>= 1) {
        if (t < st) red[t] += red[t + st];
        __syncthreads();
    }
    if (t == 0) sa.bnd_part[(int64_t)a * sa.bnd_maxch + ch] = red[0];
}

constexpr int kStateThreads = 128;

// Conversion of a per-g cell array between fluxes and deviations from the
// isothermal flux (2 pi / D) B (Sec. 2.2.3; see helios_state_convert):
// workgroup = one bin, threads over its points; each point's reference is
// formed once in FP64 and applied to the bin's n_g columns (coalesced along
// the points of a column).  mode 0: F - tpe B, 1: G + tpe B, 2: -tpe B.
template <typename R>
__global__ void __launch_bounds__(kStateThreads) state_kernel(helios_atm atm, const double* __restrict__ T_pt,
                                                               double tpe, R* __restrict__ F, int mode,
                                                               int iso_grid) {
    const int64_t b = blockIdx.x;
    const int a = find_atm(atm.bin_off, atm.n_atm, b);
    if (frozen(atm.status, a)) return;  // uniform per workgroup
    const int n = atm.n_layer[a];
    const int npt = 2 * n + 1, cs = col_stride(n);
    const double lam = atm.lambda_c[b];
    const double* __restrict__ T = T_pt + atm.pt_off[a];
    R* __restrict__ col0 = F + atm.cell_off[a] + (b - atm.bin_off[a]) * atm.n_g * cs;
    for (int p = threadIdx.x; p < npt; p += kStateThreads) {
        const int pt = (!iso_grid || (p & 1)) ? p : (p + 1 < npt ? p + 1 : p - 1);
        const double ref = tpe * planck_d(lam, T[pt]);
        for (int g = 0; g < atm.n_g; ++g) {
            R* c = col0 + (int64_t)g * cs + p;
            const double v = (mode == 2) ? -ref : (mode == 1 ? (double)*c + ref : (double)*c - ref);
            *c = (R)v;
        }
    }
}

hipError_t launch_state(const helios_atm* atm, const double* T_pt, double tpe, void* F, int mode, int iso_grid,
                        bool mixed, int64_t total_bin, hipStream_t s) {
    if (mixed)
        hipLaunchKernelGGL(state_kernel<float>, dim3((unsigned)total_bin), dim3(kStateThreads), 0, s, *atm, T_pt,
                           tpe, (float*)F, mode, iso_grid);
    else
        hipLaunchKernelGGL(state_kernel<double>, dim3((unsigned)total_bin), dim3(kStateThreads), 0, s, *atm, T_pt,
                           tpe, (double*)F, mode, iso_grid);
    return hipGetLastError();
}

hipError_t launch_planck(const helios_atm* atm, const double* T_pt, const SourceArgs& sa, const GaussTable& gt,
                         hipStream_t s) {
    hipLaunchKernelGGL(boundary_kernel, dim3(atm->n_atm, sa.bnd_maxch), dim3(kBndChunk), 0, s, *atm, sa, gt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid(atm->n_atm, (sa.npt_max + 63) / 64, (sa.nb_max + sa.chunk_bins - 1) / sa.chunk_bins);
    hipLaunchKernelGGL(planck_kernel, grid, dim3(1024), 0, s, *atm, T_pt, sa.B, sa.chunk, sa.total_pt,
                       (int)sa.iso_grid, (int)sa.chunk_bins);
    return hipGetLastError();
}

// ------------------------------------------------------ bolometric sums
// Stage 1: workgroup = (atmosphere, 64-point tile, chunk of chunk_bins bins);
// 1024 threads = 64 points x 16 groups of chunk_bins/16 bins.  Each thread
// combines the sweep's per-wave Gauss partials of a bin (fixed order) -- sums
// of deviations G = F - 2 pi eps B -- and accumulates dlambda times the up,
// down and net (up - down, where B cancels) deviations in Neumaier sums; the
// group sums are combined in order, the up and down ones plus 2 pi eps times
// the Gauss-weight sum times the chunk's width-weighted Planck sum (from the
// Planck kernel), and stored per (chunk, quantity, point) (so both stages
// access them coalesced).  Only when F_up_bin / F_dn_bin are asked for does
// a thread read B, to write F = 2 pi eps B sum(w) + G per bin.  Stage 2 sums
// a point's chunks in order.

__device__ inline double combine_partials(const void* part, int64_t base, int wpb, int npt, bool mixed) {
    if (!mixed) {
        const double* p = static_cast<const double*>(part) + base;
        double s = 0.0;
        for (int j = 0; j < wpb; ++j) s += p[(int64_t)j * npt];
        return s;
    }
    const float* p = static_cast<const float*>(part) + base;
    double acc = 0.0;
    for (int j = 0; j < wpb; ++j) acc += (double)p[(int64_t)j * npt];
    return acc;
}

// chunk sums: [n_chunk][kBolQ][total_pt]
__device__ inline int64_t chunk_at(const BolArgs& A, int ch, int v, int64_t gpt) {
    return ((int64_t)ch * kBolQ + v) * A.total_pt + gpt;
}

__global__ void __launch_bounds__(1024) bin_sum_kernel(const BolArgs A) {
    __shared__ double red[16][64][6];
    const int a = blockIdx.x;
    const int tile = blockIdx.y, ch = blockIdx.z;
    const int pl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int n = A.atm.n_layer[a];
    const int npt = 2 * n + 1;
    const int nb = (int)(A.atm.bin_off[a + 1] - A.atm.bin_off[a]);
    const int cb = A.chunk_bins;
    if (tile * 64 >= npt || ch * cb >= nb || frozen(A.atm.status, a)) return;  // uniform
    const int wpb = class_wpb(A, n);
    const int p = tile * 64 + pl;
    const int per = cb / 16;
    const int l0 = ch * cb + q * per;
    nacc au = {0.0, 0.0}, ad = {0.0, 0.0}, an = {0.0, 0.0};
    if (p < npt) {
        const double* dl = A.atm.dlambda + A.atm.bin_off[a];
        const int64_t pb = A.atm.pb_off[a];
        const bool per_bin = A.F_up_bin || A.F_dn_bin;  // uniform
#pragma unroll 4
        for (int i = 0; i < per; ++i) {
            const int l = l0 + i;
            if (l < nb) {
                const int64_t base = pb * A.wpb_stride + ((int64_t)l * A.wpb_stride) * npt + p;
                const double gu = combine_partials(A.part_up, base, wpb, npt, A.mixed);
                const double gd = combine_partials(A.part_dn, base, wpb, npt, A.mixed);
                if (per_bin) {
                    const int64_t o = pb + (int64_t)l * npt + p;
                    const double bw = A.tw * A.B[o];
                    if (A.F_up_bin) A.F_up_bin[o] = bw + gu;
                    if (A.F_dn_bin) A.F_dn_bin[o] = bw + gd;
                }
                nadd(au, dl[l] * gu);
                nadd(ad, dl[l] * gd);
                nadd(an, dl[l] * (gu - gd));
            }
        }
    }
    red[q][pl][0] = au.s;
    red[q][pl][1] = au.c;
    red[q][pl][2] = ad.s;
    red[q][pl][3] = ad.c;
    red[q][pl][4] = an.s;
    red[q][pl][5] = an.c;
    __syncthreads();
    if (q < 3 && p < npt) {  // wave v combines quantity v
        const int v = q;
        const int64_t gpt = A.atm.pt_off[a] + p;
        nacc t = {0.0, 0.0};
        double cc = 0.0;
        for (int k = 0; k < 16; ++k) {
            nadd(t, red[k][pl][2 * v]);
            cc += red[k][pl][2 * v + 1];
        }
        if (v < 2) {  // up and down: the isothermal flux's share of this chunk
            nadd(t, A.tw * A.chunk[chunk_at(A, ch, 6, gpt)]);
            cc += A.tw * A.chunk[chunk_at(A, ch, 7, gpt)];
        }
        A.chunk[chunk_at(A, ch, 2 * v, gpt)] = t.s;
        A.chunk[chunk_at(A, ch, 2 * v + 1, gpt)] = t.c + cc;
    }
}

// Stage 2 workgroup: 64 points x 16 groups; group q sums chunks q, q+16, ...
// in order, then the 16 group sums are combined in order.
__global__ void __launch_bounds__(1024) bol_final_kernel(const BolArgs A) {
    __shared__ double red[16][64][6];
    const int a = blockIdx.x, tile = blockIdx.y;
    const int pl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int npt = 2 * A.atm.n_layer[a] + 1;
    if (tile * 64 >= npt || frozen(A.atm.status, a)) return;
    const int p = tile * 64 + pl;
    const int nb = (int)(A.atm.bin_off[a + 1] - A.atm.bin_off[a]);
    const int nch = (nb + A.chunk_bins - 1) / A.chunk_bins;
    nacc t[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    double e[3] = {0.0, 0.0, 0.0};
    const int64_t gpt = A.atm.pt_off[a] + p;
    if (p < npt) {
        // U chunks' loads in flight at a time, added in chunk order
        constexpr int U = 3;
        for (int k0 = q; k0 < nch; k0 += 16 * U) {
            double c[U][6];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = k0 + 16 * u;
#pragma unroll
                for (int v = 0; v < 6; ++v) c[u][v] = (k < nch) ? A.chunk[chunk_at(A, k, v, gpt)] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (k0 + 16 * u < nch) {
#pragma unroll
                    for (int v = 0; v < 3; ++v) {
                        nadd(t[v], c[u][2 * v]);
                        e[v] += c[u][2 * v + 1];
                    }
                }
            }
        }
    }
    for (int v = 0; v < 3; ++v) {
        red[q][pl][2 * v] = t[v].s;
        red[q][pl][2 * v + 1] = t[v].c + e[v];
    }
    __syncthreads();
    if (q < 3 && p < npt) {  // wave v combines quantity v: up, down, and net summed from the deviations
        const int v = q;
        nacc sacc = {0.0, 0.0};
        double ee = 0.0;
        for (int k = 0; k < 16; ++k) {
            nadd(sacc, red[k][pl][2 * v]);
            ee += red[k][pl][2 * v + 1];
        }
        A.F_bol[3 * gpt + v] = sacc.s + (sacc.c + ee);
    }
}

hipError_t launch_bolometric(const BolArgs& a, int npt_max, int nb_max, int64_t /*total_pt*/, hipStream_t s) {
    dim3 grid(a.atm.n_atm, (npt_max + 63) / 64, (nb_max + a.chunk_bins - 1) / a.chunk_bins);
    hipLaunchKernelGGL(bin_sum_kernel, grid, dim3(1024), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bol_final_kernel, dim3(a.atm.n_atm, (npt_max + 63) / 64), dim3(1024), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------- RE update
// One workgroup per atmosphere; threads over layers.  Always FP64.  The
// points' log P are formed once in LDS (shared by the step sizes and the
// re-interpolation); the convergence reduction is a wave reduction plus one
// LDS step.
constexpr int kRadeqThreads = 256;
__global__ void __launch_bounds__(kRadeqThreads) radeq_kernel(helios_atm atm, const double* __restrict__ F_bol,
                                                              double* __restrict__ T_c, double* __restrict__ T_pt,
                                                              double* __restrict__ m, int32_t* __restrict__ hist,
                                                              int32_t* __restrict__ iter, helios_re_opts o,
                                                              int32_t* __restrict__ status,
                                                              double* __restrict__ resid) {
    __shared__ double s_lp[2 * HELIOS_MAX_LAYERS + 1];
    __shared__ double s_red[kRadeqThreads / 64];
    __shared__ int s_bad[kRadeqThreads / 64];
    const int a = blockIdx.x;
    const int n = atm.n_layer[a];
    const int npt = 2 * n + 1;
    // frozen (uniform per workgroup); a bad grid stays flagged
    if (status[a] == HELIOS_ATM_CONVERGED || status[a] == HELIOS_ATM_BADGRID) return;
    const double* F = F_bol + 3 * atm.pt_off[a];
    const double* P = atm.P_pt + atm.pt_off[a];
    double* Tc = T_c + atm.lay_off[a];
    double* ma = m + atm.lay_off[a];
    int32_t* ha = hist + atm.lay_off[a];
    const double sig = sigma_sb();
    const double ti2 = atm.T_int[a] * atm.T_int[a];
    for (int p = threadIdx.x; p < npt; p += blockDim.x) s_lp[p] = log(P[p]);
    __syncthreads();
    // the grid (Sec. 2.2.1): pressures positive, finite and strictly decreasing upward
    int badgrid = 0;
    for (int p = threadIdx.x; p < npt; p += blockDim.x)
        if (!isfinite(s_lp[p]) || (p > 0 && !(s_lp[p] < s_lp[p - 1]))) badgrid = 1;
    // convergence measure (eq:condition), on the fluxes handed in
    double worst = 0.0;
    int nonfinite = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double dF = F[3 * (2 * i + 2) + 2] - F[3 * (2 * i) + 2];
        double T = Tc[i];
        if (!isfinite(dF) || !isfinite(T)) nonfinite = 1;
        double t2 = T * T;
        double norm = (o.norm == HELIOS_NORM_SIGMA_TINT4) ? sig * ti2 * ti2 : sig * t2 * t2;
        double r = fabs(dF) / norm;
        worst = fmax(worst, r);
    }
    for (int off = 32; off > 0; off >>= 1) {
        worst = fmax(worst, __shfl_xor(worst, off, 64));
        nonfinite |= __shfl_xor(nonfinite, off, 64);
        badgrid |= __shfl_xor(badgrid, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        s_red[threadIdx.x >> 6] = worst;
        s_bad[threadIdx.x >> 6] = nonfinite | (badgrid << 1);
    }
    __syncthreads();
    worst = 0.0;
    nonfinite = 0;
    badgrid = 0;
    for (int w = 0; w < kRadeqThreads / 64; ++w) {
        worst = fmax(worst, s_red[w]);
        nonfinite |= s_bad[w] & 1;
        badgrid |= s_bad[w] >> 1;
    }
    if (badgrid) {
        if (threadIdx.x == 0) {
            status[a] = HELIOS_ATM_BADGRID;
            if (resid) resid[a] = __longlong_as_double(0x7ff8000000000000LL);
        }
        return;
    }
    if (threadIdx.x == 0 && resid) resid[a] = nonfinite ? __longlong_as_double(0x7ff8000000000000LL) : worst;
    if (nonfinite) {
        if (threadIdx.x == 0) status[a] = HELIOS_ATM_NUMERIC;
        return;
    }
    if (worst < o.tol) {
        if (threadIdx.x == 0) status[a] = HELIOS_ATM_CONVERGED;
        return;
    }
    if (threadIdx.x == 0) {
        status[a] = HELIOS_ATM_RUNNING;
        if (iter) iter[a] += 1;
    }
    const uint32_t mask = (1u << o.window) - 1u;
    // the alternating patterns ...0101 and ...1010 within the window
    uint32_t alt = 0;
    for (int k = 0; k < o.window; k += 2) alt |= 1u << k;
    const uint32_t alt1 = alt & mask, alt2 = (~alt) & mask;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double dF = F[3 * (2 * i + 2) + 2] - F[3 * (2 * i) + 2];
        double T = Tc[i];
        if (o.deadband) {  // a layer within the tolerance keeps T, m and its history
            double t2 = T * T;
            double norm = (o.norm == HELIOS_NORM_SIGMA_TINT4) ? sig * ti2 * ti2 : sig * t2 * t2;
            if (fabs(dF) / norm < o.tol) continue;
        }
        double dT = 0.0;
        if (dF != 0.0) {
            double lnR = s_lp[2 * i] - s_lp[2 * i + 2];
            double mag = pow(fabs(dF), 1.0 - o.fpre_p) * o.fpre_c * ma[i] / (sig * T * T * T * lnR);
            dT = (dF > 0.0) ? -mag : mag;
        }
        uint32_t h = (uint32_t)ha[i];
        uint32_t bits = h & 0xFFFFu, cnt = h >> 16;
        uint32_t sg = (dT > 0.0) ? 1u : (dT < 0.0) ? 0u : (cnt > 0 ? (bits & 1u) : 1u);
        bits = ((bits << 1) | sg) & mask;
        if (cnt < (uint32_t)o.window) cnt += 1;
        if (cnt >= (uint32_t)o.window) {
            if (bits == 0u || bits == mask) ma[i] *= o.grow;
            else if (o.osc_any || bits == alt1 || bits == alt2) ma[i] *= o.shrink;
        }
        ha[i] = (int32_t)((cnt << 16) | bits);
        double Tn = T + dT;
        Tc[i] = (Tn > o.T_floor) ? Tn : o.T_floor;
    }
    __syncthreads();
    // re-interpolate the point temperatures of this atmosphere (linear in log P)
    double* Tp = T_pt + atm.pt_off[a];
    for (int p = threadIdx.x; p < npt; p += blockDim.x) {
        const int i = p >> 1;
        double T;
        if (p & 1) T = Tc[i];
        else if (i == 0) T = Tc[0];
        else if (i == n) T = Tc[n - 1];
        else {
            const double f = (s_lp[p] - s_lp[p - 1]) / (s_lp[p + 1] - s_lp[p - 1]);
            T = Tc[i - 1] + f * (Tc[i] - Tc[i - 1]);
        }
        Tp[p] = T;
    }
}

hipError_t launch_radeq(const helios_atm* atm, const double* F_bol, double* T_c, double* T_pt,
                        const helios_re_state* st, const helios_re_opts& o, int32_t* status,
                        double* resid, int /*n_max*/, hipStream_t s) {
    hipLaunchKernelGGL(radeq_kernel, dim3(atm->n_atm), dim3(kRadeqThreads), 0, s, *atm, F_bol, T_c, T_pt, st->m,
                       st->hist, st->iter, o, status, resid);
    return hipGetLastError();
}

}  // namespace helios
