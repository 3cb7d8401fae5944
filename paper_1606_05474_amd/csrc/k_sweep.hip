// k_sweep.hip -- the two-stream flux solve of one temperature iteration
// (Sec. 2.1.3, 2.2.2, 2.2.3, 2.3), fused: sublayer coefficients, 1 + n_scat
// scattering passes, and the Gauss sum over g.
//
// Mapping.  One workgroup owns one wavelength bin of one atmosphere: n_g
// columns (one per Gauss point) of L lanes each.  Lane `seg` of a column owns
// K consecutive sublayers [seg*K, seg*K + K) and the K points at their lower
// ends.  Its sublayer coefficients and its upward fluxes stay in VGPRs for
// all passes, so a call reads kappa, B, w0/g0 and the warm start once and
// writes the fluxes once.
//
// Each sweep is an affine recurrence along the column:
//   down:  F_dn(s)   = a_s F_dn(s+1) + (c_s F_up(s) + S_dn,s)
//   up:    F_up(s+1) = a_s F_up(s)   + (c_s F_dn(s+1) + S_up,s)
// so a lane composes the affine maps of its K sublayers, the L lanes of a
// column combine their maps with a log2(L)-step shuffle scan (suffix scan
// from the TOA for the down sweep, prefix scan from the BOA for the up
// sweep), and each lane then replays its own K steps from its entry value.
// This is exactly the sequential Gauss-Seidel sweep of the paper, evaluated
// in a different association order.
//
// Sublayer coefficients.  With r = sqrt((1-w0)/(1-w0 g0)), zeta_pm = (1 +- r)/2,
// T = exp(-D sqrt((1-w0 g0)(1-w0)) dtau) and om = 1 - T (from expm1), the
// coefficient expressions of eq:cap simplify exactly to
//   alpha = -(zp - zm T)(zp + zm T),  alpha + beta = -r (zp + zm T^2),
//   xi = -r T,  beta + ups = om (zp + zm T),  (beta - ups)/alpha = r om / (zp + zm T)
// which are free of cancellation for thin layers.  Then
//   a = xi/alpha = r T / (zp^2 - zm^2 T^2)
//   c = -beta/alpha = zp zm om (1 + T) / (zp^2 - zm^2 T^2)
//   eq:isoscat (dtau < 1e-4):  S_up = S_dn = 2 pi eps Bbar r om / (zp + zm T)
//   eq:nonisoscat:  S_up = 2 pi eps { r [B_u (zp + zm T^2) - B_d T] / (zp^2 - zm^2 T^2)
//                                     + f B' om / (zp - zm T) }
//                   S_dn = 2 pi eps { r [B_d (zp + zm T^2) - B_u T] / (zp^2 - zm^2 T^2)
//                                     - f B' om / (zp - zm T) }
//   with B' = (B_d - B_u)/dtau and f = eps/(1 - w0 g0): the Planck value of the
//   sublayer's upper end goes with the outgoing upward flux, and B' is the
//   gradient in optical depth measured downward.
//   eq:purescat ((1 - w0) < 1e-6):  q = gamma dtau/(1 + gamma dtau),
//   gamma = D (1 - g0)/2, a = 1 - q, c = q, no source.
#include "helios_internal.hpp"

namespace helios {

template <typename R>
struct Prec;
template <>
struct Prec<double> {
    __device__ static inline void t_om(double x, double& T, double& om) {
        // one transcendental: om accurate for small x, T accurate in absolute terms
        double em = expm1(-x);
        om = -em;
        T = 1.0 + em;
    }
    __device__ static inline double rcp(double v) { return 1.0 / v; }
    __device__ static inline double sqrt_(double v) { return sqrt(v); }
};
template <>
struct Prec<float> {
    __device__ static inline void t_om(float x, float& T, float& om) {
        T = __expf(-x);
        om = -expm1f(-x);
    }
    __device__ static inline float rcp(float v) { return __frcp_rn(v); }
    __device__ static inline float sqrt_(float v) { return sqrtf(v); }
};

// Coefficients {T, a, c, S_up, S_dn} of one sublayer.
template <typename R>
__device__ inline void sub_coeffs(R dtau, R w0, R g0, R D, R Bu, R Bd, R& Tr, R& a, R& c, R& su, R& sd) {
    const R one = (R)1;
    const R eps = one / D;
    const R two_pi_eps = (R)(2.0 * kPi) * eps;
    if (one - w0 < (R)1e-6) {
        const R gd = D * (one - g0) * (R)0.5 * dtau;
        const R q = gd / (one + gd);
        Tr = one;
        a = one - q;
        c = q;
        su = (R)0;
        sd = (R)0;
        return;
    }
    const R omg = one - w0 * g0;
    const R r = Prec<R>::sqrt_((one - w0) / omg);
    const R zp = (R)0.5 * (one + r), zm = (R)0.5 * (one - r);
    const R x = D * Prec<R>::sqrt_(omg * (one - w0)) * dtau;
    R T, om;
    Prec<R>::t_om(x, T, om);
    const R den = zp * zp - zm * zm * T * T;
    const R iden = one / den;
    Tr = T;
    a = r * T * iden;
    c = zp * zm * om * (one + T) * iden;
    if (dtau < (R)1e-4) {
        const R s = two_pi_eps * (R)0.5 * (Bu + Bd) * r * om / (zp + zm * T);
        su = s;
        sd = s;
    } else {
        const R f = eps / omg;
        const R gterm = f * (Bd - Bu) / dtau * om / (zp - zm * T);
        const R e2 = zp + zm * T * T;
        su = two_pi_eps * (r * (Bu * e2 - Bd * T) * iden + gterm);
        sd = two_pi_eps * (r * (Bd * e2 - Bu * T) * iden - gterm);
    }
}

template <typename R>
__device__ inline R shfl_down_w(R v, int d, int width) {
    return __shfl_down(v, (unsigned)d, width);
}
template <typename R>
__device__ inline R shfl_up_w(R v, int d, int width) {
    return __shfl_up(v, (unsigned)d, width);
}

// Partial g-sums of one point: sum over the wave's columns by xor shuffles,
// then the first column of each wave writes its partial to LDS.
template <typename R>
struct GSum;
template <>
struct GSum<double> {
    using slot = double;
    __device__ static inline void wave_reduce_store(double v, int L, bool writer, slot* dst) {
        for (int d = L; d < 64; d <<= 1) v += __shfl_xor(v, d, 64);
        if (writer) *dst = v;
    }
    __device__ static inline double combine(const slot* src, int stride, int nw) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += src[w * stride];
        return s;
    }
};
template <>
struct GSum<float> {
    using slot = fpair;
    __device__ static inline void wave_reduce_store(float v, int L, bool writer, slot* dst) {
        fpair p = {v, 0.0f};
        for (int d = L; d < 64; d <<= 1) {
            fpair o = {__shfl_xor(p.s, d, 64), __shfl_xor(p.c, d, 64)};
            p = two_sum_add(p, o);
        }
        if (writer) *dst = p;
    }
    __device__ static inline double combine(const slot* src, int stride, int nw) {
        fpair acc = {0.0f, 0.0f};
        for (int w = 0; w < nw; ++w) acc = two_sum_add(acc, src[w * stride]);
        return (double)acc.s + (double)acc.c;
    }
};

template <int K, typename R, int MAXT>
__global__ void __launch_bounds__(MAXT) sweep_kernel(const SweepArgs A) {
    using GS = GSum<R>;
    using slot = typename GS::slot;
    extern __shared__ unsigned char smem_raw[];
    slot* part = reinterpret_cast<slot*>(smem_raw);  // [nwaves][npt_max]

    const int t = threadIdx.x;
    const int L = A.L;
    const int seg = t & (L - 1);
    const int col = t >> A.log2L;
    const int wave = t >> 6;
    const int nwaves = blockDim.x >> 6;
    const bool writer = (t & 63) < L;  // first column of its wave
    const R* __restrict__ kap_all = static_cast<const R*>(A.kappa);
    const R* __restrict__ B_all = static_cast<const R*>(A.B);
    R* __restrict__ Fu_all = static_cast<R*>(A.F_up_g);
    R* __restrict__ Fd_all = static_cast<R*>(A.F_dn_g);

    for (int64_t gb = A.gb_begin + blockIdx.x; gb < A.gb_end; gb += gridDim.x) {
        const int at = find_atm(A.bin_off, A.n_atm, gb);
        const int l = (int)(gb - A.bin_off[at]);
        const int n = A.n_layer[at];
        const int nsub = 2 * n, npt = nsub + 1;
        const int nact = (nsub + K - 1) / K;
        const bool colok = col < A.n_g;
        const int lo = seg * K;
        // points owned by this segment (its sublayers' lower ends), whatever the column
        const int scnt = (seg < nact) ? min(K, nsub - lo) : 0;
        const bool top_seg = (seg == nact - 1);  // also owns the TOA point
        const int cnt = colok ? scnt : 0;
        const int64_t cell = A.cell_off[at] + ((int64_t)l * A.n_g + (colok ? col : 0)) * npt;
        const int64_t pb = A.pb_off[at] + (int64_t)l * npt;
        const int64_t lb = A.lb_off[at] + (int64_t)l * n;
        const double* __restrict__ P = A.P_pt + A.pt_off[at];
        const double grav = A.grav[at];
        const R D = (R)A.D;
        const R Ftop = (R)A.F_top[A.bin_off[at] + l];
        const R Fint = (R)A.F_int[A.bin_off[at] + l];
        const R wg = colok ? (R)A.gw[col] : (R)0;

        // ---- load and build the sublayer coefficients (once per call)
        R ca[K], cc[K], su[K], sd[K], fu[K], bu[K];
        {
            R kp = (R)0, Bp = (R)0;
            double Pp = 1.0;
            if (cnt > 0) {
                kp = kap_all[cell + lo];
                Bp = B_all[pb + lo];
                Pp = P[lo];
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                ca[k] = (R)1;
                cc[k] = (R)0;
                su[k] = (R)0;
                sd[k] = (R)0;
                fu[k] = (R)0;
                bu[k] = (R)0;
                if (k < cnt) {
                    const int s = lo + k;
                    const R kn = kap_all[cell + s + 1];
                    const R Bn = B_all[pb + s + 1];
                    const double Pn = P[s + 1];
                    const R dtau = (R)0.5 * (kp + kn) * (R)((Pp - Pn) / grav);
                    const R w0 = (R)A.w0[lb + (s >> 1)];
                    const R g0 = (R)A.g0[lb + (s >> 1)];
                    R Tr;
                    sub_coeffs<R>(dtau, w0, g0, D, Bn, Bp, Tr, ca[k], cc[k], su[k], sd[k]);
                    fu[k] = Fu_all[cell + s];
                    kp = kn;
                    Bp = Bn;
                    Pp = Pn;
                }
            }
        }

        R ftoa = (R)0;
        const int base = (t & 63) & ~(L - 1);  // lane of seg 0 in this column
        for (int pass = 0; pass <= A.n_scat; ++pass) {
            const bool last = (pass == A.n_scat);
            // ---------------- downward sweep: compose my segment (top -> bottom)
            R MA = (R)1, MB = (R)0;
#pragma unroll
            for (int k = K - 1; k >= 0; --k) {
                const R b = cc[k] * fu[k] + sd[k];
                MB = ca[k] * MB + b;
                MA = ca[k] * MA;
            }
            for (int d = 1; d < L; d <<= 1) {  // suffix scan towards the BOA
                const R A2 = shfl_down_w(MA, d, L), B2 = shfl_down_w(MB, d, L);
                if (seg + d < L) {
                    MB = MA * B2 + MB;
                    MA = MA * A2;
                }
            }
            const R xbot = MA * Ftop + MB;
            R xtop = shfl_down_w(xbot, 1, L);
            if (seg == L - 1) xtop = Ftop;
            // replay: downward fluxes, and the up-sweep inputs b_up
            R x = xtop;
            if (last) {
                // F_dn at the TOA point is the boundary value; the top segment owns it
                GS::wave_reduce_store((top_seg && colok) ? wg * Ftop : (R)0, L, writer && top_seg,
                                      &part[wave * A.npt_max + nsub]);
                if (top_seg && colok && Fd_all) Fd_all[cell + nsub] = Ftop;
            }
#pragma unroll
            for (int k = K - 1; k >= 0; --k) {
                bu[k] = cc[k] * x + su[k];
                x = ca[k] * x + (cc[k] * fu[k] + sd[k]);
                if (last) {
                    GS::wave_reduce_store((k < cnt) ? wg * x : (R)0, L, writer && k < scnt,
                                          &part[wave * A.npt_max + min(lo + k, nsub)]);
                    if (k < cnt && Fd_all) Fd_all[cell + lo + k] = x;
                }
            }
            if (last) {
                __syncthreads();
                double* outb = A.F_dn_bin + pb;
                for (int p = t; p < npt; p += blockDim.x) outb[p] = GS::combine(part + p, A.npt_max, nwaves);
                __syncthreads();
            }
            // ---------------- BOA: F_up(0) = F_dn(0) + F_int
            const R y0 = __shfl(x, base, 64) + Fint;
            // ---------------- upward sweep: compose (bottom -> top)
            MA = (R)1;
            MB = (R)0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                MB = ca[k] * MB + bu[k];
                MA = ca[k] * MA;
            }
            for (int d = 1; d < L; d <<= 1) {  // prefix scan towards the TOA
                const R A2 = shfl_up_w(MA, d, L), B2 = shfl_up_w(MB, d, L);
                if (seg >= d) {
                    MB = MA * B2 + MB;
                    MA = MA * A2;
                }
            }
            const R ytop = MA * y0 + MB;
            R ybot = shfl_up_w(ytop, 1, L);
            if (seg == 0) ybot = y0;
            R y = ybot;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                fu[k] = y;
                y = ca[k] * y + bu[k];
            }
            ftoa = y;
        }

        // ---- outputs: upward fluxes (warm start for the next call) and their g-sum
#pragma unroll
        for (int k = 0; k < K; ++k) {
            GS::wave_reduce_store((k < cnt) ? wg * fu[k] : (R)0, L, writer && k < scnt,
                                  &part[wave * A.npt_max + min(lo + k, nsub)]);
            if (k < cnt) Fu_all[cell + lo + k] = fu[k];
        }
        GS::wave_reduce_store((top_seg && colok) ? wg * ftoa : (R)0, L, writer && top_seg,
                              &part[wave * A.npt_max + nsub]);
        if (top_seg && colok) Fu_all[cell + nsub] = ftoa;
        __syncthreads();
        double* outb = A.F_up_bin + pb;
        for (int p = t; p < npt; p += blockDim.x) outb[p] = GS::combine(part + p, A.npt_max, nwaves);
        __syncthreads();
    }
}

template <int K, int MAXT>
static hipError_t launch_k(const SweepArgs& a, bool mixed, int block, int grid, hipStream_t s) {
    const int nwaves = block / 64;
    if (mixed) {
        size_t sh = (size_t)nwaves * a.npt_max * sizeof(fpair);
        hipLaunchKernelGGL((sweep_kernel<K, float, MAXT>), dim3(grid), dim3(block), sh, s, a);
    } else {
        size_t sh = (size_t)nwaves * a.npt_max * sizeof(double);
        hipLaunchKernelGGL((sweep_kernel<K, double, MAXT>), dim3(grid), dim3(block), sh, s, a);
    }
    return hipGetLastError();
}

template <int K>
static hipError_t launch_kb(const SweepArgs& a, bool mixed, int block, int grid, hipStream_t s) {
    if (block <= 320) return launch_k<K, 320>(a, mixed, block, grid, s);
    if (block <= 640) return launch_k<K, 640>(a, mixed, block, grid, s);
    return hipErrorInvalidValue;
}

hipError_t launch_sweep(const SweepArgs& a, int K, bool mixed, int block, int grid, hipStream_t s) {
    switch (K) {
        case 4: return launch_kb<4>(a, mixed, block, grid, s);
        case 7: return launch_kb<7>(a, mixed, block, grid, s);
        case 13: return launch_kb<13>(a, mixed, block, grid, s);
        case 25: return launch_kb<25>(a, mixed, block, grid, s);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------- coefficient inspection
// One thread per (bin, g, sublayer): the same coefficient routine the sweep
// uses, written out as {T, a, c, S_up, S_dn}.
template <typename R>
__global__ void transmission_kernel(helios_atm atm, const R* __restrict__ kap, const double* __restrict__ T_pt,
                                    const double* __restrict__ w0, const double* __restrict__ g0, double D,
                                    double* __restrict__ out, int64_t total_sub) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total_sub) return;
    // sub offsets: cell_off[a] - n_g * bin_off[a] counts nb*ng*2n per atmosphere
    int lo = 0, hi = atm.n_atm;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (atm.cell_off[mid] - (int64_t)atm.n_g * atm.bin_off[mid] <= idx) lo = mid; else hi = mid;
    }
    const int a = lo;
    const int64_t rel = idx - (atm.cell_off[a] - (int64_t)atm.n_g * atm.bin_off[a]);
    const int n = atm.n_layer[a], nsub = 2 * n, npt = nsub + 1;
    const int64_t colx = rel / nsub;
    const int s = (int)(rel - colx * nsub);
    const int l = (int)(colx / atm.n_g);
    const int64_t cell = atm.cell_off[a] + colx * npt;
    const double* P = atm.P_pt + atm.pt_off[a];
    const double lam = atm.lambda_c[atm.bin_off[a] + l];
    const R Bd = (R)planck_d(lam, T_pt[atm.pt_off[a] + s]);
    const R Bu = (R)planck_d(lam, T_pt[atm.pt_off[a] + s + 1]);
    const R dtau = (R)0.5 * (kap[cell + s] + kap[cell + s + 1]) * (R)((P[s] - P[s + 1]) / atm.grav[a]);
    const int64_t lb = atm.lb_off[a] + (int64_t)l * n + (s >> 1);
    R Tr, ca, cc, su, sd;
    sub_coeffs<R>(dtau, (R)w0[lb], (R)g0[lb], (R)D, Bu, Bd, Tr, ca, cc, su, sd);
    double* o = out + 5 * idx;
    o[0] = (double)Tr;
    o[1] = (double)ca;
    o[2] = (double)cc;
    o[3] = (double)su;
    o[4] = (double)sd;
}

hipError_t launch_transmission(const helios_atm* atm, const void* kappa, const double* T_pt,
                               const double* w0, const double* g0, double D, double* out,
                               int64_t total_sub, bool mixed, hipStream_t s) {
    int block = 256;
    int64_t grid = (total_sub + block - 1) / block;
    if (mixed)
        hipLaunchKernelGGL(transmission_kernel<float>, dim3((unsigned)grid), dim3(block), 0, s, *atm,
                           (const float*)kappa, T_pt, w0, g0, D, out, total_sub);
    else
        hipLaunchKernelGGL(transmission_kernel<double>, dim3((unsigned)grid), dim3(block), 0, s, *atm,
                           (const double*)kappa, T_pt, w0, g0, D, out, total_sub);
    return hipGetLastError();
}

}  // namespace helios
