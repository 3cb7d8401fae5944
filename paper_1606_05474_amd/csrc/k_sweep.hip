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
//
// Deviation form.  An isothermal column has F_up = F_dn = 2 pi eps B at every
// point (for any coefficients), so the sweep carries G = F - 2 pi eps B(point)
// instead of F.  Substituting leaves a and c unchanged and turns both sources
// into one term linear in the Planck difference dB = B_lower - B_upper across
// the sublayer (the part proportional to B cancels exactly):
//   up:   G_up(upper)   = a G_up(lower) + c G_dn(upper) + sig
//   down: G_dn(lower)   = a G_dn(upper) + c G_up(lower) - sig
//   non-isothermal  sig = 2 pi eps f dB om / (dtau (zp - zm T))
//   isothermal      sig = pi eps (1 + a - c) dB
//   pure scattering sig = 2 pi eps a dB
// with the boundary values G_dn(TOA) = F_top - 2 pi eps B(TOA) and
// G_up(BOA) = G_dn(BOA) + F_int.  Deep in the atmosphere F_up and F_dn are both
// close to pi B and their difference (the net flux) is small; in this form
// the rounding of each stream is relative to its deviation from pi B rather
// than to pi B itself, which is what lets FP32 sweeps resolve net fluxes at
// depth.  Fluxes are recovered as F = G + 2 pi eps B in FP64 by the bin sum.
#include "helios_internal.hpp"

namespace helios {

template <typename R>
struct Prec;
template <>
struct Prec<double> {
    // T = exp(-x) and om = 1 - T from one transcendental: om is accurate for
    // thin layers, T accurate in absolute terms
    __device__ static inline void t_om(double x, double& T, double& om) {
        double em = expm1(-x);
        om = -em;
        T = 1.0 + em;
    }
    // reciprocal: hardware estimate refined by two Newton steps (the
    // arguments here are well scaled: no denormals, no overflow)
    __device__ static inline double rcp(double v) {
        double r = __builtin_amdgcn_rcp(v);
        double e = fma(-v, r, 1.0);
        r = fma(r, e, r);
        e = fma(-v, r, 1.0);
        return fma(r, e, r);
    }
    __device__ static inline double sqrt_(double v) { return sqrt(v); }
};
template <>
struct Prec<float> {
    // om = 1 - exp(-x): degree-6 Taylor polynomial below x = 0.25 (truncation
    // below one float ulp), 1 - exp(-x) above (no cancellation there)
    __device__ static inline void t_om(float x, float& T, float& om) {
        T = __expf(-x);
        float p = x * (-1.0f / 720.0f) + (1.0f / 120.0f);
        p = x * p - (1.0f / 24.0f);
        p = x * p + (1.0f / 6.0f);
        p = x * p - 0.5f;
        p = x * p + 1.0f;
        om = (x < 0.25f) ? x * p : 1.0f - T;
    }
    __device__ static inline float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
    // hardware square root (about 1 ulp), enough for the mixed path
    __device__ static inline float sqrt_(float v) { return __builtin_amdgcn_sqrtf(v); }
};

// Per-layer quantities shared by a layer's two sublayers and all g.
template <typename R>
struct LayerQ {
    R r, zp, zm, zpzm, kx, f, tpr, purescat_gd;  // tpr = 2 pi eps r; purescat_gd = D (1 - g0)/2
    bool purescat;
};

template <typename R>
__device__ inline LayerQ<R> layer_q(R w0, R g0, R D, R inv_D, R two_pi_eps) {
    LayerQ<R> q;
    const R one = (R)1;
    q.purescat = (one - w0) < (R)1e-6;
    const R omg = one - w0 * g0;
    const R iomg = Prec<R>::rcp(omg);
    q.r = Prec<R>::sqrt_((one - w0) * iomg);
    q.zp = (R)0.5 * (one + q.r);
    q.zm = (R)0.5 * (one - q.r);
    q.zpzm = q.zp * q.zm;
    q.kx = D * q.r * omg;  // D sqrt((1 - w0 g0)(1 - w0))
    q.f = iomg * inv_D;  // eps / (1 - w0 g0)
    q.tpr = two_pi_eps * q.r;
    q.purescat_gd = D * (one - g0) * (R)0.5;
    return q;
}

// Coefficients {T, a, c, S_up, S_dn} of one sublayer from its layer's
// quantities, optical depth and end Planck values.  den = zp^2 - zm^2 T^2
// factors as (zp - zm T)(zp + zm T), so one reciprocal serves all three
// denominators.  The pure-scattering override is evaluated only when some
// lane of the wave needs it (a wave-uniform branch).
template <typename R>
__device__ inline void sub_coeffs_q(const LayerQ<R>& q, R dtau, R two_pi_eps, R Bu, R Bd, R& Tr, R& a, R& c,
                                    R& su, R& sd) {
    const R one = (R)1;
    R T, om;
    Prec<R>::t_om(q.kx * dtau, T, om);
    const R u = q.zp - q.zm * T, v = q.zp + q.zm * T;
    const R iden = Prec<R>::rcp(u * v);
    const R omi = om * iden;
    a = q.r * T * iden;
    c = q.zpzm * (one + T) * omi;
    const R s_iso = (R)0.5 * q.tpr * (Bu + Bd) * u * omi;
    const R gterm = q.f * (Bd - Bu) * Prec<R>::rcp(dtau) * v * omi;
    const R e2 = q.zp + q.zm * T * T;
    const R tu = q.tpr * iden;
    R su_ = tu * (Bu * e2 - Bd * T) + two_pi_eps * gterm;
    R sd_ = tu * (Bd * e2 - Bu * T) - two_pi_eps * gterm;
    const bool iso = dtau < (R)1e-4;
    su = iso ? s_iso : su_;
    sd = iso ? s_iso : sd_;
    Tr = T;
    if (__any(q.purescat)) {  // eq:purescat
        const R gd = q.purescat_gd * dtau;
        const R qq = gd * Prec<R>::rcp(one + gd);
        Tr = q.purescat ? one : Tr;
        a = q.purescat ? one - qq : a;
        c = q.purescat ? qq : c;
        su = q.purescat ? (R)0 : su;
        sd = q.purescat ? (R)0 : sd;
    }
}

// Coefficients of one sublayer from (dtau, w0, g0): the inspection kernel's
// entry to the same arithmetic.
template <typename R>
__device__ inline void sub_coeffs(R dtau, R w0, R g0, R D, R Bu, R Bd, R& Tr, R& a, R& c, R& su, R& sd) {
    const R inv_D = (R)1 / D, tpe = (R)(2.0 * kPi) * inv_D;
    LayerQ<R> q = layer_q<R>(w0, g0, D, inv_D, tpe);
    sub_coeffs_q<R>(q, dtau, tpe, Bu, Bd, Tr, a, c, su, sd);
}

// The sweep's coefficients of one sublayer in the deviation form: a, c and
// the source sig for the Planck difference dB = B_lower - B_upper.  One
// reciprocal of (zp - zm T)(zp + zm T) serves a and c; om / (zp - zm T) is
// om (zp + zm T) times it.
template <typename R>
__device__ inline void sub_coeffs_g(const LayerQ<R>& q, R dtau, R two_pi_eps, R dB, R& a, R& c, R& sig) {
    const R one = (R)1;
    R T, om;
    Prec<R>::t_om(q.kx * dtau, T, om);
    const R u = q.zp - q.zm * T, v = q.zp + q.zm * T;
    const R iden = Prec<R>::rcp(u * v);
    const R omi = om * iden;
    a = q.r * T * iden;
    c = q.zpzm * (one + T) * omi;
    sig = two_pi_eps * q.f * v * omi * Prec<R>::rcp(dtau) * dB;
    const bool iso = dtau < (R)1e-4;
    if (__any(iso)) sig = iso ? (R)0.5 * two_pi_eps * (one + a - c) * dB : sig;  // may be inf at dtau = 0
    if (__any(q.purescat)) {  // eq:purescat
        const R gd = q.purescat_gd * dtau;
        const R qq = gd * Prec<R>::rcp(one + gd);
        a = q.purescat ? one - qq : a;
        c = q.purescat ? qq : c;
        sig = q.purescat ? two_pi_eps * (one - qq) * dB : sig;
    }
}

// Shifts within a column's group of L lanes.  For L = 16 the group is one
// DPP row, so row_shl/row_shr moves (out-of-row sources read 0) replace LDS
// permutes; wider groups use shuffles (out-of-group sources read the own
// value, which the callers never use).
template <int CTRL>
__device__ inline float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ inline double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// value of lane seg + D of the group (TOA direction)
template <int L, int D, typename R>
__device__ inline R grp_down(R v) {
    if constexpr (L == 16) return dpp_mov<0x100 + D>(v);
    else return __shfl_down(v, (unsigned)D, L);
}
// value of lane seg - D of the group (BOA direction)
template <int L, int D, typename R>
__device__ inline R grp_up(R v) {
    if constexpr (L == 16) return dpp_mov<0x110 + D>(v);
    else return __shfl_up(v, (unsigned)D, L);
}

// One scan step of affine maps whose multipliers are pass-invariant:
// MB <- mult * MB(partner) + MB.
template <int L, int T, typename R>
__device__ inline R scan_down_step(R MB, R mult) {
    return mult * grp_down<L, (1 << T)>(MB) + MB;
}
template <int L, int T, typename R>
__device__ inline R scan_up_step(R MB, R mult) {
    return mult * grp_up<L, (1 << T)>(MB) + MB;
}

// Full scan step pairs (multiplier and offset) for when the multipliers are
// not kept between passes.
template <int L, int D, typename R>
__device__ inline void down_pair(R& MA, R& MB, int seg) {
    const R a2 = grp_down<L, D>(MA), b2 = grp_down<L, D>(MB);
    const bool ok = seg + D < L;
    MB = ok ? MA * b2 + MB : MB;
    MA = ok ? MA * a2 : MA;
}
template <int L, int D, typename R>
__device__ inline void up_pair(R& MA, R& MB, int seg) {
    const R a2 = grp_up<L, D>(MA), b2 = grp_up<L, D>(MB);
    const bool ok = seg >= D;
    MB = ok ? MA * b2 + MB : MB;
    MA = ok ? MA * a2 : MA;
}
template <int L, typename R>
__device__ inline void scan_down_full(R& MA, R& MB, int seg) {
    down_pair<L, 1>(MA, MB, seg);
    down_pair<L, 2>(MA, MB, seg);
    down_pair<L, 4>(MA, MB, seg);
    down_pair<L, 8>(MA, MB, seg);
    if constexpr (L > 16) down_pair<L, 16>(MA, MB, seg);
}
template <int L, typename R>
__device__ inline void scan_up_full(R& MA, R& MB, int seg) {
    up_pair<L, 1>(MA, MB, seg);
    up_pair<L, 2>(MA, MB, seg);
    up_pair<L, 4>(MA, MB, seg);
    up_pair<L, 8>(MA, MB, seg);
    if constexpr (L > 16) up_pair<L, 16>(MA, MB, seg);
}

// Gauss partial sum of one point over the wave's ncols columns staged in
// LDS (column stride npt), in column order; compensated pairs in FP32.
template <typename R>
struct GSum;
template <>
struct GSum<double> {
    using slot = double;
    __device__ static inline slot col_sum(const double* col, int npt, int ncols, const double* w) {
        double acc = 0.0;
        for (int c = 0; c < ncols; ++c) acc += w[c] * col[c * npt];
        return acc;
    }
};
template <>
struct GSum<float> {
    // a wave's columns are at most 4 g points, so its partial is a sum of <= 4
    // products; every later sum (over the bin's waves, then over bins) is in
    // FP64 with compensation
    using slot = float;
    __device__ static inline slot col_sum(const float* col, int npt, int ncols, const float* w) {
        float acc = 0.0f;
        for (int c = 0; c < ncols; ++c) acc += w[c] * col[c * npt];
        return acc;
    }
};

// One workgroup = one wave, which owns one (bin, part) at a time: it stages
// the bin's Planck differences, sublayer column masses, w0 and g0 in LDS once,
// then solves its share of the bin's n_g columns C = 64/L at a time (group j
// covers g in [j*C, j*C + C), contiguous in the [bin][g][point] arrays, staged
// and written back through LDS with coalesced accesses), and accumulates the
// Gauss sums of its groups in LDS in a fixed order.  Large launches give a bin
// one part (one partial per (bin, point)); launches with few bins split a
// bin's groups over several waves to fill the device.  The bin-sum kernel adds
// a bin's partials in order, adds the Planck term and sums over bins.  No
// barrier spans more than the wave.
template <int K, int L, typename R, int OCC>
__global__ void __launch_bounds__(64, OCC) sweep_kernel(const SweepArgs A) {
    using GS = GSum<R>;
    using slot = typename GS::slot;
    constexpr int C = 64 / L;
    static_assert(K % 2 == 0, "segments hold whole layers");
    extern __shared__ unsigned char smem_raw[];
    const int npt_max = A.npt_max;
    R* s_kap = reinterpret_cast<R*>(smem_raw);  // [C][npt]   opacities of the group
    R* s_fu = s_kap + C * npt_max;              // [C][npt]   warm start, later F_dn / F_up of the group
    R* s_dB = s_fu + C * npt_max;               // [npt - 1]  Planck difference across each sublayer
    R* s_dm = s_dB + npt_max;                   // [npt - 1]  sublayer column masses
    R* s_w0 = s_dm + npt_max;                   // [n]
    R* s_g0 = s_w0 + npt_max / 2;               // [n]
    slot* s_pu = reinterpret_cast<slot*>(s_g0 + npt_max / 2 + 1);  // [npt] Gauss sums, up
    slot* s_pd = s_pu + npt_max;                                     // [npt] Gauss sums, down

    const int lane = threadIdx.x;
    const int seg = lane & (L - 1);
    const int cw = lane / L;
    const R* __restrict__ kap_all = static_cast<const R*>(A.kappa);
    const double* __restrict__ B_all = static_cast<const double*>(A.B);
    R* __restrict__ Fu_all = static_cast<R*>(A.F_up_g);
    R* __restrict__ Fd_all = static_cast<R*>(A.F_dn_g);
    slot* __restrict__ part_up = static_cast<slot*>(A.part_up);
    slot* __restrict__ part_dn = static_cast<slot*>(A.part_dn);

    for (int64_t item = A.w_begin + blockIdx.x; item < A.w_end; item += gridDim.x) {
        const int64_t gb = item / A.parts;
        const int part = (int)(item - gb * A.parts);
        // one group per wave: its Gauss sums go straight to the workspace
        // (no LDS accumulators are allocated for such launches)
        const bool direct = (A.parts >= A.wpb);
        const int at = A.bin_atm[gb];
        const int l = (int)(gb - A.bin_off[at]);
        const int n = A.n_layer[at];
        if (n < A.n_lo || n > A.n_hi || frozen(A.status, at)) continue;  // uniform per wave
        const int nsub = 2 * n, npt = nsub + 1;
        const int nact = (nsub + K - 1) / K;
        const int lo = seg * K;
        const int scnt = (seg < nact) ? min(K, nsub - lo) : 0;  // points owned (any column)
        const bool top_seg = (seg == nact - 1);                 // also owns the TOA point
        const int cs = col_stride(n);
        const int64_t pb = A.pb_off[at] + (int64_t)l * npt;
        const int64_t lb = A.lb_off[at] + (int64_t)l * n;
        const double* __restrict__ P = A.P_pt + A.pt_off[at];
        const double igrav = 1.0 / A.grav[at];
        const R D = (R)A.D;
        const R inv_D = (R)(1.0 / A.D);
        const R tpe = (R)(2.0 * kPi / A.D);
        // TOA value of the downward deviation, formed in FP64
        const R Ftop = (R)(A.F_top[A.bin_off[at] + l] - (2.0 * kPi / A.D) * B_all[pb + nsub]);
        const R Fint = (R)A.F_int[A.bin_off[at] + l];

        // ---- the bin's per-sublayer inputs, staged once for all g.  All loads
        // are issued before the first is consumed (compile-time bounds,
        // indices clamped into the bin's own rows).
        {
            constexpr int NCAP = K * L + 1;
            constexpr int PCH = (NCAP + 63) / 64;
            constexpr int LCH = (K * L / 2 + 63) / 64;
            double bv[PCH], pv[PCH], wv[LCH], gv[LCH];
#pragma unroll
            for (int q = 0; q < PCH; ++q) {
                const int i = min(lane + 64 * q, npt - 1);
                bv[q] = B_all[pb + i];
                pv[q] = P[i];
            }
#pragma unroll
            for (int q = 0; q < LCH; ++q) {
                const int i = min(lane + 64 * q, n - 1);
                wv[q] = A.w0[lb + i];
                gv[q] = A.g0[lb + i];
            }
            // sublayer differences from the next point's value: the next lane,
            // or lane 0 of the next chunk for lane 63 (sublayer i < npt - 1
            // never needs a chunk past the last)
#pragma unroll
            for (int q = 0; q < PCH; ++q) {
                double bn = __shfl_down(bv[q], 1u, 64), pn = __shfl_down(pv[q], 1u, 64);
                if (q + 1 < PCH) {
                    const double b0 = __shfl(bv[q + 1 < PCH ? q + 1 : q], 0, 64);
                    const double p0 = __shfl(pv[q + 1 < PCH ? q + 1 : q], 0, 64);
                    bn = (lane == 63) ? b0 : bn;
                    pn = (lane == 63) ? p0 : pn;
                }
                const int i = lane + 64 * q;
                if (i < nsub) {
                    s_dB[i] = (R)(bv[q] - bn);
                    s_dm[i] = (R)((pv[q] - pn) * igrav);
                }
                if (i < npt && !direct) {
                    s_pu[i] = (slot)0;
                    s_pd[i] = (slot)0;
                }
            }
#pragma unroll
            for (int q = 0; q < LCH; ++q) {
                const int i = lane + 64 * q;
                if (i < n) {
                    s_w0[i] = (R)wv[q];
                    s_g0[i] = (R)gv[q];
                }
            }
        }

        const int gpp = (A.wpb + A.parts - 1) / A.parts;  // groups of this wave: [j_lo, j_hi)
        const int j_lo = part * gpp, j_hi = min(A.wpb, j_lo + gpp);
      for (int j = j_lo; j < j_hi; ++j) {  // groups of C columns
        const int g = j * C + cw;
        const int ncols = min(C, A.n_g - j * C);  // columns of this group
        const bool colok = cw < ncols;
        const int cnt = colok ? scnt : 0;
        const int64_t cell0 = A.cell_off[at] + ((int64_t)l * A.n_g + j * C) * cs;  // first column
        R wcol[C];  // Gauss weights of the wave's columns
#pragma unroll
        for (int c = 0; c < C; ++c) wcol[c] = (c < ncols) ? (R)A.gw[j * C + c] : (R)0;

        // ---- stage the group's opacities and warm start in LDS (coalesced,
        // all loads issued before the first is consumed)
        {
            constexpr int NCAP = K * L + 1;
            constexpr int PCH = (NCAP + 63) / 64;
            R kv[C][PCH], fv[C][PCH];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int64_t col = cell0 + (int64_t)min(c, ncols - 1) * cs;
#pragma unroll
                for (int q = 0; q < PCH; ++q) {
                    const int i = min(lane + 64 * q, npt - 1);
                    kv[c][q] = kap_all[col + i];
                    fv[c][q] = Fu_all[col + i];
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
#pragma unroll
                for (int q = 0; q < PCH; ++q) {
                    const int i = lane + 64 * q;
                    if (c < ncols && i < npt) {
                        s_kap[c * npt + i] = kv[c][q];
                        s_fu[c * npt + i] = fv[c][q];
                    }
                }
            }
        }
        __syncthreads();

        // ---- sublayer coefficients and warm start (once per call)
        R ca[K], cc[K], sg[K], fu[K], bu[K];
        {
            const R* kc = s_kap + cw * npt + lo;
            const R* fc = s_fu + cw * npt + lo;
            const R* dBc = s_dB + lo;
            const R* dmc = s_dm + lo;
            R kp = (R)0;
            if (cnt > 0) kp = kc[0];
            LayerQ<R> q;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                ca[k] = (R)1;
                cc[k] = (R)0;
                sg[k] = (R)0;
                fu[k] = (R)0;
                bu[k] = (R)0;
                if (k < cnt) {
                    if ((k & 1) == 0) q = layer_q<R>(s_w0[(lo + k) >> 1], s_g0[(lo + k) >> 1], D, inv_D, tpe);
                    const R kn = kc[k + 1];
                    const R dtau = (R)0.5 * (kp + kn) * dmc[k];
                    sub_coeffs_g<R>(q, dtau, tpe, dBc[k], ca[k], cc[k], sg[k]);
                    fu[k] = fc[k];
                    kp = kn;
                }
            }
        }

        // ---- pass-invariant parts of the column scans.  A segment's map is
        // x -> P x + b with P the product of its a_s (the same for both sweeps
        // and every pass).  The boundary values are folded into the end
        // segments (top: F_dn = F_top; bottom: F_up = F_dn + F_int), so every
        // scanned map ends up constant and only its offset b is scanned.
        constexpr int LOG2L = (L == 16) ? 4 : 5;
        // keep the multipliers in registers unless that would spill (wide FP64 segments)
        constexpr bool PRECOMP = (sizeof(R) == 4) || (K <= 8);
        R pseg = (R)1;
#pragma unroll
        for (int k = 0; k < K; ++k) pseg *= ca[k];
        R mdn[PRECOMP ? LOG2L : 1], mup[PRECOMP ? LOG2L : 1];
        if constexpr (PRECOMP) {
            R ma = (seg == L - 1) ? (R)0 : pseg;
            R mb = (seg == 0) ? (R)0 : pseg;
#pragma unroll
            for (int t = 0; t < LOG2L; ++t) {
                const int d = 1 << t;
                R a2, b2;
                if (t == 0) { a2 = grp_down<L, 1>(ma); b2 = grp_up<L, 1>(mb); }
                else if (t == 1) { a2 = grp_down<L, 2>(ma); b2 = grp_up<L, 2>(mb); }
                else if (t == 2) { a2 = grp_down<L, 4>(ma); b2 = grp_up<L, 4>(mb); }
                else if (t == 3) { a2 = grp_down<L, 8>(ma); b2 = grp_up<L, 8>(mb); }
                else { a2 = grp_down<L, 16>(ma); b2 = grp_up<L, 16>(mb); }
                const bool okd = seg + d < L, oku = seg >= d;
                mdn[t] = okd ? ma : (R)0;
                mup[t] = oku ? mb : (R)0;
                ma = okd ? ma * a2 : ma;
                mb = oku ? mb * b2 : mb;
            }
        }
        const R ftop_fold = pseg * Ftop;

        // the down sweep's per-sublayer offsets c F_up - sig, kept for the
        // replay when registers allow
        constexpr bool KEEP_T = (sizeof(R) == 4) || (K <= 8);
        R tk[KEEP_T ? K : 1];
        R ftoa = (R)0;
        for (int pass = 0; pass <= A.n_scat; ++pass) {
            const bool last = (pass == A.n_scat);
            // ---------------- downward sweep: compose my segment (top -> bottom)
            R MB = (R)0;
            if constexpr (KEEP_T) {
#pragma unroll
                for (int k = 0; k < K; ++k) tk[k] = cc[k] * fu[k] - sg[k];
#pragma unroll
                for (int k = K - 1; k >= 0; --k) MB = ca[k] * MB + tk[k];
            } else {
#pragma unroll
                for (int k = K - 1; k >= 0; --k) MB = ca[k] * MB + (cc[k] * fu[k] - sg[k]);
            }
            if (seg == L - 1) MB = ftop_fold + MB;
            if constexpr (PRECOMP) {  // suffix scan towards the BOA
                MB = scan_down_step<L, 0>(MB, mdn[0]);
                MB = scan_down_step<L, 1>(MB, mdn[1]);
                MB = scan_down_step<L, 2>(MB, mdn[2]);
                MB = scan_down_step<L, 3>(MB, mdn[3]);
                if constexpr (LOG2L > 4) MB = scan_down_step<L, 4>(MB, mdn[LOG2L - 1]);
            } else {
                R MA = (seg == L - 1) ? (R)0 : pseg;
                scan_down_full<L>(MA, MB, seg);
            }
            R x = grp_down<L, 1>(MB);  // F_dn at my segment's top point
            if (seg == L - 1) x = Ftop;
            // downward fluxes of the final pass go straight to LDS (the staged
            // warm start is dead by then), then the Gauss partials (column
            // sums) and, optionally, the per-g values are stored coalesced
            R* s_out = s_fu;
#pragma unroll
            for (int k = K - 1; k >= 0; --k) {
                bu[k] = cc[k] * x + sg[k];
                if constexpr (KEEP_T) x = ca[k] * x + tk[k];
                else x = ca[k] * x + (cc[k] * fu[k] - sg[k]);
                if (last && k < cnt) s_out[cw * npt + lo + k] = x;
            }
            if (last) {
                if (top_seg && colok) s_out[cw * npt + nsub] = Ftop;
                __syncthreads();
                for (int i = lane; i < npt; i += 64) {
                    const slot v = GS::col_sum(s_out + i, npt, ncols, wcol);
                    if (direct) part_dn[pb * A.wpb_stride + (int64_t)part * npt + i] = v;
                    else s_pd[i] += v;
                }
                if (Fd_all) {
                    for (int cc = 0; cc < ncols; ++cc) {
                        R* db = Fd_all + cell0 + (int64_t)cc * cs;
                        for (int i = lane; i < npt; i += 64) db[i] = s_out[cc * npt + i];
                    }
                }
                __syncthreads();
            }
            // ---------------- upward sweep: compose (bottom -> top); the BOA
            // condition F_up(0) = F_dn(0) + F_int lives in segment 0
            const R y0 = x + Fint;  // meaningful in segment 0 only
            MB = (R)0;
#pragma unroll
            for (int k = 0; k < K; ++k) MB = ca[k] * MB + bu[k];
            if (seg == 0) MB = pseg * y0 + MB;
            if constexpr (PRECOMP) {  // prefix scan towards the TOA
                MB = scan_up_step<L, 0>(MB, mup[0]);
                MB = scan_up_step<L, 1>(MB, mup[1]);
                MB = scan_up_step<L, 2>(MB, mup[2]);
                MB = scan_up_step<L, 3>(MB, mup[3]);
                if constexpr (LOG2L > 4) MB = scan_up_step<L, 4>(MB, mup[LOG2L - 1]);
            } else {
                R MA = (seg == 0) ? (R)0 : pseg;
                scan_up_full<L>(MA, MB, seg);
            }
            R y = grp_up<L, 1>(MB);  // F_up at my segment's bottom point
            if (seg == 0) y = y0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                fu[k] = y;
                y = ca[k] * y + bu[k];
            }
            ftoa = y;
        }

        // ---- outputs: upward fluxes (warm start of the next call) and their
        // Gauss partials, staged in LDS and stored coalesced
        {
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k < cnt) s_fu[cw * npt + lo + k] = fu[k];
            if (top_seg && colok) s_fu[cw * npt + nsub] = ftoa;
            __syncthreads();
            for (int i = lane; i < npt; i += 64) {
                const slot v = GS::col_sum(s_fu + i, npt, ncols, wcol);
                if (direct) part_up[pb * A.wpb_stride + (int64_t)part * npt + i] = v;
                else s_pu[i] += v;
            }
            for (int cc = 0; cc < ncols; ++cc) {
                R* ub = Fu_all + cell0 + (int64_t)cc * cs;
                for (int i = lane; i < npt; i += 64) ub[i] = s_fu[cc * npt + i];
            }
            __syncthreads();
        }
      }  // groups
        // ---- this wave's Gauss sums over its groups (one partial per point)
        if (!direct) {
            // partial slot of this (bin, part): [bin x point][stride] layout
            const int64_t poff = pb * A.wpb_stride + (int64_t)part * npt;
            for (int i = lane; i < npt; i += 64) {
                part_up[poff + i] = s_pu[i];
                part_dn[poff + i] = s_pd[i];
            }
        }
    }
}

// LDS bytes of one sweep workgroup.
template <int L>
static size_t sweep_lds(const SweepArgs& a, size_t rbytes) {
    constexpr int C = 64 / L;
    // staging + per-bin inputs + two Gauss-sum accumulators (slot = R; not
    // needed when every wave has a single group)
    const size_t acc = (a.parts >= a.wpb) ? 0 : 2 * (size_t)a.npt_max;
    return (size_t)(2 * C * a.npt_max + 2 * a.npt_max + a.npt_max + 1 + acc) * rbytes + 64;
}

// Occupancy hint (waves per SIMD) so the register arrays fit without spills.
template <int K, int L, bool F64>
constexpr int sweep_occ() {
    if (F64) return (K <= 4 && L == 16) ? 3 : ((K <= 8 || (K <= 14 && L == 16)) ? 2 : 1);
    if (L == 16) return K <= 8 ? 4 : (K <= 14 ? 3 : 2);
    return K <= 4 ? 4 : (K <= 8 ? 3 : (K <= 14 ? 2 : 1));
}

template <int K, int L>
static hipError_t launch_kp(const SweepArgs& a, bool mixed, int grid, hipStream_t s) {
    if (mixed)
        hipLaunchKernelGGL((sweep_kernel<K, L, float, sweep_occ<K, L, false>()>), dim3(grid), dim3(64),
                           sweep_lds<L>(a, 4), s, a);
    else
        hipLaunchKernelGGL((sweep_kernel<K, L, double, sweep_occ<K, L, true>()>), dim3(grid), dim3(64),
                           sweep_lds<L>(a, 8), s, a);
    return hipGetLastError();
}

template <int K>
static hipError_t launch_kl(const SweepArgs& a, int L, bool mixed, int grid, hipStream_t s) {
    if (L == 16) return launch_kp<K, 16>(a, mixed, grid, s);
    if (L == 32) return launch_kp<K, 32>(a, mixed, grid, s);
    return hipErrorInvalidValue;
}

hipError_t launch_sweep(const SweepArgs& a, int K, int L, bool mixed, int grid, hipStream_t s) {
    switch (K) {
        case 4: return launch_kl<4>(a, L, mixed, grid, s);
        case 8: return launch_kl<8>(a, L, mixed, grid, s);
        case 14: return launch_kl<14>(a, L, mixed, grid, s);
        case 26: return launch_kl<26>(a, L, mixed, grid, s);
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
    // sublayer-cell offsets: nb*ng*2n per atmosphere = 2 ng lb_off
    int lo = 0, hi = atm.n_atm;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (2 * (int64_t)atm.n_g * atm.lb_off[mid] <= idx) lo = mid; else hi = mid;
    }
    const int a = lo;
    const int64_t rel = idx - 2 * (int64_t)atm.n_g * atm.lb_off[a];
    const int n = atm.n_layer[a], nsub = 2 * n;
    const int64_t colx = rel / nsub;
    const int s = (int)(rel - colx * nsub);
    const int l = (int)(colx / atm.n_g);
    const int64_t cell = atm.cell_off[a] + colx * col_stride(n);
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
