// k_sweep.hip -- the two-stream flux solve of one temperature iteration
// (Sec. 2.1.3, 2.2.2, 2.2.3, 2.3), fused: sublayer coefficients, 1 + n_scat
// scattering passes, and the Gauss sum over g.
//
// Mapping.  One workgroup owns one wavelength bin of one atmosphere: n_g
// columns (one per Gauss point) of L lanes each (L = 16 or 32; the
// long-column shape K = 26, L = 64 gives one column the whole wave).  Lane `seg` of a column owns
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
//
// Isothermal-layer grid (Sec. 2.2.1, template flag ISO).  A slot is a whole
// isothermal layer j between interfaces j (point 2j) and j+1 (point 2j+2):
// its optical thickness is the centre opacity (point 2j+1) times its column
// mass, eq:isoscat (eq:purescat) at any thickness.  Interface j carries the
// deviation from tpe B_j = (2 pi / D) B(T_j) of the layer above it (the TOA
// that of the top layer).  The layer maps tpe B_j to itself for any a, c, so
// substituting F = G + tpe B with the two references leaves as the only
// source the change of reference dB_j = B_j - B_{j+1}:
//   up:   G_up(j+1) = a G_up(j) + c G_dn(j+1) + (1 - c) tpe dB_j
//   down: G_dn(j)   = a G_dn(j+1) + c G_up(j) - a tpe dB_j
// (the composition of the layer without a source and an identity slot that
// adds tpe dB_j, both directions).  Each slot writes two points: 2j holds
// interface j, 2j+1 interface j+1 in the layer's own reference, i.e.
// G(j+1) - tpe dB_j, so the output layout is that of the sublayered grid.
//
// Rayleigh scattering (Sec. 2.1.4, template flag RAY).  The bin's H2
// scattering opacity sigma/mbar is added to every sublayer and the albedo
// follows per sublayer and g-point from the scattering share of the
// extinction (g0 = 0), so r, kx and the pure-scattering switch are formed per
// sublayer in the coefficient set-up instead of per layer in LDS; the passes
// are unchanged.
#include <type_traits>

#include "helios_internal.hpp"

namespace helios {

template <typename R>
struct Prec;
template <>
struct Prec<double> {
    // T = exp(-x) and om = 1 - T (om accurate for thin layers)
    __device__ static inline void t_om(double x, double& T, double& om) { exp_neg_om(x, T, om); }
    // the sweep's staged kx carries no unit factor in FP64
    static constexpr double kx_unit = 1.0;
    __device__ static inline void t_om_u(double x, double& T, double& om) { exp_neg_om(x, T, om); }
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
    // The sweep's FP32 kx is staged in base-2 units (times log2 e), so that
    // y = kx dtau feeds the hardware exp2 directly: T = 2^-y, and
    // om = 1 - 2^-y from its Taylor series in y (coefficients (-1)^k
    // ln2^(k+1)/(k+1)!, the same truncation as above) below y = 0.25/ln2.
    static constexpr float kx_unit = 1.4426950408889634f;
    __device__ static inline void t_om_u(float y, float& T, float& om) {
        T = __builtin_amdgcn_exp2f(-y);
        float p = y * -1.5403530393381606e-4f + 1.3333558146428441e-3f;
        p = y * p - 9.618129107628477e-3f;
        p = y * p + 5.5504108664821576e-2f;
        p = y * p - 0.2402265069591007f;
        p = y * p + 0.6931471805599453f;
        om = (y < 0.36067376f) ? y * p : 1.0f - T;
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

// Per-layer quantities of the sweep, the same for a layer's two sublayers and
// every g of a bin (staged in LDS once per bin):
//   r = sqrt((1 - w0)/(1 - w0 g0)),  kx = D sqrt((1 - w0 g0)(1 - w0)),
//   sf = 2 pi eps f = 2 pi eps / (D (1 - w0 g0)),
//   gd = D (1 - g0)/2 for a pure scatterer ((1 - w0) < 1e-6), else -1.
template <typename R>
__device__ inline void layer_g(R w0, R g0, R D, R inv_D, R tpe, R& r, R& kx, R& sf, R& gd) {
    const R one = (R)1;
    const R omg = one - w0 * g0;
    const R iomg = Prec<R>::rcp(omg);
    r = Prec<R>::sqrt_((one - w0) * iomg);
    kx = D * r * omg * Prec<R>::kx_unit;
    sf = tpe * iomg * inv_D;
    gd = ((one - w0) < (R)1e-6) ? D * (one - g0) * (R)0.5 : (R)-1;
}

// The sweep's coefficients of one sublayer in the deviation form: a, c and
// the source sig for the Planck difference dB = B_lower - B_upper, from the
// layer's quantities (zp = (1 + r)/2, zm = (1 - r)/2).  One reciprocal,
// rec = 1/((zp - zm T)(zp + zm T) dtau), serves a, c and the gradient term.
// dtau is floored at a power of two, so that a transparent sublayer stays
// finite and a padding sublayer (dtau = 0, dB = 0, r = 1, kx = sf = 0) is
// exactly the identity map (a = 1, c = sig = 0).  Thin sublayers with a
// Planck difference take the eq:isoscat form (with dB = 0 both forms give
// sig = 0).
template <typename R>
__device__ inline void sub_coeffs_g(R r, R kx, R sf, R gd, R zp, R zm, R zpzm, R dtau, R two_pi_eps, R dB,
                                    R& a, R& c, R& sig) {
    const R one = (R)1;
    R T, om;
    Prec<R>::t_om_u(kx * dtau, T, om);
    const R u = zp - zm * T, v = zp + zm * T;
    const R den = u * v;
    R dd;
    if constexpr (sizeof(R) == 4)  // dtau >= 0: the integer maximum of the bit patterns is the float one
        dd = __int_as_float(max(__float_as_int(dtau), __float_as_int(0x1p-100f)));
    else
        dd = fmax(dtau, (R)0x1p-960);
    const R rec = Prec<R>::rcp(den * dd);
    const R iden = rec * dd;  // 1/den
    const R omi = om * iden;
    a = r * T * iden;
    c = zpzm * (one + T) * omi;
    sig = sf * dB * v * om * rec;  // 2 pi eps f dB om / ((zp - zm T) dtau)
    // eq:isoscat; the wave-wide tests are ballots of the compare masks
    const bool iso = dtau < (R)1e-4 && dB != (R)0;
    if (__builtin_amdgcn_ballot_w64(iso) != 0) sig = iso ? (R)0.5 * two_pi_eps * (one + a - c) * dB : sig;
    if (__builtin_amdgcn_ballot_w64(gd >= (R)0) != 0) {  // eq:purescat
        const bool ps = gd >= (R)0;
        const R g = gd * dtau;
        const R qq = g * Prec<R>::rcp(one + g);
        a = ps ? one - qq : a;
        c = ps ? qq : c;
        sig = ps ? two_pi_eps * (one - qq) * dB : sig;
    }
}

// Lane exchanges of the column scans.  A DPP move reads another lane of the
// wave as an operand modifier of an ordinary VALU instruction (no LDS round
// trip, no wait): row_shl/row_shr:d read lane +-d within a row of 16 lanes
// (out-of-row sources read 0), wave_shl/wave_shr:1 read lane +-1 across the
// whole wave, row_bcast:15 gives every lane of a row the last lane of the
// row below it, row_newbcast:0 gives every lane of a row the row's first lane.
template <int CTRL, int ROWS = 0xF>
__device__ inline float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS = 0xF>
__device__ inline double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// gfx950's permlane16/permlane32 swaps with one register as both operands
// return in every lane the lower and the upper member of its lane pair
// (lanes i and i ^ 16, or i and i ^ 32, of each 32- or 64-lane half).
template <int S>
__device__ inline unsigned pair_lo_hi(unsigned u, unsigned& hi) {
    if constexpr (S == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        hi = r[1];
        return r[0];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        hi = r[1];
        return r[0];
    }
}
// the upper member (lane i | 16) of every lane's pair
__device__ inline float upper16(float v) {
    unsigned hi;
    (void)pair_lo_hi<16>(__float_as_uint(v), hi);
    return __uint_as_float(hi);
}
__device__ inline double upper16(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    unsigned hi_l, hi_h;
    (void)pair_lo_hi<16>((unsigned)b, hi_l);
    (void)pair_lo_hi<16>((unsigned)(b >> 32), hi_h);
    return __longlong_as_double((long long)(((unsigned long long)hi_h << 32) | hi_l));
}

// The column scans combine the lanes' affine maps in log2(L) steps.  Step T
// pairs lane seg with lane seg +- 2^T of its group.  For L = 16 the group is
// one DPP row.  For L = 32 (two rows) steps 0..3 run within each row and
// step 4 joins the rows: the lower row takes the first lane of the row above
// (row_newbcast:0, then the permlane16 swap), the upper row the last lane of
// the row below (row_bcast:15); every exchange is a VALU operation.  L = 64
// uses shuffles (out-of-group sources read the own value, which the callers
// never use).
template <int L, int T>
__device__ inline bool has_above(int seg) {  // a partner towards the TOA at step T
    if constexpr (L == 32 && T < 4) return (seg & 15) + (1 << T) < 16;
    else if constexpr (L == 32) return seg < 16;
    else return seg + (1 << T) < L;
}
template <int L, int T>
__device__ inline bool has_below(int seg) {  // a partner towards the BOA at step T
    if constexpr (L == 32 && T < 4) return (seg & 15) >= (1 << T);
    else if constexpr (L == 32) return seg >= 16;
    else return seg >= (1 << T);
}
// the partner's value at step T (towards the TOA / towards the BOA)
template <int L, int T, typename R>
__device__ inline R from_above(R v) {
    if constexpr (L == 16 || (L == 32 && T < 4)) return dpp_mov<0x100 + (1 << T)>(v);
    else if constexpr (L == 32) return upper16(dpp_mov<0x150>(v));
    else return __shfl_down(v, 1u << T, L);
}
template <int L, int T, typename R>
__device__ inline R from_below(R v) {
    if constexpr (L == 16 || (L == 32 && T < 4)) return dpp_mov<0x110 + (1 << T)>(v);
    else if constexpr (L == 32) return dpp_mov<0x142, 0xA>(v);
    else return __shfl_up(v, 1u << T, L);
}
// value of the next lane of the column (towards the TOA) and of the previous
// one (towards the BOA); the top and bottom lanes' results are not used
template <int L, typename R>
__device__ inline R next_lane(R v) {
    if constexpr (L == 16) return dpp_mov<0x101>(v);
    else if constexpr (L == 32) return dpp_mov<0x130>(v);
    else return __shfl_down(v, 1u, L);
}
template <int L, typename R>
__device__ inline R prev_lane(R v) {
    if constexpr (L == 16) return dpp_mov<0x111>(v);
    else if constexpr (L == 32) return dpp_mov<0x138>(v);
    else return __shfl_up(v, 1u, L);
}

// One scan step of affine maps whose multipliers are pass-invariant:
// MB <- mult * MB(partner) + MB (mult is 0 where there is no partner).
template <int L, int T, typename R>
__device__ inline R scan_down_step(R MB, R mult) {
    return mult * from_above<L, T>(MB) + MB;
}
template <int L, int T, typename R>
__device__ inline R scan_up_step(R MB, R mult) {
    return mult * from_below<L, T>(MB) + MB;
}

// Full scan step pairs (multiplier and offset) for when the multipliers are
// not kept between passes.
template <int L, int T, typename R>
__device__ inline void down_pair(R& MA, R& MB, int seg) {
    const R a2 = from_above<L, T>(MA), b2 = from_above<L, T>(MB);
    const bool ok = has_above<L, T>(seg);
    MB = ok ? MA * b2 + MB : MB;
    MA = ok ? MA * a2 : MA;
}
template <int L, int T, typename R>
__device__ inline void up_pair(R& MA, R& MB, int seg) {
    const R a2 = from_below<L, T>(MA), b2 = from_below<L, T>(MB);
    const bool ok = has_below<L, T>(seg);
    MB = ok ? MA * b2 + MB : MB;
    MA = ok ? MA * a2 : MA;
}
template <int L, typename R>
__device__ inline void scan_down_full(R& MA, R& MB, int seg) {
    down_pair<L, 0>(MA, MB, seg);
    down_pair<L, 1>(MA, MB, seg);
    down_pair<L, 2>(MA, MB, seg);
    down_pair<L, 3>(MA, MB, seg);
    if constexpr (L > 16) down_pair<L, 4>(MA, MB, seg);
    if constexpr (L > 32) down_pair<L, 5>(MA, MB, seg);
}
template <int L, typename R>
__device__ inline void scan_up_full(R& MA, R& MB, int seg) {
    up_pair<L, 0>(MA, MB, seg);
    up_pair<L, 1>(MA, MB, seg);
    up_pair<L, 2>(MA, MB, seg);
    up_pair<L, 3>(MA, MB, seg);
    if constexpr (L > 16) up_pair<L, 4>(MA, MB, seg);
    if constexpr (L > 32) up_pair<L, 5>(MA, MB, seg);
}

// v(lane) + v(lane ^ S) for S = 16 or 32 with the permlane swaps: both
// lanes of a pair form the same sum (lower + upper).
template <int S>
__device__ inline float xor_pair_sum(float v) {
    unsigned hi;
    const unsigned lo = pair_lo_hi<S>(__float_as_uint(v), hi);
    return __uint_as_float(lo) + __uint_as_float(hi);
}
template <int S>
__device__ inline double xor_pair_sum(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    unsigned lo_h, hi_h, lo_l, hi_l;
    lo_l = pair_lo_hi<S>((unsigned)b, hi_l);
    lo_h = pair_lo_hi<S>((unsigned)(b >> 32), hi_h);
    const double lo = __longlong_as_double((long long)(((unsigned long long)lo_h << 32) | lo_l));
    const double hi = __longlong_as_double((long long)(((unsigned long long)hi_h << 32) | hi_l));
    return lo + hi;
}

// Sum of v over the wave's C = 64/L columns (lanes seg, seg + L, ...); every
// column gets the same value, added in the order ((c0 + c1) + (c2 + c3)).
template <int L, typename R>
__device__ inline R col_sum(R v) {
    if constexpr (L <= 16) v = xor_pair_sum<16>(v);
    if constexpr (L <= 32) v = xor_pair_sum<32>(v);
    return v;
}

// LDS layout of a sweep workgroup of shape (K, L), in elements of R (each
// block starts on a multiple of 4 elements).  Arrays span the shape's full
// capacity of K*L sublayers so that every lane can address its K sublayers
// without bounds tests: sublayers past the column hold the identity.
//   dB, hdm  [K*L + 1]   Planck difference and half column mass per sublayer
//   tB       [K*L + 1]   (2 pi / D) B per point (flux-state variant only)
//   lq       [K*L/2][4]  r, kx, sf, gd per layer
//   pu, pd   [K*L + 2]   Gauss sums per point (slots past the column's
//                        points take zeros)
// On the isothermal-layer grid a slot is a whole layer with two points (its
// lower interface and the point above it), so dB, hdm and lq are per layer
// and tB, pu, pd span 2 K*L + 2 points.
struct SweepLds {
    int dB, hdm, tB, lq, pu, pd, total;
    static constexpr int r4(int v) { return (v + 3) & ~3; }
    __host__ __device__ constexpr SweepLds(int KL, bool iso = false, bool fs = false)
        : dB(0),
          hdm(r4(KL + 1)),
          tB(2 * r4(KL + 1)),
          lq(tB + (fs ? r4(iso ? 2 * KL + 2 : KL + 1) : 0)),
          pu(lq + 4 * r4(iso ? KL : KL / 2)),
          pd(pu + r4(iso ? 2 * KL + 2 : KL + 2)),
          total(pd + r4(iso ? 2 * KL + 2 : KL + 2)) {}
};

// One workgroup = one wave, which owns one (bin, part) at a time.  It stages
// the bin's Planck differences, half column masses and per-layer quantities
// in LDS once, then solves its share of the bin's n_g columns C = 64/L at a
// time (group j covers g in [j*C, j*C + C)).  Each lane reads the opacities
// and warm start of its own K points straight from HBM (pairs of values, all
// loads issued before the first is used) and writes its fluxes back the same
// way.  The Gauss sums over a group's columns are formed with cross-column
// shuffles and accumulated per point in LDS over the wave's groups, then
// written out coalesced: one partial per (bin, part, point).  Large launches
// give a bin one part; launches with few bins split a bin's groups over
// several waves.  The bin-sum kernel adds a bin's partials in order, adds the
// Planck term and sums over bins.  No barrier spans more than the wave.
// FS: the caller's per-g arrays hold fluxes (HELIOS_STATE_FLUX); the sweep
// still carries deviations, taking (2 pi / D) B off the warm start as it is
// read and adding it back to the per-g values as they are stored.
template <int K, int L, typename R, int OCC, bool RAY, bool ISO, bool FS>
__global__ void __launch_bounds__(64, OCC) sweep_kernel(const SweepArgs A) {
    using R2 = typename std::conditional<sizeof(R) == 8, double2, float2>::type;
    constexpr int C = 64 / L;
    constexpr int KH = K / 2;
    constexpr int KL = K * L;
    constexpr SweepLds lay(KL, ISO, FS);
    static_assert(K % 2 == 0, "segments hold whole layers");
    static_assert(!(RAY && ISO), "Rayleigh scattering is solved on the sublayered grid");
    extern __shared__ unsigned char smem_raw[];
    R* sm = reinterpret_cast<R*>(smem_raw);
    R* s_dB = sm + lay.dB;
    R* s_hdm = sm + lay.hdm;
    R* s_tB = sm + lay.tB;
    R* s_lq = sm + lay.lq;
    R* s_pu = sm + lay.pu;
    R* s_pd = sm + lay.pd;

    const int lane = threadIdx.x;
    const int seg = lane & (L - 1);
    const int cw = lane / L;
    const int lo = seg * K;
    const R* __restrict__ kap_all = static_cast<const R*>(A.kappa);
    const double* __restrict__ B_all = static_cast<const double*>(A.B);
    R* __restrict__ Fu_all = static_cast<R*>(A.F_up_g);
    R* __restrict__ Fd_all = static_cast<R*>(A.F_dn_g);
    R* __restrict__ part_up = static_cast<R*>(A.part_up);
    R* __restrict__ part_dn = static_cast<R*>(A.part_dn);
    const R D = (R)A.D;
    const R inv_D = (R)(1.0 / A.D);
    const R tpe = (R)(2.0 * kPi / A.D);
    const double tpe_d = 2.0 * kPi / A.D;
    // FP32: the Gauss weights held one per lane (n_g <= HELIOS_MAX_NG = 32 <
    // 64), so that a group takes its columns' weights with a lane exchange
    // instead of reloading the weight array's address
    const float gw_lane = (lane < A.n_g) ? (float)A.gw[lane] : 0.0f;

    for (int64_t item = A.w_begin + blockIdx.x; item < A.w_end; item += gridDim.x) {
        const int64_t gb = (A.parts == 1) ? item : item / A.parts;
        const int part = (int)(item - gb * A.parts);
        const int at = A.bin_atm[gb];
        const int l = (int)(gb - A.bin_off[at]);
        const int n = A.n_layer[at];
        if (n < A.n_lo || n > A.n_hi || frozen(A.status, at)) continue;  // uniform per wave
        const int nsub = 2 * n, npt = nsub + 1;  // the TOA point is nsub on both grids
        const int nsl = ISO ? n : nsub;         // slots: layers (isothermal grid) or sublayers
        const int nact = (nsl + K - 1) / K;
        const int scnt = (seg < nact) ? min(K, nsl - lo) : 0;  // slots owned (any column)
        const bool top_seg = (seg == nact - 1);                // also owns the TOA point
        const int cs = col_stride(n);
        const int64_t pb = A.pb_off[at] + (int64_t)l * npt;
        const int64_t lb = A.lb_off[at] + (int64_t)l * n;
        const double* __restrict__ P = A.P_pt + A.pt_off[at];
        const double higrav = 0.5 / A.grav[at];
        // TOA value of the downward deviation, formed in FP64
        const R Ftop = (R)(A.F_top[A.bin_off[at] + l] - (2.0 * kPi / A.D) * B_all[pb + nsub]);
        // BOA flux: pi B(T_int) scaled so that its width-weighted sum over the
        // atmosphere's bins is sigma T_int^4 (chunk sums added in order)
        R Fint;
        {
            const int nbch = (int)((A.bin_off[at + 1] - A.bin_off[at] + kBndChunk - 1) / kBndChunk);
            const double* bp = A.bnd_part + (int64_t)at * A.bnd_maxch;
            double sum = 0.0;
            for (int c = 0; c < nbch; ++c) sum += bp[c];
            const double t2 = A.T_int[at] * A.T_int[at];
            const double scale = (sum > 0.0) ? sigma_sb() * t2 * t2 / sum : 0.0;
            Fint = (R)(A.F_int[A.bin_off[at] + l] * scale);
        }
        // Rayleigh scattering (Sec. 2.1.4): twice the bin's H2 scattering
        // opacity sigma / mbar, so that its sublayer depth is kR2 times the
        // half column mass
        R kR2 = (R)0;
        if constexpr (RAY) kR2 = (R)(2.0 * rayleigh_h2(A.lambda_c[A.bin_off[at] + l]) * A.inv_mbar);

        // ---- the bin's per-sublayer and per-layer inputs, staged once for
        // all g, padded with the identity up to the shape's capacity.  All
        // loads are issued before the first is consumed (compile-time bounds,
        // indices clamped into the bin's own rows).
        if constexpr (ISO) {
            // per layer j: dB = B(2j+1) - B(2j+2) (its own Planck value minus the
            // reference of its upper interface), half its column mass, and its
            // r, kx, sf, gd; per point: the flux-state reference (FS) and the
            // Gauss-sum slots of every point of the capacity cleared
            constexpr int SCH = (KL + 63) / 64;
            constexpr int QCH = (2 * KL + 2 + 63) / 64;
            for (int q = 0; q < SCH; ++q) {  // one chunk of 64 layers at a time
                const int j = lane + 64 * q;
                const int jc = min(j, n - 1);
                const double b1 = B_all[pb + 2 * jc + 1], b2 = B_all[pb + 2 * jc + 2];
                const double p0 = P[2 * jc], p2 = P[2 * jc + 2];
                const double wv = A.w0[lb + jc], gv = A.g0[lb + jc];
                if (j < KL) {
                    const bool real = j < n;
                    s_dB[j] = real ? (R)(b1 - b2) : (R)0;
                    s_hdm[j] = real ? (R)((p0 - p2) * higrav) : (R)0;
                    R r = (R)1, kx = (R)0, sf = (R)0, gd = (R)-1;
                    if (real) layer_g<R>((R)wv, (R)gv, D, inv_D, tpe, r, kx, sf, gd);
                    s_lq[4 * j + 0] = r;
                    s_lq[4 * j + 1] = kx;
                    s_lq[4 * j + 2] = sf;
                    s_lq[4 * j + 3] = gd;
                }
            }
#pragma unroll
            for (int q = 0; q < QCH; ++q) {
                const int i = lane + 64 * q;
                if (i <= 2 * KL + 1) {
                    if constexpr (FS) s_tB[i] = (i < npt) ? (R)(tpe_d * B_all[pb + i]) : (R)0;
                    s_pu[i] = (R)0;
                    s_pd[i] = (R)0;
                }
            }
        } else {
            constexpr int PCH = (KL + 2 + 63) / 64;
            constexpr int LCH = (KL / 2 + 63) / 64;
            double bv[PCH], pv[PCH], wv[LCH], gv[LCH];
#pragma unroll
            for (int q = 0; q < PCH; ++q) {
                const int i = min(lane + 64 * q, npt - 1);
                bv[q] = B_all[pb + i];
                pv[q] = P[i];
            }
            if constexpr (!RAY) {
#pragma unroll
                for (int q = 0; q < LCH; ++q) {
                    const int i = min(lane + 64 * q, n - 1);
                    wv[q] = A.w0[lb + i];
                    gv[q] = A.g0[lb + i];
                }
            }
            // sublayer differences from the next point's value: the next lane,
            // or lane 0 of the next chunk for lane 63
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
                const bool real = i < nsub;
                if (i <= KL) {
                    s_dB[i] = real ? (R)(bv[q] - bn) : (R)0;
                    s_hdm[i] = real ? (R)((pv[q] - pn) * higrav) : (R)0;
                    if constexpr (FS) s_tB[i] = (i < npt) ? (R)(tpe_d * bv[q]) : (R)0;
                }
                if (i <= KL + 1) {
                    s_pu[i] = (R)0;
                    s_pd[i] = (R)0;
                }
            }
            if constexpr (!RAY) {
#pragma unroll
                for (int q = 0; q < LCH; ++q) {
                    const int i = lane + 64 * q;
                    if (i < KL / 2) {
                        R r = (R)1, kx = (R)0, sf = (R)0, gd = (R)-1;
                        if (i < n) layer_g<R>((R)wv[q], (R)gv[q], D, inv_D, tpe, r, kx, sf, gd);
                        s_lq[4 * i + 0] = r;
                        s_lq[4 * i + 1] = kx;
                        s_lq[4 * i + 2] = sf;
                        s_lq[4 * i + 3] = gd;
                    }
                }
            }
        }
        __syncthreads();

        const int gpp = (A.wpb + A.parts - 1) / A.parts;  // groups of this wave: [j_lo, j_hi)
        const int j_lo = part * gpp, j_hi = min(A.wpb, j_lo + gpp);
      for (int j = j_lo; j < j_hi; ++j) {  // groups of C columns
        const int ncols = min(C, A.n_g - j * C);  // columns of this group
        const bool colok = cw < ncols;
        const int cnt = colok ? scnt : 0;
        // the group's first column (uniform) and my column's offset from it
        // (a surplus column of a short last group reads the group's last
        // column and writes nothing)
        const int64_t gcol = A.cell_off[at] + ((int64_t)l * A.n_g + j * C) * cs;
        const R* __restrict__ kap_g = kap_all + gcol;
        R* __restrict__ fu_g = Fu_all + gcol;
        const uint32_t col = (uint32_t)(min(cw, ncols - 1) * cs);
        R wg;  // Gauss weight of my column
        if constexpr (sizeof(R) == 4) {
            const float wsrc = __shfl(gw_lane, min(j * C + cw, 63), 64);  // every lane takes part
            wg = colok ? wsrc : 0.0f;
        } else {
            wg = colok ? (R)A.gw[j * C + cw] : (R)0;
        }

        // ---- my points' opacities (lo .. lo + K) and warm start (lo .. lo + K - 1):
        // pairs starting at even indices, clamped to nsub; a pair at nsub also
        // reads index nsub + 1 < col_stride (npt is odd), which is not used
        R kv[K + 2], fu[K];
        if constexpr (ISO) {
            // slot k is layer lo + k: the warm start at its lower interface
            // 2(lo + k) and the opacity at its centre 2(lo + k) + 1
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t pt = (uint32_t)min(2 * (lo + k), nsub - 1);  // interface; its layer's centre is pt + 1
                kv[k] = kap_g[col + pt + 1];
                fu[k] = fu_g[col + pt];
            }
            if constexpr (FS) {
#pragma unroll
                for (int k = 0; k < K; ++k) fu[k] -= s_tB[2 * (lo + k)];
            }
        } else {
            R2 kp2[KH + 1], fp2[KH];
#pragma unroll
            for (int p = 0; p <= KH; ++p)
                kp2[p] = *reinterpret_cast<const R2*>(kap_g + (col + (uint32_t)min(lo + 2 * p, nsub)));
#pragma unroll
            for (int p = 0; p < KH; ++p)
                fp2[p] = *reinterpret_cast<const R2*>(fu_g + (col + (uint32_t)min(lo + 2 * p, nsub)));
#pragma unroll
            for (int p = 0; p <= KH; ++p) {
                kv[2 * p] = kp2[p].x;
                kv[2 * p + 1] = kp2[p].y;
            }
#pragma unroll
            for (int p = 0; p < KH; ++p) {
                fu[2 * p] = fp2[p].x;
                fu[2 * p + 1] = fp2[p].y;
            }
            if constexpr (FS) {  // the sweep carries deviations from the isothermal flux
#pragma unroll
                for (int k = 0; k < K; ++k) fu[k] -= s_tB[lo + k];
            }
        }

        // ---- sublayer coefficients (once per call); sublayers past my
        // column's end get dtau = 0 and the LDS padding, i.e. the identity
        R ca[K], cc[K], sg[K];
        {
            R r = (R)1, kx = (R)0, sf = (R)0, gd = (R)-1, zp = (R)1, zm = (R)0, zpzm = (R)0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool act = k < cnt;
                if constexpr (ISO) {
                    // the whole layer at its centre's opacity, eq:isoscat at any
                    // optical depth (eq:purescat where 1 - w0 < 1e-6); its source
                    // in the deviation form only moves the reference from the
                    // layer's own Planck value to that of its upper interface
                    const R* lq = s_lq + 4 * (lo + k);
                    r = lq[0];
                    kx = lq[1];
                    sf = lq[2];
                    gd = lq[3];
                    zp = (R)0.5 + (R)0.5 * r;
                    zm = (R)0.5 - (R)0.5 * r;
                    zpzm = zp * zm;
                    const R dtau = act ? (kv[k] + kv[k]) * s_hdm[lo + k] : (R)0;
                    fu[k] = act ? fu[k] : (R)0;
                    sub_coeffs_g<R>(r, kx, sf, gd, zp, zm, zpzm, dtau, tpe, (R)0, ca[k], cc[k], sg[k]);
                    sg[k] = tpe * s_dB[lo + k];
                    // the long shapes read one layer's LDS values at a time (all
                    // of them hoisted ahead would hold 5 K values in registers)
                    if constexpr (K >= kLongK) asm volatile("" ::: "memory");
                    continue;
                }
                if constexpr (RAY) {
                    // the sublayer's own optics: absorption (mean of its end
                    // opacities) plus H2 scattering; albedo w0 = scattering
                    // share, 1 - w0 formed as the absorption share; g0 = 0
                    const R dabs = act ? (kv[k] + kv[k + 1]) * s_hdm[lo + k] : (R)0;
                    const R dtau = act ? dabs + kR2 * s_hdm[lo + k] : (R)0;
                    const R omw = (dtau > (R)0) ? dabs * Prec<R>::rcp(dtau) : (R)1;
                    r = Prec<R>::sqrt_(omw);
                    kx = D * Prec<R>::kx_unit * r;
                    sf = tpe * inv_D;
                    gd = (omw < (R)1e-6) ? D * (R)0.5 : (R)-1;
                    zp = (R)0.5 + (R)0.5 * r;
                    zm = (R)0.5 - (R)0.5 * r;
                    zpzm = zp * zm;
                    fu[k] = act ? fu[k] : (R)0;
                    sub_coeffs_g<R>(r, kx, sf, gd, zp, zm, zpzm, dtau, tpe, s_dB[lo + k], ca[k], cc[k], sg[k]);
                    continue;
                }
                if ((k & 1) == 0) {
                    const R* lq = s_lq + 4 * ((lo + k) >> 1);
                    r = lq[0];
                    kx = lq[1];
                    sf = lq[2];
                    gd = lq[3];
                    zp = (R)0.5 + (R)0.5 * r;
                    zm = (R)0.5 - (R)0.5 * r;
                    zpzm = zp * zm;
                }
                // sublayer: mean of its end opacities times its column mass.
                // (iso_grid is 0 on this path; the long shapes keep a
                // two-branch form that compiles to fewer registers there: 440
                // against 512 plus spills in the FP64 long-column shape.)
                R dtau;
                if constexpr (K >= kLongK) {
                    if ((k & 1) == 0) {
                        const R k_lo = A.iso_grid ? kv[k + 1] : kv[k];
                        const R hm = A.iso_grid ? s_hdm[lo + k] + s_hdm[lo + k + 1] : s_hdm[lo + k];
                        dtau = act ? (k_lo + kv[k + 1]) * hm : (R)0;
                    } else {
                        dtau = (act && !A.iso_grid) ? (kv[k] + kv[k + 1]) * s_hdm[lo + k] : (R)0;
                    }
                } else {
                    // past the column's last sublayer the LDS padding gives
                    // dtau = 0 (a surplus column's lanes compute values that
                    // carry zero Gauss weight and are not stored), and the
                    // identity map's c = 0 cancels the clamped warm start
                    dtau = (kv[k] + kv[k + 1]) * s_hdm[lo + k];
                }
                if constexpr (K >= kLongK) fu[k] = act ? fu[k] : (R)0;
                sub_coeffs_g<R>(r, kx, sf, gd, zp, zm, zpzm, dtau, tpe, s_dB[lo + k], ca[k], cc[k], sg[k]);
            }
        }

        // ---- pass-invariant parts of the column scans.  A segment's map is
        // x -> P x + b with P the product of its a_s (the same for both sweeps
        // and every pass).  The boundary values are folded into the end
        // segments (top: F_dn = F_top; bottom: F_up = F_dn + F_int), so every
        // scanned map ends up constant and only its offset b is scanned.
        constexpr int LOG2L = (L == 16) ? 4 : (L == 32 ? 5 : 6);
        // keep the scan multipliers in registers unless that would spill
        constexpr bool PRECOMP = (sizeof(R) == 4) || (K <= 14);
        R pseg = (R)1;
#pragma unroll
        for (int k = 0; k < K; ++k) pseg *= ca[k];
        R mdn[PRECOMP ? LOG2L : 1], mup[PRECOMP ? LOG2L : 1];
        if constexpr (PRECOMP) {
            R ma = (seg == L - 1) ? (R)0 : pseg;
            R mb = (seg == 0) ? (R)0 : pseg;
#pragma unroll
            for (int t = 0; t < LOG2L; ++t) {
                R a2, b2;
                bool okd, oku;
                if (t == 0) { a2 = from_above<L, 0>(ma); b2 = from_below<L, 0>(mb); okd = has_above<L, 0>(seg); oku = has_below<L, 0>(seg); }
                else if (t == 1) { a2 = from_above<L, 1>(ma); b2 = from_below<L, 1>(mb); okd = has_above<L, 1>(seg); oku = has_below<L, 1>(seg); }
                else if (t == 2) { a2 = from_above<L, 2>(ma); b2 = from_below<L, 2>(mb); okd = has_above<L, 2>(seg); oku = has_below<L, 2>(seg); }
                else if (t == 3) { a2 = from_above<L, 3>(ma); b2 = from_below<L, 3>(mb); okd = has_above<L, 3>(seg); oku = has_below<L, 3>(seg); }
                else if (t == 4) { a2 = from_above<L, 4>(ma); b2 = from_below<L, 4>(mb); okd = has_above<L, 4>(seg); oku = has_below<L, 4>(seg); }
                else { a2 = from_above<L, 5>(ma); b2 = from_below<L, 5>(mb); okd = has_above<L, 5>(seg); oku = has_below<L, 5>(seg); }
                mdn[t] = okd ? ma : (R)0;
                mup[t] = oku ? mb : (R)0;
                ma = okd ? ma * a2 : ma;
                mb = oku ? mb * b2 : mb;
            }
        }
        const R ftop_fold = pseg * Ftop;

        // Gauss sums of one stream over the group's columns at my points
        // (v[k] at lo + k, vtop at the TOA for the top segment), added to the
        // wave's LDS accumulators.  Every column of a point computes the same
        // sum and writes the same value.  A lane's K slots lo .. lo + K - 1 are
        // its own; slots past the column's last sublayer take zeros, and the
        // TOA point is added last (its slot may be one of them), so all K
        // reads are issued before the first write.
        auto emit = [&](const R (&v)[K], R vtop, R* acc) {
            R* a = acc + lo;
            R prev[K];
#pragma unroll
            for (int k = 0; k < K; ++k) prev[k] = a[k];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const R sk = col_sum<L>(wg * v[k]);
                a[k] = prev[k] + ((lo + k < nsub) ? sk : (R)0);
            }
            const R st = col_sum<L>(wg * vtop);
            if (top_seg) acc[nsub] += st;
        };
        // Isothermal-layer grid: slot k has two points, its lower interface
        // 2(lo + k) (v[k]) and the point above it, which carries the flux at
        // the next interface in the layer's own Planck reference (the slot's
        // upper value, v[k + 1] or vlast, minus its reference shift sg[k]).
        auto upper_iso = [&](const auto& v, R vlast, int k) -> R {
            return (k + 1 < K ? v[k + 1 < K ? k + 1 : k] : vlast) - sg[k];
        };
        auto emit_iso = [&](const auto& v, R vlast, R* acc) {
            R* a = acc + 2 * lo;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool act = lo + k < nsl;
                const R s0 = col_sum<L>(wg * v[k]);
                const R s1 = col_sum<L>(wg * upper_iso(v, vlast, k));
                a[2 * k] += act ? s0 : (R)0;
                a[2 * k + 1] += act ? s1 : (R)0;
                // the long shapes take one slot's read-modify-writes at a time:
                // hoisting all 2K reads would hold 2K values in registers
                if constexpr (K >= kLongK) asm volatile("" ::: "memory");
            }
            const R st = col_sum<L>(wg * vlast);
            if (top_seg) acc[nsub] += st;
        };
        auto store_iso = [&](const auto& v, R vlast, R* __restrict__ dst_g) {
            if (!colok) return;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (k < cnt) {
                    R2 w;
                    w.x = v[k];
                    w.y = upper_iso(v, vlast, k);
                    if constexpr (FS) {
                        w.x += s_tB[2 * (lo + k)];
                        w.y += s_tB[2 * (lo + k) + 1];
                    }
                    *reinterpret_cast<R2*>(dst_g + (col + (uint32_t)(2 * (lo + k)))) = w;
                }
            }
            if (top_seg) dst_g[col + (uint32_t)nsub] = FS ? vlast + s_tB[nsub] : vlast;
        };
        // per-g values of one stream (pairs at my points, the TOA value
        // alone), as fluxes in the flux-state variant
        auto store = [&](const R (&v)[K], R vtop, R* __restrict__ dst_g) {
            if (!colok) return;
#pragma unroll
            for (int p = 0; p < KH; ++p) {
                if (2 * p < cnt) {
                    R2 w;
                    w.x = v[2 * p];
                    w.y = v[2 * p + 1];
                    if constexpr (FS) {
                        w.x += s_tB[lo + 2 * p];
                        w.y += s_tB[lo + 2 * p + 1];
                    }
                    *reinterpret_cast<R2*>(dst_g + (col + (uint32_t)(lo + 2 * p))) = w;
                }
            }
            if (top_seg) dst_g[col + (uint32_t)nsub] = FS ? vtop + s_tB[nsub] : vtop;
        };

        // One scattering pass: downward sweep (top -> bottom), then upward
        // (bottom -> top).  fu[k] holds sublayer k's stream state in turn:
        // F_up at its lower point, the downward map offset c F_up - sig, the
        // upward map offset c F_dn + sig (in the last pass F_dn first), and
        // the new F_up.
        R ftoa = (R)0;
        auto one_pass = [&](auto last_tag) {
            constexpr bool LAST = decltype(last_tag)::value;
            R MB = (R)0;
            // downward offsets c F_up - sig (isothermal grid: the shift a sg)
#pragma unroll
            for (int k = 0; k < K; ++k) fu[k] = cc[k] * fu[k] - (ISO ? ca[k] * sg[k] : sg[k]);
#pragma unroll
            for (int k = K - 1; k >= 0; --k) MB = ca[k] * MB + fu[k];
            if (seg == L - 1) MB = ftop_fold + MB;
            if constexpr (PRECOMP) {  // suffix scan towards the BOA
                MB = scan_down_step<L, 0>(MB, mdn[0]);
                MB = scan_down_step<L, 1>(MB, mdn[1]);
                MB = scan_down_step<L, 2>(MB, mdn[2]);
                MB = scan_down_step<L, 3>(MB, mdn[3]);
                if constexpr (LOG2L > 4) MB = scan_down_step<L, 4>(MB, mdn[4 < LOG2L ? 4 : 0]);
                if constexpr (LOG2L > 5) MB = scan_down_step<L, 5>(MB, mdn[5 < LOG2L ? 5 : 0]);
            } else {
                R MA = (seg == L - 1) ? (R)0 : pseg;
                scan_down_full<L>(MA, MB, seg);
            }
            R x = next_lane<L>(MB);  // F_dn at my segment's top point
            if (seg == L - 1) x = Ftop;
            if constexpr (!LAST) {
                // fu[k] then takes the upward sweep's offset c F_dn + sig
#pragma unroll
                for (int k = K - 1; k >= 0; --k) {
                    const R xn = ca[k] * x + fu[k];
                    fu[k] = ISO ? cc[k] * (x - sg[k]) + sg[k] : cc[k] * x + sg[k];  // (1 - c) sg on that grid
                    x = xn;
                }
            } else {
                // keep F_dn for the outputs, then form the offsets from it
                const R xtop = x;
#pragma unroll
                for (int k = K - 1; k >= 0; --k) {
                    x = ca[k] * x + fu[k];
                    fu[k] = x;
                }
                if constexpr (ISO) {
                    emit_iso(fu, xtop, s_pd);
                    if (Fd_all) store_iso(fu, xtop, Fd_all + gcol);
                } else {
                    emit(fu, Ftop, s_pd);
                    if (Fd_all) store(fu, Ftop, Fd_all + gcol);
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const R xu = k + 1 < K ? fu[k + 1 < K ? k + 1 : k] : xtop;
                    fu[k] = ISO ? cc[k] * (xu - sg[k]) + sg[k] : cc[k] * xu + sg[k];
                }
            }
            // the BOA condition F_up(0) = F_dn(0) + F_int lives in segment 0
            const R y0 = x + Fint;
            MB = (R)0;
#pragma unroll
            for (int k = 0; k < K; ++k) MB = ca[k] * MB + fu[k];
            if (seg == 0) MB = pseg * y0 + MB;
            if constexpr (PRECOMP) {  // prefix scan towards the TOA
                MB = scan_up_step<L, 0>(MB, mup[0]);
                MB = scan_up_step<L, 1>(MB, mup[1]);
                MB = scan_up_step<L, 2>(MB, mup[2]);
                MB = scan_up_step<L, 3>(MB, mup[3]);
                if constexpr (LOG2L > 4) MB = scan_up_step<L, 4>(MB, mup[4 < LOG2L ? 4 : 0]);
                if constexpr (LOG2L > 5) MB = scan_up_step<L, 5>(MB, mup[5 < LOG2L ? 5 : 0]);
            } else {
                R MA = (seg == 0) ? (R)0 : pseg;
                scan_up_full<L>(MA, MB, seg);
            }
            R y = prev_lane<L>(MB);  // F_up at my segment's bottom point
            if (seg == 0) y = y0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const R yn = ca[k] * y + fu[k];
                fu[k] = y;
                y = yn;
            }
            ftoa = y;
        };
        for (int pass = 0; pass < A.n_scat; ++pass) one_pass(std::false_type{});
        one_pass(std::true_type{});

        // ---- outputs: upward fluxes (warm start of the next call) and their
        // Gauss sums
        if constexpr (ISO) {
            emit_iso(fu, ftoa, s_pu);
            store_iso(fu, ftoa, fu_g);
        } else {
            emit(fu, ftoa, s_pu);
            store(fu, ftoa, fu_g);
        }
      }  // groups
        // ---- this wave's Gauss sums over its groups (one partial per point),
        // stored coalesced
        __syncthreads();
        const int64_t poff = pb * A.wpb_stride + (int64_t)part * npt;
        for (int i = lane; i < npt; i += 64) {
            part_up[poff + i] = s_pu[i];
            part_dn[poff + i] = s_pd[i];
        }
        __syncthreads();  // the next item restages the LDS arrays
    }
}

// LDS bytes of one sweep workgroup of shape (K, L).
static size_t sweep_lds(int K, int L, size_t rbytes, bool iso = false, bool fs = false) {
    return (size_t)SweepLds(K * L, iso, fs).total * rbytes;
}

// Occupancy hint (waves per SIMD) so the register arrays fit without spills
// (the isothermal grid's two output points per slot take one step less).
template <int K, int L, bool F64, bool ISO = false>
constexpr int sweep_occ() {
    if (L == 64) return 1;  // the long-column shape: whole register file, large LDS staging
    const int occ = F64 ? ((K <= 4) ? 4 : ((K <= 8) ? 3 : (K <= 14 ? 2 : 1))) : (K <= 8 ? 4 : (K <= 14 ? 3 : 2));
    return (ISO && occ > 1) ? occ - 1 : occ;
}

// Dynamic LDS beyond 64 KB (the FP64 long-column shape) is declared to the
// runtime once per instantiation before its first launch.
template <typename Kern>
static hipError_t allow_lds(Kern kern, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <int K, int L, bool RAY, bool ISO, bool FS>
static hipError_t launch_kprf(const SweepArgs& a, bool mixed, int grid, hipStream_t s) {
    if (mixed) {
        auto kern = sweep_kernel<K, L, float, sweep_occ<K, L, false, ISO>(), RAY, ISO, FS>;
        static const hipError_t ok = allow_lds(kern, sweep_lds(K, L, 4, ISO, FS));
        if (ok != hipSuccess) return ok;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64), sweep_lds(K, L, 4, ISO, FS), s, a);
    } else {
        auto kern = sweep_kernel<K, L, double, sweep_occ<K, L, true, ISO>(), RAY, ISO, FS>;
        static const hipError_t ok = allow_lds(kern, sweep_lds(K, L, 8, ISO, FS));
        if (ok != hipSuccess) return ok;
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64), sweep_lds(K, L, 8, ISO, FS), s, a);
    }
    return hipGetLastError();
}

template <int K, int L, bool RAY, bool ISO>
static hipError_t launch_kpr(const SweepArgs& a, bool mixed, int grid, hipStream_t s) {
    if (a.flux_state) return launch_kprf<K, L, RAY, ISO, true>(a, mixed, grid, s);
    return launch_kprf<K, L, RAY, ISO, false>(a, mixed, grid, s);
}

template <int K, int L>
static hipError_t launch_kp(const SweepArgs& a, bool mixed, int grid, hipStream_t s) {
    if (a.iso_grid) return launch_kpr<K, L, false, true>(a, mixed, grid, s);
    if (a.inv_mbar > 0.0) return launch_kpr<K, L, true, false>(a, mixed, grid, s);
    return launch_kpr<K, L, false, false>(a, mixed, grid, s);
}

template <int K>
static hipError_t launch_kl(const SweepArgs& a, int L, bool mixed, int grid, hipStream_t s) {
    if (L == 16) return launch_kp<K, 16>(a, mixed, grid, s);
    if (L == 32) return launch_kp<K, 32>(a, mixed, grid, s);
    if constexpr (K == kLongK) {
        if (L == 64) return launch_kp<K, 64>(a, mixed, grid, s);
    }
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
