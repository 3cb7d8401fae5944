// api.hip -- the C ABI of libhelios: argument validation, workspace layout,
// launch shapes, and dispatch to the kernels.  See include/helios.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "helios_internal.hpp"

using namespace helios;

namespace {

thread_local char g_err[512] = "";
thread_local hipEvent_t g_ev_before = nullptr, g_ev_after = nullptr;

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    return fail(HELIOS_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

// Size classes of the batched sweep, by layer count: atmospheres of one
// class share a sweep launch and its shape, so a short atmosphere does not
// run with the lane count of the deepest one.
constexpr int kNumClasses = 6;
constexpr int kClassNHi[kNumClasses] = {32, 64, 112, 208, 400, HELIOS_MAX_LAYERS};
static_assert(kNumClasses <= kMaxClasses, "class table");

int class_of(int n) {
    for (int k = 0; k < kNumClasses; ++k)
        if (n <= kClassNHi[k]) return k;
    return kNumClasses - 1;
}
int class_nlo(int k) { return k == 0 ? 0 : kClassNHi[k - 1] + 1; }

// Host view of the batch sizes.
struct Sizes {
    int64_t total_n = 0, total_pt = 0, total_bin = 0, total_lb = 0, total_pb = 0, total_cell = 0;
    int n_max = 0, npt_max = 0, nb_max = 0, n_atm = 0;
    // per class: deepest member, bin range [bin_lo, bin_hi) spanning its members,
    // and the member with the most bins among the deepest (autotuner sample)
    int cls_nmax[kNumClasses] = {};
    int64_t cls_bin_lo[kNumClasses] = {}, cls_bin_hi[kNumClasses] = {}, cls_bins[kNumClasses] = {};
    int cls_rep[kNumClasses] = {};
};

int check_atm(const helios_atm* atm, Sizes& z) {
    if (!atm) return fail(HELIOS_EINVAL, "atm is NULL");
    if (atm->n_atm < 1) return fail(HELIOS_EINVAL, "n_atm = %d must be >= 1", atm->n_atm);
    if (atm->n_g < 1 || atm->n_g > HELIOS_MAX_NG)
        return fail(HELIOS_EINVAL, "n_g = %d outside 1..%d", atm->n_g, HELIOS_MAX_NG);
    if (!atm->n_layer_h || !atm->n_bin_h || !atm->n_layer || !atm->n_bin || !atm->lay_off || !atm->pt_off ||
        !atm->bin_off || !atm->lb_off || !atm->pb_off || !atm->cell_off || !atm->bin_index || !atm->bin_index_h ||
        !atm->lambda_c || !atm->dlambda || !atm->P_c || !atm->P_pt || !atm->grav || !atm->T_star ||
        !atm->T_irr || !atm->T_int)
        return fail(HELIOS_EINVAL, "a helios_atm array pointer is NULL");
    for (int a = 0; a < atm->n_atm; ++a) {
        int n = atm->n_layer_h[a], nb = atm->n_bin_h[a];
        if (n < 2 || n > HELIOS_MAX_LAYERS)
            return fail(HELIOS_ESHAPE, "atmosphere %d: n_layer = %d outside 2..%d", a, n, HELIOS_MAX_LAYERS);
        if (nb < 1) return fail(HELIOS_ESHAPE, "atmosphere %d: n_bin = %d must be >= 1", a, nb);
        int npt = 2 * n + 1;
        z.total_n += n;
        z.total_pt += npt;
        z.total_bin += nb;
        z.total_lb += (int64_t)nb * n;
        z.total_pb += (int64_t)nb * npt;
        z.total_cell += (int64_t)nb * atm->n_g * col_stride(n);
        z.n_max = std::max(z.n_max, n);
        z.npt_max = std::max(z.npt_max, npt);
        z.nb_max = std::max(z.nb_max, nb);
    }
    z.n_atm = atm->n_atm;
    int64_t b0 = 0;
    for (int a = 0; a < atm->n_atm; ++a) {
        int n = atm->n_layer_h[a], nb = atm->n_bin_h[a], k = class_of(n);
        if (z.cls_nmax[k] == 0) {
            z.cls_bin_lo[k] = b0;
            z.cls_rep[k] = a;
        }
        int r = z.cls_rep[k];
        if (n > z.cls_nmax[k] || (n == atm->n_layer_h[r] && nb > atm->n_bin_h[r])) z.cls_rep[k] = a;
        z.cls_nmax[k] = std::max(z.cls_nmax[k], n);
        z.cls_bins[k] += nb;
        b0 += nb;
        z.cls_bin_hi[k] = b0;
    }
    return HELIOS_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct WsLayout {
    size_t B, F_top, F_int, gw, bin_atm, part_up, part_dn, chunk, bnd_part, total;
    int bnd_maxch;
};

// Waves per bin for L lanes per column: each wave holds 64/L columns.
int waves_per_bin(int n_g, int L) { return (n_g + (64 / L) - 1) / (64 / L); }

// A sweep launch gives each bin P waves (each takes a contiguous share of the
// bin's column groups and leaves its own partial).  P = 1 moves the least
// data; small launches may fill the device better with P > 1, which the
// autotuner can choose.  The workspace holds up to waves_per_bin(n_g, 32)
// partials per (bin, point) for batches of at most kSplitBins bins, one for
// larger ones.
constexpr int64_t kSplitBins = 65536;
int parts_stride(const Sizes& z, int n_g) {
    return z.total_bin <= kSplitBins ? waves_per_bin(n_g, 32) : 1;
}

// Gauss partials per (bin, point) and direction, sized for doubles (the
// mixed path stores floats in the first half), so the layout does not depend
// on the precision or the sweep shape.
WsLayout ws_layout(const Sizes& z, int n_g, bool /*mixed*/) {
    WsLayout w;
    const size_t wpb = (size_t)parts_stride(z, n_g);
    const int cb = bol_chunk_bins(z.total_bin);
    const size_t n_chunk = (size_t)((z.nb_max + cb - 1) / cb);
    w.B = 0;  // Planck values in FP64 for both precisions
    w.F_top = align256(w.B + (size_t)z.total_pb * sizeof(double));
    w.F_int = align256(w.F_top + (size_t)z.total_bin * sizeof(double));
    w.gw = align256(w.F_int + (size_t)z.total_bin * sizeof(double));
    w.bin_atm = align256(w.gw + HELIOS_MAX_NG * sizeof(double));
    w.part_up = align256(w.bin_atm + (size_t)z.total_bin * sizeof(int32_t));
    w.part_dn = align256(w.part_up + (size_t)z.total_pb * wpb * 8);
    w.chunk = align256(w.part_dn + (size_t)z.total_pb * wpb * 8);
    w.bnd_maxch = (z.nb_max + kBndChunk - 1) / kBndChunk;
    w.bnd_part = align256(w.chunk + (size_t)z.total_pt * n_chunk * kBolQ * sizeof(double));
    w.total = align256(w.bnd_part + (size_t)z.n_atm * w.bnd_maxch * sizeof(double));
    return w;
}

// Gauss-Legendre rule on [0,1] (Sec. 2.3): weights w_g/2 at the nodes
// (1 + y_g)/2, y_g the roots of P_n, by Newton's method on the Legendre
// three-term recurrence; nodes ascending.  Computed once per n on the host.
void legendre(int n, double y, double& pn, double& dpn) {
    double a = 1.0, b = y;  // P_0, P_1
    for (int k = 2; k <= n; ++k) {
        double c = ((2.0 * k - 1.0) * y * b - (k - 1.0) * a) / k;
        a = b;
        b = c;
    }
    if (n == 1) a = 1.0;
    pn = b;
    dpn = n * (y * b - a) / (y * y - 1.0);
}

const GaussTable& gauss_table(int n) {
    static GaussTable tab[HELIOS_MAX_NG + 1];
    static std::once_flag once;
    std::call_once(once, [] {
        for (int m = 1; m <= HELIOS_MAX_NG; ++m) {
            memset(tab[m].w, 0, sizeof(tab[m].w));
            for (int i = 0; i < m; ++i) {
                double y = cos(kPi * (i + 0.75) / (m + 0.5)), pn = 0.0, dpn = 1.0;
                for (int it = 0; it < 100; ++it) {
                    legendre(m, y, pn, dpn);
                    double step = pn / dpn;
                    y -= step;
                    if (fabs(step) < 1e-16) break;
                }
                legendre(m, y, pn, dpn);
                tab[m].w[m - 1 - i] = 1.0 / ((1.0 - y * y) * dpn * dpn);
            }
        }
    });
    return tab[n];
}

// Sum of the Gauss weights in g order (the bin sum scales B by 2 pi eps times it).
double gauss_weight_sum(int n) {
    const GaussTable& t = gauss_table(n);
    double w = 0.0;
    for (int g = 0; g < n; ++g) w += t.w[g];
    return w;
}

int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    return (v && *v) ? atoi(v) : dflt;
}

// Sweep shape: K sublayers per lane (compiled instantiations) and L lanes per
// column.  Default: the smallest register footprint that fits the deepest
// atmosphere with L = 16, else L = 32.
struct SweepShape {
    int K, L;
    int P = 1;  // waves per bin
};

bool k_allowed(int K, bool /*mixed*/) {
    for (int i = 0; i < kNumSweepK; ++i)
        if (kSweepK[i] == K) return true;
    return false;
}

// Instantiated shapes: every K with L = 16 and 32, and the long-column
// shape (kLongK, 64).
bool shape_allowed(int K, int L, bool mixed) {
    if (!k_allowed(K, mixed)) return false;
    return L == 16 || L == 32 || (L == 64 && K == kLongK);
}

// Shapes chosen by helios_autotune, per (precision, n_g, size class).
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, SweepShape> g_tuned;  // (mixed, n_g, class, isothermal grid)

int default_shape(int nsub_max, bool mixed, SweepShape& sh) {
    // fewest sublayers per lane first (smallest register footprint), then
    // the narrower column
    for (int i = 0; i < kNumSweepK; ++i) {
        for (int L : {16, 32, 64}) {
            int K = kSweepK[i];
            if (!shape_allowed(K, L, mixed)) continue;
            if (K * L >= nsub_max) {
                sh = {K, L};
                return HELIOS_OK;
            }
        }
    }
    return fail(HELIOS_ESHAPE, "no sweep shape holds %d sublayers", nsub_max);
}

// Shape of class k (deepest member nsub_max sublayers): an environment
// override (HELIOS_SWEEP_K / HELIOS_SWEEP_L / HELIOS_SWEEP_P, for measurement), else the
// autotuned one, else the default.
int pick_shape(int k, int nsub_max, int n_g, bool mixed, SweepShape& sh, bool iso_grid = false) {
    int fk = env_int("HELIOS_SWEEP_K", 0), fl = env_int("HELIOS_SWEEP_L", 0);
    if (fk || fl) {
        if (!shape_allowed(fk, fl, mixed))
            return fail(HELIOS_EINVAL, "HELIOS_SWEEP_K/L = %d/%d not available", fk, fl);
        if (fk * fl < nsub_max) return fail(HELIOS_ESHAPE, "K*L = %d < %d sublayers", fk * fl, nsub_max);
        sh = {fk, fl, std::max(1, env_int("HELIOS_SWEEP_P", 1))};
        return HELIOS_OK;
    }
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tuned.find({mixed ? 1 : 0, n_g, k, iso_grid ? 1 : 0});
        if (it != g_tuned.end() && it->second.K * it->second.L >= nsub_max) {
            sh = it->second;
            return HELIOS_OK;
        }
    }
    return default_shape(nsub_max, mixed, sh);
}

// Everything one flux call needs after validation.
struct FluxPlan {
    Sizes z;
    WsLayout w;
    bool mixed;
    bool flux_state;  // the per-g arrays hold fluxes (HELIOS_STATE_FLUX)
    SweepShape sh[kNumClasses];
};

// Splits a flux call's prec argument into the element type and the per-g
// convention; false for unknown bits.
bool split_prec(int prec_arg, bool& mixed, bool& flux_state) {
    const int base = prec_arg & 0xff, flags = prec_arg & ~0xff;
    if ((base != HELIOS_FP64 && base != HELIOS_MIXED) || (flags & ~HELIOS_STATE_FLUX)) return false;
    mixed = base == HELIOS_MIXED;
    flux_state = (flags & HELIOS_STATE_FLUX) != 0;
    return true;
}

int plan_flux(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0, const double* g0,
              int32_t n_scat, double D, const void* F_up_g, const void* ws, size_t ws_bytes, helios_prec prec,
              FluxPlan& p, bool need_optics = true, bool iso_grid = false) {
    int rc = check_atm(atm, p.z);
    if (rc) return rc;
    if (!kappa || !T_pt || (need_optics && (!w0 || !g0)) || !F_up_g || !ws)
        return fail(HELIOS_EINVAL, "flux: NULL argument");
    if (!split_prec((int)prec, p.mixed, p.flux_state))
        return fail(HELIOS_EINVAL, "unknown precision / state flags 0x%x", (int)prec);
    if (n_scat < 0 || n_scat > 100000) return fail(HELIOS_EINVAL, "n_scat = %d", n_scat);
    if (!(D > 0.0)) return fail(HELIOS_EINVAL, "D = %g must be > 0", D);
    p.w = ws_layout(p.z, atm->n_g, p.mixed);
    if (ws_bytes < p.w.total)
        return fail(HELIOS_EWORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, p.w.total);
    for (int k = 0; k < kNumClasses; ++k) {
        p.sh[k] = {0, 0};
        if (p.z.cls_nmax[k] == 0) continue;
        // slots per column: sublayers, or layers on the isothermal-layer grid
        rc = pick_shape(k, (iso_grid ? 1 : 2) * p.z.cls_nmax[k], atm->n_g, p.mixed, p.sh[k], iso_grid);
        if (rc) return rc;
    }
    return HELIOS_OK;
}

// Waves per bin of class k's launch (never more than the workspace holds or
// the bin has column groups).
int class_parts(const FluxPlan& p, int k, int n_g) {
    return std::max(1, std::min({p.sh[k].P, parts_stride(p.z, n_g), waves_per_bin(n_g, p.sh[k].L)}));
}

SweepArgs sweep_args(const helios_atm* atm, const FluxPlan& p, const void* kappa, const double* w0,
                     const double* g0, int32_t n_scat, double D, void* F_up_g, void* F_dn_g, char* wsb) {
    SweepArgs A;
    A.n_layer = atm->n_layer;
    A.pt_off = atm->pt_off;
    A.bin_off = atm->bin_off;
    A.lb_off = atm->lb_off;
    A.pb_off = atm->pb_off;
    A.cell_off = atm->cell_off;
    A.P_pt = atm->P_pt;
    A.grav = atm->grav;
    A.kappa = kappa;
    A.B = wsb + p.w.B;
    A.F_top = (double*)(wsb + p.w.F_top);
    A.F_int = (double*)(wsb + p.w.F_int);
    A.w0 = w0;
    A.g0 = g0;
    A.F_up_g = F_up_g;
    A.F_dn_g = F_dn_g;
    A.part_up = wsb + p.w.part_up;
    A.part_dn = wsb + p.w.part_dn;
    A.gw = (double*)(wsb + p.w.gw);
    A.bnd_part = (const double*)(wsb + p.w.bnd_part);
    A.T_int = atm->T_int;
    A.bnd_maxch = p.w.bnd_maxch;
    A.bin_atm = (const int32_t*)(wsb + p.w.bin_atm);
    A.status = atm->status;
    A.n_atm = atm->n_atm;
    A.n_g = atm->n_g;
    A.wpb_stride = parts_stride(p.z, atm->n_g);
    A.n_scat = n_scat;
    A.npt_max = p.z.npt_max;
    A.iso_grid = 0;
    A.flux_state = p.flux_state ? 1 : 0;
    A.D = D;
    A.lambda_c = atm->lambda_c;
    A.inv_mbar = 0.0;
    return A;
}

// One sweep launch for class k over bins [b_lo, b_hi): one wave per bin,
// looping over the bin's groups of 64/L columns.
hipError_t sweep_class(SweepArgs A, const SweepShape& sh, int k, int64_t b_lo, int64_t b_hi, int parts,
                       bool mixed, hipStream_t s) {
    A.wpb = waves_per_bin(A.n_g, sh.L);  // column groups per bin
    A.parts = parts;
    A.n_lo = class_nlo(k);
    A.n_hi = kClassNHi[k];
    A.npt_max = std::min(A.npt_max, 2 * A.n_hi + 1);  // LDS sized for the class
    A.w_begin = b_lo * parts;
    A.w_end = b_hi * parts;
    int64_t grid64 = A.w_end - A.w_begin;
    int cap = env_int("HELIOS_SWEEP_GRID", 0);
    if (cap > 0 && grid64 > cap) grid64 = cap;
    if (grid64 > 0x7fffffff) grid64 = 0x7fffffff;  // the kernel strides over the rest
    return launch_sweep(A, sh.K, sh.L, mixed, (int)grid64, s);
}

hipError_t launch_sources(const helios_atm* atm, const FluxPlan& p, const double* T_pt, char* wsb,
                          hipStream_t s, bool iso_grid = false) {
    SourceArgs sa;
    sa.iso_grid = iso_grid ? 1 : 0;
    sa.B = (double*)(wsb + p.w.B);
    sa.F_top = (double*)(wsb + p.w.F_top);
    sa.F_int = (double*)(wsb + p.w.F_int);
    sa.gw = (double*)(wsb + p.w.gw);
    sa.bin_atm = (int32_t*)(wsb + p.w.bin_atm);
    sa.bnd_part = (double*)(wsb + p.w.bnd_part);
    sa.bnd_maxch = p.w.bnd_maxch;
    sa.nb_max = p.z.nb_max;
    sa.npt_max = p.z.npt_max;
    sa.total_bin = p.z.total_bin;
    sa.chunk = (double*)(wsb + p.w.chunk);
    sa.total_pt = p.z.total_pt;
    sa.chunk_bins = bol_chunk_bins(p.z.total_bin);
    return launch_planck(atm, T_pt, sa, gauss_table(atm->n_g), s);
}

// ------------------------------------------------------ warm-start network
struct NetLayout {
    int nl;                        // affine layers (hidden + output)
    int in[9], out[9];
    size_t offW[9], offb[9], count;
};

bool net_layout(const helios_mlp* net, NetLayout& L) {
    if (!net || net->n_in < 1 || net->n_in > 64 || net->n_hidden < 1 || net->n_hidden > 1024 ||
        net->n_hidden_layers < 1 || net->n_hidden_layers > 8 || net->n_out < 1 || net->n_out > kMaxNetOut)
        return false;
    L.nl = net->n_hidden_layers + 1;
    size_t off = 0;
    for (int l = 0; l < L.nl; ++l) {
        L.in[l] = l == 0 ? net->n_in : net->n_hidden;
        L.out[l] = l == L.nl - 1 ? net->n_out : net->n_hidden;
        L.offW[l] = off;
        off += (size_t)L.in[l] * L.out[l];
        L.offb[l] = off;
        off += (size_t)L.out[l];
    }
    L.count = off;
    return true;
}

struct NetWs {
    size_t X0, Z, A, Y, dY, D0, D1, partial, T, total;  // Z, A: n_hidden_layers consecutive [B][H] blocks
};
constexpr int kLossBlocks = 512;

NetWs net_ws(const helios_mlp* net, int64_t B) {
    NetWs w;
    const size_t H = (size_t)net->n_hidden, nh = (size_t)net->n_hidden_layers, no = (size_t)net->n_out;
    w.X0 = 0;
    w.Z = align256(w.X0 + (size_t)B * net->n_in * 2);
    w.A = align256(w.Z + nh * B * H * 4);
    w.Y = align256(w.A + nh * B * H * 2);
    w.dY = align256(w.Y + (size_t)B * no * 4);
    w.D0 = align256(w.dY + (size_t)B * no * 2);
    w.D1 = align256(w.D0 + (size_t)B * H * 2);
    w.partial = align256(w.D1 + (size_t)B * H * 2);
    w.T = align256(w.partial + kLossBlocks * sizeof(double));
    w.total = align256(w.T + (size_t)B * no * 4);
    return w;
}

int check_net(const helios_mlp* net, NetLayout& L, bool training) {
    if (!net_layout(net, L)) return fail(HELIOS_EINVAL, "helios_mlp: dimensions outside the limits");
    if (!net->params || !net->params_bf16 || !net->in_shift || !net->in_scale || !net->out_shift || !net->out_scale)
        return fail(HELIOS_EINVAL, "helios_mlp: NULL array");
    if (training && (!net->adam_m || !net->adam_v)) return fail(HELIOS_EINVAL, "helios_mlp: no Adam moments");
    return HELIOS_OK;
}

GemmArgs gemm(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbn, int64_t sbk, int M, int N,
              int K) {
    GemmArgs g = {};
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbn = sbn;
    g.sbk = sbk;
    g.M = M;
    g.N = N;
    g.K = K;
    return g;
}

// Forward pass of B rows: X0, then Z_l / A_l per hidden layer, then the
// output layer into out (normalised y, or T when scaled).
hipError_t net_forward(const helios_mlp* net, const NetLayout& L, const NetWs& w, char* wsb, const float* x, int B,
                       float* out, bool scaled, hipStream_t s) {
    const int H = net->n_hidden;
    uint16_t* X0 = (uint16_t*)(wsb + w.X0);
    hipError_t e = launch_mlp_input(x, (int64_t)B * net->n_in, net->n_in, net->in_shift, net->in_scale, X0, s);
    if (e != hipSuccess) return e;
    const uint16_t* h = X0;
    for (int l = 0; l < L.nl; ++l) {
        GemmArgs g = gemm(h, L.in[l], 1, net->params_bf16 + L.offW[l], L.in[l], 1, B, L.out[l], L.in[l]);
        g.bias = net->params + L.offb[l];
        if (l < L.nl - 1) {
            g.out_f = (float*)(wsb + w.Z) + (size_t)l * B * H;
            g.ld_f = H;
            g.out_b = (uint16_t*)(wsb + w.A) + (size_t)l * B * H;
            g.ld_b = H;
            e = launch_gemm(g, kEpiGelu, s);
            h = g.out_b;
        } else {
            g.out_f = out;
            g.ld_f = net->n_out;
            if (scaled) {
                g.oshift = net->out_shift;
                g.oscale = net->out_scale;
            }
            e = launch_gemm(g, kEpiLinear, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The two-stream solve of helios_flux on either grid: iso_grid selects the
// isothermal-layer grid (the Planck kernel's and the sweep's flag);
// inv_mbar > 0 adds H2 Rayleigh scattering (w0, g0 then unused).
int flux_impl(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0, const double* g0,
              int32_t n_scat, double D, void* F_up_g, void* F_dn_g, double* F_up_bin, double* F_dn_bin,
              double* F_bol, void* ws, size_t ws_bytes, helios_prec prec, void* stream, bool iso_grid,
              double inv_mbar, const char* name) {
    FluxPlan p;
    int rc = plan_flux(atm, kappa, T_pt, w0, g0, n_scat, D, F_up_g, ws, ws_bytes, prec, p, !(inv_mbar > 0.0),
                       iso_grid);
    if (rc) return rc;
    if (!F_bol) return fail(HELIOS_EINVAL, "%s: NULL argument", name);
    hipStream_t s = (hipStream_t)stream;
    char* wsb = (char*)ws;
    hipError_t e = launch_sources(atm, p, T_pt, wsb, s, iso_grid);
    if (e != hipSuccess) return hip_fail(e, name);

    SweepArgs A = sweep_args(atm, p, kappa, w0, g0, n_scat, D, F_up_g, F_dn_g, wsb);
    A.iso_grid = iso_grid ? 1 : 0;
    A.inv_mbar = inv_mbar;
    A.flux_state = p.flux_state ? 1 : 0;  // the sweep's flux-state variant converts as it reads and stores
    if (g_ev_before && g_ev_after) {
        e = hipEventRecord(g_ev_before, s);
        if (e != hipSuccess) return hip_fail(e, name);
    }
    for (int k = 0; k < kNumClasses; ++k) {
        if (p.z.cls_nmax[k] == 0) continue;
        e = sweep_class(A, p.sh[k], k, p.z.cls_bin_lo[k], p.z.cls_bin_hi[k], class_parts(p, k, atm->n_g), p.mixed,
                        s);
        if (e != hipSuccess) return hip_fail(e, name);
    }
    if (g_ev_before && g_ev_after) {
        e = hipEventRecord(g_ev_after, s);
        if (e != hipSuccess) return hip_fail(e, name);
    }
    BolArgs Bo;
    Bo.atm = *atm;
    Bo.part_up = A.part_up;
    Bo.part_dn = A.part_dn;
    Bo.F_up_bin = F_up_bin;
    Bo.F_dn_bin = F_dn_bin;
    Bo.chunk = (double*)(wsb + p.w.chunk);
    Bo.total_pt = p.z.total_pt;
    Bo.F_bol = F_bol;
    Bo.B = (const double*)(wsb + p.w.B);
    Bo.gw = (const double*)(wsb + p.w.gw);
    Bo.tpe = 2.0 * kPi / D;
    Bo.tw = Bo.tpe * gauss_weight_sum(atm->n_g);
    Bo.wpb_stride = A.wpb_stride;
    Bo.chunk_bins = bol_chunk_bins(p.z.total_bin);
    Bo.n_chunk = (p.z.nb_max + Bo.chunk_bins - 1) / Bo.chunk_bins;
    Bo.mixed = p.mixed ? 1 : 0;
    Bo.n_cls = kNumClasses;
    for (int k = 0; k < kNumClasses; ++k) {
        Bo.cls_nhi[k] = kClassNHi[k];
        Bo.cls_wpb[k] = p.sh[k].L ? class_parts(p, k, atm->n_g) : 1;  // partials per (bin, point)
    }
    e = launch_bolometric(Bo, p.z.npt_max, p.z.nb_max, p.z.total_pt, s);
    if (e != hipSuccess) return hip_fail(e, name);
    g_err[0] = 0;
    return HELIOS_OK;
}

// Workspace of helios_flux_noalloc, for callers that cannot allocate device
// memory: a fixed array in the library's code object, one copy per device,
// held until the process ends.  Host code must not use the array's name as
// an address: each device's copy is looked up once (hipGetSymbolAddress, with
// that device current) and only that pointer is passed on.
constexpr size_t kScratchBytes = HELIOS_NOALLOC_WS_BYTES;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
void* g_scratch_ptr[kScratchDevices] = {};
std::mutex g_scratch_mu;

int scratch_for_current_device(void** out, const char* name) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, name);
    if (dev < 0 || dev >= kScratchDevices) return fail(HELIOS_EDEVICE, "%s: device %d beyond %d", name, dev,
                                                       kScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, name);
        if (!ptr) return fail(HELIOS_EDEVICE, "%s: no device address for the scratch array", name);
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HELIOS_OK;
}

}  // namespace

extern "C" {

const char* helios_last_error(void) { return g_err; }

int helios_set_sweep_events(void* before, void* after) {
    if ((before == nullptr) != (after == nullptr))
        return fail(HELIOS_EINVAL, "helios_set_sweep_events: give both events or neither");
    g_ev_before = (hipEvent_t)before;
    g_ev_after = (hipEvent_t)after;
    return HELIOS_OK;
}

int32_t helios_version(void) { return 1; }

int helios_grid(const helios_atm* atm, void* stream) {
    Sizes z;
    int rc = check_atm(atm, z);
    if (rc) return rc;
    hipError_t e = launch_grid(atm, z.total_pt, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "helios_grid");
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_profile(const helios_atm* atm, const double* T_c, double* T_pt, void* stream) {
    Sizes z;
    int rc = check_atm(atm, z);
    if (rc) return rc;
    if (!T_c || !T_pt) return fail(HELIOS_EINVAL, "helios_profile: T_c or T_pt is NULL");
    hipError_t e = launch_profile(atm, z.total_pt, T_c, T_pt, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "helios_profile");
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_mix_opacity(const helios_atm* atm, const helios_ktab* kt, const double* T_pt, const double* vmr,
                       void* kappa, helios_prec prec, void* stream) {
    Sizes z;
    int rc = check_atm(atm, z);
    if (rc) return rc;
    if (!kt || !T_pt || !vmr || !kappa) return fail(HELIOS_EINVAL, "helios_mix_opacity: NULL argument");
    if (prec != HELIOS_FP64 && prec != HELIOS_MIXED) return fail(HELIOS_EINVAL, "unknown precision %d", prec);
    if (kt->mode != HELIOS_KTAB_TABLE && kt->mode != HELIOS_KTAB_POWERLAW)
        return fail(HELIOS_EINVAL, "unknown k-table mode %d", kt->mode);
    if (kt->n_species < 1 || kt->n_species > HELIOS_MAX_SPECIES)
        return fail(HELIOS_EINVAL, "n_species = %d outside 1..%d", kt->n_species, HELIOS_MAX_SPECIES);
    if (kt->n_g != atm->n_g) return fail(HELIOS_ESHAPE, "table n_g %d != batch n_g %d", kt->n_g, atm->n_g);
    if (kt->n_bin_table < 1) return fail(HELIOS_ESHAPE, "n_bin_table = %d", kt->n_bin_table);
    for (int64_t b = 0; b < z.total_bin; ++b)  // the table lookup (Sec. 2.3) needs a bin of the table
        if (atm->bin_index_h[b] < 0 || atm->bin_index_h[b] >= kt->n_bin_table)
            return fail(HELIOS_ESHAPE, "bin %lld: bin_index %d outside the table's 0..%d", (long long)b,
                        atm->bin_index_h[b], kt->n_bin_table - 1);
    if (!kt->species_mass || !(kt->mmw > 0.0)) return fail(HELIOS_EINVAL, "species masses / mmw missing");
    if (kt->mode == HELIOS_KTAB_TABLE) {
        if (!kt->k) return fail(HELIOS_EINVAL, "TABLE mode without k");
        if (kt->n_T < 2 || kt->n_P < 2) return fail(HELIOS_ESHAPE, "table needs >= 2 nodes per axis");
        if (!(kt->T_step > 0.0) || !(kt->logP_step > 0.0)) return fail(HELIOS_EINVAL, "non-positive table step");
    } else {
        if (!kt->k0) return fail(HELIOS_EINVAL, "POWERLAW mode without k0");
        if (!(kt->P_ref > 0.0) || !(kt->T_ref > 0.0)) return fail(HELIOS_EINVAL, "non-positive P_ref/T_ref");
    }
    hipError_t e = launch_mix(atm, kt, T_pt, vmr, kappa, prec == HELIOS_MIXED, z.total_pt, atm->n_layer_h,
                              atm->n_bin_h, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "helios_mix_opacity");
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_transmission(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0,
                        const double* g0, double D, double* out, helios_prec prec, void* stream) {
    Sizes z;
    int rc = check_atm(atm, z);
    if (rc) return rc;
    if (!kappa || !T_pt || !w0 || !g0 || !out) return fail(HELIOS_EINVAL, "helios_transmission: NULL argument");
    if (prec != HELIOS_FP64 && prec != HELIOS_MIXED) return fail(HELIOS_EINVAL, "unknown precision %d", prec);
    if (!(D > 0.0)) return fail(HELIOS_EINVAL, "D = %g must be > 0", D);
    int64_t total_sub = 2 * (int64_t)atm->n_g * z.total_lb;
    hipError_t e = launch_transmission(atm, kappa, T_pt, w0, g0, D, out, total_sub, prec == HELIOS_MIXED,
                                       (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "helios_transmission");
    g_err[0] = 0;
    return HELIOS_OK;
}

size_t helios_workspace_bytes(const helios_atm* atm, helios_prec prec) {
    Sizes z;
    bool mixed = false, fstate = false;
    if (check_atm(atm, z) || !split_prec((int)prec, mixed, fstate)) return 0;
    return ws_layout(z, atm->n_g, mixed).total;
}

int helios_state_convert(const helios_atm* atm, const double* T_pt, double D, void* F_g, int32_t mode,
                         int32_t layers, helios_prec prec, void* stream) {
    Sizes z;
    int rc = check_atm(atm, z);
    if (rc) return rc;
    if (!T_pt || !F_g) return fail(HELIOS_EINVAL, "helios_state_convert: NULL argument");
    if (mode != HELIOS_CONVERT_TO_DEVIATION && mode != HELIOS_CONVERT_TO_FLUX && mode != HELIOS_CONVERT_ZERO_FLUX)
        return fail(HELIOS_EINVAL, "helios_state_convert: unknown mode %d", mode);
    if (layers != HELIOS_LAYERS_SUBLAYERED && layers != HELIOS_LAYERS_ISOTHERMAL)
        return fail(HELIOS_EINVAL, "helios_state_convert: unknown layers %d", layers);
    if (prec != HELIOS_FP64 && prec != HELIOS_MIXED) return fail(HELIOS_EINVAL, "unknown precision %d", prec);
    if (!(D > 0.0)) return fail(HELIOS_EINVAL, "D = %g must be > 0", D);
    hipError_t e = launch_state(atm, T_pt, 2.0 * kPi / D, F_g, mode, layers == HELIOS_LAYERS_ISOTHERMAL ? 1 : 0,
                                prec == HELIOS_MIXED, z.total_bin, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "helios_state_convert");
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_flux(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0,
                const double* g0, int32_t n_scat, double D, void* F_up_g, void* F_dn_g, double* F_up_bin,
                double* F_dn_bin, double* F_bol, void* ws, size_t ws_bytes, helios_prec prec, void* stream) {
    return flux_impl(atm, kappa, T_pt, w0, g0, n_scat, D, F_up_g, F_dn_g, F_up_bin, F_dn_bin, F_bol, ws, ws_bytes,
                     prec, stream, false, 0.0, "helios_flux");
}

int helios_flux_noalloc(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0,
                        const double* g0, int32_t n_scat, double D, void* F_up_g, void* F_dn_g, double* F_up_bin,
                        double* F_dn_bin, double* F_bol, helios_prec prec, void* stream) {
    Sizes z;
    bool mixed = false, fstate = false;
    int rc = check_atm(atm, z);
    if (rc) return rc;
    if (!split_prec((int)prec, mixed, fstate))
        return fail(HELIOS_EINVAL, "helios_flux_noalloc: unknown precision %d", (int)prec);
    const size_t need = ws_layout(z, atm->n_g, mixed).total;
    if (need > kScratchBytes)
        return fail(HELIOS_EWORKSPACE,
                    "helios_flux_noalloc: the batch needs %zu bytes of workspace, the static scratch holds %zu",
                    need, kScratchBytes);
    void* ws = nullptr;
    if ((rc = scratch_for_current_device(&ws, "helios_flux_noalloc"))) return rc;
    return flux_impl(atm, kappa, T_pt, w0, g0, n_scat, D, F_up_g, F_dn_g, F_up_bin, F_dn_bin, F_bol, ws,
                     kScratchBytes, prec, stream, false, 0.0, "helios_flux_noalloc");
}

int helios_flux_iso(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0,
                    const double* g0, int32_t n_scat, double D, void* F_up_g, void* F_dn_g, double* F_up_bin,
                    double* F_dn_bin, double* F_bol, void* ws, size_t ws_bytes, helios_prec prec, void* stream) {
    return flux_impl(atm, kappa, T_pt, w0, g0, n_scat, D, F_up_g, F_dn_g, F_up_bin, F_dn_bin, F_bol, ws, ws_bytes,
                     prec, stream, true, 0.0, "helios_flux_iso");
}

int helios_flux_rayleigh(const helios_atm* atm, const void* kappa, const double* T_pt, double mbar,
                         int32_t n_scat, double D, void* F_up_g, void* F_dn_g, double* F_up_bin,
                         double* F_dn_bin, double* F_bol, void* ws, size_t ws_bytes, helios_prec prec,
                         void* stream) {
    if (!(mbar > 0.0)) return fail(HELIOS_EINVAL, "helios_flux_rayleigh: mbar = %g must be > 0", mbar);
    return flux_impl(atm, kappa, T_pt, nullptr, nullptr, n_scat, D, F_up_g, F_dn_g, F_up_bin, F_dn_bin, F_bol, ws,
                     ws_bytes, prec, stream, false, 1.0 / mbar, "helios_flux_rayleigh");
}

int helios_flux_exact(const helios_atm* atm, const double* kappa, const double* T_pt, double* F_up_g,
                      double* F_dn_g, double* F_up_bin, double* F_dn_bin, double* F_bol, void* ws, size_t ws_bytes,
                      int32_t state, void* stream) {
    FluxPlan p;
    int rc = check_atm(atm, p.z);
    if (rc) return rc;
    if (!kappa || !T_pt || !F_up_g || !F_dn_g || !F_bol || !ws)
        return fail(HELIOS_EINVAL, "helios_flux_exact: NULL argument");
    if (state != HELIOS_STATE_DEVIATION && state != HELIOS_STATE_FLUX)
        return fail(HELIOS_EINVAL, "helios_flux_exact: unknown state 0x%x", state);
    p.mixed = false;
    p.flux_state = state == HELIOS_STATE_FLUX;
    p.w = ws_layout(p.z, atm->n_g, false);
    if (ws_bytes < p.w.total)
        return fail(HELIOS_EWORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, p.w.total);
    for (int k = 0; k < kNumClasses; ++k) p.sh[k] = {0, 0};
    hipStream_t s = (hipStream_t)stream;
    char* wsb = (char*)ws;
    hipError_t e = launch_sources(atm, p, T_pt, wsb, s);
    if (e != hipSuccess) return hip_fail(e, "helios_flux_exact (sources)");
    SweepArgs A = sweep_args(atm, p, kappa, nullptr, nullptr, 0, 2.0, F_up_g, F_dn_g, wsb);
    A.w_begin = 0;
    A.w_end = p.z.total_bin;
    e = launch_exact(A, p.z.total_bin, s);
    if (e != hipSuccess) return hip_fail(e, "helios_flux_exact (sweep)");
    BolArgs Bo;
    Bo.atm = *atm;
    Bo.part_up = A.part_up;
    Bo.part_dn = A.part_dn;
    Bo.F_up_bin = F_up_bin;
    Bo.F_dn_bin = F_dn_bin;
    Bo.chunk = (double*)(wsb + p.w.chunk);
    Bo.total_pt = p.z.total_pt;
    Bo.F_bol = F_bol;
    Bo.B = (const double*)(wsb + p.w.B);
    Bo.gw = (const double*)(wsb + p.w.gw);
    Bo.tpe = kPi;  // the deviations are taken from pi B
    Bo.tw = Bo.tpe * gauss_weight_sum(atm->n_g);
    Bo.wpb_stride = A.wpb_stride;
    Bo.chunk_bins = bol_chunk_bins(p.z.total_bin);
    Bo.n_chunk = (p.z.nb_max + Bo.chunk_bins - 1) / Bo.chunk_bins;
    Bo.mixed = 0;
    Bo.n_cls = kNumClasses;
    for (int k = 0; k < kNumClasses; ++k) {
        Bo.cls_nhi[k] = kClassNHi[k];
        Bo.cls_wpb[k] = 1;
    }
    e = launch_bolometric(Bo, p.z.npt_max, p.z.nb_max, p.z.total_pt, s);
    if (e != hipSuccess) return hip_fail(e, "helios_flux_exact (bolometric)");
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_autotune(const helios_atm* atm, const void* kappa, const double* T_pt, const double* w0,
                    const double* g0, int32_t n_scat, double D, void* F_up_g, void* ws, size_t ws_bytes,
                    helios_prec prec, void* stream) {
    const bool iso = ((int)prec & HELIOS_GRID_ISOTHERMAL) != 0;
    const helios_prec pr = (helios_prec)((int)prec & ~HELIOS_GRID_ISOTHERMAL);
    FluxPlan p;
    int rc = plan_flux(atm, kappa, T_pt, w0, g0, n_scat, D, F_up_g, ws, ws_bytes, pr, p, true, iso);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    char* wsb = (char*)ws;
    const size_t r = p.mixed ? sizeof(float) : sizeof(double);
    hipError_t e = launch_sources(atm, p, T_pt, wsb, s, iso);
    if (e != hipSuccess) return hip_fail(e, "helios_autotune (sources)");
    SweepArgs A = sweep_args(atm, p, kappa, w0, g0, n_scat, D, F_up_g, nullptr, wsb);
    A.iso_grid = iso ? 1 : 0;
    A.status = nullptr;  // time the work even where the batch marks a member converged
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<char> saved;
    auto cleanup = [&](int code) {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        return code;
    };
    if ((e = hipEventCreate(&ev0)) != hipSuccess || (e = hipEventCreate(&ev1)) != hipSuccess)
        return cleanup(hip_fail(e, "helios_autotune (events)"));
    for (int k = 0; k < kNumClasses; ++k) {
        if (p.z.cls_nmax[k] == 0) continue;
        // sample: up to 4096 bins of the class's deepest atmosphere
        const int a = p.z.cls_rep[k];
        int64_t b_lo = 0, c_lo = 0;
        for (int i = 0; i < a; ++i) {
            b_lo += atm->n_bin_h[i];
            c_lo += (int64_t)atm->n_bin_h[i] * atm->n_g * col_stride(atm->n_layer_h[i]);
        }
        const int64_t nbs = std::min<int64_t>(atm->n_bin_h[a], 4096);
        const size_t cells = (size_t)nbs * atm->n_g * col_stride(atm->n_layer_h[a]);
        char* fu = (char*)F_up_g + c_lo * r;
        saved.resize(cells * r);
        if ((e = hipMemcpyAsync(saved.data(), fu, cells * r, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return cleanup(hip_fail(e, "helios_autotune (save)"));
        const int nsub = (iso ? 1 : 2) * p.z.cls_nmax[k];  // slots per column
        SweepShape best = p.sh[k];
        float best_ms = 1e30f;
        for (int L : {16, 32, 64}) {
          const int groups = waves_per_bin(atm->n_g, L);
          for (int P : {1, 2, groups}) {
            if (P > std::min(groups, parts_stride(p.z, atm->n_g)) || (P == groups && P <= 2 && P != 1)) continue;
            for (int i = 0; i < kNumSweepK; ++i) {
                SweepShape c = {kSweepK[i], L, P};
                if (!shape_allowed(c.K, c.L, p.mixed) || c.K * c.L < nsub) continue;
                if (c.L == 64 && nsub <= kLongK * 32) continue;  // the long shape only where nothing else fits
                const int parts = P;
                if ((e = sweep_class(A, c, k, b_lo, b_lo + nbs, parts, p.mixed, s)) != hipSuccess)  // warm-up
                    return cleanup(hip_fail(e, "helios_autotune (sweep)"));
                float ms_min = 1e30f;
                for (int rep = 0; rep < 3; ++rep) {
                    float ms = 0.f;
                    if ((e = hipEventRecord(ev0, s)) != hipSuccess ||
                        (e = sweep_class(A, c, k, b_lo, b_lo + nbs, parts, p.mixed, s)) != hipSuccess ||
                        (e = hipEventRecord(ev1, s)) != hipSuccess || (e = hipEventSynchronize(ev1)) != hipSuccess ||
                        (e = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess)
                        return cleanup(hip_fail(e, "helios_autotune (timing)"));
                    ms_min = std::min(ms_min, ms);
                }
                if (ms_min < best_ms) {
                    best_ms = ms_min;
                    best = c;
                }
            }
          }
        }
        if ((e = hipMemcpyAsync(fu, saved.data(), cells * r, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return cleanup(hip_fail(e, "helios_autotune (restore)"));
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tuned[{p.mixed ? 1 : 0, atm->n_g, k, iso ? 1 : 0}] = best;
    }
    g_err[0] = 0;
    return cleanup(HELIOS_OK);
}

int helios_autotune_reset(void) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned.clear();
    return HELIOS_OK;
}

int helios_sweep_shapes(const helios_atm* atm, helios_prec prec, int32_t* out, int32_t max_classes) {
    Sizes z;
    int rc = check_atm(atm, z);
    if (rc) return rc;
    if (!out || max_classes < kNumClasses) return fail(HELIOS_EINVAL, "out needs %d classes", kNumClasses);
    bool mixed = false, fstate = false;
    const bool iso = ((int)prec & HELIOS_GRID_ISOTHERMAL) != 0;
    if (!split_prec((int)prec & ~HELIOS_GRID_ISOTHERMAL, mixed, fstate))
        return fail(HELIOS_EINVAL, "unknown precision 0x%x", (int)prec);
    for (int k = 0; k < kNumClasses; ++k) {
        SweepShape sh = {0, 0};
        if (z.cls_nmax[k]) {
            rc = pick_shape(k, (iso ? 1 : 2) * z.cls_nmax[k], atm->n_g, mixed, sh, iso);
            if (rc) return rc;
        }
        out[3 * k] = kClassNHi[k];
        out[3 * k + 1] = sh.K;
        out[3 * k + 2] = sh.L;
    }
    g_err[0] = 0;
    return kNumClasses;
}

size_t helios_mlp_param_count(const helios_mlp* net) {
    NetLayout L;
    return net_layout(net, L) ? L.count : 0;
}

size_t helios_mlp_workspace_bytes(const helios_mlp* net, int32_t batch) {
    NetLayout L;
    if (!net_layout(net, L) || batch < 1 || batch > (1 << 22)) return 0;
    return net_ws(net, batch).total;
}

int helios_mlp_sync(const helios_mlp* net, void* stream) {
    NetLayout L;
    int rc = check_net(net, L, false);
    if (rc) return rc;
    hipError_t e = launch_mlp_sync(net->params, net->params_bf16, (int64_t)L.count, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "helios_mlp_sync");
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_mlp_forward(const helios_mlp* net, const float* x, int32_t batch, float* T, void* ws, size_t ws_bytes,
                       void* stream) {
    NetLayout L;
    int rc = check_net(net, L, false);
    if (rc) return rc;
    if (!x || !T || !ws) return fail(HELIOS_EINVAL, "helios_mlp_forward: NULL argument");
    if (batch < 1 || batch > (1 << 22)) return fail(HELIOS_EINVAL, "batch = %d outside 1..2^22", batch);
    NetWs w = net_ws(net, batch);
    if (ws_bytes < w.total) return fail(HELIOS_EWORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, w.total);
    hipError_t e = net_forward(net, L, w, (char*)ws, x, batch, T, true, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "helios_mlp_forward");
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_mlp_backward(const helios_mlp* net, const float* x, const float* T_target, int32_t batch, float* loss,
                        float* grad, void* ws, size_t ws_bytes, void* stream) {
    NetLayout L;
    int rc = check_net(net, L, false);
    if (rc) return rc;
    if (!x || !T_target || !loss || !grad || !ws) return fail(HELIOS_EINVAL, "helios_mlp_backward: NULL argument");
    if (batch < 1 || batch > (1 << 22)) return fail(HELIOS_EINVAL, "batch = %d outside 1..2^22", batch);
    NetWs w = net_ws(net, batch);
    if (ws_bytes < w.total) return fail(HELIOS_EWORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, w.total);
    hipStream_t s = (hipStream_t)stream;
    char* wsb = (char*)ws;
    const int B = batch, H = net->n_hidden, no = net->n_out;
    float* Y = (float*)(wsb + w.Y);
    hipError_t e = net_forward(net, L, w, wsb, x, B, Y, false, s);
    if (e != hipSuccess) return hip_fail(e, "helios_mlp_backward (forward)");
    uint16_t* dY = (uint16_t*)(wsb + w.dY);
    e = launch_mlp_loss(Y, T_target, (int64_t)B * no, no, net->out_shift, net->out_scale, dY,
                        (double*)(wsb + w.partial), kLossBlocks, loss, s);
    if (e != hipSuccess) return hip_fail(e, "helios_mlp_backward (loss)");
    uint16_t* Dbuf[2] = {(uint16_t*)(wsb + w.D0), (uint16_t*)(wsb + w.D1)};
    const uint16_t* E = dY;  // error at the output of layer l, [B][out_l]
    int cur = 0;
    for (int l = L.nl - 1; l >= 0; --l) {
        const int in = L.in[l], out = L.out[l];
        const uint16_t* h = l == 0 ? (const uint16_t*)(wsb + w.X0) : (const uint16_t*)(wsb + w.A) + (size_t)(l - 1) * B * H;
        // weight gradient: dW[o][i] = sum_b E[b][o] h[b][i]
        GemmArgs g = gemm(E, 1, out, h, 1, in, out, in, B);
        g.out_f = grad + L.offW[l];
        g.ld_f = in;
        if ((e = launch_gemm(g, kEpiStore, s)) != hipSuccess) return hip_fail(e, "helios_mlp_backward (dW)");
        if ((e = launch_mlp_bias_grad(E, B, out, grad + L.offb[l], s)) != hipSuccess)
            return hip_fail(e, "helios_mlp_backward (db)");
        if (l == 0) break;
        // error at the output of layer l-1: (E W_l) * gelu'(Z_{l-1}), rounded to BF16
        GemmArgs d = gemm(E, out, 1, net->params_bf16 + L.offW[l], 1, in, B, in, out);
        d.zin = (const float*)(wsb + w.Z) + (size_t)(l - 1) * B * H;
        d.ld_z = H;
        d.out_b = Dbuf[cur];
        d.ld_b = H;
        if ((e = launch_gemm(d, kEpiDGelu, s)) != hipSuccess) return hip_fail(e, "helios_mlp_backward (dX)");
        E = Dbuf[cur];
        cur ^= 1;
    }
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_mlp_adam(const helios_mlp* net, const float* grad, int32_t step, float lr, float beta1, float beta2,
                    float eps, void* stream) {
    NetLayout L;
    int rc = check_net(net, L, true);
    if (rc) return rc;
    if (!grad) return fail(HELIOS_EINVAL, "helios_mlp_adam: grad is NULL");
    if (step < 1) return fail(HELIOS_EINVAL, "step = %d must be >= 1", step);
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(HELIOS_EINVAL, "helios_mlp_adam: bad hyper-parameters");
    const double bc1 = 1.0 - pow((double)beta1, step), bc2 = 1.0 - pow((double)beta2, step);
    hipError_t e = launch_mlp_adam(net->params, net->params_bf16, net->adam_m, net->adam_v, grad, (int64_t)L.count,
                                   lr, beta1, beta2, eps, (float)bc1, (float)bc2, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "helios_mlp_adam");
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_warm_start(const helios_atm* atm, const helios_mlp* net, const float* x, const double* logP_net,
                      double T_iso, double T_lo, double T_hi, double* T_c, int32_t* fallback, void* ws,
                      size_t ws_bytes, void* stream) {
    Sizes z;
    int rc = check_atm(atm, z);
    if (rc) return rc;
    NetLayout L;
    if ((rc = check_net(net, L, false))) return rc;
    if (!x || !logP_net || !T_c || !fallback || !ws) return fail(HELIOS_EINVAL, "helios_warm_start: NULL argument");
    if (net->n_out < 2) return fail(HELIOS_EINVAL, "helios_warm_start: the network needs >= 2 outputs");
    if (!(T_lo <= T_hi) || !(T_iso > 0.0)) return fail(HELIOS_EINVAL, "helios_warm_start: bad temperature bounds");
    if (atm->n_atm > (1 << 22)) return fail(HELIOS_EINVAL, "n_atm = %d above 2^22", atm->n_atm);
    NetWs w = net_ws(net, atm->n_atm);
    if (ws_bytes < w.total) return fail(HELIOS_EWORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, w.total);
    hipStream_t s = (hipStream_t)stream;
    char* wsb = (char*)ws;
    float* T_net = (float*)(wsb + w.T);
    hipError_t e = net_forward(net, L, w, wsb, x, atm->n_atm, T_net, true, s);
    if (e != hipSuccess) return hip_fail(e, "helios_warm_start (network)");
    e = launch_warm_start(atm, T_net, net->n_out, logP_net, T_iso, T_lo, T_hi, T_c, fallback, s);
    if (e != hipSuccess) return hip_fail(e, "helios_warm_start (profiles)");
    g_err[0] = 0;
    return HELIOS_OK;
}

int helios_radeq(const helios_atm* atm, const double* F_bol, double* T_c, double* T_pt,
                 const helios_re_state* st, const helios_re_opts* opt, int32_t* status, double* resid,
                 void* stream) {
    Sizes z;
    int rc = check_atm(atm, z);
    if (rc) return rc;
    if (!F_bol || !T_c || !T_pt || !st || !st->m || !st->hist || !opt || !status)
        return fail(HELIOS_EINVAL, "helios_radeq: NULL argument");
    if (opt->window < 2 || opt->window > 16) return fail(HELIOS_EINVAL, "window = %d outside 2..16", opt->window);
    if (opt->norm != HELIOS_NORM_SIGMA_T4 && opt->norm != HELIOS_NORM_SIGMA_TINT4)
        return fail(HELIOS_EINVAL, "unknown norm %d", opt->norm);
    if (!(opt->tol >= 0.0) || !(opt->shrink > 0.0) || !(opt->grow > 0.0) || !(opt->fpre_c > 0.0))
        return fail(HELIOS_EINVAL, "helios_radeq: bad options");
    hipError_t e = launch_radeq(atm, F_bol, T_c, T_pt, st, *opt, status, resid, z.n_max, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "helios_radeq");
    g_err[0] = 0;
    return HELIOS_OK;
}

}  // extern "C"
