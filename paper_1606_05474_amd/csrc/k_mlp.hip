// k_mlp.hip -- the learned warm start: a multilayer perceptron on the
// matrix cores (BF16 operands, FP32 accumulation), its back-propagation, the
// Adam update, and the interpolation of its profile onto each atmosphere's
// layers with the isothermal fallback.
//
// One GEMM kernel serves every product of the network: C = A * B^T over a
// K dimension, with A(m, k) and B(n, k) read through arbitrary strides, so
// the forward product (activations x weights^T), the data gradient (errors x
// weights) and the weight gradient (errors^T x activations) are the same
// code with different strides.  A workgroup of 4 waves owns a 64 x 64 output
// tile; each wave owns 32 x 32 of it as 2 x 2 tiles of the 16x16x32 BF16
// MFMA.  Per K step of 32 the two 64 x 32 operand tiles are staged in LDS.
// The epilogue is fused: bias + GELU (storing the pre-activation for the
// backward pass and the BF16 activation for the next layer), bias + output
// scaling, the GELU derivative applied to a data gradient, or a plain FP32
// store of a weight gradient.
#include <math.h>

#include "helios_internal.hpp"

namespace helios {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// float -> bfloat16 bits, round to nearest with ties to even; NaN stays NaN.
__device__ inline uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU in the exact form z * Phi(z) and its derivative Phi(z) + z phi(z).
__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

constexpr int kTile = 64, kKStep = 32, kLdsPad = 8;

template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t sA[kTile][kKStep + kLdsPad];
    __shared__ __attribute__((aligned(16))) uint16_t sB[kTile][kKStep + kLdsPad];
    const int m0 = blockIdx.x * kTile, n0 = blockIdx.y * kTile;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = t >> 2, lk = (t & 3) * 8;  // staging: row lr, k offset lk..lk+7
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int am = m0 + lr, bn = n0 + lr;
    const bool arow = am < g.M, brow = bn < g.N;
    for (int k0 = 0; k0 < g.K; k0 += kKStep) {
        const int kb = k0 + lk;
        for (int i = 0; i < 8; ++i) {
            const int k = kb + i;
            const bool kin = k < g.K;
            sA[lr][lk + i] = (arow && kin) ? g.A[(int64_t)am * g.sam + (int64_t)k * g.sak] : (uint16_t)0;
            sB[lr][lk + i] = (brow && kin) ? g.B[(int64_t)bn * g.sbn + (int64_t)k * g.sbk] : (uint16_t)0;
        }
        __syncthreads();
        bf16x8 a[2], b[2];
        // operand layout of the 16x16x32 MFMA: lane l supplies row (l mod 16)
        // and the 8 K values starting at 8 (l / 16); A and B use the same K
        // assignment, so the sum over K is the full dot product
        for (int i = 0; i < 2; ++i)
            a[i] = *reinterpret_cast<const bf16x8*>(&sA[wm + i * 16 + (lane & 15)][(lane >> 4) * 8]);
        for (int j = 0; j < 2; ++j)
            b[j] = *reinterpret_cast<const bf16x8*>(&sB[wn + j * 16 + (lane & 15)][(lane >> 4) * 8]);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // result layout: lane l holds rows 4 (l / 16) + e, e = 0..3, column l mod 16
    for (int i = 0; i < 2; ++i) {
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + j * 16 + (lane & 15);
            if (n >= g.N) continue;
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + e;
                if (m >= g.M) continue;
                const float v = acc[i][j][e];
                if constexpr (EPI == kEpiGelu) {
                    const float z = v + g.bias[n];
                    g.out_f[(int64_t)m * g.ld_f + n] = z;
                    g.out_b[(int64_t)m * g.ld_b + n] = to_bf16(gelu_f(z));
                } else if constexpr (EPI == kEpiLinear) {
                    float y = v + g.bias[n];
                    if (g.oscale) y = g.oshift[n] + g.oscale[n] * y;
                    g.out_f[(int64_t)m * g.ld_f + n] = y;
                } else if constexpr (EPI == kEpiDGelu) {
                    const float z = g.zin[(int64_t)m * g.ld_z + n];
                    g.out_b[(int64_t)m * g.ld_b + n] = to_bf16(v * gelu_grad_f(z));
                } else {
                    g.out_f[(int64_t)m * g.ld_f + n] = v;
                }
            }
        }
    }
}

hipError_t launch_gemm(const GemmArgs& g, int epi, hipStream_t s) {
    dim3 grid((unsigned)((g.M + kTile - 1) / kTile), (unsigned)((g.N + kTile - 1) / kTile));
    switch (epi) {
        case kEpiGelu: hipLaunchKernelGGL(gemm_bf16_kernel<kEpiGelu>, grid, dim3(256), 0, s, g); break;
        case kEpiLinear: hipLaunchKernelGGL(gemm_bf16_kernel<kEpiLinear>, grid, dim3(256), 0, s, g); break;
        case kEpiDGelu: hipLaunchKernelGGL(gemm_bf16_kernel<kEpiDGelu>, grid, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL(gemm_bf16_kernel<kEpiStore>, grid, dim3(256), 0, s, g); break;
    }
    return hipGetLastError();
}

// --------------------------------------------------------- elementwise
// Normalised inputs, rounded to BF16: X0[b][j] = bf16((x - shift_j) scale_j).
__global__ void mlp_input_kernel(const float* __restrict__ x, int64_t count, int n_in,
                                 const float* __restrict__ shift, const float* __restrict__ scale,
                                 uint16_t* __restrict__ X0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int j = (int)(i % n_in);
    X0[i] = to_bf16((x[i] - shift[j]) * scale[j]);
}

// Loss and output error: r = y - (T - shift)/scale, dY = bf16(2 r / count),
// per-block sums of r^2 in a fixed order (double).
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                       int64_t count, int n_out, const float* __restrict__ shift,
                                                       const float* __restrict__ scale, uint16_t* __restrict__ dY,
                                                       double* __restrict__ partial, int64_t per_block) {
    __shared__ double red[256];
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = min(count, lo + per_block);
    const float inv = 2.0f / (float)count;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const int j = (int)(i % n_out);
        const float t = (T[i] - shift[j]) / scale[j];
        const float r = Y[i] - t;
        dY[i] = to_bf16(r * inv);
        acc += (double)r * (double)r;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void mlp_loss_final_kernel(const double* __restrict__ partial, int nblk,
                                                             double inv_count, float* __restrict__ loss) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partial[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(red[0] * inv_count);
}

// Bias gradient: column sums of a BF16 error matrix D [rows][N], fixed order.
__global__ __launch_bounds__(256) void mlp_bias_grad_kernel(const uint16_t* __restrict__ D, int64_t rows, int N,
                                                            float* __restrict__ gb) {
    __shared__ float red[256];
    const int n = blockIdx.x;
    float acc = 0.f;
    for (int64_t m = threadIdx.x; m < rows; m += blockDim.x) acc += from_bf16(D[m * N + n]);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) gb[n] = red[0];
}

// Adam (Kingma & Ba, Algorithm 1) on the FP32 master parameters, refreshing
// the BF16 copy; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void mlp_adam_kernel(float* __restrict__ p, uint16_t* __restrict__ pb, float* __restrict__ m,
                                float* __restrict__ v, const float* __restrict__ grad, int64_t count, float lr,
                                float beta1, float beta2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gr = grad[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gr;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gr * gr;
    m[i] = mi;
    v[i] = vi;
    const float w = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    p[i] = w;
    pb[i] = to_bf16(w);
}

__global__ void mlp_sync_kernel(const float* __restrict__ p, uint16_t* __restrict__ pb, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) pb[i] = to_bf16(p[i]);
}

hipError_t launch_mlp_input(const float* x, int64_t count, int n_in, const float* shift, const float* scale,
                            uint16_t* X0, hipStream_t s) {
    hipLaunchKernelGGL(mlp_input_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, x, count, n_in,
                       shift, scale, X0);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(const float* Y, const float* T, int64_t count, int n_out, const float* shift,
                           const float* scale, uint16_t* dY, double* partial, int nblk, float* loss,
                           hipStream_t s) {
    const int64_t per = (count + nblk - 1) / nblk;
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(nblk), dim3(256), 0, s, Y, T, count, n_out, shift, scale, dY, partial,
                       per);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_loss_final_kernel, dim3(1), dim3(256), 0, s, partial, nblk, 1.0 / (double)count, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_bias_grad(const uint16_t* D, int64_t rows, int N, float* gb, hipStream_t s) {
    hipLaunchKernelGGL(mlp_bias_grad_kernel, dim3(N), dim3(256), 0, s, D, rows, N, gb);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, uint16_t* pb, float* m, float* v, const float* grad, int64_t count, float lr,
                           float beta1, float beta2, float eps, float bc1, float bc2, hipStream_t s) {
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, pb, m, v, grad,
                       count, lr, beta1, beta2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_mlp_sync(const float* p, uint16_t* pb, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(mlp_sync_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, pb, count);
    return hipGetLastError();
}

// ------------------------------------------------------------ warm start
// One workgroup per atmosphere: the network's n_out temperatures at the log
// pressures logP_net (monotone, either direction) are checked (finite and in
// [T_lo, T_hi]; otherwise the whole atmosphere takes T_iso) and interpolated
// linearly in log10 P onto the atmosphere's layer centres, holding the end
// values outside the network's range.
__global__ __launch_bounds__(256) void warm_start_kernel(helios_atm atm, const float* __restrict__ T_net, int n_out,
                                                         const double* __restrict__ logP_net, double T_iso,
                                                         double T_lo, double T_hi, double* __restrict__ T_c,
                                                         int32_t* __restrict__ fallback) {
    __shared__ double s_lp[kMaxNetOut];
    __shared__ double s_T[kMaxNetOut];
    const int a = blockIdx.x;
    const float* row = T_net + (int64_t)a * n_out;
    // store in ascending log P
    const bool desc = logP_net[0] > logP_net[n_out - 1];
    int bad = 0;
    for (int j = threadIdx.x; j < n_out; j += blockDim.x) {
        const int src = desc ? n_out - 1 - j : j;
        const double T = (double)row[src];
        s_lp[j] = logP_net[src];
        s_T[j] = T;
        bad |= !(T >= T_lo && T <= T_hi);  // NaN fails both
    }
    bad = __syncthreads_or(bad);
    const int n = atm.n_layer[a];
    const int64_t off = atm.lay_off[a];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double T;
        if (bad) {
            T = T_iso;
        } else {
            const double lp = log10(atm.P_c[off + i]);
            if (lp <= s_lp[0]) {
                T = s_T[0];
            } else if (lp >= s_lp[n_out - 1]) {
                T = s_T[n_out - 1];
            } else {
                int lo = 0, hi = n_out - 1;  // s_lp[lo] < lp < s_lp[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_lp[mid] <= lp) lo = mid; else hi = mid;
                }
                const double f = (lp - s_lp[lo]) / (s_lp[hi] - s_lp[lo]);
                T = s_T[lo] + f * (s_T[hi] - s_T[lo]);
            }
        }
        T_c[off + i] = T;
    }
    if (threadIdx.x == 0) fallback[a] = bad ? 1 : 0;
}

hipError_t launch_warm_start(const helios_atm* atm, const float* T_net, int n_out, const double* logP_net,
                             double T_iso, double T_lo, double T_hi, double* T_c, int32_t* fallback,
                             hipStream_t s) {
    hipLaunchKernelGGL(warm_start_kernel, dim3(atm->n_atm), dim3(256), 0, s, *atm, T_net, n_out, logP_net, T_iso,
                       T_lo, T_hi, T_c, fallback);
    return hipGetLastError();
}

}  // namespace helios
