// mlp_kernels.hip -- the false-alarm surrogate's network on gfx950 matrix cores.
//
// A 4-layer perceptron (68 -> 256 -> 256 -> 256 -> 9, GELU in tanh form after
// the first three layers) maps sampling-pattern features to nine quantiles of
// the maximum periodogram power of white noise.  Products run on BF16 MFMA
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation; FP32 master weights,
// Adam moments and all elementwise work stay in FP32.
//
// GEMM convention ("NT"): C[M][N] = sum_k A[M][K] B[N][K], both operands
// K-contiguous BF16 row-major, so every lane fetches 8 consecutive BF16 (16 B).
// Forward: A = activations [B][in], B = W [out][in].  Backward: dH = dZ W uses
// W^T [in][out]; dW = dZ^T H uses dZ^T [out][B] and H^T [in][B]; so the
// epilogues write activations and their gradients in both layouts.
//
// One wavefront owns a 32x32 tile as 2x2 MFMA blocks of 16x16.  Fragment
// layout of v_mfma_f32_16x16x32_bf16 (64 lanes, l = lane):
//   A (16x32):  lane l holds A[l % 16][8 (l / 16) .. 8 (l / 16) + 7]
//   B (32x16):  lane l holds B[8 (l / 16) .. + 7][l % 16]   (= our Bnt[l % 16][...])
//   D (16x16):  lane l holds D[4 (l / 16) + r][l % 16], r = 0..3
#include <hip/hip_bf16.h>
#include <math.h>

#include "internal.h"
#include "mlp.h"

namespace lsp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 to_bf16(float v) { return __float2bfloat16(v); }  // round to nearest even

// GELU, tanh form, and its derivative
__device__ __forceinline__ float gelu(float z)
{
    const float u = 0.7978845608028654f * (z + 0.044715f * z * z * z);
    return 0.5f * z * (1.0f + tanhf(u));
}
__device__ __forceinline__ float gelu_grad(float z)
{
    const float u = 0.7978845608028654f * (z + 0.044715f * z * z * z);
    const float th = tanhf(u);
    return 0.5f * (1.0f + th) + 0.5f * z * (1.0f - th * th) * 0.7978845608028654f * (1.0f + 0.134145f * z * z);
}

__global__ void __launch_bounds__(64) gemm_nt_kernel(GemmArgs g)
{
    const int lane = threadIdx.x;
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const __bf16 *Ar0 = g.A + (size_t)(m0 + r16) * g.lda + kq;
    const __bf16 *Ar1 = Ar0 + (size_t)16 * g.lda;
    const __bf16 *Br0 = g.B + (size_t)(n0 + r16) * g.ldb + kq;
    const __bf16 *Br1 = Br0 + (size_t)16 * g.ldb;
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(Ar0 + k0);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(Ar1 + k0);
        const bf16x8 b0 = *reinterpret_cast<const bf16x8 *>(Br0 + k0);
        const bf16x8 b1 = *reinterpret_cast<const bf16x8 *>(Br1 + k0);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + 16 * i + 4 * (lane >> 4) + r;
                const int col = n0 + 16 * j + r16;
                float v = acc[i][j][r];
                float out_b = v;  // value written to the BF16 copies
                if (g.epi == GEMM_BIAS_GELU) {
                    v += g.bias[col];
                    out_b = gelu(v);
                } else if (g.epi == GEMM_BIAS) {
                    v += g.bias[col];
                    out_b = v;
                } else if (g.epi == GEMM_DGELU) {
                    v *= gelu_grad(g.Z[(size_t)row * g.ldz + col]);
                    out_b = v;
                }
                if (g.C) g.C[(size_t)row * g.ldc + col] = v;
                if (g.Cb) g.Cb[(size_t)row * g.ldcb + col] = to_bf16(out_b);
                if (g.CbT) g.CbT[(size_t)col * g.ldcbT + row] = to_bf16(out_b);
            }
}

hipError_t launch_gemm_nt(const GemmArgs &g, hipStream_t s)
{
    if (g.M % 32 || g.N % 32 || g.K % 32 || g.lda % 8 || g.ldb % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemm_nt_kernel, dim3(g.N / 32, g.M / 32), dim3(64), 0, s, g);
    return hipGetLastError();
}

// standardized, zero-padded network input in both layouts; per-pattern max |z|
__global__ void __launch_bounds__(256) features_in_kernel(const float *feat, int B, int Bp, const float *mean,
                                                          const float *stdv, __bf16 *X, __bf16 *XT, float *zmax)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= Bp) return;
    float zm = 0.f;
    for (int i = 0; i < kMlpInPad; ++i) {
        float z = 0.f;
        if (b < B && i < kMlpIn) {
            z = (feat[(size_t)b * kMlpIn + i] - mean[i]) / stdv[i];
            zm = fmaxf(zm, fabsf(z));
        }
        const __bf16 zb = to_bf16(z);
        X[(size_t)b * kMlpInPad + i] = zb;
        XT[(size_t)i * Bp + b] = zb;
    }
    if (zmax && b < B) zmax[b] = zm;
}

hipError_t launch_features_in(const float *feat, int B, int Bp, const float *mean, const float *stdv, __bf16 *X,
                              __bf16 *XT, float *zmax, hipStream_t s)
{
    hipLaunchKernelGGL(features_in_kernel, dim3((Bp + 255) / 256), dim3(256), 0, s, feat, B, Bp, mean, stdv, X, XT,
                       zmax);
    return hipGetLastError();
}

__device__ __forceinline__ float softplus(float r) { return r > 20.f ? r : log1pf(expf(r)); }
__device__ __forceinline__ float sigmoid(float r) { return 1.f / (1.f + expf(-r)); }

// monotone head: q0 = mu + sigma r0, q_i = q_{i-1} + sigma softplus(r_i)
__device__ __forceinline__ void head(const float *raw, float mu, float sigma, float *q)
{
    float acc = mu + sigma * raw[0];
    q[0] = acc;
    for (int i = 1; i < kMlpOut; ++i) {
        acc += sigma * softplus(raw[i]);
        q[i] = acc;
    }
}

__global__ void __launch_bounds__(256) quantiles_kernel(const float *raw, int B, int ldr, float mu, float sigma,
                                                        float *q)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    head(raw + (size_t)b * ldr, mu, sigma, q + (size_t)b * kMlpOut);
}

hipError_t launch_quantiles(const float *raw, int B, int ldr, float mu, float sigma, float *q, hipStream_t s)
{
    hipLaunchKernelGGL(quantiles_kernel, dim3((B + 255) / 256), dim3(256), 0, s, raw, B, ldr, mu, sigma, q);
    return hipGetLastError();
}

// Pinball loss of the nine quantiles against R Monte-Carlo maxima per pattern,
//   L = 1/(9 B) sum_b sum_i 1/R sum_r rho_tau_i(y_br - q_bi),  rho_tau(u) = u (tau - [u < 0]),
// its gradient through the head, written as dRaw in FP32 and BF16 (both layouts).
__global__ void __launch_bounds__(256) pinball_kernel(const float *raw, int B, int Bp, int ldr, const float *y, int R,
                                                      const float *tau, float mu, float sigma, float *loss_b,
                                                      float *dR, __bf16 *dRb, __bf16 *dRbT)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= Bp) return;
    float dr[kMlpOutPad];
    for (int i = 0; i < kMlpOutPad; ++i) dr[i] = 0.f;
    float lb = 0.f;
    if (b < B) {
        const float *rb = raw + (size_t)b * ldr;
        float q[kMlpOut];
        head(rb, mu, sigma, q);
        float dq[kMlpOut];
        const float scale = 1.0f / (float)(kMlpOut * B);
        for (int i = 0; i < kMlpOut; ++i) {
            double lsum = 0.0;
            int below = 0;
            for (int r = 0; r < R; ++r) {
                const float u = y[(size_t)b * R + r] - q[i];
                below += (u < 0.f) ? 1 : 0;
                lsum += (double)(u * (tau[i] - (u < 0.f ? 1.f : 0.f)));
            }
            lb += (float)(lsum / (double)R);
            dq[i] = ((float)below / (float)R - tau[i]) * scale;
        }
        lb *= scale;
        // back through the head: q_i depends on r_0 (slope sigma) and on r_j, j <= i
        float tail = 0.f;
        for (int i = kMlpOut - 1; i >= 1; --i) {
            tail += dq[i];
            dr[i] = tail * sigma * sigmoid(rb[i]);
        }
        dr[0] = (tail + dq[0]) * sigma;
    }
    if (loss_b && b < B) loss_b[b] = lb;
    for (int i = 0; i < kMlpOutPad; ++i) {
        dR[(size_t)b * kMlpOutPad + i] = dr[i];
        dRb[(size_t)b * kMlpOutPad + i] = to_bf16(dr[i]);
        dRbT[(size_t)i * Bp + b] = to_bf16(dr[i]);
    }
}

hipError_t launch_pinball(const float *raw, int B, int Bp, int ldr, const float *y, int R, const float *tau, float mu,
                          float sigma, float *loss_b, float *dR, __bf16 *dRb, __bf16 *dRbT, hipStream_t s)
{
    hipLaunchKernelGGL(pinball_kernel, dim3((Bp + 255) / 256), dim3(256), 0, s, raw, B, Bp, ldr, y, R, tau, mu, sigma,
                       loss_b, dR, dRb, dRbT);
    return hipGetLastError();
}

// fixed-order sum of n values into out[0] (one block)
__global__ void __launch_bounds__(256) sum_kernel(const float *v, int n, float *out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += (double)v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)red[0];
}

hipError_t launch_sum(const float *v, int n, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, v, n, out);
    return hipGetLastError();
}

// bias gradient: column sums of dZ [M][N] over the first B rows, fixed order
__global__ void __launch_bounds__(256) colsum_kernel(const float *dZ, int B, int N, float *db)
{
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < B; ++m) s += dZ[(size_t)m * N + n];
    db[n] = s;
}

hipError_t launch_colsum(const float *dZ, int B, int N, float *db, hipStream_t s)
{
    hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, s, dZ, B, N, db);
    return hipGetLastError();
}

// Adam (Kingma & Ba, Algorithm 1) on a flat FP32 parameter buffer
__global__ void __launch_bounds__(256) adam_kernel(float *w, const float *g, float *m, float *v, int64_t n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    w[i] -= lr * mh / (sqrtf(vh) + eps);
}

hipError_t launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

// BF16 copies of a weight matrix [rows][cols] in both layouts
__global__ void __launch_bounds__(256) cast_weights_kernel(const float *W, int rows, int cols, __bf16 *Wb, __bf16 *WbT)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= rows * cols) return;
    const int r = i / cols, c = i % cols;
    const __bf16 v = to_bf16(W[i]);
    Wb[i] = v;
    WbT[(size_t)c * rows + r] = v;
}

hipError_t launch_cast_weights(const float *W, int rows, int cols, __bf16 *Wb, __bf16 *WbT, hipStream_t s)
{
    hipLaunchKernelGGL(cast_weights_kernel, dim3((rows * cols + 255) / 256), dim3(256), 0, s, W, rows, cols, Wb, WbT);
    return hipGetLastError();
}

// FAP of an observed maximum from predicted quantiles, per member: the CDF of
// the maximum is interpolated linearly in the Gumbel reduced variate
// y = -ln(-ln tau) against q (extrapolated along the end segments), and
// FAP = 1 - exp(-exp(-y)).  Then mean and spread over members.
__global__ void __launch_bounds__(256) fap_kernel(const float *q, int members, int B, const float *tau,
                                                  const float *p_obs, float *fap, float *sigma)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    double yl[kMlpOut];
    for (int i = 0; i < kMlpOut; ++i) yl[i] = -log(-log((double)tau[i]));
    const double p = (double)p_obs[b];
    double s1 = 0.0, s2 = 0.0;
    for (int e = 0; e < members; ++e) {
        const float *qb = q + ((size_t)e * B + b) * kMlpOut;
        int i = 0;
        while (i < kMlpOut - 2 && p > (double)qb[i + 1]) ++i;  // segment [i, i+1], ends extended
        const double dq = fmax((double)qb[i + 1] - (double)qb[i], 1e-12);
        const double y = yl[i] + (p - (double)qb[i]) * (yl[i + 1] - yl[i]) / dq;
        const double f = -expm1(-exp(-y));
        s1 += f;
        s2 += f * f;
    }
    const double mean = s1 / members;
    fap[b] = (float)mean;
    sigma[b] = (float)sqrt(fmax(s2 / members - mean * mean, 0.0));
}

hipError_t launch_fap(const float *q, int members, int B, const float *tau, const float *p_obs, float *fap,
                      float *sigma, hipStream_t s)
{
    hipLaunchKernelGGL(fap_kernel, dim3((B + 255) / 256), dim3(256), 0, s, q, members, B, tau, p_obs, fap, sigma);
    return hipGetLastError();
}

// empirical FAP of p_obs among R Monte-Carlo maxima: fraction >= p_obs
__global__ void __launch_bounds__(256) mc_fap_kernel(const float *pmax, int R, int B, const float *p_obs,
                                                     const int32_t *idx, float *fap, float *sigma)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= B) return;
    const int b = idx[i];
    int n = 0;
    for (int r = 0; r < R; ++r) n += (pmax[(size_t)i * R + r] >= p_obs[b]) ? 1 : 0;
    const float f = (float)n / (float)R;
    fap[b] = f;
    sigma[b] = sqrtf(f * (1.f - f) / (float)R);
}

hipError_t launch_mc_fap(const float *pmax, int R, int B, const float *p_obs, const int32_t *idx, float *fap,
                         float *sigma, hipStream_t s)
{
    hipLaunchKernelGGL(mc_fap_kernel, dim3((B + 255) / 256), dim3(256), 0, s, pmax, R, B, p_obs, idx, fap, sigma);
    return hipGetLastError();
}

}  // namespace lsp
