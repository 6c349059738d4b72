// mlp_kernels.hip -- the false-alarm surrogate's network on gfx950 matrix cores.
//
// A 4-layer perceptron (68 -> 256 -> 256 -> 256 -> 2, GELU in tanh form after
// the first three layers) maps sampling-pattern features to the two parameters
// (location and scale) of the law of the maximum periodogram power of white
// noise; quantiles and false-alarm probabilities follow from that law.  Products run on BF16 MFMA
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

// ---------------------------------------------------------------------------
// The law of the maximum.  A single frequency's normalized power z exceeds a
// level with the beta-law probability (1 - 2z/Nt)^((Nt-3)/2) = exp(-w(z)) of
// white noise (Section 3, beside Eq. (3)); the maximum over the grid is taken
// as Gumbel in w with location ln Nf + m and scale beta:
//   P(max <= z) = exp(-exp(-u)),  u = (w(z) - ln Nf - m) / beta,
//   m = mu + sigma r_0,  beta = softplus(r_1 + ln(e - 1)).
// m = 0, beta = 1 is Eq. (3) with Nf independent frequencies (in its Poisson
// limit).  Per-pattern arithmetic is FP64.

constexpr double kBetaShift = 0.54132485461291810;  // ln(e - 1): beta = 1 at r_1 = 0

__device__ __forceinline__ double softplus_d(double r) { return r > 30.0 ? r : log1p(exp(r)); }
__device__ __forceinline__ double sigmoid_d(double r) { return 1.0 / (1.0 + exp(-r)); }

// the nine reported quantile levels tau
__device__ __forceinline__ double quantile_level(int i)
{
    switch (i) {
    case 0: return 0.5;
    case 1: return 0.75;
    case 2: return 0.9;
    case 3: return 0.95;
    case 4: return 0.975;
    case 5: return 0.99;
    case 6: return 0.995;
    case 7: return 0.998;
    default: return 0.999;
    }
}

struct PatternSize {
    double Nt, lnNf;
};

__device__ __forceinline__ PatternSize pattern_size(const float *feat, int b)
{
    PatternSize p;
    p.Nt = rint(pow(10.0, (double)feat[(size_t)b * kMlpIn + kFeatLogNt]));
    p.lnNf = log(rint(pow(10.0, (double)feat[(size_t)b * kMlpIn + kFeatLogNf])));
    return p;
}

// exponential-equivalent power of z, and its inverse
__device__ __forceinline__ double w_of(double z, double Nt)
{
    return -0.5 * (Nt - 3.0) * log1p(-fmin(2.0 * z / Nt, 1.0 - 1e-15));
}
__device__ __forceinline__ double z_of(double w, double Nt) { return -0.5 * Nt * expm1(-2.0 * w / (Nt - 3.0)); }

__global__ void __launch_bounds__(256) head_kernel(const float *raw, int ldr, const float *feat, int B, float mu,
                                                   float sigma, float *law, float *q)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    const double m = (double)mu + (double)sigma * (double)raw[(size_t)b * ldr];
    const double beta = softplus_d((double)raw[(size_t)b * ldr + 1] + kBetaShift);
    if (law) {
        law[(size_t)b * 2] = (float)m;
        law[(size_t)b * 2 + 1] = (float)beta;
    }
    if (q) {
        const PatternSize ps = pattern_size(feat, b);
        for (int i = 0; i < kQuantiles; ++i) {
            const double w = ps.lnNf + m + beta * -log(-log(quantile_level(i)));
            q[(size_t)b * kQuantiles + i] = (float)z_of(w, ps.Nt);
        }
    }
}

hipError_t launch_head(const float *raw, int ldr, const float *feat, int B, float mu, float sigma, float *law, float *q,
                       hipStream_t s)
{
    hipLaunchKernelGGL(head_kernel, dim3((B + 255) / 256), dim3(256), 0, s, raw, ldr, feat, B, mu, sigma, law, q);
    return hipGetLastError();
}

// Negative log-likelihood of R Monte-Carlo maxima per pattern under the law,
//   L = 1/(B R) sum_b sum_r [ln beta + u + exp(-u)],  u = (w(y) - ln Nf - m) / beta,
// and its gradient through the head, written as dRaw in FP32 and BF16 (both layouts).
__global__ void __launch_bounds__(256) gumbel_nll_kernel(const float *raw, int ldr, const float *feat, int B, int Bp,
                                                         const float *y, int R, float mu, float sigma, float *loss_b,
                                                         float *dR, __bf16 *dRb, __bf16 *dRbT)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= Bp) return;
    float dr0 = 0.f, dr1 = 0.f, lb = 0.f;
    if (b < B) {
        const double r1 = (double)raw[(size_t)b * ldr + 1] + kBetaShift;
        const double m = (double)mu + (double)sigma * (double)raw[(size_t)b * ldr];
        const double beta = softplus_d(r1);
        const PatternSize ps = pattern_size(feat, b);
        double su = 0.0, se = 0.0, sue = 0.0;  // sums of u, exp(-u), u exp(-u)
        for (int r = 0; r < R; ++r) {
            const double u = (w_of((double)y[(size_t)b * R + r], ps.Nt) - ps.lnNf - m) / beta;
            const double e = exp(-u);
            su += u;
            se += e;
            sue += u * e;
        }
        const double scale = 1.0 / ((double)B * (double)R);
        lb = (float)(((double)R * log(beta) + su + se) * scale);
        const double dm = -((double)R - se) / beta * scale;          // dL/dm
        const double db = ((double)R - su + sue) / beta * scale;      // dL/dbeta
        dr0 = (float)(dm * (double)sigma);
        dr1 = (float)(db * sigmoid_d(r1));
    }
    if (loss_b && b < B) loss_b[b] = lb;
    for (int i = 0; i < kMlpOutPad; ++i) {
        const float d = (i == 0) ? dr0 : (i == 1 ? dr1 : 0.f);
        dR[(size_t)b * kMlpOutPad + i] = d;
        dRb[(size_t)b * kMlpOutPad + i] = to_bf16(d);
        dRbT[(size_t)i * Bp + b] = to_bf16(d);
    }
}

hipError_t launch_gumbel_nll(const float *raw, int ldr, const float *feat, int B, int Bp, const float *y, int R,
                             float mu, float sigma, float *loss_b, float *dR, __bf16 *dRb, __bf16 *dRbT,
                             hipStream_t s)
{
    hipLaunchKernelGGL(gumbel_nll_kernel, dim3((Bp + 255) / 256), dim3(256), 0, s, raw, ldr, feat, B, Bp, y, R, mu,
                       sigma, loss_b, dR, dRb, dRbT);
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

// FAP of an observed maximum under each member's law, 1 - exp(-exp(-u)),
// then the members' mean and spread.
// FAP of p_obs under every member's law, their mean, and a per-pattern error
// bound.  The members' spread measures how far they disagree; the calibrated
// standard errors (err_m, err_beta) of the law's location and scale, carried
// to the FAP through its derivatives at this pattern's p_obs,
//   dFAP/dm = e^{-u} exp(-e^{-u}) / beta,   dFAP/dbeta = u e^{-u} exp(-e^{-u}) / beta,
// measure how far the law itself may be off.  bound = z sqrt(spread^2 +
// (err_m dFAP/dm)^2 + (err_beta dFAP/dbeta)^2).
__global__ void __launch_bounds__(256) fap_kernel(const float *law, int members, int B, const float *feat,
                                                  const float *p_obs, float err_m, float err_beta, float z,
                                                  float *fap, float *bound)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    const PatternSize ps = pattern_size(feat, b);
    const double w = w_of((double)p_obs[b], ps.Nt) - ps.lnNf;
    double s1 = 0.0, s2 = 0.0, dm = 0.0, db = 0.0;
    for (int e = 0; e < members; ++e) {
        const float *lw = law + ((size_t)e * B + b) * 2;
        const double beta = (double)lw[1];
        const double u = (w - (double)lw[0]) / beta;
        const double eu = exp(-u);
        const double f = -expm1(-eu);
        const double g = eu * exp(-eu) / beta;
        s1 += f;
        s2 += f * f;
        dm += g;
        db += u * g;
    }
    const double mean = s1 / members;
    dm /= members;
    db /= members;
    const double spread2 = fmax(s2 / members - mean * mean, 0.0);
    const double law2 = (double)err_m * err_m * dm * dm + (double)err_beta * err_beta * db * db;
    fap[b] = (float)mean;
    bound[b] = (float)((double)z * sqrt(spread2 + law2));
}

hipError_t launch_fap(const float *law, int members, int B, const float *feat, const float *p_obs, float err_m,
                      float err_beta, float z, float *fap, float *bound, hipStream_t s)
{
    hipLaunchKernelGGL(fap_kernel, dim3((B + 255) / 256), dim3(256), 0, s, law, members, B, feat, p_obs, err_m,
                       err_beta, z, fap, bound);
    return hipGetLastError();
}

// empirical FAP of p_obs among R Monte-Carlo maxima (fraction >= p_obs) and z
// times its binomial standard error
__global__ void __launch_bounds__(256) mc_fap_kernel(const float *pmax, int R, int B, const float *p_obs,
                                                     const int32_t *idx, float z, float *fap, float *bound)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= B) return;
    const int b = idx[i];
    int n = 0;
    for (int r = 0; r < R; ++r) n += (pmax[(size_t)i * R + r] >= p_obs[b]) ? 1 : 0;
    const float f = (float)n / (float)R;
    fap[b] = f;
    bound[b] = z * sqrtf(f * (1.f - f) / (float)R);
}

hipError_t launch_mc_fap(const float *pmax, int R, int B, const float *p_obs, const int32_t *idx, float z,
                         float *fap, float *bound, hipStream_t s)
{
    hipLaunchKernelGGL(mc_fap_kernel, dim3((B + 255) / 256), dim3(256), 0, s, pmax, R, B, p_obs, idx, z, fap,
                       bound);
    return hipGetLastError();
}

}  // namespace lsp
