// mlp.h -- shapes and launchers of the surrogate network kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsp {

constexpr int kMlpIn = 68;        // features
constexpr int kMlpInPad = 96;     // padded to the MFMA K step (32)
constexpr int kMlpHidden = 256;
constexpr int kMlpOut = 2;        // location and scale of the law of the maximum
constexpr int kMlpOutPad = 32;    // padded to the 32-wide output tile
constexpr int kMlpLayers = 4;
constexpr int kQuantiles = 9;     // reported quantile levels (see quantile_level)
constexpr int kFeatLogNt = 64;    // raw feature slots holding log10 Nt and log10 Nf
constexpr int kFeatLogNf = 67;

enum { GEMM_STORE = 0, GEMM_BIAS = 1, GEMM_BIAS_GELU = 2, GEMM_DGELU = 3 };

struct GemmArgs {
    const __bf16 *A;  // [M][K], row stride lda
    int lda;
    const __bf16 *B;  // [N][K], row stride ldb
    int ldb;
    int M, N, K;      // multiples of 32
    int epi;          // GEMM_*
    const float *bias;  // [N] (BIAS, BIAS_GELU)
    const float *Z;     // [M][N] pre-activation, row stride ldz (DGELU)
    int ldz;
    float *C;         // FP32 result (pre-activation for BIAS_GELU), nullable
    int ldc;
    __bf16 *Cb;       // BF16 copy (GELU output for BIAS_GELU), nullable
    int ldcb;
    __bf16 *CbT;      // BF16 transposed copy [N][M], nullable
    int ldcbT;
};

hipError_t launch_gemm_nt(const GemmArgs &g, hipStream_t s);
hipError_t launch_features_in(const float *feat, int B, int Bp, const float *mean, const float *stdv, __bf16 *X,
                              __bf16 *XT, float *zmax, hipStream_t s);
// law [B][2] = (m, beta) and/or q [B][9] (either may be null) from the raw outputs
hipError_t launch_head(const float *raw, int ldr, const float *feat, int B, float mu, float sigma, float *law, float *q,
                       hipStream_t s);
hipError_t launch_gumbel_nll(const float *raw, int ldr, const float *feat, int B, int Bp, const float *y, int R,
                             float mu, float sigma, float *loss_b, float *dR, __bf16 *dRb, __bf16 *dRbT,
                             hipStream_t s);
hipError_t launch_sum(const float *v, int n, float *out, hipStream_t s);
hipError_t launch_colsum(const float *dZ, int B, int N, float *db, hipStream_t s);
hipError_t launch_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_cast_weights(const float *W, int rows, int cols, __bf16 *Wb, __bf16 *WbT, hipStream_t s);
// mean FAP of the members' laws and its error bound (see fap_kernel)
hipError_t launch_fap(const float *law, int members, int B, const float *feat, const float *p_obs, float err_m,
                      float err_beta, float z, float *fap, float *bound, hipStream_t s);
hipError_t launch_mc_fap(const float *pmax, int R, int B, const float *p_obs, const int32_t *idx, float z,
                         float *fap, float *bound, hipStream_t s);

}  // namespace lsp
