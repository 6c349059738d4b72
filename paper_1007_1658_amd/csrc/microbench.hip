// microbench.hip -- instruction-throughput microbenchmarks for gfx950.
//
// The paper explains its speedup by measuring the sin/cos throughput of both
// platforms (Section 5.3).  These kernels measure the rates that bound the
// periodogram kernel on this GPU: FP32 FMA, FP64 FMA, hardware sin+cos, the
// FP64 phase reduction (round + convert), each with eight independent chains
// per lane, at a chosen number of resident waves per SIMD; and how many vector
// FMAs issue alongside 32x32x16 FP16 MFMAs before they slow the matrix pipe.  Every wave runs
// a fixed trip count; the result is stored so that nothing is eliminated.
#include <string>

#include "internal.h"

namespace lsp {

constexpr int kChains = 8;

template <int KIND>
__global__ void __launch_bounds__(64) mb_kernel(float *out, int iters, float seed)
{
    const int lane = threadIdx.x;
    float a[kChains];
    double d[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        a[i] = seed + 0.001f * (float)(lane + i);
        d[i] = (double)a[i];
    }
    const float m = 0.999f, c = 1e-4f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                if constexpr (KIND == 0) {
                    a[i] = __builtin_fmaf(a[i], m, c);  // FP32 FMA
                } else if constexpr (KIND == 1) {
                    d[i] = __builtin_fma(d[i], 0.999, 1e-4);  // FP64 FMA
                } else if constexpr (KIND == 2) {
                    a[i] = __builtin_amdgcn_sinf(a[i]) + __builtin_amdgcn_cosf(a[i]);  // 2 trans + 1 add
                } else {
                    double p = d[i] * 1.0000001;  // FP64 phase: mul, round, fma, convert
                    a[i] += (float)(p - __builtin_rint(p));
                    d[i] = p;
                }
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i] + (float)d[i];
    out[blockIdx.x * 64 + lane] = s;
}

typedef _Float16 mb_halfx8 __attribute__((ext_vector_type(8)));
typedef float mb_floatx16 __attribute__((ext_vector_type(16)));

// Matrix-core / vector co-issue: per step four independent 32x32x16 FP16
// MFMAs (one per accumulator), each followed by NV independent FP32 FMAs on
// eight chains.  NV = 0 measures the matrix pipe alone; WITH_MFMA = false
// issues the same FMA stream without the MFMAs.
template <int NV, bool WITH_MFMA>
__global__ void __launch_bounds__(64) mb_coissue_kernel(float *out, int iters, float seed)
{
    const int lane = threadIdx.x;
    mb_halfx8 A, B;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        A[i] = (_Float16)(seed * (float)(lane + i));
        B[i] = (_Float16)(seed * (float)(i + 1));
    }
    mb_floatx16 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = mb_floatx16{};
    float a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = seed + 0.001f * (float)(lane + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (WITH_MFMA) acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, B, acc[q], 0, 0, 0);
#pragma unroll
                for (int k = 0; k < NV; ++k) a[k % kChains] = __builtin_fmaf(a[k % kChains], 0.999f, 1e-4f);
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) s += acc[q][r];
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i];
    out[blockIdx.x * 64 + lane] = s;
}

}  // namespace lsp

using namespace lsp;

extern "C" lsp_status lsp_microbench(int32_t kind, int32_t waves_per_simd, int32_t iters, void *stream,
                                     double *ops_per_s, double *ms)
{
    if (kind < 0 || kind > 8 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || !ops_per_s)
        return LSP_ERR_INVALID_ARG;
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (he == hipSuccess) he = hipGetDeviceProperties(&prop, dev);
    if (he != hipSuccess) {
        set_last_error(std::string("lsp_microbench: ") + hipGetErrorString(he));
        return LSP_ERR_NO_DEVICE;
    }
    const int blocks = prop.multiProcessorCount * 4 * waves_per_simd;  // one wave per block
    hipStream_t s = (hipStream_t)stream;
    float *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc(&out, sizeof(float) * 64 * (size_t)blocks) != hipSuccess) return LSP_ERR_HIP;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    typedef void (*Fn)(float *, int, float);
    const Fn fns[9] = {mb_kernel<0>,
                       mb_kernel<1>,
                       mb_kernel<2>,
                       mb_kernel<3>,
                       mb_coissue_kernel<0, true>,
                       mb_coissue_kernel<4, true>,
                       mb_coissue_kernel<8, true>,
                       mb_coissue_kernel<16, true>,
                       mb_coissue_kernel<16, false>};
    hipLaunchKernelGGL(fns[kind], dim3(blocks), dim3(64), 0, s, out, 1, 0.1f);  // warm-up
    hipEventRecord(e0, s);
    hipLaunchKernelGGL(fns[kind], dim3(blocks), dim3(64), 0, s, out, iters, 0.1f);
    hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(out);
    if (e != hipSuccess) return LSP_ERR_HIP;
    // counted operations per lane per inner step: 1 FMA / 1 FMA / sin+cos / one phase
    // reduction (kinds 0-3, eight chains); kinds 4-7: the four MFMAs' FLOPs
    // (4 x 32x32x16 x 2 per wave, i.e. 2048 per lane); kind 8: its 64 FMAs
    double per_step = kChains;
    if (kind >= 4 && kind <= 7) per_step = 4.0 * 32 * 32 * 16 * 2 / 64;
    if (kind == 8) per_step = 64.0;
    const double per_lane = (double)iters * 8.0 * per_step;
    *ops_per_s = per_lane * 64.0 * (double)blocks / (t * 1e-3);
    if (ms) *ms = t;
    return LSP_OK;
}
