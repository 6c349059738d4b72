// probe_kernels.hip -- the building blocks of the periodogram kernels run on
// caller-given inputs, one element per lane, with the very device functions
// the kernels use: the hardware sine and cosine in revolutions, the reduced
// phase of each phase mode (Section 4.4's reduction and its split-precision
// replacements) and the frequency recurrence.  They let the error of each
// block be measured on its own, against FP64 or 80-bit references on the host.
#include "pgram_device.h"

namespace lsp {

__global__ void __launch_bounds__(256) probe_sincos_kernel(const float *__restrict__ r, int64_t n,
                                                           float *__restrict__ s, float *__restrict__ c)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        s[i] = sin_rev(r[i]);
        c[i] = cos_rev(r[i]);
    }
}

// The sample as the records and the LDS tiles hold it: SPLIT and SPLIT32 keep
// t' = t - t_ref as the FP32 pair (th, tl) (SPLIT re-forms th + tl in FP64 when
// staging), NAIVE keeps raw t rounded to FP32.
template <int PHASE>
__device__ __forceinline__ Smp probe_sample(double t, double t_ref)
{
    Smp sm;
    sm.t = 0.0;
    sm.th = 0.0f;
    sm.tl = 0.0f;
    sm.x = 0.0f;
    sm.rc = 1.0f;
    sm.rs = 0.0f;
    if constexpr (PHASE == PH_NAIVE) {
        sm.th = (float)t;
    } else {
        split_time(t - t_ref, sm.th, sm.tl);
        sm.t = (double)sm.th + (double)sm.tl;
    }
    return sm;
}

template <int PHASE>
__global__ void __launch_bounds__(256) probe_phase_kernel(const double *__restrict__ t,
                                                          const double *__restrict__ f, int64_t n, double t_ref,
                                                          float *__restrict__ phi)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const Smp sm = probe_sample<PHASE>(t[i], t_ref);
        Freq<PHASE, TR_DIRECT, 1> F;
        F.set(0, f[i]);
        phi[i] = phase_of<PHASE, TR_DIRECT, 1>(F, 0, sm);
    }
}

constexpr int kProbeRecurMax = 32;

// c, s[i * M + m] = (cos, sin)(2 pi (f0 + m step_df) t'_i), m < M, as the
// recurrence form of the kernel produces them for one sample and lane.
__global__ void __launch_bounds__(256) probe_recur_kernel(const double *__restrict__ t, int64_t n, double t_ref,
                                                          double f0, double step_df, int M, float *__restrict__ c,
                                                          float *__restrict__ s)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        Smp sm = probe_sample<PH_SPLIT>(t[i], t_ref);
        step_rotation(step_df, t[i] - t_ref, sm.rc, sm.rs);
        Freq<PH_SPLIT, TR_RECUR, kProbeRecurMax> F;
        F.set(0, f0);
        const float ph = phase_of<PH_SPLIT, TR_RECUR, kProbeRecurMax>(F, 0, sm);
        recur_terms<kProbeRecurMax>(ph, sm.rc, sm.rs, [&](int m, float cm, float sn) {
            if (m < M) {
                c[i * M + m] = cm;
                s[i * M + m] = sn;
            }
        });
    }
}

static unsigned probe_blocks(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

hipError_t launch_probe_sincos(const float *r, int64_t n, float *s, float *c, hipStream_t st)
{
    hipLaunchKernelGGL(probe_sincos_kernel, dim3(probe_blocks(n)), dim3(256), 0, st, r, n, s, c);
    return hipGetLastError();
}

hipError_t launch_probe_phase(const double *t, const double *f, int64_t n, double t_ref, int phase, float *phi,
                              hipStream_t st)
{
    const dim3 g(probe_blocks(n)), b(256);
    switch (phase) {
    case PH_SPLIT: hipLaunchKernelGGL(probe_phase_kernel<PH_SPLIT>, g, b, 0, st, t, f, n, t_ref, phi); break;
    case PH_SPLIT32: hipLaunchKernelGGL(probe_phase_kernel<PH_SPLIT32>, g, b, 0, st, t, f, n, t_ref, phi); break;
    case PH_NAIVE: hipLaunchKernelGGL(probe_phase_kernel<PH_NAIVE>, g, b, 0, st, t, f, n, t_ref, phi); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int probe_recur_max() { return kProbeRecurMax; }

hipError_t launch_probe_recur(const double *t, int64_t n, double t_ref, double f0, double step_df, int M, float *c,
                              float *s, hipStream_t st)
{
    if (M < 1 || M > kProbeRecurMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(probe_recur_kernel, dim3(probe_blocks(n)), dim3(256), 0, st, t, n, t_ref, f0, step_df, M, c,
                       s);
    return hipGetLastError();
}

}  // namespace lsp
