// fast_kernels.hip -- the approximate periodogram of Press & Rybicki (1989),
// the extirpolation + FFT approach that Section 1 cites beside the direct
// sums: values are spread onto a periodic grid of N points whose period is
// 1/df with Lagrange weights (the transpose of Lagrange interpolation), the
// grids are Fourier transformed (hipFFT, FP64), and Eqs. (5)-(7) are
// evaluated on the transformed bins.  Everything here is FP64 (the spread
// sums in 64-bit fixed point, see below).
#include <algorithm>

#include "pgram_device.h"

namespace lsp {

__global__ void __launch_bounds__(256) fast_fill_kernel(double *__restrict__ g, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) g[i] = 0.0;
}

// The spreading adds into 64-bit fixed point, so that a grid point's sum does
// not depend on the order in which the atomic updates land (integer addition
// is associative; FP64 atomic addition is not, and made reruns differ in the
// last bits).  Each term is rounded to a multiple of 2^(e - 62), with 2^e
// above the largest magnitude the grid point's sum can reach: the sum of
// |value| |weight| over all samples.  |weight| < 2 for the Lagrange weights of
// the stencils built here (on the central interval of 4, 6 or 8 equispaced
// nodes no basis polynomial exceeds 1 in magnitude), and
// |x_j - mean| <= sqrt(Nt var), since one squared deviation
// cannot exceed their sum.  The sum of two's-complement words is exact modulo
// 2^64, so only the final value has to be in range.
struct FixedScale {
    double to_fixed, to_real;
};

__device__ __forceinline__ FixedScale fixed_scale(double bound)
{
    int e = 0;
    if (bound > 0.0) (void)frexp(bound, &e);  // bound < 2^e
    return FixedScale{ldexp(1.0, 62 - e), ldexp(1.0, e - 62)};
}

constexpr double kLagrangeWeightBound = 2.0;

// bounds of the two grids' sums: values x_j - mean, and ones
__device__ __forceinline__ FixedScale value_scale(const CurveStats &s, int64_t Nt)
{
    const double n = (double)Nt;
    return fixed_scale(n * sqrt(n * fmax(s.var, 0.0)) * kLagrangeWeightBound);
}

__device__ __forceinline__ FixedScale ones_scale(int64_t Nt) { return fixed_scale((double)Nt * kLagrangeWeightBound); }

// spreads value v at grid position u (grid units, 0 <= u < N) over the macc
// nearest points n0 .. n0 + macc - 1, n0 = floor(u) - macc/2 + 1, with the
// Lagrange basis weights of those points at u, as fixed-point words; indices
// wrap modulo N
template <int MACC>
__device__ __forceinline__ void spread(unsigned long long *__restrict__ g, int64_t N, double u, double v,
                                       double to_fixed)
{
    const double fl = floor(u);
    const int64_t n0 = (int64_t)fl - (MACC / 2 - 1);
    const double s = u - (double)n0;
#pragma unroll
    for (int m = 0; m < MACC; ++m) {
        double w = 1.0;
#pragma unroll
        for (int l = 0; l < MACC; ++l)
            if (l != m) w *= (s - (double)l) / (double)(m - l);
        int64_t n = (n0 + m) % N;
        if (n < 0) n += N;
        atomicAdd(&g[n], (unsigned long long)llrint(v * w * to_fixed));
    }
}

// gx: values x_j - mean at u_j = (t_j - t_min) df N; g1: ones at 2 u_j mod N
template <int MACC>
__global__ void __launch_bounds__(256) fast_extirp_kernel(const double *__restrict__ t, const float *__restrict__ x,
                                                          int64_t Nt, const CurveStats *__restrict__ st, double df,
                                                          int64_t N, unsigned long long *__restrict__ gx,
                                                          unsigned long long *__restrict__ g1)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= Nt) return;
    const CurveStats s = *st;
    double u = (t[j] - s.t_min) * df * (double)N;
    u -= floor(u / (double)N) * (double)N;
    double v = 2.0 * u;
    v -= floor(v / (double)N) * (double)N;
    spread<MACC>(gx, N, u, (double)x[j] - s.mean, value_scale(s, Nt).to_fixed);
    spread<MACC>(g1, N, v, 1.0, ones_scale(Nt).to_fixed);
}

// the fixed-point grids back to FP64, in place, for the transforms
__global__ void __launch_bounds__(256) fast_fixed_to_real_kernel(double *__restrict__ g, int64_t N, int64_t Nt,
                                                                 const CurveStats *__restrict__ st)
{
    const double ux = value_scale(*st, Nt).to_real, u1 = ones_scale(Nt).to_real;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 2 * N; i += (int64_t)gridDim.x * 256) {
        const long long q = __double_as_longlong(g[i]);
        g[i] = (double)q * (i < N ? ux : u1);
    }
}

// bin m0 + k of each transform: sum x e^{-i w t} = XC - i XS and the same at
// twice the angle = C2 - i S2; Eq. (5) with CC = (Nt + C2)/2, CS = S2/2
__global__ void __launch_bounds__(256) fast_epilogue_kernel(const double2 *__restrict__ Fx,
                                                            const double2 *__restrict__ F1, int64_t m0, int64_t Nf,
                                                            int64_t Nt, const CurveStats *__restrict__ st,
                                                            float *__restrict__ Pn)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= Nf) return;
    const double2 a = Fx[m0 + k], b = F1[m0 + k];
    const double XC = a.x, XS = -a.y;
    const double CC = 0.5 * ((double)Nt + b.x), CS = -0.5 * b.y;
    Pn[k] = pn_from_sums(XC, XS, CC, CS, (double)Nt, st->inv_var);
}

hipError_t launch_fast_extirp(const double *t, const float *x, int64_t Nt, const CurveStats *stats, double df,
                              int64_t N, int macc, double *grids, hipStream_t s)
{
    const unsigned fb = (unsigned)std::min<int64_t>((2 * N + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(fast_fill_kernel, dim3(fb), dim3(256), 0, s, grids, 2 * N);
    const unsigned nb = (unsigned)((Nt + 255) / 256);
    // the zero fill above is zero as fixed point too
    unsigned long long *gx = (unsigned long long *)grids, *g1 = gx + N;
    if (macc == 4)
        hipLaunchKernelGGL(fast_extirp_kernel<4>, dim3(nb), dim3(256), 0, s, t, x, Nt, stats, df, N, gx, g1);
    else if (macc == 6)
        hipLaunchKernelGGL(fast_extirp_kernel<6>, dim3(nb), dim3(256), 0, s, t, x, Nt, stats, df, N, gx, g1);
    else if (macc == 8)
        hipLaunchKernelGGL(fast_extirp_kernel<8>, dim3(nb), dim3(256), 0, s, t, x, Nt, stats, df, N, gx, g1);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(fast_fixed_to_real_kernel, dim3(fb), dim3(256), 0, s, grids, N, Nt, stats);
    return hipGetLastError();
}

hipError_t launch_fast_epilogue(const void *spectra, int64_t N, int64_t m0, int64_t Nf, int64_t Nt,
                                const CurveStats *stats, float *Pn, hipStream_t s)
{
    const double2 *Fx = (const double2 *)spectra;
    const double2 *F1 = Fx + (N / 2 + 1);
    hipLaunchKernelGGL(fast_epilogue_kernel, dim3((unsigned)((Nf + 255) / 256)), dim3(256), 0, s, Fx, F1, m0, Nf,
                       Nt, stats, Pn);
    return hipGetLastError();
}

}  // namespace lsp
