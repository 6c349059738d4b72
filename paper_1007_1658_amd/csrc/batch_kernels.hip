// batch_kernels.hip -- many periodograms in one persistent launch.
//
// Curves are grouped by sampling pattern: a group owns a run of times (and
// their split-time records), a curve owns values.  Ordinary batches have one
// curve per group; Monte-Carlo batches draw many white-noise curves on one
// pattern (the use the paper names for its code in Section 6.2, the false-alarm
// statistics of many noise periodograms).  The same persistent kernel also
// evaluates the spectral window |sum_j exp(2 pi i f t_j)|^2 (values all 1, no
// mean removed), from which the per-pattern band features are taken.
//
// Sequence per launch: init (queue and per-curve reductions reset by a fill
// kernel), time records per group, value records per curve, the persistent
// periodogram kernel, per-curve finalization.
#include "pgram_device.h"

namespace lsp {

constexpr int kBatchM = 8;
int batched_freq_per_item(int form) { return form == LSP_TRIG_MFMA ? kBatchMfmaFreq : kWave * kBatchM; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications and xors, key bumped by the Weyl constants.

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Standard normal deviate number j of counter stream `curve`: Box-Muller on the
// first two output words (24-bit uniforms in (0, 1), exact in FP32).
__device__ __forceinline__ float normal_deviate(uint64_t seed, uint64_t curve, int64_t j)
{
    U4 c;
    c.x = (uint32_t)j;
    c.y = (uint32_t)curve;
    c.z = (uint32_t)(curve >> 32);
    c.w = 0u;
    const U4 o = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float u1 = ((float)(o.x >> 8) + 0.5f) * 5.9604644775390625e-08f;  // 2^-24
    const float u2 = ((float)(o.y >> 8) + 0.5f) * 5.9604644775390625e-08f;
    return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

__global__ void __launch_bounds__(256) normals_kernel(uint64_t seed, uint64_t curve, int64_t n, float *out)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) out[j] = normal_deviate(seed, curve, j);
}

hipError_t launch_normals(uint64_t seed, uint64_t curve, int64_t n, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(normals_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, curve, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) batch_init_kernel(BatchArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i == 0) {
        *a.queue = 0u;
        *a.t0 = wall_clock64();
    }
    if (i < a.n_curves) {
        a.key[i] = 0ull;
        a.tbeg[i] = ~0ull;
        a.tend[i] = 0ull;
    }
}

// per group: time range, origin, split times and the recurrence step
__global__ void __launch_bounds__(256) batch_time_kernel(BatchArgs a)
{
    const BatchGroup g = a.groups[blockIdx.x];
    const double *t = a.t + g.toff;
    Moments m = moments_empty();
    for (int64_t j = threadIdx.x; j < g.Nt; j += 256) moments_push(m, 0.0, t[j]);
    m = block_merge_256(m);
    const double t_ref = 0.5 * (m.tmin + m.tmax);
    if (threadIdx.x == 0) {
        a.t_ref[3 * blockIdx.x] = t_ref;
        a.t_ref[3 * blockIdx.x + 1] = m.tmin;
        a.t_ref[3 * blockIdx.x + 2] = m.tmax;
    }
    const double step_df = (double)kWave * g.df;
    for (int64_t j = threadIdx.x; j < g.Nt; j += 256) {
        const double tp = t[j] - t_ref;
        float th, tl, rc, rs;
        split_time(tp, th, tl);
        step_rotation(step_df, tp, rc, rs);
        a.th[g.toff + j] = th;
        a.tl[g.toff + j] = tl;
        a.rc[g.toff + j] = rc;
        a.rs[g.toff + j] = rs;
    }
}

template <int VAL>
__device__ __forceinline__ float value_of(const BatchArgs &a, const BatchCurve &cv, int c, int64_t j)
{
    if constexpr (VAL == VAL_INPUT) return a.x[cv.xoff + j];
    else if constexpr (VAL == VAL_NORMAL) return normal_deviate(a.seed, a.curve_base + (uint64_t)c, j);
    else return 1.0f;
}

// per curve: mean and population variance of the values, centred value records
template <int VAL>
__global__ void __launch_bounds__(256) batch_value_kernel(BatchArgs a)
{
    const int c = blockIdx.x;
    const BatchCurve cv = a.curves[c];
    CurveStats s;
    if constexpr (VAL == VAL_ONES) {
        // the spectral window: unit values, no mean removed, no variance scaling
        s.mean = 0.0;
        s.var = 1.0;
        s.inv_var = 1.0;
        s.zero_var = 0;
    } else {
        Moments m = moments_empty();
        for (int64_t j = threadIdx.x; j < cv.Nt; j += 256) moments_push(m, (double)value_of<VAL>(a, cv, c, j), 0.0);
        m = block_merge_256(m);
        s.mean = m.mean;
        s.var = m.m2 / m.n;
        s.zero_var = (m.m2 > 0.0) ? 0 : 1;
        s.inv_var = s.zero_var ? 0.0 : 1.0 / s.var;
    }
    s.t_ref = a.t_ref[3 * cv.group];
    s.t_min = a.t_ref[3 * cv.group + 1];
    s.t_max = a.t_ref[3 * cv.group + 2];
    s.wsum = (double)cv.Nt;
    s.pad_ = 0;
    if (threadIdx.x == 0) a.stats[c] = s;
    for (int64_t j = threadIdx.x; j < cv.Nt; j += 256)
        a.xv[cv.xoff + j] = (float)((double)value_of<VAL>(a, cv, c, j) - s.mean);
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o, kWave);
        v = (w > v) ? w : v;
    }
    return v;
}

// the epilogue kept out of line so that its FP64 constants do not occupy
// registers across the persistent loop
__device__ __noinline__ float batch_epilogue(double XC, double XS, double CC, double CS, double Nt,
                                             double inv_var, int epi)
{
    if (epi == EPI_WINDOW) return (float)(XC * XC + XS * XS);
    return pn_from_sums(XC, XS, CC, CS, Nt, inv_var);
}

template <int M>
__global__ void __launch_bounds__(256) batch_pgram_kernel(BatchArgs a)
{
    __shared__ Tile<PH_SPLIT> tiles[kMaxWaves];
    __shared__ float comp_lds[CompLds<SUM_KAHAN, M>::kFloats];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // A wave never takes more than n_items items, so the bound below is a
    // guaranteed exit on top of the drained-queue test.
    for (int guard = 0; guard <= a.n_items; ++guard) {
        // Every lane executes the atomic and only lane 0 adds 1, so lane 0's return
        // value is this wave's item.  No lane-dependent branch surrounds it: with one,
        // the compiler may split this loop so that lanes other than 0 never see a new
        // item.  readfirstlane makes the index a scalar, and the exit below is a
        // wave-uniform branch that every wave reaches once the queue is drained.
        const unsigned int it =
            __builtin_amdgcn_readfirstlane(atomicAdd(a.queue, lane == 0 ? 1u : 0u));
        if (it >= (unsigned)a.n_items) break;
        const BatchItem item = a.items[it];
        const BatchCurve cv = a.curves[item.curve];
        if (lane == 0) atomicMin(&a.tbeg[item.curve], (unsigned long long)wall_clock64());
        const int64_t k0 = (int64_t)item.fblock * kWave * M;
        Records r;
        r.th = a.th + cv.toff;
        r.tl = a.tl + cv.toff;
        r.rc = a.rc + cv.toff;
        r.rs = a.rs + cv.toff;
        r.xv = a.xv + cv.xoff;
        Totals<SUM_KAHAN, M> Tot;
        Tot.init(comp_lds + wave * 3 * M * kWave, lane);
        wave_sums<PH_SPLIT, TR_RECUR, M, 4, SUM_KAHAN>(tiles[wave], r, 0, cv.Nt, cv.f_min, cv.df, k0, lane, Tot);
        const double inv_var = a.stats[item.curve].inv_var;
        const double pads = (double)pad_count(cv.Nt);
        unsigned long long best = 0ull;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int64_t k = k0 + lane + (int64_t)kWave * m;
            if (k < cv.Nf) {
                const float P = batch_epilogue(Tot.value(0, m), Tot.value(1, m), Tot.value(2, m) - pads,
                                               Tot.value(3, m), (double)cv.Nt, inv_var, a.epi_mode);
                if (a.Pn) a.Pn[cv.pn_off + k] = P;
                const unsigned long long key =
                    ((unsigned long long)__float_as_uint(P) << 32) | (unsigned long long)(0xffffffffu - (unsigned)k);
                best = (key > best) ? key : best;
            }
        }
        best = wave_max_u64(best);
        if (lane == 0) {
            atomicMax(&a.key[item.curve], best);
            atomicMax(&a.tend[item.curve], (unsigned long long)wall_clock64());
        }
    }
}

__global__ void __launch_bounds__(256) batch_final_kernel(BatchArgs a, double ns_per_tick)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= a.n_curves) return;
    const unsigned long long key = a.key[c];
    const unsigned k = 0xffffffffu - (unsigned)(key & 0xffffffffull);
    const BatchCurve cv = a.curves[c];
    const bool zero = a.stats[c].zero_var != 0;
    if (a.pmax) a.pmax[c] = zero ? __int_as_float(0x7fc00000) : __uint_as_float((unsigned)(key >> 32));
    if (a.kbest) a.kbest[c] = zero ? -1 : (int64_t)k;
    if (a.fbest) a.fbest[c] = zero ? __longlong_as_double(0x7ff8000000000000ll) : cv.f_min + (double)k * cv.df;
    if (a.t_ns) {
        const unsigned long long t0 = *a.t0;
        a.t_ns[2 * c] = (uint64_t)((double)(a.tbeg[c] - t0) * ns_per_tick);
        a.t_ns[2 * c + 1] = (uint64_t)((double)(a.tend[c] - t0) * ns_per_tick);
    }
}

hipError_t batched_occupancy(int form, int waves, int *blocks_per_cu)
{
    if (form == LSP_TRIG_MFMA) return batch_mfma_occupancy(blocks_per_cu);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_pgram_kernel<kBatchM>,
                                                        kWave * waves, 0);
}

hipError_t launch_batched(const BatchArgs &a, int form, int persistent_blocks, int waves, hipStream_t s)
{
    if (form != LSP_TRIG_RECUR && form != LSP_TRIG_MFMA) return hipErrorInvalidValue;
    int dev = 0;
    hipGetDevice(&dev);
    int rate_khz = 0;
    hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
    const double ns_per_tick = rate_khz > 0 ? 1e6 / (double)rate_khz : 10.0;
    const unsigned nb_c = (unsigned)((a.n_curves + 255) / 256);
    hipLaunchKernelGGL(batch_init_kernel, dim3(nb_c), dim3(256), 0, s, a);
    hipLaunchKernelGGL(batch_time_kernel, dim3((unsigned)a.n_groups), dim3(256), 0, s, a);
    if (a.val_mode == VAL_NORMAL)
        hipLaunchKernelGGL(batch_value_kernel<VAL_NORMAL>, dim3((unsigned)a.n_curves), dim3(256), 0, s, a);
    else if (a.val_mode == VAL_ONES)
        hipLaunchKernelGGL(batch_value_kernel<VAL_ONES>, dim3((unsigned)a.n_curves), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(batch_value_kernel<VAL_INPUT>, dim3((unsigned)a.n_curves), dim3(256), 0, s, a);
    if (form == LSP_TRIG_MFMA) {
        hipError_t e = launch_batch_mfma(a, persistent_blocks, s);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(batch_pgram_kernel<kBatchM>, dim3((unsigned)persistent_blocks), dim3(kWave * waves), 0,
                           s, a);
    }
    hipLaunchKernelGGL(batch_final_kernel, dim3(nb_c), dim3(256), 0, s, a, ns_per_tick);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Spectral-window features of each pattern (one 256-thread block per group;
// the batch holds one unit-valued curve per group whose window power sits in
// Pn at the curve's pn_off).
//   feat[0..63]: log10 of the mean window power over Nt in 64 bands of the
//                frequency index, log-spaced: band b covers k in
//                [round(Nf^(b/64)) - 1, round(Nf^((b+1)/64)) - 1) with the outer
//                edges 0 and Nf, at least one k;
//   feat[64]: log10 Nt;  feat[65]: log10 T (T = t_max - t_min);
//   feat[66]: gap fraction = sum of the spacings longer than five mean spacings,
//             over T (times sorted);  feat[67]: log10 Nf.

__global__ void __launch_bounds__(256) window_features_kernel(BatchArgs a, float *feat)
{
    const int c = blockIdx.x;
    const BatchCurve cv = a.curves[c];
    const BatchGroup g = a.groups[cv.group];
    float *out = feat + (size_t)c * kFeatures;
    const double Nf = (double)cv.Nf;
    if (threadIdx.x < kWindowBands) {
        const int b = threadIdx.x;
        // edges round(Nf^(b/64)) - 1, the outer ones fixed at 0 and Nf
        int64_t lo = (b == 0) ? 0 : (int64_t)rint(exp(log(Nf) * (double)b / kWindowBands)) - 1;
        int64_t hi = (b == kWindowBands - 1) ? cv.Nf
                                             : (int64_t)rint(exp(log(Nf) * (double)(b + 1) / kWindowBands)) - 1;
        lo = lo < 0 ? 0 : (lo > cv.Nf - 1 ? cv.Nf - 1 : lo);
        hi = hi < lo + 1 ? lo + 1 : (hi > cv.Nf ? cv.Nf : hi);
        double sum = 0.0;
        for (int64_t k = lo; k < hi; ++k) sum += (double)a.Pn[cv.pn_off + k];
        out[b] = (float)log10(sum / (double)(hi - lo) / (double)cv.Nt + 1e-30);
    }
    // gap fraction over sorted times
    const double *t = a.t + g.toff;
    const double T = a.t_ref[3 * cv.group + 2] - a.t_ref[3 * cv.group + 1];
    const double thr = 5.0 * T / (double)(g.Nt - 1);
    double gsum = 0.0;
    for (int64_t j = threadIdx.x; j + 1 < g.Nt; j += 256) {
        const double d = t[j + 1] - t[j];
        if (d > thr) gsum += d;
    }
    __shared__ double red[256];
    red[threadIdx.x] = gsum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[kWindowBands + 0] = (float)log10((double)cv.Nt);
        out[kWindowBands + 1] = (float)log10(T > 0.0 ? T : 1e-30);
        out[kWindowBands + 2] = (float)(T > 0.0 ? red[0] / T : 0.0);
        out[kWindowBands + 3] = (float)log10(Nf);
    }
}

hipError_t launch_window_features(const BatchArgs &a, float *feat, int n_feat, hipStream_t s)
{
    if (n_feat != kFeatures) return hipErrorInvalidValue;
    hipLaunchKernelGGL(window_features_kernel, dim3((unsigned)a.n_curves), dim3(256), 0, s, a, feat);
    return hipGetLastError();
}

}  // namespace lsp
