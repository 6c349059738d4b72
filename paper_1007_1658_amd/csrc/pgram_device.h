// pgram_device.h -- device-side building blocks shared by the periodogram
// kernels (single curve, batched, Monte Carlo, spectral window): moments and
// per-sample records, wave-private LDS tiles, phase reduction, the frequency
// recurrence, accumulation and the FP64 epilogue of Eqs. (5)-(7).
#pragma once

#include <math.h>

#include <hip/hip_ext.h>

#include "internal.h"

namespace lsp {

// A launch that, while the profiling hook is on, carries HIP events for its
// own start and end: the extended launch takes them from the dispatch itself,
// so the stream gets no marker commands between kernels (on MI355X a
// recorded event holds the stream for about 5 us).  No events: a plain launch.
template <typename... KArgs, typename... Args>
static inline void launch_timed(void (*kernel)(KArgs...), dim3 grid, dim3 block, hipStream_t s, hipEvent_t start,
                                hipEvent_t stop, Args... args)
{
    if (start || stop)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, start, stop, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

enum { PH_SPLIT = LSP_PHASE_SPLIT, PH_NAIVE = LSP_PHASE_NAIVE, PH_SPLIT32 = LSP_PHASE_SPLIT32 };
enum { TR_DIRECT = LSP_TRIG_DIRECT, TR_RECUR = LSP_TRIG_RECUR, TR_MFMA = LSP_TRIG_MFMA };

// hardware sin/cos take their argument in revolutions: sin_rev(r) = sin(2 pi r)
__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

// An FP64 phase p (revolutions) reduced to p - rint(p), |.| <= 1/2, then
// rounded to FP32: the reduction every split-phase path uses (Section 4.4
// reduces by the nearest integer too, but in FP32).
__device__ __forceinline__ float rev_reduce(double p) { return (float)(p - rint(p)); }

// A time offset t' as the FP32 pair the records hold: th = fl32(t'),
// tl = fl32(t' - th); th + tl in FP64 is t' to about 2^-48 relative.
__device__ __forceinline__ void split_time(double tp, float &th, float &tl)
{
    th = (float)tp;
    tl = (float)(tp - (double)th);
}

// (cos, sin) of the recurrence step angle 2 pi step_df t', reduced and
// evaluated in FP64 once per sample, rounded to FP32.
__device__ __forceinline__ void step_rotation(double step_df, double tp, float &rc, float &rs)
{
    double q = step_df * tp;  // revolutions of the step angle
    q -= rint(q);
    double sq, cq;
    sincospi(2.0 * q, &sq, &cq);
    rc = (float)cq;
    rs = (float)sq;
}

// ---------------------------------------------------------------------------
// Prep: moments of x (mean, population variance; Section 3 opening paragraph)
// and the time range, then the per-sample records.

__device__ __forceinline__ Moments moments_empty()
{
    Moments m;
    m.n = 0.0;
    m.mean = 0.0;
    m.m2 = 0.0;
    m.tmin = INFINITY;
    m.tmax = -INFINITY;
    return m;
}

__device__ __forceinline__ void moments_push(Moments &a, double x, double t)
{
    a.n += 1.0;
    double d = x - a.mean;
    a.mean += d / a.n;
    a.m2 += d * (x - a.mean);
    a.tmin = fmin(a.tmin, t);
    a.tmax = fmax(a.tmax, t);
}

// one sample with weight w >= 0 (West's weighted update; n is the weight sum)
__device__ __forceinline__ void moments_push_w(Moments &a, double x, double w, double t)
{
    a.tmin = fmin(a.tmin, t);
    a.tmax = fmax(a.tmax, t);
    if (!(w > 0.0)) return;
    a.n += w;
    double d = x - a.mean;
    a.mean += d * (w / a.n);
    a.m2 += w * d * (x - a.mean);
}

// Chan, Golub & LeVeque pairwise combination
__device__ __forceinline__ Moments moments_merge(const Moments &a, const Moments &b)
{
    if (a.n == 0.0) return b;
    if (b.n == 0.0) return a;
    Moments r;
    r.n = a.n + b.n;
    double d = b.mean - a.mean;
    r.mean = a.mean + d * (b.n / r.n);
    r.m2 = a.m2 + b.m2 + d * d * (a.n * (b.n / r.n));
    r.tmin = fmin(a.tmin, b.tmin);
    r.tmax = fmax(a.tmax, b.tmax);
    return r;
}

// fixed-order tree reduction over a 256-thread block
__device__ __forceinline__ Moments block_merge_256(Moments v)
{
    __shared__ Moments sm[256];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] = moments_merge(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    Moments r = sm[0];
    __syncthreads();
    return r;
}

// All partial moments merged in one fixed order, whatever the block size:
// leaf i < 256 folds parts i, i + 256, ..., then a 256-leaf tree (the block's
// threads take the leaves and the tree's nodes in turn).  Every block that
// calls it gets the same bits.
__device__ __forceinline__ Moments merge_parts(const Moments *__restrict__ part, int n_part)
{
    __shared__ Moments sm[256];
    const int tid = threadIdx.x;
    for (int l = tid; l < 256; l += blockDim.x) {
        Moments m = moments_empty();
        for (int i = l; i < n_part; i += 256) m = moments_merge(m, part[i]);
        sm[l] = m;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        for (int l = tid; l < w; l += blockDim.x) sm[l] = moments_merge(sm[l], sm[l + w]);
        __syncthreads();
    }
    Moments r = sm[0];
    __syncthreads();
    return r;
}

// the curve's scalars from its merged moments
__device__ __forceinline__ CurveStats stats_of(const Moments &m, int phase)
{
    CurveStats s;
    s.mean = m.mean;
    s.var = m.m2 / m.n;
    s.zero_var = (m.m2 > 0.0) ? 0 : 1;
    s.inv_var = s.zero_var ? 0.0 : 1.0 / s.var;
    s.t_min = m.tmin;
    s.t_max = m.tmax;
    s.wsum = m.n;
    s.t_ref = (phase == PH_NAIVE) ? 0.0 : 0.5 * (m.tmin + m.tmax);
    s.pad_ = 0;
    return s;
}

// one sample's record: split time, centred value, recurrence step (cos, sin)
__device__ __forceinline__ void write_record(const Records &rec, int64_t j, double tj, float xj,
                                             const CurveStats &s, double step_df, int phase)
{
    float xv = (float)((double)xj - s.mean);
    if (phase == PH_NAIVE) {
        rec.th[j] = (float)tj;
        rec.tl[j] = 0.0f;
        rec.xv[j] = xv;
        rec.rc[j] = 1.0f;
        rec.rs[j] = 0.0f;
        return;
    }
    const double tp = tj - s.t_ref;
    float th, tl, rc = 1.0f, rs = 0.0f;
    split_time(tp, th, tl);
    if (step_df != 0.0) step_rotation(step_df, tp, rc, rs);  // 0: no kernel of the call reads the step
    rec.th[j] = th;
    rec.tl[j] = tl;
    rec.xv[j] = xv;
    rec.rc[j] = rc;
    rec.rs[j] = rs;
}

// ---------------------------------------------------------------------------
// Main kernel pieces.

// Wave-private LDS tile (one record per lane of the staging wave).
template <int PHASE> struct Tile;
template <> struct alignas(16) Tile<PH_SPLIT> {
    double t[kTile];
    float x[kTile], rc[kTile], rs[kTile];
};
template <> struct alignas(16) Tile<PH_SPLIT32> {
    float th[kTile], tl[kTile];
    float x[kTile], rc[kTile], rs[kTile];
};
template <> struct alignas(16) Tile<PH_NAIVE> {
    float t[kTile];
    float x[kTile];
};

// the record a lane fetches from HBM for the next tile
struct Staged {
    float th, tl, x, rc, rs;
};

// Lanes past the end of the range stage a neutral sample: t' = 0 and x = 0,
// step angle 0.  Its phase is exactly 0 for every frequency, so it adds 0 to
// XC, XS and CS and exactly 1 (up to the rounding of the FP32 sum) to CC; the
// epilogue subtracts the number of such samples from CC.
template <int PHASE>
__device__ __forceinline__ void fetch(const Records &r, int64_t j, bool ok, Staged &s)
{
    if (ok) {
        s.th = r.th[j];
        s.x = r.xv[j];
        if (PHASE != PH_NAIVE) {
            s.tl = r.tl[j];
            s.rc = r.rc[j];
            s.rs = r.rs[j];
        }
    } else {
        s.th = 0.0f;
        s.tl = 0.0f;
        s.x = 0.0f;
        s.rc = 1.0f;
        s.rs = 0.0f;
    }
}

template <int PHASE>
__device__ __forceinline__ void stage(Tile<PHASE> &T, int lane, const Staged &s)
{
    if constexpr (PHASE == PH_SPLIT) {
        T.t[lane] = (double)s.th + (double)s.tl;  // exact: t' = th + tl
        T.x[lane] = s.x;
        T.rc[lane] = s.rc;
        T.rs[lane] = s.rs;
    } else if constexpr (PHASE == PH_SPLIT32) {
        T.th[lane] = s.th;
        T.tl[lane] = s.tl;
        T.x[lane] = s.x;
        T.rc[lane] = s.rc;
        T.rs[lane] = s.rs;
    } else {
        T.t[lane] = s.th;
        T.x[lane] = s.x;
    }
}

// Per-lane frequency constants.  DIRECT keeps all M frequencies, RECUR the
// first only (the others follow from the per-sample step).
template <int PHASE, int TRIG, int M>
struct Freq {
    static constexpr int N = (TRIG == TR_DIRECT) ? M : 1;
    double f[N];
    float fh[N], fl[N];
    __device__ __forceinline__ void set(int m, double fm)
    {
        f[m] = fm;
        fh[m] = (float)fm;
        fl[m] = (float)(fm - (double)fh[m]);
    }
    __device__ __forceinline__ void init(double f_min, double df, int64_t k)
    {
#pragma unroll
        for (int m = 0; m < N; ++m) set(m, f_min + (double)(k + (int64_t)kWave * m) * df);
    }
};

// One sample as read back from LDS.
struct Smp {
    double t;
    float th, tl, x, rc, rs;
};

// reduced phase (revolutions, |phi| <= 1/2 up to rounding) of f t'
template <int PHASE, int TRIG, int M>
__device__ __forceinline__ float phase_of(const Freq<PHASE, TRIG, M> &F, int m, const Smp &s)
{
    if constexpr (PHASE == PH_SPLIT) {
        return rev_reduce(F.f[m] * s.t);
    } else if constexpr (PHASE == PH_SPLIT32) {
#pragma clang fp contract(off)
        // (fh + fl)(th + tl) with fh*th carried exactly: p + e = fh*th (p the
        // rounded product: no contraction of p into the subtractions).  The
        // correction q (at most about half an ulp of p, ~1e-3 revolutions at
        // |p| ~ 3e4) can carry r + q just past 1/2, so the sum is reduced once
        // more (an exact subtraction of 0 or +-1).
        float p = F.fh[m] * s.th;
        float e = __builtin_fmaf(F.fh[m], s.th, -p);
        float r = p - __builtin_rintf(p);
        float q = __builtin_fmaf(F.fh[m], s.tl, e);
        q = __builtin_fmaf(F.fl[m], s.th, q);
        const float v = r + q;
        return v - __builtin_rintf(v);
    } else {
#pragma clang fp contract(off)
        float ft = F.fh[m] * s.th;  // the paper's FP32 reduction of the rounded product
        return ft - __builtin_rintf(ft);
    }
}

template <int M>
__device__ __forceinline__ void acc_term(float (&p)[4][M], int m, float x, float c, float s)
{
    p[0][m] = __builtin_fmaf(x, c, p[0][m]);  // XC
    p[1][m] = __builtin_fmaf(x, s, p[1][m]);  // XS
    p[2][m] = __builtin_fmaf(c, c, p[2][m]);  // CC
    p[3][m] = __builtin_fmaf(c, s, p[3][m]);  // CS
}

// (cos, sin) of 2 pi (f_0 + m S) t' for m = 0 .. M-1, handed to use(m, c, s):
// hardware sin/cos of the seed phase ph (of f_0), one rotation by the step
// (rc, rs) = (cos, sin)(2 pi S t'), then the three-term recurrence
// c_{m+1} = 2 rc c_m - c_{m-1} (and likewise s).
template <int M, class Use>
__device__ __forceinline__ void recur_terms(float ph, float rc, float rs, Use &&use)
{
    float c0 = cos_rev(ph), s0 = sin_rev(ph);
    use(0, c0, s0);
    if constexpr (M > 1) {
        float c1 = __builtin_fmaf(c0, rc, -(s0 * rs));
        float s1 = __builtin_fmaf(s0, rc, c0 * rs);
        use(1, c1, s1);
        const float k2 = rc + rc;
#pragma unroll
        for (int m = 2; m < M; ++m) {
            float c2 = __builtin_fmaf(k2, c1, -c0);
            float s2 = __builtin_fmaf(k2, s1, -s0);
            use(m, c2, s2);
            c0 = c1;
            c1 = c2;
            s0 = s1;
            s1 = s2;
        }
    }
}

// all M terms of one sample for this lane
template <int PHASE, int TRIG, int M>
__device__ __forceinline__ void sample_terms(float (&p)[4][M], const Freq<PHASE, TRIG, M> &F,
                                             const Smp &s)
{
    if constexpr (TRIG == TR_RECUR) {
        recur_terms<M>(phase_of<PHASE, TRIG, M>(F, 0, s), s.rc, s.rs,
                       [&](int m, float c, float sn) { acc_term<M>(p, m, s.x, c, sn); });
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            float ph = phase_of<PHASE, TRIG, M>(F, m, s);
            acc_term<M>(p, m, s.x, cos_rev(ph), sin_rev(ph));
        }
    }
}

// U consecutive samples with broadcast reads (all lanes read one address)
template <int PHASE, int U>
__device__ __forceinline__ void read_smp(const Tile<PHASE> &T, int j, Smp (&s)[U])
{
    if constexpr (U == 4) {
        if constexpr (PHASE == PH_SPLIT) {
            const double2 t01 = *reinterpret_cast<const double2 *>(&T.t[j]);
            const double2 t23 = *reinterpret_cast<const double2 *>(&T.t[j + 2]);
            s[0].t = t01.x; s[1].t = t01.y; s[2].t = t23.x; s[3].t = t23.y;
        } else if constexpr (PHASE == PH_SPLIT32) {
            const float4 h = *reinterpret_cast<const float4 *>(&T.th[j]);
            const float4 l = *reinterpret_cast<const float4 *>(&T.tl[j]);
            s[0].th = h.x; s[1].th = h.y; s[2].th = h.z; s[3].th = h.w;
            s[0].tl = l.x; s[1].tl = l.y; s[2].tl = l.z; s[3].tl = l.w;
        } else {
            const float4 h = *reinterpret_cast<const float4 *>(&T.t[j]);
            s[0].th = h.x; s[1].th = h.y; s[2].th = h.z; s[3].th = h.w;
        }
        const float4 x = *reinterpret_cast<const float4 *>(&T.x[j]);
        s[0].x = x.x; s[1].x = x.y; s[2].x = x.z; s[3].x = x.w;
        if constexpr (PHASE != PH_NAIVE) {
            const float4 c = *reinterpret_cast<const float4 *>(&T.rc[j]);
            const float4 r = *reinterpret_cast<const float4 *>(&T.rs[j]);
            s[0].rc = c.x; s[1].rc = c.y; s[2].rc = c.z; s[3].rc = c.w;
            s[0].rs = r.x; s[1].rs = r.y; s[2].rs = r.z; s[3].rs = r.w;
        }
    } else if constexpr (U == 2) {
        if constexpr (PHASE == PH_SPLIT) {
            const double2 t01 = *reinterpret_cast<const double2 *>(&T.t[j]);
            s[0].t = t01.x; s[1].t = t01.y;
        } else if constexpr (PHASE == PH_SPLIT32) {
            const float2 h = *reinterpret_cast<const float2 *>(&T.th[j]);
            const float2 l = *reinterpret_cast<const float2 *>(&T.tl[j]);
            s[0].th = h.x; s[1].th = h.y;
            s[0].tl = l.x; s[1].tl = l.y;
        } else {
            const float2 h = *reinterpret_cast<const float2 *>(&T.t[j]);
            s[0].th = h.x; s[1].th = h.y;
        }
        const float2 x = *reinterpret_cast<const float2 *>(&T.x[j]);
        s[0].x = x.x; s[1].x = x.y;
        if constexpr (PHASE != PH_NAIVE) {
            const float2 c = *reinterpret_cast<const float2 *>(&T.rc[j]);
            const float2 r = *reinterpret_cast<const float2 *>(&T.rs[j]);
            s[0].rc = c.x; s[1].rc = c.y;
            s[0].rs = r.x; s[1].rs = r.y;
        }
    } else {
        if constexpr (PHASE == PH_SPLIT) {
            s[0].t = T.t[j];
        } else if constexpr (PHASE == PH_SPLIT32) {
            s[0].th = T.th[j];
            s[0].tl = T.tl[j];
        } else {
            s[0].th = T.t[j];
        }
        s[0].x = T.x[j];
        if constexpr (PHASE != PH_NAIVE) {
            s[0].rc = T.rc[j];
            s[0].rs = T.rs[j];
        }
    }
}

// How the FP32 partials of a tile group become the wave's totals.
//   SUM_KAHAN: Kahan-compensated FP32 totals in registers for the sums that
//              cancel (XC, XS, CS), their compensation terms in wave-private
//              LDS (touched only at folds); CC, a sum of squares, needs none;
//   SUM_TWO:   plain FP32 totals (two-level summation, as the paper's chunks).
enum { SUM_KAHAN = 1, SUM_TWO = 2 };

// compensated accumulator slot of sum q (XC 0, XS 1, CS 3), -1 for CC
__device__ __forceinline__ constexpr int comp_slot(int q) { return q == 2 ? -1 : (q == 3 ? 2 : q); }

template <int SUM, int M>
struct Totals {
    float S[4][M];
    float *comp;  // SUM_KAHAN: this wave's [3][M][64] compensation terms in LDS
    int lane;

    __device__ __forceinline__ void init(float *lds_comp, int ln)
    {
        comp = lds_comp;
        lane = ln;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                S[q][m] = 0.0f;
                if constexpr (SUM == SUM_KAHAN)
                    if (comp_slot(q) >= 0) comp[(comp_slot(q) * M + m) * kWave + lane] = 0.0f;
            }
    }

    __device__ __forceinline__ void fold(float (&p)[4][M])
    {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (SUM == SUM_KAHAN && comp_slot(q) >= 0) {
                    float &c = comp[(comp_slot(q) * M + m) * kWave + lane];
                    const float y = p[q][m] - c;
                    const float t = S[q][m] + y;
                    c = (t - S[q][m]) - y;
                    S[q][m] = t;
                } else {
                    S[q][m] += p[q][m];
                }
                p[q][m] = 0.0f;
            }
    }

    // total of accumulator (q, m) in FP64
    __device__ __forceinline__ double value(int q, int m) const
    {
        if (SUM == SUM_KAHAN && comp_slot(q) >= 0)
            return (double)S[q][m] - (double)comp[(comp_slot(q) * M + m) * kWave + lane];
        return (double)S[q][m];
    }
};

template <int SUM, int M>
struct CompLds {
    static constexpr int kFloats = (SUM == SUM_KAHAN) ? kMaxWaves * 3 * M * kWave : 1;
};

// Processes samples [jb, je) for the 64*M frequencies starting at k0 (this
// lane: k0 + lane + 64 m) and leaves the totals in Tot.
template <int PHASE, int TRIG, int M, int U, int SUM>
__device__ __forceinline__ void wave_sums(Tile<PHASE> &T, const Records &rec, int64_t jb, int64_t je,
                                          double f_min, double df, int64_t k0, int lane,
                                          Totals<SUM, M> &Tot)
{
    Freq<PHASE, TRIG, M> F;
    F.init(f_min, df, k0 + lane);
    float p[4][M];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < M; ++m) p[q][m] = 0.0f;
    Staged nx;
    fetch<PHASE>(rec, jb + lane, jb + lane < je, nx);
    int since_fold = 0;
    // whole tiles only: the ragged end is padded with neutral samples (see fetch)
    for (int64_t j0 = jb; j0 < je; j0 += kTile) {
        stage<PHASE>(T, lane, nx);
        __builtin_amdgcn_wave_barrier();
        const int64_t jn = j0 + kTile + lane;
        fetch<PHASE>(rec, jn, jn < je, nx);  // prefetch the next tile
#pragma unroll 1
        for (int j = 0; j < kTile; j += U) {
            Smp s[U];
            read_smp<PHASE, U>(T, j, s);
#pragma unroll
            for (int u = 0; u < U; ++u) sample_terms<PHASE, TRIG, M>(p, F, s[u]);
        }
        __builtin_amdgcn_wave_barrier();
        if (++since_fold == kFoldTiles) {
            Tot.fold(p);
            since_fold = 0;
        }
    }
    Tot.fold(p);
}

// Eqs. (5)-(7) in FP64 from the four sums of Eq. (8) (SS = Nt - CC).
__device__ __forceinline__ float pn_from_sums(double XC, double XS, double CC, double CS, double Nt,
                                              double inv_var)
{
    const double SS = Nt - CC;
    const double d = CC - SS;
    const double two_wt = (CS == 0.0 && d == 0.0) ? 0.0 : atan2(2.0 * CS, d);  // Eq. (6)
    double st, ct;
    sincos(0.5 * two_wt, &st, &ct);                                              // Eq. (7)
    const double Dc = ct * ct * CC + 2.0 * ct * st * CS + st * st * SS;
    const double Ds = ct * ct * SS - 2.0 * ct * st * CS + st * st * CC;
    const double a = ct * XC + st * XS;
    const double b = ct * XS - st * XC;
    const double floor_d = 1e-12 * Nt;
    const double P = 0.5 * ((Dc > floor_d ? a * a / Dc : 0.0) + (Ds > floor_d ? b * b / Ds : 0.0));
    return (float)(P * inv_var);
}

// v[q] += part[(s NV + q) Nf + k] over the chunks s in ascending order (the
// split merge); U chunks' loads are issued together before they are added, so
// that U NV loads per lane are in flight and the sum is the same as one chunk at
// a time
template <int NV, int U>
__device__ __forceinline__ void sum_chunks(const float *__restrict__ part, int splits, int64_t Nf, int64_t k,
                                           double (&v)[NV])
{
    int s = 0;
    for (; s + U <= splits; s += U) {
        float f[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < NV; ++q) f[u][q] = part[((int64_t)(s + u) * NV + q) * Nf + k];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < NV; ++q) v[q] += (double)f[u][q];
    }
    for (; s < splits; ++s)
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] += (double)part[((int64_t)s * NV + q) * Nf + k];
}

// number of neutral samples that pad [0, Nt) to whole tiles
__host__ __device__ __forceinline__ int64_t pad_count(int64_t Nt)
{
    return (Nt + kTile - 1) / kTile * kTile - Nt;
}

}  // namespace lsp
