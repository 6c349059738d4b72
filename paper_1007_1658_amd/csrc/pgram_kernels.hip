// pgram_kernels.hip -- gfx950 kernels of the direct normalized Lomb-Scargle
// periodogram (Townsend, Section 3, Eqs. (5)-(8) single-pass form).
//
// Work decomposition (CDNA4, wave64):
//   * every wavefront is autonomous: it owns a block of 64*M frequencies
//     (lane l, slot m -> k = k0 + l + 64 m, so each of the M output stores is
//     one coalesced 256-byte row) and one range of samples;
//   * samples stream through a wave-private LDS tile of 64 records (one
//     coalesced global load per lane, prefetched one tile ahead); every lane
//     then reads the same LDS address (broadcast, no bank conflicts), so no
//     workgroup barrier is ever needed;
//   * per term the lane needs (cos, sin) of 2 pi f_k t'_j and four FMAs into
//     XC, XS, CC, CS (SS = Nt - CC, Section 4.4);
//   * FP32 partials are folded every kFoldTiles tiles into Kahan-compensated
//     FP32 totals (their compensation terms wait in wave-private LDS, so they
//     cost no registers) or, as an option, plain two-level FP32 totals; the
//     epilogue (tau by atan2, Eq. (5), 1/variance) is FP64;
//   * when Nf alone cannot fill 256 CUs the sample axis is split over the
//     grid's y dimension; a second kernel adds the per-chunk sums (stored
//     FP32) in FP64 in fixed split order (deterministic) and evaluates the
//     FP64 epilogue.
#include <math.h>

#include "internal.h"

namespace lsp {

enum { PH_SPLIT = LSP_PHASE_SPLIT, PH_NAIVE = LSP_PHASE_NAIVE, PH_SPLIT32 = LSP_PHASE_SPLIT32 };
enum { TR_DIRECT = LSP_TRIG_DIRECT, TR_RECUR = LSP_TRIG_RECUR };

// ---------------------------------------------------------------------------
// hardware sin/cos take their argument in revolutions: sin_rev(r) = sin(2 pi r)
__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

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
__device__ Moments block_merge_256(Moments v)
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

__global__ void __launch_bounds__(256) prep_moments_kernel(const double *__restrict__ t,
                                                           const float *__restrict__ x,
                                                           int64_t Nt, Moments *__restrict__ out)
{
    Moments m = moments_empty();
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < Nt; j += stride)
        moments_push(m, (double)x[j], t[j]);
    m = block_merge_256(m);
    if (threadIdx.x == 0) out[blockIdx.x] = m;
}

__global__ void __launch_bounds__(256) prep_finalize_kernel(const Moments *__restrict__ part, int n_part,
                                                            int phase, CurveStats *__restrict__ st)
{
    Moments m = moments_empty();
    for (int i = threadIdx.x; i < n_part; i += 256) m = moments_merge(m, part[i]);
    m = block_merge_256(m);
    if (threadIdx.x == 0) {
        CurveStats s;
        s.mean = m.mean;
        s.var = m.m2 / m.n;
        s.zero_var = (m.m2 > 0.0) ? 0 : 1;
        s.inv_var = s.zero_var ? 0.0 : 1.0 / s.var;
        s.t_min = m.tmin;
        s.t_max = m.tmax;
        s.t_ref = (phase == PH_NAIVE) ? 0.0 : 0.5 * (m.tmin + m.tmax);
        s.pad_ = 0;
        *st = s;
    }
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
    double tp = tj - s.t_ref;
    float th = (float)tp;
    float tl = (float)(tp - (double)th);
    double q = step_df * tp;  // revolutions of the step angle
    q -= rint(q);
    double sq, cq;
    sincospi(2.0 * q, &sq, &cq);
    rec.th[j] = th;
    rec.tl[j] = tl;
    rec.xv[j] = xv;
    rec.rc[j] = (float)cq;
    rec.rs[j] = (float)sq;
}

__global__ void __launch_bounds__(256) prep_records_kernel(const double *__restrict__ t,
                                                           const float *__restrict__ x, int64_t Nt,
                                                           const CurveStats *__restrict__ st,
                                                           double step_df, int phase, Records rec)
{
    int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= Nt) return;
    CurveStats s = *st;
    write_record(rec, j, t[j], x[j], s, step_df, phase);
}

hipError_t launch_prep(const double *t, const float *x, int64_t Nt, double step_df, int phase,
                       Moments *moments, int n_moment_blocks, CurveStats *stats, Records rec,
                       hipStream_t s)
{
    hipLaunchKernelGGL(prep_moments_kernel, dim3(n_moment_blocks), dim3(256), 0, s, t, x, Nt, moments);
    hipLaunchKernelGGL(prep_finalize_kernel, dim3(1), dim3(256), 0, s, (const Moments *)moments,
                       n_moment_blocks, phase, stats);
    int64_t nb = (Nt + 255) / 256;
    hipLaunchKernelGGL(prep_records_kernel, dim3((unsigned)nb), dim3(256), 0, s, t, x, Nt,
                       (const CurveStats *)stats, step_df, phase, rec);
    return hipGetLastError();
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
    __device__ __forceinline__ void init(double f_min, double df, int64_t k)
    {
#pragma unroll
        for (int m = 0; m < N; ++m) {
            double fm = f_min + (double)(k + (int64_t)kWave * m) * df;
            f[m] = fm;
            fh[m] = (float)fm;
            fl[m] = (float)(fm - (double)fh[m]);
        }
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
        double p = F.f[m] * s.t;
        return (float)(p - rint(p));
    } else if constexpr (PHASE == PH_SPLIT32) {
        // (fh + fl)(th + tl) with fh*th carried exactly: p + e = fh*th
        float p = F.fh[m] * s.th;
        float e = __builtin_fmaf(F.fh[m], s.th, -p);
        float r = p - __builtin_rintf(p);
        float q = __builtin_fmaf(F.fh[m], s.tl, e);
        q = __builtin_fmaf(F.fl[m], s.th, q);
        return r + q;
    } else {
        float ft = F.fh[m] * s.th;  // the paper's FP32 reduction
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

// all M terms of one sample for this lane
template <int PHASE, int TRIG, int M>
__device__ __forceinline__ void sample_terms(float (&p)[4][M], const Freq<PHASE, TRIG, M> &F,
                                             const Smp &s)
{
    if constexpr (TRIG == TR_RECUR) {
        float ph = phase_of<PHASE, TRIG, M>(F, 0, s);
        float c0 = cos_rev(ph), s0 = sin_rev(ph);
        acc_term<M>(p, 0, s.x, c0, s0);
        if constexpr (M > 1) {
            // one exact rotation by the step angle, then the three-term recurrence
            float c1 = __builtin_fmaf(c0, s.rc, -(s0 * s.rs));
            float s1 = __builtin_fmaf(s0, s.rc, c0 * s.rs);
            acc_term<M>(p, 1, s.x, c1, s1);
            const float k2 = s.rc + s.rc;
#pragma unroll
            for (int m = 2; m < M; ++m) {
                float c2 = __builtin_fmaf(k2, c1, -c0);
                float s2 = __builtin_fmaf(k2, s1, -s0);
                acc_term<M>(p, m, s.x, c2, s2);
                c0 = c1;
                c1 = c2;
                s0 = s1;
                s1 = s2;
            }
        }
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

template <int PHASE, int TRIG, int M, int U, int SUM>
__global__ void __launch_bounds__(256) pgram_kernel(PgramArgs a)
{
    __shared__ Tile<PHASE> tiles[kMaxWaves];
    __shared__ float comp_lds[CompLds<SUM, M>::kFloats];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    const int nw = blockDim.x / kWave;
    const int64_t fb = (int64_t)blockIdx.x * nw + wave;
    const int64_t k0 = fb * (int64_t)(kWave * M);
    if (k0 >= a.Nf) return;  // wave-uniform; no workgroup barrier follows
    const int split = blockIdx.y;
    const int64_t jb = (int64_t)split * a.chunk;
    const int64_t je = (jb + a.chunk < a.Nt) ? jb + a.chunk : a.Nt;

    Totals<SUM, M> Tot;
    Tot.init(comp_lds + (SUM == SUM_KAHAN ? wave * 3 * M * kWave : 0), lane);
    wave_sums<PHASE, TRIG, M, U, SUM>(tiles[wave], a.rec, jb, je, a.f_min, a.df, k0, lane, Tot);

    // The chunk's four sums leave as FP32 (one rounding of the compensated
    // total); the FP64 merge and the epilogue run in pgram_reduce_kernel, so the
    // epilogue's FP64 constants never occupy registers during the sample loop.
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int64_t k = k0 + lane + (int64_t)kWave * m;
        if (k < a.Nf) {
#pragma unroll
            for (int q = 0; q < 4; ++q) a.part[((int64_t)split * 4 + q) * a.Nf + k] = (float)Tot.value(q, m);
        }
    }
}

// number of neutral samples that pad [0, Nt) to whole tiles
__host__ __device__ __forceinline__ int64_t pad_count(int64_t Nt)
{
    return (Nt + kTile - 1) / kTile * kTile - Nt;
}

__global__ void __launch_bounds__(256) pgram_reduce_kernel(const float *__restrict__ part, int splits,
                                                           int64_t Nf, int64_t Nt,
                                                           const CurveStats *__restrict__ st,
                                                           float *__restrict__ Pn)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= Nf) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < splits; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += (double)part[((int64_t)s * 4 + q) * Nf + k];
    v[2] -= (double)pad_count(Nt);  // chunks are whole tiles except the last
    Pn[k] = pn_from_sums(v[0], v[1], v[2], v[3], (double)Nt, st->inv_var);
}

// ---------------------------------------------------------------------------
// dispatch table of the built launch shapes

typedef void (*PgramFn)(PgramArgs);

struct Variant {
    int phase, trig, m, unroll, sum;
    PgramFn fn;
    const char *name;
};

#define LSP_V(P, T, M, U, S) \
    {P, T, M, U, S, pgram_kernel<P, T, M, U, S>, "pgram_kernel<" #P "," #T "," #M "," #U "," #S ">"}

static const Variant kVariants[] = {
    // split phase, frequency recurrence, compensated sums
    LSP_V(PH_SPLIT, TR_RECUR, 4, 4, SUM_KAHAN),   LSP_V(PH_SPLIT, TR_RECUR, 8, 4, SUM_KAHAN),
    LSP_V(PH_SPLIT, TR_RECUR, 8, 2, SUM_KAHAN),   LSP_V(PH_SPLIT, TR_RECUR, 12, 2, SUM_KAHAN),
    LSP_V(PH_SPLIT, TR_RECUR, 12, 4, SUM_KAHAN),  LSP_V(PH_SPLIT, TR_RECUR, 14, 2, SUM_KAHAN),
    LSP_V(PH_SPLIT, TR_RECUR, 16, 2, SUM_KAHAN),  LSP_V(PH_SPLIT, TR_RECUR, 16, 1, SUM_KAHAN),
    // split phase, frequency recurrence, two-level sums
    LSP_V(PH_SPLIT, TR_RECUR, 8, 4, SUM_TWO),     LSP_V(PH_SPLIT, TR_RECUR, 12, 2, SUM_TWO),
    LSP_V(PH_SPLIT, TR_RECUR, 14, 2, SUM_TWO),    LSP_V(PH_SPLIT, TR_RECUR, 16, 2, SUM_TWO),
    LSP_V(PH_SPLIT, TR_RECUR, 20, 2, SUM_TWO),    LSP_V(PH_SPLIT, TR_RECUR, 24, 2, SUM_TWO),
    // split phase, direct trigonometry
    LSP_V(PH_SPLIT, TR_DIRECT, 1, 4, SUM_KAHAN),  LSP_V(PH_SPLIT, TR_DIRECT, 2, 4, SUM_KAHAN),
    LSP_V(PH_SPLIT, TR_DIRECT, 4, 4, SUM_KAHAN),
    // all-FP32 split phase
    LSP_V(PH_SPLIT32, TR_RECUR, 8, 4, SUM_KAHAN), LSP_V(PH_SPLIT32, TR_RECUR, 16, 2, SUM_KAHAN),
    LSP_V(PH_SPLIT32, TR_DIRECT, 1, 4, SUM_KAHAN), LSP_V(PH_SPLIT32, TR_DIRECT, 4, 4, SUM_KAHAN),
    // the paper's FP32 arithmetic (two-level sums, as its chunked totals)
    LSP_V(PH_NAIVE, TR_DIRECT, 1, 4, SUM_TWO),    LSP_V(PH_NAIVE, TR_DIRECT, 2, 4, SUM_TWO),
    LSP_V(PH_NAIVE, TR_DIRECT, 4, 4, SUM_TWO),
};

static const Variant *find_variant(int phase, const lsp_tile &t)
{
    for (const Variant &v : kVariants)
        if (v.phase == phase && v.trig == t.trig && v.m == t.m && v.unroll == t.unroll && v.sum == t.sum)
            return &v;
    return nullptr;
}

bool pgram_tile_supported(int phase, const lsp_tile &tile)
{
    if (tile.waves != 1 && tile.waves != 2 && tile.waves != 4) return false;
    if (tile.splits < 1) return false;
    return find_variant(phase, tile) != nullptr;
}

const char *pgram_kernel_name(int phase, const lsp_tile &tile)
{
    const Variant *v = find_variant(phase, tile);
    return v ? v->name : "";
}

// fills unset (zero) unroll/sum fields with the first built variant that matches the rest
void pgram_complete_tile(int phase, lsp_tile &t)
{
    for (const Variant &v : kVariants)
        if (v.phase == phase && v.trig == t.trig && v.m == t.m && (t.unroll == 0 || v.unroll == t.unroll) &&
            (t.sum == 0 || v.sum == t.sum)) {
            t.unroll = v.unroll;
            t.sum = v.sum;
            return;
        }
}

int pgram_list_tiles(int phase, lsp_tile *out, int cap)
{
    int n = 0;
    for (const Variant &v : kVariants)
        if (v.phase == phase) {
            if (out && n < cap) {
                lsp_tile t;
                t.trig = v.trig;
                t.m = v.m;
                t.waves = 0;
                t.splits = 0;
                t.unroll = v.unroll;
                t.sum = v.sum;
                out[n] = t;
            }
            ++n;
        }
    return n;
}

hipError_t pgram_occupancy(int phase, const lsp_tile &tile, int *blocks_per_cu)
{
    const Variant *v = find_variant(phase, tile);
    if (!v) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, v->fn, kWave * tile.waves, 0);
}

hipError_t launch_pgram(const PgramArgs &a, int phase, const lsp_tile &tile, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1)
{
    const Variant *v = find_variant(phase, tile);
    if (!v) return hipErrorInvalidValue;
    const int64_t per_wave = (int64_t)kWave * tile.m;
    const int64_t nfb = (a.Nf + per_wave - 1) / per_wave;
    const int64_t nblk = (nfb + tile.waves - 1) / tile.waves;
    if (ev0) hipEventRecord(ev0, s);
    hipLaunchKernelGGL(v->fn, dim3((unsigned)nblk, (unsigned)tile.splits), dim3(kWave * tile.waves), 0,
                       s, a);
    if (ev1) hipEventRecord(ev1, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = (a.Nf + 255) / 256;
    hipLaunchKernelGGL(pgram_reduce_kernel, dim3((unsigned)nb), dim3(256), 0, s, (const float *)a.part,
                       tile.splits, a.Nf, a.Nt, a.stats, a.Pn);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched: one persistent launch over many curves.

constexpr int kBatchM = 8;
int batched_m() { return kBatchM; }

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

// one 256-thread block per curve: two-pass FP64 moments, then the records
__global__ void __launch_bounds__(256) batch_prep_kernel(BatchArgs a)
{
    const int c = blockIdx.x;
    const BatchCurve cv = a.curves[c];
    const double *t = a.t + cv.off;
    const float *x = a.x + cv.off;
    Moments m = moments_empty();
    for (int64_t j = threadIdx.x; j < cv.Nt; j += 256) moments_push(m, (double)x[j], t[j]);
    m = block_merge_256(m);
    CurveStats s;
    s.mean = m.mean;
    s.var = m.m2 / m.n;
    s.zero_var = (m.m2 > 0.0) ? 0 : 1;
    s.inv_var = s.zero_var ? 0.0 : 1.0 / s.var;
    s.t_min = m.tmin;
    s.t_max = m.tmax;
    s.t_ref = 0.5 * (m.tmin + m.tmax);
    s.pad_ = 0;
    if (threadIdx.x == 0) a.stats[c] = s;
    Records r = a.rec;
    r.th += cv.off;
    r.tl += cv.off;
    r.xv += cv.off;
    r.rc += cv.off;
    r.rs += cv.off;
    const double step_df = (double)kWave * cv.df;
    for (int64_t j = threadIdx.x; j < cv.Nt; j += 256) write_record(r, j, t[j], x[j], s, step_df, PH_SPLIT);
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
        Records r = a.rec;
        r.th += cv.off;
        r.tl += cv.off;
        r.xv += cv.off;
        r.rc += cv.off;
        r.rs += cv.off;
        Totals<SUM_KAHAN, M> Tot;
        Tot.init(comp_lds + wave * 3 * M * kWave, lane);
        wave_sums<PH_SPLIT, TR_RECUR, M, 4, SUM_KAHAN>(tiles[wave], r, 0, cv.Nt, cv.f_min, cv.df, k0, lane,
                                                       Tot);
        const double inv_var = a.stats[item.curve].inv_var;
        unsigned long long best = 0ull;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int64_t k = k0 + lane + (int64_t)kWave * m;
            if (k < cv.Nf) {
                const float P = pn_from_sums(Tot.value(0, m), Tot.value(1, m),
                                             Tot.value(2, m) - (double)pad_count(cv.Nt), Tot.value(3, m),
                                             (double)cv.Nt, inv_var);
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
    a.pmax[c] = zero ? __int_as_float(0x7fc00000) : __uint_as_float((unsigned)(key >> 32));
    if (a.kbest) a.kbest[c] = zero ? -1 : (int64_t)k;
    if (a.fbest) a.fbest[c] = zero ? __longlong_as_double(0x7ff8000000000000ll) : cv.f_min + (double)k * cv.df;
    if (a.t_ns) {
        const unsigned long long t0 = *a.t0;
        a.t_ns[2 * c] = (uint64_t)((double)(a.tbeg[c] - t0) * ns_per_tick);
        a.t_ns[2 * c + 1] = (uint64_t)((double)(a.tend[c] - t0) * ns_per_tick);
    }
}

hipError_t batched_occupancy(int waves, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_pgram_kernel<kBatchM>,
                                                        kWave * waves, 0);
}

hipError_t launch_batched(const BatchArgs &a, int m, int persistent_blocks, int waves, hipStream_t s)
{
    if (m != kBatchM) return hipErrorInvalidValue;
    int dev = 0;
    hipGetDevice(&dev);
    int rate_khz = 0;
    hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
    const double ns_per_tick = rate_khz > 0 ? 1e6 / (double)rate_khz : 10.0;
    const unsigned nb_c = (unsigned)((a.n_curves + 255) / 256);
    hipLaunchKernelGGL(batch_init_kernel, dim3(nb_c), dim3(256), 0, s, a);
    hipLaunchKernelGGL(batch_prep_kernel, dim3((unsigned)a.n_curves), dim3(256), 0, s, a);
    hipLaunchKernelGGL(batch_pgram_kernel<kBatchM>, dim3((unsigned)persistent_blocks), dim3(kWave * waves), 0,
                       s, a);
    hipLaunchKernelGGL(batch_final_kernel, dim3(nb_c), dim3(256), 0, s, a, ns_per_tick);
    return hipGetLastError();
}

}  // namespace lsp
