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
#include "pgram_device.h"

namespace lsp {

// ---------------------------------------------------------------------------
// Prep kernels (single curve).

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
    const Moments m = merge_parts(part, n_part);
    if (threadIdx.x == 0) *st = stats_of(m, phase);
}

// Records, with the scalars merged by every block itself (one launch fewer than
// a separate finalize step); block 0 also stores them for the later kernels.
// The grid is bounded (kRecordBlocks) and strides over the samples, so the
// merge is repeated at most that many times.
constexpr int kRecordBlocks = 1024;

__global__ void __launch_bounds__(256) prep_records_kernel(const double *__restrict__ t,
                                                           const float *__restrict__ x, int64_t Nt,
                                                           const Moments *__restrict__ part, int n_part,
                                                           CurveStats *__restrict__ st, double step_df,
                                                           int phase, Records rec)
{
    const CurveStats s = stats_of(merge_parts(part, n_part), phase);
    if (blockIdx.x == 0 && threadIdx.x == 0) *st = s;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < Nt; j += stride)
        write_record(rec, j, t[j], x[j], s, step_df, phase);
}

static unsigned record_blocks(int64_t Nt)
{
    const int64_t nb = (Nt + 255) / 256;
    return (unsigned)(nb < kRecordBlocks ? (nb > 0 ? nb : 1) : kRecordBlocks);
}

hipError_t launch_prep(const double *t, const float *x, int64_t Nt, double step_df, int phase,
                       Moments *moments, int n_moment_blocks, CurveStats *stats, Records rec,
                       hipStream_t s, hipEvent_t call_start)
{
    launch_timed(prep_moments_kernel, dim3(n_moment_blocks), dim3(256), s, call_start, nullptr, t, x, Nt, moments);
    hipLaunchKernelGGL(prep_records_kernel, dim3(record_blocks(Nt)), dim3(256), 0, s, t, x, Nt,
                       (const Moments *)moments, n_moment_blocks, stats, step_df, phase, rec);
    return hipGetLastError();
}

// the partial moments alone: the matrix-core periodogram merges them and
// converts the samples itself, so it needs no records
hipError_t launch_moment_parts(const double *t, const float *x, int64_t Nt, Moments *moments, int n_moment_blocks,
                               hipStream_t s, hipEvent_t call_start)
{
    launch_timed(prep_moments_kernel, dim3(n_moment_blocks), dim3(256), s, call_start, nullptr, t, x, Nt, moments);
    return hipGetLastError();
}

hipError_t launch_moments(const double *t, const float *x, int64_t Nt, Moments *moments, int n_moment_blocks,
                          CurveStats *stats, hipStream_t s)
{
    hipLaunchKernelGGL(prep_moments_kernel, dim3(n_moment_blocks), dim3(256), 0, s, t, x, Nt, moments);
    hipLaunchKernelGGL(prep_finalize_kernel, dim3(1), dim3(256), 0, s, (const Moments *)moments,
                       n_moment_blocks, (int)PH_NAIVE, stats);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Prep of the generalized periodogram: weighted moments (weights w_j >= 0,
// NULL = all 1), then records t' (split), w_j (y_j - Y) / W and w_j / W.

__global__ void __launch_bounds__(256) prep_moments_w_kernel(const double *__restrict__ t,
                                                             const float *__restrict__ y,
                                                             const float *__restrict__ w, int64_t Nt,
                                                             Moments *__restrict__ out)
{
    Moments m = moments_empty();
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < Nt; j += stride)
        moments_push_w(m, (double)y[j], w ? (double)w[j] : 1.0, t[j]);
    m = block_merge_256(m);
    if (threadIdx.x == 0) out[blockIdx.x] = m;
}

// weighted records; the scalars merged per block as in prep_records_kernel
__global__ void __launch_bounds__(256) prep_records_w_kernel(const double *__restrict__ t,
                                                             const float *__restrict__ y,
                                                             const float *__restrict__ w, int64_t Nt,
                                                             const Moments *__restrict__ part, int n_part,
                                                             CurveStats *__restrict__ st, Records rec,
                                                             uint32_t *__restrict__ refine_count)
{
    const CurveStats s = stats_of(merge_parts(part, n_part), (int)PH_SPLIT);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *st = s;
        if (refine_count) *refine_count = 0u;  // the merge lists ill-conditioned bins from here on
    }
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < Nt; j += stride) {
        split_time(t[j] - s.t_ref, rec.th[j], rec.tl[j]);
        const double wn = (s.wsum > 0.0) ? (w ? (double)w[j] : 1.0) / s.wsum : 0.0;
        rec.xv[j] = (float)(wn * ((double)y[j] - s.mean));
        rec.wv[j] = (float)wn;
    }
}

hipError_t launch_prep_weighted(const double *t, const float *y, const float *w, int64_t Nt, Moments *moments,
                                int n_moment_blocks, CurveStats *stats, Records rec, uint32_t *refine_count,
                                hipStream_t s)
{
    hipLaunchKernelGGL(prep_moments_w_kernel, dim3(n_moment_blocks), dim3(256), 0, s, t, y, w, Nt, moments);
    hipLaunchKernelGGL(prep_records_w_kernel, dim3(record_blocks(Nt)), dim3(256), 0, s, t, y, w, Nt,
                       (const Moments *)moments, n_moment_blocks, stats, rec, refine_count);
    return hipGetLastError();
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

// pads: the neutral samples (t' = 0, x = 0) that the main kernel counted in
// CC, pad_count(Nt) for the vector kernels (whose last chunk is padded to
// whole tiles), 0 for the matrix-core kernel (whose pads add nothing)
__global__ void __launch_bounds__(256) pgram_reduce_kernel(const float *__restrict__ part, int splits,
                                                           int64_t Nf, int64_t Nt, int64_t pads,
                                                           const CurveStats *__restrict__ st,
                                                           float *__restrict__ Pn)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= Nf) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    sum_chunks<4, 8>(part, splits, Nf, k, v);
    v[2] -= (double)pads;
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
    // split phase on the matrix cores (per-chunk FP32 accumulation)
    {PH_SPLIT, TR_MFMA, 32, 1, SUM_TWO, pgram_mfma_kernel, "pgram_mfma_kernel<PH_SPLIT,TR_MFMA,32,1,SUM_TWO>"},
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
    const bool eight = tile.trig == TR_MFMA && tile.waves == 8;  // matrix-core form: also 8 waves
    if (tile.waves != 1 && tile.waves != 2 && tile.waves != 4 && !eight) return false;
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
                        hipEvent_t ev0, hipEvent_t ev1, hipEvent_t call_end)
{
    const Variant *v = find_variant(phase, tile);
    if (!v) return hipErrorInvalidValue;
    const int64_t per_wave = (int64_t)kWave * tile.m;
    const int64_t nfb = (a.Nf + per_wave - 1) / per_wave;
    const int64_t nblk = (nfb + tile.waves - 1) / tile.waves;
    launch_timed(v->fn, dim3((unsigned)nblk, (unsigned)tile.splits), dim3(kWave * tile.waves), s, ev0, ev1, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = (a.Nf + 255) / 256;
    const int64_t pads = (tile.trig == TR_MFMA) ? 0 : pad_count(a.Nt);
    launch_timed(pgram_reduce_kernel, dim3((unsigned)nb), dim3(256), s, nullptr, call_end, (const float *)a.part,
                 (int)tile.splits, a.Nf, a.Nt, pads, (const CurveStats *)a.stats, a.Pn);
    return hipGetLastError();
}

}  // namespace lsp
