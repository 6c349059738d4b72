// internal.h -- declarations shared by the library's host code and kernels.
// Not part of the public ABI (that is include/lsp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lsp.h"

namespace lsp {

constexpr int kWave = 64;          // gfx950 wavefront width
constexpr int kMaxWaves = 4;       // waves per workgroup of the VALU kernels (matrix-core ones: up to 8)
constexpr int kTile = 64;          // samples staged per wave per tile (one per lane)
constexpr int kFoldTiles = 8;      // tiles between compensated folds of the FP32 partials

// Per-curve scalars written by the prep kernels and read by the rest.
struct CurveStats {
    double mean;     // sample mean of x
    double var;      // population variance of x
    double inv_var;  // 1/var, 0 when var == 0
    double t_ref;    // time origin removed from t (0 in NAIVE mode)
    double t_min, t_max;
    double wsum;     // sum of the weights (Nt when unweighted)
    int32_t zero_var;
    int32_t pad_;
};

// Partial moments of a slice of the series (count, mean, M2, time range),
// merged with Chan et al.'s pairwise update.
struct Moments {
    double n, mean, m2, tmin, tmax;
};

// Per-sample records (SoA, FP32) staged by the periodogram kernels.
struct Records {
    float *th;  // t' hi  (t' = t - t_ref; NAIVE: fl32(t))
    float *tl;  // t' lo  (t' - th, rounded; NAIVE: 0)
    float *xv;  // x - mean
    float *rc;  // cos(2 pi * 64 df * t')  (step of the frequency recurrence)
    float *rs;  // sin(2 pi * 64 df * t')
    float *wv;  // generalized periodogram: normalized weight w_j / sum w (else unused)
};

struct PgramArgs {
    Records rec;
    const CurveStats *stats;
    int64_t Nt;
    int64_t chunk;      // samples per split (multiple of kTile)
    double f_min, df;
    int64_t Nf;
    float *Pn;          // output, written by the reduce/epilogue kernel
    float *part;        // [splits][4][Nf] per-chunk sums (merged in FP64)
    int32_t splits;
    // weighted periodograms: bins whose FP32-derived normal equations are
    // ill-conditioned, listed by the merge for an FP64 recomputation
    uint32_t *refine_list;   // [Nf]
    uint32_t *refine_count;  // [1], zeroed by the weighted prep
    double *refine_part;     // [kRefineBlocks][6 K + 2] partial FP64 sums of a bin split over workgroups
    // single-curve matrix-core form: the raw series and the prep's partial
    // moments; its kernel merges them, converts each sample as the record
    // kernel would, and writes the curve's scalars for the merge
    const double *t_raw;     // [Nt]
    const float *x_raw;      // [Nt]
    const Moments *mom;      // [n_mom]
    int32_t n_mom;
    CurveStats *stats_w;     // = stats, written by workgroup (0, 0)
};

// Batched work item: one wave computes 64*m frequencies of one curve.
struct BatchItem {
    int32_t curve;
    int32_t fblock;
};

// A sampling pattern: a run of times shared by one or more curves (Monte Carlo
// realizations share their pattern's times and time records).
struct BatchGroup {
    int64_t toff;       // first sample in t and in the time records
    int64_t Nt;
    double df;          // grid spacing of its curves (sets the recurrence step)
};

struct BatchCurve {
    int64_t toff;       // first sample in the time records (= its group's)
    int64_t xoff;       // first sample in x / the value records
    int64_t Nt;
    int64_t Nf;
    int64_t pn_off;     // first output frequency in the CSR Pn array
    double f_min, df;
    int32_t group;
    int32_t pad_;
};

// where the values of a batch come from
enum { VAL_INPUT = 0, VAL_NORMAL = 1, VAL_ONES = 2 };
// what the per-frequency epilogue produces
enum { EPI_PN = 0, EPI_WINDOW = 1 };

struct BatchArgs {
    float *th, *tl, *rc, *rs;  // time records, indexed by toff + j
    float *xv;                 // value records, indexed by xoff + j
    CurveStats *stats;         // [n_curves]
    double *t_ref;             // [n_groups]
    const BatchGroup *groups;  // [n_groups]
    int32_t n_groups;
    int32_t n_curves;
    const BatchCurve *curves;  // [n_curves]
    const BatchItem *items;    // [n_items], longest curves first
    int32_t n_items;
    int32_t val_mode;          // VAL_*
    int32_t epi_mode;          // EPI_*
    int32_t pad_;
    uint64_t seed;             // VAL_NORMAL: Philox key
    uint64_t curve_base;       // VAL_NORMAL: counter offset of curve 0
    uint32_t *queue;           // [1] next item
    unsigned long long *key;   // [n] (float bits of max Pn) << 32 | ~k
    unsigned long long *tbeg;  // [n]
    unsigned long long *tend;  // [n]
    unsigned long long *t0;    // [1] launch start
    float *Pn;                 // nullable (EPI_WINDOW: the window power, required)
    float *pmax;               // nullable for EPI_WINDOW
    int64_t *kbest;            // nullable
    double *fbest;             // nullable
    uint64_t *t_ns;            // nullable
    const double *t;           // raw times, indexed by toff + j
    const float *x;            // raw values (VAL_INPUT), indexed by xoff + j
};

// ---- kernel launchers (pgram_kernels.hip) --------------------------------------
hipError_t launch_prep(const double *t, const float *x, int64_t Nt, double step_df,
                       int phase, Moments *moments, int n_moment_blocks,
                       CurveStats *stats, Records rec, hipStream_t s, hipEvent_t call_start = nullptr);
hipError_t launch_pgram(const PgramArgs &a, int phase, const lsp_tile &tile, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1, hipEvent_t call_end = nullptr);
const char *pgram_kernel_name(int phase, const lsp_tile &tile);
bool pgram_tile_supported(int phase, const lsp_tile &tile);
void pgram_complete_tile(int phase, lsp_tile &tile);
int pgram_list_tiles(int phase, lsp_tile *out, int cap);
hipError_t pgram_occupancy(int phase, const lsp_tile &tile, int *blocks_per_cu);

// the matrix-core form of the main kernel (pgram_mfma.hip); 32 a-rows x 64 b per wave
__global__ void pgram_mfma_kernel(PgramArgs a);
// the generalized periodogram (pgram_mfma.hip): weighted prep, matrix-core sums
// (32 a-rows x 32 b per wave, six sums into part[splits][6][Nf]) and FP64 merge
hipError_t launch_prep_weighted(const double *t, const float *y, const float *w, int64_t Nt, Moments *moments,
                                int n_moment_blocks, CurveStats *stats, Records rec, uint32_t *refine_count,
                                hipStream_t s);
hipError_t launch_gls(const PgramArgs &a, int waves, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
// the multi-harmonic periodogram with K = 2 (pgram_mfma.hip): part[splits][12][Nf]
hipError_t launch_mh(const PgramArgs &a, int K, int waves, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
constexpr int kGlsFreqPerWave = 32 * 32;      // generalized periodogram, 8-wave workgroups
constexpr int kGlsPmFreqPerWave = 32 * 64;    // the same on conjugate pairs (up to 4 waves)
constexpr int kMhFreqPerWave = 32 * 64;       // multi-harmonic periodogram (conjugate pairs)
// FP64 recomputation of listed bins: workgroups of the pass (a listed bin is
// split over up to kRefineMaxParts of them when few bins are listed)
constexpr int kRefineBlocks = 256;
constexpr int kRefineMaxParts = 32;
// FP64 recomputation of the bins the weighted merges listed (K = 1: generalized)
hipError_t launch_refine(const PgramArgs &a, int K, hipStream_t s);

// moments and CurveStats only (no records)
hipError_t launch_moment_parts(const double *t, const float *x, int64_t Nt, Moments *moments, int n_moment_blocks,
                               hipStream_t s, hipEvent_t call_start = nullptr);
hipError_t launch_moments(const double *t, const float *x, int64_t Nt, Moments *moments, int n_moment_blocks,
                          CurveStats *stats, hipStream_t s);
// extirpolation + FFT periodogram (fast_kernels.hip): grids = 2 N doubles (values, ones at 2u);
// spectra = 2 (N/2 + 1) complex doubles, the two real-to-complex transforms back to back
hipError_t launch_fast_extirp(const double *t, const float *x, int64_t Nt, const CurveStats *stats, double df,
                              int64_t N, int macc, double *grids, hipStream_t s);
hipError_t launch_fast_epilogue(const void *spectra, int64_t N, int64_t m0, int64_t Nf, int64_t Nt,
                                const CurveStats *stats, float *Pn, hipStream_t s);

// ---- batched launchers (batch_kernels.hip) ---------------------------------------
// form: LSP_TRIG_RECUR (per-wave items of 64 kBatchM frequencies, VALU) or
// LSP_TRIG_MFMA (per-workgroup items of kBatchMfmaFreq frequencies, matrix cores)
hipError_t launch_batched(const BatchArgs &a, int form, int persistent_blocks, int waves,
                          hipStream_t s);
int batched_freq_per_item(int form);
hipError_t batched_occupancy(int form, int waves, int *blocks_per_cu);
// the matrix-core persistent kernel (pgram_mfma.hip), 256 threads per workgroup
constexpr int kBatchMfmaFreq = 4 * 32 * 64;
hipError_t batch_mfma_occupancy(int *blocks_per_cu);
hipError_t launch_batch_mfma(const BatchArgs &a, int persistent_blocks, hipStream_t s);
// window-power band features of each group (curves = groups, EPI_WINDOW done)
hipError_t launch_window_features(const BatchArgs &a, float *feat, int n_feat, hipStream_t s);
// n standard normal deviates of counter stream `curve` (testing the generator)
hipError_t launch_normals(uint64_t seed, uint64_t curve, int64_t n, float *out, hipStream_t s);

constexpr int kWindowBands = 64;    // log-spaced bands of the spectral-window features
constexpr int kFeatures = kWindowBands + 4;

// ---- probes of the kernels' building blocks (probe_kernels.hip) -------------------
hipError_t launch_probe_sincos(const float *r, int64_t n, float *s, float *c, hipStream_t st);
hipError_t launch_probe_phase(const double *t, const double *f, int64_t n, double t_ref, int phase, float *phi,
                              hipStream_t st);
hipError_t launch_probe_recur(const double *t, int64_t n, double t_ref, double f0, double step_df, int M, float *c,
                              float *s, hipStream_t st);
int probe_recur_max();
hipError_t launch_probe_cmac(const float *L, const float *R, int K, float *P, hipStream_t s);
hipError_t launch_probe_cpair(const float *L, const float *R, int K, float *Pp, float *Pm, hipStream_t s);

// records a message for lsp_last_error() on this host thread (lsp_host.cpp)
// device address and size of this GPU's fixed scratch array (noalloc.hip);
// looked up once per device, with that device current
hipError_t noalloc_scratch(int dev, void **ptr, size_t *bytes);

void set_last_error(const char *msg);
void set_last_error(const std::string &msg);

}  // namespace lsp
