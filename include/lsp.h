/*
 * lsp.h -- C ABI of libmi355lsp, a gfx950 (MI355X) implementation of the
 * direct O(Nt * Nf) normalized Lomb-Scargle periodogram of Townsend,
 * "Fast Calculation of the Lomb-Scargle Periodogram Using Graphics
 * Processing Units".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named "device" are HIP device memory owned by the caller; the
 *    library never frees or retains them after the call returns (graphs it
 *    caches hold them until the next call with another shape, see
 *    lsp_periodogram_batched).  Pointers named "host" are ordinary host
 *    memory, read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every GPU entry point is asynchronous on that stream unless stated.
 *  - Argument validation is synchronous, happens on the host before any HIP
 *    call, and reports LSP_ERR_INVALID_ARG.  HIP failures report LSP_ERR_HIP;
 *    lsp_last_error() gives the HIP message.
 *  - The frequency grid is f_k = f_min + k * df, k = 0 .. Nf-1, formed from k
 *    in FP64.  The paper's grid (Eq. (9), Section 4.3) is f_min = df;
 *    lsp_grid_paper() builds it from the oversampling and high factors of
 *    Eqs. (10)-(11).
 *  - The series is normalized inside the library (Section 3, opening
 *    paragraph): mean removed, scaled to unit population variance.  So Pn is
 *    invariant to x -> a x + b and 0 <= Pn <= Nt/2.
 *  - Thread safety: calls may come from several host threads; each device
 *    and stream gets its own workspace, guarded by a mutex.
 *  - Graph capture: a call may be captured on a stream (hipStreamBeginCapture,
 *    torch.cuda.graph) once an uncaptured call of at least that size has set
 *    up the stream's workspace (and, for lsp_periodogram_fast, its FFT plan);
 *    a capture that would allocate returns LSP_ERR_CAPTURE.  A workspace a
 *    capture used is never freed: when a later uncaptured call outgrows it,
 *    it is kept aside (until the process ends) so the graph can still replay.
 */
#ifndef MI355LSP_LSP_H
#define MI355LSP_LSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lsp_status {
    LSP_OK = 0,
    LSP_ERR_INVALID_ARG = -1,   /* rejected on the host before any GPU work */
    LSP_ERR_ZERO_VARIANCE = -2, /* x is constant (reported only when checked) */
    LSP_ERR_NO_DEVICE = -3,     /* no HIP device, or not a gfx950 device */
    LSP_ERR_HIP = -4,           /* a HIP runtime call failed */
    LSP_ERR_MODEL = -5,         /* surrogate model missing, corrupt or mismatched */
    LSP_ERR_CAPTURE = -6,       /* the call would allocate while the stream is captured */
    LSP_ERR_UNSUPPORTED = -7    /* option combination not built into the library */
} lsp_status;

/* How the phase f_k * t_j is reduced to revolutions in [-1/2, 1/2] (Section
   4.4 describes the paper's FP32 reduction by the nearest integer). */
typedef enum lsp_phase_mode {
    /* Default.  Times are shifted by t_ref = (t_min + t_max)/2 (Pn does not
       depend on a time shift) and held as t' = t_hi + t_lo (two FP32); the
       product f * t' is formed and reduced in FP64; the reduced phase and all
       trigonometry and sums are FP32. */
    LSP_PHASE_SPLIT = 0,
    /* The paper's arithmetic: raw t rounded to FP32 (epoch included), f in
       FP32, ft - rint(ft) in FP32.  Kept as the comparison baseline; it loses
       accuracy on long or epoch-offset baselines. */
    LSP_PHASE_NAIVE = 1,
    /* Like SPLIT, but the product is an all-FP32 error-free product of
       (f_hi + f_lo)(t_hi + t_lo) (FMA-based two-product), no FP64. */
    LSP_PHASE_SPLIT32 = 2
} lsp_phase_mode;

/* How (cos, sin) of each term are produced. */
typedef enum lsp_trig_mode {
    LSP_TRIG_AUTO = 0,   /* autotuned / heuristic choice */
    /* Every term evaluates its own phase and hardware sin/cos. */
    LSP_TRIG_DIRECT = 1,
    /* Each lane owns m frequencies spaced 64 df apart.  The first is
       evaluated directly per sample, the second by one rotation through the
       per-sample step angle 2 pi 64 df t'_j (computed in FP64 once per
       sample), the rest by the three-term recurrence
       c_{m+1} = 2 cos(step) c_m - c_{m-1} (and likewise for sin).  Re-seeded
       exactly at every sample.  Only with LSP_PHASE_SPLIT / SPLIT32. */
    LSP_TRIG_RECUR = 2,
    /* Matrix cores: with w_a the centre of frequencies 64a .. 64a + 63 and
       v_b = (b + 1/2) dw, b < 32, the sums of Eq. (8) at w_a +- v_b are the
       complex products sum_j [x_j e^{i w_a t'_j}] [e^{i v_b t'_j}] and
       sum_j [x_j e^{i w_a t'_j}] conj[e^{i v_b t'_j}] (and the same at twice
       the angle for CC, CS), both from the same four real products; FP16
       hi/lo operands in three passes with FP32 accumulation
       (v_mfma_f32_32x32x16_f16); one sin/cos pair per (a, j) and per (b, j).
       Only with LSP_PHASE_SPLIT; m = 32 (a wave covers 32 a-rows x 64
       frequencies = 2048), unroll 1, sum TWO. */
    LSP_TRIG_MFMA = 3
} lsp_trig_mode;

/* How each lane's FP32 partial sums (kept over groups of 256 samples) are
   folded into its totals. */
typedef enum lsp_sum_mode {
    LSP_SUM_AUTO = 0,
    LSP_SUM_KAHAN = 1,  /* Kahan-compensated FP32 totals */
    LSP_SUM_TWO = 2     /* plain FP32 totals (two-level summation) */
} lsp_sum_mode;

/* Launch shape of the periodogram kernel.  A zero field = library's choice
   (tuner cache, else heuristic).  lsp_autotune lists what is built. */
typedef struct lsp_tile {
    int32_t trig;   /* lsp_trig_mode */
    int32_t m;      /* frequencies per lane: DIRECT 1,2,4; RECUR 4..24; MFMA 32 */
    int32_t waves;  /* waves (64 lanes each) per workgroup: 1, 2 or 4 (MFMA also 8) */
    int32_t splits; /* workgroups sharing one frequency block along the sample
                       axis (1 = none); partials merged in fixed order in FP64 */
    int32_t unroll; /* samples per broadcast LDS read group: 1, 2 or 4 */
    int32_t sum;    /* lsp_sum_mode */
} lsp_tile;

typedef struct lsp_options {
    int32_t phase;  /* lsp_phase_mode */
    int32_t check;  /* non-zero: synchronize the stream at the end of the call
                       and return LSP_ERR_ZERO_VARIANCE for a constant x */
    lsp_tile tile;  /* all-zero fields = autotuned / heuristic choice */
} lsp_options;

/* ---- single light curve ------------------------------------------------------

   Normalized periodogram of Eq. (1) with tau of Eq. (2), computed in the
   single-pass form of Eqs. (5)-(8) (Section 3): per frequency the sums
   XC, XS, CC, CS over all samples, SS = Nt - CC, then tau from
   tan 2wtau = 2 CS / (CC - SS) (atan2 branch, atan2(0,0) = 0) and Pn by
   Eq. (5).  A term of Eq. (5) whose denominator is <= 1e-12 Nt is 0.

   t   device FP64 [Nt]  sampling times, any order, finite.
   x   device FP32 [Nt]  values, finite.
   Nt  >= 2.
   f_min finite, >= 0;  df finite, > 0;  Nf >= 1.
   Pn  device FP32 [Nf]  output, fully written: Pn[k] = Pn(f_min + k df).
   Errors: LSP_ERR_INVALID_ARG for null pointers or out-of-range sizes;
   a constant x yields Pn = 0 everywhere (LSP_ERR_ZERO_VARIANCE only with
   lsp_options.check). */
lsp_status lsp_periodogram(const double *t, const float *x, int64_t Nt,
                           double f_min, double df, int64_t Nf, float *Pn,
                           void *stream);

/* As lsp_periodogram, with explicit phase mode and launch shape.
   opt may be NULL (defaults).  LSP_ERR_UNSUPPORTED for a tile the library
   was not built with (see lsp_tile) or RECUR with NAIVE phase. */
lsp_status lsp_periodogram_ex(const double *t, const float *x, int64_t Nt,
                              double f_min, double df, int64_t Nf, float *Pn,
                              void *stream, const lsp_options *opt);

/* As lsp_periodogram, for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): the workspace (sample records, curve statistics and per-chunk
   sums) is a fixed array of LSP_NOALLOC_SCRATCH_BYTES that the library
   holds in each GPU's memory until the process ends; no call allocates or
   frees device memory.  The first call on a device (its set-up) looks up
   that device's array address and caches device facts; later calls do no
   host set-up either.  Default phase mode and launch shape, except that the
   sample axis is split into no more chunks than the array holds sums for
   (so results agree with lsp_periodogram to the library's tolerance, not
   always bit for bit).
   Size limit: 5 FP32 records per sample plus 4 FP32 sums per frequency
   (about 20 Nt + 16 Nf bytes, plus alignment) must fit the array, else
   LSP_ERR_INVALID_ARG before any GPU work, with the byte counts in
   lsp_last_error().
   Races: every call on one GPU uses that GPU's one array.  Calls on the same
   stream are ordered; calls that overlap on one GPU (other streams, other
   host threads without ordering) race and corrupt each other's results.
   Arguments, output and other errors as lsp_periodogram. */
#define LSP_NOALLOC_SCRATCH_BYTES (96u * 1024u * 1024u)
lsp_status lsp_periodogram_noalloc(const double *t, const float *x, int64_t Nt,
                                   double f_min, double df, int64_t Nf, float *Pn,
                                   void *stream);

/* Approximate periodogram by extirpolation and FFT (Press & Rybicki 1989,
   the approach Section 1 cites beside the direct sums), for comparison with
   the direct path: x - mean is spread onto a periodic grid of N points
   (period 1/df, N = smallest power of two >= 4 macc f_max/df) with
   the Lagrange weights of the macc nearest points, ones likewise at twice
   the positions; both grids are Fourier transformed (hipFFT, FP64) and
   Eq. (5) is evaluated on bins f_min/df .. f_min/df + Nf - 1.  Everything is
   FP64; the error against the direct sums comes from the spreading only and
   falls with macc (4, 6 or 8).  f_min must be a whole multiple of df.
   Arguments as lsp_periodogram; the grid may need up to 2^28 points
   (LSP_ERR_INVALID_ARG beyond).  The first call for a grid size creates an
   FFT plan (cached per device, stream and size until the process ends).
   Asynchronous on stream otherwise. */
lsp_status lsp_periodogram_fast(const double *t, const float *x, int64_t Nt, double f_min, double df,
                                int64_t Nf, int32_t macc, float *Pn, void *stream);

/* ---- generalized (floating-mean, weighted) periodogram -------------------------

   Section 6.3 points to the generalization of Zechmeister & Kuerster (2009):
   at every frequency the weighted least-squares fit y ~ a cos wt + b sin wt + c
   (the mean is fitted, not removed beforehand), and the power is the fraction
   of the weighted variance of y it explains,
     p = (SS YC^2 + CC YS^2 - 2 CS YC YS) / (YY (CC SS - CS^2)),
   with normalized weights (sum 1), Y = sum w y, YY = sum w (y - Y)^2,
   C = sum w cos, S = sum w sin, YC = sum w (y - Y) cos, YS likewise,
   CC = sum w cos^2 - C^2, SS = sum w sin^2 - S^2, CS = sum w cos sin - C S.
   A degenerate direction (CC or SS <= 1e-5, or CC SS - CS^2 <= 1e-10: f
   near 0, where the FP32 sums cannot resolve them) falls back to the
   one-dimensional fit on the other, else p = 0.  0 <= p <= 1.  Computed on
   the matrix cores (LSP_TRIG_MFMA form with a third complex sum), split phase.

   t  device FP64 [Nt], y device FP32 [Nt], w device FP32 [Nt] weights >= 0
   (e.g. 1/sigma^2) or NULL for equal weights; Nt >= 3; grid as above;
   p device FP32 [Nf] output, fully written.  waves: 0 (library's choice,
   4), 1, 2, 4 or 8 per workgroup (up to 4: conjugate-pair products, one
   wave per SIMD; 8: plain complex products, two per SIMD); splits: 0
   (library's choice) or the number of chunks of the sample axis.  All weights zero or a constant y give p = 0.
   Asynchronous on stream.  Errors: LSP_ERR_INVALID_ARG as above. */
lsp_status lsp_gls(const double *t, const float *y, const float *w, int64_t Nt,
                   double f_min, double df, int64_t Nf, float *p, int32_t waves,
                   int32_t splits, void *stream);

/* Multi-harmonic periodogram (Schwarzenberg-Czerny 1996, also named in
   Section 6.3): the weighted least-squares fit of
     y ~ c + sum_{h=1..K} (a_h cos h wt + b_h sin h wt)
   and p_K = fraction of the weighted variance of y it explains (K = 1 is
   lsp_gls).  Its normal equations need sum w e^{i m wt} for m = 1..2K and
   sum w (y - Y) e^{i h wt} for h = 1..K: 3K complex matrix-core products;
   the (2K x 2K) centred system is solved per frequency in FP64 by Cholesky,
   a column whose pivot falls to <= 1e-5 of its diagonal (or whose diagonal is
   <= 1e-5) being dropped.  K in 1..4 (LSP_ERR_UNSUPPORTED above; K = 3, 4
   take two passes over the samples, six complex sums each at most);
   Nt >= 2K + 1; waves 0 (library's choice, 4), 1, 2 or 4 for K >= 2; other
   arguments as lsp_gls.  The workspace holds 6K floats per frequency and
   sample chunk. */
lsp_status lsp_multiharmonic(const double *t, const float *y, const float *w, int64_t Nt,
                             int32_t K, double f_min, double df, int64_t Nf, float *p,
                             int32_t waves, int32_t splits, void *stream);

/* ---- many light curves in one persistent launch ------------------------------

   Curve c owns samples [off[c], off[c+1]) of t and x and its own grid
   f_min[c] + k df[c], k < Nf[c].  All curves are processed by one
   persistent kernel that takes (curve, frequency block) work items from a
   device queue, longest curves first; the whole sequence (queue reset,
   per-curve normalization, periodogram, per-curve reduction) is captured
   once into a hipGraph per batch shape and replayed on later calls with the
   same shape and pointers.

   t, x      device FP64 / FP32 [off[n]]
   off       host int64 [n+1], off[0] = 0, non-decreasing, each Nt >= 2
   f_min, df host FP64 [n];  Nf host int64 [n] (>= 1)
   Pn        device FP32 [sum Nf] or NULL; curve c at offset sum_{i<c} Nf[i]
   pmax      device FP32 [n]   max_k Pn of curve c (NaN if its x is constant)
   kbest     device int64 [n] or NULL: argmax k, lowest k on exact ties
   fbest     device FP64 [n] or NULL: f_min[c] + kbest df[c]
   t_ns      device uint64 [2n] or NULL: device timestamps (ns, relative to
             the start of the launch) at which curve c's first work item
             started and its last work item finished.
   The call may be captured by the caller (torch.cuda.graph or
   hipStreamBeginCapture) once an uncaptured call with the same shape has
   prepared the stream's workspace; the captured graph keeps reading that
   workspace's plan tables, so a later uncaptured call with another shape on
   the same stream moves to a fresh workspace (the captured one is kept until
   the process ends).  A captured graph and uncaptured calls of the same shape
   share one workspace: replays and calls that overlap in time (on different
   streams) race.
   Errors: LSP_ERR_INVALID_ARG; LSP_ERR_CAPTURE when the stream is being
   captured by the caller and this shape has not been prepared by an
   earlier uncaptured call. */
lsp_status lsp_periodogram_batched(const double *t, const float *x,
                                   const int64_t *off, int32_t n_curves,
                                   const double *f_min, const double *df,
                                   const int64_t *Nf, float *Pn, float *pmax,
                                   int64_t *kbest, double *fbest,
                                   uint64_t *t_ns, void *stream);

/* Kernel form of lsp_periodogram_batched, lsp_mc_maxpower and
   lsp_window_features, process-wide: LSP_TRIG_MFMA (default; a persistent
   workgroup takes (curve, 8192-frequency block) items and runs the
   matrix-core products of LSP_TRIG_MFMA over the whole curve, FP32 sums,
   FP64 epilogue) or LSP_TRIG_RECUR (a persistent wave takes (curve,
   512-frequency block) items; FP32 recurrence with compensated sums).
   LSP_ERR_INVALID_ARG for anything else.  Host-only; do not change it while
   a call on another thread is running. */
lsp_status lsp_set_batched_form(int32_t trig);
int32_t lsp_get_batched_form(void);

/* ---- Monte-Carlo noise periodograms (Section 6.2: simulations of the
   periodogram's statistics are the other use the paper names) ----------------

   For each sampling pattern p (times t[off[p]..off[p+1]), own grid
   f_min[p] + k df[p], k < Nf[p]) and each realization r < R, draws white
   Gaussian values x_j ~ N(0, 1) on the device and returns the maximum of the
   normalized periodogram: pmax[p * R + r].  Deviate j of realization (p, r)
   comes from the Philox4x32-10 counter generator (Salmon et al., SC'11) with
   key `seed` and counter (j, stream_base + p R + r), turned into a normal by
   Box-Muller on 24-bit uniforms; so results do not depend on how calls are
   batched.  t: device FP64; off, f_min, df, Nf: host arrays of the pattern
   shape; pmax: device FP32 [n_pat R].  Asynchronous.  LSP_ERR_INVALID_ARG as
   for lsp_periodogram_batched, or when n_pat R >= 2^31. */
lsp_status lsp_mc_maxpower(const double *t, const int64_t *off, int32_t n_pat,
                           const double *f_min, const double *df, const int64_t *Nf,
                           int32_t R, uint64_t seed, uint64_t stream_base, float *pmax,
                           void *stream);

/* Spectral-window features of each sampling pattern (inputs of the false-alarm
   surrogate).  W(f_k) = |sum_j exp(2 pi i f_k t_j)|^2 on the pattern's grid;
   feat[p*68 + b], b < 64: log10 of mean(W)/Nt over the 64 bands of the
   frequency index k in [round(Nf^(b/64)) - 1, round(Nf^((b+1)/64)) - 1),
   outer edges 0 and Nf (at least one k each); feat[p*68 + 64..67]: log10 Nt, log10 T, gap fraction
   (the spacings longer than five mean spacings, summed, over T; times must be
   sorted), log10 Nf.  feat: device FP32 [n_pat][68].  Asynchronous.
   lsp_mc_maxpower and this call upload their work tables synchronously, so
   neither can be captured: LSP_ERR_CAPTURE on a capturing stream. */
lsp_status lsp_window_features(const double *t, const int64_t *off, int32_t n_pat,
                               const double *f_min, const double *df, const int64_t *Nf,
                               float *feat, void *stream);

/* The first n normal deviates of counter stream `stream_id` under key `seed`,
   exactly as lsp_mc_maxpower draws them (out: device FP32 [n]). */
lsp_status lsp_normals(uint64_t seed, uint64_t stream_id, int64_t n, float *out, void *stream);

/* ---- false-alarm surrogate ---------------------------------------------------------

   Eq. (3) treats the Nf frequencies as independent; with oversampling they are
   not, and the number of independent frequencies has to be simulated (Section
   6.2).  The surrogate learns, per sampling pattern, the law of the maximum
   periodogram power of white noise, from Monte-Carlo maxima made by
   lsp_mc_maxpower.  Network: features (68, standardized) -> 256 -> 256 -> 256 -> 2,
   GELU (tanh form) after the first three layers; products on BF16 matrix
   cores with FP32 accumulation.  With the exponential-equivalent power
   w(z) = -((Nt-3)/2) ln(1 - 2z/Nt) (a single frequency exceeds z with the
   beta-law probability exp(-w), Section 3), the maximum is Gumbel in w:
     P(max <= z) = exp(-exp(-u)),  u = (w(z) - ln Nf - m) / beta,
     m = mu + sigma r_0,  beta = softplus(r_1 + ln(e - 1)),
   so m = 0, beta = 1 is Eq. (3) with Nf independent frequencies.  Training
   minimizes the negative log-likelihood of the Monte-Carlo maxima.  Reported
   quantiles: tau = 0.5, 0.75, 0.9, 0.95, 0.975, 0.99, 0.995, 0.998, 0.999.
   Nt and Nf are read back from the raw features (feat[64] = log10 Nt,
   feat[67] = log10 Nf, as lsp_window_features writes them).  A model is an
   ensemble of `members` independently initialized networks; their spread is
   the uncertainty.  All model entry points are synchronous with respect to
   the model (one model = one user at a time; they lock it). */
typedef struct lsp_model lsp_model;

/* Parameters per member (FP32 master weights): W1[256][68], b1[256],
   W2[256][256], b2, W3[256][256], b3, W4[2][256], b4[2] in this flat order. */
int64_t lsp_model_param_count(void);
/* New model with uniform(+-1/sqrt(fan_in)) weights (0.1x for the last layer),
   zero biases, seeded per member from `seed`.  members in 1..16. */
lsp_status lsp_model_create(int32_t members, uint64_t seed, lsp_model **out);
lsp_status lsp_model_destroy(lsp_model *m);
/* Feature standardization (host FP32 [68] mean and std > 0), the largest
   |standardized feature| accepted before the Monte-Carlo fallback, and the
   location scale (mu, sigma > 0) of the head. */
lsp_status lsp_model_set_scalers(lsp_model *m, const float *feat_mean, const float *feat_std,
                                 float feat_zmax, float q_mu, float q_sigma);
/* FP32 master parameters of one member, flat order above (host [n], n must
   equal lsp_model_param_count()). */
lsp_status lsp_model_get_params(const lsp_model *m, int32_t member, float *host, int64_t n);
lsp_status lsp_model_set_params(lsp_model *m, int32_t member, const float *host, int64_t n);
/* Calibrated standard errors of the law's location m (err_m) and scale beta
   (err_beta), each in [0, 10]: measured against Monte Carlo on patterns kept
   out of training.  lsp_fap_surrogate carries them to each pattern's FAP
   through the law's derivatives there (see lsp_fap_surrogate).  Zeros (the
   default) leave the members' spread alone. */
lsp_status lsp_model_set_law_error(lsp_model *m, float err_m, float err_beta);
/* Binary model file (little-endian): header (version 3), scalers, the two
   law errors, per member the step count and the weights, plus the Adam
   moments when with_optimizer != 0 (version-1 and version-2 files load with
   zero law errors).
   Load reports LSP_ERR_MODEL for a missing, truncated or mismatched file. */
lsp_status lsp_model_save(const lsp_model *m, const char *path, int32_t with_optimizer);
lsp_status lsp_model_load(const char *path, lsp_model **out);

/* The nine quantiles of the maximum under every member's law: feat device
   FP32 [B][68] (raw features), q device FP32 [members][B][9].  Asynchronous
   on stream. */
lsp_status lsp_mlp_forward(lsp_model *m, const float *feat, int32_t B, float *q, void *stream);
/* Forward, negative log-likelihood of R Monte-Carlo maxima per pattern
   (samples device FP32 [B][R], each below Nt/2),
     L = 1/(B R) sum_b sum_r [ln beta_b + u_br + exp(-u_br)],
   and backward of one member.  grad (device FP32 [param_count], flat order)
   and loss (device FP32 [1]) may be NULL; the gradient also stays inside the
   model for lsp_mlp_adam_step.  Asynchronous. */
lsp_status lsp_mlp_grad(lsp_model *m, int32_t member, const float *feat, const float *samples,
                        int32_t R, int32_t B, float *grad, float *loss, void *stream);
/* One Adam step (Kingma & Ba, Algorithm 1, bias-corrected moments) of one
   member with its last gradient; refreshes the BF16 weight copies. */
lsp_status lsp_mlp_adam_step(lsp_model *m, int32_t member, float lr, float beta1, float beta2,
                             float eps, void *stream);
/* The network's matrix product alone: C[M][N] = sum_k A[M][k] B[N][k];
   A, B device BF16 row-major (K contiguous), C device FP32; M, N, K
   multiples of 32.  Asynchronous. */
lsp_status lsp_mlp_gemm_nt(const void *A, const void *B, float *C, int32_t M, int32_t N, int32_t K,
                           void *stream);

/* FAP of observed maxima: for each pattern p (as in lsp_mc_maxpower, times
   sorted, Nt >= 4), fap[p] = P(max Pn of white noise >= p_obs[p]) =
   1 - exp(-exp(-u)) under each member's law; fap is the members' mean.
   fap_err[p] is a per-pattern error bound: 2.576 standard errors (the
   two-sided 99 % point), the standard error being
     sqrt(spread^2 + (err_m dFAP/dm)^2 + (err_beta dFAP/dbeta)^2),
   spread = the members' standard deviation, the derivatives those of the
   law at this pattern's p_obs (dFAP/dm = e^{-u} exp(-e^{-u}) / beta,
   dFAP/dbeta = u dFAP/dm) and err_m, err_beta the model's calibrated law
   errors.  Patterns with fap_err > max_err (the accuracy the caller needs,
   e.g. 0.005), or with a standardized feature beyond the model's range, are
   answered by Monte Carlo instead (mc_realizations draws, key `seed`; fap =
   fraction of maxima >= p_obs, fap_err 2.576 times its binomial standard
   error) and flagged in used_mc (may be NULL; with mc_realizations = 0
   nothing falls back and nothing is flagged).  p_obs, fap, fap_err,
   used_mc: device [n_pat].  Synchronous (the fallback decision reads the
   bounds back). */
lsp_status lsp_fap_surrogate(lsp_model *m, const double *t, const int64_t *off, int32_t n_pat,
                             const double *f_min, const double *df, const int64_t *Nf,
                             const float *p_obs, float *fap, float *fap_err, int32_t *used_mc,
                             float max_err, int32_t mc_realizations, uint64_t seed, void *stream);

/* ---- autotuner -----------------------------------------------------------------

   Times the built launch shapes of the single-curve kernel on synthetic data
   of size (Nt, Nf) on `stream` (synchronous), keeps the fastest in the
   in-memory cache (keyed by device arch, CU count, phase mode and the
   power-of-two buckets of Nt and Nf) and returns it.  Later calls in the
   same buckets with an all-zero tile use it.  best_ms may be NULL. */
lsp_status lsp_autotune(int64_t Nt, int64_t Nf, int32_t phase, void *stream,
                        lsp_tile *best, double *best_ms);
/* The launch shapes built into the library for a phase mode (waves and
   splits are 0 in the listing: 1, 2 or 4 waves, matrix-core shapes also 8, any split count).
   Writes at most cap entries to out (out may be NULL) and returns how many
   exist, or -1 for an unknown phase mode.  Host-only. */
int32_t lsp_list_tiles(int32_t phase, lsp_tile *out, int32_t cap);

/* The cached shape for (Nt, Nf, phase) on the current device, if any:
   LSP_OK and *tile filled, or LSP_ERR_INVALID_ARG when nothing is cached
   (or tile is NULL), LSP_ERR_NO_DEVICE without a gfx950 device. */
lsp_status lsp_tune_lookup(int64_t Nt, int64_t Nf, int32_t phase, lsp_tile *tile);
/* JSON persistence of the tuner cache; path NULL = $LSP_TUNE_CACHE. */
lsp_status lsp_tune_cache_save(const char *path);
lsp_status lsp_tune_cache_load(const char *path);

/* ---- microbenchmarks --------------------------------------------------------------

   Measures one instruction class on the current device with eight
   independent chains per lane and `waves_per_simd` resident waves:
   kind 0 FP32 FMA, 1 FP64 FMA, 2 hardware sin+cos pair, 3 FP64 phase
   reduction (multiply, round to nearest, subtract, convert to FP32);
   matrix-core / vector co-issue: kinds 4, 5, 6, 7 run four independent
   32x32x16 FP16 MFMAs per step with 0, 4, 8, 16 independent FP32 FMAs after
   each and report the MFMA FLOP rate; kind 8 runs kind 7's FMA stream alone
   and reports FMAs per second.  Synchronous on `stream`.  *ops_per_s =
   lane-operations (kinds 4-7: FLOPs) per second; ms may be NULL. */
lsp_status lsp_microbench(int32_t kind, int32_t waves_per_simd, int32_t iters,
                          void *stream, double *ops_per_s, double *ms);

/* ---- probes of the kernels' building blocks ---------------------------------------

   Each probe runs one building block of the periodogram kernels on
   caller-given inputs, one element per lane, with the device code the kernels
   themselves run, so that its error can be measured against an FP64 or 80-bit
   reference.  All pointers are device memory; asynchronous on `stream`;
   n = 0 does nothing.  LSP_ERR_INVALID_ARG for n < 0, NULL pointers (n > 0)
   or non-finite scalars.

   lsp_probe_sincos: s[i] = sin(2 pi r[i]), c[i] = cos(2 pi r[i]) by the
   hardware sine and cosine, which take revolutions (Section 4.4 quotes the
   maximum error of the G80 intrinsic the paper used).  r, s, c: FP32 [n].

   lsp_probe_phase: the reduced phase phi[i] (revolutions, |phi| <= 1/2) of
   frequency f[i] at time t[i] in phase mode `phase` (lsp_phase_mode), with
   the time held as the records hold it: SPLIT and SPLIT32 reduce
   f (t - t_ref) with t - t_ref in FP64 split into two FP32 halves; NAIVE
   reduces fl32(f) fl32(t) in FP32 (t_ref unused).  t, f: FP64 [n]; phi: FP32 [n].

   lsp_probe_recurrence: for each time t[i], the M values
   (c, s)[i M + m] = (cos, sin)(2 pi (f0 + m step_df) (t[i] - t_ref)), m < M,
   as the recurrence form (LSP_TRIG_RECUR) makes them: the hardware sine and
   cosine of the SPLIT phase of f0, one rotation by the per-sample step angle
   2 pi step_df t' (FP64, rounded to FP32), then the three-term recurrence.
   The kernels use step_df = 64 df.  1 <= M <= 32; c, s: FP32 [n M].

   lsp_probe_cmac: one wave of the matrix-core form's complex product,
   P[a][b] = sum_j L[a][j] R[b][j] for a, b < 32 and j < K (Eq. (8)'s sums as
   the products of the k = 64 a + b factorization), with the kernels' operand
   splitting (each value v as hi = fp16(v) plus lo = fp16(v - hi)) and
   accumulation (hi*hi + hi*lo + lo*hi per real product on FP16 matrix cores,
   FP32 sums).  L, R: FP32 complex [32][K] as interleaved (re, im); P: FP32
   complex [32][32].  The kernels scale operands so that |value| <= 2^14.5 and
   the lo halves stay normal.  K a multiple of 16 in [16, 4096].

   lsp_probe_cpair: the same operands through the conjugate-pair products of
   the plain and generalized periodograms' default kernels: the four real
   products A = sum Lr Rr, B = sum Li Ri, C = sum Lr Ri, D = sum Li Rr kept in
   separate accumulators (three FP16 passes each), then
   Pp = sum_j L[a][j] R[b][j] = (A - B, C + D) and
   Pm = sum_j L[a][j] conj(R[b][j]) = (A + B, D - C); Pp, Pm: FP32 complex
   [32][32]. */
lsp_status lsp_probe_sincos(const float *r, int64_t n, float *s, float *c, void *stream);
lsp_status lsp_probe_phase(const double *t, const double *f, int64_t n, double t_ref, int32_t phase,
                           float *phi, void *stream);
lsp_status lsp_probe_recurrence(const double *t, int64_t n, double t_ref, double f0, double step_df,
                                int32_t M, float *c, float *s, void *stream);
lsp_status lsp_probe_cmac(const float *L, const float *R, int32_t K, float *P, void *stream);
lsp_status lsp_probe_cpair(const float *L, const float *R, int32_t K, float *Pp, float *Pm, void *stream);

/* ---- profiling hook ------------------------------------------------------------

   on: 0 = off; bit 0 (1) = every launch of the main periodogram kernel
   carries HIP events for its start and end (of the first and last pass
   where the generalized or multi-harmonic periodogram makes several);
   bit 1 (2) = every lsp_periodogram / lsp_periodogram_ex call carries
   events on its first kernel's start and its last kernel's end.
   lsp_periodogram_noalloc is never profiled (creating events allocates).
   The extended launch takes the events from the dispatches themselves, so
   the stream gets no marker commands; still, on MI355X the main kernel's
   pair delays a c1-sized call by about 5 us and the call pair by about 6 us
   more.  Enabling (or disabling) clears previous records.

   lsp_profile_read synchronizes the main kernel's events and returns the
   total kernel time (ms), the number of launches and the kernel's symbol
   name (truncated to name_len).

   lsp_profile_read_calls: the device time of each recorded call, in call
   order, from the start of its first kernel to the end of its last one.
   Writes min(cap, calls) values to the host array ms (ms may be NULL when
   cap = 0) and the number of calls recorded to *calls.  Synchronizes the
   events it reads.  LSP_ERR_INVALID_ARG for cap < 0 or a NULL ms with
   cap > 0. */
lsp_status lsp_profile_enable(int32_t on);
lsp_status lsp_profile_read(double *total_ms, int64_t *launches, char *name,
                            int32_t name_len);
lsp_status lsp_profile_read_calls(double *ms, int64_t cap, int64_t *calls);

/* ---- host-only helpers (no GPU needed) -------------------------------------------

   Grid of Eqs. (9)-(11): df = 1/(F_over (t_max - t_min)), f_min = df,
   Nf = ceil(F_high F_over Nt / 2), then rounded up to a multiple of round_to
   (>= 1; the paper's kernel needs a multiple of its 256-thread block).
   Errors: LSP_ERR_INVALID_ARG for t_max <= t_min, Nt < 2, F_over <= 0,
   F_high <= 0, round_to < 1 or a null output pointer. */
lsp_status lsp_grid_paper(double t_min, double t_max, int64_t Nt,
                          double F_over, double F_high, int32_t round_to,
                          double *f_min, double *df, int64_t *Nf);

/* Eq. (3): Q = 1 - [1 - (1 - 2 Pn/Nt)^((Nt-3)/2)]^Nf, evaluated with
   log1p/expm1.  NaN when Nt < 4, Nf < 1 or Pn outside [0, Nt/2]. */
double lsp_fap_analytic(double Pn, int64_t Nt, int64_t Nf);

const char *lsp_status_string(lsp_status s);
/* Last HIP error message seen by this host thread ("" if none). */
const char *lsp_last_error(void);
/* Library version string. */
const char *lsp_version(void);
/* Number of visible gfx950 devices (0 when there is none; never fails). */
int32_t lsp_device_count(void);

#ifdef __cplusplus
}
#endif

#endif /* MI355LSP_LSP_H */
