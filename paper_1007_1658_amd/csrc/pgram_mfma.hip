// pgram_mfma.hip -- the sums of Eq. (8) as complex matrix products on the
// FP16 matrix cores (v_mfma_f32_32x32x16_f16, FP32 accumulation).
//
// Split the frequency index as k = 64 a + b (b in [0, 64)).  Then
//   f_k t' = F_a t' + b df t',   F_a = f_min + 64 a df,
// and with L_aj = x_j e^{2 pi i F_a t'_j}, R_bj = e^{2 pi i b df t'_j}
//   XC_k + i XS_k = sum_j L_aj R_bj,
//   sum_j e^{2 i w_k t'_j} = sum_j L2_aj R2_bj   (L2, R2: the same at twice the angle),
// so CC = (N + Re)/2 and CS = Im/2 of the second product (Eq. (8) with
// cos^2 = (1 + cos 2wt)/2, cos sin = sin(2wt)/2).  Both are dense products
// over the sample axis of operands that cost one sin/cos pair per (a, j) and
// per (b, j) instead of per (k, j).
//
// Precision: every operand v (|v| <= 1 after scaling) is carried as
// hi + lo, hi = fp16(v), lo = fp16(v - hi), and each real product as
// hi*hi + hi*lo + lo*hi (the dropped lo*lo term is below 2^-22 |v||w|).
// Operands are scaled by powers of two (values by 2^(14-e) with 2^e > max|x|
// over the chunk, trigonometric factors by 2^14) so that the lo parts stay
// in FP16's normal range; the scales are removed exactly at the end.
// Phases are FP64 products (as the SPLIT mode) reduced to [0, 1) revolutions.
//
// Work split: a workgroup of W waves owns a-rows [32 W blockIdx.x, +32 W) and
// all b; wave w owns 32 a-rows (64 frequencies each).  Per block of 64
// samples the workgroup writes the R operands once to LDS (shared by its
// waves); each lane builds its own L operands in registers.
//
// Conjugate pairs (the plain periodogram, mfma_sums_pm): the four real
// products Lr Rr, Li Ri, Lr Ri, Li Rr of a complex product, accumulated
// apart, give L R and L conj(R) alike, i.e. the sums at F_a + beta and at
// F_a - beta.  Centring F_a in its 64 frequencies and taking beta_b =
// (b + 1/2) df for b < 32 then covers all of them with half the matrix work
// and half the R operands of the plain product over b < 64.
//
// The same products give the generalized (floating-mean, weighted)
// periodogram named in Section 6.3 (Zechmeister & Kuerster 2009): with
// normalized weights w_j and weighted-centred values, a third complex sum
// sum_j w_j e^{i w t'_j} supplies C and S, and the double-angle sum is
// weighted (b range 32 there, k = 32a + b, to keep six accumulators).
#include "pgram_device.h"

namespace lsp {

typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kMB = 64;        // samples per LDS block (four K-steps of 16)
constexpr int kMRow = kMB + 8; // halfs per LDS row: 144 B, so 16 lanes' 16-B reads hit distinct banks
constexpr float kTrigScale = 16384.0f;  // 2^14

enum { RR_H = 0, RR_L, RI_H, RI_L, R2R_H, R2R_L, R2I_H, R2I_L, R_KINDS };

constexpr int kMfmaMaxWaves = 8;  // the matrix-core kernels take workgroups of up to 8 waves

template <int NB, bool GLS>
struct MfmaLds {
    double t[kMB];
    float x[kMB];
    float w[kMB];  // GLS: weights; plain: the scale of the R2 operands, 0 for pads
    float red[2][kMfmaMaxWaves];
    alignas(16) _Float16 R[R_KINDS][32 * NB][kMRow];  // 16-B rows: whole-row b128 reads and writes
};

__device__ __forceinline__ void split16(float v, _Float16 &hi, _Float16 &lo)
{
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

// A phase product reduced to [0, 1) revolutions by one v_fract_f64 (the
// hardware sine and cosine take any such argument; one instruction fewer than
// rounding to the nearest integer and subtracting it)
__device__ __forceinline__ float rev_fract(double p) { return (float)__builtin_amdgcn_fract(p); }

// 1.0f in a register the compiler cannot see into (an operand of the split
// sequences below, which take their inputs in registers)
__device__ __forceinline__ float opaque_one()
{
    float one = 1.0f;
    asm volatile("" : "+v"(one));
    return one;
}

// g e^{2i theta} from c = cos theta, s = sin theta: cos 2theta = 2c^2 - 1 and
// sin 2theta = 2cs.  Returns t = 2 g c and the real part t c - g (one product,
// one fused multiply-add); the imaginary part is the product t s, which the
// hi/lo split below forms itself.
__device__ __forceinline__ float double_angle(float c, float g, float &c2g)
{
    const float t = c * (2.0f * g);
    c2g = fmaf(t, c, -g);
    return t;
}

// Debug build (LSP_POISON_LDS): once a block's shared operands have been
// consumed, every byte of the staging area is set to NaN bits before the next
// block is written, so a read that no barrier orders after its write yields
// NaN and fails the parity tests.  A no-op in the normal build.
template <class T>
__device__ __forceinline__ void lds_poison(T &s)
{
#ifdef LSP_POISON_LDS
    uint32_t *p = reinterpret_cast<uint32_t *>(&s);
    for (int i = threadIdx.x; i < (int)(sizeof(T) / 4); i += blockDim.x) p[i] = 0xffffffffu;
    __syncthreads();
#else
    (void)s;
#endif
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ halfx8 neg8(halfx8 v)
{
    return __builtin_bit_cast(halfx8, __builtin_bit_cast(u32x4, v) ^ 0x80008000u);
}

// Two complex products z_i = p_i (c_i + i s_i), i = 0, 1, as FP16 hi/lo
// halves packed two to a register (element i in half i): hi = fp16(p c),
// lo = fp16(p c - hi), each one mixed-precision FMA on the exact product, so
// the product itself is never rounded to FP32.  Written out because the
// compiler forms each hi twice otherwise (once packed, once as the residual's
// operand).  The leading s_nop covers a transcendental result read at once,
// the trailing one the two wait states that a matrix instruction needs before
// it reads a register a vector instruction wrote: hazards the compiler does
// not track through inline assembly.
__device__ __forceinline__ void split_cprod2(float p0, float c0, float s0, float p1, float c1, float s1,
                                             unsigned &rh, unsigned &rl, unsigned &ih, unsigned &il)
{
    asm("s_nop 0\n\t"
        "v_fma_mixlo_f16 %0, %4, %5, 0\n\t"
        "v_fma_mixlo_f16 %2, %4, %6, 0\n\t"
        "v_fma_mixhi_f16 %0, %7, %8, 0\n\t"
        "v_fma_mixhi_f16 %2, %7, %9, 0\n\t"
        "v_fma_mixlo_f16 %1, %4, %5, -%0 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixlo_f16 %3, %4, %6, -%2 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %1, %7, %8, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %3, %7, %9, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]\n\t"
        "s_nop 1"
        : "=&v"(rh), "=&v"(rl), "=&v"(ih), "=&v"(il)
        : "v"(p0), "v"(c0), "v"(s0), "v"(p1), "v"(c1), "v"(s1));
}

// The same for (r_i + i t_i s_i): the real parts r_i given as FP32 values
// (hi by one packed conversion, lo = fp16(r - hi)), the imaginary parts as
// products.
__device__ __forceinline__ void split_csum2(float r0, float r1, float t0, float s0, float t1, float s1, float one,
                                            unsigned &rh, unsigned &rl, unsigned &ih, unsigned &il)
{
    asm("s_nop 0\n\t"
        "v_cvt_pk_f16_f32 %0, %4, %5\n\t"
        "v_fma_mixlo_f16 %2, %6, %7, 0\n\t"
        "v_fma_mixhi_f16 %2, %8, %9, 0\n\t"
        "v_fma_mixlo_f16 %1, %4, %10, -%0 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixlo_f16 %3, %6, %7, -%2 op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %1, %5, %10, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]\n\t"
        "v_fma_mixhi_f16 %3, %8, %9, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]\n\t"
        "s_nop 1"
        : "=&v"(rh), "=&v"(rl), "=&v"(ih), "=&v"(il)
        : "v"(r0), "v"(r1), "v"(t0), "v"(s0), "v"(t1), "v"(s1), "v"(one));
}

__device__ __forceinline__ void put2(halfx8 &v, int k, unsigned d)
{
    u32x4 t = __builtin_bit_cast(u32x4, v);
    t[k] = d;
    v = __builtin_bit_cast(halfx8, t);
}

// the complex operand v = (re, im) of 8 samples as hi/lo FP16 halves, plus -im
// for the real part (filled by set_cprod() / set_csum() for each pair of
// samples, then finish())
struct COp {
    halfx8 rh, rl, ih, il, nih, nil;
    // samples 2k, 2k + 1: v = p (c + i s)
    __device__ __forceinline__ void set_cprod(int k, float p0, float c0, float s0, float p1, float c1, float s1)
    {
        unsigned a, b, c, d;
        split_cprod2(p0, c0, s0, p1, c1, s1, a, b, c, d);
        put2(rh, k, a);
        put2(rl, k, b);
        put2(ih, k, c);
        put2(il, k, d);
    }
    // samples 2k, 2k + 1: v = r + i t s
    __device__ __forceinline__ void set_csum(int k, float r0, float r1, float t0, float s0, float t1, float s1,
                                             float one)
    {
        unsigned a, b, c, d;
        split_csum2(r0, r1, t0, s0, t1, s1, one, a, b, c, d);
        put2(rh, k, a);
        put2(rl, k, b);
        put2(ih, k, c);
        put2(il, k, d);
    }
    // -im from im, a sign flip of both halves of each 32-bit word
    __device__ __forceinline__ void finish()
    {
        nih = neg8(ih);
        nil = neg8(il);
    }
};

// R operands of 8 samples (times t[0..7], one b): R = 2^14 e^{2 pi i b df t'}
// and R2 = g e^{4 pi i b df t'}, as hi/lo halves; g = g2[i] (0 for the pads
// of a ragged block, so that they add nothing to the double-angle sums) or
// 2^14 for g2 = nullptr
__device__ __forceinline__ void build_r8(double bdf, const double *t, const float *g2, float one, COp &R, COp &R2)
{
    const float scale = kTrigScale;
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
        float c[2], s[2], tt[2], c2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const float ph = rev_fract(bdf * t[i + u]);
            c[u] = cos_rev(ph);
            s[u] = sin_rev(ph);
            tt[u] = double_angle(c[u], g2 ? g2[i + u] : kTrigScale, c2[u]);
        }
        R.set_cprod(i / 2, scale, c[0], s[0], scale, c[1], s[1]);
        R2.set_csum(i / 2, c2[0], c2[1], tt[0], s[0], tt[1], s[1], one);
    }
}

// The same for 4 samples, written straight to the LDS staging area (row b,
// samples s0 .. s0+3 of each operand kind)
template <int NBR>
__device__ __forceinline__ void build_r4(double bdf, const double *t, const float *g2, float one,
                                         _Float16 (&R)[R_KINDS][NBR][kMRow], int b, int s0)
{
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    u32x2 v[R_KINDS];
    const float scale = kTrigScale;
#pragma unroll
    for (int i = 0; i < 4; i += 2) {
        float c[2], s[2], tt[2], c2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const float ph = rev_fract(bdf * t[i + u]);
            c[u] = cos_rev(ph);
            s[u] = sin_rev(ph);
            tt[u] = double_angle(c[u], g2 ? g2[i + u] : kTrigScale, c2[u]);
        }
        unsigned p, q, r, w;
        split_cprod2(scale, c[0], s[0], scale, c[1], s[1], p, q, r, w);
        v[RR_H][i / 2] = p;
        v[RR_L][i / 2] = q;
        v[RI_H][i / 2] = r;
        v[RI_L][i / 2] = w;
        split_csum2(c2[0], c2[1], tt[0], s[0], tt[1], s[1], one, p, q, r, w);
        v[R2R_H][i / 2] = p;
        v[R2R_L][i / 2] = q;
        v[R2I_H][i / 2] = r;
        v[R2I_L][i / 2] = w;
    }
#pragma unroll
    for (int k = 0; k < R_KINDS; ++k) *reinterpret_cast<u32x2 *>(&R[k][b][s0]) = v[k];
}

#define LSP_MFMA(A, B, C) C = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, B, C, 0, 0, 0)

// accR += Re(L R), accI += Im(L R), three FP16 passes each
#define LSP_CMAC(L, BRH, BRL, BIH, BIL, ACCR, ACCI)                             \
    do {                                                                       \
        LSP_MFMA(L.rh, BRH, ACCR); LSP_MFMA(L.rh, BIH, ACCI);                  \
        LSP_MFMA(L.rh, BRL, ACCR); LSP_MFMA(L.rh, BIL, ACCI);                  \
        LSP_MFMA(L.rl, BRH, ACCR); LSP_MFMA(L.rl, BIH, ACCI);                  \
        LSP_MFMA(L.nih, BIH, ACCR); LSP_MFMA(L.ih, BRH, ACCI);                 \
        LSP_MFMA(L.nih, BIL, ACCR); LSP_MFMA(L.ih, BRL, ACCI);                 \
        LSP_MFMA(L.nil, BIH, ACCR); LSP_MFMA(L.il, BRH, ACCI);                 \
    } while (0)

// The generalized periodogram's sums, b range 32 (k = 32 a + b): YC + i YS,
// C + i S and sum w e^{2i wt}; slots [C, S, YC, YS, Re/2, Im/2] (weights
// normalized to 1).  Six accumulators of 16.
__device__ __forceinline__ void gls_sums(const PgramArgs &a)
{
    constexpr int NB = 1, BW = 32, NACC = 6;
    __shared__ MfmaLds<NB, true> S;
    const int tid = threadIdx.x;
    const float one = opaque_one();
    const int nw = blockDim.x / kWave;  // waves in the workgroup (1 to 8)
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int half = lane >> 5;   // which 8 samples of a K-step this lane carries
    const int row = lane & 31;    // A: the lane's a-row; B: the lane's b-column
    const int split = blockIdx.y;
    const int64_t jb = (int64_t)split * a.chunk;
    const int64_t je = (jb + a.chunk < a.Nt) ? jb + a.chunk : a.Nt;

    // chunk scales: 2^(14 - e) with max|value| < 2^e (values and weights)
    float mx = 0.f, mw = 0.f;
    for (int64_t j = jb + tid; j < je; j += blockDim.x) {
        mx = fmaxf(mx, fabsf(a.rec.xv[j]));
        mw = fmaxf(mw, a.rec.wv[j]);
    }
    mx = wave_max(mx);
    mw = wave_max(mw);
    if (lane == 0) {
        S.red[0][wave] = mx;
        S.red[1][wave] = mw;
    }
    __syncthreads();
    mx = S.red[0][0];
    mw = S.red[1][0];
    for (int w = 1; w < nw; ++w) {
        mx = fmaxf(mx, S.red[0][w]);
        mw = fmaxf(mw, S.red[1][w]);
    }
    int ex = 0, ew = 0;
    (void)frexpf(mx, &ex);  // mx = m 2^ex, 0.5 <= m < 1 (ex = 0 for mx = 0)
    (void)frexpf(mw, &ew);
    const float xscale = ldexpf(1.0f, 14 - ex);
    const float wscale = ldexpf(1.0f, 14 - ew);

    const int64_t a_row = ((int64_t)blockIdx.x * nw + wave) * 32 + row;
    const double Fa = a.f_min + (double)(a_row * BW) * a.df;

    floatx16 acc[NB][NACC];
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int q = 0; q < NACC; ++q) acc[n][q] = floatx16{};

    for (int64_t j0 = jb; j0 < je; j0 += kMB) {
        __syncthreads();  // the previous block's LDS is consumed
        lds_poison(S);
        if (tid < kMB) {
            const int64_t j = j0 + tid;
            const bool ok = j < je;  // ragged end: neutral samples t' = 0, x = 0, w = 0
            S.t[tid] = ok ? (double)a.rec.th[j] + (double)a.rec.tl[j] : 0.0;
            S.x[tid] = ok ? a.rec.xv[j] * xscale : 0.0f;
            S.w[tid] = ok ? a.rec.wv[j] * wscale : 0.0f;
        }
        __syncthreads();
        // R operands: BW b x 4 groups of 8 samples
        for (int task = tid; task < BW * (kMB / 8); task += blockDim.x) {
            const int b = task / (kMB / 8);
            const int g = task % (kMB / 8);
            const double bdf = (double)b * a.df;
            COp R, R2;
            build_r8(bdf, &S.t[8 * g], nullptr, one, R, R2);
            *reinterpret_cast<halfx8 *>(&S.R[RR_H][b][8 * g]) = R.rh;
            *reinterpret_cast<halfx8 *>(&S.R[RR_L][b][8 * g]) = R.rl;
            *reinterpret_cast<halfx8 *>(&S.R[RI_H][b][8 * g]) = R.ih;
            *reinterpret_cast<halfx8 *>(&S.R[RI_L][b][8 * g]) = R.il;
            *reinterpret_cast<halfx8 *>(&S.R[R2R_H][b][8 * g]) = R2.rh;
            *reinterpret_cast<halfx8 *>(&S.R[R2R_L][b][8 * g]) = R2.rl;
            *reinterpret_cast<halfx8 *>(&S.R[R2I_H][b][8 * g]) = R2.ih;
            *reinterpret_cast<halfx8 *>(&S.R[R2I_L][b][8 * g]) = R2.il;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kMB / 16; ++ks) {
            const int js = 16 * ks + 8 * half;
            // this lane's L operands: a-row `row`, samples js .. js+7
            COp L, L2, LW;
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                float c[2], s[2], t[2], c2[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const float ph = rev_fract(Fa * S.t[js + i + u]);
                    c[u] = cos_rev(ph);
                    s[u] = sin_rev(ph);
                    t[u] = double_angle(c[u], S.w[js + i + u], c2[u]);
                }
                L.set_cprod(i / 2, S.x[js + i], c[0], s[0], S.x[js + i + 1], c[1], s[1]);
                LW.set_cprod(i / 2, S.w[js + i], c[0], s[0], S.w[js + i + 1], c[1], s[1]);
                L2.set_csum(i / 2, c2[0], c2[1], t[0], s[0], t[1], s[1], one);
            }
            L.finish();
            L2.finish();
            LW.finish();
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int bcol = 32 * n + row;
                const halfx8 rrh = *reinterpret_cast<const halfx8 *>(&S.R[RR_H][bcol][js]);
                const halfx8 rrl = *reinterpret_cast<const halfx8 *>(&S.R[RR_L][bcol][js]);
                const halfx8 rih = *reinterpret_cast<const halfx8 *>(&S.R[RI_H][bcol][js]);
                const halfx8 ril = *reinterpret_cast<const halfx8 *>(&S.R[RI_L][bcol][js]);
                const halfx8 qrh = *reinterpret_cast<const halfx8 *>(&S.R[R2R_H][bcol][js]);
                const halfx8 qrl = *reinterpret_cast<const halfx8 *>(&S.R[R2R_L][bcol][js]);
                const halfx8 qih = *reinterpret_cast<const halfx8 *>(&S.R[R2I_H][bcol][js]);
                const halfx8 qil = *reinterpret_cast<const halfx8 *>(&S.R[R2I_L][bcol][js]);
                LSP_CMAC(LW, rrh, rrl, rih, ril, acc[n][0], acc[n][1]);
                LSP_CMAC(L, rrh, rrl, rih, ril, acc[n][2], acc[n][3]);
                LSP_CMAC(L2, qrh, qrl, qih, qil, acc[n][4], acc[n][5]);
            }
        }
    }

    const float ux = ldexpf(1.0f, ex - 28);   // 1 / (xscale 2^14)
    const float uw = ldexpf(1.0f, ew - 28);   // 1 / (wscale 2^14)
#pragma unroll
    for (int n = 0; n < NB; ++n)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t ar = ((int64_t)blockIdx.x * nw + wave) * 32 + 8 * (r / 4) + 4 * half + (r % 4);
            const int64_t k = ar * BW + 32 * n + row;
            if (k < a.Nf) {
                float *p = a.part + (int64_t)split * 6 * a.Nf + k;
                p[0] = acc[n][0][r] * uw;
                p[a.Nf] = acc[n][1][r] * uw;
                p[2 * a.Nf] = acc[n][2][r] * ux;
                p[3 * a.Nf] = acc[n][3][r] * ux;
                p[4 * a.Nf] = 0.5f * acc[n][4][r] * uw;
                p[5 * a.Nf] = 0.5f * acc[n][5][r] * uw;
            }
        }
}

// acc A += sum Lr Rr, B += sum Li Ri, C += sum Lr Ri, D += sum Li Rr, each in
// three FP16 passes (hi x hi, hi x lo, lo x hi)
#define LSP_PMAC(L, RRH, RRL, RIH, RIL, A, B, C, D)                             \
    do {                                                                       \
        LSP_MFMA(L.rh, RRH, A); LSP_MFMA(L.ih, RIH, B);                        \
        LSP_MFMA(L.rh, RIH, C); LSP_MFMA(L.ih, RRH, D);                        \
        LSP_MFMA(L.rh, RRL, A); LSP_MFMA(L.ih, RIL, B);                        \
        LSP_MFMA(L.rh, RIL, C); LSP_MFMA(L.ih, RRL, D);                        \
        LSP_MFMA(L.rl, RRH, A); LSP_MFMA(L.il, RIH, B);                        \
        LSP_MFMA(L.rl, RIH, C); LSP_MFMA(L.il, RRH, D);                        \
    } while (0)

// The conjugate-pair products of one K-step: acc[0..3] += A, B, C, D of L R
// (A = sum Lr Rr, B = sum Li Ri, C = sum Lr Ri, D = sum Li Rr), acc[4..7] the
// same of L2 R2, each real product as hi x hi + hi x lo + lo x hi; R operands
// of b-column `row` from the LDS staging area
template <int NBR>
__device__ __forceinline__ void pm_products(const COp &L, const COp &L2, const _Float16 (&R)[R_KINDS][NBR][kMRow],
                                            int row, int js, floatx16 (&acc)[8])
{
    const halfx8 rrh = *reinterpret_cast<const halfx8 *>(&R[RR_H][row][js]);
    const halfx8 rrl = *reinterpret_cast<const halfx8 *>(&R[RR_L][row][js]);
    const halfx8 rih = *reinterpret_cast<const halfx8 *>(&R[RI_H][row][js]);
    const halfx8 ril = *reinterpret_cast<const halfx8 *>(&R[RI_L][row][js]);
    const halfx8 qrh = *reinterpret_cast<const halfx8 *>(&R[R2R_H][row][js]);
    const halfx8 qrl = *reinterpret_cast<const halfx8 *>(&R[R2R_L][row][js]);
    const halfx8 qih = *reinterpret_cast<const halfx8 *>(&R[R2I_H][row][js]);
    const halfx8 qil = *reinterpret_cast<const halfx8 *>(&R[R2I_L][row][js]);
    LSP_MFMA(L.rh, rrh, acc[0]); LSP_MFMA(L.ih, rih, acc[1]);
    LSP_MFMA(L.rh, rih, acc[2]); LSP_MFMA(L.ih, rrh, acc[3]);
    LSP_MFMA(L2.rh, qrh, acc[4]); LSP_MFMA(L2.ih, qih, acc[5]);
    LSP_MFMA(L2.rh, qih, acc[6]); LSP_MFMA(L2.ih, qrh, acc[7]);
    LSP_MFMA(L.rh, rrl, acc[0]); LSP_MFMA(L.ih, ril, acc[1]);
    LSP_MFMA(L.rh, ril, acc[2]); LSP_MFMA(L.ih, rrl, acc[3]);
    LSP_MFMA(L2.rh, qrl, acc[4]); LSP_MFMA(L2.ih, qil, acc[5]);
    LSP_MFMA(L2.rh, qil, acc[6]); LSP_MFMA(L2.ih, qrl, acc[7]);
    LSP_MFMA(L.rl, rrh, acc[0]); LSP_MFMA(L.il, rih, acc[1]);
    LSP_MFMA(L.rl, rih, acc[2]); LSP_MFMA(L.il, rrh, acc[3]);
    LSP_MFMA(L2.rl, qrh, acc[4]); LSP_MFMA(L2.il, qih, acc[5]);
    LSP_MFMA(L2.rl, qih, acc[6]); LSP_MFMA(L2.il, qrh, acc[7]);
}

// The sums of Eq. (8) for the plain periodogram.  The four real products of
// each complex product are kept apart,
//   A = sum Lr Rr, B = sum Li Ri, C = sum Lr Ri, D = sum Li Rr,
// and give both L R (A - B, C + D) and L conj(R) (A + B, D - C), i.e. the
// sums at F_a + beta_b and at F_a - beta_b.  With F_a = f_min + (64 a + 31.5) df
// and beta_b = (b + 1/2) df, b < 32, the two cover k = 64 a + 32 + b and
// k = 64 a + 31 - b: all 64 frequencies of the a-row from one 32-wide b
// range.  Same for the double-angle product.  Eight accumulators of 16 (a
// 32 x 32 tile each), as many as a complex product over b < 64 holds for the
// same frequencies, with 24 instead of 48 matrix instructions per K-step,
// half the R operands and no negated operands.
__device__ __forceinline__ void mfma_sums_pm(const PgramArgs &a)
{
    __shared__ MfmaLds<1, false> S;
    const int tid = threadIdx.x;
    const float one = opaque_one();
    const int nw = blockDim.x / kWave;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int half = lane >> 5;   // which 8 samples of a K-step this lane carries
    const int row = lane & 31;    // A: the lane's a-row; B: the lane's b-column
    const int split = blockIdx.y;
    const int64_t jb = (int64_t)split * a.chunk;
    const int64_t je = (jb + a.chunk < a.Nt) ? jb + a.chunk : a.Nt;

    // the chunk's range of raw values (before the curve's mean is known: the
    // centred values' extremes are those of the raw ones, rounding being
    // monotonic), and the first block's samples, loaded into registers one
    // block ahead so that global-memory latency overlaps other work
    float xlo = INFINITY, xhi = -INFINITY;
    for (int64_t j = jb + tid; j < je; j += blockDim.x) {
        const float v = a.x_raw[j];
        xlo = fminf(xlo, v);
        xhi = fmaxf(xhi, v);
    }
    double pt = 0.0;
    float px = 0.f;
    bool pok = false;
    if (tid < kMB) {
        const int64_t j = jb + tid;
        pok = j < je;
        if (pok) {
            pt = a.t_raw[j];
            px = a.x_raw[j];
        }
    }
    // the curve's mean and time reference, merged from the prep's partial
    // moments in the record kernel's order (the same bits in every workgroup)
    const CurveStats cs = stats_of(merge_parts(a.mom, a.n_mom), (int)PH_SPLIT);
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) *a.stats_w = cs;

    // chunk scale: 2^(14 - e) with max|x - mean| < 2^e, the centred values
    // rounded to FP32 as the records hold them
    xlo = -wave_max(-xlo);
    xhi = wave_max(xhi);
    if (lane == 0) {
        S.red[0][wave] = xhi;
        S.red[1][wave] = xlo;
    }
    __syncthreads();
    xhi = S.red[0][0];
    xlo = S.red[1][0];
    for (int w = 1; w < nw; ++w) {
        xhi = fmaxf(xhi, S.red[0][w]);
        xlo = fminf(xlo, S.red[1][w]);
    }
    const float mx = (xlo <= xhi) ? fmaxf(fabsf((float)((double)xhi - cs.mean)), fabsf((float)((double)xlo - cs.mean)))
                                  : 0.0f;
    int ex = 0;
    (void)frexpf(mx, &ex);
    const float xscale = ldexpf(1.0f, 14 - ex);

    const int64_t a_row = ((int64_t)blockIdx.x * nw + wave) * 32 + row;
    const double Fa = a.f_min + ((double)(a_row * 64) + 31.5) * a.df;

    // [A, B, C, D] of L R, then of L2 R2
    floatx16 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = floatx16{};

    for (int64_t j0 = jb; j0 < je; j0 += kMB) {
        __syncthreads();  // the previous block's LDS is consumed
        lds_poison(S);
        if (tid < kMB) {
            // t' = t - t_ref split into FP32 hi + lo and x - mean rounded to
            // FP32, as the record kernel writes them; ragged end: neutral
            // samples t' = 0, x = 0, and a double-angle scale of 0 so that
            // they add nothing to CC
            float th = 0.f, tl = 0.f;
            if (pok) split_time(pt - cs.t_ref, th, tl);
            S.t[tid] = pok ? (double)th + (double)tl : 0.0;
            S.x[tid] = pok ? (float)((double)px - cs.mean) * xscale : 0.0f;
            S.w[tid] = pok ? kTrigScale : 0.0f;  // R2 of the pads: 0
            const int64_t j = j0 + kMB + tid;
            pok = j < je;
            if (pok) {
                pt = a.t_raw[j];
                px = a.x_raw[j];
            }
        }
        __syncthreads();
        // R operands: 32 b x 16 groups of 4 samples, beta_b = (b + 1/2) df,
        // one task per thread of an 8-wave workgroup
        for (int task = tid; task < 32 * (kMB / 4); task += blockDim.x) {
            const int b = task / (kMB / 4);
            const int g = task % (kMB / 4);
            build_r4(((double)b + 0.5) * a.df, &S.t[4 * g], &S.w[4 * g], one, S.R, b, 4 * g);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kMB / 16; ++ks) {
            const int js = 16 * ks + 8 * half;
            COp L, L2;
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                float c[2], s[2], t[2], c2[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const float ph = rev_fract(Fa * S.t[js + i + u]);
                    c[u] = cos_rev(ph);
                    s[u] = sin_rev(ph);
                    t[u] = double_angle(c[u], kTrigScale, c2[u]);
                }
                L.set_cprod(i / 2, S.x[js + i], c[0], s[0], S.x[js + i + 1], c[1], s[1]);
                L2.set_csum(i / 2, c2[0], c2[1], t[0], s[0], t[1], s[1], one);
            }
            pm_products(L, L2, S.R, row, js, acc);
        }
    }

    // FP32 chunk sums, scales removed (the pads of the last block add
    // nothing, and the merge subtracts none for this kernel)
    const float ux = ldexpf(1.0f, ex - 28);   // 1 / (xscale 2^14)
    const float uz = 1.0f / (kTrigScale * kTrigScale);
    const float count = (float)(je - jb);
    float *part = a.part + (int64_t)split * 4 * a.Nf;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t ar = ((int64_t)blockIdx.x * nw + wave) * 32 + 8 * (r / 4) + 4 * half + (r % 4);
        const float A = acc[0][r], B = acc[1][r], C = acc[2][r], D = acc[3][r];
        const float A2 = acc[4][r], B2 = acc[5][r], C2 = acc[6][r], D2 = acc[7][r];
        const int64_t kp = ar * 64 + 32 + row;  // F_a + beta_b: L R
        const int64_t km = ar * 64 + 31 - row;  // F_a - beta_b: L conj(R)
        if (kp < a.Nf) {
            float *p = part + kp;
            p[0] = (A - B) * ux;
            p[a.Nf] = (C + D) * ux;
            p[2 * a.Nf] = 0.5f * (count + (A2 - B2) * uz);
            p[3 * a.Nf] = 0.5f * (C2 + D2) * uz;
        }
        if (km < a.Nf) {
            float *p = part + km;
            p[0] = (A + B) * ux;
            p[a.Nf] = (D - C) * ux;
            p[2 * a.Nf] = 0.5f * (count + (A2 + B2) * uz);
            p[3 * a.Nf] = 0.5f * (D2 - C2) * uz;
        }
    }
}

// The generalized periodogram's sums on conjugate pairs (as mfma_sums_pm):
// LW R, L R and L2W R2 with L = x e^{i theta}, LW = w e^{i theta},
// L2W = w e^{2 i theta}, each as its four real products, so that one 32-wide
// b range gives the a-row's 64 frequencies F_a +- beta_b.  Twelve
// accumulators of 16 need one wave per SIMD (workgroups of at most 4 waves).
// Slots as gls_sums: [C, S, YC, YS, Re/2, Im/2] of sum w e^{2i wt}.
__device__ __forceinline__ void gls_sums_pm(const PgramArgs &a)
{
    __shared__ MfmaLds<1, true> S;
    const int tid = threadIdx.x;
    const float one = opaque_one();
    const int nw = blockDim.x / kWave;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int half = lane >> 5;
    const int row = lane & 31;
    const int split = blockIdx.y;
    const int64_t jb = (int64_t)split * a.chunk;
    const int64_t je = (jb + a.chunk < a.Nt) ? jb + a.chunk : a.Nt;

    // chunk scales: 2^(14 - e) with max|value| < 2^e (values and weights)
    float mx = 0.f, mw = 0.f;
    for (int64_t j = jb + tid; j < je; j += blockDim.x) {
        mx = fmaxf(mx, fabsf(a.rec.xv[j]));
        mw = fmaxf(mw, a.rec.wv[j]);
    }
    mx = wave_max(mx);
    mw = wave_max(mw);
    if (lane == 0) {
        S.red[0][wave] = mx;
        S.red[1][wave] = mw;
    }
    __syncthreads();
    mx = S.red[0][0];
    mw = S.red[1][0];
    for (int w = 1; w < nw; ++w) {
        mx = fmaxf(mx, S.red[0][w]);
        mw = fmaxf(mw, S.red[1][w]);
    }
    int ex = 0, ew = 0;
    (void)frexpf(mx, &ex);
    (void)frexpf(mw, &ew);
    const float xscale = ldexpf(1.0f, 14 - ex);
    const float wscale = ldexpf(1.0f, 14 - ew);

    const int64_t a_row = ((int64_t)blockIdx.x * nw + wave) * 32 + row;
    const double Fa = a.f_min + ((double)(a_row * 64) + 31.5) * a.df;

    floatx16 acc[12];  // [A, B, C, D] of LW R, of L R, of L2W R2
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = floatx16{};

    for (int64_t j0 = jb; j0 < je; j0 += kMB) {
        __syncthreads();  // the previous block's LDS is consumed
        lds_poison(S);
        if (tid < kMB) {
            const int64_t j = j0 + tid;
            const bool ok = j < je;  // ragged end: neutral samples t' = 0, x = 0, w = 0
            S.t[tid] = ok ? (double)a.rec.th[j] + (double)a.rec.tl[j] : 0.0;
            S.x[tid] = ok ? a.rec.xv[j] * xscale : 0.0f;
            S.w[tid] = ok ? a.rec.wv[j] * wscale : 0.0f;
        }
        __syncthreads();
        for (int task = tid; task < 32 * (kMB / 4); task += blockDim.x) {
            const int b = task / (kMB / 4);
            const int g = task % (kMB / 4);
            build_r4(((double)b + 0.5) * a.df, &S.t[4 * g], nullptr, one, S.R, b, 4 * g);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kMB / 16; ++ks) {
            const int js = 16 * ks + 8 * half;
            COp L, LW, L2;
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                float c[2], s[2], t[2], c2[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const float ph = rev_fract(Fa * S.t[js + i + u]);
                    c[u] = cos_rev(ph);
                    s[u] = sin_rev(ph);
                    t[u] = double_angle(c[u], S.w[js + i + u], c2[u]);
                }
                L.set_cprod(i / 2, S.x[js + i], c[0], s[0], S.x[js + i + 1], c[1], s[1]);
                LW.set_cprod(i / 2, S.w[js + i], c[0], s[0], S.w[js + i + 1], c[1], s[1]);
                L2.set_csum(i / 2, c2[0], c2[1], t[0], s[0], t[1], s[1], one);
            }
            const halfx8 rrh = *reinterpret_cast<const halfx8 *>(&S.R[RR_H][row][js]);
            const halfx8 rrl = *reinterpret_cast<const halfx8 *>(&S.R[RR_L][row][js]);
            const halfx8 rih = *reinterpret_cast<const halfx8 *>(&S.R[RI_H][row][js]);
            const halfx8 ril = *reinterpret_cast<const halfx8 *>(&S.R[RI_L][row][js]);
            LSP_PMAC(LW, rrh, rrl, rih, ril, acc[0], acc[1], acc[2], acc[3]);
            LSP_PMAC(L, rrh, rrl, rih, ril, acc[4], acc[5], acc[6], acc[7]);
            const halfx8 qrh = *reinterpret_cast<const halfx8 *>(&S.R[R2R_H][row][js]);
            const halfx8 qrl = *reinterpret_cast<const halfx8 *>(&S.R[R2R_L][row][js]);
            const halfx8 qih = *reinterpret_cast<const halfx8 *>(&S.R[R2I_H][row][js]);
            const halfx8 qil = *reinterpret_cast<const halfx8 *>(&S.R[R2I_L][row][js]);
            LSP_PMAC(L2, qrh, qrl, qih, qil, acc[8], acc[9], acc[10], acc[11]);
        }
    }

    const float ux = ldexpf(1.0f, ex - 28);   // 1 / (xscale 2^14)
    const float uw = ldexpf(1.0f, ew - 28);   // 1 / (wscale 2^14)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t ar = ((int64_t)blockIdx.x * nw + wave) * 32 + 8 * (r / 4) + 4 * half + (r % 4);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            // n = 0: F_a + beta_b (L R), n = 1: F_a - beta_b (L conj(R))
            const int64_t k = n == 0 ? ar * 64 + 32 + row : ar * 64 + 31 - row;
            if (k < a.Nf) {
                const float sg = n == 0 ? -1.0f : 1.0f;
                float *p = a.part + (int64_t)split * 6 * a.Nf + k;
                p[0] = (acc[0][r] + sg * acc[1][r]) * uw;
                p[a.Nf] = (n == 0 ? acc[2][r] + acc[3][r] : acc[3][r] - acc[2][r]) * uw;
                p[2 * a.Nf] = (acc[4][r] + sg * acc[5][r]) * ux;
                p[3 * a.Nf] = (n == 0 ? acc[6][r] + acc[7][r] : acc[7][r] - acc[6][r]) * ux;
                p[4 * a.Nf] = 0.5f * (acc[8][r] + sg * acc[9][r]) * uw;
                p[5 * a.Nf] = 0.5f * (n == 0 ? acc[10][r] + acc[11][r] : acc[11][r] - acc[10][r]) * uw;
            }
        }
    }
}

// Probe of the matrix-core complex product on caller-given operands: one wave
// forms P[a][b] = sum_j L[a][j] R[b][j] (a, b < 32, j < 16 K-steps of 16 j each,
// i.e. K = 16 ks) with the kernels' own operand splitting (COp: hi/lo halves,
// the -im halves by sign flip) and accumulation (LSP_CMAC: three FP16 passes
// per real product into FP32).  L, R: FP32 complex [32][K] as (re, im) pairs;
// P: FP32 complex [32][32].
__global__ void __launch_bounds__(64) probe_cmac_kernel(const float *__restrict__ L, const float *__restrict__ R,
                                                        int K, float *__restrict__ P)
{
    const int lane = threadIdx.x;
    const int half = lane >> 5;
    const int row = lane & 31;
    const float one = opaque_one();
    floatx16 accR = floatx16{}, accI = floatx16{};
    for (int j0 = 0; j0 < K; j0 += 16) {
        const int js = j0 + 8 * half;
        COp A, B;
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            const float *la = L + 2 * ((int64_t)row * K + js + i);
            const float *rb = R + 2 * ((int64_t)row * K + js + i);
            A.set_cprod(i / 2, one, la[0], la[1], one, la[2], la[3]);
            B.set_cprod(i / 2, one, rb[0], rb[1], one, rb[2], rb[3]);
        }
        A.finish();
        LSP_CMAC(A, B.rh, B.rl, B.ih, B.il, accR, accI);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int a = 8 * (r / 4) + 4 * half + (r % 4);
        float *o = P + 2 * (a * 32 + row);
        o[0] = accR[r];
        o[1] = accI[r];
    }
}

// The same operands through the conjugate-pair products of the plain and
// generalized kernels: the four real products accumulated apart (LSP_PMAC),
// then Pp = sum L R = (A - B, C + D) and Pm = sum L conj(R) = (A + B, D - C).
__global__ void __launch_bounds__(64) probe_cpair_kernel(const float *__restrict__ L, const float *__restrict__ R,
                                                         int K, float *__restrict__ Pp, float *__restrict__ Pm)
{
    const int lane = threadIdx.x;
    const int half = lane >> 5;
    const int row = lane & 31;
    const float one = opaque_one();
    floatx16 A = floatx16{}, B = floatx16{}, C = floatx16{}, D = floatx16{};
    for (int j0 = 0; j0 < K; j0 += 16) {
        const int js = j0 + 8 * half;
        COp X, Y;
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            const float *la = L + 2 * ((int64_t)row * K + js + i);
            const float *rb = R + 2 * ((int64_t)row * K + js + i);
            X.set_cprod(i / 2, one, la[0], la[1], one, la[2], la[3]);
            Y.set_cprod(i / 2, one, rb[0], rb[1], one, rb[2], rb[3]);
        }
        LSP_PMAC(X, Y.rh, Y.rl, Y.ih, Y.il, A, B, C, D);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int a = 8 * (r / 4) + 4 * half + (r % 4);
        float *op = Pp + 2 * (a * 32 + row);
        float *om = Pm + 2 * (a * 32 + row);
        op[0] = A[r] - B[r];
        op[1] = C[r] + D[r];
        om[0] = A[r] + B[r];
        om[1] = D[r] - C[r];
    }
}

hipError_t launch_probe_cpair(const float *L, const float *R, int K, float *Pp, float *Pm, hipStream_t s)
{
    hipLaunchKernelGGL(probe_cpair_kernel, dim3(1), dim3(64), 0, s, L, R, K, Pp, Pm);
    return hipGetLastError();
}

hipError_t launch_probe_cmac(const float *L, const float *R, int K, float *P, hipStream_t s)
{
    hipLaunchKernelGGL(probe_cmac_kernel, dim3(1), dim3(64), 0, s, L, R, K, P);
    return hipGetLastError();
}

// 4- or 8-wave workgroups (an 8-wave group shares each block's R operands among
// twice as many waves); 256 VGPRs at most either way, two waves per SIMD
__global__ void __launch_bounds__(512, 1) pgram_mfma_kernel(PgramArgs a) { mfma_sums_pm(a); }

__global__ void __launch_bounds__(512, 1) gls_mfma_kernel(PgramArgs a) { gls_sums(a); }
// the conjugate-pair form: one wave per SIMD (at most 4 waves per workgroup)
__global__ void __launch_bounds__(256, 1) gls_pm_kernel(PgramArgs a) { gls_sums_pm(a); }

// ---------------------------------------------------------------------------
// Batched form: a persistent workgroup takes (curve, block of 4 x 32 a-rows =
// 8192 frequencies) items from the queue (longest curves first) and runs the
// products above over the whole curve, then evaluates Eq. (5) in FP64 from the
// FP32 sums and folds (Pn, k) into the curve's 64-bit max key.

__device__ __forceinline__ unsigned long long wave_max_key(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o, kWave);
        v = (w > v) ? w : v;
    }
    return v;
}

// Eq. (5) of the per-frequency sums, or the window power for unit values;
// out of line so that its FP64 constants stay out of the product loop's registers
__device__ __noinline__ float mfma_batch_epilogue(double XC, double XS, double CC, double CS, double Nt,
                                                  double inv_var, int epi)
{
    if (epi == EPI_WINDOW) return (float)(XC * XC + XS * XS);
    return pn_from_sums(XC, XS, CC, CS, Nt, inv_var);
}

__global__ void __launch_bounds__(256, 2) batch_mfma_kernel(BatchArgs a)
{
    __shared__ MfmaLds<2, false> S;
    __shared__ unsigned int s_item;
    const int tid = threadIdx.x;
    const float one = opaque_one();
    const int nw = blockDim.x / kWave;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int half = lane >> 5;
    const int row = lane & 31;
    // A workgroup never takes more than n_items items: the bound is a guaranteed
    // exit on top of the drained-queue test, which every thread sees alike.
    for (int guard = 0; guard <= a.n_items; ++guard) {
        if (tid == 0) s_item = atomicAdd(a.queue, 1u);
        __syncthreads();
        const unsigned int it = s_item;
        __syncthreads();  // every thread has read s_item before the next write
        if (it >= (unsigned)a.n_items) break;
        const BatchItem item = a.items[it];
        const BatchCurve cv = a.curves[item.curve];
        if (tid == 0) atomicMin(&a.tbeg[item.curve], (unsigned long long)wall_clock64());
        const float *th = a.th + cv.toff;
        const float *tl = a.tl + cv.toff;
        const float *xr = a.xv + cv.xoff;
        const int64_t Nt = cv.Nt;

        float mx = 0.f;
        for (int64_t j = tid; j < Nt; j += blockDim.x) mx = fmaxf(mx, fabsf(xr[j]));
        mx = wave_max(mx);
        if (lane == 0) S.red[0][wave] = mx;
        __syncthreads();
        mx = S.red[0][0];
        for (int w = 1; w < nw; ++w) mx = fmaxf(mx, S.red[0][w]);
        int ex = 0;
        (void)frexpf(mx, &ex);
        const float xscale = ldexpf(1.0f, 14 - ex);

        // A curve's last item may hold fewer than nw row tiles with frequencies
        // below Nf.  With at most two (one), the waves group in twos (fours) on
        // them: the waves of a group take one row tile and split each block's
        // four K-steps between them (all waves still share the block's R
        // operands), and their sums are added through LDS at the end.
        const int64_t k_first = (int64_t)item.fblock * nw * 32 * 64;
        const int64_t n_act = (cv.Nf - k_first + 2047) / 2048;
        const int grp = (nw != 4) ? 1 : (n_act <= 1 ? 4 : (n_act <= 2 ? 2 : 1));  // waves per row tile
        const int tiles = nw / grp;
        const int tile = wave % tiles;
        const int kg = wave / tiles;   // the wave's share of the K-steps within its group
        const int64_t a0 = ((int64_t)item.fblock * nw + tile) * 32;
        // conjugate pairs as in mfma_sums_pm: F_a centred in the a-row's 64
        // frequencies, beta_b = (b + 1/2) df for b < 32
        const double Fa = cv.f_min + ((double)((a0 + row) * 64) + 31.5) * cv.df;
        floatx16 acc[8];  // [A, B, C, D] of L R, then of L2 R2
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = floatx16{};

        // the next block's samples, loaded one block ahead (as in mfma_sums_pm)
        float pth = 0.f, ptl = 0.f, pxv = 0.f;
        bool pok = false;
        if (tid < kMB) {
            pok = tid < Nt;
            if (pok) {
                pth = th[tid];
                ptl = tl[tid];
                pxv = xr[tid];
            }
        }
        for (int64_t j0 = 0; j0 < Nt; j0 += kMB) {
            __syncthreads();
            lds_poison(S);
            if (tid < kMB) {
                S.t[tid] = pok ? (double)pth + (double)ptl : 0.0;
                S.x[tid] = pok ? pxv * xscale : 0.0f;
                S.w[tid] = pok ? kTrigScale : 0.0f;  // pads: R2 = 0
                const int64_t j = j0 + kMB + tid;
                pok = j < Nt;
                if (pok) {
                    pth = th[j];
                    ptl = tl[j];
                    pxv = xr[j];
                }
            }
            __syncthreads();
            for (int task = tid; task < 32 * (kMB / 8); task += blockDim.x) {
                const int b = task / (kMB / 8);
                const int g = task % (kMB / 8);
                const double bdf = ((double)b + 0.5) * cv.df;
                COp R, R2;
                build_r8(bdf, &S.t[8 * g], &S.w[8 * g], one, R, R2);
                *reinterpret_cast<halfx8 *>(&S.R[RR_H][b][8 * g]) = R.rh;
                *reinterpret_cast<halfx8 *>(&S.R[RR_L][b][8 * g]) = R.rl;
                *reinterpret_cast<halfx8 *>(&S.R[RI_H][b][8 * g]) = R.ih;
                *reinterpret_cast<halfx8 *>(&S.R[RI_L][b][8 * g]) = R.il;
                *reinterpret_cast<halfx8 *>(&S.R[R2R_H][b][8 * g]) = R2.rh;
                *reinterpret_cast<halfx8 *>(&S.R[R2R_L][b][8 * g]) = R2.rl;
                *reinterpret_cast<halfx8 *>(&S.R[R2I_H][b][8 * g]) = R2.ih;
                *reinterpret_cast<halfx8 *>(&S.R[R2I_L][b][8 * g]) = R2.il;
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < kMB / 16; ++ks) {
                if (ks / (4 / grp) != kg) continue;  // another wave of the group takes it
                const int js = 16 * ks + 8 * half;
                COp L, L2;
#pragma unroll
                for (int i = 0; i < 8; i += 2) {
                    float c[2], s[2], t[2], c2[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const float ph = rev_fract(Fa * S.t[js + i + u]);
                        c[u] = cos_rev(ph);
                        s[u] = sin_rev(ph);
                        t[u] = double_angle(c[u], kTrigScale, c2[u]);
                    }
                    L.set_cprod(i / 2, S.x[js + i], c[0], s[0], S.x[js + i + 1], c[1], s[1]);
                    L2.set_csum(i / 2, c2[0], c2[1], t[0], s[0], t[1], s[1], one);
                }
                pm_products(L, L2, S.R, row, js, acc);
            }
        }

        // group sums by a fixed tree through the LDS staging area: in each
        // round the upper half of the group (two waves in all, 64 KB of the
        // 72 KB) stores its sums and the lower half adds them
        float *ps = reinterpret_cast<float *>(&S.R[0][0][0]);
        for (int h = grp / 2; h >= 1; h /= 2) {
            __syncthreads();  // the R operands (first round) or the last round's sums are read
            if (kg >= h && kg < 2 * h) {
                const int slot = (kg - h) * tiles + tile;
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int r = 0; r < 16; ++r) ps[(slot * 128 + q * 16 + r) * kWave + lane] = acc[q][r];
            }
            __syncthreads();
            if (kg < h) {
                const int slot = kg * tiles + tile;
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[q][r] += ps[(slot * 128 + q * 16 + r) * kWave + lane];
            }
        }
        if (kg > 0) continue;  // the group's first wave evaluates the tile
        // whole-curve sums (the ragged end's pads add nothing)
        const double ux = ldexp(1.0, ex - 28);
        const double uz = 1.0 / ((double)kTrigScale * (double)kTrigScale);
        const double inv_var = a.stats[item.curve].inv_var;
        unsigned long long best = 0ull;
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                // n = 0: F_a + beta_b (L R), n = 1: F_a - beta_b (L conj(R))
                const int64_t ar = a0 + 8 * (r / 4) + 4 * half + (r % 4);
                const int64_t k = n == 0 ? ar * 64 + 32 + row : ar * 64 + 31 - row;
                if (k < cv.Nf) {
                    const float sg = n == 0 ? -1.0f : 1.0f;
                    const double XC = (double)(acc[0][r] + sg * acc[1][r]) * ux;
                    const double XS = (double)(n == 0 ? acc[2][r] + acc[3][r] : acc[3][r] - acc[2][r]) * ux;
                    const double CC = 0.5 * ((double)Nt + (double)(acc[4][r] + sg * acc[5][r]) * uz);
                    const double CS = 0.5 * (double)(n == 0 ? acc[6][r] + acc[7][r] : acc[7][r] - acc[6][r]) * uz;
                    const float P = mfma_batch_epilogue(XC, XS, CC, CS, (double)Nt, inv_var, a.epi_mode);
                    if (a.Pn) a.Pn[cv.pn_off + k] = P;
                    const unsigned long long key = ((unsigned long long)__float_as_uint(P) << 32) |
                                                   (unsigned long long)(0xffffffffu - (unsigned)k);
                    best = (key > best) ? key : best;
                }
            }
        best = wave_max_key(best);
        if (lane == 0) {
            atomicMax(&a.key[item.curve], best);
            atomicMax(&a.tend[item.curve], (unsigned long long)wall_clock64());
        }
    }
}

hipError_t batch_mfma_occupancy(int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_mfma_kernel, 256, 0);
}

hipError_t launch_batch_mfma(const BatchArgs &a, int persistent_blocks, hipStream_t s)
{
    hipLaunchKernelGGL(batch_mfma_kernel, dim3((unsigned)persistent_blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The weighted least-squares powers from their sums (weights normalized to 1).
//
// A bin whose smallest pivot of the centred normal equations (for K = 1 the
// smaller eigenvalue of the 2x2 system) falls below kRefinePivot is listed by
// the merge and recomputed in FP64 (mh_refine_kernel): the FP32 chunk sums
// carry absolute errors of a few 1e-7, which a pivot of 1e-2 turns into a few
// 1e-5 of p at most, while near f = 0 (less than a cycle over the baseline)
// or at aliases of the sampling the pivot falls far lower.
constexpr double kRefinePivot = 1e-2;

// Generalized power (Section 6.3's pointer to Zechmeister & Kuerster):
//   CC = sum w cos^2 - C^2, SS = sum w sin^2 - S^2, CS = sum w cos sin - C S,
//   p = (SS YC^2 + CC YS^2 - 2 CS YC YS) / (YY (CC SS - CS^2)),
// with sum w cos^2 = (1 + C2)/2, sum w sin^2 = (1 - C2)/2, sum w cos sin = S2/2
// (C2 + i S2 = sum w e^{2i wt}).  A degenerate direction falls back to the
// one-dimensional fit on the other, else p = 0.  FP32-derived sums: a
// direction with CC or SS <= 1e-5 (or a determinant <= 1e-10) is degenerate;
// FP64 sums (fp64 = true): the determinant or the direction <= 1e-12, the
// oracle's rule.  *lmin: the smaller eigenvalue of [[CC, CS], [CS, SS]].
__device__ __forceinline__ double gls_power(double C, double Sn, double YC, double YS, double C2, double S2,
                                            double YY, bool fp64, double *lmin, bool dform = false)
{
    // dform: C and C2 carried as C - 1 and C2 - 1 (see mh_power)
    const double CCh = 0.5 + 0.5 * C2, CSh = 0.5 * S2;
    const double CC = dform ? 0.5 * C2 - 2.0 * C - C * C : CCh - C * C;
    const double SS = dform ? -0.5 * C2 - Sn * Sn : (1.0 - CCh) - Sn * Sn;
    const double CS = dform ? CSh - (1.0 + C) * Sn : CSh - C * Sn;
    const double D = CC * SS - CS * CS;
    const double h = 0.5 * (CC - SS);
    *lmin = 0.5 * (CC + SS) - sqrt(h * h + CS * CS);
    if (!(YY > 0.0)) return 0.0;
    const double eps = fp64 ? 1e-12 : 1e-5;
    const bool two = fp64 ? (D > 1e-12) : (CC > eps && SS > eps && D > eps * eps);
    // a fraction of the variance, [0, 1] up to rounding, which is clipped
    double p = 0.0;
    if (two) p = (SS * YC * YC + CC * YS * YS - 2.0 * CS * YC * YS) / (YY * D);
    else if (CC > eps) p = YC * YC / (YY * CC);
    else if (SS > eps) p = YS * YS / (YY * SS);
    return fmin(fmax(p, 0.0), 1.0);
}

// FP64 merge of the six chunk sums (slots C, S, YC, YS, C2/2, S2/2) and the
// generalized power; ill-conditioned bins are listed for the FP64 recomputation.
__global__ void __launch_bounds__(256) gls_reduce_kernel(const float *__restrict__ part, int splits, int64_t Nf,
                                                         const CurveStats *__restrict__ st, float *__restrict__ P,
                                                         uint32_t *__restrict__ list, uint32_t *__restrict__ count)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= Nf) return;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    sum_chunks<6, 4>(part, splits, Nf, k, v);
    const double YY = st->var;
    double lmin;
    P[k] = (float)gls_power(v[0], v[1], v[2], v[3], 2.0 * v[4], 2.0 * v[5], YY, false, &lmin);
    if (YY > 0.0 && !(lmin >= kRefinePivot)) list[atomicAdd(count, 1u)] = (uint32_t)k;
}

hipError_t launch_gls(const PgramArgs &a, int waves, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    // 8-wave workgroups: the plain complex products (32 frequencies per a-row);
    // up to 4 waves: conjugate pairs (64 per a-row, one wave per SIMD)
    const bool pm = waves <= 4;
    const int64_t per_wave = pm ? kGlsPmFreqPerWave : kGlsFreqPerWave;
    const int64_t nfb = (a.Nf + per_wave - 1) / per_wave;
    const int64_t nblk = (nfb + waves - 1) / waves;
    launch_timed(pm ? gls_pm_kernel : gls_mfma_kernel, dim3((unsigned)nblk, (unsigned)a.splits), dim3(kWave * waves),
                 s, ev0, ev1, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gls_reduce_kernel, dim3((unsigned)((a.Nf + 255) / 256)), dim3(256), 0, s,
                       (const float *)a.part, a.splits, a.Nf, a.stats, a.Pn, a.refine_list, a.refine_count);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_refine(a, 1, s);
}

// ---------------------------------------------------------------------------
// Multi-harmonic periodogram (Section 6.3's pointer to Schwarzenberg-Czerny
// 1996): the weighted least-squares fit of c + sum_{h<=K} (a_h cos h wt +
// b_h sin h wt).  Its normal equations need, per frequency,
//   C_m + i S_m = sum_j w_j e^{i m w t'_j}, m = 1..2K  (Gram entries through
//   cos A cos B = (cos(A-B) + cos(A+B))/2 and the like), and
//   YC_h + i YS_h = sum_j w_j (y_j - Y) e^{i h w t'_j}, h = 1..K,
// i.e. 3K complex products of the same kind, with the R operands of the
// harmonics involved.  b range 32 (k = 32a + b); a wave holds at most six
// complex sums (twelve 32x32 accumulators, one wave per SIMD), so K = 2 is one
// pass over the samples and K = 3, 4 are two passes, each writing its own
// slots of the per-chunk partial sums.

// One pass: weight sums of harmonics W0..W1 (none when W1 < W0) and value sums
// of harmonics 1..V (none when V = 0).
template <int W0, int W1, int V0, int V1>
struct MhPass {
    static constexpr int NW = (W1 >= W0) ? W1 - W0 + 1 : 0;  // weight harmonics W0..W1
    static constexpr int NV = (V1 >= V0) ? V1 - V0 + 1 : 0;  // value harmonics V0..V1
    static constexpr int NS = NW + NV;
    static constexpr int HMAX = (W1 > V1) ? W1 : V1;
    static constexpr bool weight(int m) { return NW > 0 && m >= W0 && m <= W1; }
    static constexpr bool value(int m) { return NV > 0 && m >= V0 && m <= V1; }
    static constexpr bool needed(int m) { return weight(m) || value(m); }
    static constexpr int rslot(int m)
    {
        int r = 0;
        for (int i = 1; i < m; ++i) r += needed(i) ? 1 : 0;
        return r;
    }
    static constexpr int wslot(int m) { return m - W0; }       // accumulators of weight harmonic m
    static constexpr int vslot(int h) { return NW + h - V0; }  // accumulators of value harmonic h
    static constexpr int NR = rslot(HMAX + 1);                 // harmonics with R operands in LDS
    static_assert(NS >= 1 && NS <= 3, "a pass holds one to three complex sums");
};

template <int NR>
struct MhLds {
    double t[kMB];
    float x[kMB];
    float w[kMB];
    float red[2][kMaxWaves];
    alignas(16) _Float16 R[4 * NR][32][kMRow];  // per harmonic: (re hi, re lo, im hi, im lo)
};

// z = u v for complex u, v
__device__ __forceinline__ void cmul(float ur, float ui, float vr, float vi, float &zr, float &zi)
{
    zr = ur * vr - ui * vi;
    zi = ur * vi + ui * vr;
}

// R operands of harmonic M for sample i of a group (e^{i M phi} from e^{i phi}
// by repeated products), then the next harmonic
template <class P, int M>
struct MhRBuild {
    __device__ __forceinline__ static void run(float c1, float s1, float cr, float ci, halfx8 (&v)[4 * P::NR], int i)
    {
        if constexpr (M > 1) cmul(cr, ci, c1, s1, cr, ci);
        if constexpr (P::needed(M)) {
            constexpr int r = P::rslot(M);
            _Float16 h, l;
            split16(cr * kTrigScale, h, l);
            v[4 * r][i] = h;
            v[4 * r + 1][i] = l;
            split16(ci * kTrigScale, h, l);
            v[4 * r + 2][i] = h;
            v[4 * r + 3][i] = l;
        }
        if constexpr (M < P::HMAX) MhRBuild<P, M + 1>::run(c1, s1, cr, ci, v, i);
    }
};

// the products of harmonic M over this lane's 8 samples, then the next
// harmonic: each complex sum as its four real products (conjugate pairs)
template <class P, int M>
struct MhStep {
    __device__ __forceinline__ static void run(const float (&e1r)[8], const float (&e1i)[8], float (&er)[8],
                                               float (&ei)[8], const float (&xv)[8], const float (&wv)[8],
                                               const MhLds<P::NR> &S, int row, int js,
                                               floatx16 (&acc)[P::NS][4])
    {
        if constexpr (M > 1) {
#pragma unroll
            for (int i = 0; i < 8; ++i) cmul(er[i], ei[i], e1r[i], e1i[i], er[i], ei[i]);
        }
        if constexpr (P::needed(M)) {
            constexpr int r = P::rslot(M);
            const halfx8 rrh = *reinterpret_cast<const halfx8 *>(&S.R[4 * r][row][js]);
            const halfx8 rrl = *reinterpret_cast<const halfx8 *>(&S.R[4 * r + 1][row][js]);
            const halfx8 rih = *reinterpret_cast<const halfx8 *>(&S.R[4 * r + 2][row][js]);
            const halfx8 ril = *reinterpret_cast<const halfx8 *>(&S.R[4 * r + 3][row][js]);
            if constexpr (P::weight(M)) {
                constexpr int q = P::wslot(M);
                COp LW;
#pragma unroll
                for (int i = 0; i < 8; i += 2) LW.set_cprod(i / 2, wv[i], er[i], ei[i], wv[i + 1], er[i + 1], ei[i + 1]);
                LSP_PMAC(LW, rrh, rrl, rih, ril, acc[q][0], acc[q][1], acc[q][2], acc[q][3]);
            }
            if constexpr (P::value(M)) {
                constexpr int q = P::vslot(M);
                COp LX;
#pragma unroll
                for (int i = 0; i < 8; i += 2) LX.set_cprod(i / 2, xv[i], er[i], ei[i], xv[i + 1], er[i + 1], ei[i + 1]);
                LSP_PMAC(LX, rrh, rrl, rih, ril, acc[q][0], acc[q][1], acc[q][2], acc[q][3]);
            }
        }
        if constexpr (M < P::HMAX) MhStep<P, M + 1>::run(e1r, e1i, er, ei, xv, wv, S, row, js, acc);
    }
};

// Per-chunk partial sums of one pass, written to the slots of the K-harmonic
// layout: sum g (0..3K-1) = weight harmonic g + 1 for g < 2K, value harmonic
// g - 2K + 1 after that; its real and imaginary parts at slots 2g and 2g + 1.
// Conjugate pairs as in mfma_sums_pm: F_a = f_min + (64 a + 31.5) df,
// harmonic m of beta_b = (b + 1/2) df, and each sum's four real products give
// frequencies k = 64 a + 32 + b and 64 a + 31 - b.  At most three complex
// sums (twelve accumulators) per pass, one wave per SIMD.
template <int K, int W0, int W1, int V0, int V1>
__global__ void __launch_bounds__(256, 1) mh_mfma_kernel(PgramArgs a)
{
    using P = MhPass<W0, W1, V0, V1>;
    constexpr int NS = P::NS;
    __shared__ MhLds<P::NR> S;
    const int tid = threadIdx.x;
    const int nw = blockDim.x / kWave;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int half = lane >> 5;
    const int row = lane & 31;
    const int split = blockIdx.y;
    const int64_t jb = (int64_t)split * a.chunk;
    const int64_t je = (jb + a.chunk < a.Nt) ? jb + a.chunk : a.Nt;

    float mx = 0.f, mw = 0.f;
    for (int64_t j = jb + tid; j < je; j += blockDim.x) {
        mx = fmaxf(mx, fabsf(a.rec.xv[j]));
        mw = fmaxf(mw, a.rec.wv[j]);
    }
    mx = wave_max(mx);
    mw = wave_max(mw);
    if (lane == 0) {
        S.red[0][wave] = mx;
        S.red[1][wave] = mw;
    }
    __syncthreads();
    mx = S.red[0][0];
    mw = S.red[1][0];
    for (int w = 1; w < nw; ++w) {
        mx = fmaxf(mx, S.red[0][w]);
        mw = fmaxf(mw, S.red[1][w]);
    }
    int ex = 0, ew = 0;
    (void)frexpf(mx, &ex);
    (void)frexpf(mw, &ew);
    const float xscale = ldexpf(1.0f, 14 - ex);
    const float wscale = ldexpf(1.0f, 14 - ew);

    const int64_t a_row = ((int64_t)blockIdx.x * nw + wave) * 32 + row;
    const double Fa = a.f_min + ((double)(a_row * 64) + 31.5) * a.df;

    floatx16 acc[NS][4];  // [sum][A, B, C, D], sums in the pass's order (weights, then values)
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[q][c] = floatx16{};

    for (int64_t j0 = jb; j0 < je; j0 += kMB) {
        __syncthreads();
        lds_poison(S);
        if (tid < kMB) {
            const int64_t j = j0 + tid;
            const bool ok = j < je;  // ragged end: t' = 0, x = 0, w = 0 (adds nothing)
            S.t[tid] = ok ? (double)a.rec.th[j] + (double)a.rec.tl[j] : 0.0;
            S.x[tid] = ok ? a.rec.xv[j] * xscale : 0.0f;
            S.w[tid] = ok ? a.rec.wv[j] * wscale : 0.0f;
        }
        __syncthreads();
        // R operands of the pass's harmonics: 32 b x 8 groups of 8 samples
        for (int task = tid; task < 32 * (kMB / 8); task += blockDim.x) {
            const int b = task / (kMB / 8);
            const int g = task % (kMB / 8);
            const double bdf = ((double)b + 0.5) * a.df;
            halfx8 v[4 * P::NR];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float ph = rev_fract(bdf * S.t[8 * g + i]);
                const float c1 = cos_rev(ph), s1 = sin_rev(ph);
                MhRBuild<P, 1>::run(c1, s1, c1, s1, v, i);
            }
#pragma unroll
            for (int q = 0; q < 4 * P::NR; ++q) *reinterpret_cast<halfx8 *>(&S.R[q][b][8 * g]) = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kMB / 16; ++ks) {
            const int js = 16 * ks + 8 * half;
            float e1r[8], e1i[8], er[8], ei[8], xv[8], wv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float ph = rev_fract(Fa * S.t[js + i]);
                e1r[i] = cos_rev(ph);
                e1i[i] = sin_rev(ph);
                er[i] = e1r[i];
                ei[i] = e1i[i];
                xv[i] = S.x[js + i];
                wv[i] = S.w[js + i];
            }
            MhStep<P, 1>::run(e1r, e1i, er, ei, xv, wv, S, row, js, acc);
        }
    }

    const float ux = ldexpf(1.0f, ex - 28);
    const float uw = ldexpf(1.0f, ew - 28);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t ar = ((int64_t)blockIdx.x * nw + wave) * 32 + 8 * (r / 4) + 4 * half + (r % 4);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            // n = 0: F_a + beta_b (L R), n = 1: F_a - beta_b (L conj(R))
            const int64_t k = n == 0 ? ar * 64 + 32 + row : ar * 64 + 31 - row;
            if (k < a.Nf) {
                const float sg = n == 0 ? -1.0f : 1.0f;
                float *p = a.part + (int64_t)split * 6 * K * a.Nf + k;
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    const int gq = (q < P::NW) ? (W0 - 1 + q) : (2 * K + V0 - 1 + q - P::NW);
                    const float u = (q < P::NW) ? uw : ux;
                    const float re = acc[q][0][r] + sg * acc[q][1][r];
                    const float im = n == 0 ? acc[q][2][r] + acc[q][3][r] : acc[q][3][r] - acc[q][2][r];
                    p[(int64_t)(2 * gq) * a.Nf] = re * u;
                    p[(int64_t)(2 * gq + 1) * a.Nf] = im * u;
                }
            }
        }
    }
}

// The multi-harmonic power from the sums v (C_m, S_m for m = 1..2K at
// v[2(m-1)], v[2(m-1)+1]; YC_h, YS_h for h = 1..K at v[4K + 2(h-1)], +1).
// Columns u = (cos hwt, sin hwt), h = 1..K, centred by their weighted means
// (the constant is fitted):
//   G_ik = sum w u_i u_k - mean_i mean_k,  b_i = sum w (y - Y) u_i,
// with sum w cos(Aw t) cos(Bw t) = (C_{A-B} + C_{A+B})/2 and the like
// (C_0 = 1, S_0 = 0, C_{-m} = C_m, S_{-m} = -S_m).  Cholesky (in place, lower
// triangle) with column dropping; p = |L^{-1} b|^2 / YY.  FP32-derived sums:
// a column whose centred diagonal or pivot is <= 1e-5 (of that diagonal) is
// dropped (columns the FP32 sums cannot separate); FP64 sums (fp64 = true): a
// pivot <= 1e-12 of the uncentred diagonal sum w u_i^2, the oracle's rule.
// *min_pivot: the smallest pivot met (dropped columns included).
template <int K>
__device__ __forceinline__ double mh_power(const double *v, double YY, bool fp64, double *min_pivot,
                                          bool dform = false)
{
    constexpr int M2 = 2 * K, n = 2 * K;
    // dform: the cosine sums are carried as C_m - 1 (d_m), which keeps the
    // centred Gram entries of low frequencies (wt << 1 over the baseline, where
    // C_m - C_A C_B cancels to O((wt)^4)) to FP64 precision relative to them
    double C[M2 + 1], Sn[M2 + 1];
    C[0] = dform ? 0.0 : 1.0;
    Sn[0] = 0.0;
#pragma unroll
    for (int m = 1; m <= M2; ++m) {
        C[m] = v[2 * (m - 1)];
        Sn[m] = v[2 * (m - 1) + 1];
    }
    auto Cm = [&](int m) { return C[m < 0 ? -m : m]; };
    auto Sm = [&](int m) { return m < 0 ? -Sn[-m] : Sn[m]; };
    // column i: harmonic 1 + i/2, cos for even i, sin for odd i
    double G[n][n], b[n], mean[n], raw[n];
#pragma unroll
    for (int i = 0; i < n; ++i) {
        const int h = 1 + i / 2;
        mean[i] = (i % 2 == 0) ? C[h] : Sn[h];  // dform: the cosine means less 1
        b[i] = v[2 * M2 + 2 * (h - 1) + (i % 2)];
    }
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            const int A = 1 + i / 2, B = 1 + j / 2;
            const bool ci = i % 2 == 0, cj = j % 2 == 0;
            double r;
            if (ci && cj) r = 0.5 * (Cm(A - B) + Cm(A + B));
            else if (!ci && !cj) r = 0.5 * (Cm(A - B) - Cm(A + B));
            else if (ci) r = 0.5 * (Sm(A + B) - Sm(A - B));  // cos(A) sin(B)
            else r = 0.5 * (Sm(A + B) + Sm(A - B));          // sin(A) cos(B)
            if (!dform) {
                if (i == j) raw[i] = r;
                G[i][j] = r - mean[i] * mean[j];
            } else {
                // with C = 1 + d: E[cos cos] = 1 + r and mean = 1 + d, so the
                // centred entry is r - d_A - d_B - d_A d_B; cos sin: r - (1 + d_A) s_B
                if (i == j) raw[i] = ci ? 1.0 + r : r;
                if (ci && cj) G[i][j] = r - mean[i] - mean[j] - mean[i] * mean[j];
                else if (!ci && !cj) G[i][j] = r - mean[i] * mean[j];
                else if (ci) G[i][j] = r - (1.0 + mean[i]) * mean[j];
                else G[i][j] = r - mean[i] * (1.0 + mean[j]);
            }
        }
    const double eps = 1e-5;
    double z[n];
    double explained = 0.0;
    double mp = INFINITY;
#pragma unroll
    for (int i = 0; i < n; ++i) {
        // G[i][0..i-1] already hold L[i][0..i-1] (zero for dropped columns)
        const double gii = G[i][i];
        double d = gii;
#pragma unroll
        for (int c = 0; c < i; ++c) d -= G[i][c] * G[i][c];
        mp = fmin(mp, d);
        z[i] = 0.0;
        const bool drop = fp64 ? (!(raw[i] > 0.0) || !(d > 1e-12 * raw[i])) : (!(gii > eps) || !(d > eps * gii));
        if (drop) {
#pragma unroll
            for (int r = i + 1; r < n; ++r) G[r][i] = 0.0;  // column dropped
            continue;
        }
        const double lii = sqrt(d);
#pragma unroll
        for (int r = i + 1; r < n; ++r) {
            double t = G[r][i];
#pragma unroll
            for (int c = 0; c < i; ++c) t -= G[r][c] * G[i][c];
            G[r][i] = t / lii;
        }
        double t = b[i];
#pragma unroll
        for (int c = 0; c < i; ++c) t -= G[i][c] * z[c];
        z[i] = t / lii;
        explained += z[i] * z[i];
    }
    *min_pivot = mp;
    // a fraction of the variance: 1 at most (rounding in an interpolating fit,
    // Nt = 2K + 1, can carry explained / YY past 1 by ~1e-5)
    return (YY > 0.0) ? fmin(explained / YY, 1.0) : 0.0;
}

// FP64 merge of the 6K chunk sums and the least-squares solve; ill-conditioned
// bins are listed for the FP64 recomputation.
template <int K>
__global__ void __launch_bounds__(256) mh_reduce_kernel(const float *__restrict__ part, int splits, int64_t Nf,
                                                        const CurveStats *__restrict__ st, float *__restrict__ P,
                                                        uint32_t *__restrict__ list, uint32_t *__restrict__ count)
{
    constexpr int NS = 3 * K;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= Nf) return;
    double v[2 * NS];
#pragma unroll
    for (int q = 0; q < 2 * NS; ++q) v[q] = 0.0;
    sum_chunks<2 * NS, (2 * NS >= 24 ? 1 : 2)>(part, splits, Nf, k, v);
    const double YY = st->var;
    double piv;
    P[k] = (float)mh_power<K>(v, YY, false, &piv);
    if (YY > 0.0 && !(piv >= kRefinePivot)) list[atomicAdd(count, 1u)] = (uint32_t)k;
}

// FP64 recomputation of the listed bins: each thread sums samples tid,
// tid + 256, ... from the records the matrix-core kernels read (t' = th + tl,
// w/W, w (y - Y)/W), with the phase reduced and the sine and cosine evaluated
// in FP64 and the harmonics by complex products; a fixed-order tree adds the
// threads' sums, then the solve runs with the FP64 rule.  The harmonics are
// carried as e^{i m theta} - 1 (from the half angle), so that the cosine sums
// are C_m - 1: at frequencies with less than a cycle over the baseline the
// centred Gram entries are O((wt)^4) and would cancel against the raw sums'
// O(1) to FP64 rounding.  A bin takes one
// workgroup, or, when few bins are listed (typically only f = 0), P of them
// over consecutive sample ranges, whose sums a second kernel adds in range
// order; P depends only on the number of listed bins, so a bin's value does
// not depend on which workgroups take it.
// The records hold the normalized weights and centred values rounded to FP32,
// so their own totals W0 = sum w/W and Y0 = sum w (y - Y)/W (summed alongside,
// in the same order) differ from 1 and 0 by rounding: every weight sum is
// divided by W0 and every value sum is centred on Y0/W0, which makes the
// normal equations those of the records' own weights exactly (at f = 0 every
// sum of e^{i m theta} - 1 is 0, and the constant direction is dropped as the
// oracle drops it).
// workgroups per listed bin: the pass's kRefineBlocks workgroups spread over
// the n listed bins, at most kRefineMaxParts each (1: a workgroup per bin,
// which then also evaluates the power)
__host__ __device__ __forceinline__ int refine_parts(uint32_t n)
{
    if (n == 0) return 1;
    const uint32_t p = kRefineBlocks / n;
    return p < 1 ? 1 : (p > (uint32_t)kRefineMaxParts ? kRefineMaxParts : (int)p);
}

// the FP64 power of one bin from its harmonic sums v[0 .. 6K) and the records'
// weight and value totals v[6K], v[6K + 1] (normalized here)
template <int K>
__device__ __forceinline__ float refine_power(double *v, double YY)
{
    constexpr int NS = 6 * K;
    const double W0 = v[NS], ybar = v[NS + 1] / W0;
#pragma unroll
    for (int q = 0; q < 4 * K; ++q) v[q] /= W0;
#pragma unroll
    for (int q = 0; q < 2 * K; ++q) v[4 * K + q] = v[4 * K + q] / W0 - ybar * v[q];
    double d;
    double p = 0.0;
    if (W0 > 0.0)
        p = (K == 1) ? gls_power(v[0], v[1], v[4], v[5], v[2], v[3], YY, true, &d, true)
                     : mh_power<K>(v, YY, true, &d, true);
    return (float)p;
}

template <int K>
__global__ void __launch_bounds__(256) mh_refine_kernel(PgramArgs a)
{
    constexpr int NS = 6 * K;      // harmonic sums
    constexpr int NV = NS + 2;     // and the records' weight and value totals
    __shared__ double red[NV][256];
    const int tid = threadIdx.x;
    const uint32_t n = *a.refine_count;
    const int P = refine_parts(n);
    // P = 1: bins i = blockIdx.x, + gridDim.x, ...; P > 1: item q = blockIdx.x
    // is part q % P of bin q / P (n P <= kRefineBlocks items)
    const uint32_t items = (P == 1) ? n : n * (uint32_t)P;
    for (uint32_t q = blockIdx.x; q < items; q += gridDim.x) {
        const uint32_t i = q / (uint32_t)P;
        const int part = (int)(q % (uint32_t)P);
        const int64_t k = (int64_t)a.refine_list[i];
        const double f = a.f_min + (double)k * a.df;
        const int64_t jb = a.Nt * part / P, je = a.Nt * (part + 1) / P;
        double v[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c] = 0.0;
        for (int64_t j = jb + tid; j < je; j += 256) {
            const double tp = (double)a.rec.th[j] + (double)a.rec.tl[j];
            double ph = f * tp;
            ph -= rint(ph);
            // e^{i m theta} - 1 = u_m + i v_m, from the half angle without
            // cancellation: u_1 = -2 sin^2(theta/2), v_1 = sin theta, then
            // (1 + u_m + i v_m)(1 + u_1 + i v_1) with the 1 kept out
            double sh, ch;
            sincospi(ph, &sh, &ch);
            const double u1 = -2.0 * sh * sh, v1 = 2.0 * sh * ch;
            const double w = (double)a.rec.wv[j], y = (double)a.rec.xv[j];
            double u = u1, vv = v1;
#pragma unroll
            for (int m = 1; m <= 2 * K; ++m) {
                if (m > 1) {
                    const double un = u + u1 + (u * u1 - vv * v1);
                    vv = vv + v1 + (u * v1 + vv * u1);
                    u = un;
                }
                v[2 * (m - 1)] += w * u;
                v[2 * (m - 1) + 1] += w * vv;
                if (m <= K) {
                    v[4 * K + 2 * (m - 1)] += y * u;
                    v[4 * K + 2 * (m - 1) + 1] += y * vv;
                }
            }
            v[NS] += w;
            v[NS + 1] += y;
        }
#pragma unroll
        for (int c = 0; c < NV; ++c) red[c][tid] = v[c];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) {
#pragma unroll
                for (int c = 0; c < NV; ++c) red[c][tid] += red[c][tid + w];
            }
            __syncthreads();
        }
        if (tid == 0) {
            if (P == 1) {
#pragma unroll
                for (int c = 0; c < NV; ++c) v[c] = red[c][0];
                a.Pn[k] = refine_power<K>(v, a.stats->var);
            } else {
#pragma unroll
                for (int c = 0; c < NV; ++c) a.refine_part[(size_t)q * NV + c] = red[c][0];
            }
        }
        __syncthreads();  // red is reused by the next item
    }
}

// the bins split over workgroups: their parts added in order, then the power
template <int K>
__global__ void __launch_bounds__(256) mh_refine_finish_kernel(PgramArgs a)
{
    constexpr int NV = 6 * K + 2;
    const uint32_t n = *a.refine_count;
    const int P = refine_parts(n);
    if (P == 1) return;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        double v[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c] = 0.0;
        for (int part = 0; part < P; ++part)
#pragma unroll
            for (int c = 0; c < NV; ++c) v[c] += a.refine_part[((size_t)i * P + part) * NV + c];
        a.Pn[a.refine_list[i]] = refine_power<K>(v, a.stats->var);
    }
}

// the refinement pass: kRefineBlocks workgroups (fewer for a short grid);
// items past the list's length (read on the device) are skipped at once
hipError_t launch_refine(const PgramArgs &a, int K, hipStream_t s)
{
    const dim3 g((unsigned)kRefineBlocks), b(256), g1(1);
    switch (K) {
    case 1:
        hipLaunchKernelGGL(mh_refine_kernel<1>, g, b, 0, s, a);
        hipLaunchKernelGGL(mh_refine_finish_kernel<1>, g1, b, 0, s, a);
        break;
    case 2:
        hipLaunchKernelGGL(mh_refine_kernel<2>, g, b, 0, s, a);
        hipLaunchKernelGGL(mh_refine_finish_kernel<2>, g1, b, 0, s, a);
        break;
    case 3:
        hipLaunchKernelGGL(mh_refine_kernel<3>, g, b, 0, s, a);
        hipLaunchKernelGGL(mh_refine_finish_kernel<3>, g1, b, 0, s, a);
        break;
    case 4:
        hipLaunchKernelGGL(mh_refine_kernel<4>, g, b, 0, s, a);
        hipLaunchKernelGGL(mh_refine_finish_kernel<4>, g1, b, 0, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int K>
static hipError_t launch_mh_k(const PgramArgs &a, int waves, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    const int64_t per_wave = kMhFreqPerWave;
    const int64_t nfb = (a.Nf + per_wave - 1) / per_wave;
    const int64_t nblk = (nfb + waves - 1) / waves;
    const dim3 grid((unsigned)nblk, (unsigned)a.splits), block(kWave * waves);
    // passes of at most three complex sums: weight harmonics 1..2K, then the
    // value harmonics 1..K; the hook's events span the first pass's start to
    // the last pass's end
    if constexpr (K == 2) {
        launch_timed(mh_mfma_kernel<2, 1, 3, 1, 0>, grid, block, s, ev0, nullptr, a);
        launch_timed(mh_mfma_kernel<2, 4, 4, 1, 2>, grid, block, s, nullptr, ev1, a);
    } else if constexpr (K == 3) {
        launch_timed(mh_mfma_kernel<3, 1, 3, 1, 0>, grid, block, s, ev0, nullptr, a);
        launch_timed(mh_mfma_kernel<3, 4, 6, 1, 0>, grid, block, s, nullptr, nullptr, a);
        launch_timed(mh_mfma_kernel<3, 1, 0, 1, 3>, grid, block, s, nullptr, ev1, a);
    } else {
        static_assert(K == 4, "K = 2, 3 or 4");
        launch_timed(mh_mfma_kernel<4, 1, 3, 1, 0>, grid, block, s, ev0, nullptr, a);
        launch_timed(mh_mfma_kernel<4, 4, 6, 1, 0>, grid, block, s, nullptr, nullptr, a);
        launch_timed(mh_mfma_kernel<4, 7, 8, 1, 1>, grid, block, s, nullptr, nullptr, a);
        launch_timed(mh_mfma_kernel<4, 1, 0, 2, 4>, grid, block, s, nullptr, ev1, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((mh_reduce_kernel<K>), dim3((unsigned)((a.Nf + 255) / 256)), dim3(256), 0, s,
                       (const float *)a.part, a.splits, a.Nf, a.stats, a.Pn, a.refine_list, a.refine_count);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_refine(a, K, s);
}

hipError_t launch_mh(const PgramArgs &a, int K, int waves, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    switch (K) {
    case 2: return launch_mh_k<2>(a, waves, s, ev0, ev1);
    case 3: return launch_mh_k<3>(a, waves, s, ev0, ev1);
    case 4: return launch_mh_k<4>(a, waves, s, ev0, ev1);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lsp
