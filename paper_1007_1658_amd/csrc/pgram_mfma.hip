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
// Phases are FP64 products reduced to revolutions (as the SPLIT mode).
//
// Work split: a workgroup of W waves owns a-rows [32 W blockIdx.x, +32 W) and
// all 64 b; wave w owns 32 a-rows (one 32 x 64 output tile per sum).  Per
// block of 32 samples the workgroup writes the R operands once to LDS (shared
// by its waves); each lane builds its own L operands in registers.
#include "pgram_device.h"

namespace lsp {

typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kMB = 32;        // samples per LDS block (two K-steps of 16)
constexpr int kMRow = kMB + 8; // halfs per LDS row: 80 B, so 16 lanes' 16-B reads hit distinct banks
constexpr float kTrigScale = 16384.0f;  // 2^14

enum { RR_H = 0, RR_L, RI_H, RI_L, R2R_H, R2R_L, R2I_H, R2I_L, R_KINDS };

struct MfmaLds {
    double t[kMB];
    float x[kMB];
    float red[kMaxWaves];
    _Float16 R[R_KINDS][64][kMRow];
};

__device__ __forceinline__ void split16(float v, _Float16 &hi, _Float16 &lo)
{
    hi = (_Float16)v;
    lo = (_Float16)(v - (float)hi);
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

#define LSP_MFMA(A, B, C) C = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, B, C, 0, 0, 0)

__global__ void __launch_bounds__(256) pgram_mfma_kernel(PgramArgs a)
{
    __shared__ MfmaLds S;
    const int tid = threadIdx.x;
    const int nw = blockDim.x / kWave;  // waves in the workgroup (1, 2 or 4)
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int half = lane >> 5;   // which 8 samples of a K-step this lane carries
    const int row = lane & 31;    // A: the lane's a-row; B: the lane's b-column
    const int split = blockIdx.y;
    const int64_t jb = (int64_t)split * a.chunk;
    const int64_t je = (jb + a.chunk < a.Nt) ? jb + a.chunk : a.Nt;

    // value scale for this chunk: 2^(14 - e) with max|x - mean| < 2^e
    float mx = 0.f;
    for (int64_t j = jb + tid; j < je; j += blockDim.x) mx = fmaxf(mx, fabsf(a.rec.xv[j]));
    mx = wave_max(mx);
    if (lane == 0) S.red[wave] = mx;
    __syncthreads();
    mx = S.red[0];
    for (int w = 1; w < nw; ++w) mx = fmaxf(mx, S.red[w]);
    int ex = 0;
    (void)frexpf(mx, &ex);  // mx = m 2^ex, 0.5 <= m < 1 (ex = 0 for mx = 0)
    const float xscale = ldexpf(1.0f, 14 - ex);

    const int64_t a_row = ((int64_t)blockIdx.x * nw + wave) * 32 + row;
    const double Fa = a.f_min + (double)(a_row * 64) * a.df;

    floatx16 acc[2][4];  // [b half][ReX, ImX, ReZ, ImZ]
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[n][q] = floatx16{};

    for (int64_t j0 = jb; j0 < je; j0 += kMB) {
        __syncthreads();  // the previous block's LDS is consumed
        if (tid < kMB) {
            const int64_t j = j0 + tid;
            const bool ok = j < je;  // ragged end: neutral samples t' = 0, x = 0
            S.t[tid] = ok ? (double)a.rec.th[j] + (double)a.rec.tl[j] : 0.0;
            S.x[tid] = ok ? a.rec.xv[j] * xscale : 0.0f;
        }
        __syncthreads();
        // R operands: 64 b x 4 groups of 8 samples, one task per thread and round
        for (int task = tid; task < 64 * (kMB / 8); task += blockDim.x) {
            const int b = task / (kMB / 8);
            const int g = task % (kMB / 8);
            const double bdf = (double)b * a.df;
            halfx8 v[R_KINDS];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                double p = bdf * S.t[8 * g + i];
                p -= rint(p);
                const float ph = (float)p;
                const float c = cos_rev(ph), s = sin_rev(ph);
                const float c2 = (c - s) * (c + s), s2 = 2.0f * c * s;
                _Float16 h, l;
                split16(c * kTrigScale, h, l); v[RR_H][i] = h; v[RR_L][i] = l;
                split16(s * kTrigScale, h, l); v[RI_H][i] = h; v[RI_L][i] = l;
                split16(c2 * kTrigScale, h, l); v[R2R_H][i] = h; v[R2R_L][i] = l;
                split16(s2 * kTrigScale, h, l); v[R2I_H][i] = h; v[R2I_L][i] = l;
            }
#pragma unroll
            for (int q = 0; q < R_KINDS; ++q) *reinterpret_cast<halfx8 *>(&S.R[q][b][8 * g]) = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kMB / 16; ++ks) {
            const int js = 16 * ks + 8 * half;
            // this lane's L operands: a-row `row`, samples js .. js+7
            halfx8 lrh, lrl, lih, lil, nih, nil, zrh, zrl, zih, zil, nzh, nzl;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                double p = Fa * S.t[js + i];
                p -= rint(p);
                const float ph = (float)p;
                const float c = cos_rev(ph), s = sin_rev(ph);
                const float xv = S.x[js + i];
                const float c2 = (c - s) * (c + s), s2 = 2.0f * c * s;
                _Float16 h, l;
                split16(xv * c, h, l); lrh[i] = h; lrl[i] = l;
                split16(xv * s, h, l); lih[i] = h; lil[i] = l; nih[i] = -h; nil[i] = -l;
                split16(c2 * kTrigScale, h, l); zrh[i] = h; zrl[i] = l;
                split16(s2 * kTrigScale, h, l); zih[i] = h; zil[i] = l; nzh[i] = -h; nzl[i] = -l;
            }
#pragma unroll
            for (int n = 0; n < 2; ++n) {
                const int bcol = 32 * n + row;
                const halfx8 rrh = *reinterpret_cast<const halfx8 *>(&S.R[RR_H][bcol][js]);
                const halfx8 rrl = *reinterpret_cast<const halfx8 *>(&S.R[RR_L][bcol][js]);
                const halfx8 rih = *reinterpret_cast<const halfx8 *>(&S.R[RI_H][bcol][js]);
                const halfx8 ril = *reinterpret_cast<const halfx8 *>(&S.R[RI_L][bcol][js]);
                const halfx8 qrh = *reinterpret_cast<const halfx8 *>(&S.R[R2R_H][bcol][js]);
                const halfx8 qrl = *reinterpret_cast<const halfx8 *>(&S.R[R2R_L][bcol][js]);
                const halfx8 qih = *reinterpret_cast<const halfx8 *>(&S.R[R2I_H][bcol][js]);
                const halfx8 qil = *reinterpret_cast<const halfx8 *>(&S.R[R2I_L][bcol][js]);
                // Re = Lr Rr - Li Ri,  Im = Lr Ri + Li Rr, each in three FP16 passes;
                // the four sums interleaved so consecutive products are independent
                LSP_MFMA(lrh, rrh, acc[n][0]); LSP_MFMA(lrh, rih, acc[n][1]);
                LSP_MFMA(zrh, qrh, acc[n][2]); LSP_MFMA(zrh, qih, acc[n][3]);
                LSP_MFMA(lrh, rrl, acc[n][0]); LSP_MFMA(lrh, ril, acc[n][1]);
                LSP_MFMA(zrh, qrl, acc[n][2]); LSP_MFMA(zrh, qil, acc[n][3]);
                LSP_MFMA(lrl, rrh, acc[n][0]); LSP_MFMA(lrl, rih, acc[n][1]);
                LSP_MFMA(zrl, qrh, acc[n][2]); LSP_MFMA(zrl, qih, acc[n][3]);
                LSP_MFMA(nih, rih, acc[n][0]); LSP_MFMA(lih, rrh, acc[n][1]);
                LSP_MFMA(nzh, qih, acc[n][2]); LSP_MFMA(zih, qrh, acc[n][3]);
                LSP_MFMA(nih, ril, acc[n][0]); LSP_MFMA(lih, rrl, acc[n][1]);
                LSP_MFMA(nzh, qil, acc[n][2]); LSP_MFMA(zih, qrl, acc[n][3]);
                LSP_MFMA(nil, rih, acc[n][0]); LSP_MFMA(lil, rrh, acc[n][1]);
                LSP_MFMA(nzl, qih, acc[n][2]); LSP_MFMA(zil, qrh, acc[n][3]);
            }
        }
    }

    // FP32 chunk sums, scales removed.  The merge subtracts one per sample that
    // pads the series to whole 64-sample tiles (what the other kernels' neutral
    // samples add to CC); here the ragged end is padded to 32 samples, whose
    // pads add 1 to Re of the second product, so CC gets the difference.
    const float ux = ldexpf(1.0f, ex - 28);   // 1 / (xscale 2^14)
    const float uz = 1.0f / (kTrigScale * kTrigScale);
    const int64_t len = je - jb;
    const int64_t p32 = (len + kMB - 1) / kMB * kMB - len;
    const int64_t p64 = (len + kTile - 1) / kTile * kTile - len;
    const float count = (float)(len - p32 + 2 * p64);
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t ar = ((int64_t)blockIdx.x * nw + wave) * 32 + 8 * (r / 4) + 4 * half + (r % 4);
            const int64_t k = ar * 64 + 32 * n + row;
            if (k < a.Nf) {
                float *p = a.part + (int64_t)split * 4 * a.Nf + k;
                p[0] = acc[n][0][r] * ux;
                p[a.Nf] = acc[n][1][r] * ux;
                p[2 * a.Nf] = 0.5f * (count + acc[n][2][r] * uz);
                p[3 * a.Nf] = 0.5f * acc[n][3][r] * uz;
            }
        }
}


}  // namespace lsp
