// fast_host.cpp -- host side of the extirpolation + FFT periodogram
// (Press & Rybicki 1989, cited in Section 1): argument checks, workspace,
// the cached hipFFT plans (FP64 real-to-complex, two transforms per plan)
// and the launch sequence moments -> extirpolation -> FFT -> Eq. (5).
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

namespace lsp {
namespace {

struct FastState {
    std::mutex mu;
    // plans and workspaces per (device, stream, N)
    std::map<std::pair<int, hipStream_t>, std::map<int64_t, hipfftHandle>> plans;
    std::map<std::pair<int, hipStream_t>, std::pair<void *, size_t>> ws;
    std::map<std::pair<int, hipStream_t>, bool> captured;  // a captured graph refers to ws
    std::vector<void *> retired;                            // outgrown captured workspaces (never freed)
};

FastState &fs()
{
    static FastState *s = new FastState();  // lives until the process ends
    return *s;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

lsp_status fail(const char *what, hipError_t e)
{
    set_last_error(std::string(what) + ": " + hipGetErrorString(e));
    return LSP_ERR_HIP;
}

}  // namespace

int64_t fast_grid_size(int64_t k_max, int macc)
{
    const int64_t need = 4 * (int64_t)macc * std::max<int64_t>(k_max, 1);
    int64_t n = 1;
    while (n < need) n <<= 1;
    return n;
}

}  // namespace lsp

using namespace lsp;

extern "C" lsp_status lsp_periodogram_fast(const double *t, const float *x, int64_t Nt, double f_min, double df,
                                           int64_t Nf, int32_t macc, float *Pn, void *stream)
{
    if (!t || !x || !Pn || Nt < 2 || Nf < 1 || !(df > 0.0) || !std::isfinite(df) || !(f_min >= 0.0) ||
        !std::isfinite(f_min) || (macc != 4 && macc != 6 && macc != 8)) {
        set_last_error("invalid argument");
        return LSP_ERR_INVALID_ARG;
    }
    const double q = f_min / df;
    const int64_t m0 = (int64_t)std::llround(q);
    if (std::fabs(q - (double)m0) > 1e-9 * std::max(1.0, q)) {
        set_last_error("f_min must be a whole multiple of df");
        return LSP_ERR_INVALID_ARG;
    }
    const int64_t N = fast_grid_size(m0 + Nf - 1, macc);
    if (N > ((int64_t)1 << 28) || Nt > ((int64_t)1 << 31)) {
        set_last_error("grid too large (4 macc f_max / df > 2^28)");
        return LSP_ERR_INVALID_ARG;
    }
    if (lsp_device_count() < 1) return LSP_ERR_NO_DEVICE;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail("hipGetDevice", e);
    hipStream_t s = (hipStream_t)stream;
    FastState &F = fs();
    std::lock_guard<std::mutex> lock(F.mu);
    const auto key = std::make_pair(dev, s);

    // workspace: stats | moments | grids (2N doubles) | spectra (2 (N/2+1) complex)
    const int n_mom = (int)std::min<int64_t>(256, std::max<int64_t>(1, (Nt + 1023) / 1024));
    const size_t o_stats = 0;
    const size_t o_mom = align256(sizeof(CurveStats));
    const size_t o_grid = o_mom + align256(sizeof(Moments) * (size_t)n_mom);
    const size_t o_spec = o_grid + align256(sizeof(double) * 2 * (size_t)N);
    const size_t total = o_spec + align256(sizeof(double) * 4 * (size_t)(N / 2 + 1));
    auto &w = F.ws[key];
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusActive;
    if (capturing && (w.second < total || F.plans[key].find(N) == F.plans[key].end())) {
        set_last_error("workspace or FFT plan would be created during stream capture (call once uncaptured first)");
        return LSP_ERR_CAPTURE;
    }
    if (capturing) F.captured[key] = true;
    if (w.second < total) {
        if (w.first) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return fail("workspace release", e);
            if (F.captured[key]) {
                F.retired.push_back(w.first);  // a captured graph may still replay into it
            } else {
                e = hipFree(w.first);
                if (e != hipSuccess) return fail("workspace release", e);
            }
            F.captured[key] = false;
            w.first = nullptr;
            w.second = 0;
        }
        e = hipMalloc(&w.first, total);
        if (e != hipSuccess) return fail("hipMalloc(fast workspace)", e);
        w.second = total;
    }
    char *base = (char *)w.first;
    CurveStats *stats = (CurveStats *)(base + o_stats);

    auto &pl = F.plans[key];
    hipfftHandle plan;
    auto it = pl.find(N);
    if (it == pl.end()) {
        int n = (int)N;
        if (hipfftPlanMany(&plan, 1, &n, nullptr, 1, n, nullptr, 1, n / 2 + 1, HIPFFT_D2Z, 2) != HIPFFT_SUCCESS) {
            set_last_error("hipfftPlanMany failed");
            return LSP_ERR_HIP;
        }
        pl[N] = plan;
    } else {
        plan = it->second;
    }
    if (hipfftSetStream(plan, s) != HIPFFT_SUCCESS) {
        set_last_error("hipfftSetStream failed");
        return LSP_ERR_HIP;
    }
    e = launch_moments(t, x, Nt, (Moments *)(base + o_mom), n_mom, stats, s);
    if (e == hipSuccess) e = launch_fast_extirp(t, x, Nt, stats, df, N, macc, (double *)(base + o_grid), s);
    if (e != hipSuccess) return fail("extirpolation launch", e);
    if (hipfftExecD2Z(plan, (hipfftDoubleReal *)(base + o_grid), (hipfftDoubleComplex *)(base + o_spec)) !=
        HIPFFT_SUCCESS) {
        set_last_error("hipfftExecD2Z failed");
        return LSP_ERR_HIP;
    }
    e = launch_fast_epilogue(base + o_spec, N, m0, Nf, Nt, stats, Pn, s);
    if (e != hipSuccess) return fail("epilogue launch", e);
    return LSP_OK;
}
