// tuner.cpp -- launch-shape autotuner for the single-curve periodogram.
//
// The paper picked its 256-thread block by trying sizes (Section 4.3,
// footnote on the block size).  Here the candidates are every built
// (trig mode, frequencies per lane) of the requested phase mode, crossed
// with waves per workgroup and sample-axis splits around the occupancy
// heuristic (for the split phases only the compensated-sum variants).  Each candidate is timed with HIP events on synthetic data of
// the requested size; the fastest is kept per (arch, CU count, phase,
// power-of-two bucket of Nt and of Nf), in memory and optionally in a JSON
// file.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <random>
#include <sstream>
#include <string>
#include <vector>

#include "tuner.h"

namespace lsp {

namespace {

struct Entry {
    lsp_tile tile;
    double ms;
};

std::mutex g_mu;
std::map<std::string, Entry> g_cache;

int bucket(int64_t v)
{
    int b = 0;
    while (((int64_t)1 << b) < v) ++b;
    return b;
}

std::string make_key(const std::string &arch, int cus, int phase, int64_t Nt, int64_t Nf)
{
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%s|%d|%d|%d|%d", arch.c_str(), cus, phase, bucket(Nt), bucket(Nf));
    return buf;
}

const char *default_path()
{
    const char *p = std::getenv("LSP_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

}  // namespace

bool tuner_lookup(const std::string &arch, int cus, int phase, int64_t Nt, int64_t Nf, lsp_tile *out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find(make_key(arch, cus, phase, Nt, Nf));
    if (it == g_cache.end()) return false;
    *out = it->second.tile;
    return true;
}

}  // namespace lsp

using namespace lsp;

extern "C" {

lsp_status lsp_autotune(int64_t Nt, int64_t Nf, int32_t phase, void *stream, lsp_tile *best, double *best_ms)
{
    if (Nt < 2 || Nf < 1 || Nt > ((int64_t)1 << 31) || Nf > ((int64_t)1 << 32) - 1 ||
        (phase != LSP_PHASE_SPLIT && phase != LSP_PHASE_NAIVE && phase != LSP_PHASE_SPLIT32))
        return LSP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const int cus = device_cus();
    const std::string arch = device_arch();
    if (cus <= 0) return LSP_ERR_NO_DEVICE;

    // synthetic series: sorted uniform times over Nt/2 days, Gaussian values
    std::vector<double> th((size_t)Nt);
    std::vector<float> xh((size_t)Nt);
    std::mt19937_64 g(12345);
    std::uniform_real_distribution<double> U(0.0, 0.5 * (double)Nt);
    std::normal_distribution<float> Nrm(0.f, 1.f);
    for (auto &v : th) v = U(g);
    std::sort(th.begin(), th.end());
    for (auto &v : xh) v = Nrm(g);
    const double T = th.back() - th.front();
    const double df = 1.0 / (4.0 * (T > 0 ? T : 1.0));

    double *dt = nullptr;
    float *dx = nullptr, *dp = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lsp_status result = LSP_OK;
    hipError_t e = hipMalloc(&dt, sizeof(double) * (size_t)Nt);
    if (e == hipSuccess) e = hipMalloc(&dx, sizeof(float) * (size_t)Nt);
    if (e == hipSuccess) e = hipMalloc(&dp, sizeof(float) * (size_t)Nf);
    if (e == hipSuccess) e = hipMemcpy(dt, th.data(), sizeof(double) * (size_t)Nt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dx, xh.data(), sizeof(float) * (size_t)Nt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        set_last_error(std::string("autotune setup: ") + hipGetErrorString(e));
        result = LSP_ERR_HIP;
    }

    std::vector<lsp_tile> cand;
    if (result == LSP_OK) {
        const int nv = pgram_list_tiles(phase, nullptr, 0);
        std::vector<lsp_tile> built((size_t)nv);
        pgram_list_tiles(phase, built.data(), nv);
        // the split phases keep their compensated sums: two-level variants are
        // reachable by explicit request only (the matrix-core form, whose sums
        // are the FP32 accumulators of its products, is a candidate)
        const int want_sum = (phase == LSP_PHASE_NAIVE) ? LSP_SUM_TWO : LSP_SUM_KAHAN;
        for (lsp_tile t : built)
            for (int w : {2, 4, 8}) {
                if (t.sum != want_sum && t.trig != LSP_TRIG_MFMA) continue;
                if (w == 8 && t.trig != LSP_TRIG_MFMA) continue;  // 8 waves: matrix-core form only
                if (w == 2 && t.trig == LSP_TRIG_MFMA) continue;  // too few waves to share R
                t.waves = w;
                int per_cu = 0;
                t.splits = 1;
                if (pgram_occupancy(phase, t, &per_cu) != hipSuccess) per_cu = 0;
                const int h = heuristic_splits(Nt, Nf, t.m, cus, w, per_cu);
                // around the heuristic, plus, for short grids, the finest split
                // a series allows (one 64-sample block per chunk): few
                // frequencies leave most CUs idle unless the samples split
                // (bounded so that the chunk sums stay within 2^24 floats per sum)
                int finest = (int)std::min<int64_t>(256, std::max<int64_t>(1, (Nt + 63) / 64));
                if ((int64_t)finest * Nf > ((int64_t)1 << 24)) finest = h;
                for (int sp : {h, std::max(1, (h * 3) / 4), (h * 3 + 1) / 2, 2 * h, finest}) {
                    t.splits = sp;
                    if (!pgram_tile_supported(phase, t)) continue;
                    bool dup = false;
                    for (auto &c : cand)
                        dup |= (c.trig == t.trig && c.m == t.m && c.waves == t.waves && c.splits == t.splits &&
                                c.unroll == t.unroll && c.sum == t.sum);
                    if (!dup) cand.push_back(t);
                }
            }
    }
    lsp_tile win;
    std::memset(&win, 0, sizeof(win));
    double win_ms = 1e300;
    for (const lsp_tile &t : cand) {
        if (result != LSP_OK) break;
        lsp_status st = run_single_timed(dt, dx, Nt, df, df, Nf, dp, s, phase, t);  // warm-up
        if (st != LSP_OK) {
            result = st;
            break;
        }
        // per-call time from batches of back-to-back calls between the two
        // events: one call sizes the batch to about half a millisecond, so
        // that the events' own cost and launch jitter do not rank short calls
        double best_rep = 1e300;
        int batch = 1;
        for (int r = 0; r < 4 && result == LSP_OK; ++r) {
            hipEventRecord(e0, s);
            for (int i = 0; i < batch && st == LSP_OK; ++i)
                st = run_single_timed(dt, dx, Nt, df, df, Nf, dp, s, phase, t);
            hipEventRecord(e1, s);
            if (st != LSP_OK) {
                result = st;
                break;
            }
            e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                set_last_error(std::string("autotune timing: ") + hipGetErrorString(e));
                result = LSP_ERR_HIP;
                break;
            }
            if (r == 0) {  // the sizing call
                batch = (int)std::min(50.0, std::max(1.0, 0.5 / std::max((double)ms, 1e-3)));
                continue;
            }
            best_rep = std::min(best_rep, (double)ms / batch);
        }
        if (result == LSP_OK && best_rep < win_ms) {
            win_ms = best_rep;
            win = t;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (dt) hipFree(dt);
    if (dx) hipFree(dx);
    if (dp) hipFree(dp);
    if (result != LSP_OK) return result;
    if (win.m == 0) return LSP_ERR_UNSUPPORTED;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_cache[make_key(arch, cus, phase, Nt, Nf)] = Entry{win, win_ms};
    }
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return LSP_OK;
}

int32_t lsp_list_tiles(int32_t phase, lsp_tile *out, int32_t cap)
{
    if (phase != LSP_PHASE_SPLIT && phase != LSP_PHASE_NAIVE && phase != LSP_PHASE_SPLIT32) return -1;
    return pgram_list_tiles(phase, out, cap < 0 ? 0 : cap);
}

lsp_status lsp_tune_lookup(int64_t Nt, int64_t Nf, int32_t phase, lsp_tile *tile)
{
    if (!tile || Nt < 1 || Nf < 1) return LSP_ERR_INVALID_ARG;
    const int cus = device_cus();
    if (cus <= 0) return LSP_ERR_NO_DEVICE;
    return tuner_lookup(device_arch(), cus, phase, Nt, Nf, tile) ? LSP_OK : LSP_ERR_INVALID_ARG;
}

lsp_status lsp_tune_cache_save(const char *path)
{
    if (!path) path = default_path();
    if (!path) return LSP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    std::ofstream f(path);
    if (!f) return LSP_ERR_INVALID_ARG;
    f << "{\n  \"format\": \"mi355lsp-tune-2\",\n  \"entries\": [";
    bool first = true;
    for (auto &kv : g_cache) {
        const lsp_tile &t = kv.second.tile;
        f << (first ? "\n" : ",\n") << "    {\"key\": \"" << kv.first << "\", \"trig\": " << t.trig
          << ", \"m\": " << t.m << ", \"waves\": " << t.waves << ", \"splits\": " << t.splits
          << ", \"unroll\": " << t.unroll << ", \"sum\": " << t.sum << ", \"ms\": " << kv.second.ms << "}";
        first = false;
    }
    f << "\n  ]\n}\n";
    return f.good() ? LSP_OK : LSP_ERR_INVALID_ARG;
}

// reads the flat format written above; unknown fields are ignored
lsp_status lsp_tune_cache_load(const char *path)
{
    if (!path) path = default_path();
    if (!path) return LSP_ERR_INVALID_ARG;
    std::ifstream f(path);
    if (!f) return LSP_ERR_INVALID_ARG;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    if (s.find("mi355lsp-tune-2") == std::string::npos) return LSP_ERR_INVALID_ARG;
    auto num = [&](size_t from, size_t to, const char *field, double *v) {
        const std::string pat = std::string("\"") + field + "\":";
        size_t p = s.find(pat, from);
        if (p == std::string::npos || p > to) return false;
        *v = std::strtod(s.c_str() + p + pat.size(), nullptr);
        return true;
    };
    std::map<std::string, Entry> loaded;
    size_t pos = 0;
    while ((pos = s.find("{\"key\": \"", pos)) != std::string::npos) {
        const size_t kb = pos + 9;
        const size_t ke = s.find('"', kb);
        const size_t end = s.find('}', kb);
        if (ke == std::string::npos || end == std::string::npos) return LSP_ERR_INVALID_ARG;
        double tr, m, w, sp, un, su, ms;
        if (!num(ke, end, "trig", &tr) || !num(ke, end, "m", &m) || !num(ke, end, "waves", &w) ||
            !num(ke, end, "splits", &sp) || !num(ke, end, "unroll", &un) || !num(ke, end, "sum", &su) ||
            !num(ke, end, "ms", &ms))
            return LSP_ERR_INVALID_ARG;
        // every shape field a small non-negative integer (a foreign or damaged file is refused)
        for (double v : {tr, m, w, sp, un, su})
            if (!(v >= 0.0 && v <= 1048576.0) || v != std::floor(v)) return LSP_ERR_INVALID_ARG;
        if (!std::isfinite(ms)) return LSP_ERR_INVALID_ARG;
        Entry e;
        e.tile.trig = (int32_t)tr;
        e.tile.m = (int32_t)m;
        e.tile.waves = (int32_t)w;
        e.tile.splits = (int32_t)sp;
        e.tile.unroll = (int32_t)un;
        e.tile.sum = (int32_t)su;
        e.ms = ms;
        loaded[s.substr(kb, ke - kb)] = e;
        pos = end;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &kv : loaded) g_cache[kv.first] = kv.second;
    return LSP_OK;
}

}  // extern "C"
