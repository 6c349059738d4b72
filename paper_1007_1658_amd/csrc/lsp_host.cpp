// lsp_host.cpp -- host side of the C ABI declared in include/lsp.h:
// validation, device checks, per-(device, stream) workspaces, launch-shape
// choice, hipGraph capture of batched calls, profiling hook, host helpers.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "tuner.h"

namespace lsp {

namespace {

thread_local std::string g_last_error;

constexpr int64_t kMaxNt = (int64_t)1 << 31;   // sample count limit (32-bit tile indices)
constexpr int64_t kMaxNf = ((int64_t)1 << 32) - 1;  // batched argmax key holds k in 32 bits
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

lsp_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return LSP_ERR_HIP;
}

struct DeviceInfo {
    bool ok = false;
    int cus = 0;
    std::string arch;
};

struct Buffer {
    void *ptr = nullptr;
    size_t size = 0;
    bool captured = false;       // a captured graph refers to ptr
    std::vector<void *> retired;  // outgrown buffers a captured graph may still replay into (never freed)
};

struct BatchGraph {
    uint64_t key = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct StreamCtx {
    Buffer ws;        // single-curve workspace
    Buffer bws;       // batched workspace
    Buffer mws;       // Monte-Carlo / window workspace
    uint64_t plan_key = 0;  // batch plan currently resident in bws
    BatchGraph graph;
};

struct Context {
    std::mutex mu;
    std::map<int, DeviceInfo> dev;
    std::map<std::pair<int, hipStream_t>, std::unique_ptr<StreamCtx>> streams;
    int prof = 0;  // profiling hook: bit 0 the main kernel's events, bit 1 per-call events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_calls;  // single-curve calls: first kernel .. last kernel
    std::string prof_name;
};

Context &ctx()
{
    static Context *c = new Context();  // never destroyed: safe at process exit
    return *c;
}

// requires ctx().mu held
lsp_status device_info(int *dev_out, DeviceInfo **info)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        g_last_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return LSP_ERR_NO_DEVICE;
    }
    auto it = ctx().dev.find(dev);
    if (it == ctx().dev.end()) {
        DeviceInfo di;
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e == hipSuccess) {
            di.arch = prop.gcnArchName;
            di.cus = prop.multiProcessorCount;
            di.ok = di.arch.rfind("gfx950", 0) == 0;
        }
        it = ctx().dev.emplace(dev, di).first;
    }
    if (!it->second.ok) {
        g_last_error = "device " + std::to_string(dev) + " is not gfx950 (" + it->second.arch + ")";
        return LSP_ERR_NO_DEVICE;
    }
    *dev_out = dev;
    *info = &it->second;
    return LSP_OK;
}

StreamCtx &stream_ctx(int dev, hipStream_t s)
{
    auto &p = ctx().streams[{dev, s}];
    if (!p) p.reset(new StreamCtx());
    return *p;
}

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st == hipStreamCaptureStatusActive;
}

// Sets a buffer that a captured graph refers to aside for the rest of the
// process (it is never freed); the next ensure() allocates a fresh one.
void retire(Buffer &b)
{
    if (b.ptr) b.retired.push_back(b.ptr);
    b.ptr = nullptr;
    b.size = 0;
    b.captured = false;
}

// Grow-only buffer.  It never grows while the stream is captured, and a buffer
// that a capture used is retired, not freed, when a later eager call outgrows
// it: the captured graph keeps replaying into it.
lsp_status ensure(Buffer &b, size_t need, hipStream_t s)
{
    if (stream_capturing(s)) {
        if (b.size < need) {
            g_last_error = "workspace would grow during stream capture";
            return LSP_ERR_CAPTURE;
        }
        b.captured = true;
        return LSP_OK;
    }
    if (b.size >= need) return LSP_OK;
    hipError_t e;
    if (b.ptr) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        if (b.captured) {
            b.retired.push_back(b.ptr);
        } else {
            e = hipFree(b.ptr);
            if (e != hipSuccess) return hip_fail(e, "hipFree");
        }
        b.ptr = nullptr;
        b.size = 0;
        b.captured = false;
    }
    size_t sz = std::max(need, (size_t)1 << 20);
    e = hipMalloc(&b.ptr, sz);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
    b.size = sz;
    return LSP_OK;
}

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }
bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// ---- single-curve workspace layout ----------------------------------------------
struct Layout {
    size_t stats, moments, th, tl, xv, rc, rs, part, total;
};

Layout layout(int64_t Nt, int64_t Nf, int splits, int n_mom)
{
    Layout L;
    size_t o = 0;
    L.stats = o;
    o = align_up(o + sizeof(CurveStats));
    L.moments = o;
    o = align_up(o + sizeof(Moments) * (size_t)n_mom);
    const size_t fb = align_up(sizeof(float) * (size_t)Nt);
    L.th = o;
    o += fb;
    L.tl = o;
    o += fb;
    L.xv = o;
    o += fb;
    L.rc = o;
    o += fb;
    L.rs = o;
    o += fb;
    L.part = o;
    o = align_up(o + sizeof(float) * 4 * (size_t)Nf * (size_t)splits);
    L.total = o;
    return L;
}

int moment_blocks(int64_t Nt) { return (int)std::min<int64_t>(256, std::max<int64_t>(1, (Nt + 1023) / 1024)); }

}  // namespace

// ---- launch-shape choice -------------------------------------------------------------

// Split count along the sample axis.  Resident workgroup slots come from the
// occupancy of the variant; the cost model counts dispatch rounds times the
// samples per wave (plus a fixed per-wave overhead), so that the last round is
// not a nearly empty one.  blocks_per_cu <= 0: assume two workgroups per CU.
int heuristic_splits(int64_t Nt, int64_t Nf, int m, int cus, int waves, int blocks_per_cu, int sums_per_freq)
{
    if (waves < 1) waves = 4;
    if (blocks_per_cu <= 0) blocks_per_cu = 2;
    const int64_t per_wave = (int64_t)kWave * m;
    const int64_t nfb = (Nf + per_wave - 1) / per_wave;
    const int64_t fwg = (nfb + waves - 1) / waves;
    const int64_t slots = (int64_t)cus * blocks_per_cu;
    // chunks of at least 256 samples, or down to one tile for short series
    // (Nt <= 8192), where few chunks leave most CUs idle: measured untuned
    // on MI355X, Nt 1000-5000 ran 1.3-2x faster with one-tile chunks allowed
    // and Nt 12,000 14 % slower (its per-workgroup overheads and chunk sums)
    const int64_t min_chunk = (Nt <= 8192) ? kTile : 256;
    int64_t smax = std::max<int64_t>(1, std::min<int64_t>(256, (Nt + min_chunk - 1) / min_chunk));
    // keep the per-chunk partial sums (FP32, sums_per_freq per frequency) under 1 GiB
    const double bytes_per_split = 4.0 * (double)std::max(1, sums_per_freq) * (double)Nf;
    while (smax > 1 && (double)smax * bytes_per_split > (double)(1u << 30)) --smax;
    int64_t best_s = 1;
    double best_cost = 1e300;
    for (int64_t s = 1; s <= smax; ++s) {
        int64_t chunk = (Nt + s - 1) / s;
        chunk = (chunk + kTile - 1) / kTile * kTile;
        const int64_t eff = (Nt + chunk - 1) / chunk;
        const int64_t wgs = fwg * eff;
        const int64_t rounds = (wgs + slots - 1) / slots;
        const double cost = (double)rounds * (double)(chunk + 64) + 2.0 * (double)eff;
        if (cost < best_cost * 0.999) {
            best_cost = cost;
            best_s = eff;
        }
    }
    return (int)best_s;
}

lsp_tile default_tile(int phase, int64_t Nt, int64_t Nf, int cus)
{
    lsp_tile t;
    if (phase == LSP_PHASE_NAIVE) {
        t.trig = LSP_TRIG_DIRECT;
        t.m = 1;
        t.sum = LSP_SUM_TWO;
        t.unroll = 4;
    } else if (phase == LSP_PHASE_SPLIT) {
        // matrix-core form: FP16 hi/lo products with FP32 accumulation
        t.trig = LSP_TRIG_MFMA;
        t.m = 32;
        t.sum = LSP_SUM_TWO;
        t.unroll = 1;
    } else {
        t.trig = LSP_TRIG_RECUR;
        t.m = 8;
        t.sum = LSP_SUM_KAHAN;
        t.unroll = 4;
    }
    // matrix-core form: 8-wave groups (one per CU, sharing each block's R
    // operands) from ~1e9 terms on; smaller problems want more, smaller groups
    t.waves = (t.trig == LSP_TRIG_MFMA && (double)Nt * (double)Nf >= 1e9) ? 8 : 4;
    t.splits = heuristic_splits(Nt, Nf, t.m, cus, t.waves, 0);
    return t;
}

// chunk (multiple of the tile) and effective number of splits
static void split_geometry(int64_t Nt, int splits, int64_t *chunk, int *eff)
{
    int64_t c = (Nt + splits - 1) / splits;
    c = (c + kTile - 1) / kTile * kTile;
    *chunk = c;
    *eff = (int)((Nt + c - 1) / c);
}

// Runs prep + main (+ reduce) for one curve on `s`.  Caller holds no lock.
// fixed_cap > 0: the workspace is this device's fixed scratch array instead of
// the stream's grow-only buffer (nothing is allocated); the sample axis is then
// split into no more chunks than the array holds sums for.
static lsp_status run_single(const double *t, const float *x, int64_t Nt, double f_min, double df,
                             int64_t Nf, float *Pn, hipStream_t s, int phase, lsp_tile tile,
                             const CurveStats **stats_out, bool allow_profile, size_t fixed_cap = 0)
{
    std::lock_guard<std::mutex> lock(ctx().mu);
    int dev = 0;
    DeviceInfo *di = nullptr;
    lsp_status st = device_info(&dev, &di);
    if (st != LSP_OK) return st;
    if (tile.trig == 0 || tile.m == 0 || tile.waves == 0 || tile.unroll == 0 || tile.sum == 0) {
        lsp_tile tuned;
        if (tuner_lookup(di->arch, di->cus, phase, Nt, Nf, &tuned) &&
            (tile.trig == 0 || tile.trig == tuned.trig) && (tile.m == 0 || tile.m == tuned.m)) {
            if (tile.trig == 0) tile.trig = tuned.trig;
            if (tile.m == 0) tile.m = tuned.m;
            if (tile.waves == 0) tile.waves = tuned.waves;
            if (tile.splits == 0) tile.splits = tuned.splits;
            if (tile.unroll == 0) tile.unroll = tuned.unroll;
            if (tile.sum == 0) tile.sum = tuned.sum;
        }
        const lsp_tile d = default_tile(phase, Nt, Nf, di->cus);
        if (tile.trig == 0) tile.trig = d.trig;
        if (tile.m == 0)
            tile.m = (tile.trig == d.trig) ? d.m
                                           : (tile.trig == LSP_TRIG_DIRECT ? 1 : (tile.trig == LSP_TRIG_MFMA ? 32 : 8));
        if (tile.waves == 0) tile.waves = (tile.trig == d.trig) ? d.waves : 4;
        if (tile.sum == 0 && tile.trig == d.trig && tile.m == d.m) tile.sum = d.sum;
        pgram_complete_tile(phase, tile);
    }
    if (tile.splits == 0) {
        int per_cu = 0;
        if (pgram_occupancy(phase, tile, &per_cu) != hipSuccess) per_cu = 0;
        tile.splits = heuristic_splits(Nt, Nf, tile.m, di->cus, tile.waves, per_cu);
    }
    if (!pgram_tile_supported(phase, tile)) {
        g_last_error = "launch shape not built into the library";
        return LSP_ERR_UNSUPPORTED;
    }
    const int n_mom = moment_blocks(Nt);
    char *base = nullptr;
    if (fixed_cap > 0) {
        void *p = nullptr;
        size_t cap = 0;
        const hipError_t he = noalloc_scratch(dev, &p, &cap);
        if (he != hipSuccess) return hip_fail(he, "hipGetSymbolAddress(scratch)");
        cap = std::min(cap, fixed_cap);
        const Layout L1 = layout(Nt, Nf, 1, n_mom);
        if (L1.total > cap) {
            g_last_error = "needs " + std::to_string(L1.total) + " bytes of scratch, the fixed array holds " +
                           std::to_string(cap);
            return LSP_ERR_INVALID_ARG;
        }
        const size_t per_split = sizeof(float) * 4 * (size_t)Nf;
        const size_t fit = cap >= L1.part + kAlign ? (cap - L1.part - (kAlign - 1)) / per_split : 1;
        if ((size_t)tile.splits > fit) tile.splits = (int)std::max<size_t>(1, fit);
        base = (char *)p;
    }
    int64_t chunk = 0;
    int eff = 1;
    split_geometry(Nt, tile.splits, &chunk, &eff);
    tile.splits = eff;

    const Layout L = layout(Nt, Nf, tile.splits, n_mom);
    if (!base) {
        StreamCtx &sc = stream_ctx(dev, s);
        st = ensure(sc.ws, L.total, s);
        if (st != LSP_OK) return st;
        base = (char *)sc.ws.ptr;
    }
    Records rec;
    rec.th = (float *)(base + L.th);
    rec.tl = (float *)(base + L.tl);
    rec.xv = (float *)(base + L.xv);
    rec.rc = (float *)(base + L.rc);
    rec.rs = (float *)(base + L.rs);
    rec.wv = nullptr;
    CurveStats *stats = (CurveStats *)(base + L.stats);
    // the matrix-core kernel merges the partial moments and converts the raw
    // samples itself; the other forms read records (the step rotations serve
    // the recurrence form)
    // profiling hook: events on the main kernel, and on the call's first and
    // last kernels (the whole call), all attached to the launches themselves
    hipEvent_t ev0 = nullptr, ev1 = nullptr, call0 = nullptr, call1 = nullptr;
    if (allow_profile && (ctx().prof & 1)) {
        if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
            return hip_fail(hipGetLastError(), "hipEventCreate");
        ctx().prof_events.emplace_back(ev0, ev1);
        ctx().prof_name = pgram_kernel_name(phase, tile);
    }
    if (allow_profile && (ctx().prof & 2)) {
        if (hipEventCreate(&call0) != hipSuccess || hipEventCreate(&call1) != hipSuccess)
            return hip_fail(hipGetLastError(), "hipEventCreate");
        ctx().prof_calls.emplace_back(call0, call1);
    }
    Moments *moments = (Moments *)(base + L.moments);
    const bool mfma = tile.trig == LSP_TRIG_MFMA;
    hipError_t e = mfma ? launch_moment_parts(t, x, Nt, moments, n_mom, s, call0)
                        : launch_prep(t, x, Nt, (double)kWave * df, phase, moments, n_mom, stats, rec, s, call0);
    if (e != hipSuccess) return hip_fail(e, "prep launch");

    PgramArgs a;
    a.rec = rec;
    a.stats = stats;
    a.Nt = Nt;
    a.chunk = chunk;
    a.f_min = f_min;
    a.df = df;
    a.Nf = Nf;
    a.Pn = Pn;
    a.part = (float *)(base + L.part);
    a.splits = tile.splits;
    a.refine_list = nullptr;
    a.refine_count = nullptr;
    a.refine_part = nullptr;
    a.t_raw = mfma ? t : nullptr;
    a.x_raw = mfma ? x : nullptr;
    a.mom = mfma ? moments : nullptr;
    a.n_mom = n_mom;
    a.stats_w = stats;

    e = launch_pgram(a, phase, tile, s, ev0, ev1, call1);
    if (e != hipSuccess) return hip_fail(e, "periodogram launch");
    if (stats_out) *stats_out = stats;
    return LSP_OK;
}

lsp_status run_single_timed(const double *t, const float *x, int64_t Nt, double f_min, double df,
                            int64_t Nf, float *Pn, hipStream_t s, int phase, const lsp_tile &tile)
{
    return run_single(t, x, Nt, f_min, df, Nf, Pn, s, phase, tile, nullptr, false);
}

int device_cus()
{
    std::lock_guard<std::mutex> lock(ctx().mu);
    int dev = 0;
    DeviceInfo *di = nullptr;
    if (device_info(&dev, &di) != LSP_OK) return 0;
    return di->cus;
}

std::string device_arch()
{
    std::lock_guard<std::mutex> lock(ctx().mu);
    int dev = 0;
    DeviceInfo *di = nullptr;
    if (device_info(&dev, &di) != LSP_OK) return "";
    return di->arch;
}

void set_last_error(const std::string &m) { g_last_error = m; }
void set_last_error(const char *m) { g_last_error = m ? m : ""; }

// ---- batched -------------------------------------------------------------------------

namespace {

uint64_t fnv1a(uint64_t h, const void *p, size_t n)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Host description of one batched launch.
struct BatchPlan {
    std::vector<BatchGroup> groups;
    std::vector<BatchCurve> curves;
    std::vector<BatchItem> items;
    int64_t total_t = 0;   // time samples (sum over groups)
    int64_t total_x = 0;   // value samples (sum over curves)
    int64_t total_nf = 0;  // output frequencies (sum over curves)
};

// Groups are given by off[] (host, CSR over t); curve c of group g uses the
// grid of g.  reps curves per group (Monte Carlo), values laid out curve by
// curve.  Items in longest-processing-time order.
// kernel form of the batched, Monte-Carlo and window paths (lsp_set_batched_form)
int g_batch_form = LSP_TRIG_MFMA;

void build_plan(const int64_t *off, int32_t n_groups, const double *f_min, const double *df, const int64_t *Nf,
                int32_t reps, BatchPlan &P)
{
    const int64_t per_wave = batched_freq_per_item(g_batch_form);
    P.groups.resize((size_t)n_groups);
    P.curves.resize((size_t)n_groups * (size_t)reps);
    int64_t xoff = 0, pn = 0;
    for (int32_t g = 0; g < n_groups; ++g) {
        BatchGroup &G = P.groups[(size_t)g];
        G.toff = off[g];
        G.Nt = off[g + 1] - off[g];
        G.df = df[g];
        for (int32_t r = 0; r < reps; ++r) {
            BatchCurve &cv = P.curves[(size_t)g * reps + r];
            cv.toff = G.toff;
            cv.xoff = xoff;
            cv.Nt = G.Nt;
            cv.Nf = Nf[g];
            cv.pn_off = pn;
            cv.f_min = f_min[g];
            cv.df = df[g];
            cv.group = g;
            cv.pad_ = 0;
            xoff += G.Nt;
            pn += Nf[g];
        }
    }
    P.total_t = off[n_groups];
    P.total_x = xoff;
    P.total_nf = pn;
    P.items.clear();
    for (size_t c = 0; c < P.curves.size(); ++c) {
        const int64_t nfb = (P.curves[c].Nf + per_wave - 1) / per_wave;
        for (int64_t b = 0; b < nfb; ++b) P.items.push_back(BatchItem{(int32_t)c, (int32_t)b});
    }
    // every item of curve c costs ~Nt_c * 64 m terms: longest curves first
    std::stable_sort(P.items.begin(), P.items.end(), [&](const BatchItem &a, const BatchItem &b) {
        return P.curves[(size_t)a.curve].Nt > P.curves[(size_t)b.curve].Nt;
    });
}

uint64_t plan_hash(const BatchPlan &P)
{
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &g_batch_form, sizeof(g_batch_form));
    h = fnv1a(h, P.groups.data(), sizeof(BatchGroup) * P.groups.size());
    h = fnv1a(h, P.curves.data(), sizeof(BatchCurve) * P.curves.size());
    return h;
}

struct BatchLayout {
    size_t stats, tref, groups, curves, items, queue, key, tbeg, tend, t0, th, tl, rc, rs, xv, pn, pmax, total;
};

BatchLayout batch_layout(const BatchPlan &P, bool own_pn, bool own_pmax)
{
    BatchLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t nc = P.curves.size(), ng = P.groups.size();
    L.stats = take(sizeof(CurveStats) * nc);
    L.tref = take(sizeof(double) * 3 * ng);
    L.groups = take(sizeof(BatchGroup) * ng);
    L.curves = take(sizeof(BatchCurve) * nc);
    L.items = take(sizeof(BatchItem) * P.items.size());
    L.queue = take(sizeof(uint32_t));
    L.key = take(8 * nc);
    L.tbeg = take(8 * nc);
    L.tend = take(8 * nc);
    L.t0 = take(8);
    L.th = take(4 * (size_t)P.total_t);
    L.tl = take(4 * (size_t)P.total_t);
    L.rc = take(4 * (size_t)P.total_t);
    L.rs = take(4 * (size_t)P.total_t);
    L.xv = take(4 * (size_t)P.total_x);
    L.pn = own_pn ? take(4 * (size_t)P.total_nf) : 0;
    L.pmax = own_pmax ? take(4 * nc) : 0;
    L.total = o;
    return L;
}

BatchArgs batch_args(char *b, const BatchLayout &L, const BatchPlan &P)
{
    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.th = (float *)(b + L.th);
    a.tl = (float *)(b + L.tl);
    a.rc = (float *)(b + L.rc);
    a.rs = (float *)(b + L.rs);
    a.xv = (float *)(b + L.xv);
    a.stats = (CurveStats *)(b + L.stats);
    a.t_ref = (double *)(b + L.tref);
    a.groups = (const BatchGroup *)(b + L.groups);
    a.n_groups = (int32_t)P.groups.size();
    a.curves = (const BatchCurve *)(b + L.curves);
    a.n_curves = (int32_t)P.curves.size();
    a.items = (const BatchItem *)(b + L.items);
    a.n_items = (int32_t)P.items.size();
    a.queue = (uint32_t *)(b + L.queue);
    a.key = (unsigned long long *)(b + L.key);
    a.tbeg = (unsigned long long *)(b + L.tbeg);
    a.tend = (unsigned long long *)(b + L.tend);
    a.t0 = (unsigned long long *)(b + L.t0);
    return a;
}

// copies the plan tables to the workspace (synchronous: the host vectors are temporary)
lsp_status upload_plan(char *b, const BatchLayout &L, const BatchPlan &P, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(b + L.groups, P.groups.data(), sizeof(BatchGroup) * P.groups.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b + L.curves, P.curves.data(), sizeof(BatchCurve) * P.curves.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !P.items.empty())
        e = hipMemcpyAsync(b + L.items, P.items.data(), sizeof(BatchItem) * P.items.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch plan upload");
    return LSP_OK;
}

lsp_status persistent_blocks(const DeviceInfo *di, int waves, int *blocks)
{
    int per_cu = 0;
    hipError_t e = batched_occupancy(g_batch_form, waves, &per_cu);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    *blocks = std::max(1, per_cu) * di->cus;
    return LSP_OK;
}

bool valid_groups(const int64_t *off, int32_t n, const double *f_min, const double *df, const int64_t *Nf)
{
    if (!off || !f_min || !df || !Nf || n < 1 || off[0] != 0) return false;
    for (int32_t c = 0; c < n; ++c) {
        const int64_t nt = off[c + 1] - off[c];
        if (nt < 2 || nt > kMaxNt || Nf[c] < 1 || Nf[c] > kMaxNf || !finite_nonneg(f_min[c]) ||
            !finite_pos(df[c]) || !std::isfinite(f_min[c] + (double)(Nf[c] - 1) * df[c])) {
            g_last_error = "invalid curve " + std::to_string(c);
            return false;
        }
    }
    return true;
}

}  // namespace

static lsp_status batched_impl(const double *t, const float *x, const int64_t *off, int32_t n,
                               const double *f_min, const double *df, const int64_t *Nf, float *Pn,
                               float *pmax, int64_t *kbest, double *fbest, uint64_t *t_ns, hipStream_t s)
{
    std::lock_guard<std::mutex> lock(ctx().mu);
    int dev = 0;
    DeviceInfo *di = nullptr;
    lsp_status st = device_info(&dev, &di);
    if (st != LSP_OK) return st;

    BatchPlan P;
    build_plan(off, n, f_min, df, Nf, 1, P);
    const uint64_t plan_key = plan_hash(P);
    const void *ptrs[] = {t, x, Pn, pmax, kbest, fbest, t_ns};
    const uint64_t key = fnv1a(plan_key, ptrs, sizeof(ptrs));

    StreamCtx &sc = stream_ctx(dev, s);
    const bool capturing = stream_capturing(s);
    // fast path: same shape and pointers as the cached graph
    if (!capturing && sc.graph.exec && sc.graph.key == key) {
        hipError_t e = hipGraphLaunch(sc.graph.exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        return LSP_OK;
    }
    const BatchLayout L = batch_layout(P, false, false);
    if (capturing) {
        // launched into the caller's capture: the plan must already be resident
        if (sc.plan_key != plan_key || sc.bws.size < L.total) {
            g_last_error = "batch shape not prepared before capture";
            return LSP_ERR_CAPTURE;
        }
        // the caller's graph now reads this buffer's plan tables and writes its
        // records: a later eager call with another plan must not touch it
        sc.bws.captured = true;
    } else if (sc.plan_key != plan_key || sc.bws.size < L.total) {
        // a plan that a captured graph replays is never overwritten or freed:
        // the new plan goes to a fresh buffer and the old one is retired
        if (sc.bws.captured) retire(sc.bws);
        st = ensure(sc.bws, L.total, s);
        if (st != LSP_OK) return st;
        st = upload_plan((char *)sc.bws.ptr, L, P, s);
        if (st != LSP_OK) return st;
        sc.plan_key = plan_key;
    }
    BatchArgs a = batch_args((char *)sc.bws.ptr, L, P);
    a.val_mode = VAL_INPUT;
    a.epi_mode = EPI_PN;
    a.Pn = Pn;
    a.pmax = pmax;
    a.kbest = kbest;
    a.fbest = fbest;
    a.t_ns = t_ns;
    a.t = t;
    a.x = x;
    const int waves = 4;
    int blocks = 0;
    st = persistent_blocks(di, waves, &blocks);
    if (st != LSP_OK) return st;

    hipError_t e;
    if (capturing || s == nullptr) {
        e = launch_batched(a, g_batch_form, blocks, waves, s);
        if (e != hipSuccess) return hip_fail(e, "batched launch");
        return LSP_OK;
    }
    // capture once, replay afterwards
    if (sc.graph.exec) {
        hipGraphExecDestroy(sc.graph.exec);
        hipGraphDestroy(sc.graph.graph);
        sc.graph = BatchGraph();
    }
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t el = launch_batched(a, g_batch_form, blocks, waves, s);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (el != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return hip_fail(el, "batched launch (capture)");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    sc.graph.key = key;
    sc.graph.graph = g;
    sc.graph.exec = ex;
    e = hipGraphLaunch(ex, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return LSP_OK;
}

// Monte-Carlo max power and window features: direct launches on the stream.
static lsp_status mc_or_window(const double *t, const int64_t *off, int32_t n, const double *f_min,
                               const double *df, const int64_t *Nf, int32_t reps, uint64_t seed,
                               uint64_t curve_base, float *pmax, float *feat, hipStream_t s)
{
    std::lock_guard<std::mutex> lock(ctx().mu);
    int dev = 0;
    DeviceInfo *di = nullptr;
    lsp_status st = device_info(&dev, &di);
    if (st != LSP_OK) return st;
    if (stream_capturing(s)) {
        // every call uploads its plan tables synchronously
        g_last_error = "Monte-Carlo and window calls cannot be captured";
        return LSP_ERR_CAPTURE;
    }
    const bool window = feat != nullptr;
    BatchPlan P;
    build_plan(off, n, f_min, df, Nf, window ? 1 : reps, P);
    const BatchLayout L = batch_layout(P, window, false);
    StreamCtx &sc = stream_ctx(dev, s);
    st = ensure(sc.mws, L.total, s);
    if (st != LSP_OK) return st;
    st = upload_plan((char *)sc.mws.ptr, L, P, s);
    if (st != LSP_OK) return st;
    BatchArgs a = batch_args((char *)sc.mws.ptr, L, P);
    a.val_mode = window ? VAL_ONES : VAL_NORMAL;
    a.epi_mode = window ? EPI_WINDOW : EPI_PN;
    a.seed = seed;
    a.curve_base = curve_base;
    a.Pn = window ? (float *)((char *)sc.mws.ptr + L.pn) : nullptr;
    a.pmax = window ? nullptr : pmax;
    a.t = t;
    a.x = nullptr;
    const int waves = 4;
    int blocks = 0;
    st = persistent_blocks(di, waves, &blocks);
    if (st != LSP_OK) return st;
    hipError_t e = launch_batched(a, g_batch_form, blocks, waves, s);
    if (e == hipSuccess && window) e = launch_window_features(a, feat, kFeatures, s);
    if (e != hipSuccess) return hip_fail(e, window ? "window features launch" : "Monte-Carlo launch");
    return LSP_OK;
}

}  // namespace lsp

using namespace lsp;

// =====================================================================================
// C ABI

extern "C" {

const char *lsp_status_string(lsp_status s)
{
    // a C caller may pass any int: read the bits, not the (range-limited) enum
    int code = 0;
    std::memcpy(&code, &s, sizeof(code) < sizeof(s) ? sizeof(code) : sizeof(s));
    switch (code) {
    case LSP_OK: return "ok";
    case LSP_ERR_INVALID_ARG: return "invalid argument";
    case LSP_ERR_ZERO_VARIANCE: return "zero variance (constant series)";
    case LSP_ERR_NO_DEVICE: return "no gfx950 device";
    case LSP_ERR_HIP: return "HIP runtime error";
    case LSP_ERR_MODEL: return "surrogate model error";
    case LSP_ERR_CAPTURE: return "not allowed during stream capture";
    case LSP_ERR_UNSUPPORTED: return "unsupported option";
    }
    return "unknown status";
}

const char *lsp_last_error(void) { return g_last_error.c_str(); }

const char *lsp_version(void) { return "mi355lsp 0.1.0"; }

int32_t lsp_device_count(void)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    int good = 0;
    for (int d = 0; d < n; ++d) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, d) == hipSuccess && std::string(p.gcnArchName).rfind("gfx950", 0) == 0)
            ++good;
    }
    return good;
}

lsp_status lsp_grid_paper(double t_min, double t_max, int64_t Nt, double F_over, double F_high,
                          int32_t round_to, double *f_min, double *df, int64_t *Nf)
{
    if (!f_min || !df || !Nf) return LSP_ERR_INVALID_ARG;
    if (!std::isfinite(t_min) || !std::isfinite(t_max) || !(t_max > t_min) || Nt < 2 ||
        !finite_pos(F_over) || !finite_pos(F_high) || round_to < 1)
        return LSP_ERR_INVALID_ARG;
    const double d = 1.0 / (F_over * (t_max - t_min));  // Eq. (10)
    const double nf = std::ceil(F_high * F_over * (double)Nt / 2.0 - 1e-9);  // Eq. (11)
    if (!finite_pos(d) || !(nf >= 1.0) || nf > 9e15) return LSP_ERR_INVALID_ARG;
    int64_t n = (int64_t)nf;
    n = (n + round_to - 1) / round_to * round_to;
    *df = d;
    *f_min = d;  // Eq. (9): f_i = i df, i = 1..Nf
    *Nf = n;
    return LSP_OK;
}

double lsp_fap_analytic(double Pn, int64_t Nt, int64_t Nf)
{
    if (Nt < 4 || Nf < 1 || !(Pn >= 0.0) || Pn > 0.5 * (double)Nt) return NAN;
    // Eq. (3) as -expm1(Nf * log1p(-q)), q = (1 - 2Pn/Nt)^((Nt-3)/2)
    const double lq = 0.5 * (double)(Nt - 3) * std::log1p(-2.0 * Pn / (double)Nt);
    const double q = std::exp(lq);
    if (q >= 1.0) return 1.0;
    return -std::expm1((double)Nf * std::log1p(-q));
}

lsp_status lsp_periodogram_ex(const double *t, const float *x, int64_t Nt, double f_min, double df,
                              int64_t Nf, float *Pn, void *stream, const lsp_options *opt)
{
    g_last_error.clear();
    if (!t || !x || !Pn || Nt < 2 || Nt > kMaxNt || Nf < 1 || Nf > kMaxNf || !finite_nonneg(f_min) ||
        !finite_pos(df) || !std::isfinite(f_min + (double)(Nf - 1) * df)) {
        g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    lsp_options o;
    std::memset(&o, 0, sizeof(o));
    if (opt) o = *opt;
    if (o.phase != LSP_PHASE_SPLIT && o.phase != LSP_PHASE_NAIVE && o.phase != LSP_PHASE_SPLIT32) {
        g_last_error = "unknown phase mode";
        return LSP_ERR_INVALID_ARG;
    }
    if (o.tile.trig != 0 && o.tile.trig != LSP_TRIG_DIRECT && o.tile.trig != LSP_TRIG_RECUR &&
        o.tile.trig != LSP_TRIG_MFMA) {
        g_last_error = "unknown trig mode";
        return LSP_ERR_INVALID_ARG;
    }
    if (o.tile.m < 0 || o.tile.waves < 0 || o.tile.splits < 0) {
        g_last_error = "negative launch-shape field";
        return LSP_ERR_INVALID_ARG;
    }
    if (o.phase == LSP_PHASE_NAIVE && o.tile.trig == LSP_TRIG_RECUR) {
        g_last_error = "the recurrence needs the split phase";
        return LSP_ERR_UNSUPPORTED;
    }
    if (o.phase != LSP_PHASE_SPLIT && o.tile.trig == LSP_TRIG_MFMA) {
        g_last_error = "the matrix-core form needs the split phase";
        return LSP_ERR_UNSUPPORTED;
    }
    hipStream_t s = (hipStream_t)stream;
    const CurveStats *stats = nullptr;
    lsp_status st = run_single(t, x, Nt, f_min, df, Nf, Pn, s, o.phase, o.tile, &stats, true);
    if (st != LSP_OK || !o.check) return st;
    CurveStats h;
    hipError_t e = hipMemcpyAsync(&h, stats, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "status read-back");
    return h.zero_var ? LSP_ERR_ZERO_VARIANCE : LSP_OK;
}

// the generalized (K = 1) and multi-harmonic (K = 2..4) periodograms
static lsp_status run_weighted(const double *t, const float *y, const float *w, int64_t Nt, int K, double f_min,
                               double df, int64_t Nf, float *p, int32_t waves, int32_t splits, void *stream);

lsp_status lsp_gls(const double *t, const float *y, const float *w, int64_t Nt, double f_min, double df,
                   int64_t Nf, float *p, int32_t waves, int32_t splits, void *stream)
{
    return run_weighted(t, y, w, Nt, 1, f_min, df, Nf, p, waves, splits, stream);
}

lsp_status lsp_multiharmonic(const double *t, const float *y, const float *w, int64_t Nt, int32_t K, double f_min,
                             double df, int64_t Nf, float *p, int32_t waves, int32_t splits, void *stream)
{
    if (K < 1 || K > 4) {
        g_last_error = "harmonic count K must be 1 to 4";
        return K < 1 ? LSP_ERR_INVALID_ARG : LSP_ERR_UNSUPPORTED;
    }
    return run_weighted(t, y, w, Nt, K, f_min, df, Nf, p, waves, splits, stream);
}

static lsp_status run_weighted(const double *t, const float *y, const float *w, int64_t Nt, int K, double f_min,
                               double df, int64_t Nf, float *p, int32_t waves, int32_t splits, void *stream)
{
    if (!t || !y || !p || Nt < 2 * K + 1 || Nt > kMaxNt || Nf < 1 || Nf > kMaxNf || !finite_nonneg(f_min) ||
        !finite_pos(df) || !std::isfinite(f_min + (double)(Nf - 1) * df)) {
        g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    if (waves != 0 && waves != 1 && waves != 2 && waves != 4 && !(K == 1 && waves == 8)) {
        g_last_error = "waves must be 0 (library's choice), 1, 2 or 4 (generalized periodogram: also 8)";
        return LSP_ERR_INVALID_ARG;
    }
    if (splits < 0) {
        g_last_error = "negative split count";
        return LSP_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(ctx().mu);
    int dev = 0;
    DeviceInfo *di = nullptr;
    lsp_status st = device_info(&dev, &di);
    if (st != LSP_OK) return st;
    if (waves == 0) waves = 4;
    if (splits == 0) {
        // up to 4 waves: conjugate pairs, one wave per SIMD, 64 frequencies
        // per a-row (the multi-harmonic kernels always; GLS with 8 waves:
        // complex products, 32 per a-row)
        const bool pm = waves <= 4;
        const int per_wave = (K == 1) ? (pm ? kGlsPmFreqPerWave : kGlsFreqPerWave) : kMhFreqPerWave;
        splits = heuristic_splits(Nt, Nf, per_wave / kWave, di->cus, waves, pm ? 4 / waves : 2,
                                  (K == 1) ? 6 : 6 * K);
    }
    int64_t chunk = 0;
    int eff = 1;
    split_geometry(Nt, splits, &chunk, &eff);

    // workspace: stats, moments, th, tl, xv, wv, six partial sums per chunk
    const int n_mom = moment_blocks(Nt);
    size_t o = 0;
    const size_t o_stats = o;
    o = align_up(o + sizeof(CurveStats));
    const size_t o_mom = o;
    o = align_up(o + sizeof(Moments) * (size_t)n_mom);
    const size_t fb = align_up(sizeof(float) * (size_t)Nt);
    const size_t o_th = o, o_tl = o + fb, o_xv = o + 2 * fb, o_wv = o + 3 * fb;
    o += 4 * fb;
    const size_t o_part = o;
    const int slots = (K == 1) ? 6 : 6 * K;  // partial sums per frequency and chunk
    o = align_up(o + sizeof(float) * (size_t)slots * (size_t)Nf * (size_t)eff);
    const size_t o_list = o;  // bins listed for the FP64 recomputation, and their count
    o = align_up(o + sizeof(uint32_t) * (size_t)Nf);
    const size_t o_count = o;
    o = align_up(o + sizeof(uint32_t));
    const size_t o_rpart = o;  // partial FP64 sums of bins split over workgroups
    o = align_up(o + sizeof(double) * (size_t)kRefineBlocks * (size_t)(6 * K + 2));
    StreamCtx &sc = stream_ctx(dev, s);
    st = ensure(sc.ws, o, s);
    if (st != LSP_OK) return st;
    char *base = (char *)sc.ws.ptr;
    Records rec;
    rec.th = (float *)(base + o_th);
    rec.tl = (float *)(base + o_tl);
    rec.xv = (float *)(base + o_xv);
    rec.wv = (float *)(base + o_wv);
    rec.rc = nullptr;
    rec.rs = nullptr;
    CurveStats *stats = (CurveStats *)(base + o_stats);
    uint32_t *refine_count = (uint32_t *)(base + o_count);
    hipError_t e = launch_prep_weighted(t, y, w, Nt, (Moments *)(base + o_mom), n_mom, stats, rec, refine_count, s);
    if (e != hipSuccess) return hip_fail(e, "prep launch");
    PgramArgs a;
    a.rec = rec;
    a.stats = stats;
    a.Nt = Nt;
    a.chunk = chunk;
    a.f_min = f_min;
    a.df = df;
    a.Nf = Nf;
    a.Pn = p;
    a.part = (float *)(base + o_part);
    a.splits = eff;
    a.refine_list = (uint32_t *)(base + o_list);
    a.refine_count = refine_count;
    a.refine_part = (double *)(base + o_rpart);
    a.t_raw = nullptr;
    a.x_raw = nullptr;
    a.mom = nullptr;
    a.n_mom = 0;
    a.stats_w = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx().prof & 1) {
        if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
            return hip_fail(hipGetLastError(), "hipEventCreate");
        ctx().prof_events.emplace_back(ev0, ev1);
        ctx().prof_name = (K == 1) ? (waves <= 4 ? "gls_pm_kernel" : "gls_mfma_kernel") : "mh_mfma_kernel";
    }
    e = (K == 1) ? launch_gls(a, waves, s, ev0, ev1) : launch_mh(a, K, waves, s, ev0, ev1);
    if (e != hipSuccess) return hip_fail(e, "generalized periodogram launch");
    return LSP_OK;
}

lsp_status lsp_set_batched_form(int32_t trig)
{
    if (trig != LSP_TRIG_RECUR && trig != LSP_TRIG_MFMA) {
        g_last_error = "batched form must be LSP_TRIG_RECUR or LSP_TRIG_MFMA";
        return LSP_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(ctx().mu);
    g_batch_form = trig;
    return LSP_OK;
}

int32_t lsp_get_batched_form(void) { return g_batch_form; }

lsp_status lsp_periodogram(const double *t, const float *x, int64_t Nt, double f_min, double df,
                           int64_t Nf, float *Pn, void *stream)
{
    return lsp_periodogram_ex(t, x, Nt, f_min, df, Nf, Pn, stream, nullptr);
}

lsp_status lsp_periodogram_noalloc(const double *t, const float *x, int64_t Nt, double f_min, double df,
                                   int64_t Nf, float *Pn, void *stream)
{
    g_last_error.clear();
    if (!t || !x || !Pn || Nt < 2 || Nt > kMaxNt || Nf < 1 || Nf > kMaxNf || !finite_nonneg(f_min) ||
        !finite_pos(df) || !std::isfinite(f_min + (double)(Nf - 1) * df)) {
        g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    // the smallest workspace (one chunk of samples) must fit the fixed array
    const Layout L1 = layout(Nt, Nf, 1, moment_blocks(Nt));
    if (L1.total > (size_t)LSP_NOALLOC_SCRATCH_BYTES) {
        g_last_error = "needs " + std::to_string(L1.total) + " bytes of scratch, the fixed array holds " +
                       std::to_string((size_t)LSP_NOALLOC_SCRATCH_BYTES);
        return LSP_ERR_INVALID_ARG;
    }
    lsp_tile tile;
    std::memset(&tile, 0, sizeof(tile));
    return run_single(t, x, Nt, f_min, df, Nf, Pn, (hipStream_t)stream, LSP_PHASE_SPLIT, tile, nullptr, false,
                      (size_t)LSP_NOALLOC_SCRATCH_BYTES);
}

lsp_status lsp_periodogram_batched(const double *t, const float *x, const int64_t *off, int32_t n_curves,
                                   const double *f_min, const double *df, const int64_t *Nf, float *Pn,
                                   float *pmax, int64_t *kbest, double *fbest, uint64_t *t_ns,
                                   void *stream)
{
    g_last_error.clear();
    if (!t || !x || !pmax || !valid_groups(off, n_curves, f_min, df, Nf)) {
        if (g_last_error.empty()) g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    return batched_impl(t, x, off, n_curves, f_min, df, Nf, Pn, pmax, kbest, fbest, t_ns, (hipStream_t)stream);
}

lsp_status lsp_mc_maxpower(const double *t, const int64_t *off, int32_t n_pat, const double *f_min,
                           const double *df, const int64_t *Nf, int32_t R, uint64_t seed, uint64_t stream_base,
                           float *pmax, void *stream)
{
    g_last_error.clear();
    if (!t || !pmax || R < 1 || !valid_groups(off, n_pat, f_min, df, Nf) ||
        (int64_t)n_pat * (int64_t)R > ((int64_t)1 << 31) - 1) {
        if (g_last_error.empty()) g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    return mc_or_window(t, off, n_pat, f_min, df, Nf, R, seed, stream_base, pmax, nullptr, (hipStream_t)stream);
}

lsp_status lsp_window_features(const double *t, const int64_t *off, int32_t n_pat, const double *f_min,
                               const double *df, const int64_t *Nf, float *feat, void *stream)
{
    g_last_error.clear();
    if (!t || !feat || !valid_groups(off, n_pat, f_min, df, Nf)) {
        if (g_last_error.empty()) g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    return mc_or_window(t, off, n_pat, f_min, df, Nf, 1, 0, 0, nullptr, feat, (hipStream_t)stream);
}

lsp_status lsp_normals(uint64_t seed, uint64_t stream_id, int64_t n, float *out, void *stream)
{
    g_last_error.clear();
    if (!out || n < 0 || n > ((int64_t)1 << 32)) return LSP_ERR_INVALID_ARG;
    if (n == 0) return LSP_OK;
    std::lock_guard<std::mutex> lock(ctx().mu);
    int dev = 0;
    DeviceInfo *di = nullptr;
    lsp_status st = device_info(&dev, &di);
    if (st != LSP_OK) return st;
    hipError_t e = launch_normals(seed, stream_id, n, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "normals launch");
    return LSP_OK;
}

// ---- probes ------------------------------------------------------------------------

static lsp_status probe_device()
{
    std::lock_guard<std::mutex> lock(ctx().mu);
    int dev = 0;
    DeviceInfo *di = nullptr;
    return device_info(&dev, &di);
}

lsp_status lsp_probe_sincos(const float *r, int64_t n, float *s, float *c, void *stream)
{
    g_last_error.clear();
    if (n < 0 || (n > 0 && (!r || !s || !c))) {
        g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    if (n == 0) return LSP_OK;
    lsp_status st = probe_device();
    if (st != LSP_OK) return st;
    hipError_t e = launch_probe_sincos(r, n, s, c, (hipStream_t)stream);
    return e == hipSuccess ? LSP_OK : hip_fail(e, "probe launch");
}

lsp_status lsp_probe_cmac(const float *L, const float *R, int32_t K, float *P, void *stream)
{
    g_last_error.clear();
    if (!L || !R || !P || K < 16 || K > 4096 || K % 16 != 0) {
        g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    lsp_status st = probe_device();
    if (st != LSP_OK) return st;
    hipError_t e = launch_probe_cmac(L, R, K, P, (hipStream_t)stream);
    return e == hipSuccess ? LSP_OK : hip_fail(e, "probe launch");
}

lsp_status lsp_probe_cpair(const float *L, const float *R, int32_t K, float *Pp, float *Pm, void *stream)
{
    g_last_error.clear();
    if (!L || !R || !Pp || !Pm || K < 16 || K > 4096 || K % 16 != 0) {
        g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    lsp_status st = probe_device();
    if (st != LSP_OK) return st;
    hipError_t e = launch_probe_cpair(L, R, K, Pp, Pm, (hipStream_t)stream);
    return e == hipSuccess ? LSP_OK : hip_fail(e, "probe launch");
}

lsp_status lsp_probe_phase(const double *t, const double *f, int64_t n, double t_ref, int32_t phase, float *phi,
                           void *stream)
{
    g_last_error.clear();
    if (n < 0 || (n > 0 && (!t || !f || !phi)) || !std::isfinite(t_ref) ||
        (phase != LSP_PHASE_SPLIT && phase != LSP_PHASE_SPLIT32 && phase != LSP_PHASE_NAIVE)) {
        g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    if (n == 0) return LSP_OK;
    lsp_status st = probe_device();
    if (st != LSP_OK) return st;
    hipError_t e = launch_probe_phase(t, f, n, t_ref, phase, phi, (hipStream_t)stream);
    return e == hipSuccess ? LSP_OK : hip_fail(e, "probe launch");
}

lsp_status lsp_probe_recurrence(const double *t, int64_t n, double t_ref, double f0, double step_df, int32_t M,
                                float *c, float *s, void *stream)
{
    g_last_error.clear();
    if (n < 0 || (n > 0 && (!t || !c || !s)) || !std::isfinite(t_ref) || !std::isfinite(f0) ||
        !std::isfinite(step_df) || M < 1 || M > probe_recur_max() || n > ((int64_t)1 << 40) / M) {
        g_last_error = "invalid argument";
        return LSP_ERR_INVALID_ARG;
    }
    if (n == 0) return LSP_OK;
    lsp_status st = probe_device();
    if (st != LSP_OK) return st;
    hipError_t e = launch_probe_recur(t, n, t_ref, f0, step_df, M, c, s, (hipStream_t)stream);
    return e == hipSuccess ? LSP_OK : hip_fail(e, "probe launch");
}

lsp_status lsp_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lock(ctx().mu);
    for (auto *v : {&ctx().prof_events, &ctx().prof_calls}) {
        for (auto &p : *v) {
            hipEventDestroy(p.first);
            hipEventDestroy(p.second);
        }
        v->clear();
    }
    ctx().prof_name.clear();
    ctx().prof = on & 3;
    return LSP_OK;
}

lsp_status lsp_profile_read(double *total_ms, int64_t *launches, char *name, int32_t name_len)
{
    std::lock_guard<std::mutex> lock(ctx().mu);
    double tot = 0.0;
    for (auto &p : ctx().prof_events) {
        hipError_t e = hipEventSynchronize(p.second);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p.first, p.second);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int64_t)ctx().prof_events.size();
    if (name && name_len > 0) {
        std::strncpy(name, ctx().prof_name.c_str(), (size_t)name_len - 1);
        name[name_len - 1] = 0;
    }
    return LSP_OK;
}

lsp_status lsp_profile_read_calls(double *ms, int64_t cap, int64_t *calls)
{
    if (cap < 0 || (cap > 0 && !ms)) {
        g_last_error = "ms must hold cap values";
        return LSP_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(ctx().mu);
    const auto &v = ctx().prof_calls;
    for (size_t i = 0; i < v.size() && (int64_t)i < cap; ++i) {
        hipError_t e = hipEventSynchronize(v[i].second);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float t = 0.f;
        e = hipEventElapsedTime(&t, v[i].first, v[i].second);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        ms[i] = t;
    }
    if (calls) *calls = (int64_t)v.size();
    return LSP_OK;
}

}  // extern "C"
