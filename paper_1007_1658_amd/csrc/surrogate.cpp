// surrogate.cpp -- host side of the false-alarm surrogate: model lifecycle,
// forward / backward / Adam orchestration of the BF16-MFMA kernels, and the
// FAP entry point with its Monte-Carlo fallback.
//
// The maximum of a white-noise periodogram over Nf correlated frequencies has
// no closed-form law (Eq. (3) assumes independent frequencies, Section 3, and
// Section 6.2 points to simulations for the effective number); the surrogate
// learns the law of that maximum (a Gumbel law in the exponential-equivalent
// power, two numbers per pattern, from which the nine reported quantiles and
// the FAP follow) from Monte-Carlo periodograms this library generates, and
// keeps plain Monte Carlo as its fallback.
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "internal.h"
#include "mlp.h"

namespace lsp {
namespace {

struct LayerShape {
    int out_p, in_p, out, in;
    size_t w, b;  // offsets in the padded flat buffer
};

constexpr LayerShape kL[kMlpLayers] = {
    {kMlpHidden, kMlpInPad, kMlpHidden, kMlpIn, 0, 256 * 96},
    {kMlpHidden, kMlpHidden, kMlpHidden, kMlpHidden, 256 * 96 + 256, 256 * 96 + 256 + 65536},
    {kMlpHidden, kMlpHidden, kMlpHidden, kMlpHidden, 256 * 96 + 256 + 65536 + 256,
     256 * 96 + 256 + 2 * 65536 + 256},
    {kMlpOutPad, kMlpHidden, kMlpOut, kMlpHidden, 256 * 96 + 256 + 2 * 65536 + 2 * 256,
     256 * 96 + 256 + 2 * 65536 + 2 * 256 + 32 * 256},
};
constexpr size_t kPadded = 256 * 96 + 256 + 2 * (65536 + 256) + 32 * 256 + 32;
constexpr int64_t kParams = 256 * 68 + 256 + 2 * (65536 + 256) + kMlpOut * 256 + kMlpOut;  // unpadded, per member

size_t round32(size_t v) { return (v + 31) / 32 * 32; }

// The error bound lsp_fap_surrogate reports is this many standard errors
// (the two-sided 99 % point of the normal law).
constexpr float kBoundZ = 2.5758293f;

}  // namespace
}  // namespace lsp

using namespace lsp;

struct lsp_model {
    int members = 0;
    uint64_t seed = 0;
    float feat_mean[kMlpIn];
    float feat_std[kMlpIn];
    float feat_zmax = 1e30f;  // patterns whose standardized features exceed this fall back to Monte Carlo
    float q_mu = 0.f, q_sigma = 1.f;
    // calibrated standard errors of the law's location m and scale beta on
    // patterns kept out of training (0: the members' spread alone)
    float law_err[2] = {0.f, 0.f};
    std::vector<float *> P, G, M1, M2;
    std::vector<int> step;
    std::vector<std::array<__bf16 *, kMlpLayers>> Wb, WbT;
    float *d_mean = nullptr, *d_std = nullptr;
    // activation workspace for batches up to cap rows
    size_t cap = 0;
    __bf16 *X = nullptr, *XT = nullptr;
    float *Z[3] = {nullptr, nullptr, nullptr};
    __bf16 *H[3] = {nullptr, nullptr, nullptr}, *HT[3] = {nullptr, nullptr, nullptr};
    float *raw = nullptr;
    float *dZ[2] = {nullptr, nullptr};
    __bf16 *dZb[2] = {nullptr, nullptr}, *dZbT[2] = {nullptr, nullptr};
    float *dR = nullptr;
    __bf16 *dRb = nullptr, *dRbT = nullptr;
    float *loss_b = nullptr, *zmax = nullptr, *law = nullptr;  // law: [members][B][2] (m, beta)
    std::vector<void *> ws;  // everything of the activation workspace, for freeing
    std::mutex mu;
};

namespace {

lsp_status fail(hipError_t e, const char *what)
{
    set_last_error(std::string(what) + ": " + hipGetErrorString(e));
    return LSP_ERR_HIP;
}

template <class T>
hipError_t dalloc(T **p, size_t n, std::vector<void *> *track)
{
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (n ? n : 1));
    if (e == hipSuccess && track) track->push_back((void *)*p);
    return e;
}

hipError_t ensure_ws(lsp_model *m, size_t Bp, hipStream_t s)
{
    if (Bp <= m->cap) return hipSuccess;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (void *p : m->ws) hipFree(p);
    m->ws.clear();
    const size_t H = kMlpHidden;
    e = dalloc(&m->X, Bp * kMlpInPad, &m->ws);
    if (e == hipSuccess) e = dalloc(&m->XT, Bp * kMlpInPad, &m->ws);
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        e = dalloc(&m->Z[l], Bp * H, &m->ws);
        if (e == hipSuccess) e = dalloc(&m->H[l], Bp * H, &m->ws);
        if (e == hipSuccess) e = dalloc(&m->HT[l], Bp * H, &m->ws);
    }
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = dalloc(&m->dZ[i], Bp * H, &m->ws);
        if (e == hipSuccess) e = dalloc(&m->dZb[i], Bp * H, &m->ws);
        if (e == hipSuccess) e = dalloc(&m->dZbT[i], Bp * H, &m->ws);
    }
    if (e == hipSuccess) e = dalloc(&m->raw, Bp * kMlpOutPad, &m->ws);
    if (e == hipSuccess) e = dalloc(&m->dR, Bp * kMlpOutPad, &m->ws);
    if (e == hipSuccess) e = dalloc(&m->dRb, Bp * kMlpOutPad, &m->ws);
    if (e == hipSuccess) e = dalloc(&m->dRbT, Bp * kMlpOutPad, &m->ws);
    if (e == hipSuccess) e = dalloc(&m->loss_b, Bp, &m->ws);
    if (e == hipSuccess) e = dalloc(&m->zmax, Bp, &m->ws);
    if (e == hipSuccess) e = dalloc(&m->law, (size_t)m->members * Bp * 2, &m->ws);
    m->cap = (e == hipSuccess) ? Bp : 0;
    return e;
}

hipError_t cast_all(lsp_model *m, int e_, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int l = 0; l < kMlpLayers && e == hipSuccess; ++l)
        e = launch_cast_weights(m->P[e_] + kL[l].w, kL[l].out_p, kL[l].in_p, m->Wb[e_][l], m->WbT[e_][l], s);
    return e;
}

GemmArgs gemm(const __bf16 *A, int lda, const __bf16 *B, int ldb, int M, int N, int K, int epi)
{
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    g.epi = epi;
    return g;
}

// forward of member e on Bp padded rows (features already in X/XT); raw outputs in m->raw
hipError_t forward_member(lsp_model *m, int e_, int Bp, hipStream_t s)
{
    hipError_t e = hipSuccess;
    const __bf16 *in = m->X;
    int ld_in = kMlpInPad, K = kMlpInPad;
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        GemmArgs g = gemm(in, ld_in, m->Wb[e_][l], kL[l].in_p, Bp, kMlpHidden, K, GEMM_BIAS_GELU);
        g.bias = m->P[e_] + kL[l].b;
        g.C = m->Z[l];
        g.ldc = kMlpHidden;
        g.Cb = m->H[l];
        g.ldcb = kMlpHidden;
        g.CbT = m->HT[l];
        g.ldcbT = Bp;
        e = launch_gemm_nt(g, s);
        in = m->H[l];
        ld_in = kMlpHidden;
        K = kMlpHidden;
    }
    if (e != hipSuccess) return e;
    GemmArgs g = gemm(in, ld_in, m->Wb[e_][3], kL[3].in_p, Bp, kMlpOutPad, K, GEMM_BIAS);
    g.bias = m->P[e_] + kL[3].b;
    g.C = m->raw;
    g.ldc = kMlpOutPad;
    return launch_gemm_nt(g, s);
}

// likelihood loss and backward of member e into m->G[e]; loss (device scalar) optional
hipError_t backward_member(lsp_model *m, int e_, const float *feat, int B, int Bp, const float *y, int R, float *loss,
                           hipStream_t s)
{
    hipError_t e = launch_gumbel_nll(m->raw, kMlpOutPad, feat, B, Bp, y, R, m->q_mu, m->q_sigma, m->loss_b, m->dR,
                                     m->dRb, m->dRbT, s);
    if (e == hipSuccess && loss) e = launch_sum(m->loss_b, B, loss, s);
    float *G = m->G[e_];
    // layer 4: dW4 = dR^T H3, db4 = colsum dR, dZ3 = (dR W4) * gelu'(Z3)
    const float *dz = m->dR;
    const __bf16 *dzb = m->dRb, *dzbT = m->dRbT;
    int n_out = kMlpOutPad;
    int ping = 0;
    for (int l = 3; l >= 0 && e == hipSuccess; --l) {
        const __bf16 *inT = (l == 0) ? m->XT : m->HT[l - 1];
        const int in_p = kL[l].in_p;
        GemmArgs gw = gemm(dzbT, Bp, inT, Bp, n_out, in_p, Bp, GEMM_STORE);
        gw.C = G + kL[l].w;
        gw.ldc = in_p;
        e = launch_gemm_nt(gw, s);
        if (e == hipSuccess) e = launch_colsum(dz, B, n_out, G + kL[l].b, s);
        if (l == 0 || e != hipSuccess) break;
        GemmArgs gx = gemm(dzb, n_out, m->WbT[e_][l], kL[l].out_p, Bp, in_p, n_out, GEMM_DGELU);
        gx.Z = m->Z[l - 1];
        gx.ldz = kMlpHidden;
        gx.C = m->dZ[ping];
        gx.ldc = kMlpHidden;
        gx.Cb = m->dZb[ping];
        gx.ldcb = kMlpHidden;
        gx.CbT = m->dZbT[ping];
        gx.ldcbT = Bp;
        e = launch_gemm_nt(gx, s);
        dz = m->dZ[ping];
        dzb = m->dZb[ping];
        dzbT = m->dZbT[ping];
        n_out = kMlpHidden;
        ping ^= 1;
    }
    return e;
}

// unpadded flat <-> padded device buffer
hipError_t copy_params(float *padded, float *flat, bool to_flat, hipMemcpyKind kind, hipStream_t s)
{
    size_t o = 0;
    hipError_t e = hipSuccess;
    for (int l = 0; l < kMlpLayers && e == hipSuccess; ++l) {
        const LayerShape &L = kL[l];
        float *pw = padded + L.w, *fw = flat + o;
        if (to_flat)
            e = hipMemcpy2DAsync(fw, sizeof(float) * L.in, pw, sizeof(float) * L.in_p, sizeof(float) * L.in, L.out,
                                 kind, s);
        else
            e = hipMemcpy2DAsync(pw, sizeof(float) * L.in_p, fw, sizeof(float) * L.in, sizeof(float) * L.in, L.out,
                                 kind, s);
        o += (size_t)L.out * L.in;
        if (e != hipSuccess) break;
        if (to_flat)
            e = hipMemcpyAsync(flat + o, padded + L.b, sizeof(float) * L.out, kind, s);
        else
            e = hipMemcpyAsync(padded + L.b, flat + o, sizeof(float) * L.out, kind, s);
        o += (size_t)L.out;
    }
    return e;
}

bool good_model(const lsp_model *m) { return m && m->members > 0 && (int)m->P.size() == m->members; }

lsp_status alloc_model(lsp_model *m)
{
    hipError_t e = hipSuccess;
    for (int i = 0; i < m->members && e == hipSuccess; ++i) {
        float *P, *G, *M1, *M2;
        e = dalloc(&P, kPadded, nullptr);
        if (e == hipSuccess) e = dalloc(&G, kPadded, nullptr);
        if (e == hipSuccess) e = dalloc(&M1, kPadded, nullptr);
        if (e == hipSuccess) e = dalloc(&M2, kPadded, nullptr);
        if (e != hipSuccess) break;
        m->P.push_back(P);
        m->G.push_back(G);
        m->M1.push_back(M1);
        m->M2.push_back(M2);
        m->step.push_back(0);
        std::array<__bf16 *, kMlpLayers> wb{}, wbt{};
        for (int l = 0; l < kMlpLayers && e == hipSuccess; ++l) {
            e = dalloc(&wb[l], (size_t)kL[l].out_p * kL[l].in_p, nullptr);
            if (e == hipSuccess) e = dalloc(&wbt[l], (size_t)kL[l].out_p * kL[l].in_p, nullptr);
        }
        m->Wb.push_back(wb);
        m->WbT.push_back(wbt);
    }
    if (e == hipSuccess) e = dalloc(&m->d_mean, kMlpIn, nullptr);
    if (e == hipSuccess) e = dalloc(&m->d_std, kMlpIn, nullptr);
    return e == hipSuccess ? LSP_OK : fail(e, "model allocation");
}

lsp_status upload_scalers(lsp_model *m)
{
    hipError_t e = hipMemcpy(m->d_mean, m->feat_mean, sizeof(m->feat_mean), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_std, m->feat_std, sizeof(m->feat_std), hipMemcpyHostToDevice);
    return e == hipSuccess ? LSP_OK : fail(e, "scaler upload");
}

const char kMagic[16] = "MI355LSP-FAP-2";

}  // namespace

extern "C" {

int64_t lsp_model_param_count(void) { return kParams; }

lsp_status lsp_model_create(int32_t members, uint64_t seed, lsp_model **out)
{
    if (!out || members < 1 || members > 16) return LSP_ERR_INVALID_ARG;
    *out = nullptr;
    if (lsp_device_count() < 1) return LSP_ERR_NO_DEVICE;
    lsp_model *m = new lsp_model();
    m->members = members;
    m->seed = seed;
    for (int i = 0; i < kMlpIn; ++i) {
        m->feat_mean[i] = 0.f;
        m->feat_std[i] = 1.f;
    }
    lsp_status st = alloc_model(m);
    if (st == LSP_OK) st = upload_scalers(m);
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases, padding zero
    std::vector<float> h(kPadded);
    for (int e = 0; e < members && st == LSP_OK; ++e) {
        std::mt19937_64 g(seed * 1000003ull + (uint64_t)e);
        std::fill(h.begin(), h.end(), 0.f);
        for (int l = 0; l < kMlpLayers; ++l) {
            const float a = (l == kMlpLayers - 1 ? 0.1f : 1.0f) / std::sqrt((float)kL[l].in);
            std::uniform_real_distribution<float> U(-a, a);
            for (int o = 0; o < kL[l].out; ++o)
                for (int i = 0; i < kL[l].in; ++i) h[kL[l].w + (size_t)o * kL[l].in_p + i] = U(g);
        }
        hipError_t he = hipMemcpy(m->P[e], h.data(), sizeof(float) * kPadded, hipMemcpyHostToDevice);
        if (he == hipSuccess) he = hipMemset(m->M1[e], 0, sizeof(float) * kPadded);
        if (he == hipSuccess) he = hipMemset(m->M2[e], 0, sizeof(float) * kPadded);
        if (he == hipSuccess) he = hipMemset(m->G[e], 0, sizeof(float) * kPadded);
        if (he == hipSuccess) he = cast_all(m, e, nullptr);
        if (he == hipSuccess) he = hipDeviceSynchronize();
        if (he != hipSuccess) st = fail(he, "model init");
    }
    if (st != LSP_OK) {
        lsp_model_destroy(m);
        return st;
    }
    *out = m;
    return LSP_OK;
}

lsp_status lsp_model_destroy(lsp_model *m)
{
    if (!m) return LSP_OK;
    for (size_t e = 0; e < m->P.size(); ++e) {
        hipFree(m->P[e]);
        hipFree(m->G[e]);
        hipFree(m->M1[e]);
        hipFree(m->M2[e]);
        for (int l = 0; l < kMlpLayers; ++l) {
            hipFree(m->Wb[e][l]);
            hipFree(m->WbT[e][l]);
        }
    }
    for (void *p : m->ws) hipFree(p);
    hipFree(m->d_mean);
    hipFree(m->d_std);
    delete m;
    return LSP_OK;
}

lsp_status lsp_model_set_scalers(lsp_model *m, const float *feat_mean, const float *feat_std, float feat_zmax,
                                 float q_mu, float q_sigma)
{
    if (!good_model(m) || !feat_mean || !feat_std || !(q_sigma > 0.f) || !(feat_zmax > 0.f))
        return LSP_ERR_INVALID_ARG;
    for (int i = 0; i < kMlpIn; ++i)
        if (!(feat_std[i] > 0.f) || !std::isfinite(feat_mean[i])) return LSP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(m->mu);
    std::memcpy(m->feat_mean, feat_mean, sizeof(m->feat_mean));
    std::memcpy(m->feat_std, feat_std, sizeof(m->feat_std));
    m->feat_zmax = feat_zmax;
    m->q_mu = q_mu;
    m->q_sigma = q_sigma;
    return upload_scalers(m);
}

lsp_status lsp_model_get_params(const lsp_model *m, int32_t member, float *host, int64_t n)
{
    if (!good_model(m) || member < 0 || member >= m->members || !host || n != kParams) return LSP_ERR_INVALID_ARG;
    hipError_t e = copy_params(m->P[member], host, true, hipMemcpyDeviceToHost, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e == hipSuccess ? LSP_OK : fail(e, "get params");
}

lsp_status lsp_model_set_params(lsp_model *m, int32_t member, const float *host, int64_t n)
{
    if (!good_model(m) || member < 0 || member >= m->members || !host || n != kParams) return LSP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(m->mu);
    hipError_t e = copy_params(m->P[member], const_cast<float *>(host), false, hipMemcpyHostToDevice, nullptr);
    if (e == hipSuccess) e = cast_all(m, member, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e == hipSuccess ? LSP_OK : fail(e, "set params");
}

lsp_status lsp_mlp_forward(lsp_model *m, const float *feat, int32_t B, float *q, void *stream)
{
    if (!good_model(m) || !feat || !q || B < 1) return LSP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(m->mu);
    hipStream_t s = (hipStream_t)stream;
    const int Bp = (int)round32((size_t)B);
    hipError_t e = ensure_ws(m, Bp, s);
    if (e == hipSuccess) e = launch_features_in(feat, B, Bp, m->d_mean, m->d_std, m->X, m->XT, m->zmax, s);
    for (int i = 0; i < m->members && e == hipSuccess; ++i) {
        e = forward_member(m, i, Bp, s);
        if (e == hipSuccess)
            e = launch_head(m->raw, kMlpOutPad, feat, B, m->q_mu, m->q_sigma, nullptr, q + (size_t)i * B * kQuantiles,
                            s);
    }
    return e == hipSuccess ? LSP_OK : fail(e, "lsp_mlp_forward");
}

lsp_status lsp_mlp_grad(lsp_model *m, int32_t member, const float *feat, const float *samples, int32_t R, int32_t B,
                        float *grad, float *loss, void *stream)
{
    if (!good_model(m) || member < 0 || member >= m->members || !feat || !samples || R < 1 || B < 1)
        return LSP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(m->mu);
    hipStream_t s = (hipStream_t)stream;
    const int Bp = (int)round32((size_t)B);
    hipError_t e = ensure_ws(m, Bp, s);
    if (e == hipSuccess) e = launch_features_in(feat, B, Bp, m->d_mean, m->d_std, m->X, m->XT, nullptr, s);
    if (e == hipSuccess) e = forward_member(m, member, Bp, s);
    if (e == hipSuccess) e = backward_member(m, member, feat, B, Bp, samples, R, loss, s);
    if (e == hipSuccess && grad) e = copy_params(m->G[member], grad, true, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? LSP_OK : fail(e, "lsp_mlp_grad");
}

lsp_status lsp_mlp_adam_step(lsp_model *m, int32_t member, float lr, float beta1, float beta2, float eps,
                             void *stream)
{
    if (!good_model(m) || member < 0 || member >= m->members || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return LSP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(m->mu);
    hipStream_t s = (hipStream_t)stream;
    const int t = ++m->step[member];
    hipError_t e = launch_adam(m->P[member], m->G[member], m->M1[member], m->M2[member], (int64_t)kPadded, lr, beta1,
                               beta2, eps, t, s);
    if (e == hipSuccess) e = cast_all(m, member, s);
    return e == hipSuccess ? LSP_OK : fail(e, "lsp_mlp_adam_step");
}

lsp_status lsp_model_set_law_error(lsp_model *m, float err_m, float err_beta)
{
    if (!good_model(m) || !(err_m >= 0.f && err_m <= 10.f) || !(err_beta >= 0.f && err_beta <= 10.f))
        return LSP_ERR_INVALID_ARG;
    m->law_err[0] = err_m;
    m->law_err[1] = err_beta;
    return LSP_OK;
}

lsp_status lsp_model_save(const lsp_model *m, const char *path, int32_t with_optimizer)
{
    if (!good_model(m) || !path) return LSP_ERR_INVALID_ARG;
    std::ofstream f(path, std::ios::binary);
    if (!f) return LSP_ERR_INVALID_ARG;
    const int32_t hdr[8] = {3, m->members, kMlpIn, kMlpInPad, kMlpHidden, kMlpOut, kMlpOutPad, with_optimizer ? 1 : 0};
    f.write(kMagic, 16);
    f.write((const char *)hdr, sizeof(hdr));
    f.write((const char *)&m->seed, 8);
    f.write((const char *)m->feat_mean, sizeof(m->feat_mean));
    f.write((const char *)m->feat_std, sizeof(m->feat_std));
    const float sc[3] = {m->feat_zmax, m->q_mu, m->q_sigma};
    f.write((const char *)sc, sizeof(sc));
    f.write((const char *)m->law_err, sizeof(m->law_err));  // version 3
    std::vector<float> h(kPadded);
    for (int e = 0; e < m->members; ++e) {
        const int32_t st = m->step[e];
        f.write((const char *)&st, 4);
        const int nbuf = with_optimizer ? 3 : 1;
        float *bufs[3] = {m->P[e], m->M1[e], m->M2[e]};
        for (int b = 0; b < nbuf; ++b) {
            if (hipMemcpy(h.data(), bufs[b], sizeof(float) * kPadded, hipMemcpyDeviceToHost) != hipSuccess)
                return fail(hipGetLastError(), "model save");
            f.write((const char *)h.data(), sizeof(float) * kPadded);
        }
    }
    return f.good() ? LSP_OK : LSP_ERR_INVALID_ARG;
}

lsp_status lsp_model_load(const char *path, lsp_model **out)
{
    if (!path || !out) return LSP_ERR_INVALID_ARG;
    *out = nullptr;
    std::ifstream f(path, std::ios::binary);
    if (!f) {
        set_last_error(std::string("cannot open model file ") + path);
        return LSP_ERR_MODEL;
    }
    char magic[16];
    int32_t hdr[8];
    f.read(magic, 16);
    f.read((char *)hdr, sizeof(hdr));
    if (!f || std::memcmp(magic, kMagic, 16) != 0 || (hdr[0] < 1 || hdr[0] > 3) || hdr[2] != kMlpIn ||
        hdr[3] != kMlpInPad ||
        hdr[4] != kMlpHidden || hdr[5] != kMlpOut || hdr[6] != kMlpOutPad || hdr[1] < 1 || hdr[1] > 16) {
        set_last_error("model file header mismatch");
        return LSP_ERR_MODEL;
    }
    lsp_model *m = nullptr;
    lsp_status st = lsp_model_create(hdr[1], 0, &m);
    if (st != LSP_OK) return st;
    f.read((char *)&m->seed, 8);
    f.read((char *)m->feat_mean, sizeof(m->feat_mean));
    f.read((char *)m->feat_std, sizeof(m->feat_std));
    float sc[3];
    f.read((char *)sc, sizeof(sc));
    m->feat_zmax = sc[0];
    m->q_mu = sc[1];
    m->q_sigma = sc[2];
    if (hdr[0] == 2) {  // a per-FAP-bin error table (7 floats), no longer used: skipped
        float table[7];
        f.read((char *)table, sizeof(table));
    } else if (hdr[0] >= 3) {  // calibrated errors of the law's location and scale
        f.read((char *)m->law_err, sizeof(m->law_err));
        for (float v : m->law_err)
            if (!(v >= 0.f && v <= 10.f)) {
                lsp_model_destroy(m);
                set_last_error("model file: bad law errors");
                return LSP_ERR_MODEL;
            }
    }
    std::vector<float> h(kPadded);
    for (int e = 0; e < m->members && f; ++e) {
        int32_t stp = 0;
        f.read((char *)&stp, 4);
        m->step[e] = stp;
        float *bufs[3] = {m->P[e], m->M1[e], m->M2[e]};
        const int nbuf = hdr[7] ? 3 : 1;
        for (int b = 0; b < nbuf && f; ++b) {
            f.read((char *)h.data(), sizeof(float) * kPadded);
            if (f && hipMemcpy(bufs[b], h.data(), sizeof(float) * kPadded, hipMemcpyHostToDevice) != hipSuccess) {
                lsp_model_destroy(m);
                return fail(hipGetLastError(), "model load");
            }
        }
        if (cast_all(m, e, nullptr) != hipSuccess) {
            lsp_model_destroy(m);
            return fail(hipGetLastError(), "model load");
        }
    }
    if (!f) {
        lsp_model_destroy(m);
        set_last_error("model file truncated");
        return LSP_ERR_MODEL;
    }
    st = upload_scalers(m);
    if (st == LSP_OK && hipDeviceSynchronize() != hipSuccess) st = fail(hipGetLastError(), "model load");
    if (st != LSP_OK) {
        lsp_model_destroy(m);
        return st;
    }
    *out = m;
    return LSP_OK;
}

lsp_status lsp_mlp_gemm_nt(const void *A, const void *B, float *C, int32_t M, int32_t N, int32_t K, void *stream)
{
    if (!A || !B || !C || M < 32 || N < 32 || K < 32 || M % 32 || N % 32 || K % 32) return LSP_ERR_INVALID_ARG;
    if (lsp_device_count() < 1) return LSP_ERR_NO_DEVICE;
    GemmArgs g = gemm((const __bf16 *)A, K, (const __bf16 *)B, K, M, N, K, GEMM_STORE);
    g.C = C;
    g.ldc = N;
    hipError_t e = launch_gemm_nt(g, (hipStream_t)stream);
    return e == hipSuccess ? LSP_OK : fail(e, "lsp_mlp_gemm_nt");
}

lsp_status lsp_fap_surrogate(lsp_model *m, const double *t, const int64_t *off, int32_t n_pat, const double *f_min,
                             const double *df, const int64_t *Nf, const float *p_obs, float *fap, float *fap_err,
                             int32_t *used_mc, float max_err, int32_t mc_realizations, uint64_t seed, void *stream)
{
    if (!good_model(m) || !t || !off || !f_min || !df || !Nf || !p_obs || !fap || !fap_err || n_pat < 1 ||
        !(max_err >= 0.f) || mc_realizations < 0)
        return LSP_ERR_INVALID_ARG;
    for (int32_t p = 0; p < n_pat; ++p)
        if (off[p + 1] - off[p] < 4) return LSP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    // 1. features of every pattern
    float *feat = nullptr;
    hipError_t he = hipMalloc(&feat, sizeof(float) * kFeatures * (size_t)n_pat);
    if (he != hipSuccess) return fail(he, "feature buffer");
    lsp_status st = lsp_window_features(t, off, n_pat, f_min, df, Nf, feat, stream);
    // 2. the law from every member, 3. FAP and its error bound
    std::vector<float> hz((size_t)n_pat), hs((size_t)n_pat);
    if (st == LSP_OK) {
        std::lock_guard<std::mutex> lock(m->mu);
        const int Bp = (int)round32((size_t)n_pat);
        he = ensure_ws(m, Bp, s);
        if (he == hipSuccess) he = launch_features_in(feat, n_pat, Bp, m->d_mean, m->d_std, m->X, m->XT, m->zmax, s);
        for (int i = 0; i < m->members && he == hipSuccess; ++i) {
            he = forward_member(m, i, Bp, s);
            if (he == hipSuccess)
                he = launch_head(m->raw, kMlpOutPad, feat, n_pat, m->q_mu, m->q_sigma,
                                 m->law + (size_t)i * n_pat * 2, nullptr, s);
        }
        if (he == hipSuccess)
            he = launch_fap(m->law, m->members, n_pat, feat, p_obs, m->law_err[0], m->law_err[1], kBoundZ, fap,
                            fap_err, s);
        if (he == hipSuccess) he = hipMemcpyAsync(hz.data(), m->zmax, sizeof(float) * n_pat, hipMemcpyDeviceToHost, s);
        if (he == hipSuccess)
            he = hipMemcpyAsync(hs.data(), fap_err, sizeof(float) * n_pat, hipMemcpyDeviceToHost, s);
        if (he == hipSuccess) he = hipStreamSynchronize(s);
    }
    hipFree(feat);
    if (st != LSP_OK) return st;
    if (he != hipSuccess) return fail(he, "lsp_fap_surrogate");
    // 4. Monte-Carlo fallback where the bound exceeds max_err or the pattern is out of range
    std::vector<int32_t> fb, flags((size_t)n_pat, 0);
    for (int32_t p = 0; p < n_pat; ++p)
        if (!(hs[p] <= max_err) || !(hz[p] <= m->feat_zmax)) fb.push_back(p);
    if (!fb.empty() && mc_realizations > 0) {
        std::vector<int64_t> o2(1, 0), n2;
        std::vector<double> fm2, df2;
        for (int32_t p : fb) {
            o2.push_back(o2.back() + (off[p + 1] - off[p]));
            fm2.push_back(f_min[p]);
            df2.push_back(df[p]);
            n2.push_back(Nf[p]);
            flags[p] = 1;
        }
        double *t2 = nullptr;
        float *pm = nullptr;
        int32_t *idx = nullptr;
        he = hipMalloc(&t2, sizeof(double) * (size_t)o2.back());
        if (he == hipSuccess) he = hipMalloc(&pm, sizeof(float) * fb.size() * (size_t)mc_realizations);
        if (he == hipSuccess) he = hipMalloc(&idx, sizeof(int32_t) * fb.size());
        for (size_t i = 0; i < fb.size() && he == hipSuccess; ++i)
            he = hipMemcpyAsync(t2 + o2[i], t + off[fb[i]], sizeof(double) * (size_t)(o2[i + 1] - o2[i]),
                                hipMemcpyDeviceToDevice, s);
        if (he == hipSuccess)
            he = hipMemcpyAsync(idx, fb.data(), sizeof(int32_t) * fb.size(), hipMemcpyHostToDevice, s);
        if (he == hipSuccess) {
            st = lsp_mc_maxpower(t2, o2.data(), (int32_t)fb.size(), fm2.data(), df2.data(), n2.data(),
                                 mc_realizations, seed, 0, pm, stream);
            if (st == LSP_OK)
                he = launch_mc_fap(pm, mc_realizations, (int)fb.size(), p_obs, idx, kBoundZ, fap, fap_err, s);
            if (he == hipSuccess) he = hipStreamSynchronize(s);
        }
        hipFree(t2);
        hipFree(pm);
        hipFree(idx);
        if (st != LSP_OK) return st;
        if (he != hipSuccess) return fail(he, "Monte-Carlo fallback");
    }
    if (used_mc) {
        he = hipMemcpyAsync(used_mc, flags.data(), sizeof(int32_t) * n_pat, hipMemcpyHostToDevice, s);
        if (he == hipSuccess) he = hipStreamSynchronize(s);
        if (he != hipSuccess) return fail(he, "used_mc");
    }
    return LSP_OK;
}

}  // extern "C"
