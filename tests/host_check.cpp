// Host-side checks of libmi355lsp under AddressSanitizer / UndefinedBehavior-
// Sanitizer (built without a GPU in mind): every entry point's argument
// validation, the host helpers over wide input ranges, and the two file
// parsers (tuner cache JSON, surrogate model header) on malformed inputs.
// Prints one line per group; exit status 0 when every expectation holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lsp.h"

static int g_fail = 0;
#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++g_fail;                                                       \
        }                                                                   \
    } while (0)

static std::string write_file(const std::string &name, const std::string &body)
{
    const std::string path = std::string(std::getenv("HOST_CHECK_DIR") ? std::getenv("HOST_CHECK_DIR") : "/tmp") +
                             "/" + name;
    FILE *f = std::fopen(path.c_str(), "wb");
    if (f) {
        std::fwrite(body.data(), 1, body.size(), f);
        std::fclose(f);
    }
    return path;
}

int main()
{
    double *fake_d = reinterpret_cast<double *>(16);
    float *fake_f = reinterpret_cast<float *>(16);

    // argument validation: rejected on the host before any HIP call
    EXPECT(lsp_periodogram(nullptr, fake_f, 10, 0.1, 0.1, 10, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_periodogram(fake_d, fake_f, 1, 0.1, 0.1, 10, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_periodogram(fake_d, fake_f, 10, -1.0, 0.1, 10, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_periodogram(fake_d, fake_f, 10, 0.1, 0.0, 10, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_periodogram(fake_d, fake_f, 10, 0.1, NAN, 10, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_periodogram(fake_d, fake_f, 10, 0.1, 0.1, 0, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_periodogram(fake_d, fake_f, 10, 0.1, 1e308, 10, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    lsp_options opt;
    std::memset(&opt, 0, sizeof(opt));
    opt.tile.waves = -3;
    EXPECT(lsp_periodogram_ex(fake_d, fake_f, 10, 0.1, 0.1, 10, fake_f, nullptr, &opt) == LSP_ERR_INVALID_ARG);
    opt.tile.waves = 0;
    opt.phase = 7;
    EXPECT(lsp_periodogram_ex(fake_d, fake_f, 10, 0.1, 0.1, 10, fake_f, nullptr, &opt) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_periodogram_fast(fake_d, fake_f, 10, 0.1, 0.1, 10, 5, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_gls(fake_d, fake_f, nullptr, 2, 0.1, 0.1, 10, fake_f, 0, 0, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_gls(fake_d, fake_f, nullptr, 10, 0.1, 0.1, 10, fake_f, 3, 0, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_multiharmonic(fake_d, fake_f, nullptr, 10, 9, 0.1, 0.1, 10, fake_f, 0, 0, nullptr) ==
           LSP_ERR_UNSUPPORTED);
    EXPECT(lsp_multiharmonic(fake_d, fake_f, nullptr, 10, 0, 0.1, 0.1, 10, fake_f, 0, 0, nullptr) ==
           LSP_ERR_INVALID_ARG);
    const int64_t off_bad[3] = {0, 5, 3};  // decreasing offsets
    const double fm[2] = {0.1, 0.1}, dfs[2] = {0.1, 0.1};
    const int64_t nfs[2] = {10, 10};
    float pmax[2];
    EXPECT(lsp_periodogram_batched(fake_d, fake_f, off_bad, 2, fm, dfs, nfs, nullptr, pmax, nullptr, nullptr,
                                   nullptr, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_mc_maxpower(fake_d, off_bad, 2, fm, dfs, nfs, 10, 1, 0, pmax, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_normals(1, 0, -1, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    double ops = 0;
    EXPECT(lsp_microbench(42, 2, 10, nullptr, &ops, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_probe_sincos(nullptr, 4, fake_f, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_probe_phase(fake_d, fake_d, 4, NAN, 0, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_probe_recurrence(fake_d, 4, 0.0, 1.0, 0.1, 33, fake_f, fake_f, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_probe_recurrence(fake_d, (int64_t)1 << 40, 0.0, 1.0, 0.1, 32, fake_f, fake_f, nullptr) ==
           LSP_ERR_INVALID_ARG);
    std::printf("validation: ok\n");

    // host helpers over wide ranges (no crash, finite or NaN as documented)
    const double vals[] = {-1e300, -1.0, 0.0, 1e-300, 0.5, 1.0, 7.0, 1e6, 1e300, NAN, INFINITY};
    for (double a : vals)
        for (double b : vals) {
            double f_min = 0, df = 0;
            int64_t Nf = 0;
            (void)lsp_grid_paper(a, b, 1000, 4.0, 1.0, 256, &f_min, &df, &Nf);
            (void)lsp_grid_paper(0.0, 10.0, 100, a, b, 1, &f_min, &df, &Nf);
            for (int64_t nt : {(int64_t)-5, (int64_t)3, (int64_t)4, (int64_t)1000, (int64_t)1 << 40}) {
                const double q = lsp_fap_analytic(a, nt, (b > 0 && b < 1e18) ? (int64_t)b : 1000);
                EXPECT(std::isnan(q) || (q >= 0.0 && q <= 1.0));
            }
        }
    {
        double f_min = 0, df = 0;
        int64_t Nf = 0;
        EXPECT(lsp_grid_paper(0.0, 150.0, 382003, 4.0, 2.0, 256, &f_min, &df, &Nf) == LSP_OK);
        EXPECT(Nf == 1528064);
    }
    for (int s = -20; s <= 20; ++s) EXPECT(lsp_status_string((lsp_status)s) != nullptr);
    EXPECT(lsp_last_error() != nullptr && lsp_version() != nullptr);
    for (int ph = -2; ph <= 4; ++ph) {
        const int n = lsp_list_tiles(ph, nullptr, 0);
        std::vector<lsp_tile> v(n > 0 ? n : 1);
        EXPECT(lsp_list_tiles(ph, v.data(), n > 0 ? n : 0) == n);
    }
    std::printf("helpers: ok\n");

    // tuner cache parser on malformed input: an error or a clean load, never a crash
    const std::string hdr = "{\"format\": \"mi355lsp-tune-2\", \"entries\": [";
    const std::vector<std::string> bodies = {
        "",
        "mi355lsp-tune-2",
        hdr,
        hdr + "{\"key\": \"",
        hdr + "{\"key\": \"abc",
        hdr + "{\"key\": \"abc\", \"trig\": 3}",
        hdr + "{\"key\": \"abc\", \"trig\": 1e300, \"m\": -1e300, \"waves\": 1e20, \"splits\": nan, \"unroll\": inf, "
              "\"sum\": 2, \"ms\": 1}]}",
        hdr + "{\"key\": \"x|256|0|10|11\", \"trig\": 3, \"m\": 32, \"waves\": 8, \"splits\": 99999999999, "
              "\"unroll\": 1, \"sum\": 2, \"ms\": 0.1}]}",
        hdr + std::string(100000, '{') + "]}",
        hdr + "{\"key\": \"" + std::string(5000, 'k') + "\", \"trig\": 1, \"m\": 1, \"waves\": 4, \"splits\": 1, "
              "\"unroll\": 4, \"sum\": 1, \"ms\": 1}]}",
    };
    for (size_t i = 0; i < bodies.size(); ++i) {
        const lsp_status st = lsp_tune_cache_load(write_file("host_check_tune_" + std::to_string(i) + ".json",
                                                             bodies[i]).c_str());
        EXPECT(st == LSP_OK || st == LSP_ERR_INVALID_ARG);
    }
    EXPECT(lsp_tune_cache_load("/nonexistent/dir/tune.json") == LSP_ERR_INVALID_ARG);
    std::printf("tuner cache parser: ok\n");

    // surrogate model header on malformed files: LSP_ERR_MODEL before any device work
    const std::vector<std::string> models = {"", "short", std::string(16, 'M'), std::string(200, '\xff'),
                                             std::string("MI355LSP-MODEL") + std::string(40, '\0')};
    for (size_t i = 0; i < models.size(); ++i) {
        lsp_model *m = nullptr;
        const lsp_status st = lsp_model_load(write_file("host_check_model_" + std::to_string(i) + ".bin",
                                                        models[i]).c_str(), &m);
        EXPECT(st == LSP_ERR_MODEL && m == nullptr);
    }
    EXPECT(lsp_model_load(nullptr, nullptr) == LSP_ERR_INVALID_ARG);
    EXPECT(lsp_model_set_law_error(nullptr, 0.05f, 0.01f) == LSP_ERR_INVALID_ARG);
    std::printf("model header parser: ok\n");

    std::printf("%s (%d failed expectations)\n", g_fail ? "FAILED" : "PASSED", g_fail);
    return g_fail ? 1 : 0;
}
