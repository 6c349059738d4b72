// tuner.h -- launch-shape autotuner cache (host only).
#pragma once

#include <string>

#include "internal.h"

namespace lsp {

// Tuned shape for the power-of-two buckets of (Nt, Nf) on this device, if any.
bool tuner_lookup(const std::string &arch, int cus, int phase, int64_t Nt, int64_t Nf, lsp_tile *out);

// Host-side pieces of lsp_host.cpp used by the tuner.
lsp_status run_single_timed(const double *t, const float *x, int64_t Nt, double f_min, double df,
                            int64_t Nf, float *Pn, hipStream_t s, int phase, const lsp_tile &tile);
// splits of the sample axis for a launch shape; sums_per_freq FP32 chunk sums
// per frequency and split (4 for the plain periodogram) bound the workspace
int heuristic_splits(int64_t Nt, int64_t Nf, int m, int cus, int waves, int blocks_per_cu, int sums_per_freq = 4);
int device_cus();
std::string device_arch();
hipError_t batched_occupancy(int waves, int *blocks_per_cu);

}  // namespace lsp
