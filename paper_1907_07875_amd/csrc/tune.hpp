// Plan-time launch tuning: candidate timing on the device and the tuning cache.
//
// A plan's launch choices (tile heights, grid sizes, batch partition, large-engine pass
// shapes) change how work is spread over the GPU, never the arithmetic of a signal, so every
// choice gives the same results bit for bit; preparation times the candidates on a
// synthetic batch and keeps the fastest.  Results are cached by a key naming the device
// (architecture, compute units), the engine and a hash of the plan's device image, in
// memory and in a text file (GFT_TUNE_CACHE; default $HOME/.cache/libgft/tuning-v1.txt;
// empty or "off": memory only), so a plan whose image was tuned before skips the timing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace gft {

// FNV-1a over bytes, chained through h.
uint64_t fnv1a(const void *data, size_t n, uint64_t h = 1469598103934665603ull);

// "<arch>:<compute units>" of device dev (e.g. "gfx950:256").
std::string device_tag(int dev);

// Cached choice for key, if any.
bool tune_cache_get(const std::string &key, std::vector<int32_t> &values);
// Record a choice (memory, and the cache file when one is configured).
void tune_cache_put(const std::string &key, const std::vector<int32_t> &values);

// Times `ncand` launch candidates on stream st: a warm-up of six launches of the built-in
// candidate `base`, then four rounds taking the candidates in turn, two launches each, each
// candidate keeping its best time.  Returns the fastest candidate when it is at least 3%
// faster than `base`, else `base`; -1 when a launch or event call failed.
int time_candidates(int ncand, int base, const std::function<hipError_t(int, hipStream_t)> &launch,
                    hipStream_t st);

}  // namespace gft
