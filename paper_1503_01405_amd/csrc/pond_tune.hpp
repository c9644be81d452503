// Blocks-per-launch autotuner (pond_tune.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <vector>

namespace pond {

// What a tuned choice depends on (with the device, which the tuner adds).
struct TuneKey {
    const char* path = "dedisperse";  // which launch sequence is timed
    int64_t nfft = 0;
    int precision = 0;
    int kind = 0;              // input kind (complex, real LSB/USB)
    bool global_hist = false;  // fold histogram in global memory (else LDS)
};

struct TuneResult {
    int batch = 0;                      // chosen blocks per launch
    double ms_per_block = 0;            // its time per block
    int default_batch = 0;              // the fixed rule's choice
    double default_ms_per_block = 0;    // its time per block
    bool from_cache = false;            // read from POND_AUTOTUNE_CACHE, not measured
};

// Times run(nb) (one launch sequence over nb blocks, on the null stream)
// for every candidate, after one untimed run each, as the median of three
// samples of back-to-back runs (about 10 ms or more each), and picks the
// least time per block (a larger batch must win by more than 0.5%).  With POND_AUTOTUNE_CACHE set, a stored result for the same key
// and device is used instead (if its batch is still a candidate), and a new
// result is appended.  Synchronous.
hipError_t autotune_batch(const TuneKey& key, const std::vector<int>& candidates, int default_batch,
                          const std::function<hipError_t(int)>& run, TuneResult* out);

// The tuner's input: a ring of pseudo-random int8 samples of at least 1 GiB
// (four times the 256 MB Infinity Cache; less only where the device has
// not that much to spare), through which successive runs advance, so that
// every run reads input that the caches do not hold.
struct TuneRing {
    int64_t bytes = 0;   // allocation, a multiple of 8
    int64_t blocks = 0;  // overlap-save blocks the ring holds
    // first block of run `run` of nb blocks
    int64_t start(int64_t run, int nb) const { return (run * nb) % (blocks - nb + 1); }
};
TuneRing tune_ring(int64_t nfft, int64_t hop, int64_t bytes_per_sample, int nb_max, int64_t spare_bytes);

// 1, 2, 3, 4, 6, 8, 12, 16, 24, 32 blocks where they fit in cap_bytes (1
// always), plus the default.
std::vector<int> batch_candidates(int64_t block_bytes, int64_t cap_bytes, int default_batch);

}  // namespace pond
