// Blocks-per-launch autotuner: times candidate launch sizes of a path on
// the device it will run on and keeps the fastest per block, with a
// persistent cache (POND_AUTOTUNE_CACHE: a text file, one result per line)
// so that a configuration is measured once per device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pond_tune.hpp"

namespace pond {

namespace {

std::mutex g_cache_mu;

// Device identity for the cache key: architecture name and compute units.
std::string device_tag(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);  // drop feature flags
    return arch + "-" + std::to_string(prop.multiProcessorCount) + "cu";
}

std::string key_line(const TuneKey& k, const std::string& dev) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "pond-tune-4 %s %s nfft=%lld form=%d kind=%d hist=%s", dev.c_str(), k.path,
                  (long long)k.nfft, k.precision, k.kind, k.global_hist ? "global" : "lds");
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, TuneResult* r) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, key.c_str(), key.size()) != 0 || line[key.size()] != ' ') continue;
        int b = 0, d = 0;
        double t = 0, td = 0;
        if (std::sscanf(line + key.size(), " batch=%d ms_per_block=%lf default_batch=%d default_ms_per_block=%lf", &b,
                        &t, &d, &td) == 4 &&
            b > 0 && d > 0) {
            r->batch = b;
            r->ms_per_block = t;
            r->default_batch = d;
            r->default_ms_per_block = td;
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const TuneResult& r) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    FILE* f = std::fopen(path, "a");
    if (!f) return;  // an unwritable cache only costs a new measurement next time
    std::fprintf(f, "%s batch=%d ms_per_block=%.6f default_batch=%d default_ms_per_block=%.6f\n", key.c_str(),
                 r.batch, r.ms_per_block, r.default_batch, r.default_ms_per_block);
    std::fclose(f);
}

}  // namespace

hipError_t autotune_batch(const TuneKey& key, const std::vector<int>& candidates, int default_batch,
                          const std::function<hipError_t(int)>& run, TuneResult* out) {
    *out = TuneResult{};
    if (candidates.empty()) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const char* path = std::getenv("POND_AUTOTUNE_CACHE");
    const std::string k = key_line(key, device_tag(dev));
    if (path && *path && cache_lookup(path, k, out)) {
        if (std::find(candidates.begin(), candidates.end(), out->batch) != candidates.end()) {
            out->from_cache = true;
            return hipSuccess;
        }
        *out = TuneResult{};  // cached choice no longer allowed here (memory cap): measure
    }
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    double best = 0, dflt = 0;
    int best_b = 0;
    for (int nb : candidates) {
        if (e != hipSuccess) break;
        // one untimed launch (first-use costs), one to size the samples,
        // then the median of three samples of at least ~10 ms each
        auto sample = [&](int reps, float* ms) {
            hipError_t r = hipEventRecord(a, nullptr);
            for (int i = 0; i < reps && r == hipSuccess; ++i) r = run(nb);
            if (r == hipSuccess) r = hipEventRecord(b, nullptr);
            if (r == hipSuccess) r = hipEventSynchronize(b);
            if (r == hipSuccess) r = hipEventElapsedTime(ms, a, b);
            return r;
        };
        e = run(nb);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        float t1 = 0;
        if (e == hipSuccess) e = sample(1, &t1);
        const int reps = t1 > 0 ? std::max(1, std::min(64, (int)(10.0f / t1) + 1)) : 1;
        float t[3] = {0, 0, 0};
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = sample(reps, &t[r]);
        if (e != hipSuccess) break;
        std::sort(t, t + 3);
        const double per = (double)t[1] / ((double)reps * nb);
        // a larger launch must win by more than 0.5% (it costs memory; the
        // samples' spread is below that)
        if (best_b == 0 || per < best * 0.995) {
            best = per;
            best_b = nb;
        }
        if (nb == default_batch) dflt = per;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return e;
    out->batch = best_b;
    out->ms_per_block = best;
    out->default_batch = default_batch;
    out->default_ms_per_block = dflt;
    out->from_cache = false;
    if (path && *path) cache_store(path, k, *out);
    return hipSuccess;
}

TuneRing tune_ring(int64_t nfft, int64_t hop, int64_t bytes_per_sample, int nb_max, int64_t spare_bytes) {
    const int64_t span = ((int64_t)(nb_max - 1) * hop + nfft) * bytes_per_sample;  // one run of nb_max
    int64_t want = (int64_t)1 << 30;
    if (want > spare_bytes) want = spare_bytes;
    if (want < span) want = span;
    TuneRing r;
    r.blocks = (want / bytes_per_sample - nfft) / hop + 1;
    if (r.blocks < nb_max) r.blocks = nb_max;
    r.bytes = (((r.blocks - 1) * hop + nfft) * bytes_per_sample + 7) & ~(int64_t)7;
    return r;
}

std::vector<int> batch_candidates(int64_t block_bytes, int64_t cap_bytes, int default_batch) {
    std::vector<int> c;
    for (int nb : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32})
        if ((int64_t)nb * block_bytes <= cap_bytes || nb == 1) c.push_back(nb);
    if (std::find(c.begin(), c.end(), default_batch) == c.end()) c.push_back(default_batch);
    std::sort(c.begin(), c.end());
    return c;
}

}  // namespace pond
