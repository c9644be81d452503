// Host-runtime driver for the sanitizer build: the library's host sources
// compiled with AddressSanitizer and UndefinedBehaviorSanitizer (host code
// only; the kernels come from libpond.so), exercised through the C ABI.
//   host_driver cpu   argument checking, geometry, error text, host-only
//                     queries: no device needed
//   host_driver gpu   plans (streaming calls, taper, timing, autotune and
//                     its cache file), search, server with deferred
//                     admission, real input, AID, the no-allocation entry
// Exits 0 when every check holds; a sanitizer report aborts the process.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <unistd.h>

#include "../../include/pond.h"

namespace {

int g_fail = 0;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
            ++g_fail;                                                            \
        }                                                                        \
    } while (0)

const double F0 = 326.5, BW = 16.0, P0 = 0.0891;

void run_cpu() {
    int64_t nf = 0, disc = 0, hop = 0;
    CHECK(pond_geometry(F0, BW, 50.0, (int64_t)1 << 23, &nf, &disc, &hop) == POND_OK);
    CHECK(nf > 0 && disc == ((int64_t)1 << 22) && hop == ((int64_t)1 << 22));
    CHECK(pond_geometry(F0, BW, 50.0, 1000, &nf, &disc, &hop) == POND_EINVAL);
    CHECK(pond_geometry(F0, -1.0, 1.0, 1 << 18, nullptr, nullptr, nullptr) == POND_EINVAL);
    CHECK(pond_geometry(F0, BW, NAN, 1 << 18, nullptr, nullptr, nullptr) == POND_EINVAL);
    for (int64_t c : {0, -1, -2, -3, -4, -5, -99, 7}) CHECK(std::strlen(pond_strerror(c)) > 0);
    // invalid plans are rejected before any device call
    CHECK(pond_plan_create(F0, BW, 1.0, (1 << 18) + 1, 256, P0) == nullptr);
    CHECK(pond_plan_create(F0, BW, 1.0, (int64_t)1 << 28, 256, P0) == nullptr);
    CHECK(pond_plan_create_ex(F0, BW, 1.0, 1 << 18, 256, P0, 9, 0) == nullptr);
    CHECK(pond_create_status() == POND_EINVAL);
    CHECK(pond_real_plan_create(F0, BW, 1.0, (int64_t)1 << 26, 256, P0, POND_FP32, 0, POND_LSB) == nullptr);
    // null handles
    CHECK(pond_dedisperse_fold(nullptr, nullptr, 0, 0, nullptr, 0, nullptr) == POND_EINVAL);
    CHECK(pond_plan_expect(nullptr, 10, 0, nullptr, nullptr) == POND_EINVAL);
    CHECK(pond_plan_autotune(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == POND_EINVAL);
    pond_plan_destroy(nullptr);
    const double dms[2] = {1.0, 2.0};
    CHECK(pond_search_create(F0, BW, dms, 0, 64, P0, 1 << 16, 1 << 18, POND_FP32) == nullptr);
    CHECK(pond_search_create_ex(F0, BW, dms, 2, 64, P0, 1 << 16, 1 << 30, POND_FP32, 0) == nullptr);
    CHECK(pond_search_autotune(nullptr, 1 << 16, nullptr, nullptr, nullptr, nullptr, nullptr) == POND_EINVAL);
    pond_search_destroy(nullptr);
    CHECK(pond_server_create(0, 4) == nullptr);
    CHECK(pond_server_create(1 << 30, 0) == nullptr);
    pond_stream_desc d{};
    d.f0_mhz = F0;
    d.bw_mhz = BW;
    d.dm = 1.0;
    d.period_s = P0;
    d.nfft = 1 << 18;
    d.subint_nsamp = 1 << 20;
    d.max_block_nsamp = 1 << 20;
    d.nbins = 256;
    d.precision = POND_HALF;
    CHECK(pond_server_stream_bytes(&d) > 0);
    d.nfft = 12345;
    CHECK(pond_server_stream_bytes(&d) == POND_EINVAL);
    CHECK(pond_server_poll(nullptr, nullptr, 0, 0) == POND_EINVAL);
    pond_server_destroy(nullptr);
    CHECK(pond_aid_create(F0, BW, 1.0, 100, 4, 64, P0) == nullptr);
    pond_aid_destroy(nullptr);
    CHECK(pond_copy_device(nullptr, nullptr, 15, nullptr) == POND_EINVAL);
}

// Device buffer of pseudo-random int8 samples (xorshift64 on the host).
int8_t* device_noise(int64_t bytes, uint64_t seed) {
    std::vector<int8_t> h((size_t)bytes);
    uint64_t x = seed | 1;
    for (auto& v : h) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        v = (int8_t)((int)(x >> 56) % 41 - 20);
    }
    int8_t* d = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&d), (size_t)bytes) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), (size_t)bytes, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return d;
}

void run_plans(int8_t* iq, int64_t nsamp) {
    const int64_t nfft = 1 << 18, S = 1 << 20;
    float *prof = nullptr, *ser = nullptr;
    CHECK(hipMalloc(reinterpret_cast<void**>(&prof), 64 * 256 * sizeof(float)) == hipSuccess);
    CHECK(hipMalloc(reinterpret_cast<void**>(&ser), (size_t)(nsamp / 16 + 16) * sizeof(float)) == hipSuccess);
    for (int prec : {POND_FP32, POND_MIXED, POND_MIXED_VALU, POND_HALF}) {
        pond_plan* p = pond_plan_create_ex(F0, BW, 1.0, nfft, 256, P0, prec, 0);
        CHECK(p != nullptr);
        if (!p) continue;
        CHECK(pond_plan_set_taper(p, 0.1) == POND_OK);
        CHECK(pond_plan_set_timing(p, 1) == POND_OK);
        int64_t pos = 0, nprof = 0;
        const int64_t cuts[] = {nfft / 3, nfft, 5 * nfft / 2, nsamp};
        for (int64_t c : cuts) {
            const int64_t n = std::min(c, nsamp) - pos;
            if (n <= 0) continue;
            int64_t np = 0, no = 0;
            CHECK(pond_plan_expect(p, n, S, &np, &no) == POND_OK);
            int64_t ns = 0;
            const int64_t r = pond_dedisperse_series(p, iq + 2 * pos, n, S, prof, 64, 16, ser, nsamp / 16 + 16, &ns,
                                                     nullptr);
            CHECK(r == np && ns == no / 16);
            nprof += r > 0 ? r : 0;
            pos += n;
        }
        CHECK(pond_plan_set_taper(p, 0.2) == POND_EINVAL);  // mid-stream
        const int64_t last = pond_dedisperse_fold(p, nullptr, 0, S, prof, 64, nullptr);
        CHECK(last == 1);
        pond_info info{};
        CHECK(pond_plan_query(p, &info) == POND_OK);
        pond_kernel_times kt{};
        CHECK(pond_plan_kernel_times(p, &kt) == POND_OK);
        CHECK(kt.launches[0] > 0);
        pond_plan_destroy(p);
    }
    (void)hipFree(prof);
    (void)hipFree(ser);
}

void run_autotune() {
    const char* tmp = std::getenv("TMPDIR");
    const std::string spath = std::string(tmp && *tmp ? tmp : "/tmp") + "/pond_tune_asan_" + std::to_string(getpid()) + ".txt";
    const char* path = spath.c_str();
    std::remove(path);
    setenv("POND_AUTOTUNE_CACHE", path, 1);
    int32_t b = 0, db = 0, fc = -1;
    double t = 0, td = 0;
    pond_plan* p = pond_plan_create_ex(F0, BW, 1.0, 1 << 18, 256, P0, POND_HALF, POND_BATCH_AUTOTUNE);
    CHECK(p != nullptr);
    CHECK(pond_plan_autotune(p, &b, &t, &db, &td, &fc) == POND_OK && b >= 1 && fc == 0 && t > 0);
    pond_plan_destroy(p);
    p = pond_plan_create_ex(F0, BW, 1.0, 1 << 18, 256, P0, POND_HALF, POND_BATCH_AUTOTUNE);
    int32_t b2 = 0;
    CHECK(p != nullptr);
    CHECK(pond_plan_autotune(p, &b2, nullptr, nullptr, nullptr, &fc) == POND_OK && b2 == b && fc == 1);
    pond_plan_destroy(p);
    // a damaged cache file is ignored line by line
    FILE* f = std::fopen(path, "a");
    if (f) {
        std::fputs("pond-tune-1 garbage\n", f);
        std::fputs(std::string(2000, 'x').c_str(), f);
        std::fputs("\n", f);
        std::fclose(f);
    }
    p = pond_plan_create_ex(F0, BW, 1.0, 1 << 18, 256, P0, POND_HALF, POND_BATCH_AUTOTUNE);
    CHECK(p != nullptr);
    CHECK(pond_plan_autotune(p, &b2, nullptr, nullptr, nullptr, &fc) == POND_OK && b2 == b);
    pond_plan_destroy(p);
    unsetenv("POND_AUTOTUNE_CACHE");
    std::remove(path);
}

void run_search(int8_t* iq, int64_t nsamp) {
    const double dms[4] = {0.0, 0.5, 1.0, 2.0};
    float* out = nullptr;
    CHECK(hipMalloc(reinterpret_cast<void**>(&out), 4 * 128 * sizeof(float)) == hipSuccess);
    for (int32_t mb : {0, POND_BATCH_AUTOTUNE}) {
        pond_search* s = pond_search_create_ex(F0, BW, dms, 4, 128, P0, 1 << 16, 1 << 19, POND_HALF, mb);
        CHECK(s != nullptr);
        if (!s) continue;
        for (int t = 0; t < 4; ++t) {
            int64_t n = 0, nf = 0, h = 0;
            CHECK(pond_search_trial(s, t, &n, &nf, &h) == POND_OK);
            int32_t b = 0;
            CHECK((pond_search_autotune(s, n, &b, nullptr, nullptr, nullptr, nullptr) == POND_OK) ==
                  (mb == POND_BATCH_AUTOTUNE));
        }
        CHECK(pond_search_run(s, iq, nsamp, out, nullptr) == POND_OK);
        pond_search_destroy(s);
    }
    (void)hipFree(out);
}

void run_server() {
    pond_stream_desc d{};
    d.f0_mhz = F0;
    d.bw_mhz = BW;
    d.dm = 1.0;
    d.period_s = P0;
    d.nfft = 1 << 18;
    d.subint_nsamp = 1 << 20;
    d.max_block_nsamp = 1 << 19;
    d.nbins = 128;
    d.precision = POND_HALF;
    const int64_t one = pond_server_stream_bytes(&d);
    CHECK(one > 0);
    // room for two streams: the third waits for a close
    pond_server* s = pond_server_create(2 * one + one / 8, 8);
    CHECK(s != nullptr);
    if (!s) return;
    int32_t id[3];
    for (int i = 0; i < 3; ++i) id[i] = pond_server_open(s, &d);
    CHECK(id[0] >= 0 && id[1] >= 0 && id[2] >= 0);
    CHECK(pond_server_stream_state(s, id[2]) == POND_STREAM_WAITING);
    std::vector<int8_t> block((size_t)2 * (1 << 19));
    uint64_t x = 88172645463325252ull;
    for (auto& v : block) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        v = (int8_t)((int)(x >> 56) % 21 - 10);
    }
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) CHECK(pond_server_submit(s, id[i], block.data(), 1 << 19) >= 0);
    pond_completion c[16];
    for (int k = 0; k < 20; ++k) CHECK(pond_server_poll(s, c, 16, 1) >= 0);
    CHECK(pond_server_close(s, id[0]) == POND_OK);  // admits the waiting stream
    for (int k = 0; k < 20; ++k) CHECK(pond_server_poll(s, c, 16, 1) >= 0);
    CHECK(pond_server_stream_state(s, id[2]) == POND_STREAM_OPEN);
    std::vector<float> prof(16 * 128);
    CHECK(pond_server_take_profiles(s, id[0], prof.data(), 16) >= 1);
    int64_t used = 0, budget = 0, queued = 0;
    int32_t open = 0;
    CHECK(pond_server_query(s, &used, &budget, &open, &queued) == POND_OK && open == 2);
    CHECK(pond_server_close(s, id[1]) == POND_OK);
    pond_server_destroy(s);  // closes the last stream
}

void run_misc(int8_t* iq, int64_t nsamp) {
    // real input (A/B pairs: the same bytes read as pairs)
    pond_plan* r = pond_real_plan_create(F0, BW, 1.0, 1 << 19, 128, P0, POND_FP32, 0, POND_USB);
    CHECK(r != nullptr);
    float *prof = nullptr, *ser = nullptr;
    CHECK(hipMalloc(reinterpret_cast<void**>(&prof), 64 * 256 * sizeof(float)) == hipSuccess);
    CHECK(hipMalloc(reinterpret_cast<void**>(&ser), (size_t)(nsamp / 8 + 64) * sizeof(float)) == hipSuccess);
    if (r) {
        int64_t ns = 0;
        CHECK(pond_real_dedisperse(r, iq, nsamp, 0, prof, 64, 32, ser, nsamp / 8 + 64, &ns, nullptr) >= 0);
        pond_plan_destroy(r);
    }
    pond_aid* a = pond_aid_create(F0, BW, 1.0, 256, 16, 128, P0);
    CHECK(a != nullptr);
    if (a) {
        int64_t nspec = 0, nser = 0;
        CHECK(pond_aid_geometry(a, nsamp, &nspec, &nser, nullptr, nullptr, nullptr) == POND_OK);
        CHECK(pond_aid_run(a, iq, nsamp, prof, ser, nsamp / 8 + 64, nullptr) == nser);
        pond_aid_destroy(a);
    }
    CHECK(pond_dedisperse_segment_noalloc(F0, BW, 1.0, 1 << 18, 256, P0, POND_FP32, iq, nsamp, 16, prof, ser,
                                          nsamp / 8 + 64, nullptr) > 0);
    void *x = nullptr, *y = nullptr;
    CHECK(hipMalloc(&x, 1 << 20) == hipSuccess && hipMalloc(&y, 1 << 20) == hipSuccess);
    CHECK(pond_copy_device(y, x, 1 << 20, nullptr) == POND_OK);
    (void)hipFree(x);
    (void)hipFree(y);
    (void)hipFree(prof);
    (void)hipFree(ser);
}

}  // namespace

int main(int argc, char** argv) {
    const std::string mode = argc > 1 ? argv[1] : "cpu";
    run_cpu();
    if (mode == "gpu") {
        const int64_t nsamp = 3 << 20;
        int8_t* iq = device_noise(2 * nsamp, 12345);
        CHECK(iq != nullptr);
        if (iq) {
            std::printf("driver: plans\n");
            std::fflush(stdout);
            run_plans(iq, nsamp);
            std::printf("driver: autotune\n");
            std::fflush(stdout);
            run_autotune();
            std::printf("driver: search\n");
            std::fflush(stdout);
            run_search(iq, nsamp);
            std::printf("driver: server\n");
            std::fflush(stdout);
            run_server();
            std::printf("driver: real, aid, no-alloc, copy\n");
            std::fflush(stdout);
            run_misc(iq, nsamp);
            CHECK(hipDeviceSynchronize() == hipSuccess);
            (void)hipFree(iq);
        }
    }
    std::printf("driver %s: %d failed checks\n", mode.c_str(), g_fail);
    return g_fail == 0 ? 0 : 1;
}
