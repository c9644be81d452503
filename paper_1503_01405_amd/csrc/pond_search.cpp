// DM-trial search: one stream dedispersed and folded at many trial DMs.
//
// Trials are grouped by FFT length (N_t = clamp(2 discard_t, nfft_min,
// nfft_max), discard_t by the plan rule of the single-DM path); a group
// shares one block grid with hop = N_t / 2, so each block's forward
// transform (int8 unpack + column FFTs + twiddle + row FFTs) runs once per
// group.  Each trial then multiplies the stored spectrum by its own inverse
// ISM response (Sec. 3.7, Eq. (4)), inverts the row and column transforms,
// detects and folds into its own integer accumulators.  The response's
// phase is DM times a per-bin geometry factor, so one float64 table of that
// factor per group serves every trial (no per-trial tables).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/pond.h"
#include "pond_internal.hpp"
#include "pond_tune.hpp"

using namespace pond;

namespace {

constexpr int kSearchMaxLog2N = 24;

struct Group {
    int64_t nfft = 0, hop = 0;
    int log2n = 0, log2n1 = 0, log2n2 = 0;
    int max_batch = 1;
    float pscale = 1.0f;  // detected-power scale of K3 (packed float16: see pond_api.cpp)
    std::vector<int> trials;
    float2* tw1 = nullptr;    // exp(-2 pi i t / n1)
    float2* tw2 = nullptr;    // exp(-2 pi i t / n2)
    float2* tw4 = nullptr;    // [n2][n1] four-step twiddle
    void* htw4 = nullptr;     // packed float16 form: [n2][n1] twiddle / 16
    double* geo = nullptr;    // [n2][n1] chirp turns per unit DM, shared by the group's trials
    void* spec = nullptr;     // max_batch blocks of spectrum
    void* out = nullptr;      // max_batch blocks of one trial's row-inverse output
    bool tuned = false;       // max_batch chosen by the autotuner
    TuneResult tune;
};

int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

}  // namespace

struct pond_search {
    int device = 0;
    double f0 = 0, bw = 0, period = 0, fs = 0, inv_pfs = 0;
    int32_t nbins = 0, precision = 0, ntrials = 0;
    size_t elem = 8;
    std::vector<double> dm;
    std::vector<int64_t> n_front;
    std::vector<int> group_of;
    std::vector<Group> groups;
    uint64_t* acc_sum = nullptr;  // [ntrials][nbins]
    uint64_t* acc_cnt = nullptr;
    uint64_t* part_sum = nullptr;
    uint32_t* part_cnt = nullptr;
    uint64_t* status = nullptr;
    bool sticky = false;
    hipStream_t last_stream = nullptr;
};

namespace {

void free_search(pond_search* s) {
    for (auto& g : s->groups) {
        void* ptrs[] = {g.tw1, g.tw2, g.tw4, g.htw4, g.geo, g.spec, g.out};
        for (void* q : ptrs)
            if (q) (void)hipFree(q);
    }
    void* ptrs[] = {s->acc_sum, s->acc_cnt, s->part_sum, s->part_cnt, s->status};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
}

// Plan geometry of the single-DM path (same expressions, float64).
void trial_geometry(double f0, double bw, double dm, int64_t* n_front, int64_t* discard) {
    const double fs = bw * 1e6;
    const double k_dm = 1.0 / 2.41e-4;
    const double f_lo = f0 - bw / 2, f_hi = f0 + bw / 2;
    const double delta_lo = k_dm * dm * (1.0 / (f_lo * f_lo) - 1.0 / (f0 * f0));
    const double delta_hi = k_dm * dm * (1.0 / (f0 * f0) - 1.0 / (f_hi * f_hi));
    const int64_t nf = (int64_t)std::ceil(delta_hi * fs);
    const int64_t s = nf + (int64_t)std::ceil(delta_lo * fs);
    int64_t d = 0;
    if (s > 0) {
        d = 16;
        while (d < s) d <<= 1;
    }
    *n_front = nf;
    *discard = d;
}

// The group's work for blocks block0 .. block0 + nb - 1 of `iq` (absolute
// sample 0 at iq): K1 and the forward rows into `spec`, then for each of
// the first `ntr` trials of the group the inverse rows into `out`, K3 and
// the fold reduction into that trial's accumulators.
hipError_t run_group(const pond_search* s, const Group& g, void* spec, void* out, const int8_t* iq, int64_t block0,
                     int nb, size_t ntr, hipStream_t stream, ReduceQueue& rq) {
    const int32_t nbins = s->nbins;
    const int64_t n1 = (int64_t)1 << g.log2n1;
    const int64_t cap = hist_capacity(g.log2n2, s->precision);
    const bool global_mode = nbins > cap;
    K1Args a1{};
    a1.tail = iq;
    a1.tail_start = 0;
    a1.in = iq;
    a1.in_start = 0;
    a1.hop = g.hop;
    a1.block0 = block0;
    a1.nblocks = nb;
    a1.log2n1 = g.log2n1;
    a1.work = spec;
    a1.tw2 = g.tw2;
    a1.scale = std::ldexp(1.0f, -g.log2n2);
    a1.f16_cols = 2 * g.hop == g.nfft;
    hipError_t e = launch_k1(s->precision, g.log2n2, a1, stream);
    if (e != hipSuccess) return e;
    K2Args f{};
    f.work = spec;
    f.nblocks = nb;
    f.log2n2 = g.log2n2;
    f.tw1 = g.tw1;
    f.tw4 = g.tw4;
    f.htw4 = g.htw4;
    f.scale = std::ldexp(1.0f, -g.log2n1);
    e = launch_k2(s->precision, kRowFwd, g.log2n1, f, stream);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < ntr && i < g.trials.size(); ++i) {
        const int t = g.trials[i];
        K2Args v{};
        v.in = spec;
        v.out = out;
        v.nblocks = nb;
        v.log2n2 = g.log2n2;
        v.tw1 = g.tw1;
        v.tw4 = g.tw4;
        v.htw4 = g.htw4;
        v.geo = g.geo;
        v.dm = s->dm[t];
        v.scale = 1.0f;
        e = launch_k2(s->precision, kRowInv, g.log2n1, v, stream);
        if (e != hipSuccess) return e;
        K3Args a3{};
        a3.work = out;
        a3.nblocks = nb;
        a3.log2n1 = g.log2n1;
        a3.hop = g.hop;
        a3.n_front = s->n_front[t];
        a3.block0 = block0;
        a3.tw2 = g.tw2;
        a3.scale = 1.0f;
        a3.pscale = g.pscale;
        a3.series = nullptr;
        a3.series_base = 0;
        a3.decim = 16;
        a3.nbins = nbins;
        a3.inv_pfs = s->inv_pfs;
        a3.subint = 0;
        a3.s_base = 0;
        a3.entries = nbins;
        a3.global_mode = global_mode ? 1 : 0;
        a3.acc_sum = s->acc_sum + (int64_t)t * nbins;
        a3.acc_cnt = s->acc_cnt + (int64_t)t * nbins;
        a3.acc_s0 = 0;
        a3.status = reinterpret_cast<uint32_t*>(s->status);
        const size_t dyn = global_mode ? 0 : (size_t)nbins * 12;
        const int grid = k3_grid(g.log2n2, s->precision, dyn, (int64_t)nb * (n1 / 16), nbins, global_mode);
        // the trials' fold reductions are queued (ReduceQueue), four per launch
        const bool deferred = !global_mode && (int64_t)grid * nbins <= kPartRegion;
        if (!global_mode && !deferred) e = rq.flush(stream);
        if (e != hipSuccess) return e;
        a3.part_sum = deferred ? rq.part_sum(s->part_sum) : s->part_sum;
        a3.part_cnt = deferred ? rq.part_cnt(s->part_cnt) : s->part_cnt;
        e = launch_k3(s->precision, g.log2n2, a3, grid, dyn, stream);
        if (e != hipSuccess) return e;
        if (!global_mode) {
            const ReduceJob job{a3.part_sum, a3.part_cnt, a3.acc_sum, a3.acc_cnt, 0, grid, nbins};
            if (deferred) {
                e = rq.push(job, stream);
            } else {
                ReduceBatch one;
                one.job[0] = job;
                one.n = 1;
                e = launch_fold_reduce_batch(one, stream);
            }
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Autotuned blocks per launch of one group (tables built, fold buffers in
// place, spec/out not allocated): the group's pass with two trials (the
// per-trial part is the same for every trial) on pseudo-random input.
hipError_t tune_group(pond_search* s, Group& g, int default_batch) {
    size_t free_b = 0, total_b = 0;
    hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return e;
    const int64_t block_bytes = 2 * g.nfft * (int64_t)s->elem;  // spec + out
    const int64_t cap = std::min<int64_t>((int64_t)4 << 30, (int64_t)(free_b / 3));
    const std::vector<int> cand = batch_candidates(block_bytes, cap, default_batch);
    const int nb_max = cand.back();
    void *spec = nullptr, *out = nullptr;
    int8_t* in = nullptr;
    // input streamed through a ring larger than the caches (TuneRing)
    const TuneRing ring = tune_ring(g.nfft, g.hop, 2, nb_max, (int64_t)(free_b / 6));
    e = hipMalloc(&spec, (size_t)nb_max * g.nfft * s->elem);
    if (e == hipSuccess) e = hipMalloc(&out, (size_t)nb_max * g.nfft * s->elem);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&in), (size_t)ring.bytes);
    if (e == hipSuccess)
        e = launch_fill_noise_u64(reinterpret_cast<uint64_t*>(in), ring.bytes / 8, 0x706f6e64ull, nullptr);
    if (e == hipSuccess) {
        TuneKey key;
        key.path = "search2";
        key.nfft = g.nfft;
        key.precision = s->precision;
        key.kind = POND_INPUT_COMPLEX;
        key.global_hist = s->nbins > hist_capacity(g.log2n2, s->precision);
        int64_t runs = 0;
        ReduceQueue rq;
        e = autotune_batch(
            key, cand, default_batch,
            [&](int nb) { return run_group(s, g, spec, out, in, ring.start(runs++, nb), nb, 2, nullptr, rq); },
            &g.tune);
        if (e == hipSuccess) e = rq.flush(nullptr);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (spec) (void)hipFree(spec);
    if (out) (void)hipFree(out);
    if (in) (void)hipFree(in);
    if (e == hipSuccess) {
        g.max_batch = g.tune.batch;
        g.tuned = true;
    }
    return e;
}

}  // namespace

extern "C" {

pond_search* pond_search_create(double f0_mhz, double bw_mhz, const double* dms, int32_t ntrials, int32_t nbins,
                                double period_s, int64_t nfft_min, int64_t nfft_max, int32_t precision) {
    return pond_search_create_ex(f0_mhz, bw_mhz, dms, ntrials, nbins, period_s, nfft_min, nfft_max, precision, 0);
}

pond_search* pond_search_create_ex(double f0_mhz, double bw_mhz, const double* dms, int32_t ntrials, int32_t nbins,
                                   double period_s, int64_t nfft_min, int64_t nfft_max, int32_t precision,
                                   int32_t max_batch) {
    if (!dms || ntrials < 1 || nbins < 1 || nbins > 65536) return nullptr;
    if (!std::isfinite(f0_mhz) || !std::isfinite(bw_mhz) || !std::isfinite(period_s)) return nullptr;
    if (!(bw_mhz > 0) || !(f0_mhz - bw_mhz / 2 > 0)) return nullptr;
    if (precision != POND_FP32 && precision != POND_MIXED && precision != POND_MIXED_VALU && precision != POND_HALF)
        return nullptr;
    if (nfft_min <= 0 || (nfft_min & (nfft_min - 1)) || nfft_max < nfft_min || (nfft_max & (nfft_max - 1)))
        return nullptr;
    if (ilog2(nfft_min) < 10 || ilog2(nfft_max) > kSearchMaxLog2N) return nullptr;
    const double fs = bw_mhz * 1e6;
    if (!(period_s > 0) || !(period_s * fs >= 1.0)) return nullptr;
    for (int t = 0; t < ntrials; ++t)
        if (!std::isfinite(dms[t]) || !(dms[t] >= 0) || dms[t] > 1e6) return nullptr;

    pond_search* s = new (std::nothrow) pond_search();
    if (!s) return nullptr;
    s->f0 = f0_mhz;
    s->bw = bw_mhz;
    s->period = period_s;
    s->fs = fs;
    s->inv_pfs = 1.0 / (period_s * fs);
    s->nbins = nbins;
    s->precision = precision;
    s->ntrials = ntrials;
    s->elem = precision == POND_FP32 ? 8 : 4;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return nullptr;
    }
    // Trial geometry and grouping by FFT length.
    s->dm.assign(dms, dms + ntrials);
    s->n_front.resize(ntrials);
    s->group_of.resize(ntrials);
    for (int t = 0; t < ntrials; ++t) {
        int64_t nf, d;
        trial_geometry(f0_mhz, bw_mhz, dms[t], &nf, &d);
        if (d > nfft_max / 2) {
            delete s;
            return nullptr;
        }
        int64_t n = 2 * d;
        n = n < nfft_min ? nfft_min : (n > nfft_max ? nfft_max : n);
        s->n_front[t] = nf;
        int gi = -1;
        for (size_t i = 0; i < s->groups.size(); ++i)
            if (s->groups[i].nfft == n) gi = (int)i;
        if (gi < 0) {
            Group g;
            g.nfft = n;
            g.hop = n / 2;
            g.log2n = ilog2(n);
            g.log2n2 = g.log2n / 2 < 10 ? g.log2n / 2 : 10;
            g.log2n1 = g.log2n - g.log2n2;
            int64_t b = ((int64_t)1 << 28) / (n * (int64_t)s->elem);
            g.max_batch = max_batch > 0 ? max_batch : (int)(b < 1 ? 1 : (b > 16 ? 16 : b));
            s->groups.push_back(g);
            gi = (int)s->groups.size() - 1;
        }
        s->group_of[t] = gi;
        s->groups[gi].trials.push_back(t);
    }

    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    // fold buffers first (the autotuner's launches fold too; every run
    // clears the accumulators it uses)
    chk(hipMalloc(reinterpret_cast<void**>(&s->acc_sum), (size_t)ntrials * nbins * 8));
    chk(hipMalloc(reinterpret_cast<void**>(&s->acc_cnt), (size_t)ntrials * nbins * 8));
    chk(hipMalloc(reinterpret_cast<void**>(&s->part_sum), (size_t)kPartEntries * 8));
    chk(hipMalloc(reinterpret_cast<void**>(&s->part_cnt), (size_t)kPartEntries * 4));
    chk(hipMalloc(reinterpret_cast<void**>(&s->status), 8));
    for (auto& g : s->groups) {
        const int64_t n1 = (int64_t)1 << g.log2n1, n2 = (int64_t)1 << g.log2n2;
        chk(hipMalloc(reinterpret_cast<void**>(&g.tw1), n1 * sizeof(float2)));
        chk(hipMalloc(reinterpret_cast<void**>(&g.tw2), n2 * sizeof(float2)));
        if (e == hipSuccess) chk(launch_stage_twiddles(g.tw1, n1, nullptr));
        if (e == hipSuccess) chk(launch_stage_twiddles(g.tw2, n2, nullptr));
        // One table per group for every trial: the four-step twiddle, and the
        // chirp's turns per unit DM of each bin (each trial's chirp is formed
        // from it and its DM in the inverse rows).
        const bool half = f16_arith(precision);
        const double df = bw_mhz / (double)g.nfft;
        if (half) chk(hipMalloc(&g.htw4, g.nfft * 4));
        else chk(hipMalloc(reinterpret_cast<void**>(&g.tw4), g.nfft * sizeof(float2)));
        chk(hipMalloc(reinterpret_cast<void**>(&g.geo), g.nfft * sizeof(double)));
        if (e == hipSuccess) {
            if (half) chk(launch_k2_build_split_tables_h(g.htw4, nullptr, g.log2n1, g.log2n2, 0.0, f0_mhz, df, nullptr));
            else chk(launch_k2_build_split_tables(g.tw4, nullptr, g.log2n1, g.log2n2, 0.0, f0_mhz, df, nullptr));
        }
        if (e == hipSuccess) chk(launch_build_dm_geometry(g.geo, g.log2n1, g.log2n2, f0_mhz, df, nullptr));
        if (e == hipSuccess && max_batch == POND_BATCH_AUTOTUNE) chk(tune_group(s, g, g.max_batch));
        chk(hipMalloc(&g.spec, (size_t)g.max_batch * g.nfft * s->elem));
        chk(hipMalloc(&g.out, (size_t)g.max_batch * g.nfft * s->elem));
        // Packed float16: power scale 256 over the measured gain of the
        // group's float16 path (forward rows, then the inverse rows of the
        // group's first trial; every trial's chirp rounds alike).
        if (half && e == hipSuccess) {
            HalfCal cal;
            cal.prec = precision;
            cal.log2n1 = g.log2n1;
            cal.log2n2 = g.log2n2;
            cal.tw2 = g.tw2;
            cal.work = g.spec;
            cal.max_batch = g.max_batch;
            cal.f16_cols = 2 * g.hop == g.nfft;
            double gain = 1.0;
            chk(half_power_gain(
                cal,
                [&](int nb, const void** res) {
                    K2Args f{};
                    f.work = g.spec;
                    f.nblocks = nb;
                    f.log2n2 = g.log2n2;
                    f.tw1 = g.tw1;
                    f.htw4 = g.htw4;
                    hipError_t r = launch_k2(precision, kRowFwd, g.log2n1, f, nullptr);
                    K2Args v = f;
                    v.in = g.spec;
                    v.out = g.out;
                    v.geo = g.geo;
                    v.dm = s->dm[g.trials[0]];
                    if (r == hipSuccess) r = launch_k2(precision, kRowInv, g.log2n1, v, nullptr);
                    *res = g.out;
                    return r;
                },
                &gain));
            g.pscale = (float)(256.0 / gain);
        }
    }
    if (e == hipSuccess) chk(hipMemset(s->status, 0, 8));
    if (e == hipSuccess) chk(hipStreamSynchronize(nullptr));
    if (e != hipSuccess) {
        free_search(s);
        delete s;
        (void)hipGetLastError();
        return nullptr;
    }
    return s;
}

int32_t pond_search_autotune(const pond_search* s, int64_t nfft, int32_t* batch, double* ms_per_block,
                             int32_t* default_batch, double* default_ms_per_block, int32_t* from_cache) {
    if (!s) return POND_EINVAL;
    for (const Group& g : s->groups) {
        if (g.nfft != nfft) continue;
        if (!g.tuned) return POND_EINVAL;
        if (batch) *batch = g.tune.batch;
        if (ms_per_block) *ms_per_block = g.tune.ms_per_block;
        if (default_batch) *default_batch = g.tune.default_batch;
        if (default_ms_per_block) *default_ms_per_block = g.tune.default_ms_per_block;
        if (from_cache) *from_cache = g.tune.from_cache ? 1 : 0;
        return POND_OK;
    }
    return POND_EINVAL;
}

int32_t pond_search_trial(const pond_search* s, int32_t t, int64_t* nfft, int64_t* n_front, int64_t* hop) {
    if (!s || t < 0 || t >= s->ntrials) return POND_EINVAL;
    const Group& g = s->groups[s->group_of[t]];
    if (nfft) *nfft = g.nfft;
    if (n_front) *n_front = s->n_front[t];
    if (hop) *hop = g.hop;
    return POND_OK;
}

int32_t pond_search_run(pond_search* s, const int8_t* iq, int64_t nsamp, float* profiles, void* stream_ptr) {
    if (!s) return POND_EINVAL;
    if (s->sticky) return POND_EDEVICE;
    if (nsamp < 0 || (nsamp > 0 && (!iq || (reinterpret_cast<uintptr_t>(iq) & 1u))) || !profiles)
        return POND_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_ptr);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return POND_EDEVICE;
    if (cur != s->device && hipSetDevice(s->device) != hipSuccess) return POND_EDEVICE;
    hipError_t e = hipSuccess;
    auto done = [&](int32_t r) {
        if (cur != s->device) (void)hipSetDevice(cur);
        return r;
    };
    auto fail = [&]() {
        (void)hipGetLastError();
        s->sticky = true;
        return done(POND_EDEVICE);
    };
    const int32_t nbins = s->nbins;
    e = launch_zero_u64(s->acc_sum, (int64_t)s->ntrials * nbins, stream);
    if (e == hipSuccess) e = launch_zero_u64(s->acc_cnt, (int64_t)s->ntrials * nbins, stream);
    if (e != hipSuccess) return fail();

    ReduceQueue rq;
    for (auto& g : s->groups) {
        const int64_t nb_total = nsamp < g.nfft ? 0 : (nsamp - g.nfft) / g.hop + 1;
        for (int64_t b = 0; b < nb_total; b += g.max_batch) {
            const int nb = (int)(nb_total - b < g.max_batch ? nb_total - b : g.max_batch);
            e = run_group(s, g, g.spec, g.out, iq, b, nb, g.trials.size(), stream, rq);
            if (e != hipSuccess) return fail();
        }
    }
    e = rq.flush(stream);
    if (e != hipSuccess) return fail();
    e = launch_fold_profiles(s->acc_sum, s->acc_cnt, (int64_t)s->ntrials * nbins, profiles, stream);
    if (e != hipSuccess) return fail();
    s->last_stream = stream;
    return done(POND_OK);
}

void pond_search_destroy(pond_search* s) {
    if (!s) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != s->device) (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->last_stream);
    free_search(s);
    if (cur >= 0 && cur != s->device) (void)hipSetDevice(cur);
    delete s;
}

}  // extern "C"
