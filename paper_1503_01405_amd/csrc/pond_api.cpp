// Host runtime behind include/pond.h: plan geometry (float64), device
// workspace, streaming state (input tail, block counter, sub-integration
// accumulators) and the launch sequence K1 -> K2 -> K3 -> fold reduction per
// batch of overlap-save blocks, then the profile finalisation.
#include <hip/hip_runtime.h>

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

thread_local int32_t g_create_status = POND_OK;

constexpr int64_t kMinLog2N = 10;
constexpr int64_t kMaxLog2N = 27;       // complex input; rows past 2^14 take the split middle pass
constexpr int64_t kMaxLog2NReal = 24;   // real input (its middle passes transform whole rows)
constexpr int kMaxLog2N2 = 10;          // column length cap (K1/K3 tile = 16 columns in LDS)
constexpr int64_t kDefaultAccSlots = 4; // sub-integrations the accumulator ring holds at creation

int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

struct Geometry {
    double delta_lo = 0, delta_hi = 0;
    int64_t n_front = 0, discard = 0, hop = 0;
};

// Overlap-save geometry of a block of nfft samples (Sec. 3.7: the filter is
// longer than the smear, the cyclic edges are dropped), float64: the delays
// of the band edges relative to f0 (the constant of Eq. (1)), n_front =
// ceil(delta_hi fs), s = n_front + ceil(delta_lo fs), discard =
// next_pow2(max(s, 16)) if that is <= nfft / 2, else s rounded up to 16 (0
// when s = 0), hop = nfft - discard.  False if hop would not be positive.
bool plan_geometry(double f0_mhz, double bw_mhz, double dm, int64_t nfft, Geometry* g) {
    const double fs = bw_mhz * 1e6;
    const double k_dm = 1.0 / 2.41e-4;  // s MHz^2 per unit DM, the constant of Eq. (1)
    const double f_lo = f0_mhz - bw_mhz / 2;
    const double f_hi = f0_mhz + bw_mhz / 2;
    g->delta_lo = k_dm * dm * (1.0 / (f_lo * f_lo) - 1.0 / (f0_mhz * f0_mhz));
    g->delta_hi = k_dm * dm * (1.0 / (f0_mhz * f0_mhz) - 1.0 / (f_hi * f_hi));
    const double front_d = std::ceil(g->delta_hi * fs);
    const double back_d = std::ceil(g->delta_lo * fs);
    if (!(front_d + back_d < (double)nfft)) return false;
    g->n_front = (int64_t)front_d;
    const int64_t s = g->n_front + (int64_t)back_d;
    g->discard = 0;
    if (s > 0) {
        int64_t p2 = 16;
        while (p2 < s) p2 <<= 1;
        g->discard = p2 <= nfft / 2 ? p2 : ((s + 15) / 16) * 16;
    }
    g->hop = nfft - g->discard;
    return g->hop > 0;
}

}  // namespace

struct pond_plan {
    int device = 0;
    double f0 = 0, bw = 0, dm = 0, period = 0;
    double fs = 0, delta_lo = 0, delta_hi = 0, inv_pfs = 0, chirp_a = 0, df = 0;
    int64_t nfft = 0, n_front = 0, discard = 0, hop = 0;
    int log2n = 0, log2n1 = 0, log2n2 = 0, hbits = 0;
    int32_t nbins = 0, precision = 0;
    int max_batch = 1;
    size_t elem = 8;
    // Real two-channel input (Sec. 3.1: channels A and B added in phase):
    // element m packs real samples 2m, 2m+1; every count above is in
    // elements, the filter and fold in real samples.
    int32_t kind = POND_INPUT_COMPLEX;
    int bpe = 2;                // input bytes per element
    // Rows up to 2^13: one fused middle pass (k2_real_pair) with rtab =
    // (four-step twiddle, filter) and wk; longer rows: forward rows, split,
    // inverse rows with tw4 and rtab = (split twiddle, filter).
    bool real_fused = false;
    float2* tw4 = nullptr;
    float4* rtab = nullptr;     // [nfft + 1]
    float2* wk = nullptr;       // [n2 + n1]

    void* work = nullptr;
    int8_t* tail[2] = {nullptr, nullptr};
    int tcur = 0;
    int64_t tail_start = 0;
    float2* tw1 = nullptr;
    float2* tw2 = nullptr;
    void* table = nullptr;      // float32 arithmetic forms: chirp (float32 storage) or twiddle and chirp
    void* htable = nullptr;     // float16 arithmetic forms: twiddle / 16 and chirp (8 bytes per entry)
    // Split middle pass (rows n1 = m2 2^13 longer than 2^14): tw1 then holds
    // the sub-row twiddles, tw_n1 the row's, tw_hi / tw_lo the two-level
    // block twiddle, chirp_split the chirp in sub-row order (float2, or
    // float16 pairs for the float16 arithmetic forms).
    int log2m2 = 0;             // 0: rows transformed whole
    int log2s = 0;
    float2* tw_n1 = nullptr;
    float2* tw_hi = nullptr;
    float2* tw_lo = nullptr;
    void* chirp_split = nullptr;
    float pscale = 1.0f;        // detected-power scale applied in K3
    bool tuned = false;         // max_batch chosen by the autotuner
    TuneResult tune;
    // Packed float16: the middle pass leaves 1/16 of the value (its twiddle
    // table carries the first stage's 1/16), so the power scale is 256
    // divided by half_gain, the measured power gain of the float16
    // arithmetic (half_power_gain).
    double half_gain = 1.0;
    double taper = 0.0;         // Tukey edge fraction of the inverse filter (0: unit taper)
    uint64_t* acc_sum = nullptr;
    uint64_t* acc_cnt = nullptr;
    int64_t acc_slots = 0;
    uint64_t* part_sum = nullptr;
    uint32_t* part_cnt = nullptr;
    int64_t hist_cap = 0;
    uint64_t* status = nullptr;  // low 32 bits used

    // per-kernel timing (measurement only)
    bool timing = false;
    struct Mark {
        int kernel;
        int64_t blocks;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> event_pool;
    double t_ms[POND_NKERNELS] = {0};
    int64_t t_launch[POND_NKERNELS] = {0};
    int64_t t_blocks[POND_NKERNELS] = {0};

    int64_t samples_in = 0;
    int64_t blocks_done = 0;
    int64_t subint = -1;
    bool sticky = false;
    hipStream_t last_stream = nullptr;
};

namespace {

struct DeviceGuard {
    int old = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) { ok = false; return; }
        if (old != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

hipEvent_t take_event(pond_plan* p) {
    if (!p->event_pool.empty()) {
        hipEvent_t e = p->event_pool.back();
        p->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Fold finished marks into the sums (events must have completed).
hipError_t collect_marks(pond_plan* p) {
    hipError_t err = hipSuccess;
    for (auto& m : p->marks) {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, m.a, m.b);
        if (e == hipSuccess) {
            p->t_ms[m.kernel] += ms;
            p->t_launch[m.kernel] += 1;
            p->t_blocks[m.kernel] += m.blocks;
        } else if (err == hipSuccess) {
            err = e;
        }
        p->event_pool.push_back(m.a);
        p->event_pool.push_back(m.b);
    }
    p->marks.clear();
    return err;
}

void free_plan_memory(pond_plan* p) {
    for (auto& m : p->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    p->marks.clear();
    for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
    p->event_pool.clear();
    void* ptrs[] = {p->work,   p->tail[0], p->tail[1], p->tw1,     p->tw2,         p->table,
                    p->htable, p->tw4,     p->rtab,    p->wk,      p->tw_n1,       p->tw_hi,
                    p->tw_lo,  p->acc_sum, p->acc_cnt, p->part_sum, p->part_cnt, p->status, p->chirp_split};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
}

// The middle pass of a complex-input plan over nb blocks in p->work: K2 in
// kRowFull mode, or for rows longer than 2^14 the split pass (forward column
// pass, K2 kRowChirp on the sub-rows of 2^13, inverse column pass).  The
// normalisation is the same either way: 1/n1 on the forward side (split:
// 1/m2 in the column pass, 1/m1 in the sub-rows), and the float16 forms'
// output keeps 1/16 of the value (K2 multiplies by the twiddle / 16; the
// split pass's inverse columns scale by 1/16; the forward columns carry the
// first row stage's 1/16, which K2 otherwise takes from its table).
hipError_t run_middle(const pond_plan* p, void* work, int nb, hipStream_t stream) {
    K2Args a2{};
    a2.work = work;
    a2.nblocks = nb;
    a2.tw1 = p->tw1;
    if (p->log2m2 == 0) {
        a2.log2n2 = p->log2n2;
        a2.table = p->table;
        a2.htable = p->htable;
        a2.scale = std::ldexp(1.0f, -p->log2n1);
        return launch_k2(p->precision, kRowFull, p->log2n1, a2, stream);
    }
    const bool h = f16_arith(p->precision);
    SplitColArgs sc{work, nb, p->log2n1, p->log2n2, p->tw_n1, p->tw_hi, p->tw_lo, p->log2s, 1.0f};
    sc.scale = std::ldexp(1.0f, -p->log2m2 - (h ? 4 : 0));
    hipError_t e = launch_split_cols(p->precision, false, sc, stream);
    if (e != hipSuccess) return e;
    a2.log2n2 = p->log2n2 + p->log2m2;
    a2.chirp = reinterpret_cast<const float2*>(p->chirp_split);
    a2.hchirp = p->chirp_split;
    a2.scale = std::ldexp(1.0f, -kSplitLog2M1);
    e = launch_k2(p->precision, kRowChirp, kSplitLog2M1, a2, stream);
    if (e != hipSuccess) return e;
    sc.scale = h ? 1.0f / 16.0f : 1.0f;
    return launch_split_cols(p->precision, true, sc, stream);
}

// One launch sequence of a complex-input plan (K1, middle pass, K3, fold
// reduction) over blocks 0 .. nb-1 of `in`, with one open sub-integration
// and no series: what the autotuner times.  Null stream.
hipError_t run_blocks(pond_plan* p, void* work, const int8_t* in, int nb, float* series, ReduceQueue& rq) {
    K1Args a1{};
    a1.tail = in;
    a1.tail_start = 0;
    a1.in = in;
    a1.in_start = 0;
    a1.hop = p->hop;
    a1.block0 = 0;
    a1.nblocks = nb;
    a1.log2n1 = p->log2n1;
    a1.work = work;
    a1.tw2 = p->tw2;
    a1.scale = std::ldexp(1.0f, -p->log2n2);
    a1.f16_cols = 2 * p->hop == p->nfft;
    hipError_t e = launch_k1(p->precision, p->log2n2, a1, nullptr);
    if (e == hipSuccess) e = run_middle(p, work, nb, nullptr);
    if (e != hipSuccess) return e;
    const bool global_mode = p->nbins > p->hist_cap;
    K3Args a3{};
    a3.work = work;
    a3.nblocks = nb;
    a3.log2n1 = p->log2n1;
    a3.hop = p->hop;
    a3.n_front = p->n_front;
    a3.block0 = 0;
    a3.tw2 = p->tw2;
    a3.scale = 1.0f;
    a3.pscale = p->pscale;
    a3.series = series;
    a3.series_base = 0;
    a3.decim = 16;
    a3.nbins = p->nbins;
    a3.inv_pfs = p->inv_pfs;
    a3.subint = 0;
    a3.s_base = 0;
    a3.entries = p->nbins;
    a3.global_mode = global_mode ? 1 : 0;
    a3.acc_sum = p->acc_sum;
    a3.acc_cnt = p->acc_cnt;
    a3.acc_s0 = 0;
    a3.status = reinterpret_cast<uint32_t*>(p->status);
    const size_t dyn = global_mode ? 0 : (size_t)p->nbins * 12;
    const int grid = k3_grid(p->log2n2, p->precision, dyn, (int64_t)nb << (p->log2n1 - 4), p->nbins, global_mode);
    // fold reductions queued as in a call
    const bool deferred = !global_mode && (int64_t)grid * p->nbins <= kPartRegion;
    if (!global_mode && !deferred) e = rq.flush(nullptr);
    if (e != hipSuccess) return e;
    a3.part_sum = deferred ? rq.part_sum(p->part_sum) : p->part_sum;
    a3.part_cnt = deferred ? rq.part_cnt(p->part_cnt) : p->part_cnt;
    e = launch_k3(p->precision, p->log2n2, a3, grid, dyn, nullptr);
    if (e == hipSuccess && !global_mode) {
        const ReduceJob job{a3.part_sum, a3.part_cnt, p->acc_sum, p->acc_cnt, 0, grid, p->nbins};
        if (deferred) {
            e = rq.push(job, nullptr);
        } else {
            ReduceBatch one;
            one.job[0] = job;
            one.n = 1;
            e = launch_fold_reduce_batch(one, nullptr);
        }
    }
    return e;
}

int default_max_batch(int64_t nfft, int32_t precision, int32_t max_batch);

// Autotuned blocks per launch of a complex-input plan (tables, twiddles and
// fold buffers in place, p->work not yet allocated): candidates whose work
// area fits in min(4 GiB, a third of the free device memory), timed on a
// pseudo-random int8 stream.  Leaves the fold buffers dirty (the caller
// clears them).
hipError_t tune_plan(pond_plan* p) {
    size_t free_b = 0, total_b = 0;
    hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return e;
    const int64_t block_bytes = p->nfft * (int64_t)p->elem;
    const int64_t cap = std::min<int64_t>((int64_t)4 << 30, (int64_t)(free_b / 3));
    const int dflt = default_max_batch(p->nfft, p->precision, 0);
    const std::vector<int> cand = batch_candidates(block_bytes, cap, dflt);
    const int nb_max = cand.back();
    void* work = nullptr;
    int8_t* in = nullptr;
    float* series = nullptr;
    // The input streams through a ring several times the size of the
    // Infinity Cache, so that each timed run reads samples no earlier run
    // left in the caches (as a recorded stream is read); the work area is
    // reused from run to run, as in a call.
    const TuneRing ring = tune_ring(p->nfft, p->hop, p->bpe, nb_max, (int64_t)(free_b / 6));
    const int64_t ser_floats = (int64_t)nb_max * (p->hop / 16 + 1);
    e = hipMalloc(&work, (size_t)nb_max * block_bytes);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&in), (size_t)ring.bytes);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&series), (size_t)ser_floats * sizeof(float));
    if (e == hipSuccess)
        e = launch_fill_noise_u64(reinterpret_cast<uint64_t*>(in), ring.bytes / 8, 0x706f6e64ull, nullptr);
    if (e == hipSuccess) {
        TuneKey key;
        key.path = "dedisperse";
        key.nfft = p->nfft;
        key.precision = p->precision;
        key.kind = p->kind;
        key.global_hist = p->nbins > p->hist_cap;
        int64_t runs = 0;
        ReduceQueue rq;
        e = autotune_batch(key, cand, dflt,
                           [&](int nb) {
                               const int64_t b0 = ring.start(runs++, nb);
                               return run_blocks(p, work, in + b0 * p->hop * p->bpe, nb, series, rq);
                           },
                           &p->tune);
        if (e == hipSuccess) e = rq.flush(nullptr);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (work) (void)hipFree(work);
    if (in) (void)hipFree(in);
    if (series) (void)hipFree(series);
    if (e == hipSuccess) {
        p->max_batch = p->tune.batch;
        p->tuned = true;
    }
    return e;
}

int default_max_batch(int64_t nfft, int32_t precision, int32_t max_batch) {
    if (max_batch > 0) return max_batch;
    const int64_t elem = precision == POND_FP32 ? 8 : 4;
    const int64_t b = ((int64_t)1 << 29) / (nfft * elem);
    return (int)(b < 1 ? 1 : (b > 16 ? 16 : b));
}

int64_t n_blocks_for(int64_t nsamp, int64_t nfft, int64_t hop) {
    return nsamp < nfft ? 0 : (nsamp - nfft) / hop + 1;
}

}  // namespace

namespace pond {

namespace {
// splitmix64 (Steele, Lea & Flood 2014): the calibration noise generator.
uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}
}  // namespace

hipError_t half_power_gain(const HalfCal& c, const std::function<hipError_t(int, const void**)>& middle,
                           double* gain) {
    const int log2n = c.log2n1 + c.log2n2;
    const int64_t n = (int64_t)1 << log2n;
    const int64_t nblk = n >= ((int64_t)1 << 22) ? 1 : ((int64_t)1 << 22) / n;
    const int64_t nsamp = nblk * n;
    std::vector<int8_t> iq((size_t)(2 * nsamp));
    int64_t energy = 0;
    for (int64_t i = 0; i < nsamp; i += 4) {
        const uint64_t h = splitmix64((uint64_t)i);
        for (int k = 0; k < 8; ++k) {
            const int8_t v = (int8_t)((h >> (8 * k)) & 0xff);
            iq[(size_t)(2 * i + k)] = v;
            energy += (int64_t)v * v;
        }
    }
    int8_t* d_iq = nullptr;
    float* d_ser = nullptr;
    uint64_t* d_part = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&d_iq), iq.size());
    const int64_t nser = nsamp / 16;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d_ser), (size_t)nser * sizeof(float));
    // per-workgroup partials of a one-bin fold (unused) and the status word
    constexpr int64_t kParts = 4096;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&d_part), (size_t)kParts * 12 + 8);
    if (e == hipSuccess) e = hipMemcpy(d_iq, iq.data(), iq.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(d_part, 0, (size_t)kParts * 12 + 8);
    for (int64_t b = 0; b < nblk && e == hipSuccess; b += c.max_batch) {
        const int nb = (int)(nblk - b < c.max_batch ? nblk - b : c.max_batch);
        K1Args a1{};
        a1.tail = d_iq;
        a1.in = d_iq;
        a1.hop = n;
        a1.block0 = b;
        a1.nblocks = nb;
        a1.log2n1 = c.log2n1;
        a1.work = c.work;
        a1.tw2 = c.tw2;
        a1.f16_cols = c.f16_cols;
        e = launch_k1(c.prec, c.log2n2, a1, nullptr);
        const void* mid = nullptr;
        if (e == hipSuccess) e = middle(nb, &mid);
        if (e != hipSuccess) break;
        K3Args a3{};
        a3.work = mid;
        a3.nblocks = nb;
        a3.log2n1 = c.log2n1;
        a3.hop = n;
        a3.n_front = 0;
        a3.block0 = b;
        a3.tw2 = c.tw2;
        a3.scale = 1.0f;
        a3.pscale = 256.0f;
        a3.series = d_ser;
        a3.series_base = 0;
        a3.decim = 16;
        a3.nbins = 1;
        a3.inv_pfs = 1.0 / (double)n;
        a3.subint = 0;
        a3.entries = 1;
        a3.part_sum = d_part;
        a3.part_cnt = reinterpret_cast<uint32_t*>(d_part + kParts);
        a3.status = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(d_part) + kParts * 12);
        const int64_t items = (int64_t)nb << (c.log2n1 - 4);
        int grid = k3_grid(c.log2n2, c.prec, 12, items, 1, false);
        if (grid > kParts) grid = (int)kParts;
        e = launch_k3(c.prec, c.log2n2, a3, grid, 12, nullptr);
    }
    std::vector<float> ser((size_t)nser);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess) e = hipMemcpy(ser.data(), d_ser, (size_t)nser * sizeof(float), hipMemcpyDeviceToHost);
    if (d_iq) (void)hipFree(d_iq);
    if (d_ser) (void)hipFree(d_ser);
    if (d_part) (void)hipFree(d_part);
    if (e != hipSuccess) return e;
    double power = 0.0;
    for (float v : ser) power += (double)v;
    *gain = power / (double)energy;
    return std::isfinite(*gain) && *gain > 0.5 && *gain < 2.0 ? hipSuccess : hipErrorInvalidValue;
}

// Device bytes a plan allocates in pond_plan_create_ex (the accumulator
// ring at acc_slots sub-integrations, at least the default 4; it grows only
// for calls that span more).
int64_t plan_footprint(int64_t nfft, int32_t nbins, int32_t precision, int32_t max_batch, int64_t acc_slots) {
    const int log2n = ilog2(nfft);
    const int log2n2 = log2n / 2 < kMaxLog2N2 ? log2n / 2 : kMaxLog2N2;
    const int64_t n1 = (int64_t)1 << (log2n - log2n2), n2 = (int64_t)1 << log2n2;
    const int64_t elem = precision == POND_FP32 ? 8 : 4;
    const int64_t mb = default_max_batch(nfft, precision, max_batch);
    const bool split = (log2n - log2n2) > kMaxLog2RowN1;
    // float2 chirp (float32), two float16 pairs (float16 arithmetic), float4 otherwise
    int64_t tables = nfft * (precision == POND_FP32 || f16_arith(precision) ? 8 : 16) + (n1 + n2) * 8;
    if (split) {
        const int log2s = (log2n + 1) / 2;
        const int64_t m1 = (int64_t)1 << kSplitLog2M1;
        tables = nfft * (f16_arith(precision) ? 4 : 8) + (m1 + n2 + n1 + (nfft >> log2s) + ((int64_t)1 << log2s)) * 8;
    }
    const int64_t slots = acc_slots > kDefaultAccSlots ? acc_slots : kDefaultAccSlots;
    return mb * nfft * elem + 2 * nfft * 2 + tables + 2 * slots * (int64_t)nbins * 8 + kPartEntries * 12 + 8;
}

int plan_max_batch(int64_t nfft, int32_t precision, int32_t max_batch) {
    return default_max_batch(nfft, precision, max_batch);
}

}  // namespace pond

extern "C" {

int32_t pond_create_status(void) { return g_create_status; }

int32_t pond_copy_device(void* dst, const void* src, int64_t bytes, void* hip_stream) {
    if (bytes < 0 || (bytes > 0 && (!dst || !src))) return POND_EINVAL;
    if ((bytes & 15) || (reinterpret_cast<uintptr_t>(dst) & 15) || (reinterpret_cast<uintptr_t>(src) & 15))
        return POND_EINVAL;
    const hipError_t e = launch_copy_u128(dst, src, bytes / 16, reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return POND_EDEVICE;
    }
    return POND_OK;
}

int32_t pond_geometry(double f0_mhz, double bw_mhz, double dm, int64_t nfft, int64_t* n_front, int64_t* discard,
                      int64_t* hop) {
    if (!std::isfinite(f0_mhz) || !std::isfinite(bw_mhz) || !std::isfinite(dm)) return POND_EINVAL;
    if (!(bw_mhz > 0) || !(f0_mhz - bw_mhz / 2 > 0) || !(dm >= 0)) return POND_EINVAL;
    if (nfft <= 0 || (nfft & (nfft - 1)) != 0) return POND_EINVAL;
    Geometry g;
    if (!plan_geometry(f0_mhz, bw_mhz, dm, nfft, &g)) return POND_EINVAL;
    if (n_front) *n_front = g.n_front;
    if (discard) *discard = g.discard;
    if (hop) *hop = g.hop;
    return POND_OK;
}

const char* pond_strerror(int64_t code) {
    switch (code) {
        case POND_OK: return "ok";
        case POND_EINVAL: return "invalid argument or call sequence";
        case POND_ENOMEM: return "device allocation failed";
        case POND_EDEVICE: return "HIP runtime error (plan unusable)";
        case POND_EBUSY: return "can never fit the device-memory budget, or too many streams";
        case POND_ECANCELED: return "cancelled: its stream was closed before admission";
        default: return code > 0 ? "ok" : "unknown error";
    }
}

}  // extern "C"

namespace {

// Builds the filter table of the plan's middle pass (for the taper alpha).
hipError_t build_filter(pond_plan* p, double alpha) {
    const int lsb = p->kind == POND_INPUT_REAL_LSB ? 1 : 0;
    if (p->kind != POND_INPUT_COMPLEX && p->real_fused)
        return launch_real_build_pair_table(p->rtab, p->wk, p->log2n1, p->log2n2, p->chirp_a, p->f0, p->bw, lsb,
                                            alpha, nullptr);
    if (p->kind != POND_INPUT_COMPLEX)
        return launch_real_build_table(p->rtab, p->log2n1, p->log2n2, p->chirp_a, p->f0, p->bw, lsb, alpha, nullptr);
    if (p->log2m2 > 0)
        return launch_build_split_chirp(p->chirp_split, f16_arith(p->precision), p->log2n1, p->log2n2, p->chirp_a,
                                        p->f0, p->df, alpha, nullptr);
    if (f16_arith(p->precision))
        return launch_k2_build_table_h(p->htable, p->log2n1, p->log2n2, p->chirp_a, p->f0, p->df, alpha, nullptr);
    return launch_k2_build_table(p->table, p->precision != POND_FP32, p->log2n1, p->log2n2, p->chirp_a, p->f0, p->df,
                                 alpha, nullptr);
}

pond_plan* create_plan(double f0_mhz, double bw_mhz, double dm, int64_t nfft, int32_t nbins, double period_s,
                       int32_t precision, int32_t max_batch, int32_t kind, int64_t acc_slots = 0) {
    g_create_status = POND_EINVAL;
    if (kind != POND_INPUT_COMPLEX && precision != POND_FP32 && precision != POND_MIXED_VALU) return nullptr;
    if (!std::isfinite(f0_mhz) || !std::isfinite(bw_mhz) || !std::isfinite(dm) || !std::isfinite(period_s))
        return nullptr;
    if (!(bw_mhz > 0) || !(f0_mhz - bw_mhz / 2 > 0) || !(dm >= 0)) return nullptr;
    if (nfft <= 0 || (nfft & (nfft - 1)) != 0) return nullptr;
    const int log2n = ilog2(nfft);
    if (log2n < kMinLog2N || log2n > (kind == POND_INPUT_COMPLEX ? kMaxLog2N : kMaxLog2NReal)) return nullptr;
    if (nbins < 1 || nbins > 65536) return nullptr;
    if (precision != POND_FP32 && precision != POND_MIXED && precision != POND_MIXED_VALU && precision != POND_HALF &&
        precision != POND_BF16)
        return nullptr;
    const double fs = bw_mhz * 1e6;
    if (!(period_s > 0) || !(period_s * fs >= 1.0)) return nullptr;

    Geometry geo;
    if (!plan_geometry(f0_mhz, bw_mhz, dm, nfft, &geo)) return nullptr;
    const double delta_lo = geo.delta_lo, delta_hi = geo.delta_hi;
    const int64_t n_front = geo.n_front, discard = geo.discard, hop = geo.hop;

    pond_plan* p = new (std::nothrow) pond_plan();
    if (!p) {
        g_create_status = POND_ENOMEM;
        return nullptr;
    }
    g_create_status = POND_EDEVICE;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return nullptr;
    }
    p->f0 = f0_mhz;
    p->bw = bw_mhz;
    p->dm = dm;
    p->period = period_s;
    p->fs = fs;
    p->delta_lo = delta_lo;
    p->delta_hi = delta_hi;
    p->kind = kind;
    p->bpe = kind == POND_INPUT_COMPLEX ? 2 : 4;
    // The fold counts real samples at 2 fs on the real path.
    p->inv_pfs = 1.0 / (period_s * fs * (kind == POND_INPUT_COMPLEX ? 1.0 : 2.0));
    p->chirp_a = dm / (2.41e-10 * f0_mhz * f0_mhz);
    p->df = bw_mhz / (double)nfft;
    p->nfft = nfft;
    p->n_front = n_front;
    p->discard = discard;
    p->hop = hop;
    p->log2n = log2n;
    p->log2n2 = log2n / 2 < kMaxLog2N2 ? log2n / 2 : kMaxLog2N2;
    p->log2n1 = log2n - p->log2n2;
    p->hbits = (log2n + 1) / 2;
    p->nbins = nbins;
    p->precision = precision;
    p->elem = precision == POND_FP32 ? 8 : 4;
    const bool autotune = max_batch == POND_BATCH_AUTOTUNE;
    p->max_batch = max_batch = default_max_batch(nfft, precision, max_batch);

    p->hist_cap = hist_capacity(p->log2n2, p->precision);

    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    chk(hipMalloc(reinterpret_cast<void**>(&p->tail[0]), (size_t)nfft * p->bpe));
    chk(hipMalloc(reinterpret_cast<void**>(&p->tail[1]), (size_t)nfft * p->bpe));
    const int64_t n1 = (int64_t)1 << p->log2n1, n2 = (int64_t)1 << p->log2n2;
    // rows longer than one workgroup transforms: the split middle pass
    p->log2m2 = p->log2n1 > kMaxLog2RowN1 ? p->log2n1 - kSplitLog2M1 : 0;
    const int64_t row = p->log2m2 ? (int64_t)1 << kSplitLog2M1 : n1;  // K2's row length
    chk(hipMalloc(reinterpret_cast<void**>(&p->tw1), (size_t)row * sizeof(float2)));
    chk(hipMalloc(reinterpret_cast<void**>(&p->tw2), (size_t)n2 * sizeof(float2)));
    if (e == hipSuccess) chk(launch_stage_twiddles(p->tw1, row, nullptr));
    if (e == hipSuccess) chk(launch_stage_twiddles(p->tw2, n2, nullptr));
    if (p->log2m2) {
        p->log2s = (log2n + 1) / 2;
        const int64_t nlo = (int64_t)1 << p->log2s, nhi = nfft >> p->log2s;
        chk(hipMalloc(reinterpret_cast<void**>(&p->tw_n1), (size_t)n1 * sizeof(float2)));
        chk(hipMalloc(reinterpret_cast<void**>(&p->tw_hi), (size_t)nhi * sizeof(float2)));
        chk(hipMalloc(reinterpret_cast<void**>(&p->tw_lo), (size_t)nlo * sizeof(float2)));
        chk(hipMalloc(&p->chirp_split, (size_t)nfft * (f16_arith(precision) ? 4 : 8)));
        if (e == hipSuccess) chk(launch_stage_twiddles(p->tw_n1, n1, nullptr));
        if (e == hipSuccess) chk(launch_stage_twiddles(p->tw_hi, nhi, nullptr));
        if (e == hipSuccess) chk(launch_partial_twiddles(p->tw_lo, nlo, nfft, nullptr));
    }
    if (kind != POND_INPUT_COMPLEX) {
        p->real_fused = p->log2n1 <= kRealPairMaxLog2N1;
        chk(hipMalloc(reinterpret_cast<void**>(&p->rtab), (size_t)(nfft + 1) * sizeof(float4)));
        if (p->real_fused) {
            chk(hipMalloc(reinterpret_cast<void**>(&p->wk), (size_t)(n1 + n2) * sizeof(float2)));
        } else {
            chk(hipMalloc(reinterpret_cast<void**>(&p->tw4), (size_t)nfft * sizeof(float2)));
            if (e == hipSuccess)
                chk(launch_k2_build_split_tables(p->tw4, nullptr, p->log2n1, p->log2n2, 0.0, p->f0, p->df, nullptr));
        }
    } else if (p->log2m2) {
        // chirp_split, above
    } else if (f16_arith(precision)) {
        chk(hipMalloc(&p->htable, (size_t)nfft * 8));
    } else {
        chk(hipMalloc(&p->table, (size_t)nfft * (precision == POND_FP32 ? sizeof(float2) : sizeof(float4))));
    }
    if (e == hipSuccess) chk(build_filter(p, 0.0));
    // Fold buffers before the tuner (its launches fold too), cleared below.
    p->acc_slots = acc_slots > kDefaultAccSlots ? acc_slots : kDefaultAccSlots;
    chk(hipMalloc(reinterpret_cast<void**>(&p->acc_sum), (size_t)p->acc_slots * nbins * 8));
    chk(hipMalloc(reinterpret_cast<void**>(&p->acc_cnt), (size_t)p->acc_slots * nbins * 8));
    chk(hipMalloc(reinterpret_cast<void**>(&p->part_sum), (size_t)kPartEntries * 8));
    chk(hipMalloc(reinterpret_cast<void**>(&p->part_cnt), (size_t)kPartEntries * 4));
    chk(hipMalloc(reinterpret_cast<void**>(&p->status), 8));
    if (e == hipSuccess && autotune && kind == POND_INPUT_COMPLEX) chk(tune_plan(p));
    chk(hipMalloc(&p->work, (size_t)p->max_batch * (size_t)nfft * p->elem));
    // Float16 arithmetic (packed float16 and matrix-core forms): the power
    // scale is 256 over the measured gain of the plan's float16 arithmetic
    // (the unit-taper table just built).
    if (e == hipSuccess && f16_arith(precision) && kind == POND_INPUT_COMPLEX) {
        HalfCal cal;
        cal.prec = precision;
        cal.log2n1 = p->log2n1;
        cal.log2n2 = p->log2n2;
        cal.tw2 = p->tw2;
        cal.work = p->work;
        cal.max_batch = p->max_batch;
        cal.f16_cols = 2 * p->hop == p->nfft;
        double g = 1.0;
        chk(half_power_gain(
            cal,
            [&](int nb, const void** res) {
                *res = p->work;
                return run_middle(p, p->work, nb, nullptr);
            },
            &g));
        p->half_gain = g;
        p->pscale = (float)(256.0 / g);
    }
    if (e == hipSuccess) chk(hipMemset(p->acc_sum, 0, (size_t)p->acc_slots * nbins * 8));
    if (e == hipSuccess) chk(hipMemset(p->acc_cnt, 0, (size_t)p->acc_slots * nbins * 8));
    if (e == hipSuccess) chk(hipMemset(p->status, 0, 8));
    // The set-up work ran on the null stream; other streams' work is not waited for.
    if (e == hipSuccess) chk(hipStreamSynchronize(nullptr));
    if (e != hipSuccess) {
        g_create_status = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? POND_ENOMEM : POND_EDEVICE;
        free_plan_memory(p);
        delete p;
        (void)hipGetLastError();
        return nullptr;
    }
    g_create_status = POND_OK;
    return p;
}

}  // namespace

namespace pond {
pond_plan* plan_create_slots(double f0_mhz, double bw_mhz, double dm, int64_t nfft, int32_t nbins, double period_s,
                             int32_t precision, int32_t max_batch, int64_t acc_slots) {
    return create_plan(f0_mhz, bw_mhz, dm, nfft, nbins, period_s, precision, max_batch, POND_INPUT_COMPLEX,
                       acc_slots);
}
}  // namespace pond

extern "C" {

pond_plan* pond_plan_create_ex(double f0_mhz, double bw_mhz, double dm, int64_t nfft, int32_t nbins,
                               double period_s, int32_t precision, int32_t max_batch) {
    return create_plan(f0_mhz, bw_mhz, dm, nfft, nbins, period_s, precision, max_batch, POND_INPUT_COMPLEX);
}

pond_plan* pond_real_plan_create(double f0_mhz, double bw_mhz, double dm, int64_t nfft, int32_t nbins,
                                 double period_s, int32_t precision, int32_t max_batch, int32_t sideband) {
    g_create_status = POND_EINVAL;
    if (sideband != POND_LSB && sideband != POND_USB) return nullptr;
    if (nfft < 2 || (nfft & 1)) return nullptr;
    return create_plan(f0_mhz, bw_mhz, dm, nfft / 2, nbins, period_s, precision, max_batch,
                       sideband == POND_LSB ? POND_INPUT_REAL_LSB : POND_INPUT_REAL_USB);
}

pond_plan* pond_plan_create(double f0_mhz, double bw_mhz, double dm, int64_t nfft, int32_t nbins,
                            double period_s) {
    return pond_plan_create_ex(f0_mhz, bw_mhz, dm, nfft, nbins, period_s, POND_FP32, 0);
}

void pond_plan_destroy(pond_plan* p) {
    if (!p) return;
    {
        DeviceGuard g(p->device);
        // Calls on a plan are ordered on the device, so its last stream
        // having passed the last call means all of its work is done.
        (void)hipStreamSynchronize(p->last_stream);
        free_plan_memory(p);
    }
    delete p;
}

int32_t pond_plan_set_taper(pond_plan* p, double alpha) {
    if (!p || !std::isfinite(alpha) || alpha < 0.0 || alpha > 1.0) return POND_EINVAL;
    if (p->sticky) return POND_EDEVICE;
    if (p->samples_in != 0) return POND_EINVAL;
    DeviceGuard g(p->device);
    if (p->last_stream && hipStreamSynchronize(p->last_stream) != hipSuccess) {
        p->sticky = true;
        return POND_EDEVICE;
    }
    hipError_t e = build_filter(p, alpha);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p->sticky = true;
        return POND_EDEVICE;
    }
    p->taper = alpha;
    return POND_OK;
}

int32_t pond_plan_autotune(const pond_plan* p, int32_t* batch, double* ms_per_block, int32_t* default_batch,
                           double* default_ms_per_block, int32_t* from_cache) {
    if (!p || !p->tuned) return POND_EINVAL;
    if (batch) *batch = p->tune.batch;
    if (ms_per_block) *ms_per_block = p->tune.ms_per_block;
    if (default_batch) *default_batch = p->tune.default_batch;
    if (default_ms_per_block) *default_ms_per_block = p->tune.default_ms_per_block;
    if (from_cache) *from_cache = p->tune.from_cache ? 1 : 0;
    return POND_OK;
}

int32_t pond_plan_query(pond_plan* p, pond_info* out) {
    if (!p || !out) return POND_EINVAL;
    std::memset(out, 0, sizeof(*out));
    const int64_t u = p->kind == POND_INPUT_COMPLEX ? 1 : 2;  // samples per element
    out->nfft = u * p->nfft;
    out->n_front = u * p->n_front;
    out->discard = u * p->discard;
    out->hop = u * p->hop;
    out->n1 = (int64_t)1 << p->log2n1;
    out->n2 = (int64_t)1 << p->log2n2;
    out->samples_in = u * p->samples_in;
    out->outputs_done = u * p->blocks_done * p->hop;
    out->max_batch = p->max_batch;
    out->fs_hz = (double)u * p->fs;
    out->input_kind = p->kind;
    out->delta_lo_s = p->delta_lo;
    out->delta_hi_s = p->delta_hi;
    out->inv_pfs = p->inv_pfs;
    out->nbins = p->nbins;
    out->precision = p->precision;
    out->power_gain = p->half_gain;
    if (p->sticky) return POND_EDEVICE;
    DeviceGuard g(p->device);
    uint64_t st = 0;
    hipError_t e = hipStreamSynchronize(p->last_stream);
    if (e == hipSuccess) e = hipMemcpy(&st, p->status, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        p->sticky = true;
        return POND_EDEVICE;
    }
    out->status = (uint32_t)st;
    return POND_OK;
}

int32_t pond_plan_set_timing(pond_plan* p, int32_t enable) {
    if (!p) return POND_EINVAL;
    if (p->sticky) return POND_EDEVICE;
    DeviceGuard g(p->device);
    if (!p->marks.empty()) {
        if (hipStreamSynchronize(p->last_stream) != hipSuccess) {
            p->sticky = true;
            return POND_EDEVICE;
        }
        (void)collect_marks(p);
    }
    for (int k = 0; k < POND_NKERNELS; ++k) {
        p->t_ms[k] = 0;
        p->t_launch[k] = 0;
        p->t_blocks[k] = 0;
    }
    p->timing = enable != 0;
    return POND_OK;
}

int32_t pond_plan_kernel_times(pond_plan* p, pond_kernel_times* out) {
    if (!p || !out) return POND_EINVAL;
    if (p->sticky) return POND_EDEVICE;
    DeviceGuard g(p->device);
    if (hipStreamSynchronize(p->last_stream) != hipSuccess || collect_marks(p) != hipSuccess) {
        p->sticky = true;
        return POND_EDEVICE;
    }
    for (int k = 0; k < POND_NKERNELS; ++k) {
        out->ms[k] = p->t_ms[k];
        out->launches[k] = p->t_launch[k];
        out->blocks[k] = p->t_blocks[k];
    }
    return POND_OK;
}

static int32_t expect(const pond_plan* p, int64_t nsamp, int64_t subint, int64_t* n_profiles,
                      int64_t* n_outputs) {
    if (!p || nsamp < 0 || subint < 0) return POND_EINVAL;
    const int64_t m_before = p->blocks_done * p->hop;
    const int64_t s_open = subint > 0 ? m_before / subint : 0;
    int64_t np = 0, no = 0;
    if (nsamp == 0) {
        const int64_t in_open = subint > 0 ? m_before - s_open * subint : m_before;
        np = in_open > 0 ? 1 : 0;
    } else {
        const int64_t m_after = n_blocks_for(p->samples_in + nsamp, p->nfft, p->hop) * p->hop;
        no = m_after - m_before;
        np = subint > 0 ? m_after / subint - s_open : 0;
    }
    if (n_profiles) *n_profiles = np;
    if (n_outputs) *n_outputs = no;
    return POND_OK;
}

int32_t pond_plan_expect(const pond_plan* p, int64_t nsamp, int64_t subint, int64_t* n_profiles,
                         int64_t* n_outputs) {
    if (!p || p->kind != POND_INPUT_COMPLEX) return POND_EINVAL;
    return expect(p, nsamp, subint, n_profiles, n_outputs);
}

int32_t pond_real_expect(const pond_plan* p, int64_t nsamp, int64_t subint_nsamp, int64_t* n_profiles,
                         int64_t* n_outputs) {
    if (!p || p->kind == POND_INPUT_COMPLEX || (nsamp & 1) || (subint_nsamp & 1)) return POND_EINVAL;
    int64_t no = 0;
    const int32_t r = expect(p, nsamp / 2, subint_nsamp / 2, n_profiles, &no);
    if (r == POND_OK && n_outputs) *n_outputs = 2 * no;
    return r;
}

// nsamp, subint and decim in elements of the plan (complex samples, or
// pairs of real samples on the real path).
static int64_t run_call(pond_plan* p, const int8_t* iq, int64_t nsamp, int64_t subint, float* profiles,
                        int64_t max_profiles, int32_t decim, float* series, int64_t series_cap,
                        int64_t* n_series_out, bool want_series, void* stream_ptr) {
    if (!p) return POND_EINVAL;
    if (p->sticky) return POND_EDEVICE;
    if (n_series_out) *n_series_out = 0;
    const bool flush = (iq == nullptr && nsamp == 0);
    if (!flush) {
        if (nsamp < 0) return POND_EINVAL;
        if (nsamp > 0 && (iq == nullptr || (reinterpret_cast<uintptr_t>(iq) & (uintptr_t)(p->bpe - 1))))
            return POND_EINVAL;
    }
    if (subint < 0 || max_profiles < 0) return POND_EINVAL;
    if (p->subint >= 0 && subint != p->subint) return POND_EINVAL;
    if (decim <= 0) decim = (int32_t)std::lround(p->bw);  // 1 us (bw_mhz samples)
    if (decim != 1 && decim != 2 && decim != 4 && decim != 8 && decim != 16) return POND_EINVAL;
    if (want_series && series_cap < 0) return POND_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_ptr);

    const int64_t hop = p->hop;
    const int32_t nbins = p->nbins;
    const int64_t m_before = p->blocks_done * hop;
    const int64_t s_open = subint > 0 ? m_before / subint : 0;

    DeviceGuard guard(p->device);
    if (!guard.ok) {
        p->sticky = true;
        return POND_EDEVICE;
    }
    hipError_t e = hipSuccess;
    auto fail = [&](hipError_t x) -> int64_t {
        (void)x;
        (void)hipGetLastError();
        p->sticky = true;
        return POND_EDEVICE;
    };
    // Launch through `timed` so that, with timing on, each kernel is
    // bracketed by events on the call's stream.
    auto timed = [&](int kernel, int64_t blocks, auto&& launch) -> hipError_t {
        if (!p->timing) return launch();
        hipEvent_t ea = take_event(p), eb = take_event(p);
        if (!ea || !eb) return hipErrorOutOfMemory;
        hipError_t r = hipEventRecord(ea, stream);
        if (r == hipSuccess) r = launch();
        if (r == hipSuccess) r = hipEventRecord(eb, stream);
        p->marks.push_back({kernel, blocks, ea, eb});
        return r;
    };

    if (flush) {
        const int64_t in_open = subint > 0 ? m_before - s_open * subint : m_before;
        const int64_t nprof = in_open > 0 ? 1 : 0;
        if (nprof > max_profiles || (nprof && !profiles)) return POND_EINVAL;
        if (nprof) {
            e = timed(4, 0, [&] { return launch_fold_finalize(p->acc_sum, p->acc_cnt, nbins, 1, 1, profiles, stream); });
            if (e != hipSuccess) return fail(e);
        }
        e = launch_zero_u64(p->status, 1, stream);
        if (e != hipSuccess) return fail(e);
        p->samples_in = 0;
        p->blocks_done = 0;
        p->tail_start = 0;
        p->subint = -1;
        p->last_stream = stream;
        return nprof;
    }

    const int64_t total = p->samples_in + nsamp;
    const int64_t nb_total = n_blocks_for(total, p->nfft, hop);
    const int64_t m_after = nb_total * hop;
    int64_t n_complete = 0, n_touched = 0;
    if (subint > 0) {
        n_complete = m_after / subint - s_open;
        n_touched = m_after > m_before ? (m_after - 1) / subint - s_open + 1 : 0;
    } else {
        n_touched = m_after > m_before ? 1 : 0;
    }
    if (n_complete > max_profiles || (n_complete > 0 && !profiles)) return POND_EINVAL;
    const int64_t groups = (m_after - m_before) / decim;
    if (want_series && (groups > series_cap || (groups > 0 && !series))) return POND_EINVAL;

    // Grow the accumulator ring if this call touches more sub-integrations
    // than it holds: never while the stream is being captured into a graph
    // (the graph would own the new memory), otherwise with plain
    // allocations once the plan's work has finished.  Slot 0 (the open
    // sub-integration) carries over; the rest start at zero.
    if (n_touched > p->acc_slots) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return fail(hipErrorUnknown);
        if (cs != hipStreamCaptureStatusNone) return POND_EINVAL;
        int64_t slots = p->acc_slots;
        while (slots < n_touched) slots *= 2;
        const size_t bytes = (size_t)slots * nbins * 8;
        e = hipStreamSynchronize(stream);
        if (e == hipSuccess && p->last_stream != stream) e = hipStreamSynchronize(p->last_stream);
        if (e != hipSuccess) return fail(e);
        uint64_t *ns = nullptr, *nc = nullptr;
        e = hipMalloc(reinterpret_cast<void**>(&ns), bytes);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&nc), bytes);
        if (e != hipSuccess) {
            if (ns) (void)hipFree(ns);
            (void)hipGetLastError();
            return POND_ENOMEM;
        }
        e = hipMemset(ns, 0, bytes);
        if (e == hipSuccess) e = hipMemset(nc, 0, bytes);
        if (e == hipSuccess) e = hipMemcpy(ns, p->acc_sum, (size_t)nbins * 8, hipMemcpyDeviceToDevice);
        if (e == hipSuccess) e = hipMemcpy(nc, p->acc_cnt, (size_t)nbins * 8, hipMemcpyDeviceToDevice);
        if (e != hipSuccess) {
            (void)hipFree(ns);
            (void)hipFree(nc);
            return fail(e);
        }
        (void)hipFree(p->acc_sum);
        (void)hipFree(p->acc_cnt);
        p->acc_sum = ns;
        p->acc_cnt = nc;
        p->acc_slots = slots;
    }

    const int64_t n1 = (int64_t)1 << p->log2n1;
    const int n2log = p->log2n2;
    // Power-of-two pass scales, 1/n overall: the forward column pass is
    // normalised (1/n2), the row pass scales by 1/n1, the inverse column
    // pass by 1, so every stored intermediate stays within the input range.
    const float k1_scale = std::ldexp(1.0f, -n2log);
    const float k2_scale = std::ldexp(1.0f, -p->log2n1);
    const float k3_scale = 1.0f;

    int64_t b = p->blocks_done;
    ReduceQueue rq;
    int64_t rq_blocks = 0;  // blocks whose fold partials are queued
    while (b < nb_total) {
        int64_t nb = nb_total - b < p->max_batch ? nb_total - b : p->max_batch;
        int64_t s_lo = 0, nsub = 1;
        for (;;) {
            if (subint > 0) {
                s_lo = (b * hop) / subint;
                const int64_t s_hi = ((b + nb) * hop - 1) / subint;
                nsub = s_hi - s_lo + 1;
            }
            if (nsub * nbins <= p->hist_cap || nb == 1) break;
            nb = (nb + 1) / 2;
        }
        const int64_t entries = nsub * nbins;
        const bool global_mode = entries > p->hist_cap;

        K1Args a1;
        a1.tail = p->tail[p->tcur];
        a1.tail_start = p->tail_start;
        a1.in = iq;
        a1.in_start = p->samples_in;
        a1.hop = hop;
        a1.block0 = b;
        a1.nblocks = (int32_t)nb;
        a1.log2n1 = p->log2n1;
        a1.work = p->work;
        a1.tw2 = p->tw2;
        a1.scale = k1_scale;
        a1.f16_cols = 2 * hop == p->nfft;
        const bool real = p->kind != POND_INPUT_COMPLEX;
        e = timed(0, nb, [&] {
            return real ? launch_k1_aip(p->precision, n2log, a1, stream) : launch_k1(p->precision, n2log, a1, stream);
        });
        if (e != hipSuccess) return fail(e);

        K2Args a2{};
        a2.work = p->work;
        a2.nblocks = (int32_t)nb;
        a2.log2n2 = n2log;
        a2.tw1 = p->tw1;
        a2.table = p->table;
        a2.htable = p->htable;
        a2.scale = k2_scale;
        if (real && p->real_fused) {
            RealPairArgs rp{p->work, (int32_t)nb, n2log, p->tw1, p->rtab, p->wk, k2_scale};
            e = timed(1, nb, [&] { return launch_real_pair(p->precision, p->log2n1, rp, stream); });
        } else if (real) {
            // Forward rows, the real split with the filter (in place), then
            // the inverse rows with no further filter: one timed middle pass.
            a2.tw4 = p->tw4;
            a2.in = p->work;
            a2.out = p->work;
            a2.chirp = nullptr;
            RealSplitArgs rs{p->work, (int32_t)nb, p->log2n1, n2log, p->rtab};
            e = timed(1, nb, [&] {
                hipError_t r = launch_k2(p->precision, kRowFwd, p->log2n1, a2, stream);
                if (r == hipSuccess) r = launch_real_split(p->precision, rs, stream);
                K2Args ai = a2;
                ai.scale = 1.0f;
                if (r == hipSuccess) r = launch_k2(p->precision, kRowInvPlain, p->log2n1, ai, stream);
                return r;
            });
        } else {
            e = timed(1, nb, [&] { return run_middle(p, p->work, (int)nb, stream); });
        }
        if (e != hipSuccess) return fail(e);

        K3Args a3;
        a3.work = p->work;
        a3.nblocks = (int32_t)nb;
        a3.log2n1 = p->log2n1;
        a3.hop = hop;
        a3.n_front = p->n_front;
        a3.block0 = b;
        a3.tw2 = p->tw2;
        a3.scale = k3_scale;
        // The packed-float16 middle pass leaves 1/16 of the value (its
        // twiddle table carries the first stage's 1/16): power x 256.
        a3.pscale = p->pscale;
        a3.series = want_series ? series : nullptr;
        a3.series_base = m_before / decim;
        a3.decim = decim;
        a3.nbins = nbins;
        a3.inv_pfs = p->inv_pfs;
        a3.subint = subint;
        a3.s_base = s_lo;
        a3.entries = (int32_t)entries;
        a3.global_mode = global_mode ? 1 : 0;
        a3.acc_sum = p->acc_sum;
        a3.acc_cnt = p->acc_cnt;
        a3.acc_s0 = s_open;
        a3.status = reinterpret_cast<uint32_t*>(p->status);
        const size_t dyn = global_mode ? 0 : (size_t)entries * 12;
        const int grid = k3_grid(n2log, p->precision, dyn, nb * (n1 / 16), entries, global_mode);
        // Partials in the next quarter of the buffers with a queued reduction
        // when they fit there; otherwise the whole buffers, reduced at once
        // (after the queued reductions, which read them).
        const bool deferred = !global_mode && (int64_t)grid * entries <= kPartRegion;
        if (!global_mode && !deferred && rq.pending()) {
            e = timed(3, rq_blocks, [&] { return rq.flush(stream); });
            rq_blocks = 0;
            if (e != hipSuccess) return fail(e);
        }
        a3.part_sum = deferred ? rq.part_sum(p->part_sum) : p->part_sum;
        a3.part_cnt = deferred ? rq.part_cnt(p->part_cnt) : p->part_cnt;
        e = timed(2, nb, [&] {
            return real ? launch_k3_real(p->precision, n2log, a3, (int)grid, dyn, stream)
                        : launch_k3(p->precision, n2log, a3, (int)grid, dyn, stream);
        });
        if (e != hipSuccess) return fail(e);
        if (!global_mode) {
            const ReduceJob job{a3.part_sum, a3.part_cnt, p->acc_sum, p->acc_cnt, (s_lo - s_open) * nbins,
                                (int32_t)grid, (int32_t)entries};
            if (deferred && !rq.push_flushes()) {
                e = rq.push(job, stream);  // queued: nothing launched yet
                rq_blocks += nb;
            } else if (deferred) {
                e = timed(3, rq_blocks + nb, [&] { return rq.push(job, stream); });
                rq_blocks = 0;
            } else {
                e = timed(3, nb, [&] {
                    ReduceBatch one;
                    one.job[0] = job;
                    one.n = 1;
                    return launch_fold_reduce_batch(one, stream);
                });
            }
            if (e != hipSuccess) return fail(e);
        }
        b += nb;
    }
    if (rq.pending()) {
        e = timed(3, rq_blocks, [&] { return rq.flush(stream); });
        if (e != hipSuccess) return fail(e);
    }

    if (n_complete > 0) {
        e = timed(4, 0, [&] {
            return launch_fold_finalize(p->acc_sum, p->acc_cnt, nbins, (int)n_complete, (int)n_touched, profiles,
                                        stream);
        });
        if (e != hipSuccess) return fail(e);
    }

    // Keep the samples future blocks need: absolute [nb_total * hop, total).
    const int64_t new_start = nb_total * hop;
    int8_t* dst = p->tail[p->tcur ^ 1];
    int64_t filled = 0;
    if (p->samples_in > new_start) {
        const int64_t from = new_start > p->tail_start ? new_start : p->tail_start;
        const int64_t cnt = p->samples_in - from;
        if (cnt > 0) {
            e = hipMemcpyAsync(dst, p->tail[p->tcur] + p->bpe * (from - p->tail_start), (size_t)cnt * p->bpe,
                               hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return fail(e);
            filled = cnt;
        }
    }
    {
        const int64_t from = new_start > p->samples_in ? new_start : p->samples_in;
        const int64_t cnt = total - from;
        if (cnt > 0) {
            e = hipMemcpyAsync(dst + p->bpe * filled, iq + p->bpe * (from - p->samples_in), (size_t)cnt * p->bpe,
                               hipMemcpyDeviceToDevice, stream);
            if (e != hipSuccess) return fail(e);
        }
    }
    p->tcur ^= 1;
    p->tail_start = new_start;
    p->samples_in = total;
    p->blocks_done = nb_total;
    p->subint = subint;
    p->last_stream = stream;
    if (n_series_out) *n_series_out = want_series ? groups : 0;
    return n_complete;
}

int64_t pond_dedisperse_fold(pond_plan* p, const int8_t* iq, int64_t nsamp, int64_t subint_nsamp, float* profiles,
                             int64_t max_profiles, void* hip_stream) {
    if (p && p->kind != POND_INPUT_COMPLEX) return POND_EINVAL;
    return run_call(p, iq, nsamp, subint_nsamp, profiles, max_profiles, 16, nullptr, 0, nullptr, false, hip_stream);
}

int64_t pond_dedisperse_series(pond_plan* p, const int8_t* iq, int64_t nsamp, int64_t subint_nsamp, float* profiles,
                               int64_t max_profiles, int32_t decim, float* series, int64_t series_cap,
                               int64_t* n_series_out, void* hip_stream) {
    if (p && p->kind != POND_INPUT_COMPLEX) return POND_EINVAL;
    return run_call(p, iq, nsamp, subint_nsamp, profiles, max_profiles, decim, series, series_cap, n_series_out, true,
                    hip_stream);
}

int64_t pond_real_dedisperse(pond_plan* p, const int8_t* raw, int64_t nsamp, int64_t subint_nsamp, float* profiles,
                             int64_t max_profiles, int32_t decim, float* series, int64_t series_cap,
                             int64_t* n_series_out, void* hip_stream) {
    if (n_series_out) *n_series_out = 0;
    if (!p || p->kind == POND_INPUT_COMPLEX) return POND_EINVAL;
    if ((nsamp & 1) || (subint_nsamp & 1)) return POND_EINVAL;
    if (decim <= 0) decim = (int32_t)std::lround(2.0 * p->bw);  // 1 us of real samples
    if (decim != 2 && decim != 4 && decim != 8 && decim != 16 && decim != 32) return POND_EINVAL;
    return run_call(p, raw, nsamp / 2, subint_nsamp / 2, profiles, max_profiles, decim / 2, series, series_cap,
                    n_series_out, series != nullptr, hip_stream);
}

}  // extern "C"
