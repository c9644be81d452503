// Internal interface between the host runtime (pond_api.cpp) and the HIP
// kernels (pond_k1/k2/k3/fold/real/aid_kernels.hip).  Plain structs of
// pointers and sizes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

struct pond_plan;

namespace pond {

// Fixed-point scale of the fold accumulators: a power p is accumulated as
// round(p * 2^16) in an unsigned 64-bit integer, so sums are exact and
// independent of the order in which workgroups add them.
constexpr double kFoldScale = 65536.0;
constexpr double kFoldRangeLimit = 1099511627776.0;  // 2^40: flag larger single contributions

enum Precision { kFp32 = 0, kMixed = 1, kMixedValu = 2, kHalf = 3, kBf16 = 4 };
// Forms whose arithmetic is packed float16 (float16 tables, measured power gain).
constexpr bool f16_arith(int prec) { return prec == kHalf || prec == kMixed; }

// K1: int8 unpack + forward column FFTs (length n2, stride n1).
struct K1Args {
    const int8_t* tail;     // device ring holding absolute samples [tail_start, in_start)
    int64_t tail_start;
    const int8_t* in;       // this call's samples, absolute [in_start, ...)
    int64_t in_start;
    int64_t hop;
    int64_t block0;         // absolute index of the launch's first block
    int32_t nblocks;
    int32_t log2n1;
    void* work;             // [nblocks][n2][n1] complex, storage type of the form
    const float2* tw2;      // exp(-2 pi i t / n2), t < n2
    float scale;            // power-of-two output scale
    int32_t chain = 1;      // blocks per workgroup (set by launch_k1)
    // matrix-core form: 1 = the packed-float16 column pass instead (a
    // plan's choice where its blocks overlap by half, also for its
    // calibration, so that every launch of the plan gives the same bits)
    int32_t f16_cols = 0;
};

// K2: four-step twiddle, forward row FFT (length n1), chirp, inverse row
// FFT, conjugate twiddle.
// kRowInvPlain: kRowInv with no filter (float32 arithmetic forms; the real
// input path's longest rows, filtered by real_split before).
// kRowChirp: forward row FFT, chirp, inverse row FFT, no twiddles (the
// sub-rows of the split middle pass, rows of 2^kSplitLog2M1; chirp table in
// their order).
enum RowMode { kRowFull = 0, kRowFwd = 1, kRowInv = 2, kRowInvPlain = 3, kRowChirp = 4 };
constexpr int kMaxLog2RowN1 = 14;  // longest row one workgroup transforms in LDS
constexpr int kSplitLog2M1 = 13;   // sub-row length of the split middle pass

struct K2Args {
    void* work;             // rows, in place (kRowFull, kRowFwd)
    const void* in;         // spectrum rows (kRowInv)
    void* out;              // result rows (kRowInv)
    int32_t nblocks;
    int32_t log2n2;
    const float2* tw1;      // exp(-2 pi i t / n1), t < n1
    const void* table;      // kRowFull, float32 arithmetic: [n2][n1] chirp (float2, float32 storage) or
                            // twiddle and chirp (float4, float16 / bfloat16 storage)
    const float2* tw4;      // kRowFwd, kRowInv: [n2][n1] four-step twiddle
    const float2* chirp;    // kRowChirp: split middle pass chirp (float32 forms)
    float scale;            // power-of-two scale applied on output (float32 arithmetic)
    const void* htable;     // packed float16, kRowFull: [n2][n1] 4 halves (twiddle / 16, chirp * 2^-rem)
    const void* htw4;       // packed float16, split modes: [n2][n1] twiddle / 16
    const void* hchirp;     // packed float16, kRowChirp: split middle pass chirp
    const double* geo;      // kRowInv: [n2][n1] turns per unit DM of each bin (shared by the trials)
    double dm;              // kRowInv: the trial's DM (chirp exp(-2 pi i frac(dm geo)))
};

// Split middle pass, for rows longer than one workgroup's LDS holds (n1 =
// m2 * m1, m1 = 2^kSplitLog2M1, m2 = 2..16): the row transform of length n1
// is itself done in four steps.  Forward: for each row k2 and column c < m1,
// the m2 values at c + m1 i are multiplied by the block twiddle
// exp(-2 pi i k2 (c + m1 i) / N), transformed (length m2), multiplied by
// exp(-2 pi i c k / n1) and stored at c + m1 k (sub-row k).  Inverse: the
// same steps conjugated, in reverse order.  Float32 arithmetic for every
// storage type.
struct SplitColArgs {
    void* work;             // [nblocks][n2][n1], in place
    int32_t nblocks;
    int32_t log2n1, log2n2;
    const float2* tw_n1;    // exp(-2 pi i t / n1), t < n1
    const float2* tw_hi;    // exp(-2 pi i t 2^log2s / N), t < N / 2^log2s
    const float2* tw_lo;    // exp(-2 pi i t / N), t < 2^log2s
    int32_t log2s;
    float scale;            // applied to every output
};
hipError_t launch_split_cols(int prec, bool inverse, const SplitColArgs& a, hipStream_t s);
// Chirp tables of the split middle pass, in sub-row order: entry (k2 m2 + k)
// m1 + c' holds the inverse ISM response at frequency k2 + n2 (k + m2 c').
// Float32 (float2) or packed float16 (times 2^-half_row_rem(kSplitLog2M1)).
hipError_t launch_build_split_chirp(void* tab, bool f16, int log2n1, int log2n2, double chirp_a, double f0, double df,
                                    double taper, hipStream_t s);
// w[t] = exp(-2 pi i t / n) for t < count (count <= n), float64 sine/cosine
// rounded to float32.
hipError_t launch_partial_twiddles(float2* w, int64_t count, int64_t n, hipStream_t s);

// K3: inverse column FFTs, detection, decimation, fold partials.
struct K3Args {
    const void* work;
    int32_t nblocks;
    int32_t log2n1;
    int64_t hop;
    int64_t n_front;
    int64_t block0;
    const float2* tw2;
    float scale;            // power-of-two scale of the inverse column output (float32 arithmetic)
    float pscale;           // scale of the detected power (packed float16: 256, else 1)
    // series
    float* series;          // NULL: no series this call
    int64_t series_base;    // group index (in units of decim) of series[0]
    int32_t decim;
    // fold
    int32_t nbins;
    double inv_pfs;
    int64_t subint;         // outputs per sub-integration, 0 = one open-ended
    int64_t s_base;         // first sub-integration this launch can touch
    int32_t entries;        // (sub-integrations spanned) * nbins
    int32_t global_mode;    // 1: atomics straight into acc (histogram too big for LDS)
    uint64_t* part_sum;     // [grid][entries]
    uint32_t* part_cnt;
    uint64_t* acc_sum;      // global accumulators, slot-major [slot][nbins]
    uint64_t* acc_cnt;
    int64_t acc_s0;         // sub-integration held by accumulator slot 0
    uint32_t* status;
};

// Real input path: split of the packed spectrum into the real transform's
// bins, filter, recombination (see real_split).
struct RealSplitArgs {
    void* data;             // [nblocks][n2][n1] spectrum of the packed block (/N), replaced in place
                            // by the spectrum of the filtered packed block
    int32_t nblocks;
    int32_t log2n1, log2n2;
    const float4* tab;      // [N + 1] (W^k, M[k]) of the bin at each position, then bin N
};
// Real input path, fused middle pass (rows up to 2^13; see k2_real_pair).
struct RealPairArgs {
    void* data;             // [nblocks][n2][n1], forward column pass output, replaced in place
    int32_t nblocks;
    int32_t log2n2;
    const float2* tw1;      // exp(-2 pi i t / n1), t < n1
    const float4* tab;      // [N + 1] (four-step twiddle, M[k]) per block position; tab[N].z = M[N]
    const float2* wk;       // [n2 + n1] exp(-i pi k2 / N), then exp(-i pi k1 / n1)
    float scale;            // power-of-two scale of the forward row output
};
constexpr int kRealPairMaxLog2N1 = 13;
hipError_t launch_real_pair(int prec, int log2n1, const RealPairArgs& a, hipStream_t s);
hipError_t launch_real_build_pair_table(float4* tab, float2* wk, int log2n1, int log2n2, double chirp_a, double f0,
                                        double bw, int lsb, double taper, hipStream_t s);
hipError_t launch_k1_aip(int prec, int log2n2, const K1Args& a, hipStream_t s);
hipError_t launch_real_split(int prec, const RealSplitArgs& a, hipStream_t s);
hipError_t launch_k3_real(int prec, int log2n2, const K3Args& a, int grid, size_t dyn, hipStream_t s);
hipError_t launch_real_build_table(float4* tab, int log2n1, int log2n2, double chirp_a, double f0, double bw,
                                   int lsb, double taper, hipStream_t s);

// Incoherent (AID) mode: filterbank, then channel shift-and-sum and fold.
struct AidArgs {
    const int8_t* iq;       // nspec * nint * nchan complex int8 samples
    int64_t nspec;          // integrated spectra (output times of the filterbank)
    int32_t nint;           // spectra summed per output time
    int32_t nchan;          // channels (FFT length)
    const float2* tw;       // exp(-2 pi i t / nchan), t < nchan
    float* F;               // [nchan][nspec] integrated powers, channel-major
    const int32_t* dd;      // [nchan] delay minus the smallest delay (integrated samples)
    int32_t d_min;          // smallest delay
    int64_t nout;           // dedispersed outputs
    float* series;          // [nout] or NULL
    int32_t nbins;
    double inv_pfs;         // 1 / (period * fs)
    uint64_t* part_sum;     // [grid][nbins]
    uint32_t* part_cnt;
    uint32_t* status;
};
hipError_t launch_aid_filterbank(int log2c, const AidArgs& a, hipStream_t s);
hipError_t launch_aid_dedisperse_fold(const AidArgs& a, int grid, hipStream_t s);

// Launchers; each returns the HIP error of the launch.
hipError_t launch_k1(int prec, int log2n2, const K1Args& a, hipStream_t s);
hipError_t launch_k2(int prec, int mode, int log2n1, const K2Args& a, hipStream_t s);
hipError_t launch_k3(int prec, int log2n2, const K3Args& a, int grid, size_t dyn_lds, hipStream_t s);
hipError_t launch_fold_reduce(const uint64_t* part_sum, const uint32_t* part_cnt, int nparts, int entries,
                              uint64_t* acc_sum, uint64_t* acc_cnt, int64_t acc_off, hipStream_t s);
hipError_t launch_fold_finalize(uint64_t* acc_sum, uint64_t* acc_cnt, int nbins, int n_complete, int n_touched,
                                float* profiles, hipStream_t s);
hipError_t launch_copy_u128(void* dst, const void* src, int64_t n16, hipStream_t s);
hipError_t launch_zero_u64(uint64_t* p, int64_t n, hipStream_t s);
// n words of pseudo-random bits (splitmix64 of index and seed): timing input.
hipError_t launch_fill_noise_u64(uint64_t* p, int64_t n, uint64_t seed, hipStream_t s);
// w[t] = exp(-2 pi i t / n) for t < n, float64 sine/cosine rounded to float32.
hipError_t launch_stage_twiddles(float2* w, int64_t n, hipStream_t s);
// twiddle: float4 entries (twiddle, chirp), else float2 (chirp).
hipError_t launch_k2_build_table(void* tab, bool twiddle, int log2n1, int log2n2, double chirp_a, double f0,
                                 double df, double taper, hipStream_t s);
hipError_t launch_k2_build_split_tables(float2* tw, float2* chirp, int log2n1, int log2n2, double chirp_a, double f0,
                                        double df, hipStream_t s);

hipError_t launch_k2_build_table_h(void* tab, int log2n1, int log2n2, double chirp_a, double f0, double df,
                                   double taper, hipStream_t s);
hipError_t launch_k2_build_split_tables_h(void* tw, void* chirp, int log2n1, int log2n2, double chirp_a, double f0,
                                          double df, hipStream_t s);
// geo[i] = f^2 / (2.41e-10 f0^2 (f0 + f)), the chirp's turns per unit DM at
// the bin f = k df of entry i = k2 n1 + k1 (k = k2 + n2 k1, k >= n/2 taken
// as k - n), float64.
hipError_t launch_build_dm_geometry(double* geo, int log2n1, int log2n2, double f0, double df, hipStream_t s);
// Packed-float16 row transforms apply 2^-half_row_rem(log2n1) of their
// 1/n1 normalisation after the stages (the rest is spread over them).
constexpr int half_row_rem(int log2n1) {
    return log2n1 - 4 * ((log2n1 / 4 + (log2n1 % 4 ? 1 : 0) + 1) / 2);
}

hipError_t launch_fold_profiles(const uint64_t* acc_sum, const uint64_t* acc_cnt, int64_t n, float* profiles,
                                hipStream_t s);

constexpr int64_t kPartEntries = 1 << 21;  // per-workgroup fold partials: grid * entries <= this

// Deferred fold reductions.  A K3 launch whose partials fit in a quarter
// of the partial buffers writes them to the next free quarter and queues
// its reduction; the queued reductions run as one launch when four are
// pending, before a launch that needs the whole buffer, and before anything
// reads the accumulators (integer sums: the order does not change a bit).
constexpr int kReduceSlots = 4;
constexpr int64_t kPartRegion = kPartEntries / kReduceSlots;
struct ReduceJob {
    const uint64_t* part_sum;  // nparts x entries partials, part-major
    const uint32_t* part_cnt;
    uint64_t* acc_sum;  // accumulators; entry i goes to acc_off + i
    uint64_t* acc_cnt;
    int64_t acc_off;
    int32_t nparts;
    int32_t entries;
};
struct ReduceBatch {
    ReduceJob job[kReduceSlots];
    int32_t n = 0;
};
hipError_t launch_fold_reduce_batch(const ReduceBatch& b, hipStream_t s);
class ReduceQueue {
   public:
    // partial buffers of the next queued launch (a quarter of the full ones)
    uint64_t* part_sum(uint64_t* full) const { return full + (int64_t)b_.n * kPartRegion; }
    uint32_t* part_cnt(uint32_t* full) const { return full + (int64_t)b_.n * kPartRegion; }
    bool pending() const { return b_.n > 0; }
    bool push_flushes() const { return b_.n + 1 == kReduceSlots; }
    hipError_t push(const ReduceJob& j, hipStream_t s) {
        b_.job[b_.n++] = j;
        return b_.n == kReduceSlots ? flush(s) : hipSuccess;
    }
    hipError_t flush(hipStream_t s) {
        if (b_.n == 0) return hipSuccess;
        const hipError_t e = launch_fold_reduce_batch(b_, s);
        b_.n = 0;
        return e;
    }

   private:
    ReduceBatch b_;
};
// Workgroups of a K3 launch: enough to fill the chip at the occupancy the
// LDS allows, at most one per item, a multiple of 8, and within the
// partial-histogram budget.
int k3_grid(int log2n2, int prec, size_t dyn_lds, int64_t items, int64_t entries, bool global_mode,
            int64_t part_entries = kPartEntries);
constexpr int64_t kHistCapMax = 8192;      // fold histogram entries held in LDS
constexpr size_t kLdsBytes = 160 * 1024;   // gfx950 LDS per workgroup
int64_t hist_capacity(int log2n2, int prec);

// Device bytes pond_plan_create_ex allocates for these arguments (with an
// accumulator ring of acc_slots sub-integrations, at least 4), and the
// blocks per launch it picks (max_batch <= 0: the default).
int64_t plan_footprint(int64_t nfft, int32_t nbins, int32_t precision, int32_t max_batch, int64_t acc_slots);
// pond_plan_create_ex with an accumulator ring of at least acc_slots
// sub-integrations from the start (callers that know their largest call).
pond_plan* plan_create_slots(double f0_mhz, double bw_mhz, double dm, int64_t nfft, int32_t nbins, double period_s,
                             int32_t precision, int32_t max_batch, int64_t acc_slots);
int plan_max_batch(int64_t nfft, int32_t precision, int32_t max_batch);
// Power gain of a packed-float16 path, measured.  White int8 noise of at
// least 2^22 samples, cut into blocks of n = 2^(log2n1 + log2n2), is pushed
// through K1, the caller's middle pass and K3 with the whole block kept
// (n_front 0, hop n) and detected at scale 256; since the transform pair and
// every filter the path applies are all-pass, the exact output power is the
// input power (Parseval), and the ratio of the two is the gain of the
// float16 arithmetic (rounded twiddles, constants, table entries and
// roundings), to about 1e-6.  middle(nb, &result) runs the middle pass on nb
// blocks in `work` and names the buffer K3 reads.  Synchronous; runs on the
// null stream.
struct HalfCal {
    int prec = kHalf;             // kHalf or kMixed (float16 arithmetic forms)
    int log2n1 = 0, log2n2 = 0;
    const float2* tw2 = nullptr;  // exp(-2 pi i t / n2)
    void* work = nullptr;         // max_batch blocks of float16 pairs
    int max_batch = 1;
    int f16_cols = 0;             // the plan's K1Args::f16_cols
};
hipError_t half_power_gain(const HalfCal& c, const std::function<hipError_t(int, const void**)>& middle,
                           double* gain);

// Static LDS bytes of the K3 tile for a column length 2^log2n2.
size_t k3_static_lds(int log2n2, int prec);
// Threads per workgroup of each kernel.
int k1_threads(int log2n2);
int k2_threads(int log2n1);
int k3_threads(int log2n2);

}  // namespace pond
