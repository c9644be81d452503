// The whole dedispersion + fold of one resident segment with no device
// allocation: every buffer the kernels need beyond the caller's input and
// outputs (stage twiddles, the middle-pass table, the block work area, the
// per-workgroup fold partials, the accumulators and the status word) lives
// in one file-scope device array, `scratch`, which each GPU the library
// runs on holds until the process ends.  For callers that cannot allocate
// (graph capture, tight serving loops).  Every call on a GPU uses that GPU's
// one array, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/pond.h"
#include "pond_internal.hpp"

using namespace pond;

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // POND_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == (size_t)POND_NOALLOC_SCRATCH_BYTES, "header and library agree");

static __device__ __align__(256) char scratch[kScratchBytes];

// Device address of `scratch` per device (the array's name on the host is
// only a stand-in), looked up once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

hipError_t scratch_ptr(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

constexpr int64_t kMaxNfft = (int64_t)1 << POND_NOALLOC_MAX_LOG2N;
constexpr int32_t kMaxBins = POND_NOALLOC_MAX_BINS;
constexpr int64_t kPartCap = (int64_t)1 << 19;  // per-workgroup partial entries

int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int64_t pond_dedisperse_segment_noalloc(double f0_mhz, double bw_mhz, double dm, int64_t nfft, int32_t nbins,
                                        double period_s, int32_t precision, const int8_t* iq, int64_t nsamp,
                                        int32_t decim, float* profile, float* series, int64_t series_cap,
                                        void* hip_stream) {
    if (precision != POND_FP32 && precision != POND_MIXED_VALU) return POND_EINVAL;
    if (nfft <= 0 || (nfft & (nfft - 1)) || nfft < 1024 || nfft > kMaxNfft) return POND_EINVAL;
    if (nbins < 1 || nbins > kMaxBins || nsamp < 0 || (nsamp > 0 && !iq) || !profile) return POND_EINVAL;
    if ((reinterpret_cast<uintptr_t>(iq) & 1u) || !std::isfinite(period_s)) return POND_EINVAL;
    if (decim <= 0) decim = (int32_t)std::lround(bw_mhz);
    if (decim != 1 && decim != 2 && decim != 4 && decim != 8 && decim != 16) return POND_EINVAL;
    int64_t n_front = 0, discard = 0, hop = 0;
    if (pond_geometry(f0_mhz, bw_mhz, dm, nfft, &n_front, &discard, &hop) != POND_OK) return POND_EINVAL;
    const double fs = bw_mhz * 1e6;
    if (!(period_s > 0) || !(period_s * fs >= 1.0)) return POND_EINVAL;
    const int64_t nb_total = nsamp < nfft ? 0 : (nsamp - nfft) / hop + 1;
    const int64_t n_out = nb_total * hop;
    if (n_out / decim > series_cap || (n_out >= decim && !series)) return POND_EINVAL;

    const int log2n = ilog2(nfft);
    const int log2n2 = log2n / 2 < 10 ? log2n / 2 : 10;
    const int log2n1 = log2n - log2n2;
    const int64_t n1 = (int64_t)1 << log2n1, n2 = (int64_t)1 << log2n2;
    const size_t elem = precision == POND_FP32 ? 8 : 4;

    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return POND_EDEVICE;
    char* base = nullptr;
    if (scratch_ptr(dev, &base) != hipSuccess) {
        (void)hipGetLastError();
        return POND_EDEVICE;
    }
    // Layout of the scratch array.
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = base + off;
        off += align256(bytes);
        return q;
    };
    float2* tw1 = reinterpret_cast<float2*>(take((size_t)n1 * sizeof(float2)));
    float2* tw2 = reinterpret_cast<float2*>(take((size_t)n2 * sizeof(float2)));
    void* table = take((size_t)nfft * (precision == POND_FP32 ? sizeof(float2) : sizeof(float4)));
    uint64_t* acc_sum = reinterpret_cast<uint64_t*>(take((size_t)nbins * 8));
    uint64_t* acc_cnt = reinterpret_cast<uint64_t*>(take((size_t)nbins * 8));
    uint64_t* status = reinterpret_cast<uint64_t*>(take(8));
    uint64_t* part_sum = reinterpret_cast<uint64_t*>(take((size_t)kPartCap * 8));
    uint32_t* part_cnt = reinterpret_cast<uint32_t*>(take((size_t)kPartCap * 4));
    const size_t block_bytes = (size_t)nfft * elem;
    if (off + block_bytes > kScratchBytes) return POND_EINVAL;
    const int64_t fit = (int64_t)((kScratchBytes - off) / block_bytes);
    const int max_batch = (int)(fit > 16 ? 16 : fit);
    void* work = take((size_t)max_batch * block_bytes);

    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    auto fail = [&]() -> int64_t {
        (void)hipGetLastError();
        return POND_EDEVICE;
    };
    hipError_t e = launch_stage_twiddles(tw1, n1, stream);
    if (e == hipSuccess) e = launch_stage_twiddles(tw2, n2, stream);
    if (e == hipSuccess)
        e = launch_k2_build_table(table, precision != POND_FP32, log2n1, log2n2, dm / (2.41e-10 * f0_mhz * f0_mhz),
                                  f0_mhz, bw_mhz / (double)nfft, 0.0, stream);
    // accumulators and status start at zero (fill kernels, no memset nodes)
    if (e == hipSuccess) e = launch_zero_u64(acc_sum, nbins, stream);
    if (e == hipSuccess) e = launch_zero_u64(acc_cnt, nbins, stream);
    if (e == hipSuccess) e = launch_zero_u64(status, 1, stream);
    if (e != hipSuccess) return fail();

    const int64_t cap = hist_capacity(log2n2, precision);
    const bool global_mode = nbins > cap;
    const double inv_pfs = 1.0 / (period_s * fs);
    for (int64_t b = 0; b < nb_total; b += max_batch) {
        const int nb = (int)(nb_total - b < max_batch ? nb_total - b : max_batch);
        K1Args a1{};
        a1.tail = iq;
        a1.in = iq;
        a1.hop = hop;
        a1.block0 = b;
        a1.nblocks = nb;
        a1.log2n1 = log2n1;
        a1.work = work;
        a1.tw2 = tw2;
        a1.scale = std::ldexp(1.0f, -log2n2);
        e = launch_k1(precision, log2n2, a1, stream);
        if (e != hipSuccess) return fail();
        K2Args a2{};
        a2.work = work;
        a2.nblocks = nb;
        a2.log2n2 = log2n2;
        a2.tw1 = tw1;
        a2.table = table;
        a2.scale = std::ldexp(1.0f, -log2n1);
        e = launch_k2(precision, kRowFull, log2n1, a2, stream);
        if (e != hipSuccess) return fail();
        K3Args a3{};
        a3.work = work;
        a3.nblocks = nb;
        a3.log2n1 = log2n1;
        a3.hop = hop;
        a3.n_front = n_front;
        a3.block0 = b;
        a3.tw2 = tw2;
        a3.scale = 1.0f;
        a3.pscale = 1.0f;
        a3.series = series;
        a3.series_base = 0;
        a3.decim = decim;
        a3.nbins = nbins;
        a3.inv_pfs = inv_pfs;
        a3.subint = 0;
        a3.s_base = 0;
        a3.entries = nbins;
        a3.global_mode = global_mode ? 1 : 0;
        a3.part_sum = part_sum;
        a3.part_cnt = part_cnt;
        a3.acc_sum = acc_sum;
        a3.acc_cnt = acc_cnt;
        a3.acc_s0 = 0;
        a3.status = reinterpret_cast<uint32_t*>(status);
        const size_t dyn = global_mode ? 0 : (size_t)nbins * 12;
        const int grid = k3_grid(log2n2, precision, dyn, (int64_t)nb * (n1 / 16), nbins, global_mode, kPartCap);
        e = launch_k3(precision, log2n2, a3, grid, dyn, stream);
        if (e == hipSuccess && !global_mode)
            e = launch_fold_reduce(part_sum, part_cnt, grid, nbins, acc_sum, acc_cnt, 0, stream);
        if (e != hipSuccess) return fail();
    }
    e = launch_fold_finalize(acc_sum, acc_cnt, nbins, 1, 1, profile, stream);
    if (e != hipSuccess) return fail();
    return n_out / decim;
}

}  // extern "C"
