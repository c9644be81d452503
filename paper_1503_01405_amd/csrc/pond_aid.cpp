// Incoherent dedispersion with an FFT filterbank (the AID pulsar mode,
// Sec. 3.4 and Sec. 3.4.1): spectra of consecutive nchan-sample blocks,
// squared and summed over nint spectra, each channel shifted by its
// dispersive delay (Eq. (3), referred to f0 and rounded to the integrated
// sample), channels summed, then folded at the period.  One call processes
// one resident stream segment; nothing is carried between calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/pond.h"
#include "pond_internal.hpp"

using namespace pond;

struct pond_aid {
    int device = 0;
    double f0 = 0, bw = 0, dm = 0, period = 0, inv_pfs = 0, ts = 0;
    int32_t nchan = 0, log2c = 0, nint = 0, nbins = 0;
    int32_t d_min = 0, d_max = 0;
    float2* tw = nullptr;
    int32_t* dd = nullptr;
    float* F = nullptr;
    size_t F_cap = 0;  // floats
    uint64_t* acc_sum = nullptr;
    uint64_t* acc_cnt = nullptr;
    uint64_t* part_sum = nullptr;
    uint32_t* part_cnt = nullptr;
    uint64_t* status = nullptr;
    hipStream_t last_stream = nullptr;
    bool sticky = false;
};

namespace {

void free_aid(pond_aid* a) {
    void* ptrs[] = {a->tw, a->dd, a->F, a->acc_sum, a->acc_cnt, a->part_sum, a->part_cnt, a->status};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
}

int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}

}  // namespace

extern "C" {

pond_aid* pond_aid_create(double f0_mhz, double bw_mhz, double dm, int32_t nchan, int32_t nint, int32_t nbins,
                          double period_s) {
    if (!std::isfinite(f0_mhz) || !std::isfinite(bw_mhz) || !std::isfinite(dm) || !std::isfinite(period_s))
        return nullptr;
    if (!(bw_mhz > 0) || !(f0_mhz - bw_mhz / 2 > 0) || !(dm >= 0)) return nullptr;
    if (nchan < 64 || nchan > 4096 || (nchan & (nchan - 1))) return nullptr;
    if (nint < 1 || nint > 65536 || nbins < 1 || nbins > 65536) return nullptr;
    const double fs = bw_mhz * 1e6;
    if (!(period_s > 0) || !(period_s * fs >= 1.0)) return nullptr;

    pond_aid* a = new (std::nothrow) pond_aid();
    if (!a) return nullptr;
    if (hipGetDevice(&a->device) != hipSuccess) {
        delete a;
        return nullptr;
    }
    a->f0 = f0_mhz;
    a->bw = bw_mhz;
    a->dm = dm;
    a->period = period_s;
    a->inv_pfs = 1.0 / (period_s * fs);
    a->nchan = nchan;
    a->log2c = ilog2(nchan);
    a->nint = nint;
    a->nbins = nbins;
    // Channel c is baseband frequency fftfreq(nchan) * bw (sky f0 + f);
    // delay (1/2.41e-4) DM (f^-2 - f0^-2) s in integrated samples of
    // t_s = nchan nint / fs, rounded to nearest (float64 throughout).
    a->ts = (double)nchan * (double)nint / (bw_mhz * 1e6);
    const double val = 1.0 / ((double)nchan * (1.0 / bw_mhz));
    std::vector<int32_t> d((size_t)nchan);
    const int32_t half = (nchan - 1) / 2 + 1;
    for (int32_t c = 0; c < nchan; ++c) {
        const double k = c < half ? (double)c : (double)(c - nchan);
        const double f = f0_mhz + k * val;
        const double dt = (1.0 / 2.41e-4) * dm * (1.0 / (f * f) - 1.0 / (f0_mhz * f0_mhz));
        const double q = std::floor(dt / a->ts + 0.5);
        if (!(std::fabs(q) < 1e9)) {
            delete a;
            return nullptr;
        }
        d[(size_t)c] = (int32_t)q;
    }
    a->d_min = d[0];
    a->d_max = d[0];
    for (int32_t v : d) {
        a->d_min = v < a->d_min ? v : a->d_min;
        a->d_max = v > a->d_max ? v : a->d_max;
    }
    for (int32_t& v : d) v -= a->d_min;
    std::vector<float2> tw((size_t)nchan);
    for (int32_t t = 0; t < nchan; ++t) {
        const double ang = 2.0 * M_PI * (double)t / (double)nchan;
        tw[(size_t)t] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
    }
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    chk(hipMalloc(reinterpret_cast<void**>(&a->tw), (size_t)nchan * sizeof(float2)));
    chk(hipMalloc(reinterpret_cast<void**>(&a->dd), (size_t)nchan * 4));
    chk(hipMalloc(reinterpret_cast<void**>(&a->acc_sum), (size_t)nbins * 8));
    chk(hipMalloc(reinterpret_cast<void**>(&a->acc_cnt), (size_t)nbins * 8));
    chk(hipMalloc(reinterpret_cast<void**>(&a->part_sum), (size_t)kPartEntries * 8));
    chk(hipMalloc(reinterpret_cast<void**>(&a->part_cnt), (size_t)kPartEntries * 4));
    chk(hipMalloc(reinterpret_cast<void**>(&a->status), 8));
    if (e == hipSuccess) chk(hipMemcpy(a->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
    if (e == hipSuccess) chk(hipMemcpy(a->dd, d.data(), d.size() * 4, hipMemcpyHostToDevice));
    if (e == hipSuccess) chk(hipMemset(a->status, 0, 8));
    if (e == hipSuccess) chk(hipStreamSynchronize(nullptr));
    if (e != hipSuccess) {
        free_aid(a);
        delete a;
        (void)hipGetLastError();
        return nullptr;
    }
    return a;
}

int32_t pond_aid_geometry(const pond_aid* a, int64_t nsamp, int64_t* n_spectra, int64_t* n_series, int32_t* d_min,
                          int32_t* d_max, double* t_s) {
    if (!a || nsamp < 0) return POND_EINVAL;
    const int64_t nspec = nsamp / ((int64_t)a->nchan * a->nint);
    const int64_t nout = nspec - (int64_t)(a->d_max - a->d_min);
    if (n_spectra) *n_spectra = nspec;
    if (n_series) *n_series = nout > 0 ? nout : 0;
    if (d_min) *d_min = a->d_min;
    if (d_max) *d_max = a->d_max;
    if (t_s) *t_s = a->ts;
    return POND_OK;
}

int64_t pond_aid_run(pond_aid* a, const int8_t* iq, int64_t nsamp, float* profile, float* series, int64_t series_cap,
                     void* stream_ptr) {
    if (!a) return POND_EINVAL;
    if (a->sticky) return POND_EDEVICE;
    if (nsamp < 0 || (nsamp > 0 && (!iq || (reinterpret_cast<uintptr_t>(iq) & 1u))) || !profile) return POND_EINVAL;
    int64_t nspec = 0, nout = 0;
    (void)pond_aid_geometry(a, nsamp, &nspec, &nout, nullptr, nullptr, nullptr);
    if (series && series_cap < nout) return POND_EINVAL;
    hipStream_t stream = reinterpret_cast<hipStream_t>(stream_ptr);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return POND_EDEVICE;
    if (cur != a->device && hipSetDevice(a->device) != hipSuccess) return POND_EDEVICE;
    auto done = [&](int64_t r) {
        if (cur != a->device) (void)hipSetDevice(cur);
        return r;
    };
    auto fail = [&]() {
        (void)hipGetLastError();
        a->sticky = true;
        return done(POND_EDEVICE);
    };
    const size_t need = (size_t)a->nchan * (size_t)nspec;
    if (need > a->F_cap) {
        float* nf = nullptr;
        if (hipMallocAsync(reinterpret_cast<void**>(&nf), need * 4, stream) != hipSuccess) {
            (void)hipGetLastError();
            return done(POND_ENOMEM);
        }
        if (a->F && hipFreeAsync(a->F, stream) != hipSuccess) return fail();
        a->F = nf;
        a->F_cap = need;
    }
    hipError_t e = launch_zero_u64(a->acc_sum, a->nbins, stream);
    if (e == hipSuccess) e = launch_zero_u64(a->acc_cnt, a->nbins, stream);
    if (e != hipSuccess) return fail();
    AidArgs g{};
    g.iq = iq;
    g.nspec = nspec;
    g.nint = a->nint;
    g.nchan = a->nchan;
    g.tw = a->tw;
    g.F = a->F;
    g.dd = a->dd;
    g.d_min = a->d_min;
    g.nout = nout;
    g.series = series;
    g.nbins = a->nbins;
    g.inv_pfs = a->inv_pfs;
    g.part_sum = a->part_sum;
    g.part_cnt = a->part_cnt;
    g.status = reinterpret_cast<uint32_t*>(a->status);
    if (nspec > 0) {
        e = launch_aid_filterbank(a->log2c, g, stream);
        if (e != hipSuccess) return fail();
    }
    if (nout > 0) {
        int64_t grid = (nout + 255) / 256;
        const int64_t cap = kPartEntries / a->nbins;
        grid = grid < 2048 ? grid : 2048;
        grid = grid < cap ? grid : cap;
        grid = grid < 1 ? 1 : grid;
        e = launch_aid_dedisperse_fold(g, (int)grid, stream);
        if (e == hipSuccess)
            e = launch_fold_reduce(a->part_sum, a->part_cnt, (int)grid, a->nbins, a->acc_sum, a->acc_cnt, 0, stream);
        if (e != hipSuccess) return fail();
    }
    e = launch_fold_profiles(a->acc_sum, a->acc_cnt, a->nbins, profile, stream);
    if (e != hipSuccess) return fail();
    a->last_stream = stream;
    return done(nout);
}

void pond_aid_destroy(pond_aid* a) {
    if (!a) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != a->device) (void)hipSetDevice(a->device);
    (void)hipStreamSynchronize(a->last_stream);
    free_aid(a);
    if (cur >= 0 && cur != a->device) (void)hipSetDevice(cur);
    delete a;
}

}  // extern "C"
