// Incoherent (AID) mode kernels: filterbank, channel shift-and-sum, fold.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "pond_device.hpp"

namespace pond {

// ------------------------------------------------- incoherent (AID) mode
// Filterbank: spectra of consecutive nchan-sample blocks (square window, no
// overlap), |X|^2 summed over nint spectra per output time.  One FFT group
// of nchan/16 threads per row of the workgroup (as K2's short rows); each
// group takes AID_TS consecutive output times and keeps their powers in
// registers; the workgroup then writes them channel-major, F[c][t], through
// an LDS transpose (rows of ROWS*AID_TS consecutive times per channel).
constexpr int AID_TS = 4;

template <int LOG2C>
__global__ void __launch_bounds__(K2Shape<LOG2C>::THREADS) aid_filterbank(AidArgs a) {
    using Sh = K2Shape<LOG2C>;
    constexpr int C = 1 << LOG2C;
    constexpr int TPV = Sh::TPV;
    constexpr int ROWS = Sh::ROWS;
    constexpr int COLS = ROWS * AID_TS;  // output times per workgroup
    constexpr int FFT_LDS = ROWS * Sh::STRIDE * 8;
    constexpr int TILE_LDS = C * COLS * 4;
    __shared__ __align__(16) char lds_raw[FFT_LDS > TILE_LDS ? FFT_LDS : TILE_LDS];
    float2* lds = reinterpret_cast<float2*>(lds_raw);
    float* tile = reinterpret_cast<float*>(lds_raw);

    const int g = threadIdx.x / TPV;
    const int j = threadIdx.x - g * TPV;
    const PadLds<float2> lrow{lds + g * Sh::STRIDE};
    StageBases<LOG2C> tb;
    tb.load(j, a.tw);
    const int64_t tbase = (int64_t)blockIdx.x * COLS;

    float acc[AID_TS][16];
#pragma unroll
    for (int ts = 0; ts < AID_TS; ++ts) {
        const int64_t t = tbase + g * AID_TS + ts;
        const bool live = t < a.nspec;
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[ts][e] = 0.f;
        for (int i = 0; i < a.nint; ++i) {
            float2 v[16];
            const int8_t* blk = a.iq + 2 * ((live ? t : 0) * a.nint + i) * (int64_t)C;
            const uint32_t o = opaque((uint32_t)j);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const short sv = *at(reinterpret_cast<const short*>(blk), (o + TPV * e) * 2u);
                v[e] = make_float2((float)(int8_t)(sv & 0xff), (float)(int8_t)(sv >> 8));
            }
            fft_wg<LOG2C, -1>(v, j, tb, lrow);
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[ts][e] = fmaf(v[e].x, v[e].x, fmaf(v[e].y, v[e].y, acc[ts][e]));
        }
    }
    __syncthreads();  // the FFT scratch becomes the transpose tile
#pragma unroll
    for (int ts = 0; ts < AID_TS; ++ts)
#pragma unroll
        for (int e = 0; e < 16; ++e) tile[(j + TPV * e) * COLS + g * AID_TS + ts] = acc[ts][e];
    __syncthreads();
    const int64_t ncols = a.nspec - tbase < COLS ? a.nspec - tbase : COLS;
    for (int idx = threadIdx.x; idx < C * COLS; idx += blockDim.x) {
        const int c = idx / COLS, col = idx - c * COLS;
        if (col < ncols) a.F[(int64_t)c * a.nspec + tbase + col] = tile[idx];
    }
}

// Channel shift-and-sum and fold: output m = sum_c F[c][m + dd_c], with
// dd_c = d_c - d_min >= 0 (Eq. (3) delays in integrated samples); the
// series value and its fold into integer (sub-integration-free) histograms
// as K3 does, fold phase x = (m - d_min) * nchan * nint * inv_pfs.
__global__ void __launch_bounds__(256) aid_dedisperse_fold(AidArgs a) {
    extern __shared__ uint64_t dyn_u64[];
    uint64_t* hsum = dyn_u64;
    uint32_t* hcnt = reinterpret_cast<uint32_t*>(dyn_u64 + a.nbins);
    int32_t* dd = reinterpret_cast<int32_t*>(hcnt + a.nbins);
    for (int i = threadIdx.x; i < a.nbins; i += blockDim.x) {
        hsum[i] = 0;
        hcnt[i] = 0;
    }
    for (int c = threadIdx.x; c < a.nchan; c += blockDim.x) dd[c] = a.dd[c];
    __syncthreads();
    uint32_t flags = 0;
    const double spec = (double)a.nchan * (double)a.nint;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < a.nout;
         m += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        const float* f = a.F + m;
        for (int c = 0; c < a.nchan; ++c) s += f[(int64_t)c * a.nspec + dd[c]];
        if (a.series) a.series[m] = s;
        const double x = (double)(m - a.d_min) * spec * a.inv_pfs;
        int bin = (int)((x - floor(x)) * (double)a.nbins);
        bin = bin < a.nbins - 1 ? bin : a.nbins - 1;
        const double dv = (double)s * kFoldScale;
        if (!(dv < kFoldRangeLimit * kFoldScale)) flags |= 2u;
        if (!isfinite(s)) flags |= 1u;
        const uint64_t fx = isfinite(s) ? (uint64_t)__double2ull_rn(dv) : 0ull;
        atomicAdd((unsigned long long*)&hsum[bin], (unsigned long long)fx);
        atomicAdd(&hcnt[bin], 1u);
    }
    if (flags) atomicOr(a.status, flags);
    __syncthreads();
    uint64_t* ps = a.part_sum + (int64_t)blockIdx.x * a.nbins;
    uint32_t* pc = a.part_cnt + (int64_t)blockIdx.x * a.nbins;
    for (int i = threadIdx.x; i < a.nbins; i += blockDim.x) {
        ps[i] = hsum[i];
        pc[i] = hcnt[i];
    }
}

template <int LOG2C>
static hipError_t aid_fb_one(const AidArgs& a, hipStream_t s) {
    using Sh = K2Shape<LOG2C>;
    const int64_t cols = Sh::ROWS * AID_TS;
    const int64_t grid = (a.nspec + cols - 1) / cols;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(aid_filterbank<LOG2C>, dim3((unsigned)grid), dim3(Sh::THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_aid_filterbank(int log2c, const AidArgs& a, hipStream_t s) {
    switch (log2c) {
        case 6: return aid_fb_one<6>(a, s);
        case 7: return aid_fb_one<7>(a, s);
        case 8: return aid_fb_one<8>(a, s);
        case 9: return aid_fb_one<9>(a, s);
        case 10: return aid_fb_one<10>(a, s);
        case 11: return aid_fb_one<11>(a, s);
        case 12: return aid_fb_one<12>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_aid_dedisperse_fold(const AidArgs& a, int grid, hipStream_t s) {
    const size_t dyn = (size_t)a.nbins * 12 + (size_t)a.nchan * 4;
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&aid_dedisperse_fold),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(aid_dedisperse_fold, dim3(grid), dim3(256), dyn, s, a);
    return hipGetLastError();
}

}  // namespace pond
