// Split middle pass for blocks of 2^25 .. 2^27 samples: the row transform
// of length n1 = m2 m1 (m1 = 2^13, m2 = 4 .. 16), too long for one
// workgroup's LDS, is done in four steps of its own (Sec. 3.7 computes the
// whole block's spectrum; this only changes how the transform is cut):
//   split_cols (forward): per row k2 and column c < m1, the m2 values at
//     c + m1 i times the block twiddle exp(-2 pi i k2 (c + m1 i) / N),
//     transformed over i, times exp(-2 pi i c k / n1), stored at c + m1 k;
//   K2 kRowChirp: each sub-row k (m1 contiguous values) transformed, times
//     the chirp at frequency k2 + n2 (k + m2 c'), transformed back;
//   split_cols (inverse): the first step conjugated, in reverse order.
// One thread holds the m2 values of one (k2, c): the loads of a wave are 64
// consecutive columns (coalesced) and the transform is in registers.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>

#include "pond_device.hpp"

namespace pond {

namespace {

__device__ __forceinline__ float2 ld_f2(const float2* p) { return *p; }
__device__ __forceinline__ float2 ld_f2(const __half2* p) { return to_f2(__builtin_bit_cast(h2, *p)); }
__device__ __forceinline__ void st_f2(float2* p, float2 v) { *p = v; }
__device__ __forceinline__ void st_f2(__half2* p, float2 v) { *p = __builtin_bit_cast(__half2, to_h2(v)); }
__device__ __forceinline__ float2 ld_f2(const bf16x2* p) { return Elem<bf16x2>::load(p); }
__device__ __forceinline__ void st_f2(bf16x2* p, float2 v) { Elem<bf16x2>::store(p, v); }

// exp(-2 pi i r / N) from the two-level table: r = hi 2^s + lo.
__device__ __forceinline__ float2 block_twiddle(const SplitColArgs& a, uint32_t r) {
    const float2 h = a.tw_hi[r >> a.log2s];
    const float2 l = a.tw_lo[r & ((1u << a.log2s) - 1u)];
    return cmul(h, l);
}

template <int LOG2M2, bool INV, class T>
__global__ void __launch_bounds__(256) split_cols(SplitColArgs a) {
    constexpr int M2 = 1 << LOG2M2;
    constexpr int LOG2M1 = kSplitLog2M1;
    constexpr int M1 = 1 << LOG2M1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)a.nblocks << (a.log2n2 + LOG2M1);
    if (t >= total) return;
    const uint32_t c = (uint32_t)(t & (M1 - 1));
    const uint32_t k2 = (uint32_t)((t >> LOG2M1) & ((1 << a.log2n2) - 1));
    const int64_t b = t >> (LOG2M1 + a.log2n2);
    const uint32_t nmask = (1u << (a.log2n1 + a.log2n2)) - 1u;
    T* row = reinterpret_cast<T*>(a.work) + (((b << a.log2n2) + k2) << a.log2n1) + c;
    float2 v[M2];
#pragma unroll
    for (int i = 0; i < M2; ++i) v[i] = ld_f2(row + (int64_t)i * M1);
    if constexpr (!INV) {
#pragma unroll
        for (int i = 0; i < M2; ++i) v[i] = cmul(v[i], block_twiddle(a, (k2 * (c + (uint32_t)i * M1)) & nmask));
        Dft<M2, -1, float2>::run(v);
#pragma unroll
        for (int k = 0; k < M2; ++k) st_f2(row + (int64_t)k * M1, cscale(cmul(v[k], a.tw_n1[c * k]), a.scale));
    } else {
#pragma unroll
        for (int k = 0; k < M2; ++k) v[k] = cmulc(v[k], a.tw_n1[c * k]);
        Dft<M2, +1, float2>::run(v);
#pragma unroll
        for (int i = 0; i < M2; ++i)
            st_f2(row + (int64_t)i * M1,
                  cscale(cmulc(v[i], block_twiddle(a, (k2 * (c + (uint32_t)i * M1)) & nmask)), a.scale));
    }
}

// Chirp of the split middle pass in sub-row order (see the header).
template <bool F16>
__global__ void __launch_bounds__(256) build_split_chirp(void* tab, int log2n1, int log2n2, double chirp_a, double f0,
                                                         double df, double chirp_scale, double taper) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int log2n = log2n1 + log2n2;
    const int64_t n = 1ll << log2n;
    if (i >= n) return;
    const int log2m2 = log2n1 - kSplitLog2M1;
    const int64_t cp = i & ((1ll << kSplitLog2M1) - 1);
    const int64_t k = (i >> kSplitLog2M1) & ((1ll << log2m2) - 1);
    const int64_t k2 = i >> log2n1;
    const int64_t kf = k2 + ((k + (cp << log2m2)) << log2n2);
    const int64_t kk = kf < (n >> 1) ? kf : kf - n;
    const double f = (double)kk * df;
    const double turns = chirp_a * (f * f) / (f0 + f);
    const double frac = turns - rint(turns);
    double cs, cc;
    sincospi(2.0 * frac, &cs, &cc);
    const double w = taper_w(f, df * (double)n, taper);
    if constexpr (F16) {
        const double m = chirp_scale * w;
        reinterpret_cast<h2*>(tab)[i] = f16_unit(cc * m, -cs * m, m);
    } else {
        reinterpret_cast<float2*>(tab)[i] = make_float2((float)(cc * w), (float)(-cs * w));
    }
}

template <int LOG2M2, class T>
hipError_t split_one(bool inverse, const SplitColArgs& a, hipStream_t s) {
    const int64_t total = (int64_t)a.nblocks << (a.log2n2 + kSplitLog2M1);
    const dim3 grid((unsigned)((total + 255) / 256));
    if (inverse) hipLaunchKernelGGL((split_cols<LOG2M2, true, T>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((split_cols<LOG2M2, false, T>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <class T>
hipError_t split_dispatch(bool inverse, const SplitColArgs& a, hipStream_t s) {
    switch (a.log2n1 - kSplitLog2M1) {
        case 1: return split_one<1, T>(inverse, a, s);
        case 2: return split_one<2, T>(inverse, a, s);
        case 3: return split_one<3, T>(inverse, a, s);
        case 4: return split_one<4, T>(inverse, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_split_cols(int prec, bool inverse, const SplitColArgs& a, hipStream_t s) {
    if (a.log2n1 + a.log2n2 > 31 || a.log2s <= 0 || a.log2s > a.log2n1 + a.log2n2) return hipErrorInvalidValue;
    if (prec == kFp32) return split_dispatch<float2>(inverse, a, s);
    if (prec == kBf16) return split_dispatch<bf16x2>(inverse, a, s);
    return split_dispatch<__half2>(inverse, a, s);
}

hipError_t launch_build_split_chirp(void* tab, bool f16, int log2n1, int log2n2, double chirp_a, double f0, double df,
                                    double taper, hipStream_t s) {
    if (log2n1 <= kSplitLog2M1 || log2n1 > kSplitLog2M1 + 4) return hipErrorInvalidValue;
    const int64_t n = 1ll << (log2n1 + log2n2);
    const dim3 grid((unsigned)((n + 255) / 256));
    const double chirp_scale = std::ldexp(1.0, -half_row_rem(kSplitLog2M1));
    if (f16)
        hipLaunchKernelGGL(build_split_chirp<true>, grid, dim3(256), 0, s, tab, log2n1, log2n2, chirp_a, f0, df,
                           chirp_scale, taper);
    else
        hipLaunchKernelGGL(build_split_chirp<false>, grid, dim3(256), 0, s, tab, log2n1, log2n2, chirp_a, f0, df,
                           chirp_scale, taper);
    return hipGetLastError();
}

}  // namespace pond
