// Fold reduction and finalisation, the streaming copy and small fills.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "pond_device.hpp"

namespace pond {

// ------------------------------------------------------ fold reduction
// Sum the per-workgroup partial histograms (integer, so order-free) and
// add them to the accumulators.  Grid: x over entries, y over part chunks.
// The partials were just written and sit in cache: a full chunk issues all
// its loads at once, so a call costs about one load latency, not a chain.
constexpr int kReduceChunk = 8;
__global__ void __launch_bounds__(256) fold_reduce(const uint64_t* __restrict__ ps, const uint32_t* __restrict__ pc,
                                                   int nparts, int entries, uint64_t* acc_sum, uint64_t* acc_cnt,
                                                   int64_t acc_off) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= entries) return;
    const int p0 = blockIdx.y * kReduceChunk;
    const int p1 = min(nparts, p0 + kReduceChunk);
    uint64_t s = 0, n = 0;
    if (p1 - p0 == kReduceChunk) {
        uint64_t sv[kReduceChunk];
        uint32_t nv[kReduceChunk];
#pragma unroll
        for (int k = 0; k < kReduceChunk; ++k) {
            sv[k] = ps[(int64_t)(p0 + k) * entries + i];
            nv[k] = pc[(int64_t)(p0 + k) * entries + i];
        }
#pragma unroll
        for (int k = 0; k < kReduceChunk; ++k) {
            s += sv[k];
            n += nv[k];
        }
    } else {
        for (int q = p0; q < p1; ++q) {
            s += ps[(int64_t)q * entries + i];
            n += pc[(int64_t)q * entries + i];
        }
    }
    if (n) {
        atomicAdd((unsigned long long*)&acc_sum[acc_off + i], (unsigned long long)s);
        atomicAdd((unsigned long long*)&acc_cnt[acc_off + i], (unsigned long long)n);
    }
}

// The same for up to kReduceSlots queued launches at once (blockIdx.z
// picks the launch; each has its own partials, accumulators and sizes).
__global__ void __launch_bounds__(256) fold_reduce_batch(ReduceBatch b) {
    const ReduceJob& j = b.job[blockIdx.z];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= j.entries) return;
    const int p0 = blockIdx.y * kReduceChunk;
    if (p0 >= j.nparts) return;
    const int p1 = min(j.nparts, p0 + kReduceChunk);
    const uint64_t* ps = j.part_sum;
    const uint32_t* pc = j.part_cnt;
    const int entries = j.entries;
    uint64_t s = 0, n = 0;
    if (p1 - p0 == kReduceChunk) {
        uint64_t sv[kReduceChunk];
        uint32_t nv[kReduceChunk];
#pragma unroll
        for (int k = 0; k < kReduceChunk; ++k) {
            sv[k] = ps[(int64_t)(p0 + k) * entries + i];
            nv[k] = pc[(int64_t)(p0 + k) * entries + i];
        }
#pragma unroll
        for (int k = 0; k < kReduceChunk; ++k) {
            s += sv[k];
            n += nv[k];
        }
    } else {
        for (int q = p0; q < p1; ++q) {
            s += ps[(int64_t)q * entries + i];
            n += pc[(int64_t)q * entries + i];
        }
    }
    if (n) {
        atomicAdd((unsigned long long*)&j.acc_sum[j.acc_off + i], (unsigned long long)s);
        atomicAdd((unsigned long long*)&j.acc_cnt[j.acc_off + i], (unsigned long long)n);
    }
}

// Write the profiles of the first n_complete slots, then move slot
// n_complete (the still-open sub-integration, if any) to slot 0 and clear
// the rest of the n_touched slots.  One thread per bin.
__global__ void __launch_bounds__(256) fold_finalize(uint64_t* acc_sum, uint64_t* acc_cnt, int nbins, int n_complete,
                                                     int n_touched, float* profiles) {
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    if (bin >= nbins) return;
    for (int k = 0; k < n_complete; ++k) {
        const uint64_t s = acc_sum[(int64_t)k * nbins + bin];
        const uint64_t n = acc_cnt[(int64_t)k * nbins + bin];
        profiles[(int64_t)k * nbins + bin] = n ? (float)(((double)s / kFoldScale) / (double)n) : 0.f;
    }
    if (n_complete > 0) {
        uint64_t cs = 0, cn = 0;
        if (n_complete < n_touched) {
            cs = acc_sum[(int64_t)n_complete * nbins + bin];
            cn = acc_cnt[(int64_t)n_complete * nbins + bin];
        }
        acc_sum[bin] = cs;
        acc_cnt[bin] = cn;
        for (int k = 1; k < n_touched; ++k) {
            acc_sum[(int64_t)k * nbins + bin] = 0;
            acc_cnt[(int64_t)k * nbins + bin] = 0;
        }
    }
}

// Mean power per (trial, bin): sum / count, 0 for an empty bin.
__global__ void __launch_bounds__(256) fold_profiles(const uint64_t* acc_sum, const uint64_t* acc_cnt, int64_t n,
                                                     float* profiles) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t c = acc_cnt[i];
    profiles[i] = c ? (float)(((double)acc_sum[i] / kFoldScale) / (double)c) : 0.f;
}

// Streaming copy of n16 16-byte words (measurement of the achievable HBM
// bandwidth): each workgroup moves contiguous 16 KB chunks, a thread's four
// loads of a chunk in flight before its stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) copy_u128(u32x4* __restrict__ dst, const u32x4* __restrict__ src,
                                                 int64_t n16) {
    constexpr int U = 4;
    constexpr int64_t kChunk = 256 * U;
    for (int64_t base = (int64_t)blockIdx.x * kChunk; base < n16; base += (int64_t)gridDim.x * kChunk) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = base + u * 256 + threadIdx.x;
            v[u] = k < n16 ? src[k] : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = base + u * 256 + threadIdx.x;
            if (k < n16) dst[k] = v[u];
        }
    }
}

// Stage twiddles of a length-n transform: w[t] = exp(-2 pi i t / n) for
// t < count, float64 sine and cosine rounded to float32.
__global__ void __launch_bounds__(256) stage_twiddles(float2* w, int64_t count, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    double sn, cs;
    sincospi(2.0 * (double)t / (double)n, &sn, &cs);
    w[t] = make_float2((float)cs, (float)-sn);
}

// Pseudo-random bytes (splitmix64 of the word index and a seed, Steele,
// Lea & Flood 2014): timing input for the autotuner, not part of the method.
__global__ void __launch_bounds__(256) fill_noise_u64(uint64_t* p, int64_t n, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t x = seed + 0x9e3779b97f4a7c15ull * (uint64_t)(i + 1);
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    p[i] = x ^ (x >> 31);
}

__global__ void __launch_bounds__(256) zero_u64(uint64_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_fold_reduce(const uint64_t* ps, const uint32_t* pc, int nparts, int entries, uint64_t* acc_sum,
                              uint64_t* acc_cnt, int64_t acc_off, hipStream_t s) {
    dim3 grid((entries + 255) / 256, (nparts + kReduceChunk - 1) / kReduceChunk);
    hipLaunchKernelGGL(fold_reduce, grid, dim3(256), 0, s, ps, pc, nparts, entries, acc_sum, acc_cnt, acc_off);
    return hipGetLastError();
}

hipError_t launch_fold_reduce_batch(const ReduceBatch& b, hipStream_t s) {
    if (b.n < 1 || b.n > kReduceSlots) return hipErrorInvalidValue;
    int entries = 0, nparts = 0;
    for (int k = 0; k < b.n; ++k) {
        entries = std::max(entries, (int)b.job[k].entries);
        nparts = std::max(nparts, (int)b.job[k].nparts);
    }
    if (entries <= 0 || nparts <= 0) return hipSuccess;
    const dim3 grid((entries + 255) / 256, (nparts + kReduceChunk - 1) / kReduceChunk, b.n);
    hipLaunchKernelGGL(fold_reduce_batch, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_fold_finalize(uint64_t* acc_sum, uint64_t* acc_cnt, int nbins, int n_complete, int n_touched,
                                float* profiles, hipStream_t s) {
    hipLaunchKernelGGL(fold_finalize, dim3((nbins + 255) / 256), dim3(256), 0, s, acc_sum, acc_cnt, nbins,
                       n_complete, n_touched, profiles);
    return hipGetLastError();
}

hipError_t launch_copy_u128(void* dst, const void* src, int64_t n16, hipStream_t s) {
    if (n16 <= 0) return hipSuccess;
    const int64_t chunks = (n16 + 1023) / 1024;
    const unsigned grid = (unsigned)(chunks < 16384 ? chunks : 16384);
    hipLaunchKernelGGL(copy_u128, dim3(grid), dim3(256), 0, s, reinterpret_cast<u32x4*>(dst),
                       reinterpret_cast<const u32x4*>(src), n16);
    return hipGetLastError();
}

hipError_t launch_stage_twiddles(float2* w, int64_t n, hipStream_t s) { return launch_partial_twiddles(w, n, n, s); }

hipError_t launch_partial_twiddles(float2* w, int64_t count, int64_t n, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (count > n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stage_twiddles, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, w, count, n);
    return hipGetLastError();
}

hipError_t launch_fill_noise_u64(uint64_t* p, int64_t n, uint64_t seed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_noise_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, seed);
    return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fold_profiles(const uint64_t* acc_sum, const uint64_t* acc_cnt, int64_t n, float* profiles,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fold_profiles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, acc_sum, acc_cnt, n,
                       profiles);
    return hipGetLastError();
}

}  // namespace pond
