// K3: inverse column FFTs, square-law detection, the integrated series
// and the fold into per-workgroup integer histograms.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "pond_device.hpp"

namespace pond {

// Power buffer of the packed-float16 K3: row-major, 16 floats per row, the
// four float4 quarters of a row rotated by (row / 4) mod 4, so that the
// epilogue's float4 reads of 16 consecutive rows (one per lane) and the
// detection's writes of four rows per wave use every bank once.
__device__ __forceinline__ int k3h_pidx(int row, int col) {
    return row * 16 + ((((col >> 2) + (row >> 2)) & 3) << 2) + (col & 3);
}

// REAL (real input path, float32 arithmetic): element m of the output is
// y[2m] + i y[2m+1] of the real dedispersed voltage, detected per real
// sample (y^2); the group of 16 elements is 32 real outputs, the series
// (sums over decim elements = 2 decim real samples) is unchanged, and the
// fold takes real sample r = 2 m + j with phase (r + 2 n_front) inv_pfs
// (inv_pfs of the real sample rate).
template <int LOG2N2, class T, int FORM, bool REAL = false>
__global__ void __launch_bounds__(1 << LOG2N2) k3_colinv_detect_fold(K3Args a) {
    using Sh = K3Shape<LOG2N2>;
    constexpr int L = Sh::L;
    constexpr int TPV = Sh::TPV;
    // floats per row of the power buffer: 16 + 4 pad, 16-byte aligned; REAL:
    // two powers per column, 32 with no pad (the buffer then fills the FFT
    // tile exactly) but rotated by 4 (row mod 8) floats, so that the row
    // reads of the epilogue spread over the banks
    constexpr int PSTRIDE = REAL ? 32 : 20;
    auto rot = [](int row, int x) { return (x + 4 * (row & 7)) & 31; };
    __shared__ __align__(16) char lds_raw[Sh::lds(FORM)];
    extern __shared__ uint64_t dyn_u64[];
    uint64_t* hsum = dyn_u64;
    uint32_t* hcnt = reinterpret_cast<uint32_t*>(dyn_u64 + (a.global_mode ? 0 : a.entries));
    float2* lds = reinterpret_cast<float2*>(lds_raw);
    constexpr bool H16 = FORM == kFormF16 || FORM == kFormMfma;  // float16 arithmetic
    constexpr bool MX = FORM == kFormMfma && kMxShape<LOG2N2, true>;  // radix-16 sums on matrix cores
    float* pf = reinterpret_cast<float*>(lds_raw + (H16 ? Sh::kHalfTile : 0));

    const int c = threadIdx.x & 15;
    const int j = threadIdx.x >> 4;
    const int n1 = 1 << a.log2n1;
    const int log2tiles = a.log2n1 - 4;  // tiles of 16 columns per block
    const int items = a.nblocks << log2tiles;
    const int r0 = (int)(a.n_front & 15);
    const double inv_s = a.subint > 0 ? 1.0 / (double)a.subint : 0.0;
    const int log2d = __builtin_ctz((unsigned)a.decim);  // decim is a power of two

    if (!a.global_mode) {
        for (int i = threadIdx.x; i < a.entries; i += blockDim.x) {
            hsum[i] = 0;
            hcnt[i] = 0;
        }
    }
    // Items are split into 8 contiguous chunks, one per XCD, so that the
    // workgroups running together on one XCD handle neighbouring tiles.
    const int per_xcd = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7;
    const int local = blockIdx.x >> 3;
    const int chunk = (items + 7) >> 3;
    const int it_end = min(items, (xcd + 1) * chunk);
    uint32_t flags = 0;
    StageBases<LOG2N2, LdsVal<FORM>> tb;
    tb.load(j, a.tw2);
    // packed float16: the stage-1 twiddle table follows the power buffer
    h2* ttab = reinterpret_cast<h2*>(lds_raw + Sh::kHalfTile + Sh::kHalfPf);
    if constexpr (H16) if (threadIdx.x < 64) fill_twiddle_tables<LOG2N2, 64>(ttab, a.tw2, threadIdx.x);

    // Float16 storage with VALU arithmetic, columns of 2^9 and 2^10: the
    // next item's column tile is loaded (as float16 pairs) while this one
    // is transformed and folded, so its latency is not exposed once per
    // item (the 16 registers are free there: the LDS already limits the
    // kernel to four waves per SIMD).
    constexpr bool kPrefetch = (H16 || (FORM == kFormF32 && std::is_same<T, __half2>::value)) &&
                               (LOG2N2 == 10 || (LOG2N2 == 9 && !REAL));  // (else past 128 registers)
    h2 nxt[16];
    auto load_tile = [&](int it, h2(&dst)[16]) {
        const int bb = it >> log2tiles;
        const int tt = it & ((1 << log2tiles) - 1);
        const uint32_t cc = opaque((uint32_t)((r0 + 16 * tt + c) & (n1 - 1)));
        const __half2* const ib =
            uniform_ptr(reinterpret_cast<const __half2*>(a.work) + ((int64_t)bb << (a.log2n1 + LOG2N2)));
        // the block through a buffer descriptor: the lane's offset in a
        // vector register, the row offset of value e in a scalar one
        const BufRes rb = buf_res(ib, (uint32_t)sizeof(__half2) << (a.log2n1 + LOG2N2));
        if constexpr (MX) {
            // matrix-core layout: value e = 4b + t at position
            // 4 (j / 4) + b + (4 (j mod 4) + t) TPV
            const uint32_t ioff =
                (cc + ((uint32_t)(4 * (j >> 2) + 4 * (j & 3) * TPV) << a.log2n1)) * (uint32_t)sizeof(__half2);
#pragma unroll
            for (int e = 0; e < 16; ++e)
                dst[e] = buf_ld<h2>(rb, ioff, (int)(((e >> 2) + (e & 3) * TPV) * sizeof(__half2)) << a.log2n1);
        } else {
            const uint32_t ioff = (cc + ((uint32_t)j << a.log2n1)) * (uint32_t)sizeof(__half2);
#pragma unroll
            for (int e = 0; e < 16; ++e) dst[e] = buf_ld<h2>(rb, ioff, (int)(TPV * e * sizeof(__half2)) << a.log2n1);
        }
    };
    if constexpr (kPrefetch) {
        if (xcd * chunk + local < it_end) load_tile(xcd * chunk + local, nxt);
    }
    for (int item = xcd * chunk + local; item < it_end; item += per_xcd) {
        const int b = item >> log2tiles;
        const int t = item & ((1 << log2tiles) - 1);
        const int col = (r0 + 16 * t + c) & (n1 - 1);

        const T* in = reinterpret_cast<const T*>(a.work) + ((int64_t)b << (a.log2n1 + LOG2N2));
        const uint32_t o0 = opaque((uint32_t)col);
        if constexpr (H16) {
            // Packed float16 inverse transform (unnormalised; matrix-core
            // form: radix-16 sums on the matrix cores), then the power in
            // float32 from the float16 pair (exact products).
            h2* lh = reinterpret_cast<h2*>(lds);
            h2 v[16];
            if constexpr (kPrefetch) {
#pragma unroll
                for (int e = 0; e < 16; ++e) v[e] = nxt[e];
                if (item + per_xcd < it_end) load_tile(item + per_xcd, nxt);
            } else {
                load_tile(item, v);
            }
            // no barrier before the first exchange: every wave has left the
            // previous item's transform (the barrier after its powers)
            if constexpr (MX) fft_mx<LOG2N2, +1, false, true, false>(v, j, lh + c, ttab);
            else fft_wg<LOG2N2, +1, false, 2, false>(v, j, tb, ColLds<h2, true>{lh + c}, ttab);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const float yx = (float)v[e].x, yy = (float)v[e].y;
                pf[k3h_pidx(j + TPV * e, c)] = fmaf(yx, yx, yy * yy) * a.pscale;
            }
            __syncthreads();
        } else {
            float2 v[16];
            if constexpr (kPrefetch) {
#pragma unroll
                for (int e = 0; e < 16; ++e) v[e] = to_f2(nxt[e]);
                if (item + per_xcd < it_end) load_tile(item + per_xcd, nxt);
            } else {
                const T* const ib = uniform_ptr(in);
                const uint32_t ioff = (o0 + ((uint32_t)j << a.log2n1)) * (uint32_t)sizeof(T);
#pragma unroll
                for (int e = 0; e < 16; ++e) v[e] = Elem<T>::load(at(ib + ((int64_t)(TPV * e) << a.log2n1), ioff));
            }
            fft_wg<LOG2N2, +1>(v, j, tb, ColLds<float2>{lds + c});

            // Detected powers to LDS, one row of 16 columns per output row.
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const float2 y = cscale(v[e], a.scale);
                if constexpr (REAL) {
                    const int row = j + TPV * e;
                    *reinterpret_cast<float2*>(pf + row * PSTRIDE + rot(row, 2 * c)) = make_float2(y.x * y.x, y.y * y.y);
                } else {
                    pf[(j + TPV * e) * PSTRIDE + c] = fmaf(y.x, y.x, y.y * y.y);
                }
            }
            __syncthreads();
        }

        // Thread q takes group q: outputs n = r0 + 16 t + n1 q + [0, 16),
        // i.e. 16 consecutive kept outputs (columns that wrap past n1 hold
        // them one row further down).
        const int q = threadIdx.x;
        const int64_t nstart = (int64_t)(r0 + 16 * t) + ((int64_t)q << a.log2n1);
        const int64_t off = nstart - a.n_front;
        float p[16];
        float pr[REAL ? 32 : 1];  // REAL: the 32 real-sample powers of the group
        if constexpr (REAL) {
            if (r0 + 16 * t + 15 < n1) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float4 x4 = *reinterpret_cast<const float4*>(pf + q * PSTRIDE + rot(q, 4 * i));
                    pr[4 * i] = x4.x;
                    pr[4 * i + 1] = x4.y;
                    pr[4 * i + 2] = x4.z;
                    pr[4 * i + 3] = x4.w;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int rsrc = q + ((r0 + 16 * t + i) >> a.log2n1);
                    pr[2 * i] = rsrc < L ? pf[rsrc * PSTRIDE + rot(rsrc, 2 * i)] : 0.f;
                    pr[2 * i + 1] = rsrc < L ? pf[rsrc * PSTRIDE + rot(rsrc, 2 * i) + 1] : 0.f;
                }
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) p[i] = pr[2 * i] + pr[2 * i + 1];
        } else if (r0 + 16 * t + 15 < n1) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 x4 = *reinterpret_cast<const float4*>(
                    pf + (H16 ? k3h_pidx(q, 4 * i) : q * PSTRIDE + 4 * i));
                p[4 * i] = x4.x;
                p[4 * i + 1] = x4.y;
                p[4 * i + 2] = x4.z;
                p[4 * i + 3] = x4.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int rsrc = q + ((r0 + 16 * t + i) >> a.log2n1);
                p[i] = rsrc < L ? pf[H16 ? k3h_pidx(rsrc, i) : rsrc * PSTRIDE + i] : 0.f;
            }
        }
        if (off < 0 || off >= a.hop) continue;

        // Group sum and the decimated series (sums of `decim` consecutive
        // powers, pairwise).
        float s2[8], s4[4], s8[2];
#pragma unroll
        for (int i = 0; i < 8; ++i) s2[i] = p[2 * i] + p[2 * i + 1];
#pragma unroll
        for (int i = 0; i < 4; ++i) s4[i] = s2[2 * i] + s2[2 * i + 1];
        s8[0] = s4[0] + s4[1];
        s8[1] = s4[2] + s4[3];
        const float s16 = s8[0] + s8[1];
        const int64_t m0 = (a.block0 + b) * a.hop + off;  // first output of the group
        if (a.series) {
            float* sp = a.series + ((m0 >> log2d) - a.series_base);
            if (a.decim == 16) {
                sp[0] = s16;
            } else if (a.decim == 8) {
                sp[0] = s8[0];
                sp[1] = s8[1];
            } else if (a.decim == 4) {
#pragma unroll
                for (int i = 0; i < 4; ++i) sp[i] = s4[i];
            } else if (a.decim == 2) {
#pragma unroll
                for (int i = 0; i < 8; ++i) sp[i] = s2[i];
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i) sp[i] = p[i];
            }
        }
        if (!isfinite(s16)) flags |= 1u;

        // Fold: one contribution when all outputs of the group share pulse,
        // bin and sub-integration (the first and last decide, phase being
        // monotone).
        double t0, t15;
        constexpr int G = REAL ? 32 : 16;  // fold samples of the group
        const int64_t f0i = REAL ? 2 * m0 : m0, fnf = REAL ? 2 * a.n_front : a.n_front;
        const int bin0 = fold_bin(f0i, fnf, a.inv_pfs, a.nbins, &t0);
        const int bin15 = fold_bin(f0i + G - 1, fnf, a.inv_pfs, a.nbins, &t15);
        const int64_t d0 = m0 - a.s_base * a.subint;
        const int64_t sub0 = a.subint > 0 ? subint_rel(d0, a.subint, inv_s) : 0;
        // the group's 16 outputs share sub0 unless it ends within them
        const bool one_sub = a.subint <= 0 || d0 - sub0 * a.subint + 15 < a.subint;
        if (bin0 == bin15 && t0 == t15 && one_sub) {
            fold_add(a, hsum, hcnt, sub0, bin0, s16, G, flags);
            continue;
        }
        // Phase grows with the sample index, so each (pulse, bin) cell holds
        // consecutive samples: bisect for the end of the first cell (with
        // the per-sample float64 evaluation itself) and, if the rest of the
        // group is one cell, add two partial sums; otherwise (a bin shorter
        // than the group, or a sub-integration edge) one add per sample.
        int hi = G - 1;
        bool two = one_sub;
        if (two) {
            int lo = 0;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                double tm;
                const int bm = fold_bin(f0i + mid, fnf, a.inv_pfs, a.nbins, &tm);
                if (bm == bin0 && tm == t0) lo = mid;
                else hi = mid;
            }
            double th;
            const int bh = fold_bin(f0i + hi, fnf, a.inv_pfs, a.nbins, &th);
            two = bh == bin15 && th == t15;
        }
        if (two) {
            float sa = 0.f, sb = 0.f;
#pragma unroll
            for (int i = 0; i < G; ++i) {
                const float v = REAL ? pr[i] : p[i];
                sa += i < hi ? v : 0.f;
                sb += i < hi ? 0.f : v;
            }
            fold_add(a, hsum, hcnt, sub0, bin0, sa, (uint32_t)hi, flags);
            fold_add(a, hsum, hcnt, sub0, bin15, sb, (uint32_t)(G - hi), flags);
        } else {
            for (int i = 0; i < G; ++i) {
                double ti;
                const int bi = fold_bin(f0i + i, fnf, a.inv_pfs, a.nbins, &ti);
                const int64_t si = a.subint > 0 ? subint_rel(d0 + (REAL ? i / 2 : i), a.subint, inv_s) : 0;
                fold_add(a, hsum, hcnt, si, bi, REAL ? pr[i] : p[i], 1, flags);
            }
        }
    }
    if (flags) atomicOr(a.status, flags);
    if (!a.global_mode) {
        __syncthreads();
        uint64_t* ps = a.part_sum + (int64_t)blockIdx.x * a.entries;
        uint32_t* pc = a.part_cnt + (int64_t)blockIdx.x * a.entries;
        for (int i = threadIdx.x; i < a.entries; i += blockDim.x) {
            ps[i] = hsum[i];
            pc[i] = hcnt[i];
        }
    }
}

template <class T, int FORM, int LOG2N2>
static hipError_t k3_one(const K3Args& a, int grid, size_t dyn, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k3_colinv_detect_fold<LOG2N2, T, FORM>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)(160 * 1024 - K3Shape<LOG2N2>::lds(FORM)));
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k3_colinv_detect_fold<LOG2N2, T, FORM>), dim3(grid), dim3(1 << LOG2N2), dyn, s, a);
    return hipGetLastError();
}

template <class T, int FORM>
static hipError_t k3_dispatch(int log2n2, const K3Args& a, int grid, size_t dyn, hipStream_t s) {
    switch (log2n2) {
        case 5: return k3_one<T, FORM, 5>(a, grid, dyn, s);
        case 6: return k3_one<T, FORM, 6>(a, grid, dyn, s);
        case 7: return k3_one<T, FORM, 7>(a, grid, dyn, s);
        case 8: return k3_one<T, FORM, 8>(a, grid, dyn, s);
        case 9: return k3_one<T, FORM, 9>(a, grid, dyn, s);
        case 10: return k3_one<T, FORM, 10>(a, grid, dyn, s);
        default: return hipErrorInvalidValue;
    }
}

template <class T, int LOG2N2>
static hipError_t k3_real_one(const K3Args& a, int grid, size_t dyn, hipStream_t s) {
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k3_colinv_detect_fold<LOG2N2, T, kFormF32, true>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)(160 * 1024 - K3Shape<LOG2N2>::LDS));
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k3_colinv_detect_fold<LOG2N2, T, kFormF32, true>), dim3(grid), dim3(1 << LOG2N2), dyn, s, a);
    return hipGetLastError();
}

template <class T>
static hipError_t k3_real_dispatch(int log2n2, const K3Args& a, int grid, size_t dyn, hipStream_t s) {
    switch (log2n2) {
        case 5: return k3_real_one<T, 5>(a, grid, dyn, s);
        case 6: return k3_real_one<T, 6>(a, grid, dyn, s);
        case 7: return k3_real_one<T, 7>(a, grid, dyn, s);
        case 8: return k3_real_one<T, 8>(a, grid, dyn, s);
        case 9: return k3_real_one<T, 9>(a, grid, dyn, s);
        case 10: return k3_real_one<T, 10>(a, grid, dyn, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_k3_real(int prec, int log2n2, const K3Args& a, int grid, size_t dyn, hipStream_t s) {
    switch (prec) {
        case kFp32: return k3_real_dispatch<float2>(log2n2, a, grid, dyn, s);
        case kMixedValu: return k3_real_dispatch<__half2>(log2n2, a, grid, dyn, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_k3(int prec, int log2n2, const K3Args& a, int grid, size_t dyn, hipStream_t s) {
    switch (prec) {
        case kMixed: return k3_dispatch<__half2, kFormMfma>(log2n2, a, grid, dyn, s);
        case kMixedValu: return k3_dispatch<__half2, kFormF32>(log2n2, a, grid, dyn, s);
        case kHalf: return k3_dispatch<__half2, kFormF16>(log2n2, a, grid, dyn, s);
        case kBf16: return k3_dispatch<bf16x2, kFormF32>(log2n2, a, grid, dyn, s);
        default: return k3_dispatch<float2, kFormF32>(log2n2, a, grid, dyn, s);
    }
}

int64_t hist_capacity(int log2n2, int prec) {
    const int64_t cap = (int64_t)((kLdsBytes - k3_static_lds(log2n2, prec)) / 12);
    return cap < kHistCapMax ? cap : kHistCapMax;
}

int k3_grid(int log2n2, int prec, size_t dyn_lds, int64_t items, int64_t entries, bool global_mode,
            int64_t part_entries) {
    const size_t lds = k3_static_lds(log2n2, prec) + dyn_lds;
    int per_cu = (int)(kLdsBytes / lds);
    per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
    int64_t grid = 256 * per_cu;
    if (!global_mode && grid * entries > part_entries) grid = part_entries / entries;
    const int64_t items8 = (items + 7) & ~int64_t(7);
    if (grid > items8) grid = items8;
    grid &= ~int64_t(7);
    if (grid < 8) grid = 8;
    return (int)grid;
}

size_t k3_static_lds(int log2n2, int prec) {
    if (prec != kHalf && prec != kMixed) return sizeof(float2) * 16 * ((size_t)1 << log2n2);
    switch (log2n2) {
        case 5: return K3Shape<5>::LDS_HALF;
        case 6: return K3Shape<6>::LDS_HALF;
        case 7: return K3Shape<7>::LDS_HALF;
        case 8: return K3Shape<8>::LDS_HALF;
        case 9: return K3Shape<9>::LDS_HALF;
        default: return K3Shape<10>::LDS_HALF;
    }
}
int k1_threads(int log2n2) { return 1 << log2n2; }
int k3_threads(int log2n2) { return 1 << log2n2; }
int k2_threads(int log2n1) {
    const int tpv = (1 << log2n1) / 16;
    return tpv >= 256 ? tpv : 256;
}

// The host-side table scale must match the device schedule.
static_assert(half_row_rem(5) == Sched<5>::kHalfRem && half_row_rem(6) == Sched<6>::kHalfRem &&
                  half_row_rem(7) == Sched<7>::kHalfRem && half_row_rem(8) == Sched<8>::kHalfRem &&
                  half_row_rem(9) == Sched<9>::kHalfRem && half_row_rem(10) == Sched<10>::kHalfRem &&
                  half_row_rem(11) == Sched<11>::kHalfRem && half_row_rem(12) == Sched<12>::kHalfRem &&
                  half_row_rem(13) == Sched<13>::kHalfRem && half_row_rem(14) == Sched<14>::kHalfRem,
              "row normalisation split");
}  // namespace pond
