// K1: int8 unpack and forward column FFTs of the four-step transform
// (length n2, stride n1), written as rows [k2][n1].
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "pond_device.hpp"

namespace pond {

// AIP: the input is two real-sampled channels interleaved (A0 B0 A1 B1 ...);
// element m packs the added-in-phase samples 2m and 2m+1 as (re, im), so a
// block of 2N real samples is read as N complex elements of 4 bytes.
// The packed-float16 tile (about 69 KB at n2 = 2^10) lets two workgroups
// share a CU, if each thread stays within 64 registers.
template <int LOG2N2, class T, int FORM, bool AIP = false>
__global__ void __launch_bounds__(1 << LOG2N2) k1_unpack_colfft(K1Args a) {
    constexpr int BPE = AIP ? 4 : 2;  // input bytes per element
    constexpr int L = 1 << LOG2N2;
    constexpr int TPV = L / 16;
    __shared__ LdsVal<FORM> lds[ColLds<LdsVal<FORM>, true>::kSlots(L)];

    const int n1 = 1 << a.log2n1;
    const int tiles_per_block = n1 >> 4;
    const int ntiles = a.nblocks * tiles_per_block;
    const int tile = xcd_logical(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int b = tile / tiles_per_block;
    const int t = tile - b * tiles_per_block;
    const int c = threadIdx.x & 15;
    const int j = threadIdx.x >> 4;
    const int col = 16 * t + c;

    // Block samples [0, split) come from the carried tail, the rest from
    // this call's input; both bases are uniform, offsets are 32-bit.  Every
    // block but the one that straddles the tail's end reads one buffer
    // only (UNI: no per-sample choice of base).
    const int64_t bstart = (a.block0 + b) * a.hop;
    const int64_t split64 = a.in_start - bstart;
    const uint32_t split = split64 <= 0 ? 0u : (uint32_t)min(split64, (int64_t)1 << (a.log2n1 + LOG2N2));
    const int8_t* tbase = a.tail + BPE * (bstart - a.tail_start);
    const int8_t* ibase = a.in + BPE * (bstart - a.in_start);
    const bool one_src = split == 0 || split == (uint32_t)1 << (a.log2n1 + LOG2N2);
    const int8_t* ubase = uniform_ptr(split == 0 ? ibase : tbase);
    const uint32_t o0 = opaque((uint32_t)col);
    // Address of value e (position j + TPV e) of the thread; UNI: a uniform
    // base advanced by whole rows, plus the thread's own 32-bit offset.
    const uint32_t uoff = BPE * (o0 + ((uint32_t)j << a.log2n1));
    auto src_pos = [&](int pos) -> const int8_t* {
        const uint32_t off = o0 + ((uint32_t)pos << a.log2n1);
        return off < split ? tbase + BPE * off : ibase + BPE * off;
    };
    auto src = [&](int e, auto uni) -> const int8_t* {
        if constexpr (decltype(uni)::value) return at(ubase + ((int64_t)(BPE * TPV * e) << a.log2n1), uoff);
        else return src_pos(j + TPV * e);
    };
    auto cvt_in = [](const int8_t* p) {
        if constexpr (AIP) {
            const int w = *reinterpret_cast<const int*>(p);
            return make_float2((float)((int)(int8_t)(w & 0xff) + (int)(int8_t)((w >> 8) & 0xff)),
                               (float)((int)(int8_t)((w >> 16) & 0xff) + (int)(int8_t)(w >> 24)));
        } else {
            const short s = *reinterpret_cast<const short*>(p);
            return make_float2((float)(int8_t)(s & 0xff), (float)(int8_t)(s >> 8));
        }
    };
    // Loads of the 16 values of the thread, with or without the choice.
    auto load_all = [&](auto&& each) {
        if (one_src) {
#pragma unroll
            for (int e = 0; e < 16; ++e) each(e, std::true_type{});
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) each(e, std::false_type{});
        }
    };
    T* out = reinterpret_cast<T*>(a.work) + ((int64_t)b << (a.log2n1 + LOG2N2));
    if constexpr (FORM == kFormF16 || FORM == kFormMfma) {
        // Packed float16: int8 is exact in float16; the first stage's 1/16
        // is applied here, the even stages scale themselves, and the rest
        // of the 1/n2 normalisation is applied on output, so no value
        // exceeds 16x the input bound.  Matrix-core form: the radix-16
        // stages' butterfly sums on the matrix cores (inputs loaded in
        // their layout), the same numbers otherwise.
        constexpr bool MX = FORM == kFormMfma && kMxShape<LOG2N2, true>;
        StageBases<LOG2N2, h2> tb;
        tb.load(j, a.tw2);
        __shared__ __align__(16) h2 ttab[TwTab<LOG2N2>::kSize];
        if (threadIdx.x < 64) fill_twiddle_tables<LOG2N2, 64>(ttab, a.tw2, threadIdx.x);  // one wave
        // int8 pair -> float16 pair / 16, exactly: the bytes, sign bit
        // flipped, become the low mantissa bits of 1024 (1152 + x), and
        // (1152 + x) / 16 - 72 = x / 16 is representable.
        auto unpack = [](const int8_t* p) {
            const uint32_t s = *reinterpret_cast<const uint16_t*>(p);
            const uint32_t w = ((s & 0xffu) | ((s & 0xff00u) << 8)) ^ 0x64806480u;
            return __builtin_elementwise_fma(__builtin_bit_cast(h2, w), h2{(_Float16)0.0625f, (_Float16)0.0625f},
                                             h2{(_Float16)-72.0f, (_Float16)-72.0f});
        };
        h2 v[16];
        if constexpr (MX) {
            // value e = 4b + t at position 4 (j / 4) + b + (4 (j mod 4) + t) TPV
            const uint32_t mxoff = BPE * (o0 + ((uint32_t)(4 * (j >> 2) + 4 * (j & 3) * TPV) << a.log2n1));
            if (one_src) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    v[e] = unpack(at(ubase + ((int64_t)(BPE * ((e >> 2) + (e & 3) * TPV)) << a.log2n1), mxoff));
            } else {
#pragma unroll
                for (int e = 0; e < 16; ++e) v[e] = unpack(src_pos(mx_pos<true, TPV>(j, e)));
            }
            fft_mx<LOG2N2, -1, true, true, false>(v, j, lds + c, ttab);  // first LDS use
        } else {
            load_all([&](int e, auto uni) { v[e] = unpack(src(e, uni)); });
            fft_wg<LOG2N2, -1, true, 2, false>(v, j, tb, ColLds<h2, true>{lds + c}, ttab);  // first LDS use
        }
        constexpr float osc = 1.0f / (float)(1 << Sched<LOG2N2>::kHalfRem);
        const uint32_t woff = (opaque((uint32_t)col) + ((uint32_t)j << a.log2n1)) * (uint32_t)sizeof(T);
        T* const ob = uniform_ptr(out);
#pragma unroll
        for (int e = 0; e < 16; ++e) st_h2(at(ob + ((int64_t)(TPV * e) << a.log2n1), woff), v[e] * (_Float16)osc);
    } else {
        StageBases<LOG2N2> tb;
        tb.load(j, a.tw2);
        {
            float2 v[16];
            load_all([&](int e, auto uni) { v[e] = cvt_in(src(e, uni)); });
            fft_wg<LOG2N2, -1, false, false, false>(v, j, tb, ColLds<float2, true>{lds + c});  // first LDS use
            const uint32_t woff = (opaque((uint32_t)col) + ((uint32_t)j << a.log2n1)) * (uint32_t)sizeof(T);
            T* const ob = uniform_ptr(out);
#pragma unroll
            for (int e = 0; e < 16; ++e)
                Elem<T>::store(at(ob + ((int64_t)(TPV * e) << a.log2n1), woff), cscale(v[e], a.scale));
        }
    }
}

// The same pass for blocks that overlap by half (hop = N / 2, a discard of
// N / 2: the production shape and every DM-search group), one workgroup
// taking its column tile in `chain` consecutive blocks.  Thread j holds rows
// j + TPV e; block b + 1 starts N / 2 = 8 TPV rows of n1 samples after block
// b, so its rows with e < 8 are block b's rows with e + 8, already loaded:
// each block after the first reads only its second half (the input is read
// (chain + 1) / (2 chain) as often), and those loads are issued before the
// previous block's transform, so that their latency is hidden behind it.
// The values and the arithmetic are those of k1_unpack_colfft (AIP: the
// real two-channel input, 4 bytes per element, float32 arithmetic forms).
template <int LOG2N2, class T, int FORM, bool AIP = false>
__global__ void __launch_bounds__(1 << LOG2N2)
    __attribute__((amdgpu_waves_per_eu(FORM == kFormF16 ? 8 : 4)))  // float16: two workgroups per CU
k1_chain_colfft(K1Args a) {
    static_assert(FORM == kFormF16 || FORM == kFormF32, "VALU forms");
    static_assert(!AIP || FORM == kFormF32, "the real input path has float32 arithmetic");
    constexpr int BPE = AIP ? 4 : 2;  // input bytes per element
    constexpr int L = 1 << LOG2N2;
    constexpr int TPV = L / 16;
    constexpr bool H16 = FORM == kFormF16;
    using V = std::conditional_t<H16, h2, float2>;
    __shared__ LdsVal<FORM> lds[ColLds<LdsVal<FORM>, true>::kSlots(L)];

    const int n1 = 1 << a.log2n1;
    const int tiles_per_block = n1 >> 4;
    const int nchains = (a.nblocks + a.chain - 1) / a.chain;
    const int logical = xcd_logical(blockIdx.x, gridDim.x);
    if (logical >= nchains * tiles_per_block) return;
    const int ch = logical / tiles_per_block;
    const int t = logical - ch * tiles_per_block;
    const int bfirst = ch * a.chain;
    const int bend = min(a.nblocks, bfirst + a.chain);
    const int c = threadIdx.x & 15;
    const int j = threadIdx.x >> 4;
    const int col = 16 * t + c;
    const uint32_t o0 = opaque((uint32_t)col);
    const uint32_t uoff = (uint32_t)BPE * (o0 + ((uint32_t)j << a.log2n1));

    // raw int8 pairs of values e = E0 .. 15 of block b, which lies in the
    // carried tail or in the call's input entirely (launch_k1 uses this
    // pass only then)
    auto load_raw = [&](int b, auto e0, uint32_t (&r)[16]) {
        constexpr int E0 = decltype(e0)::value;
        const int64_t bstart = (a.block0 + b) * a.hop;
        const int8_t* ub = uniform_ptr(bstart >= a.in_start ? a.in + BPE * (bstart - a.in_start)
                                                            : a.tail + BPE * (bstart - a.tail_start));
#pragma unroll
        for (int e = E0; e < 16; ++e) {
            const int8_t* p = at(ub + ((int64_t)(BPE * TPV * e) << a.log2n1), uoff);
            if constexpr (AIP) r[e] = *reinterpret_cast<const uint32_t*>(p);
            else r[e] = *reinterpret_cast<const uint16_t*>(p);
        }
    };
    // int8 pair -> value (packed float16: exact, scaled by 1/16 as in
    // k1_unpack_colfft; float32: exact)
    auto unpack = [](uint32_t s) -> V {
        if constexpr (H16) {
            const uint32_t w = ((s & 0xffu) | ((s & 0xff00u) << 8)) ^ 0x64806480u;
            return __builtin_elementwise_fma(__builtin_bit_cast(h2, w), h2{(_Float16)0.0625f, (_Float16)0.0625f},
                                             h2{(_Float16)-72.0f, (_Float16)-72.0f});
        } else if constexpr (AIP) {
            // samples 2m and 2m+1 of channels A and B, added in phase
            return make_float2((float)((int)(int8_t)(s & 0xff) + (int)(int8_t)((s >> 8) & 0xff)),
                               (float)((int)(int8_t)((s >> 16) & 0xff) + (int)(int8_t)(s >> 24)));
        } else {
            return make_float2((float)(int8_t)(s & 0xff), (float)(int8_t)((s >> 8) & 0xff));
        }
    };

    StageBases<LOG2N2, V> tb;
    tb.load(j, a.tw2);
    __shared__ __align__(16) h2 ttab[H16 ? TwTab<LOG2N2>::kSize : 1];
    if constexpr (H16) {
        if (threadIdx.x < 64) fill_twiddle_tables<LOG2N2, 64>(ttab, a.tw2, threadIdx.x);  // one wave
    }
    const uint32_t woff = (opaque((uint32_t)col) + ((uint32_t)j << a.log2n1)) * (uint32_t)sizeof(T);

    uint32_t r[16];
    load_raw(bfirst, std::integral_constant<int, 0>{}, r);
    V v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = unpack(r[e]);
    for (int b = bfirst; b < bend; ++b) {
        V keep[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) keep[e] = v[e + 8];
        if (b + 1 < bend) load_raw(b + 1, std::integral_constant<int, 8>{}, r);
        // lead barrier: the previous block's transform may still be read
        if constexpr (H16) fft_wg<LOG2N2, -1, true, 2, true>(v, j, tb, ColLds<h2, true>{lds + c}, ttab);
        else fft_wg<LOG2N2, -1, false, false, true>(v, j, tb, ColLds<float2, true>{lds + c});
        T* const ob = uniform_ptr(reinterpret_cast<T*>(a.work) + ((int64_t)b << (a.log2n1 + LOG2N2)));
        if constexpr (H16) {
            constexpr float osc = 1.0f / (float)(1 << Sched<LOG2N2>::kHalfRem);
#pragma unroll
            for (int e = 0; e < 16; ++e)
                st_h2(at(ob + ((int64_t)(TPV * e) << a.log2n1), woff), v[e] * (_Float16)osc);
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                Elem<T>::store(at(ob + ((int64_t)(TPV * e) << a.log2n1), woff), cscale(v[e], a.scale));
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            v[e] = keep[e];
            v[e + 8] = unpack(r[e + 8]);
        }
    }
}

// ---------------------------------------------------------- launchers
// Blocks per workgroup of the chained pass: at most kK1Chain, the launch's
// blocks spread evenly over the chains.
constexpr int kK1Chain = 4;

template <class T, int FORM, int LOG2N2>
static hipError_t k1_one(const K1Args& a, hipStream_t s) {
    const int tiles_per_block = (1 << a.log2n1) >> 4;
    // half-overlapping blocks: the chained pass (VALU forms)
    // half-overlapping blocks, none straddling the end of the carried tail
    const int64_t n = (int64_t)1 << (a.log2n1 + LOG2N2);
    const int64_t first = a.block0 * a.hop, last = (a.block0 + a.nblocks - 1) * a.hop;
    // (the blocks cover [first, last + n) without gaps, so a tail end
    // strictly inside that range falls strictly inside some block)
    const bool straddle = first < a.in_start && a.in_start < last + n;
    // Where blocks overlap by half, plans of the matrix-core form ask for the
    // packed-float16 column pass (f16_cols), chained or not: the matrix-core
    // load layout puts the shifted rows in another thread (32 lanes up),
    // and keeping them for the hand-off spills, so the chained VALU pass,
    // which reads half the input, is the faster column pass there (the
    // matrix cores carry the form's row pass and inverse column pass).
    const bool half_overlap = (a.hop << 1) == n;
    const bool mx16 = FORM == kFormMfma && a.f16_cols;
    const bool chained = a.nblocks >= 2 && half_overlap && !straddle && (FORM != kFormMfma || mx16);
    constexpr int CFORM = FORM == kFormMfma ? kFormF16 : FORM;
    if (chained) {
        K1Args c = a;
        const int nchains = (a.nblocks + kK1Chain - 1) / kK1Chain;
        c.chain = (a.nblocks + nchains - 1) / nchains;
        const int grid = ((a.nblocks + c.chain - 1) / c.chain * tiles_per_block + 7) & ~7;
        hipLaunchKernelGGL((k1_chain_colfft<LOG2N2, T, CFORM>), dim3(grid), dim3(1 << LOG2N2), 0, s, c);
        return hipGetLastError();
    }
    const int grid = (a.nblocks * tiles_per_block + 7) & ~7;
    if (mx16)
        hipLaunchKernelGGL((k1_unpack_colfft<LOG2N2, T, CFORM>), dim3(grid), dim3(1 << LOG2N2), 0, s, a);
    else
        hipLaunchKernelGGL((k1_unpack_colfft<LOG2N2, T, FORM>), dim3(grid), dim3(1 << LOG2N2), 0, s, a);
    return hipGetLastError();
}

template <class T, int FORM>
static hipError_t k1_dispatch(int log2n2, const K1Args& a, hipStream_t s) {
    switch (log2n2) {
        case 5: return k1_one<T, FORM, 5>(a, s);
        case 6: return k1_one<T, FORM, 6>(a, s);
        case 7: return k1_one<T, FORM, 7>(a, s);
        case 8: return k1_one<T, FORM, 8>(a, s);
        case 9: return k1_one<T, FORM, 9>(a, s);
        case 10: return k1_one<T, FORM, 10>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <class T, int LOG2N2>
static hipError_t k1_aip_one(const K1Args& a, hipStream_t s) {
    const int tiles_per_block = (1 << a.log2n1) >> 4;
    // half-overlapping blocks, none straddling the end of the carried tail:
    // the chained pass (as in k1_one)
    const int64_t n = (int64_t)1 << (a.log2n1 + LOG2N2);
    const int64_t first = a.block0 * a.hop, last = (a.block0 + a.nblocks - 1) * a.hop;
    const bool straddle = first < a.in_start && a.in_start < last + n;
    if (a.nblocks >= 2 && (a.hop << 1) == n && !straddle) {
        K1Args c = a;
        const int nchains = (a.nblocks + kK1Chain - 1) / kK1Chain;
        c.chain = (a.nblocks + nchains - 1) / nchains;
        const int grid = ((a.nblocks + c.chain - 1) / c.chain * tiles_per_block + 7) & ~7;
        hipLaunchKernelGGL((k1_chain_colfft<LOG2N2, T, kFormF32, true>), dim3(grid), dim3(1 << LOG2N2), 0, s, c);
        return hipGetLastError();
    }
    const int grid = (a.nblocks * tiles_per_block + 7) & ~7;
    hipLaunchKernelGGL((k1_unpack_colfft<LOG2N2, T, kFormF32, true>), dim3(grid), dim3(1 << LOG2N2), 0, s, a);
    return hipGetLastError();
}

template <class T>
static hipError_t k1_aip_dispatch(int log2n2, const K1Args& a, hipStream_t s) {
    switch (log2n2) {
        case 5: return k1_aip_one<T, 5>(a, s);
        case 6: return k1_aip_one<T, 6>(a, s);
        case 7: return k1_aip_one<T, 7>(a, s);
        case 8: return k1_aip_one<T, 8>(a, s);
        case 9: return k1_aip_one<T, 9>(a, s);
        case 10: return k1_aip_one<T, 10>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_k1_aip(int prec, int log2n2, const K1Args& a, hipStream_t s) {
    switch (prec) {
        case kFp32: return k1_aip_dispatch<float2>(log2n2, a, s);
        case kMixedValu: return k1_aip_dispatch<__half2>(log2n2, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_k1(int prec, int log2n2, const K1Args& a, hipStream_t s) {
    switch (prec) {
        case kMixed: return k1_dispatch<__half2, kFormMfma>(log2n2, a, s);
        case kMixedValu: return k1_dispatch<__half2, kFormF32>(log2n2, a, s);
        case kHalf: return k1_dispatch<__half2, kFormF16>(log2n2, a, s);
        case kBf16: return k1_dispatch<bf16x2, kFormF32>(log2n2, a, s);
        default: return k1_dispatch<float2, kFormF32>(log2n2, a, s);
    }
}

}  // namespace pond
