// HIP kernels of the coherent-dedispersion + fold path (gfx950).
//
// One overlap-save block of n = n1 * n2 samples is transformed with the
// four-step factorisation (input index n = n1_ + n1 * n2_, spectrum index
// k = k2 + n2 * k1):
//   K1  column FFTs of length n2 over the int8 input (stride n1), written as
//       rows [k2][n1];
//   K2  per row k2: twiddle W_n^(n1_ k2), forward row FFT of length n1,
//       multiply bin k by the inverse ISM response exp(-2 pi i turns_k)
//       (Sec. 3.7, Eq. (4); turns in float64 reduced mod 1 before the
//       float32 sine/cosine), inverse row FFT, twiddle W_n^-(n1_ k2);
//   K3  inverse column FFTs of length n2, 1/n scaling, |y|^2 (square-law
//       detection), sums of `decim` consecutive powers (the integrated time
//       series of Sec. 4) and the fold of every kept output into
//       (sub-integration, bin) accumulators (Sec. 3.4.1 / Sec. 3.7).
// Only K1 reads the input and only K3 produces outputs, so one block costs
// three passes over its complex intermediate.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "pond_fft.hpp"
#include "pond_internal.hpp"

namespace pond {

// --------------------------------------------------------- storage forms
template <class T>
struct Elem;
template <>
struct Elem<float2> {
    __device__ __forceinline__ static float2 load(const float2* p) { return *p; }
    __device__ __forceinline__ static void store(float2* p, float2 v) { *p = v; }
};
template <>
struct Elem<__half2> {
    __device__ __forceinline__ static float2 load(const __half2* p) { return __half22float2(*p); }
    __device__ __forceinline__ static void store(__half2* p, float2 v) { *p = __float22half2_rn(v); }
};

// Access at a uniform base pointer plus a 32-bit byte offset (lets the
// compiler use the scalar-base + vector-offset addressing form).
template <class T>
__device__ __forceinline__ const T* at(const T* base, uint32_t byte_off) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ T* at(T* base, uint32_t byte_off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}
// A pointer that is the same in every lane, moved to scalar registers, so
// that bases derived from it stay scalar.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}
// Hide a value from the optimiser so that expressions depending on it are
// recomputed where used instead of being hoisted and kept in registers.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}

// ------------------------------------------------------------------- K1
// Arithmetic of a kernel instance: float32 vector, float16 matrix-core
// DFT-16 stages (float32 elsewhere), or packed float16 vector.
constexpr int kFormF32 = 0, kFormMfma = 1, kFormF16 = 2;

template <int FORM>
using LdsVal = std::conditional_t<FORM == kFormF16, h2, float2>;

// Float16 pair for the complex value (c, s) of magnitude m (float64 in):
// among the neighbouring float16 values of each component, the pair whose
// squared magnitude is closest to m^2.  Nearest rounding of each component
// would leave |w|^2 errors of ~3e-4 that do not average out over a small
// table (every stage of every block reuses the same few hundred entries).
__device__ __forceinline__ void f16_neighbours(double x, _Float16 (&h)[2]) {
    h[0] = (_Float16)x;
    const uint16_t b = __builtin_bit_cast(uint16_t, h[0]);
    const double d = (double)h[0];
    uint16_t o;
    if (d == x) o = b;
    else if ((d < x) == (d >= 0.0 && !(b & 0x8000u))) o = (uint16_t)(b + 1);  // away from zero
    else o = (b & 0x7fffu) ? (uint16_t)(b - 1) : (uint16_t)(b ^ 0x8000u);     // toward zero (or past it)
    h[1] = __builtin_bit_cast(_Float16, o);
}
__device__ __forceinline__ h2 f16_unit(double c, double s, double m) {
    _Float16 hc[2], hs[2];
    f16_neighbours(c, hc);
    f16_neighbours(s, hs);
    h2 best = {hc[0], hs[0]};
    double be = 1e300;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double cc = (double)hc[i], ss = (double)hs[k];
            const double err = fabs(cc * cc + ss * ss - m * m);
            if (err < be) {
                be = err;
                best = h2{hc[i], hs[k]};
            }
        }
    return best;
}

// Reinterpret float16 storage as a packed pair.
__device__ __forceinline__ h2 ld_h2(const __half2* p) { return *reinterpret_cast<const h2*>(p); }
__device__ __forceinline__ void st_h2(__half2* p, h2 v) { *reinterpret_cast<h2*>(p) = v; }

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
    if constexpr (FORM == kFormF16) {
        // Packed float16: int8 is exact in float16; the first stage's 1/16
        // is applied here, the even stages scale themselves, and the rest
        // of the 1/n2 normalisation is applied on output, so no value
        // exceeds 16x the input bound.
        StageBases<LOG2N2, h2> tb;
        tb.load(j, a.tw2);
        // int8 pair -> float16 pair / 16, exactly: the bytes, sign bit
        // flipped, become the low mantissa bits of 1024 (1152 + x), and
        // (1152 + x) / 16 - 72 = x / 16 is representable.
        h2 v[16];
        load_all([&](int e, auto uni) {
            const uint32_t s = *reinterpret_cast<const uint16_t*>(src(e, uni));
            const uint32_t w = ((s & 0xffu) | ((s & 0xff00u) << 8)) ^ 0x64806480u;
            v[e] = __builtin_elementwise_fma(__builtin_bit_cast(h2, w), h2{(_Float16)0.0625f, (_Float16)0.0625f},
                                             h2{(_Float16)-72.0f, (_Float16)-72.0f});
        });
        fft_wg<LOG2N2, -1, true, false, false>(v, j, tb, ColLds<h2, true>{lds + c});  // first LDS use: no lead barrier
        constexpr float osc = 1.0f / (float)(1 << Sched<LOG2N2>::kHalfRem);
        const uint32_t woff = (opaque((uint32_t)col) + ((uint32_t)j << a.log2n1)) * (uint32_t)sizeof(T);
        T* const ob = uniform_ptr(out);
#pragma unroll
        for (int e = 0; e < 16; ++e) st_h2(at(ob + ((int64_t)(TPV * e) << a.log2n1), woff), v[e] * (_Float16)osc);
    } else {
        StageBases<LOG2N2> tb;
        tb.load(j, a.tw2);
        if constexpr (FORM == kFormMfma && LOG2N2 >= 6) {
            // Normalised forward pass (1/16 per radix-16 stage, folded into
            // the DFT matrix): no float16 value can exceed the input range.
            const uint32_t w0 = opaque((uint32_t)col);
            colfft_mfma<LOG2N2, -1, false>(
                c, j, a.tw2, tb, 1.0f / 16.0f, 1.0f / (float)Sched<LOG2N2>::kRem,
                [&](int pos) { return cvt_in(src_pos(pos)); },
                [&](int pos) -> float2& { return lds[pos * 16 + c]; },
                [&](int pos, float2 y) {
                    Elem<T>::store(at(out, (w0 + ((uint32_t)pos << a.log2n1)) * (uint32_t)sizeof(T)), y);
                });
        } else {
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

// ------------------------------------------------------------------- K2
template <int LOG2N1>
struct K2Shape {
    static constexpr int L = 1 << LOG2N1;
    static constexpr int TPV = L / 16;
    static constexpr int ROWS = TPV >= 256 ? 1 : 256 / TPV;
    static constexpr int THREADS = ROWS * TPV;
    static constexpr int STRIDE = L + L / 16;  // LDS row stride: one pad slot per 16 values
};

// Frequency-domain taper of the inverse filter at baseband frequency f
// (MHz): a Tukey window of edge fraction alpha over [-bw/2, bw/2]
// (alpha = 0: unit taper).  The paper applies an unspecified taper with the
// inverse ISM response against leakage of the square window (Sec. 3.7).
__device__ __forceinline__ double taper_w(double f, double bw, double alpha) {
    if (!(alpha > 0.0)) return 1.0;
    const double af = fabs(f), flat = (1.0 - alpha) * bw * 0.5, edge = alpha * bw * 0.5;
    if (af <= flat) return 1.0;
    return 0.5 * (1.0 + cos(M_PI * fmin(af - flat, edge) / edge));
}

// Row table of the middle pass, one float4 per (k2, k1):
//   (x, y) = W_n^(k1 k2) = exp(-2 pi i (k1 k2 mod n) / n), the four-step twiddle
//   (z, w) = exp(-2 pi i turns_k), k = k2 + n2 k1, the inverse ISM response
//            of Sec. 3.7 / Eq. (4); turns_k and its reduction mod 1 are float64.
// Built once per plan; every block reads the same table.
__global__ void __launch_bounds__(256) k2_build_table(float4* __restrict__ tab, int log2n1, int log2n2,
                                                       double chirp_a, double f0, double df, double taper) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int log2n = log2n1 + log2n2;
    const int64_t n = 1ll << log2n;
    if (i >= n) return;
    const int64_t k2 = i >> log2n1;
    const int64_t k1 = i & ((1ll << log2n1) - 1);
    const int64_t r = (k1 * k2) & (n - 1);
    double s, c;
    sincospi(2.0 * (double)r / (double)n, &s, &c);
    const int64_t k = k2 + (k1 << log2n2);
    const int64_t kk = k < (n >> 1) ? k : k - n;
    const double f = (double)kk * df;
    const double turns = chirp_a * (f * f) / (f0 + f);
    const double frac = turns - rint(turns);
    double cs, cc;
    sincospi(2.0 * frac, &cs, &cc);
    const double w = taper_w(f, df * (double)n, taper);
    tab[i] = make_float4((float)c, (float)-s, (float)(cc * w), (float)(-cs * w));
}

// One workgroup takes row k2 (ROWS rows for short rows) of one block.  The
// workgroups of one row for all blocks of the launch get consecutive logical
// indices on one XCD, so they run together and share the row's table entries
// through that XCD's L2 (the table is then fetched from HBM about once per
// launch).
//   MODE kRowFull: twiddle, forward FFT, chirp, inverse FFT, conjugate
//                  twiddle, in place (float4 table: twiddle, chirp).
//   MODE kRowFwd:  twiddle and forward FFT only, in place: leaves the block's
//                  spectrum, row k2 holding bins k2 + n2 k1 (float2 twiddle table).
//   MODE kRowInv:  spectrum (in) times one trial's chirp (float2 table),
//                  inverse FFT, conjugate twiddle, to `out`.
//   MODE kRowInvPlain: kRowInv without the chirp (float32 arithmetic only).
// F16: packed float16 arithmetic on float16 storage with float16 tables
// (kRowFull: 4 halves per entry, twiddle/16 and chirp*2^-kHalfRem; split
// modes: twiddle/16 and chirp).  The forward transform is normalised stage
// by stage (1/16 of the first stage in the twiddle table), so the spectrum
// is the block's spectrum / n; the output is 1/16 of the float32 forms'.
template <int LOG2N1, class T, int MODE, bool F16>
__global__ void __launch_bounds__(K2Shape<LOG2N1>::THREADS) __attribute__((amdgpu_waves_per_eu(4)))
k2_row(K2Args a) {
    using Sh = K2Shape<LOG2N1>;
    using V = std::conditional_t<F16, h2, float2>;
    constexpr int TPV = Sh::TPV;
    __shared__ V lds[Sh::ROWS * Sh::STRIDE];

    const int logical = xcd_logical(blockIdx.x, gridDim.x);
    const int n2 = 1 << a.log2n2;
    const int row_groups = (n2 + Sh::ROWS - 1) / Sh::ROWS;
    if (logical >= row_groups * a.nblocks) return;
    const int rg = logical / a.nblocks;
    const int b = logical - rg * a.nblocks;

    const int r = threadIdx.x / TPV;
    const int j = threadIdx.x - r * TPV;
    const int row = rg * Sh::ROWS + r;
    const bool valid = row < n2;
    // packed float16 rows of 2^12 and more: per-stage bank-conflict-free layouts
    using RowL = std::conditional_t<F16 && LOG2N1 >= 12, StageRowLds<V>, PadLds<V>>;
    const RowL lrow{lds + r * Sh::STRIDE};
    static_assert(!(F16 && LOG2N1 >= 12) || (Sh::STRIDE >= (1 << LOG2N1) + 16 * ((1 << LOG2N1) >> 8)),
                  "per-stage layouts fit the row");

    StageBases<LOG2N1, V> tb;
    tb.load(j, a.tw1);
    // Uniform base pointers plus 32-bit per-thread offsets (rows beyond n2,
    // possible only for the shortest rows, re-read the last row and never
    // store).
    const int row0 = min(rg * Sh::ROWS, n2 - 1);
    const uint32_t toff = (uint32_t)(min(r, n2 - 1 - row0) << LOG2N1) + (uint32_t)j;
    const int64_t rowbase = (((int64_t)b << a.log2n2) + row0) << LOG2N1;
    T* rows = reinterpret_cast<T*>(a.work) + rowbase;
    constexpr bool INV = MODE == kRowInv || MODE == kRowInvPlain;
    const T* src = INV ? reinterpret_cast<const T*>(a.in) + rowbase : rows;
    T* dst = INV ? reinterpret_cast<T*>(a.out) + rowbase : rows;

    if constexpr (F16) {
        __shared__ h2 s1tab[kS1Pairs];
        fill_stage1_table<LOG2N1>(s1tab, a.tw1, threadIdx.x);
        const uint2* tab = reinterpret_cast<const uint2*>(a.htable) + ((int64_t)row0 << LOG2N1);
        const h2* tw4 = reinterpret_cast<const h2*>(a.htw4) + ((int64_t)row0 << LOG2N1);
        const h2* chirp = reinterpret_cast<const h2*>(a.hchirp) + ((int64_t)row0 << LOG2N1);
        auto tw_at = [&](uint32_t i) {
            if constexpr (MODE == kRowFull) return __builtin_bit_cast(h2, at(tab, i * 8u)->x);
            else return *at(tw4, i * 4u);
        };
        h2 v[16];
        uint32_t to = opaque(toff);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const uint32_t i = to + TPV * e;
            const h2 x = ld_h2(at(src, i * (uint32_t)sizeof(T)));
            if constexpr (MODE == kRowInv) v[e] = cmul(x, *at(chirp, i * 4u));
            else v[e] = cmul(x, tw_at(i));
        }
        // kRowFull: the chirp of each element is fetched during the forward
        // transform's last exchange.
        h2 ch[16];
        auto fetch_chirp = [&] {
            const uint32_t t2 = opaque(toff);
#pragma unroll
            for (int e = 0; e < 16; ++e) ch[e] = __builtin_bit_cast(h2, at(tab, (t2 + TPV * e) * 8u)->y);
        };
        if constexpr (MODE == kRowFull) fft_wg<LOG2N1, -1, true, true>(v, j, tb, lrow, s1tab, fetch_chirp);
        else if constexpr (MODE != kRowInv) fft_wg<LOG2N1, -1, true, true>(v, j, tb, lrow, s1tab);
        if constexpr (MODE == kRowFwd) {
            constexpr float osc = 1.0f / (float)(1 << Sched<LOG2N1>::kHalfRem);
            if (valid) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    st_h2(at(dst, (to + TPV * e) * (uint32_t)sizeof(T)), v[e] * (_Float16)osc);
            }
            return;
        }
        if constexpr (MODE == kRowFull) {
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = cmul(v[e], ch[e]);
        }
        // the output twiddles are fetched during the inverse transform's
        // last exchange (rather than one dependent load per store)
        h2 wo[16];
        auto fetch_tw = [&] {
            const uint32_t t2 = opaque(toff);
#pragma unroll
            for (int e = 0; e < 16; ++e) wo[e] = tw_at(t2 + TPV * e);
        };
        fft_wg<LOG2N1, +1, false, true>(v, j, tb, lrow, s1tab, fetch_tw);
        asm volatile("" ::: "memory");
        to = opaque(toff);
        if (valid) {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                st_h2(at(dst, (to + TPV * e) * (uint32_t)sizeof(T)), cmulc(v[e], wo[e]));
        }
        return;
    } else {
        const float4* tab = a.table + ((int64_t)row0 << LOG2N1);
        const float2* tw4 = a.tw4 + ((int64_t)row0 << LOG2N1);
        const float2* chirp = a.chirp + ((int64_t)row0 << LOG2N1);
        float2 v[16];
        uint32_t to = opaque(toff);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const float2 x = Elem<T>::load(at(src, (to + TPV * e) * (uint32_t)sizeof(T)));
            if constexpr (MODE == kRowFull) {
                const float4 t = *at(tab, (to + TPV * e) * 16u);
                v[e] = cmul(x, make_float2(t.x, t.y));
            } else if constexpr (MODE == kRowFwd) {
                v[e] = cmul(x, *at(tw4, (to + TPV * e) * 8u));
            } else if constexpr (MODE == kRowInv) {
                v[e] = cmul(x, *at(chirp, (to + TPV * e) * 8u));
            } else {
                v[e] = x;  // kRowInvPlain: the filter was applied before (real input path)
            }
        }
        // kRowFull: the chirp is fetched again (from L2) during the forward
        // transform's last exchange rather than kept live across it.
        float2 ch[16];
        auto fetch_chirp = [&] {
            const uint32_t t2 = opaque(toff);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const float4 t = *at(tab, (t2 + TPV * e) * 16u);
                ch[e] = make_float2(t.z, t.w);
            }
        };
        if constexpr (MODE == kRowFull) {
            fft_wg<LOG2N1, -1>(v, j, tb, lrow, nullptr, fetch_chirp);
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = cmul(v[e], ch[e]);
        } else if constexpr (MODE != kRowInv && MODE != kRowInvPlain) {
            fft_wg<LOG2N1, -1>(v, j, tb, lrow);
        }
        if constexpr (MODE == kRowFwd) {
            if (valid) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    Elem<T>::store(at(dst, (to + TPV * e) * (uint32_t)sizeof(T)), cscale(v[e], a.scale));
            }
            return;
        }
        // output twiddles fetched during the inverse transform's last exchange
        float2 wo[16];
        auto fetch_tw = [&] {
            const uint32_t t2 = opaque(toff);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                if constexpr (MODE == kRowFull) {
                    const float4 t = *at(tab, (t2 + TPV * e) * 16u);
                    wo[e] = make_float2(t.x, t.y);
                } else {
                    wo[e] = *at(tw4, (t2 + TPV * e) * 8u);
                }
            }
        };
        fft_wg<LOG2N1, +1>(v, j, tb, lrow, nullptr, fetch_tw);
        asm volatile("" ::: "memory");
        to = opaque(toff);
        if (valid) {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                Elem<T>::store(at(dst, (to + TPV * e) * (uint32_t)sizeof(T)), cscale(cmulc(v[e], wo[e]), a.scale));
        }
    }
}

// Float16 table of the middle pass for the packed-float16 form, 8 bytes per
// (k2, k1): the four-step twiddle / 16 and the inverse ISM response times
// 2^-rem (rem: the part of the row normalisation not applied by the
// transform's stages), both evaluated in float64 as in k2_build_table.
__global__ void __launch_bounds__(256) k2_build_table_h(uint2* __restrict__ tab, int log2n1, int log2n2,
                                                         double chirp_a, double f0, double df, double chirp_scale,
                                                         double taper) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int log2n = log2n1 + log2n2;
    const int64_t n = 1ll << log2n;
    if (i >= n) return;
    const int64_t k2 = i >> log2n1;
    const int64_t k1 = i & ((1ll << log2n1) - 1);
    const int64_t r = (k1 * k2) & (n - 1);
    double s, c;
    sincospi(2.0 * (double)r / (double)n, &s, &c);
    const int64_t k = k2 + (k1 << log2n2);
    const int64_t kk = k < (n >> 1) ? k : k - n;
    const double f = (double)kk * df;
    const double turns = chirp_a * (f * f) / (f0 + f);
    const double frac = turns - rint(turns);
    double cs, cc;
    sincospi(2.0 * frac, &cs, &cc);
    const h2 tw = f16_unit(c / 16.0, -s / 16.0, 1.0 / 16.0);
    const double m = chirp_scale * taper_w(f, df * (double)n, taper);
    const h2 ch = f16_unit(cc * m, -cs * m, m);
    tab[i] = make_uint2(__builtin_bit_cast(uint32_t, tw), __builtin_bit_cast(uint32_t, ch));
}

// Float16 tables of the split middle pass: twiddle / 16 (tw) and, per trial
// DM, the inverse ISM response (chirp).
__global__ void __launch_bounds__(256) k2_build_split_tables_h(h2* __restrict__ tw, h2* __restrict__ chirp,
                                                                int log2n1, int log2n2, double chirp_a, double f0,
                                                                double df) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int log2n = log2n1 + log2n2;
    const int64_t n = 1ll << log2n;
    if (i >= n) return;
    const int64_t k2 = i >> log2n1;
    const int64_t k1 = i & ((1ll << log2n1) - 1);
    if (tw) {
        const int64_t r = (k1 * k2) & (n - 1);
        double s, c;
        sincospi(2.0 * (double)r / (double)n, &s, &c);
        tw[i] = f16_unit(c / 16.0, -s / 16.0, 1.0 / 16.0);
    }
    const int64_t k = k2 + (k1 << log2n2);
    const int64_t kk = k < (n >> 1) ? k : k - n;
    const double f = (double)kk * df;
    const double turns = chirp_a * (f * f) / (f0 + f);
    const double frac = turns - rint(turns);
    double cs, cc;
    sincospi(2.0 * frac, &cs, &cc);
    chirp[i] = f16_unit(cc, -cs, 1.0);
}

// Tables of the split middle pass: tw[i] = W_n^(k1 k2) for i = k2 n1 + k1;
// per trial DM, chirp[i] = exp(-2 pi i turns_k), k = k2 + n2 k1, turns in
// float64 reduced mod 1 (Sec. 3.7 / Eq. (4)).
__global__ void __launch_bounds__(256) k2_build_split_tables(float2* __restrict__ tw, float2* __restrict__ chirp,
                                                              int log2n1, int log2n2, double chirp_a, double f0,
                                                              double df) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int log2n = log2n1 + log2n2;
    const int64_t n = 1ll << log2n;
    if (i >= n) return;
    const int64_t k2 = i >> log2n1;
    const int64_t k1 = i & ((1ll << log2n1) - 1);
    if (tw) {
        const int64_t r = (k1 * k2) & (n - 1);
        double s, c;
        sincospi(2.0 * (double)r / (double)n, &s, &c);
        tw[i] = make_float2((float)c, (float)-s);
    }
    if (!chirp) return;
    const int64_t k = k2 + (k1 << log2n2);
    const int64_t kk = k < (n >> 1) ? k : k - n;
    const double f = (double)kk * df;
    const double turns = chirp_a * (f * f) / (f0 + f);
    const double frac = turns - rint(turns);
    double cs, cc;
    sincospi(2.0 * frac, &cs, &cc);
    chirp[i] = make_float2((float)cc, (float)-cs);
}

// ------------------------------------------------------------------- K3
// Static LDS.  Float32 arithmetic: one float2 tile of 16 columns, reused for
// the detected powers.  Packed float16: the padded float16 tile, a power
// buffer of its own (16 floats per row) and the stage-1 twiddle table, so
// that an item's powers are written without a barrier after the transform
// and the next item's transform starts without one before its first
// exchange.
template <int LOG2N2>
struct K3Shape {
    static constexpr int L = 1 << LOG2N2;
    static constexpr int TPV = L / 16;
    static constexpr int THREADS = L;
    static constexpr size_t LDS = sizeof(float2) * 16 * L;
    static constexpr size_t kHalfTile = ColLds<h2, true>::kSlots(L) * sizeof(h2);
    static constexpr size_t kHalfPf = 16 * L * sizeof(float);
    static constexpr size_t LDS_HALF = kHalfTile + kHalfPf + kS1Pairs * sizeof(h2);
    static constexpr size_t lds(int form) { return form == kFormF16 ? LDS_HALF : LDS; }
};
// Power buffer of the packed-float16 K3: row-major, 16 floats per row, the
// four float4 quarters of a row rotated by (row / 4) mod 4, so that the
// epilogue's float4 reads of 16 consecutive rows (one per lane) and the
// detection's writes of four rows per wave use every bank once.
__device__ __forceinline__ int k3h_pidx(int row, int col) {
    return row * 16 + ((((col >> 2) + (row >> 2)) & 3) << 2) + (col & 3);
}

// Fold phase of output m (float64, as specified): x = (m + n_front) * inv_pfs,
// bin = min(floor(frac(x) * nbins), nbins - 1); also returns floor(x), the
// pulse number, so that equal bins in different periods are told apart.
__device__ __forceinline__ int fold_bin(int64_t m, int64_t n_front, double inv_pfs, int nbins, double* turn) {
    const double x = (double)(m + n_front) * inv_pfs;
    const double fl = floor(x);
    *turn = fl;
    const int bin = (int)((x - fl) * (double)nbins);
    return bin < nbins - 1 ? bin : nbins - 1;
}

// Sub-integration of output m relative to s_base (d = m - s_base*S >= 0),
// without a 64-bit division: float64 estimate, then an exact integer fix-up.
__device__ __forceinline__ int64_t subint_rel(int64_t d, int64_t S, double inv_s) {
    int64_t k = (int64_t)((double)d * inv_s);
    const int64_t r = d - k * S;
    if (r < 0) --k;
    else if (r >= S) ++k;
    return k;
}

// Add `val` (a power or a sum of `cnt` powers) to histogram entry `key`.
__device__ __forceinline__ void fold_add(const K3Args& a, uint64_t* hsum, uint32_t* hcnt, int64_t sub_rel, int bin,
                                         float val, uint32_t cnt, uint32_t& flags) {
    const double dv = (double)val * kFoldScale;
    if (!(dv < kFoldRangeLimit * kFoldScale)) flags |= 2u;
    const uint64_t fx = isfinite(val) ? (uint64_t)__double2ull_rn(dv) : 0ull;
    if (a.global_mode) {
        const int64_t gk = (sub_rel + a.s_base - a.acc_s0) * a.nbins + bin;
        atomicAdd((unsigned long long*)&a.acc_sum[gk], (unsigned long long)fx);
        atomicAdd((unsigned long long*)&a.acc_cnt[gk], (unsigned long long)cnt);
    } else {
        const int key = (int)sub_rel * a.nbins + bin;
        atomicAdd((unsigned long long*)&hsum[key], (unsigned long long)fx);
        atomicAdd(&hcnt[key], cnt);
    }
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
    float* pf = reinterpret_cast<float*>(lds_raw + (FORM == kFormF16 ? Sh::kHalfTile : 0));

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
    h2* s1tab = reinterpret_cast<h2*>(lds_raw + Sh::kHalfTile + Sh::kHalfPf);
    if constexpr (FORM == kFormF16) fill_stage1_table<LOG2N2>(s1tab, a.tw2, threadIdx.x);

    // Float16 storage with VALU arithmetic, columns of 2^9 and 2^10: the
    // next item's column tile is loaded (as float16 pairs) while this one
    // is transformed and folded, so its latency is not exposed once per
    // item (the 16 registers are free there: the LDS already limits the
    // kernel to four waves per SIMD).
    constexpr bool kPrefetch = (FORM == kFormF16 || (FORM == kFormF32 && std::is_same<T, __half2>::value)) &&
                               (LOG2N2 == 10 || (LOG2N2 == 9 && !REAL));  // (else past 128 registers)
    h2 nxt[16];
    auto load_tile = [&](int it, h2(&dst)[16]) {
        const int bb = it >> log2tiles;
        const int tt = it & ((1 << log2tiles) - 1);
        const uint32_t cc = opaque((uint32_t)((r0 + 16 * tt + c) & (n1 - 1)));
        const __half2* const ib =
            uniform_ptr(reinterpret_cast<const __half2*>(a.work) + ((int64_t)bb << (a.log2n1 + LOG2N2)));
        const uint32_t ioff = (cc + ((uint32_t)j << a.log2n1)) * (uint32_t)sizeof(__half2);
#pragma unroll
        for (int e = 0; e < 16; ++e) dst[e] = ld_h2(at(ib + ((int64_t)(TPV * e) << a.log2n1), ioff));
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
        auto load_in = [&](int pos) {
            return Elem<T>::load(at(in, (o0 + ((uint32_t)pos << a.log2n1)) * (uint32_t)sizeof(T)));
        };
        if constexpr (FORM == kFormF16) {
            // Packed float16 inverse transform (unnormalised), then the
            // power in float32 from the float16 pair (exact products).
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
            fft_wg<LOG2N2, +1, false, true, false>(v, j, tb, ColLds<h2, true>{lh + c}, s1tab);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const float yx = (float)v[e].x, yy = (float)v[e].y;
                pf[k3h_pidx(j + TPV * e, c)] = fmaf(yx, yx, yy * yy) * a.pscale;
            }
            __syncthreads();
        } else if constexpr (FORM == kFormMfma && LOG2N2 >= 6) {
            __syncthreads();  // the previous item's epilogue has finished with the LDS
            colfft_mfma<LOG2N2, +1, true>(
                c, j, a.tw2, tb, 1.0f, 1.0f, load_in, [&](int pos) -> float2& { return lds[pos * 16 + c]; },
                [&](int pos, float2 y) {
                    const float2 z = cscale(y, a.scale);
                    pf[pos * PSTRIDE + c] = fmaf(z.x, z.x, z.y * z.y);
                });
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
                    pf + (FORM == kFormF16 ? k3h_pidx(q, 4 * i) : q * PSTRIDE + 4 * i));
                p[4 * i] = x4.x;
                p[4 * i + 1] = x4.y;
                p[4 * i + 2] = x4.z;
                p[4 * i + 3] = x4.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int rsrc = q + ((r0 + 16 * t + i) >> a.log2n1);
                p[i] = rsrc < L ? pf[FORM == kFormF16 ? k3h_pidx(rsrc, i) : rsrc * PSTRIDE + i] : 0.f;
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

__global__ void __launch_bounds__(256) zero_u64(uint64_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ----------------------------------------------------- real input path
// The block holds Z = FFT_N(z) / N of z[m] = x[2m] + i x[2m+1] (x real, 2N
// samples), row k2 / column k1 holding bin k = k2 + n2 k1 (after the
// forward row pass).  Per bin, with its partner bin N - k (row n2 - k2,
// column n1 - 1 - k1; row 0: column -k1 mod n1):
//   E = (Z[k] + conj Z[N-k]) / 2,  O = -i (Z[k] - conj Z[N-k]) / 2
//   X[k] = E + W^k O,  X[N-k] = conj(E - W^k O)      (W = exp(-2 pi i / 2N))
// X are the bins 0..N of the real 2N-point transform.  Y = X M (the real
// path's filter per bin, with the DC and Nyquist factors real), then
//   Z'[k] = e + i o,  e = (Y[k] + conj Y[N-k]) / 2,  o = conj(W^k) (Y[k] - conj Y[N-k]) / 2
//   Z'[N-k] = conj(e) + i conj(o)
// is the N-point spectrum of z'[m] = y[2m] + i y[2m+1], y the filtered real
// signal.  tab[i] = (W^k, M[k]) for the bin k held at position i of the
// block (so that both table reads are contiguous), tab[N] = (-1, M[N]).
// In place: one thread per pair
// {k, N-k} (rows 0..n2/2; on the two rows that pair with themselves, the
// thread of the lower index), which reads and writes both bins.
template <class T>
__global__ void __launch_bounds__(256) real_split(RealSplitArgs a) {
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int log2n = a.log2n1 + a.log2n2;
    const int n1 = 1 << a.log2n1, n2 = 1 << a.log2n2, N = 1 << log2n;
    const int per_block = (n2 / 2 + 1) << a.log2n1;  // rows 0..n2/2
    if (gi >= (int64_t)a.nblocks * per_block) return;
    const int64_t b = gi / per_block;
    const int i = (int)(gi - b * per_block);
    const int k2 = i >> a.log2n1, k1 = i & (n1 - 1);
    const int ip = k2 == 0 ? ((n1 - k1) & (n1 - 1)) : (((n2 - k2) << a.log2n1) + (n1 - 1 - k1));
    if (ip < i) return;  // the pair belongs to the thread of index ip
    T* z = reinterpret_cast<T*>(a.data) + (b << log2n);
    const float2 A = Elem<T>::load(z + i), B = Elem<T>::load(z + ip);
    const float4 tk = a.tab[i], tn = a.tab[i == 0 ? N : ip];
    const float2 w = make_float2(tk.x, tk.y), mk = make_float2(tk.z, tk.w), mn = make_float2(tn.z, tn.w);
    const float2 E = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
    const float2 D = make_float2(0.5f * (A.x - B.x), 0.5f * (A.y + B.y));  // (Z[k] - conj Z[N-k]) / 2
    const float2 O = make_float2(D.y, -D.x);                                // -i D
    const float2 wo = cmul(w, O);
    const float2 yk = cmul(cadd(E, wo), mk);
    const float2 en = csub(E, wo);
    const float2 yn = cmul(make_float2(en.x, -en.y), mn);                    // Y[N-k]
    const float2 ync = make_float2(yn.x, -yn.y);
    const float2 e2 = cscale(cadd(yk, ync), 0.5f);
    const float2 o2 = cmulc(cscale(csub(yk, ync), 0.5f), w);
    Elem<T>::store(z + i, make_float2(e2.x - o2.y, e2.y + o2.x));
    if (ip != i) Elem<T>::store(z + ip, make_float2(e2.x + o2.y, o2.x - e2.y));
}

// Table of the real path's split, in the block's layout: entry i < N (row
// k2 = i / n1, column k1 = i mod n1) holds bin k = k2 + n2 k1, entry N bin
// N; each is (W^k, M[k]) with W^k = exp(-i pi k / N) and M[k] the filter of
// real-transform bin k (baseband k bw / N): upper sideband
// exp(-2 pi i turns(f)), f = k bw/N - bw/2; lower sideband
// exp(+2 pi i turns(f)), f = bw/2 - k bw/N; times the taper; real part only
// at k = 0 and k = N.  Float64, reduced mod 1 turn.
__global__ void __launch_bounds__(256) real_build_table(float4* __restrict__ tab, int log2n1, int log2n2,
                                                         double chirp_a, double f0, double bw, int lsb,
                                                         double taper) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int log2n = log2n1 + log2n2;
    const int64_t N = 1ll << log2n;
    if (i > N) return;
    const int64_t k = i == N ? N : (i >> log2n1) + ((i & ((1ll << log2n1) - 1)) << log2n2);
    double sw, cw;
    sincospi((double)k / (double)N, &sw, &cw);
    const double fb = (double)k * bw / (double)N;
    const double f = lsb ? bw * 0.5 - fb : fb - bw * 0.5;
    const double turns = chirp_a * (f * f) / (f0 + f);
    const double frac = turns - rint(turns);
    double sm, cm;
    sincospi(2.0 * frac, &sm, &cm);
    const double wt = taper_w(f, bw, taper);
    double mx = cm * wt, my = (lsb ? sm : -sm) * wt;
    if (k == 0 || k == N) my = 0.0;
    tab[i] = make_float4((float)cw, (float)-sw, (float)mx, (float)my);
}

// The real path's whole middle pass in one kernel, for rows up to 2^13:
// a workgroup takes row pairs {k2, n2 - k2} (pair 0: rows 0 and n2/2, each
// its own partner), since bin k = k2 + n2 k1 and its partner N - k lie in
// the two rows of one pair.  Per row: four-step twiddle, forward row FFT,
// scale; the pair's spectra meet in LDS, each element takes its partner's
// value and does the split, filter and recombination of real_split for its
// own bin; then inverse row FFT, conjugate twiddle, store (in place).  The
// block therefore crosses HBM once, as in the complex path's middle pass.
// tab[i] = (four-step twiddle, M[k]) at block position i, tab[N].z = M[N];
// W^k = wk[k2] wk[n2 + k1] (exp(-i pi k2 / N) and exp(-i pi k1 / n1)).
template <int LOG2N1>
struct K2PairShape {
    static constexpr int L = 1 << LOG2N1;
    static constexpr int TPV = L / 16;
    static constexpr int ROWS = TPV >= 256 ? 2 : 256 / TPV;  // even: whole pairs
    static constexpr int THREADS = ROWS * TPV;
    static constexpr int STRIDE = L + L / 16;
};

template <int LOG2N1, class T>
__global__ void __launch_bounds__(K2PairShape<LOG2N1>::THREADS) k2_real_pair(RealPairArgs a) {
    using Sh = K2PairShape<LOG2N1>;
    constexpr int L = Sh::L;
    constexpr int TPV = Sh::TPV;
    constexpr int PAIRS = Sh::ROWS / 2;
    __shared__ float2 lds[Sh::ROWS * Sh::STRIDE];

    const int logical = xcd_logical(blockIdx.x, gridDim.x);
    const int n2 = 1 << a.log2n2;
    const int npairs = n2 / 2;
    const int pair_groups = (npairs + PAIRS - 1) / PAIRS;
    if (logical >= pair_groups * a.nblocks) return;
    const int pg = logical / a.nblocks;
    const int b = logical - pg * a.nblocks;

    const int r = threadIdx.x / TPV;  // LDS row slot
    const int j = threadIdx.x - r * TPV;
    const int side = r & 1;
    const int pr = pg * PAIRS + (r >> 1);
    const bool valid = pr < npairs;   // pairs beyond the last re-run it and never store
    const int pc = min(pr, npairs - 1);
    const int row = side == 0 ? pc : (pc == 0 ? n2 / 2 : n2 - pc);
    const PadLds<float2> lrow{lds + r * Sh::STRIDE};

    StageBases<LOG2N1> tb;
    tb.load(j, a.tw1);
    T* data = reinterpret_cast<T*>(a.data) + (((int64_t)b << a.log2n2) << LOG2N1);
    const uint32_t rowoff = (uint32_t)row << LOG2N1;
    const float4* tab = a.tab;

    float2 v[16];
    uint32_t to = opaque(rowoff + (uint32_t)j);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const float2 x = Elem<T>::load(at(data, (to + TPV * e) * (uint32_t)sizeof(T)));
        const float4 t = *at(tab, (to + TPV * e) * 16u);
        v[e] = cmul(x, make_float2(t.x, t.y));
    }
    // this element's filter value, fetched while the forward transform's
    // last exchange is under way
    float2 mkp[16];
    auto fetch_m = [&] {
        const uint32_t t2 = opaque(rowoff + (uint32_t)j);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const float4 t = *at(tab, (t2 + TPV * e) * 16u);
            mkp[e] = make_float2(t.z, t.w);
        }
    };
    fft_wg<LOG2N1, -1, false, false, false>(v, j, tb, lrow, nullptr, fetch_m);  // first LDS use

    // The pair's spectra (scaled) to LDS, then each element reads its partner.
    __syncthreads();
    static_for<16>([&](auto ei) {
        constexpr int e = decltype(ei)::value;
        lrow.template put<TPV * e>(j, cscale(v[e], a.scale));
    });
    __syncthreads();
    // partner of (row, k1): row 0 -> (0, -k1 mod n1); row n2/2 -> (n2/2,
    // n1-1-k1); otherwise the other row of the pair at n1-1-k1
    const int pslot = (pc == 0) ? r : (r ^ 1);
    const PadLds<float2> prow{lds + pslot * Sh::STRIDE};
    const uint32_t prowoff = (pc == 0 ? (uint32_t)row : (uint32_t)(n2 - row)) << LOG2N1;
    const float2 wr = a.wk[row];
    const float m_nyq = tab[(int64_t)1 << (LOG2N1 + a.log2n2)].z;
    asm volatile("" ::: "memory");
    to = opaque(rowoff + (uint32_t)j);
    static_for<16>([&](auto ei) {
        constexpr int e = decltype(ei)::value;
        const int k1 = j + TPV * e;
        const int kp = (row == 0) ? ((L - k1) & (L - 1)) : (L - 1 - k1);
        const float2 A = lrow.template get<TPV * e>(j);
        const float2 B = *prow.template addr<0>(kp);
        const float4 tn = *at(tab, (prowoff + (uint32_t)kp) * 16u);
        const float2 mk = mkp[e];
        const float2 mn = (row == 0 && k1 == 0) ? make_float2(m_nyq, 0.f) : make_float2(tn.z, tn.w);
        const float2 w = cmul(wr, a.wk[n2 + k1]);
        const float2 E = make_float2(0.5f * (A.x + B.x), 0.5f * (A.y - B.y));
        const float2 D = make_float2(0.5f * (A.x - B.x), 0.5f * (A.y + B.y));
        const float2 O = make_float2(D.y, -D.x);
        const float2 wo = cmul(w, O);
        const float2 yk = cmul(cadd(E, wo), mk);
        const float2 en = csub(E, wo);
        const float2 yn = cmul(make_float2(en.x, -en.y), mn);
        const float2 ync = make_float2(yn.x, -yn.y);
        const float2 e2 = cscale(cadd(yk, ync), 0.5f);
        const float2 o2 = cmulc(cscale(csub(yk, ync), 0.5f), w);
        v[e] = make_float2(e2.x - o2.y, e2.y + o2.x);
    });
    // output twiddles fetched during the inverse transform's last exchange
    float2 wo[16];
    auto fetch_tw = [&] {
        const uint32_t t2 = opaque(rowoff + (uint32_t)j);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const float4 t = *at(tab, (t2 + TPV * e) * 16u);
            wo[e] = make_float2(t.x, t.y);
        }
    };
    fft_wg<LOG2N1, +1>(v, j, tb, lrow, nullptr, fetch_tw);
    asm volatile("" ::: "memory");
    to = opaque(rowoff + (uint32_t)j);
    if (valid) {
#pragma unroll
        for (int e = 0; e < 16; ++e)
            Elem<T>::store(at(data, (to + TPV * e) * (uint32_t)sizeof(T)), cmulc(v[e], wo[e]));
    }
}

// Table of k2_real_pair: tab[i] = (W_N^(k1 k2), M[k]) at block position i
// (row k2, column k1, bin k = k2 + n2 k1), tab[N] = (0, 0, M[N], 0);
// wk[k2] = exp(-i pi k2 / N) for k2 < n2, wk[n2 + k1] = exp(-i pi k1 / n1).
// M as real_build_table (float64, reduced mod 1 turn).
__global__ void __launch_bounds__(256) real_build_pair_table(float4* __restrict__ tab, float2* __restrict__ wk,
                                                              int log2n1, int log2n2, double chirp_a, double f0,
                                                              double bw, int lsb, double taper) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int log2n = log2n1 + log2n2;
    const int64_t N = 1ll << log2n, n1 = 1ll << log2n1, n2 = 1ll << log2n2;
    if (i > N) return;
    const int64_t k2 = i >> log2n1, k1 = i & (n1 - 1);
    const int64_t k = i == N ? N : k2 + (k1 << log2n2);
    const double fb = (double)k * bw / (double)N;
    const double f = lsb ? bw * 0.5 - fb : fb - bw * 0.5;
    const double turns = chirp_a * (f * f) / (f0 + f);
    const double frac = turns - rint(turns);
    double sm, cm;
    sincospi(2.0 * frac, &sm, &cm);
    const double wt = taper_w(f, bw, taper);
    double mx = cm * wt, my = (lsb ? sm : -sm) * wt;
    if (k == 0 || k == N) my = 0.0;
    if (i == N) {
        tab[i] = make_float4(0.f, 0.f, (float)mx, 0.f);
        return;
    }
    double st, ct;
    sincospi(2.0 * (double)((k1 * k2) & (N - 1)) / (double)N, &st, &ct);
    tab[i] = make_float4((float)ct, (float)-st, (float)mx, (float)my);
    if (i < n2) {
        double s2, c2;
        sincospi((double)i / (double)N, &s2, &c2);
        wk[i] = make_float2((float)c2, (float)-s2);
    }
    if (i < n1) {
        double s1, c1;
        sincospi((double)i / (double)n1, &s1, &c1);
        wk[n2 + i] = make_float2((float)c1, (float)-s1);
    }
}

template <class T, int LOG2N1>
static hipError_t real_pair_one(const RealPairArgs& a, hipStream_t s) {
    using Sh = K2PairShape<LOG2N1>;
    const int npairs = (1 << a.log2n2) / 2;
    const int groups = (npairs + Sh::ROWS / 2 - 1) / (Sh::ROWS / 2) * a.nblocks;
    const int grid = (groups + 7) & ~7;
    hipLaunchKernelGGL((k2_real_pair<LOG2N1, T>), dim3(grid), dim3(Sh::THREADS), 0, s, a);
    return hipGetLastError();
}

template <class T>
static hipError_t real_pair_dispatch(int log2n1, const RealPairArgs& a, hipStream_t s) {
    switch (log2n1) {
        case 5: return real_pair_one<T, 5>(a, s);
        case 6: return real_pair_one<T, 6>(a, s);
        case 7: return real_pair_one<T, 7>(a, s);
        case 8: return real_pair_one<T, 8>(a, s);
        case 9: return real_pair_one<T, 9>(a, s);
        case 10: return real_pair_one<T, 10>(a, s);
        case 11: return real_pair_one<T, 11>(a, s);
        case 12: return real_pair_one<T, 12>(a, s);
        case 13: return real_pair_one<T, 13>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_real_pair(int prec, int log2n1, const RealPairArgs& a, hipStream_t s) {
    switch (prec) {
        case kFp32: return real_pair_dispatch<float2>(log2n1, a, s);
        case kMixedValu: return real_pair_dispatch<__half2>(log2n1, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_real_build_pair_table(float4* tab, float2* wk, int log2n1, int log2n2, double chirp_a, double f0,
                                        double bw, int lsb, double taper, hipStream_t s) {
    const int64_t n = (1ll << (log2n1 + log2n2)) + 1;
    hipLaunchKernelGGL(real_build_pair_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, wk, log2n1,
                       log2n2, chirp_a, f0, bw, lsb, taper);
    return hipGetLastError();
}

template <class T>
static hipError_t real_split_t(const RealSplitArgs& a, hipStream_t s) {
    const int64_t n = (int64_t)a.nblocks * (((1 << a.log2n2) / 2 + 1) << a.log2n1);
    hipLaunchKernelGGL(real_split<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_real_split(int prec, const RealSplitArgs& a, hipStream_t s) {
    switch (prec) {
        case kFp32: return real_split_t<float2>(a, s);
        case kMixedValu: return real_split_t<__half2>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_real_build_table(float4* tab, int log2n1, int log2n2, double chirp_a, double f0, double bw,
                                   int lsb, double taper, hipStream_t s) {
    const int64_t n = (1ll << (log2n1 + log2n2)) + 1;
    hipLaunchKernelGGL(real_build_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, log2n1, log2n2,
                       chirp_a, f0, bw, lsb, taper);
    return hipGetLastError();
}

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

// ---------------------------------------------------------- launchers
template <class T, int FORM, int LOG2N2>
static hipError_t k1_one(const K1Args& a, hipStream_t s) {
    const int ntiles = a.nblocks * ((1 << a.log2n1) >> 4);
    const int grid = (ntiles + 7) & ~7;
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
    const int ntiles = a.nblocks * ((1 << a.log2n1) >> 4);
    const int grid = (ntiles + 7) & ~7;
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
        default: return k1_dispatch<float2, kFormF32>(log2n2, a, s);
    }
}

template <class T, int MODE, bool F16, int LOG2N1>
static hipError_t k2_one(const K2Args& a, hipStream_t s) {
    using Sh = K2Shape<LOG2N1>;
    const int groups = ((1 << a.log2n2) + Sh::ROWS - 1) / Sh::ROWS * a.nblocks;
    const int grid = (groups + 7) & ~7;
    hipLaunchKernelGGL((k2_row<LOG2N1, T, MODE, F16>), dim3(grid), dim3(Sh::THREADS), 0, s, a);
    return hipGetLastError();
}

template <class T, int MODE, bool F16>
static hipError_t k2_dispatch(int log2n1, const K2Args& a, hipStream_t s) {
    switch (log2n1) {
        case 5: return k2_one<T, MODE, F16, 5>(a, s);
        case 6: return k2_one<T, MODE, F16, 6>(a, s);
        case 7: return k2_one<T, MODE, F16, 7>(a, s);
        case 8: return k2_one<T, MODE, F16, 8>(a, s);
        case 9: return k2_one<T, MODE, F16, 9>(a, s);
        case 10: return k2_one<T, MODE, F16, 10>(a, s);
        case 11: return k2_one<T, MODE, F16, 11>(a, s);
        case 12: return k2_one<T, MODE, F16, 12>(a, s);
        case 13: return k2_one<T, MODE, F16, 13>(a, s);
        case 14: return k2_one<T, MODE, F16, 14>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t k2_prec(int prec, int log2n1, const K2Args& a, hipStream_t s) {
    switch (prec) {
        case kFp32: return k2_dispatch<float2, MODE, false>(log2n1, a, s);
        case kHalf: return k2_dispatch<__half2, MODE, true>(log2n1, a, s);
        default: return k2_dispatch<__half2, MODE, false>(log2n1, a, s);
    }
}

hipError_t launch_k2(int prec, int mode, int log2n1, const K2Args& a, hipStream_t s) {
    switch (mode) {
        case kRowFull: return k2_prec<kRowFull>(prec, log2n1, a, s);
        case kRowFwd: return k2_prec<kRowFwd>(prec, log2n1, a, s);
        case kRowInv: return k2_prec<kRowInv>(prec, log2n1, a, s);
        case kRowInvPlain:
            // float32 arithmetic forms only (the real input path)
            if (prec == kFp32) return k2_dispatch<float2, kRowInvPlain, false>(log2n1, a, s);
            if (prec == kMixedValu) return k2_dispatch<__half2, kRowInvPlain, false>(log2n1, a, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_k2_build_split_tables(float2* tw, float2* chirp, int log2n1, int log2n2, double chirp_a, double f0,
                                        double df, hipStream_t s) {
    const int64_t n = 1ll << (log2n1 + log2n2);
    hipLaunchKernelGGL(k2_build_split_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tw, chirp, log2n1,
                       log2n2, chirp_a, f0, df);
    return hipGetLastError();
}

hipError_t launch_k2_build_split_tables_h(void* tw, void* chirp, int log2n1, int log2n2, double chirp_a, double f0,
                                          double df, hipStream_t s) {
    const int64_t n = 1ll << (log2n1 + log2n2);
    hipLaunchKernelGGL(k2_build_split_tables_h, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<h2*>(tw), reinterpret_cast<h2*>(chirp), log2n1, log2n2, chirp_a, f0, df);
    return hipGetLastError();
}

hipError_t launch_k2_build_table_h(void* tab, int log2n1, int log2n2, double chirp_a, double f0, double df,
                                   double taper, hipStream_t s) {
    const int64_t n = 1ll << (log2n1 + log2n2);
    const double chirp_scale = std::ldexp(1.0, -half_row_rem(log2n1));
    hipLaunchKernelGGL(k2_build_table_h, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<uint2*>(tab), log2n1, log2n2, chirp_a, f0, df, chirp_scale, taper);
    return hipGetLastError();
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
        default: return k3_dispatch<float2, kFormF32>(log2n2, a, grid, dyn, s);
    }
}

hipError_t launch_fold_reduce(const uint64_t* ps, const uint32_t* pc, int nparts, int entries, uint64_t* acc_sum,
                              uint64_t* acc_cnt, int64_t acc_off, hipStream_t s) {
    dim3 grid((entries + 255) / 256, (nparts + kReduceChunk - 1) / kReduceChunk);
    hipLaunchKernelGGL(fold_reduce, grid, dim3(256), 0, s, ps, pc, nparts, entries, acc_sum, acc_cnt, acc_off);
    return hipGetLastError();
}

hipError_t launch_fold_finalize(uint64_t* acc_sum, uint64_t* acc_cnt, int nbins, int n_complete, int n_touched,
                                float* profiles, hipStream_t s) {
    hipLaunchKernelGGL(fold_finalize, dim3((nbins + 255) / 256), dim3(256), 0, s, acc_sum, acc_cnt, nbins,
                       n_complete, n_touched, profiles);
    return hipGetLastError();
}

hipError_t launch_k2_build_table(float4* tab, int log2n1, int log2n2, double chirp_a, double f0, double df,
                                 double taper, hipStream_t s) {
    const int64_t n = 1ll << (log2n1 + log2n2);
    hipLaunchKernelGGL(k2_build_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, log2n1, log2n2,
                       chirp_a, f0, df, taper);
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

int64_t hist_capacity(int log2n2, int prec) {
    const int64_t cap = (int64_t)((kLdsBytes - k3_static_lds(log2n2, prec)) / 12);
    return cap < kHistCapMax ? cap : kHistCapMax;
}

int k3_grid(int log2n2, int prec, size_t dyn_lds, int64_t items, int64_t entries, bool global_mode) {
    const size_t lds = k3_static_lds(log2n2, prec) + dyn_lds;
    int per_cu = (int)(kLdsBytes / lds);
    per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
    int64_t grid = 256 * per_cu;
    if (!global_mode && grid * entries > kPartEntries) grid = kPartEntries / entries;
    const int64_t items8 = (items + 7) & ~int64_t(7);
    if (grid > items8) grid = items8;
    grid &= ~int64_t(7);
    if (grid < 8) grid = 8;
    return (int)grid;
}

size_t k3_static_lds(int log2n2, int prec) {
    const size_t l = (size_t)1 << log2n2;
    if (prec == kHalf) return (16 * l + l) * sizeof(h2) + 16 * l * sizeof(float) + kS1Pairs * sizeof(h2);
    return sizeof(float2) * 16 * l;
}
static_assert(K3Shape<10>::LDS_HALF == (16 * 1024 + 1024) * 4 + 16 * 1024 * 4 + kS1Pairs * 4, "host copy of the K3 layout");
int k1_threads(int log2n2) { return 1 << log2n2; }
int k3_threads(int log2n2) { return 1 << log2n2; }
int k2_threads(int log2n1) {
    const int tpv = (1 << log2n1) / 16;
    return tpv >= 256 ? tpv : 256;
}

}  // namespace pond

namespace pond {
// The host-side table scale must match the device schedule.
static_assert(half_row_rem(5) == Sched<5>::kHalfRem && half_row_rem(6) == Sched<6>::kHalfRem &&
                  half_row_rem(7) == Sched<7>::kHalfRem && half_row_rem(8) == Sched<8>::kHalfRem &&
                  half_row_rem(9) == Sched<9>::kHalfRem && half_row_rem(10) == Sched<10>::kHalfRem &&
                  half_row_rem(11) == Sched<11>::kHalfRem && half_row_rem(12) == Sched<12>::kHalfRem &&
                  half_row_rem(13) == Sched<13>::kHalfRem && half_row_rem(14) == Sched<14>::kHalfRem,
              "row normalisation split");
}  // namespace pond
