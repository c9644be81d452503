// Device helpers shared by the kernel translation units: storage forms,
// uniform addressing, float16 table rounding, the frequency-domain taper,
// launch shapes, and the float64 fold phase and integer fold accumulation.
#pragma once

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
// A complex value as two bfloat16 (the upper halves of float32, real part
// in the low 16 bits), rounded to nearest even on store.
struct __align__(4) bf16x2 {
    uint32_t u;
};
__device__ __forceinline__ uint32_t bf16_rne(float f) {
    const uint32_t b = __builtin_bit_cast(uint32_t, f);
    return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
}
template <>
struct Elem<bf16x2> {
    __device__ __forceinline__ static float2 load(const bf16x2* p) {
        const uint32_t u = p->u;
        return make_float2(__builtin_bit_cast(float, u << 16), __builtin_bit_cast(float, u & 0xffff0000u));
    }
    __device__ __forceinline__ static void store(bf16x2* p, float2 v) {
        p->u = bf16_rne(v.x) | (bf16_rne(v.y) << 16);
    }
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
// A pointer into global memory that is the same in every lane, moved to
// scalar registers, so that bases derived from it stay scalar.  It is
// rebuilt as a global-address-space pointer: accesses through a pointer
// made from an integer would otherwise be flat ones, which also count as
// LDS operations, so that every wait for an LDS result would wait for them
// too.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    using G = __attribute__((address_space(1))) T;
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    G* g = reinterpret_cast<G*>(((uint64_t)hi << 32) | lo);
    return (T*)g;
}
// Raw buffer accesses (MUBUF): a uniform base and size in a resource
// descriptor, the lane's 32-bit byte offset in a vector register and a
// uniform byte offset in a scalar one, so that a thread's accesses at fixed
// strides from one lane offset cost no vector address arithmetic (global
// accesses fold such constants into 64-bit vector addresses instead).
// Accesses at or beyond `bytes` read 0 and write nothing.
struct BufRes {
    __amdgpu_buffer_rsrc_t r;
};
__device__ __forceinline__ BufRes buf_res(const void* base, uint32_t bytes) {
    // descriptor word 3 of the gfx9 family: 32-bit data format
    return {__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000)};
}
template <class V>
__device__ __forceinline__ V buf_ld(const BufRes& b, uint32_t voff, int soff) {
    static_assert(sizeof(V) == 4, "32-bit values");
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)voff, soff, 0));
}
template <class V>
__device__ __forceinline__ void buf_st(const BufRes& b, uint32_t voff, int soff, V v) {
    static_assert(sizeof(V) == 4, "32-bit values");
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), b.r, (int)voff, soff, 0);
}

// Hide a value from the optimiser so that expressions depending on it are
// recomputed where used instead of being hoisted and kept in registers.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Arithmetic of a kernel instance: float32 vector, float16 matrix-core
// DFT-16 stages (float32 elsewhere), or packed float16 vector.
constexpr int kFormF32 = 0, kFormMfma = 1, kFormF16 = 2;

template <int FORM>
using LdsVal = std::conditional_t<FORM == kFormF16 || FORM == kFormMfma, h2, float2>;

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
// ------------------------------------------------------------------- K3
// Static LDS.  Float32 arithmetic: one float2 tile of 16 columns, reused for
// the detected powers.  Packed float16: the padded float16 tile, a power
// buffer of its own (16 floats per row) and the twiddle tables, so
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
    static constexpr size_t LDS_HALF = kHalfTile + kHalfPf + ((TwTab<LOG2N2>::kSize + 3) & ~3) * sizeof(h2);
    static constexpr size_t lds(int form) { return form == kFormF16 || form == kFormMfma ? LDS_HALF : LDS; }
};

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
}  // namespace pond
