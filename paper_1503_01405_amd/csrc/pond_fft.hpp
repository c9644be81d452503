// Device-side building blocks: complex arithmetic, small in-register DFTs
// and a workgroup Stockham FFT whose stages exchange data through LDS.
//
// Data distribution (every FFT in the library): a vector of length L is
// held by L/16 threads, 16 complex values each; thread j holds positions
// j + (L/16)*e, e = 0..15, before the first stage and after the last one.
// Every stage reads its inputs from those positions, so the first stage
// reads straight from registers (filled by coalesced global loads) and the
// last stage leaves its outputs in registers (for coalesced global stores
// or further in-register work).  Between stages the values go through LDS
// at the Stockham output positions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace pond {

// ---------------------------------------------------------------- complex
// Two value types carry a complex number: float2 (float32 arithmetic) and
// h2, a pair of float16 that the packed instructions (v_pk_add_f16,
// v_pk_mul_f16, v_pk_fma_f16) process in one operation -- swaps and sign
// changes of halves fold into their op_sel / neg modifiers.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * b
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}

__device__ __forceinline__ h2 cadd(h2 a, h2 b) { return a + b; }
__device__ __forceinline__ h2 csub(h2 a, h2 b) { return a - b; }
__device__ __forceinline__ h2 cscale(h2 a, _Float16 s) { return a * s; }
__device__ __forceinline__ h2 cmul(h2 a, h2 b) {
    const h2 m = {-b.y, b.y};
    return __builtin_elementwise_fma(a.yx, m, a * b.xx);
}
__device__ __forceinline__ h2 cmulc(h2 a, h2 b) {
    const h2 m = {b.y, -b.y};
    return __builtin_elementwise_fma(a.yx, m, a * b.xx);
}

__device__ __forceinline__ float2 cneg(float2 a) { return make_float2(-a.x, -a.y); }
__device__ __forceinline__ h2 cneg(h2 a) { return -a; }

__device__ __forceinline__ h2 to_h2(float2 a) {
    const h2 r = {(_Float16)a.x, (_Float16)a.y};
    return r;
}
__device__ __forceinline__ float2 to_f2(h2 a) { return make_float2((float)a.x, (float)a.y); }

template <class V>
__device__ __forceinline__ V cone();
template <>
__device__ __forceinline__ float2 cone<float2>() { return make_float2(1.f, 0.f); }
template <>
__device__ __forceinline__ h2 cone<h2>() {
    const h2 r = {(_Float16)1.f, (_Float16)0.f};
    return r;
}

// Constants of the in-register DFTs.  cos(pi/8), sin(pi/8) and 1/sqrt(2)
// in float32; for float16 the cos/sin pair is chosen among neighbouring
// float16 values so that c^2 + s^2 = 1 + 4e-6 (the nearest values would
// lose 1.8e-4 of power per use), and products by 1/sqrt(2) are formed in
// float32 and rounded once (the nearest float16 constant would lose 2.1e-4
// of power per use).  Folded profiles are means of power, so such a fixed
// gain would not average out.
constexpr float kC8 = 0.92387953251128675613f, kS8 = 0.38268343236508977173f;
constexpr float kRs2 = 0.70710678118654752440f;
constexpr float kC8h = 0.923828125f, kS8h = 0.3828125f;  // float16-exact

// a * exp(DIR * i pi / 2): DIR = -1 multiplies by -i, DIR = +1 by +i
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
    if constexpr (DIR < 0) return make_float2(a.y, -a.x);
    else return make_float2(-a.y, a.x);
}
template <int DIR>
__device__ __forceinline__ h2 mul_i(h2 a) {
    if constexpr (DIR < 0) {
        const h2 r = {a.y, -a.x};
        return r;
    } else {
        const h2 r = {-a.y, a.x};
        return r;
    }
}
// a * exp(DIR * i pi / 4)
template <int DIR>
__device__ __forceinline__ float2 mul_w8(float2 a) {
    constexpr float h = kRs2;
    if constexpr (DIR < 0) return make_float2((a.x + a.y) * h, (a.y - a.x) * h);
    else return make_float2((a.x - a.y) * h, (a.x + a.y) * h);
}
// t * c for a float32 constant c, each half rounded once from the float32
// product (v_fma_mix*_f16): 1/sqrt(2) itself is not a float16 value.
__device__ __forceinline__ h2 scale_f32(h2 t, float c) {
    const h2 r = {(_Float16)fmaf((float)t.x, c, 0.0f), (_Float16)fmaf((float)t.y, c, 0.0f)};
    return r;
}
template <int DIR>
__device__ __forceinline__ h2 mul_w8(h2 a) {
    const h2 t = a + mul_i<DIR>(a);  // DIR < 0: (x + y, y - x); DIR > 0: (x - y, x + y)
    return scale_f32(t, kRs2);
}
// a * exp(DIR * 3 i pi / 4)
template <int DIR>
__device__ __forceinline__ float2 mul_w8_3(float2 a) {
    constexpr float h = kRs2;
    if constexpr (DIR < 0) return make_float2((a.y - a.x) * h, -(a.x + a.y) * h);
    else return make_float2(-(a.x + a.y) * h, (a.x - a.y) * h);
}
template <int DIR>
__device__ __forceinline__ h2 mul_w8_3(h2 a) {
    const h2 t = a + mul_i<-DIR>(a);  // DIR < 0: (x - y, x + y); DIR > 0: (x + y, y - x)
    return scale_f32(t, -kRs2);
}
// a * (c + DIR*i*s) for a constant point on the unit circle
template <int DIR>
__device__ __forceinline__ float2 mul_cs(float2 a, float c, float s) {
    if constexpr (DIR < 0) return make_float2(fmaf(a.x, c, a.y * s), fmaf(a.y, c, -(a.x * s)));
    else return make_float2(fmaf(a.x, c, -(a.y * s)), fmaf(a.y, c, a.x * s));
}
template <int DIR>
__device__ __forceinline__ h2 mul_cs(h2 a, float c, float s) {
    const _Float16 ch = (_Float16)c, sh = (_Float16)s;
    const h2 m = DIR < 0 ? h2{sh, -sh} : h2{-sh, sh};
    return __builtin_elementwise_fma(a.yx, m, a * ch);
}
template <class V>
struct DftConst;
template <>
struct DftConst<float2> {
    static constexpr float c8 = kC8, s8 = kS8;
};
template <>
struct DftConst<h2> {
    static constexpr float c8 = kC8h, s8 = kS8h;
};

// --------------------------------------------------------- small DFTs
// In-place DFT of R values, natural order in and out:
//   V[s] = sum_q v[q] exp(DIR * 2 pi i q s / R)   (DIR = -1 forward)
template <int DIR, class V>
__device__ __forceinline__ void dft2(V& a, V& b) {
    V t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int DIR, class V>
__device__ __forceinline__ void dft4(V& v0, V& v1, V& v2, V& v3) {
    V a0 = cadd(v0, v2), a1 = csub(v0, v2);
    V a2 = cadd(v1, v3), a3 = mul_i<DIR>(csub(v1, v3));
    v0 = cadd(a0, a2);
    v2 = csub(a0, a2);
    v1 = cadd(a1, a3);
    v3 = csub(a1, a3);
}

template <int R, int DIR, class V>
struct Dft;

template <int DIR, class V>
struct Dft<2, DIR, V> {
    __device__ __forceinline__ static void run(V* v) { dft2<DIR>(v[0], v[1]); }
};

template <int DIR, class V>
struct Dft<4, DIR, V> {
    __device__ __forceinline__ static void run(V* v) { dft4<DIR>(v[0], v[1], v[2], v[3]); }
};

// 8 = 2 x 4: two 4-point DFTs on the even/odd subsequences, twiddle, 2-point.
template <int DIR, class V>
struct Dft<8, DIR, V> {
    __device__ __forceinline__ static void run(V* v) {
        dft4<DIR>(v[0], v[2], v[4], v[6]);
        dft4<DIR>(v[1], v[3], v[5], v[7]);
        v[3] = mul_w8<DIR>(v[3]);
        v[5] = mul_i<DIR>(v[5]);
        v[7] = mul_w8_3<DIR>(v[7]);
        V o[8];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            V a = v[2 * sb], b = v[2 * sb + 1];
            o[sb] = cadd(a, b);
            o[sb + 4] = csub(a, b);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = o[i];
    }
};

// 16 = 4 x 4: q = qa + 4 qb, s = sb + 4 sa.
template <int DIR, class V>
struct Dft<16, DIR, V> {
    __device__ __forceinline__ static void run(V* v) {
        constexpr float c1 = DftConst<V>::c8;  // cos(pi/8)
        constexpr float s1 = DftConst<V>::s8;  // sin(pi/8)
#pragma unroll
        for (int qa = 0; qa < 4; ++qa) dft4<DIR>(v[qa], v[qa + 4], v[qa + 8], v[qa + 12]);
        // twiddle T[qa][sb] (stored at v[qa + 4 sb]) by W16^(qa sb)
        v[1 + 4 * 1] = mul_cs<DIR>(v[1 + 4 * 1], c1, s1);   // W^1
        v[1 + 4 * 2] = mul_w8<DIR>(v[1 + 4 * 2]);           // W^2
        v[1 + 4 * 3] = mul_cs<DIR>(v[1 + 4 * 3], s1, c1);   // W^3
        v[2 + 4 * 1] = mul_w8<DIR>(v[2 + 4 * 1]);           // W^2
        v[2 + 4 * 2] = mul_i<DIR>(v[2 + 4 * 2]);            // W^4
        v[2 + 4 * 3] = mul_w8_3<DIR>(v[2 + 4 * 3]);         // W^6
        v[3 + 4 * 1] = mul_cs<DIR>(v[3 + 4 * 1], s1, c1);   // W^3
        v[3 + 4 * 2] = mul_w8_3<DIR>(v[3 + 4 * 2]);         // W^6
        v[3 + 4 * 3] = mul_cs<DIR>(v[3 + 4 * 3], -c1, -s1); // W^9
        V o[16];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            V a0 = v[0 + 4 * sb], a1 = v[1 + 4 * sb], a2 = v[2 + 4 * sb], a3 = v[3 + 4 * sb];
            dft4<DIR>(a0, a1, a2, a3);
            o[sb + 0] = a0;
            o[sb + 4] = a1;
            o[sb + 8] = a2;
            o[sb + 12] = a3;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = o[i];
    }
};

// ------------------------------------------------------ radix schedule
// log2 L = 4 a + b: a radix-16 stages followed by one radix-2^b stage.
template <int LOG2L>
struct Sched {
    static constexpr int kFull = LOG2L / 4;
    static constexpr int kRem = 1 << (LOG2L % 4);
    static constexpr int kStages = kFull + (kRem > 1 ? 1 : 0);
    static constexpr int radix(int s) { return s < kFull ? 16 : kRem; }
    static constexpr int ns(int s) { return s == 0 ? 1 : ns(s - 1) * radix(s - 1); }
    // float16 forward transforms scale the input of every even stage by
    // 1/16 (stage 0 by the caller), so that no value exceeds 16x the input
    // bound between scalings; the rest of the 1/L normalisation is left
    // to the caller: 2^-kHalfRem.
    static constexpr int kHalfScaled = 4 * ((kStages + 1) / 2);
    static constexpr int kHalfRem = LOG2L - kHalfScaled;
};

template <int N, class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl<N>(static_cast<F&&>(f), std::make_integer_sequence<int, N>{});
}

// ------------------------------------------------------------ twiddles
// a * exp(-2 pi i u / 16) for a compile-time u (DIR-independent: the
// twiddle bases are always the forward ones).
template <int U, class V>
__device__ __forceinline__ V mul_w16(V a) {
    constexpr int u = U & 15;
    constexpr float c1 = DftConst<V>::c8, s1 = DftConst<V>::s8;
    if constexpr (u == 0) return a;
    else if constexpr (u == 4) return mul_i<-1>(a);
    else if constexpr (u == 8) return cneg(a);
    else if constexpr (u == 12) return mul_i<+1>(a);
    else if constexpr (u == 2) return mul_w8<-1>(a);
    else if constexpr (u == 6) return mul_w8_3<-1>(a);
    else if constexpr (u == 10) return mul_w8_3<+1>(a);
    else if constexpr (u == 14) return mul_w8<+1>(a);
    else if constexpr (u == 1) return mul_cs<-1>(a, c1, s1);
    else if constexpr (u == 3) return mul_cs<-1>(a, s1, c1);
    else if constexpr (u == 5) return mul_cs<-1>(a, -s1, c1);
    else if constexpr (u == 7) return mul_cs<-1>(a, -c1, s1);
    else if constexpr (u == 9) return mul_cs<-1>(a, -c1, -s1);
    else if constexpr (u == 11) return mul_cs<-1>(a, -s1, -c1);
    else if constexpr (u == 13) return mul_cs<-1>(a, s1, -c1);
    else return mul_cs<-1>(a, c1, -s1);
}

// p[q] = w^q for q = 1..R-1 (p[0] unused), products at most four deep.
template <int R, class V>
__device__ __forceinline__ void powers(V w, V (&p)[R]) {
    p[0] = cone<V>();
    if constexpr (R > 1) p[1] = w;
    if constexpr (R > 2) p[2] = cmul(w, w);
    if constexpr (R > 3) p[3] = cmul(p[2], w);
    if constexpr (R > 4) {
        p[4] = cmul(p[2], p[2]);
        p[5] = cmul(p[4], w);
        p[6] = cmul(p[4], p[2]);
        p[7] = cmul(p[4], p[3]);
    }
    if constexpr (R > 8) {
        p[8] = cmul(p[4], p[4]);
#pragma unroll
        for (int q = 9; q < 16; ++q) p[q] = cmul(p[8], p[q - 8]);
    }
}

// Per-thread twiddle bases of every stage of a length-L transform, read once
// from tw[t] = exp(-2 pi i t / L):
//   radix-16 stage with NS > 1: exp(-2 pi i k / (16 NS)), k = j mod NS
//     (one butterfly per thread; its twiddles are the powers of the base);
//   final stage of radix R < 16 (NS = L / R): exp(-2 pi i j / L); butterfly
//     u of the thread has base exp(-2 pi i (j + u L/16) / L) = base * W16^u.
template <int LOG2L, class V = float2>
struct StageBases {
    V b[Sched<LOG2L>::kStages];
    __device__ __forceinline__ void load(int j, const float2* __restrict__ tw) {
        using S = Sched<LOG2L>;
        constexpr int L = 1 << LOG2L;
        static_for<S::kStages>([&](auto si) {
            constexpr int s = decltype(si)::value;
            constexpr int NS = S::ns(s);
            constexpr int R = S::radix(s);
            float2 x = make_float2(1.f, 0.f);
            if constexpr (NS > 1) {
                if constexpr (R == 16) x = tw[(j & (NS - 1)) * (L / (16 * NS))];
                else x = tw[j];
            }
            b[s] = x;
        });
    }
};

// The packed-float16 transforms use the float32 stage bases.
template <int LOG2L>
struct StageBases<LOG2L, h2> : StageBases<LOG2L, float2> {};

// LDS layouts of a transform's vector (the position of an element is its
// index in the vector).  put<D>(p0, x) / get<D>(p0) access position p0 + D
// for a compile-time D, so that D's part of the address is an immediate.
// Columns interleaved by 16 (K1/K3 tiles): index = pos * 16 (from the
// column's base).  PAD adds four spare slots per four positions (index =
// 16 pos + 4 (pos / 4)): the first stage's stores, 16 positions apart in
// the four column groups of a wave, then fall in different banks, and the
// other accesses stay contiguous.  The split p0 + D -> idx(p0) + idx(D)
// holds when D is a multiple of 4, or when p0 is (AL).
template <class V, bool PAD = false>
struct ColLds {
    V* base;
    static constexpr uint32_t kSlots(uint32_t n) { return PAD ? n * 16 + 4 * (n / 4) : n * 16; }
    static __device__ __forceinline__ uint32_t idx(uint32_t p) { return PAD ? p * 16 + 4 * (p >> 2) : p * 16; }
    template <int D, bool AL = false>
    __device__ __forceinline__ V* addr(int p0) const {
        if constexpr (!PAD || D % 4 == 0 || AL) {
            return base + idx((uint32_t)p0) + kSlots(D);
        } else {
            return base + idx((uint32_t)(p0 + D));
        }
    }
    template <int D, bool AL = false>
    __device__ __forceinline__ void put(int p0, V x) const { *addr<D, AL>(p0) = x; }
    template <int D>
    __device__ __forceinline__ V get(int p0) const { return *addr<D>(p0); }
};
// One row with a pad slot per 16 values (K2): index = pos + pos / 16.  The
// split p0 + D -> (p0 + p0/16) + (D + D/16) holds when D is a multiple of 16,
// or when p0 is (AL) and D < 16.
template <class V>
struct PadLds {
    V* base;
    template <int D, bool AL = false>
    __device__ __forceinline__ V* addr(int p0) const {
        if constexpr (D % 16 == 0 || AL) {
            const uint32_t u = (uint32_t)p0;
            return base + (u + (u >> 4)) + (D + D / 16);
        } else {
            const uint32_t u = (uint32_t)(p0 + D);
            return base + (u + (u >> 4));
        }
    }
    template <int D, bool AL = false>
    __device__ __forceinline__ void put(int p0, V x) const { *addr<D, AL>(p0) = x; }
    template <int D>
    __device__ __forceinline__ V get(int p0) const { return *addr<D>(p0); }
};
// For a last stage, whose outputs stay in registers.
// Row layouts for float16 rows of 2^12 .. 2^14 (K2), chosen per stage so
// that the stage's stores and the following reads (runs of 64 consecutive
// positions per wave) both avoid bank conflicts (64 banks of 4 bytes):
// stage 0 (stores 16 positions apart) at p + p/64, stage 1 (runs of 16
// stores, 256 apart) at p + 16 (p/256), later stages (contiguous stores)
// at p.  Each fits in L + L/16 slots.  Use: stage_view<s>(lds).
template <class V>
struct StageRowLds {
    V* base;
    template <int S>
    struct At {
        V* base;
        static constexpr uint32_t idx(uint32_t p) { return S == 0 ? p + (p >> 6) : S == 1 ? p + 16 * (p >> 8) : p; }
        // idx(p0 + D) = idx(p0) + idx(D) for D a multiple of the layout's
        // period, and for the stage's own stores: stage 0 (AL: p0 a
        // multiple of 16, D < 16) and stage 1 (p0 mod 256 < 16, D <= 240).
        template <int D, bool AL = false>
        __device__ __forceinline__ V* addr(int p0) const {
            constexpr int period = S == 0 ? 64 : (S == 1 ? 256 : 1);
            if constexpr (D % period == 0 || (S == 0 && AL && D < 16) || (S == 1 && D <= 240)) {
                return base + idx((uint32_t)p0) + idx((uint32_t)D);
            } else {
                return base + idx((uint32_t)(p0 + D));
            }
        }
        template <int D, bool AL = false>
        __device__ __forceinline__ void put(int p0, V x) const { *addr<D, AL>(p0) = x; }
        template <int D>
        __device__ __forceinline__ V get(int p0) const { return *addr<D>(p0); }
    };
    template <int S>
    __device__ __forceinline__ At<S> stage() const { return At<S>{base}; }
};

// The layout a stage uses: the accessor itself, or its per-stage view.
template <int S, class Lds>
__device__ __forceinline__ Lds stage_view(const Lds& l) { return l; }
template <int S, class V>
__device__ __forceinline__ typename StageRowLds<V>::template At<S> stage_view(const StageRowLds<V>& l) {
    return l.template stage<S>();
}

template <class V>
struct NoLds {
    template <int D, bool AL = false>
    __device__ __forceinline__ void put(int, V) const {}
    template <int D>
    __device__ __forceinline__ V get(int) const { return V{}; }
};

// All float16 twiddles thread j needs for stage s of a length-2^LOG2L
// transform: 16 values (R = 16: its one butterfly; R < 16: R per butterfly
// u at u*R).  The powers of the stage's float32 base are formed in float32
// and each rounded once to float16 (raising a rounded float16 base to
// powers up to 15 would multiply its magnitude error, and the few distinct
// bases of a stage would leave that error as a gain bias).
template <int LOG2L, int s>
__device__ __forceinline__ void stage_tw_h(float2 base, h2 (&t)[16]) {
    using S = Sched<LOG2L>;
    constexpr int R = S::radix(s);
    if constexpr (R == 16) {
        float2 p[16];
        powers<16>(base, p);
#pragma unroll
        for (int q = 0; q < 16; ++q) t[q] = to_h2(p[q]);
    } else {
        static_for<16 / R>([&](auto ui) {
            constexpr int u = decltype(ui)::value;
            float2 p[R];
            powers<R>(mul_w16<u>(base), p);
#pragma unroll
            for (int q = 0; q < R; ++q) t[u * R + q] = to_h2(p[q]);
        });
    }
}

// One Stockham stage of radix R on the 16 values of thread j.  Butterfly u
// (index jp = j + TPV u, k = jp mod NS) reads positions jp + q L/R, which
// are registers u + q BF, twiddles input q by W_{NS R}^(q k), and writes
// output q to position (jp - k) R + k + q NS.  With SCALE_IN the inputs
// are first multiplied by 1/16 (float16 forward transforms).
template <int L, int R, int NS, int DIR, bool LAST, bool SCALE_IN = false, class V, class Lds>
__device__ __forceinline__ void stockham_stage(V (&v)[16], int j, V base, const Lds& st,
                                               const h2* htw = nullptr) {
    // htw (float16 only): the stage's 16 twiddles of this thread (stage_tw_h).
    constexpr bool HALF = std::is_same<V, h2>::value;
    // Opaque to the optimiser: the twiddle powers and LDS addresses of a
    // stage are recomputed at each use instead of being shared between the
    // forward and inverse transforms (or hoisted out of loops) and held in
    // registers, which costs occupancy.
    if constexpr (std::is_same<V, h2>::value) {
        asm volatile("" : "+v"(base), "+v"(j));
    } else {
        asm volatile("" : "+v"(base.x), "+v"(base.y), "+v"(j));
    }
    constexpr int BF = 16 / R;
    constexpr int TPV = L / 16;
    V pw[R];
    if constexpr (NS > 1 && R == 16) {
        if constexpr (HALF) {
#pragma unroll
            for (int q = 0; q < 16; ++q) pw[q] = htw[q];
        } else {
            powers<R>(base, pw);
        }
    }
    static_for<BF>([&](auto ui) {
        constexpr int u = decltype(ui)::value;
        const int jp = j + TPV * u;
        const int k = jp & (NS - 1);
        V w[R];
#pragma unroll
        for (int q = 0; q < R; ++q) w[q] = v[u + q * BF];
        if constexpr (SCALE_IN) {
#pragma unroll
            for (int q = 0; q < R; ++q) w[q] = cscale(w[q], (_Float16)0.0625f);
        }
        if constexpr (NS > 1) {
            if constexpr (R < 16) {
                if constexpr (HALF) {
#pragma unroll
                    for (int q = 0; q < R; ++q) pw[q] = htw[u * R + q];
                } else {
                    const V bu = mul_w16<u>(base);
                    powers<R>(bu, pw);
                }
            }
#pragma unroll
            for (int q = 1; q < R; ++q) w[q] = DIR < 0 ? cmul(w[q], pw[q]) : cmulc(w[q], pw[q]);
        }
        Dft<R, DIR, V>::run(w);
        if constexpr (LAST) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[u + q * BF] = w[q];
        } else {
            // basep is a multiple of 16 when NS = 1 (R = 16).
            const int basep = (jp - k) * R + k;
            static_for<R>([&](auto qi) {
                constexpr int q = decltype(qi)::value;
                st.template put<q * NS, NS == 1 && R == 16>(basep, w[q]);
            });
        }
    });
}

// LDS twiddle tables of a packed-float16 transform.  Stage s (radix R,
// NS > 1) multiplies input q of the butterfly with index k by
//   w_q(k) = exp(-2 pi i q k / (R NS)),
// and k = hi F + lo factors it as A_q(hi) B_q(lo), with
//   A_q(hi) = exp(-2 pi i q hi F / (R NS)),  B_q(lo) = exp(-2 pi i q lo / (R NS)),
// each a float16 rounding of a float32 value of the stage-twiddle array.
// The stage then costs one float16 complex product per twiddle (A B) in
// place of a float32 power chain and its conversions.  Layouts:
//   R = 16 (NS = 16 or 256, F = 16): rows of 16 pairs (q = 0..15) at a
//     stride of 20 pairs, so that 16-byte reads of 16 different rows fall
//     in distinct banks; B has 16 rows, A has NS / 16 rows (none if 1);
//   R < 16 (the last stage, NS = L / R, k = j + TPV u): F = min(64, TPV),
//     q-major, B[q-1][lo] over F entries and A[q-1][hi] over NS / F,
//     lo = j mod F (the same for every u of the thread).
// A workgroup fills the tables once (fill_twiddle_tables) from the float32
// array tw[t] = exp(-2 pi i t / L), and every transform it runs reads them.
constexpr int kTabStride = 20;
template <int LOG2L>
struct TwTab {
    using S = Sched<LOG2L>;
    static constexpr int L = 1 << LOG2L;
    static constexpr int TPV = L / 16;
    static constexpr int R(int s) { return S::radix(s); }
    static constexpr int NS(int s) { return S::ns(s); }
    static constexpr int F(int s) { return R(s) == 16 ? 16 : (TPV < 64 ? TPV : 64); }
    static constexpr int nA(int s) { return NS(s) / F(s); }
    static constexpr bool used(int s) { return s < S::kStages && NS(s) > 1; }
    static constexpr int sizeA(int s) {
        return !used(s) || nA(s) <= 1 ? 0 : (R(s) == 16 ? kTabStride * nA(s) : (R(s) - 1) * nA(s));
    }
    static constexpr int sizeB(int s) { return !used(s) ? 0 : (R(s) == 16 ? kTabStride * 16 : (R(s) - 1) * F(s)); }
    static constexpr int off(int s) { return s == 0 ? 0 : off(s - 1) + sizeA(s - 1) + sizeB(s - 1); }
    static constexpr int offA(int s) { return off(s); }
    static constexpr int offB(int s) { return off(s) + sizeA(s); }
    static constexpr int kSize = off(S::kStages);  // pairs
    static_assert(S::kFull <= 3, "radix-16 stages beyond NS = 256 are not tabled");
};

// Entries of the tables of stage s, in fill order: R = 16: B rows (16 x
// 16 pairs, q fastest) then A rows (nA x 16); R < 16: B (q-major, F per q)
// then A (q-major, nA per q).  Entry i: its table index and the index of
// its value in tw.
template <int LOG2L, int s>
struct TwFill {
    using T = TwTab<LOG2L>;
    static constexpr int L = T::L, R = T::R(s), F = T::F(s), nA = T::nA(s);
    static constexpr int D = L / (R * T::NS(s));  // tw index step of one turn / (R NS)
    static constexpr int nB = R == 16 ? 256 : (R - 1) * F;
    static constexpr int nAe = nA > 1 ? (R == 16 ? nA * 16 : (R - 1) * nA) : 0;
    static constexpr int count = T::used(s) ? nB + nAe : 0;
    static constexpr int oA = T::offA(s), oB = T::offB(s);
    __device__ __forceinline__ static void entry(int i, int& dst, int& src) {
        if (i < nB) {
            if constexpr (R == 16) {
                const int lo = i >> 4, q = i & 15;
                dst = oB + lo * kTabStride + q;
                src = q * lo * D;
            } else {
                const int q = i / F + 1, lo = i % F;
                dst = oB + i;
                src = q * lo * D;
            }
        } else {
            const int k = i - nB;
            if constexpr (R == 16) {
                const int hi = k >> 4, q = k & 15;
                dst = oA + hi * kTabStride + q;
                src = q * hi * F * D;
            } else {
                const int q = k / nA + 1, hi = k % nA;
                dst = oA + k;
                src = q * hi * F * D;
            }
        }
    }
};

// Fill every stage table of a length-2^LOG2L transform (ONLY_S1: the
// stage-1 table only); NT threads (tid < NT) share the work.  Every load of a thread is issued before its first
// store (indices past a table's end re-read a valid entry and are not
// stored), so the fill costs one memory latency, which overlaps the
// caller's own loads issued before it.
template <int LOG2L, int NT, bool ONLY_S1 = false>
__device__ __forceinline__ void fill_twiddle_tables(h2* tab, const float2* __restrict__ tw, int tid) {
    using S = Sched<LOG2L>;
    constexpr int L = 1 << LOG2L;
    static_for<S::kStages>([&](auto si) {
        constexpr int s = decltype(si)::value;
        using Fi = TwFill<LOG2L, s>;
        if constexpr (Fi::count > 0 && (!ONLY_S1 || s == 1)) {
            constexpr int kIt = (Fi::count + NT - 1) / NT;
            float2 val[kIt];
            int dst[kIt];
#pragma unroll
            for (int it = 0; it < kIt; ++it) {
                const int i = tid + it * NT;
                int d, src;
                Fi::entry(i < Fi::count ? i : Fi::count - 1, d, src);
                dst[it] = i < Fi::count ? d : -1;
                val[it] = tw[src & (L - 1)];
            }
#pragma unroll
            for (int it = 0; it < kIt; ++it)
                if (dst[it] >= 0) tab[dst[it]] = to_h2(val[it]);
        }
    });
    // keep the caller's later loads after the table work, so that their
    // registers and the table's temporaries are not live together
    asm volatile("" ::: "memory");
}

// The float16 twiddles of thread j for stage s, from the tables (same
// placement as stage_tw_h: R = 16 at t[q], R < 16 at t[u R + q]).
template <int LOG2L, int s>
__device__ __forceinline__ void stage_tw_tab(const h2* tab, int j, h2 (&t)[16]) {
    using T = TwTab<LOG2L>;
    constexpr int R = T::R(s), F = T::F(s), nA = T::nA(s);
    constexpr int oA = T::offA(s), oB = T::offB(s), NS = T::NS(s), TPV = T::TPV;
    // Opaque index: the reads are issued at each use instead of being
    // shared between transforms (or hoisted out of loops) and held live.
    asm volatile("" : "+v"(j));
    if constexpr (R == 16) {
        const int k = j & (NS - 1);
        const uint4* rb = reinterpret_cast<const uint4*>(tab + oB + (k & 15) * kTabStride);
        h2 b[16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint4 x = rb[i];
            b[4 * i] = __builtin_bit_cast(h2, x.x);
            b[4 * i + 1] = __builtin_bit_cast(h2, x.y);
            b[4 * i + 2] = __builtin_bit_cast(h2, x.z);
            b[4 * i + 3] = __builtin_bit_cast(h2, x.w);
        }
        if constexpr (nA > 1) {
            const uint4* ra = reinterpret_cast<const uint4*>(tab + oA + (k >> 4) * kTabStride);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint4 x = ra[i];
                const h2 a4[4] = {__builtin_bit_cast(h2, x.x), __builtin_bit_cast(h2, x.y),
                                  __builtin_bit_cast(h2, x.z), __builtin_bit_cast(h2, x.w)};
#pragma unroll
                for (int m = 0; m < 4; ++m) t[4 * i + m] = cmul(a4[m], b[4 * i + m]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) t[q] = b[q];
        }
    } else {
        const int lo = j & (F - 1);
        static_for<16 / R>([&](auto ui) {
            constexpr int u = decltype(ui)::value;
            const int hi = (j >> __builtin_ctz(F)) + (TPV / F) * u;
#pragma unroll
            for (int q = 1; q < R; ++q) {
                const h2 bq = tab[oB + (q - 1) * F + lo];
                if constexpr (nA > 1) t[u * R + q] = cmul(tab[oA + (q - 1) * nA + hi], bq);
                else t[u * R + q] = bq;
            }
        });
    }
}

// Full length-L transform (DIR = -1 forward, +1 inverse, unnormalised) of
// the vector held by thread j.  lds is the vector's LDS layout (ColLds or
// PadLds); every thread of the workgroup must call this together
// (it contains barriers).  With HALF_NORM (float16 forward transforms)
// every even stage but the first scales its input by 1/16 (the caller
// scales the first stage's input and applies the remaining 2^-kHalfRem).
// Float16 transforms read their stage twiddles from the LDS tables ttab
// (fill_twiddle_tables) as TW says: 0 none (float32 powers of the stage
// bases, rounded once), 1 stage 1 only, 2 every stage.  Without LEAD the caller
// guarantees that no thread still reads the vector's LDS, and the barrier
// before the first exchange's stores is left out.  hook() runs after the stores
// of the last exchange, before its barrier: global loads issued there for
// use after the transform wait out their latency behind the exchange.
struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};
template <int LOG2L, int DIR, bool HALF_NORM = false, int TW = 0, bool LEAD = true, class V, class Lds,
          class Hook = NoHook>
__device__ __forceinline__ void fft_wg(V (&v)[16], int j, const StageBases<LOG2L, V>& tb, const Lds& lds,
                                       const h2* ttab = nullptr, const Hook& hook = Hook{}) {
    using S = Sched<LOG2L>;
    constexpr int L = 1 << LOG2L;
    constexpr int TPV = L / 16;
    constexpr bool HALF = std::is_same<V, h2>::value;
    static_for<S::kStages>([&](auto si) {
        constexpr int s = decltype(si)::value;
        constexpr int R = S::radix(s);
        constexpr int NS = S::ns(s);
        constexpr bool LAST = (s == S::kStages - 1);
        constexpr bool SC = HALF_NORM && s > 0 && (s % 2 == 0);
        V base;
        h2 tw[16];
        if constexpr (HALF) {
            base = cone<V>();
            if constexpr (NS > 1 && (TW == 2 || (TW == 1 && s == 1))) {
                stage_tw_tab<LOG2L, s>(ttab, j, tw);
            } else if constexpr (NS > 1) {
                float2 b = tb.b[s];
                asm volatile("" : "+v"(b.x), "+v"(b.y));  // recompute per use, not hoisted
                stage_tw_h<LOG2L, s>(b, tw);
            }
        } else {
            base = tb.b[s];
        }
        if constexpr (!LAST) {
            const auto st = stage_view<s>(lds);
            if constexpr (s > 0 || LEAD) __syncthreads();
            stockham_stage<L, R, NS, DIR, false, SC>(v, j, base, st, tw);
            if constexpr (s == S::kStages - 2) hook();
            __syncthreads();
            static_for<16>([&](auto ei) {
                constexpr int e = decltype(ei)::value;
                v[e] = st.template get<TPV * e>(j);
            });
        } else {
            stockham_stage<L, R, NS, DIR, true, SC>(v, j, base, lds, tw);
        }
    });
}

// ------------------------------------------------- matrix-core DFT-16
// A 16-point complex DFT is a real 32 x 32 matrix product; the 16 x 32 half
// that yields real (or imaginary) outputs is one v_mfma_f32_16x16x32_f16
// operand.  Lane layout of that instruction (wave64): lane l holds
//   A[l % 16][8 (l / 16) + t]   and   B[8 (l / 16) + t][l % 16],  t < 8,
//   D[4 (l / 16) + t][l % 16],  t < 4.
// With the input vector interleaved as (Re x0, Im x0, Re x1, ...) along K,
// lane (g = l / 16, n = l % 16) supplies inputs q = 4g..4g+3 of vector n
// and receives outputs s = 4g..4g+3 of vector n.
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// cos(2 pi e / 16), e < 16 (float32 nearest to the exact values).
__constant__ const float kCos16[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                       0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                                       -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                                       0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};

// The A operands of scale * exp(DIR 2 pi i s q / 16), one float16 per entry:
// lane l holds row s = l % 16 (real outputs: (Re c, -Im c) per input q;
// imaginary outputs: (Im c, Re c)) for inputs q = 4 (l / 16) .. +3.  A fixed
// rounding of an entry changes the power gain of its output position by
// about 1e-4, which the measured power gain of the path takes out on
// average (float32 accumulation keeps the sums themselves exact).
struct Dft16H {
    half8_t re, im;
};
template <int DIR>
__device__ __forceinline__ Dft16H dft16_h(int lane, float scale) {
    const int srow = lane & 15, g = (lane >> 4) & 3;
    Dft16H m;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int e = ((4 * g + t) * srow) & 15;
        const float c = scale * kCos16[e];
        const float sn = scale * kCos16[(e + 12) & 15];  // sin x = cos(x - pi/2)
        const float si = DIR < 0 ? -sn : sn;
        m.re[2 * t] = (_Float16)c;
        m.re[2 * t + 1] = (_Float16)(-si);
        m.im[2 * t] = (_Float16)si;
        m.im[2 * t + 1] = (_Float16)c;
    }
    return m;
}

// Outputs s = 4g..4g+3 of the 16 vectors of a batch from their inputs q =
// 4g..4g+3 (x), rounded once from the float32 accumulators.
__device__ __forceinline__ void mfma_dft16_h(const Dft16H& m, const h2* x, h2* y) {
    half8_t b;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        b[2 * t] = x[t].x;
        b[2 * t + 1] = x[t].y;
    }
    const floatx4_t z = {0.f, 0.f, 0.f, 0.f};
    const floatx4_t dr = __builtin_amdgcn_mfma_f32_16x16x32_f16(m.re, b, z, 0, 0, 0);
    const floatx4_t di = __builtin_amdgcn_mfma_f32_16x16x32_f16(m.im, b, z, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t) y[t] = to_h2(make_float2(dr[t], di[t]));
}

// Matrix-core layout of a float16 transform of length L = 2^LOG2L (TPV =
// L / 16 threads per vector).  Each wave holds 64 butterflies of a
// radix-16 stage as 4 batches b of 16: lane (g, n) takes inputs q = 4g+t
// (t < 4) of butterfly jp(b), in its registers v[4b + t].
//   Rows (one vector per TPV threads, TPV >= 64, thread j of the vector):
//     g = (j / 16) mod 4, n = j mod 16, jp(b) = 64 (j / 64) + 16 b + n.
//   Columns (16 interleaved vectors, thread (c, j) with c = tid mod 16 the
//     vector, j = tid / 16, TPV >= 4): g = j mod 4, n = c,
//     jp(b) = 4 (j / 4) + b.
template <bool COLS>
__device__ __forceinline__ int mx_g(int j) {
    return COLS ? (j & 3) : ((j >> 4) & 3);
}
template <bool COLS>
__device__ __forceinline__ int mx_jp(int j, int b) {
    return COLS ? 4 * (j >> 2) + b : (j & ~63) + 16 * b + (j & 15);
}
// Position of register e = 4b + t of thread j (the first stage's input).
template <bool COLS, int TPV>
__device__ __forceinline__ int mx_pos(int j, int e) {
    return mx_jp<COLS>(j, e >> 2) + (4 * mx_g<COLS>(j) + (e & 3)) * TPV;
}
template <int LOG2L, bool COLS>
constexpr bool kMxShape = COLS ? (LOG2L >= 6) : (LOG2L >= 10);

// An int the optimiser cannot see through: values derived from it are
// computed where used instead of being shared and held in registers.
__device__ __forceinline__ int opaque_i(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// LDS layouts of the matrix-core transform's exchanges.  A float16 pair is
// one dword; a wave's 32-bit LDS access is served half a wave (32 lanes) at
// a time from 32 banks (dword index mod 32), so an access is free of bank
// conflicts when the 16 butterflies n and the two input groups g mod 2 of
// each half wave land on 32 distinct banks.  The stores of one stage and
// the reads of the next put g on different position bits (4 g TPV for the
// reads, 4 g NS for the stores), so each exchange X (0: the canonical input
// moved in, s + 1: after radix-16 stage s) has its own layout: position p
// is stored at index p ^ F(p), where F copies a few high bits of p onto low
// (bank) bits (columns, 16 interleaved vectors at index 16 p' + vector: bit
// 0 of p').  Sources and targets are disjoint, so the map is a bijection of
// [0, L).  An access at base p0 plus a compile-time offset d (p0 and d with
// no common bits) becomes (index(p0) ^ X(d)) + C(d): target bits of d XOR
// into the base, the rest is an immediate offset.
//
// Rows keep the plain layout (F = 0).  Conflict-free row layouts exist
// (after stage 0: bits 5, 6, 7, L-2 onto 0, 1, 3, 4; after stage 1: bits 6
// and L-2 onto 4), but both make the stage's stores XOR in their output
// index t, which splits the stores of a thread over several bases and
// holds them until every matrix product of the stage has finished; the row
// kernel measured 10-15% slower with them, while its bank conflicts (up to
// 8-way on the stage-0 stores) cost it nothing measurable: it is bound by
// exchange latency, not by LDS cycles.
template <int LOG2L, bool COLS, int X>
struct MxSwz {
    static constexpr int SH = COLS ? 4 : 0;
    // target bit of source bit k, or -1
    static constexpr int tgt(int k) {
        if (COLS) {
            if (X == 1) return (k == 2 || (LOG2L >= 8 && k == LOG2L - 2)) ? 0 : -1;
            if (X == 2) return k == 6 ? 0 : -1;
        }
        return -1;
    }
    static constexpr uint32_t F(uint32_t p) {
        uint32_t r = 0;
        for (int k = 0; k < LOG2L; ++k)
            if (tgt(k) >= 0 && ((p >> k) & 1u)) r ^= 1u << tgt(k);
        return r;
    }
    static constexpr uint32_t tmask() {
        uint32_t r = 0;
        for (int k = 0; k < LOG2L; ++k)
            if (tgt(k) >= 0) r |= 1u << tgt(k);
        return r;
    }
    static constexpr uint32_t kT = tmask();
    // the part of an offset that XORs into the base
    static constexpr uint32_t xpart(uint32_t d) { return (d & kT) ^ F(d); }
    // scaled index of a base position (computed where used)
    __device__ static __forceinline__ uint32_t base(int p0) {
        const uint32_t p = (uint32_t)opaque_i(p0);
        uint32_t r = p;
        static_for<LOG2L>([&](auto ki) {
            constexpr int k = decltype(ki)::value;
            constexpr int m = tgt(k);
            if constexpr (m >= 0) r ^= (p >> (k - m)) & (1u << m);
        });
        return r << SH;
    }
    // scaled index of base + D (D a compile-time offset disjoint from the base)
    template <uint32_t D>
    __device__ static __forceinline__ uint32_t at(uint32_t mb) {
        constexpr uint32_t xd = xpart(D) << SH;
        constexpr uint32_t cd = (D & ~kT) << SH;
        if constexpr (xd != 0) return (mb ^ xd) + cd;
        else return mb + cd;
    }
};

// Offsets of the 16 accesses of a thread: reads of a stage (inputs q = 4g + t
// of butterfly batch b), stores of a stage with NS = ns, canonical (j + TPV e).
template <bool COLS, int TPV>
struct MxRead {
    static constexpr uint32_t d(int e) { return (COLS ? (e >> 2) : 16 * (e >> 2)) + (e & 3) * TPV; }
};
template <bool COLS, int NS>
struct MxStore {
    // columns: k = (J0 mod NS) + b (NS >= 16) or 0 (NS = 1); rows: k = 0
    // (NS = 1; jp - k moves by 16 b), k = n for NS = 16 (jp - k moves by
    // 16 b), k = (J0 mod NS) + 16 b for NS >= 64 (jp - k fixed)
    static constexpr uint32_t d(int e) {
        const int b = e >> 2, t = e & 3;
        if (COLS) return NS == 1 ? 16 * b + t : b + t * NS;
        return NS == 1 ? 256 * b + t : NS == 16 ? 256 * b + 16 * t : 16 * b + t * NS;
    }
};
template <int TPV>
struct MxCanon {
    static constexpr uint32_t d(int e) { return TPV * e; }
};
// The 16 accesses grouped by their XOR term (first appearance order):
// accesses from one base are issued next to each other, so the compiler
// can merge pairs of them into one two-address instruction.
struct Ord16 {
    int v[16];
};
template <class W, class D>
constexpr Ord16 mx_order() {
    Ord16 o{};
    uint32_t key[16] = {};
    for (int e = 0; e < 16; ++e) key[e] = W::xpart(D::d(e));
    int k = 0;
    for (int e = 0; e < 16; ++e) {
        bool first = true;
        for (int f = 0; f < e; ++f)
            if (key[f] == key[e]) first = false;
        if (!first) continue;
        for (int f = e; f < 16; ++f)
            if (key[f] == key[e]) o.v[k++] = f;
    }
    return o;
}
// fn(e, D(e)) for the 16 accesses, grouped by base
template <class W, class D, class Fn>
__device__ __forceinline__ void mx_each(Fn&& fn) {
    constexpr Ord16 o = mx_order<W, D>();
    static_for<16>([&](auto ii) {
        constexpr int e = o.v[decltype(ii)::value];
        fn(std::integral_constant<int, e>{}, std::integral_constant<uint32_t, D::d(e)>{});
    });
}

// Full length-L float16 transform with its radix-16 stages on the matrix
// cores and the final small-radix stage (if any) in packed float16 vector
// arithmetic: the same numbers as fft_wg<..., HALF_NORM, TT> but for the
// butterfly sums.  v holds the input in the matrix-core layout (mx_pos),
// or with IN_CANON in the canonical one (positions j + TPV e, moved
// through LDS first), and receives the output in the canonical layout.
// Twiddles come from the tables ttab (fill_twiddle_tables).  buf is the
// vector's LDS: L dwords for a row, or for columns the first of 16
// interleaved vectors (16 L dwords from the tile, offset by the vector).
// Every thread of the workgroup calls this together.  Without LEAD the
// caller guarantees that no thread still reads the vector's LDS.  hook()
// runs after the stores of the last exchange, before its barrier.
template <int LOG2L, int DIR, bool HALF_NORM, bool COLS, bool LEAD = true, bool IN_CANON = false,
          class Hook = NoHook>
__device__ __forceinline__ void fft_mx(h2 (&v)[16], int j, h2* buf, const h2* ttab, const Hook& hook = Hook{}) {
    using S = Sched<LOG2L>;
    using T = TwTab<LOG2L>;
    constexpr int L = 1 << LOG2L;
    constexpr int TPV = L / 16;
    static_assert(kMxShape<LOG2L, COLS>, "matrix-core transform shape");
    asm volatile("" : "+v"(j));
    const int g = mx_g<COLS>(j);
    const Dft16H m = dft16_h<DIR>((int)(threadIdx.x & 63), 1.0f);
    // Batch-0 butterfly of the thread: rows J0 = 64 (j / 64) + n, columns
    // J0 = 4 (j / 4); batch b is J0 + 16 b (rows) or J0 + b (columns).
    const int n = COLS ? 0 : (j & 15);
    const int J0 = COLS ? 4 * (j >> 2) : (j & ~63) + n;
    // inputs q = 4g + t of butterfly J0 + db: position J0 + 4g TPV + (db + t TPV)
    auto read_mx = [&](auto xi, h2(&x)[16]) {
        using W = MxSwz<LOG2L, COLS, decltype(xi)::value>;
        const uint32_t mb = W::base(J0 + 4 * g * TPV);
        mx_each<W, MxRead<COLS, TPV>>([&](auto ei, auto di) {
            x[decltype(ei)::value] = buf[W::template at<decltype(di)::value>(mb)];
        });
    };
    if constexpr (IN_CANON) {
        using W = MxSwz<LOG2L, COLS, 0>;
        if constexpr (LEAD) __syncthreads();
        const uint32_t mb = W::base(j);
        mx_each<W, MxCanon<TPV>>([&](auto ei, auto di) {
            buf[W::template at<decltype(di)::value>(mb)] = v[decltype(ei)::value];
        });
        __syncthreads();
        read_mx(std::integral_constant<int, 0>{}, v);
    }
    static_for<S::kFull>([&](auto si) {
        constexpr int s = decltype(si)::value;
        constexpr int NS = S::ns(s);
        constexpr bool SC = HALF_NORM && s > 0 && (s % 2 == 0);
        constexpr bool LASTMX = s == S::kFull - 1;
        h2 x[16];
        if constexpr (s == 0) {
#pragma unroll
            for (int e = 0; e < 16; ++e) x[e] = v[e];
        } else {
            read_mx(std::integral_constant<int, s>{}, x);
        }
        if constexpr (NS > 1) {
            constexpr int oA = T::offA(s), oB = T::offB(s);
            // k = jp mod NS: rows k = (J0 mod NS) + 16 b (no wrap: 16 b + n < 64);
            // columns k = (J0 mod NS) + b (J0 mod NS a multiple of 4)
            const int k0 = opaque_i(J0 & (NS - 1));
            const h2* tb0 = ttab + oB + (k0 & 15) * kTabStride + 4 * g;
            const h2* ta0 = ttab + oA + (k0 >> 4) * kTabStride + 4 * g;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                // B row lo = k mod 16, A row hi = k / 16
                const int dlo = COLS ? b : 0, dhi = COLS ? 0 : b;
                const uint4 wb = *reinterpret_cast<const uint4*>(tb0 + dlo * kTabStride);
                h2 w[4] = {__builtin_bit_cast(h2, wb.x), __builtin_bit_cast(h2, wb.y), __builtin_bit_cast(h2, wb.z),
                           __builtin_bit_cast(h2, wb.w)};
                if constexpr (NS > 16) {
                    const uint4 wa = *reinterpret_cast<const uint4*>(ta0 + dhi * kTabStride);
                    w[0] = cmul(__builtin_bit_cast(h2, wa.x), w[0]);
                    w[1] = cmul(__builtin_bit_cast(h2, wa.y), w[1]);
                    w[2] = cmul(__builtin_bit_cast(h2, wa.z), w[2]);
                    w[3] = cmul(__builtin_bit_cast(h2, wa.w), w[3]);
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) x[4 * b + t] = DIR < 0 ? cmul(x[4 * b + t], w[t]) : cmulc(x[4 * b + t], w[t]);
            }
        }
        if constexpr (SC) {
#pragma unroll
            for (int e = 0; e < 16; ++e) x[e] = cscale(x[e], (_Float16)0.0625f);
        }
        h2 y[16];
#pragma unroll
        for (int b = 0; b < 4; ++b) mfma_dft16_h(m, x + 4 * b, y + 4 * b);
        // every thread has read this stage's inputs before any output lands
        if constexpr (s > 0 || LEAD || IN_CANON) __syncthreads();
        // output s' = 4g + t of butterfly jp = J0 + db (k = jp mod NS) goes to
        // (jp - k) 16 + k + s' NS; the base is that of batch 0, t = 0
        {
            using W = MxSwz<LOG2L, COLS, s + 1>;
            const int kk = J0 & (NS - 1);
            const uint32_t mb = W::base((J0 - kk) * 16 + kk + 4 * g * NS);
            mx_each<W, MxStore<COLS, NS>>([&](auto ei, auto di) {
                buf[W::template at<decltype(di)::value>(mb)] = y[decltype(ei)::value];
            });
        }
        if constexpr (LASTMX) hook();
        __syncthreads();
    });
    {
        using W = MxSwz<LOG2L, COLS, S::kFull>;
        const uint32_t mb = W::base(j);
        mx_each<W, MxCanon<TPV>>([&](auto ei, auto di) {
            v[decltype(ei)::value] = buf[W::template at<decltype(di)::value>(mb)];
        });
    }
    if constexpr (S::kRem > 1) {
        constexpr int s = S::kStages - 1;
        constexpr bool SC = HALF_NORM && s > 0 && (s % 2 == 0);
        h2 tw[16];
        stage_tw_tab<LOG2L, s>(ttab, j, tw);
        stockham_stage<L, S::kRem, S::ns(s), DIR, true, SC>(v, j, cone<h2>(), NoLds<h2>{}, tw);
    }
}

// ------------------------------------------------------------- misc
// Workgroup index remapped so that consecutive logical indices run on the
// same XCD (workgroups are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_logical(int bid, int grid) {
    const int per = grid >> 3;  // grid is a multiple of 8
    return (bid & 7) * per + (bid >> 3);
}

}  // namespace pond
