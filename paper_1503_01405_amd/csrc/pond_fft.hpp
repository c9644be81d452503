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

#include <utility>

namespace pond {

// ---------------------------------------------------------------- complex
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
// a * exp(DIR * i pi / 2): DIR = -1 multiplies by -i, DIR = +1 by +i
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
    if constexpr (DIR < 0) return make_float2(a.y, -a.x);
    else return make_float2(-a.y, a.x);
}
// a * exp(DIR * i pi / 4)
template <int DIR>
__device__ __forceinline__ float2 mul_w8(float2 a) {
    constexpr float h = 0.70710678118654752440f;
    if constexpr (DIR < 0) return make_float2((a.x + a.y) * h, (a.y - a.x) * h);
    else return make_float2((a.x - a.y) * h, (a.x + a.y) * h);
}
// a * exp(DIR * 3 i pi / 4)
template <int DIR>
__device__ __forceinline__ float2 mul_w8_3(float2 a) {
    constexpr float h = 0.70710678118654752440f;
    if constexpr (DIR < 0) return make_float2((a.y - a.x) * h, -(a.x + a.y) * h);
    else return make_float2(-(a.x + a.y) * h, (a.x - a.y) * h);
}
// a * (c + DIR*i*s) for a constant point on the unit circle
template <int DIR>
__device__ __forceinline__ float2 mul_cs(float2 a, float c, float s) {
    if constexpr (DIR < 0) return make_float2(fmaf(a.x, c, a.y * s), fmaf(a.y, c, -(a.x * s)));
    else return make_float2(fmaf(a.x, c, -(a.y * s)), fmaf(a.y, c, a.x * s));
}

// --------------------------------------------------------- small DFTs
// In-place DFT of R values, natural order in and out:
//   V[s] = sum_q v[q] exp(DIR * 2 pi i q s / R)   (DIR = -1 forward)
template <int DIR>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
    float2 a0 = cadd(v0, v2), a1 = csub(v0, v2);
    float2 a2 = cadd(v1, v3), a3 = mul_i<DIR>(csub(v1, v3));
    v0 = cadd(a0, a2);
    v2 = csub(a0, a2);
    v1 = cadd(a1, a3);
    v3 = csub(a1, a3);
}

template <int R, int DIR>
struct Dft;

template <int DIR>
struct Dft<2, DIR> {
    __device__ __forceinline__ static void run(float2* v) { dft2<DIR>(v[0], v[1]); }
};

template <int DIR>
struct Dft<4, DIR> {
    __device__ __forceinline__ static void run(float2* v) { dft4<DIR>(v[0], v[1], v[2], v[3]); }
};

// 8 = 2 x 4: two 4-point DFTs on the even/odd subsequences, twiddle, 2-point.
template <int DIR>
struct Dft<8, DIR> {
    __device__ __forceinline__ static void run(float2* v) {
        dft4<DIR>(v[0], v[2], v[4], v[6]);
        dft4<DIR>(v[1], v[3], v[5], v[7]);
        v[3] = mul_w8<DIR>(v[3]);
        v[5] = mul_i<DIR>(v[5]);
        v[7] = mul_w8_3<DIR>(v[7]);
        float2 o[8];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            float2 a = v[2 * sb], b = v[2 * sb + 1];
            o[sb] = cadd(a, b);
            o[sb + 4] = csub(a, b);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = o[i];
    }
};

// 16 = 4 x 4: q = qa + 4 qb, s = sb + 4 sa.
template <int DIR>
struct Dft<16, DIR> {
    __device__ __forceinline__ static void run(float2* v) {
        constexpr float c1 = 0.92387953251128675613f;  // cos(pi/8)
        constexpr float s1 = 0.38268343236508977173f;  // sin(pi/8)
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
        float2 o[16];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) {
            float2 a0 = v[0 + 4 * sb], a1 = v[1 + 4 * sb], a2 = v[2 + 4 * sb], a3 = v[3 + 4 * sb];
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
// exp(-2 pi i u / 16) for a compile-time u.
template <int U>
__device__ __forceinline__ float2 w16() {
    constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    constexpr float h = 0.70710678118654752440f;
    constexpr float cs[16][2] = {{1.f, 0.f},  {c1, -s1},  {h, -h},   {s1, -c1},  {0.f, -1.f}, {-s1, -c1},
                                 {-h, -h},    {-c1, -s1}, {-1.f, 0.f}, {-c1, s1}, {-h, h},     {-s1, c1},
                                 {0.f, 1.f},  {s1, c1},   {h, h},    {c1, s1}};
    return make_float2(cs[U & 15][0], cs[U & 15][1]);
}

// p[q] = w^q for q = 1..R-1 (p[0] unused), products at most four deep.
template <int R>
__device__ __forceinline__ void powers(float2 w, float2 (&p)[R]) {
    p[0] = make_float2(1.f, 0.f);
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
template <int LOG2L>
struct StageBases {
    float2 b[Sched<LOG2L>::kStages];
    __device__ __forceinline__ void load(int j, const float2* __restrict__ tw) {
        using S = Sched<LOG2L>;
        constexpr int L = 1 << LOG2L;
        static_for<S::kStages>([&](auto si) {
            constexpr int s = decltype(si)::value;
            constexpr int NS = S::ns(s);
            constexpr int R = S::radix(s);
            if constexpr (NS > 1) {
                if constexpr (R == 16) b[s] = tw[(j & (NS - 1)) * (L / (16 * NS))];
                else b[s] = tw[j];
            } else {
                b[s] = make_float2(1.f, 0.f);
            }
        });
    }
};

// One Stockham stage of radix R on the 16 values of thread j.  Butterfly u
// (index jp = j + TPV u, k = jp mod NS) reads positions jp + q L/R, which
// are registers u + q BF, twiddles input q by W_{NS R}^(q k), and writes
// output q to position (jp - k) R + k + q NS.
template <int L, int R, int NS, int DIR, bool LAST, class Store>
__device__ __forceinline__ void stockham_stage(float2 (&v)[16], int j, float2 base, Store&& st) {
    // Opaque to the optimiser: the twiddle powers and LDS addresses of a
    // stage are recomputed at each use instead of being shared between the
    // forward and inverse transforms (or hoisted out of loops) and held in
    // registers, which costs occupancy.
    asm volatile("" : "+v"(base.x), "+v"(base.y), "+v"(j));
    constexpr int BF = 16 / R;
    constexpr int TPV = L / 16;
    float2 pw[R];
    if constexpr (NS > 1 && R == 16) powers<R>(base, pw);
    static_for<BF>([&](auto ui) {
        constexpr int u = decltype(ui)::value;
        const int jp = j + TPV * u;
        const int k = jp & (NS - 1);
        float2 w[R];
#pragma unroll
        for (int q = 0; q < R; ++q) w[q] = v[u + q * BF];
        if constexpr (NS > 1) {
            if constexpr (R < 16) {
                const float2 bu = u == 0 ? base : cmul(base, w16<u>());
                powers<R>(bu, pw);
            }
#pragma unroll
            for (int q = 1; q < R; ++q) w[q] = DIR < 0 ? cmul(w[q], pw[q]) : cmulc(w[q], pw[q]);
        }
        Dft<R, DIR>::run(w);
        if constexpr (LAST) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[u + q * BF] = w[q];
        } else {
            const int basep = (jp - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) st(basep + q * NS, w[q]);
        }
    });
}

// Full length-L transform (DIR = -1 forward, +1 inverse, unnormalised) of
// the vector held by thread j.  ld(pos) / st(pos, val) access this
// vector's LDS slot; every thread of the workgroup must call this together
// (it contains barriers).
template <int LOG2L, int DIR, class Load, class Store>
__device__ __forceinline__ void fft_wg(float2 (&v)[16], int j, const StageBases<LOG2L>& tb, Load&& ld,
                                       Store&& st) {
    using S = Sched<LOG2L>;
    constexpr int L = 1 << LOG2L;
    constexpr int TPV = L / 16;
    static_for<S::kStages>([&](auto si) {
        constexpr int s = decltype(si)::value;
        constexpr int R = S::radix(s);
        constexpr int NS = S::ns(s);
        constexpr bool LAST = (s == S::kStages - 1);
        if constexpr (!LAST) {
            __syncthreads();
            stockham_stage<L, R, NS, DIR, false>(v, j, tb.b[s], st);
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = ld(j + TPV * e);
        } else {
            stockham_stage<L, R, NS, DIR, true>(v, j, tb.b[s], st);
        }
    });
}

// ------------------------------------------------------------- misc
// Workgroup index remapped so that consecutive logical indices run on the
// same XCD (workgroups are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_logical(int bid, int grid) {
    const int per = grid >> 3;  // grid is a multiple of 8
    return (bid & 7) * per + (bid >> 3);
}

}  // namespace pond
