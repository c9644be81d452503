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

// ------------------------------------------------- matrix-core DFT-16
// A 16-point complex DFT is a real 32 x 32 matrix product; the 16 x 32 half
// that yields real (or imaginary) outputs is one v_mfma_f32_16x16x32_f16
// operand.  Lane layout of that instruction (wave64): lane l holds
//   A[l % 16][8 (l / 16) + t]   and   B[8 (l / 16) + t][l % 16],  t < 8,
//   D[4 (l / 16) + t][l % 16],  t < 4.
// With the input vector interleaved as (Re x0, Im x0, Re x1, ...) along K,
// lane (g = l / 16, n = l % 16) supplies inputs q = 4g..4g+3 of vector n and
// receives outputs s = 4g..4g+3 of vector n.
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// The DFT matrix is carried as a float16 pair hi + lo (lo = the rounding
// error of hi): a single float16 matrix would give every output a fixed
// ~1e-4 gain error, which does not average out in a folded profile.
struct Dft16Operands {
    half8_t re_hi, re_lo, im_hi, im_lo;
};

__device__ __forceinline__ floatx4_t mfma16x16x32(const half8_t& hi, const half8_t& lo, const half8_t& b) {
    const floatx4_t z = {0.f, 0.f, 0.f, 0.f};
    const floatx4_t c = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo, b, z, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(hi, b, c, 0, 0, 0);
}

__device__ __forceinline__ void split_half(float x, _Float16& hi, _Float16& lo) {
    hi = (_Float16)x;
    lo = (_Float16)(x - (float)hi);
}

// cos and sin of 2 pi e / 16, e < 16 (float32 nearest to the exact values).
__constant__ const float kCos16[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                                       0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                                       -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                                       0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};

// This lane's A operands for scale * exp(DIR 2 pi i q s / 16): rows of real
// outputs hold (Re c, -Im c) per input q, rows of imaginary outputs (Im c, Re c).
template <int DIR>
__device__ __forceinline__ Dft16Operands dft16_operands(int lane, float scale) {
    const int s = lane & 15;
    const int g = lane >> 4;
    Dft16Operands m;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int e = ((4 * g + t) * s) & 15;
        const float cs = kCos16[e], sn = kCos16[(e + 12) & 15];  // sin x = cos(x - pi/2)
        const float cr = scale * cs, ci = scale * (DIR < 0 ? -sn : sn);
        _Float16 h, l;
        split_half(cr, h, l);
        m.re_hi[2 * t] = h;
        m.re_lo[2 * t] = l;
        m.im_hi[2 * t + 1] = h;
        m.im_lo[2 * t + 1] = l;
        split_half(-ci, h, l);
        m.re_hi[2 * t + 1] = h;
        m.re_lo[2 * t + 1] = l;
        split_half(ci, h, l);
        m.im_hi[2 * t] = h;
        m.im_lo[2 * t] = l;
    }
    return m;
}

// One radix-16 Stockham stage on matrix cores for 16 interleaved columns of
// length L (thread c = tid % 16, j = tid / 16; wave lane = 16 (j % 4) + c).
// The wave owns butterflies jp = (j & ~3) + b, b < 4, one MFMA batch each
// (the 16 columns share the butterfly's twiddles).  src(pos) returns this
// lane's column at pos; dst(pos, y) receives outputs.  If SYNC, a barrier
// separates all reads from all writes (in-place LDS stages).
template <int L, int NS, int DIR, bool SYNC, class Src, class Dst>
__device__ __forceinline__ void mfma16_stage_cols(int j, const Dft16Operands& m, const float2* __restrict__ tw,
                                                  Src&& src, Dst&& dst) {
    asm volatile("" : "+v"(j));
    const int g = j & 3;
    const int jb = j & ~3;
    floatx4_t dre[4], dim[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int jp = jb + b;
        const int k = jp & (NS - 1);
        half8_t bv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int q = 4 * g + t;
            float2 x = src(jp + q * (L / 16));
            if constexpr (NS > 1) {
                const float2 w = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(tw) +
                                                                  (uint32_t)(q * k * (L / (16 * NS))) * 8u);
                x = DIR < 0 ? cmul(x, w) : cmulc(x, w);
            }
            bv[2 * t] = (_Float16)x.x;
            bv[2 * t + 1] = (_Float16)x.y;
        }
        dre[b] = mfma16x16x32(m.re_hi, m.re_lo, bv);
        dim[b] = mfma16x16x32(m.im_hi, m.im_lo, bv);
    }
    if constexpr (SYNC) __syncthreads();
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int jp = jb + b;
        const int k = jp & (NS - 1);
#pragma unroll
        for (int t = 0; t < 4; ++t) dst((jp - k) * 16 + k + (4 * g + t) * NS, make_float2(dre[b][t], dim[b][t]));
    }
}

// Length-L transform of 16 interleaved columns with the radix-16 stages on
// matrix cores (operands in float16, accumulation in float32) and the final
// small-radix stage, if any, in float32 arithmetic.  Each radix-16 stage is
// scaled by scale16 (folded into the matrix), the small stage by scale_rem.
// in(pos) gives the first stage's input for this lane's column; out(pos, y)
// receives every output of this lane's column exactly once.  lds(pos) is
// the float2 slot of this column at pos.  With OUT_SYNC a barrier precedes
// the first out() call (out may then reuse the LDS).  Contains barriers.
template <int LOG2L, int DIR, bool OUT_SYNC, class In, class Lds, class Out>
__device__ __forceinline__ void colfft_mfma(int c, int j, const float2* __restrict__ tw, const StageBases<LOG2L>& tb,
                                            float scale16, float scale_rem, In&& in, Lds&& lds, Out&& out) {
    using S = Sched<LOG2L>;
    constexpr int L = 1 << LOG2L;
    constexpr int TPV = L / 16;
    // A wave must hold 4 butterflies of 16 columns: L >= 64.
    static_assert(LOG2L >= 6, "matrix-core column transform needs columns of at least 64 points");
    const Dft16Operands m = dft16_operands<DIR>(threadIdx.x & 63, scale16);
    auto from_lds = [&](int pos) { return lds(pos); };
    auto to_lds = [&](int pos, float2 y) { lds(pos) = y; };
    static_for<S::kFull>([&](auto si) {
        constexpr int s = decltype(si)::value;
        constexpr int NS = S::ns(s);
        constexpr bool LAST = (s == S::kStages - 1);
        if constexpr (s == 0) {
            if constexpr (LAST) mfma16_stage_cols<L, NS, DIR, OUT_SYNC>(j, m, tw, in, out);
            else mfma16_stage_cols<L, NS, DIR, false>(j, m, tw, in, to_lds);
        } else {
            __syncthreads();
            if constexpr (LAST) mfma16_stage_cols<L, NS, DIR, true>(j, m, tw, from_lds, out);
            else mfma16_stage_cols<L, NS, DIR, true>(j, m, tw, from_lds, to_lds);
        }
    });
    if constexpr (S::kRem > 1) {
        constexpr int s = S::kStages - 1;
        __syncthreads();
        float2 v[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = lds(j + TPV * e);
        stockham_stage<L, S::kRem, S::ns(s), DIR, true>(v, j, tb.b[s], [](int, float2) {});
        if constexpr (OUT_SYNC) __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) out(j + TPV * e, cscale(v[e], scale_rem));
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
