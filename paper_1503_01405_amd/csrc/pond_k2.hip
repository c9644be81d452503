// K2: the middle (row) pass of the four-step transform: four-step
// twiddle, forward row FFT, inverse ISM response, inverse row FFT,
// conjugate twiddle; and the tables it reads.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "pond_device.hpp"

namespace pond {

// Row table of the middle pass per (k2, k1): exp(-2 pi i turns_k) times the
// taper, k = k2 + n2 k1, the inverse ISM response of Sec. 3.7 / Eq. (4)
// (turns_k and its reduction mod 1 in float64), preceded with TW by the
// four-step twiddle W_n^(k1 k2) (float4; float2 without, for the float32
// form, whose row kernel forms the twiddle itself).
// Built once per plan; every block reads the same table.
template <bool TW>
__global__ void __launch_bounds__(256) k2_build_table(void* __restrict__ tab, int log2n1, int log2n2, double chirp_a,
                                                       double f0, double df, double taper) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int log2n = log2n1 + log2n2;
    const int64_t n = 1ll << log2n;
    if (i >= n) return;
    const int64_t k2 = i >> log2n1;
    const int64_t k1 = i & ((1ll << log2n1) - 1);
    const int64_t k = k2 + (k1 << log2n2);
    const int64_t kk = k < (n >> 1) ? k : k - n;
    const double f = (double)kk * df;
    const double turns = chirp_a * (f * f) / (f0 + f);
    const double frac = turns - rint(turns);
    double cs, cc;
    sincospi(2.0 * frac, &cs, &cc);
    const double w = taper_w(f, df * (double)n, taper);
    if constexpr (TW) {
        const int64_t r = (k1 * k2) & (n - 1);
        double s, c;
        sincospi(2.0 * (double)r / (double)n, &s, &c);
        reinterpret_cast<float4*>(tab)[i] = make_float4((float)c, (float)-s, (float)(cc * w), (float)(-cs * w));
    } else {
        reinterpret_cast<float2*>(tab)[i] = make_float2((float)(cc * w), (float)(-cs * w));
    }
}

// One workgroup takes row k2 (ROWS rows for short rows) of one block.  The
// workgroups of one row for all blocks of the launch get consecutive logical
// indices on one XCD, so they run together and share the row's table entries
// through that XCD's L2 (the table is then fetched from HBM about once per
// launch).
//   MODE kRowFull: twiddle, forward FFT, chirp, inverse FFT, conjugate
//                  twiddle, in place.  Float32 form: float2 chirp table, the
//                  twiddle W_N^(k2 n) = lo[n mod LO] hi[n / LO] from two
//                  per-row float32 tables the workgroup forms in LDS (RowTw;
//                  the float32 rows read 16 bytes per element besides it).
//                  Float16 / bfloat16 storage with float32 arithmetic: a
//                  float4 table (twiddle, chirp).  Float16 arithmetic: two
//                  float16 pairs per element (twiddle / 16, chirp * 2^-rem).
//                  Forming the twiddle in the row kernel measured faster only
//                  in the float32 form; in the others it costs registers
//                  (float16: 61 -> 92, occupancy 8 -> 5 waves) and time.
//   MODE kRowFwd:  twiddle and forward FFT only, in place: leaves the block's
//                  spectrum, row k2 holding bins k2 + n2 k1 (float2 twiddle table).
//   MODE kRowInv:  spectrum (in) times one trial's chirp, inverse FFT,
//                  conjugate twiddle, to `out`; the chirp is formed from the
//                  trial's DM and the shared float64 table of turns per unit
//                  DM (dm_chirp).
//   MODE kRowInvPlain: kRowInv without the chirp (float32 arithmetic only).
//   MODE kRowChirp: forward FFT, chirp (float2 or float16 table in the rows'
//                  order), inverse FFT, in place, no twiddles (the sub-rows
//                  of the split middle pass; the float16 forms' input already
//                  carries the first stage's 1/16).
// F16: packed float16 arithmetic on float16 storage with float16 tables
// (kRowFull: 4 halves per entry, twiddle/16 and chirp*2^-kHalfRem; split
// modes: twiddle/16 and chirp).  The forward transform is normalised stage
// by stage (1/16 of the first stage in the twiddle table), so the spectrum
// is the block's spectrum / n; the output is 1/16 of the float32 forms'.
// MXF (with F16, rows of 2^10 and more): the radix-16 stages' butterfly
// sums on the matrix cores (fft_mx), inputs loaded in their layout.
// Four-step twiddles of a workgroup's rows for the full middle pass:
// W_N^(k2 n) = lo[n mod LO] * hi[n / LO] with lo[t] = W_N^(k2 t) and hi[u] =
// W_N^(k2 LO u), LO = 2^floor(log2(n1) / 2), each entry the float32 sine and
// cosine of an exactly representable phase (k2 t mod N < 2^24): the product
// is within a few float32 ulps of the exact twiddle, and the tables cost the
// workgroup (LO + n1 / LO) sine/cosine pairs instead of a table read per
// element.
template <int LOG2N1>
struct RowTw {
    static constexpr int LOG2LO = LOG2N1 / 2;
    static constexpr int LO = 1 << LOG2LO;
    static constexpr int HI = (1 << LOG2N1) >> LOG2LO;
    static constexpr int PER_ROW = LO + HI;
    // rows row0 .. row0 + ROWS - 1 (k2), all threads of the workgroup
    template <int ROWS, int THREADS>
    __device__ __forceinline__ static void fill(float2* t, int row0, int log2n, int tid) {
        const uint32_t nmask = (1u << log2n) - 1u;
        const float scale = 2.0f / (float)(1u << log2n);  // exact: a power of two
        for (int i = tid; i < ROWS * PER_ROW; i += THREADS) {
            const int rr = i / PER_ROW, k = i - rr * PER_ROW;
            const uint32_t k2 = (uint32_t)(row0 + rr);
            const uint32_t e = k < LO ? (uint32_t)k : (uint32_t)(k - LO) << LOG2LO;
            float sn, cs;
            sincospif((float)((k2 * e) & nmask) * scale, &sn, &cs);
            t[i] = make_float2(cs, -sn);
        }
    }
    // W_N^(k2 n) of row rr of the workgroup at position n of the row
    __device__ __forceinline__ static float2 at(const float2* t, uint32_t rr, uint32_t n) {
        const float2* b = t + rr * PER_ROW;
        return cmul(b[n & (LO - 1)], b[LO + (n >> LOG2LO)]);
    }
};

// exp(-2 pi i turns) of one trial's chirp at a bin with turns = dm g (Eq.
// (4) with the DM factored out): the product and the reduction mod 1 in
// float64, the sine and cosine of the reduced phase in float32.
__device__ __forceinline__ float2 dm_chirp(double dm, double g) {
    const double turns = dm * g;
    const float frac = (float)(turns - rint(turns));
    float sn, cs;
    sincospif(2.0f * frac, &sn, &cs);
    return make_float2(cs, -sn);
}

template <int LOG2N1, class T, int MODE, bool F16, bool MXF = false>
__global__ void __launch_bounds__(K2Shape<LOG2N1>::THREADS)
    __attribute__((amdgpu_waves_per_eu(MXF && (MODE == kRowFull || MODE == kRowChirp) && LOG2N1 >= 13 ? 8 : 4)))
k2_row(K2Args a) {
    using Sh = K2Shape<LOG2N1>;
    using V = std::conditional_t<F16, h2, float2>;
    constexpr bool MX = F16 && MXF && kMxShape<LOG2N1, false>;
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
    using RowL = std::conditional_t<F16 && !MX && LOG2N1 >= 12, StageRowLds<V>, PadLds<V>>;
    const RowL lrow{lds + r * Sh::STRIDE};
    static_assert(!(F16 && !MX && LOG2N1 >= 12) || (Sh::STRIDE >= (1 << LOG2N1) + 16 * ((1 << LOG2N1) >> 8)),
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
        __shared__ __align__(16) h2 ttab[TwTab<LOG2N1>::kSize];
        // one wave fills the tables: every stage's for the matrix-core form,
        // stage 1's for the packed-float16 form (its other stages form their
        // twiddles from float32 powers, which measures faster here)
        if (threadIdx.x < 64) fill_twiddle_tables<LOG2N1, 64, !MX>(ttab, a.tw1, threadIdx.x);
        const uint2* tab = reinterpret_cast<const uint2*>(a.htable) + ((int64_t)row0 << LOG2N1);
        const h2* tw4 = reinterpret_cast<const h2*>(a.htw4) + ((int64_t)row0 << LOG2N1);
        const h2* chirp = reinterpret_cast<const h2*>(a.hchirp) + ((int64_t)row0 << LOG2N1);
        const double* geo = a.geo + ((int64_t)row0 << LOG2N1);
        // Element u + i of the workgroup's rows through buffer descriptors:
        // u (uniform) is the scalar offset, i the lane's, so that a thread's
        // 16 accesses share one vector offset per array.
        constexpr uint32_t kEl = (uint32_t)Sh::ROWS << LOG2N1;  // elements of the rows
        const BufRes rsrc = buf_res(src, kEl * (uint32_t)sizeof(T));
        const BufRes rdst = buf_res(dst, kEl * (uint32_t)sizeof(T));
        const BufRes rtab = buf_res(tab, kEl * 8u);
        const BufRes rtw4 = buf_res(tw4, kEl * 4u);
        const BufRes rchirp = buf_res(chirp, kEl * 4u);
        auto tw_at = [&](int u, uint32_t i) {
            if constexpr (MODE == kRowFull) return buf_ld<h2>(rtab, i * 8u, u * 8);
            else return buf_ld<h2>(rtw4, i * 4u, u * 4);
        };
        h2 v[16];
        uint32_t to = opaque(toff);
        // MX: value e at the matrix-core position mx_pos(j, e) of the row
        const uint32_t mxo = opaque(toff - (uint32_t)j + (uint32_t)mx_pos<false, TPV>(j, 0));
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int u = MX ? 16 * (e >> 2) + (e & 3) * TPV : TPV * e;
            const uint32_t i = MX ? mxo : to;
            const h2 x = buf_ld<h2>(rsrc, i * (uint32_t)sizeof(T), u * (int)sizeof(T));
            if constexpr (MODE == kRowInv) v[e] = cmul(x, to_h2(dm_chirp(a.dm, *at(geo + u, i * 8u))));
            else if constexpr (MODE == kRowChirp) v[e] = x;
            else v[e] = cmul(x, tw_at(u, i));
        }
        // kRowFull: the chirp of each element is fetched during the forward
        // transform's last exchange.
        h2 ch[16];
        auto fetch_chirp = [&] {
            const uint32_t t2 = opaque(toff);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                if constexpr (MODE == kRowChirp) ch[e] = buf_ld<h2>(rchirp, t2 * 4u, TPV * e * 4);
                else ch[e] = buf_ld<h2>(rtab, t2 * 8u, TPV * e * 8 + 4);
            }
        };
        if constexpr (MX) {
            // first LDS use of the row: no barrier before the first stores
            if constexpr (MODE == kRowFull || MODE == kRowChirp)
                fft_mx<LOG2N1, -1, true, false, false>(v, j, lrow.base, ttab, fetch_chirp);
            else if constexpr (MODE != kRowInv) fft_mx<LOG2N1, -1, true, false, false>(v, j, lrow.base, ttab);
        } else {
            if constexpr (MODE == kRowFull || MODE == kRowChirp)
                fft_wg<LOG2N1, -1, true, 1>(v, j, tb, lrow, ttab, fetch_chirp);
            else if constexpr (MODE != kRowInv) fft_wg<LOG2N1, -1, true, 1>(v, j, tb, lrow, ttab);
        }
        if constexpr (MODE == kRowFwd) {
            constexpr float osc = 1.0f / (float)(1 << Sched<LOG2N1>::kHalfRem);
            if (valid) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    buf_st<h2>(rdst, to * (uint32_t)sizeof(T), TPV * e * (int)sizeof(T), v[e] * (_Float16)osc);
            }
            return;
        }
        if constexpr (MODE == kRowFull || MODE == kRowChirp) {
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = cmul(v[e], ch[e]);
        }
        if constexpr (MODE == kRowChirp) {
            if constexpr (MX) fft_mx<LOG2N1, +1, false, false, true, true>(v, j, lrow.base, ttab);
            else fft_wg<LOG2N1, +1, false, 1>(v, j, tb, lrow, ttab);
            asm volatile("" ::: "memory");
            to = opaque(toff);
            if (valid) {
#pragma unroll
                for (int e = 0; e < 16; ++e) buf_st<h2>(rdst, to * (uint32_t)sizeof(T), TPV * e * (int)sizeof(T), v[e]);
            }
            return;
        }
        // the output twiddles are fetched during the inverse transform's
        // last exchange (rather than one dependent load per store)
        h2 wo[16];
        auto fetch_tw = [&] {
            const uint32_t t2 = opaque(toff);
#pragma unroll
            for (int e = 0; e < 16; ++e) wo[e] = tw_at(TPV * e, t2);
        };
        if constexpr (MX && MODE == kRowFull)  // input in registers (canonical), moved through LDS
            fft_mx<LOG2N1, +1, false, false, true, true>(v, j, lrow.base, ttab, fetch_tw);
        else if constexpr (MX)  // kRowInv: input loaded in the matrix-core layout, first LDS use
            fft_mx<LOG2N1, +1, false, false, false>(v, j, lrow.base, ttab, fetch_tw);
        else fft_wg<LOG2N1, +1, false, 1>(v, j, tb, lrow, ttab, fetch_tw);
        asm volatile("" ::: "memory");
        to = opaque(toff);
        if (valid) {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                buf_st<h2>(rdst, to * (uint32_t)sizeof(T), TPV * e * (int)sizeof(T), cmulc(v[e], wo[e]));
        }
        return;
    } else {
        // float32 storage: twiddles formed here, float2 chirp table;
        // otherwise the float4 table (twiddle, chirp)
        constexpr bool OTF = std::is_same<T, float2>::value;
        const float2* tab = reinterpret_cast<const float2*>(a.table) + ((int64_t)row0 << LOG2N1);
        const float4* tab4 = reinterpret_cast<const float4*>(a.table) + ((int64_t)row0 << LOG2N1);
        __shared__ float2 rtw[MODE == kRowFull && OTF ? Sh::ROWS * RowTw<LOG2N1>::PER_ROW : 1];
        if constexpr (MODE == kRowFull && OTF) {
            RowTw<LOG2N1>::template fill<Sh::ROWS, Sh::THREADS>(rtw, row0, LOG2N1 + a.log2n2, threadIdx.x);
            __syncthreads();
        }
        auto tw_row = [&](int u, uint32_t i) {
            if constexpr (OTF) {
                const uint32_t k = i + (uint32_t)u;
                return RowTw<LOG2N1>::at(rtw, k >> LOG2N1, k & ((1u << LOG2N1) - 1u));
            } else {
                const float4 t = *at(tab4 + u, i * 16u);
                return make_float2(t.x, t.y);
            }
        };
        const float2* tw4 = a.tw4 + ((int64_t)row0 << LOG2N1);
        const float2* chirp = a.chirp + ((int64_t)row0 << LOG2N1);
        const double* geo = a.geo + ((int64_t)row0 << LOG2N1);
        float2 v[16];
        uint32_t to = opaque(toff);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const float2 x = Elem<T>::load(at(src + TPV * e, to * (uint32_t)sizeof(T)));
            if constexpr (MODE == kRowFull) {
                v[e] = cmul(x, tw_row(TPV * e, to));
            } else if constexpr (MODE == kRowFwd) {
                v[e] = cmul(x, *at(tw4 + TPV * e, to * 8u));
            } else if constexpr (MODE == kRowInv) {
                v[e] = cmul(x, dm_chirp(a.dm, *at(geo + TPV * e, to * 8u)));
            } else {
                v[e] = x;  // kRowInvPlain: the filter was applied before (real input path); kRowChirp
            }
        }
        // kRowFull: the chirp is fetched again (from L2) during the forward
        // transform's last exchange rather than kept live across it.
        float2 ch[16];
        auto fetch_chirp = [&] {
            const uint32_t t2 = opaque(toff);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                if constexpr (MODE == kRowChirp) {
                    ch[e] = *at(chirp + TPV * e, t2 * 8u);
                } else if constexpr (OTF) {
                    ch[e] = *at(tab + TPV * e, t2 * 8u);
                } else {
                    const float4 t = *at(tab4 + TPV * e, t2 * 16u);
                    ch[e] = make_float2(t.z, t.w);
                }
            }
        };
        if constexpr (MODE == kRowFull || MODE == kRowChirp) {
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
                    Elem<T>::store(at(dst + TPV * e, to * (uint32_t)sizeof(T)), cscale(v[e], a.scale));
            }
            return;
        }
        if constexpr (MODE == kRowChirp) {
            fft_wg<LOG2N1, +1>(v, j, tb, lrow);
            asm volatile("" ::: "memory");
            to = opaque(toff);
            if (valid) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    Elem<T>::store(at(dst + TPV * e, to * (uint32_t)sizeof(T)), cscale(v[e], a.scale));
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
                    wo[e] = tw_row(TPV * e, t2);
                } else {
                    wo[e] = *at(tw4 + TPV * e, t2 * 8u);
                }
            }
        };
        fft_wg<LOG2N1, +1>(v, j, tb, lrow, nullptr, fetch_tw);
        asm volatile("" ::: "memory");
        to = opaque(toff);
        if (valid) {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                Elem<T>::store(at(dst + TPV * e, to * (uint32_t)sizeof(T)), cscale(cmulc(v[e], wo[e]), a.scale));
        }
    }
}

// Float16 table of the middle pass for the float16 arithmetic forms, 8
// bytes per (k2, k1): the four-step twiddle / 16 and the inverse ISM
// response times 2^-rem (rem: the part of the row normalisation not applied
// by the transform's stages), both evaluated in float64 as in
// k2_build_table.
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
    if (!chirp) return;
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

template <class T, int MODE, bool F16, bool MX, int LOG2N1>
static hipError_t k2_one(const K2Args& a, hipStream_t s) {
    using Sh = K2Shape<LOG2N1>;
    const int groups = ((1 << a.log2n2) + Sh::ROWS - 1) / Sh::ROWS * a.nblocks;
    const int grid = (groups + 7) & ~7;
    hipLaunchKernelGGL((k2_row<LOG2N1, T, MODE, F16, MX>), dim3(grid), dim3(Sh::THREADS), 0, s, a);
    return hipGetLastError();
}

template <class T, int MODE, bool F16, bool MX = false>
static hipError_t k2_dispatch(int log2n1, const K2Args& a, hipStream_t s) {
    switch (log2n1) {
        case 5: return k2_one<T, MODE, F16, MX, 5>(a, s);
        case 6: return k2_one<T, MODE, F16, MX, 6>(a, s);
        case 7: return k2_one<T, MODE, F16, MX, 7>(a, s);
        case 8: return k2_one<T, MODE, F16, MX, 8>(a, s);
        case 9: return k2_one<T, MODE, F16, MX, 9>(a, s);
        case 10: return k2_one<T, MODE, F16, MX, 10>(a, s);
        case 11: return k2_one<T, MODE, F16, MX, 11>(a, s);
        case 12: return k2_one<T, MODE, F16, MX, 12>(a, s);
        case 13: return k2_one<T, MODE, F16, MX, 13>(a, s);
        case 14: return k2_one<T, MODE, F16, MX, 14>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t k2_prec(int prec, int log2n1, const K2Args& a, hipStream_t s) {
    switch (prec) {
        case kFp32: return k2_dispatch<float2, MODE, false>(log2n1, a, s);
        case kHalf: return k2_dispatch<__half2, MODE, true>(log2n1, a, s);
        case kMixed: return k2_dispatch<__half2, MODE, true, true>(log2n1, a, s);
        case kBf16: return k2_dispatch<bf16x2, MODE, false>(log2n1, a, s);
        default: return k2_dispatch<__half2, MODE, false>(log2n1, a, s);
    }
}

hipError_t launch_k2(int prec, int mode, int log2n1, const K2Args& a, hipStream_t s) {
    switch (mode) {
        case kRowFull: return k2_prec<kRowFull>(prec, log2n1, a, s);
        case kRowFwd: return k2_prec<kRowFwd>(prec, log2n1, a, s);
        case kRowInv: return k2_prec<kRowInv>(prec, log2n1, a, s);
        case kRowChirp:
            // sub-rows of the split middle pass only
            if (log2n1 != kSplitLog2M1) return hipErrorInvalidValue;
            switch (prec) {
                case kFp32: return k2_one<float2, kRowChirp, false, false, kSplitLog2M1>(a, s);
                case kHalf: return k2_one<__half2, kRowChirp, true, false, kSplitLog2M1>(a, s);
                case kMixed: return k2_one<__half2, kRowChirp, true, true, kSplitLog2M1>(a, s);
                case kBf16: return k2_one<bf16x2, kRowChirp, false, false, kSplitLog2M1>(a, s);
                default: return k2_one<__half2, kRowChirp, false, false, kSplitLog2M1>(a, s);
            }
        case kRowInvPlain:
            // float32 arithmetic forms only (the real input path)
            if (prec == kFp32) return k2_dispatch<float2, kRowInvPlain, false>(log2n1, a, s);
            if (prec == kMixedValu) return k2_dispatch<__half2, kRowInvPlain, false>(log2n1, a, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

// Turns per unit DM of every bin, in the row layout (see the header).
__global__ void __launch_bounds__(256) build_dm_geometry(double* __restrict__ geo, int log2n1, int log2n2, double f0,
                                                         double df) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = 1ll << (log2n1 + log2n2);
    if (i >= n) return;
    const int64_t k2 = i >> log2n1;
    const int64_t k1 = i & ((1ll << log2n1) - 1);
    const int64_t k = k2 + (k1 << log2n2);
    const int64_t kk = k < (n >> 1) ? k : k - n;
    const double f = (double)kk * df;
    geo[i] = (f * f) / (2.41e-10 * f0 * f0 * (f0 + f));
}

hipError_t launch_build_dm_geometry(double* geo, int log2n1, int log2n2, double f0, double df, hipStream_t s) {
    const int64_t n = 1ll << (log2n1 + log2n2);
    hipLaunchKernelGGL(build_dm_geometry, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, geo, log2n1, log2n2, f0,
                       df);
    return hipGetLastError();
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

hipError_t launch_k2_build_table(void* tab, bool twiddle, int log2n1, int log2n2, double chirp_a, double f0,
                                 double df, double taper, hipStream_t s) {
    const int64_t n = 1ll << (log2n1 + log2n2);
    if (twiddle)
        hipLaunchKernelGGL(k2_build_table<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, log2n1,
                           log2n2, chirp_a, f0, df, taper);
    else
        hipLaunchKernelGGL(k2_build_table<false>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, log2n1,
                           log2n2, chirp_a, f0, df, taper);
    return hipGetLastError();
}

}  // namespace pond
