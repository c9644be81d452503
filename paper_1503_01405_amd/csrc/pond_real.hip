// The real two-channel input path (channels added in phase, packed
// real-to-complex transforms).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "pond_device.hpp"

namespace pond {

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

}  // namespace pond
