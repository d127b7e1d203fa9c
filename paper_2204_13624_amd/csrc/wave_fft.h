// Row FFTs held by a group of W lanes (W a power of two <= 64, m = L/W values per
// lane), with no LDS and no barriers.
//
// Layout "natural": lane l, slot r holds index l + W r.
// Layout "scrambled": lane l, slot s holds index s + m bitrev_W(l).
//
// Natural -> scrambled (used for the inverse transform): with j = l + W r and
// k = s + m t,  X[s + m t] = sum_l w_W^{l t} [ w_L^{l s} sum_r x[l + W r] w_m^{r s} ]:
// an m-point DFT over the slots of each lane, the twiddles w_L^{l s}, then a
// W-point decimation-in-frequency FFT across lanes (xor shuffles), whose output
// is bit-reversed over the lanes.
// Scrambled -> natural (forward transform): the mirror image, a W-point
// decimation-in-time FFT across lanes on bit-reversed input, the twiddles
// w_L^{s l}, then the m-point DFT over the slots: X[l + W r].
#pragma once

#include "common.h"
#include "fft_reg.h"

namespace combo {

template <int W>
__device__ __forceinline__ int bitrev_lane(int l) {
    if constexpr (W == 1) {
        return 0;
    } else {
        constexpr int bits = (W == 2) ? 1 : (W == 4) ? 2 : (W == 8) ? 3 : (W == 16) ? 4 : (W == 32) ? 5 : 6;
        return (int)(__brev((unsigned)l) >> (32 - bits));
    }
}

template <typename T>
__device__ __forceinline__ cpx<T> shfl_xor_c(cpx<T> v, int mask) {
    cpx<T> r;
    r.x = __shfl_xor(v.x, mask, 64);
    r.y = __shfl_xor(v.y, mask, 64);
    return r;
}

// read v from lane `src` of the same group of W lanes
template <int W, typename T>
__device__ __forceinline__ cpx<T> shfl_c(cpx<T> v, int src) {
    cpx<T> r;
    r.x = __shfl(v.x, src, W);
    r.y = __shfl(v.y, src, W);
    return r;
}

// Per-lane twiddles: step[s] = w_L^{l s} (s < m) and stage[b] = w_{2h}^{l mod h}
// for h = 2^b (b < log2 W), all as forward values exp(-2 pi i ./L).
template <typename T, int M, int W>
struct WaveTwiddles {
    static constexpr int L = M * W;
    static constexpr int NB = (W == 1) ? 0 : (W == 2) ? 1 : (W == 4) ? 2 : (W == 8) ? 3 : (W == 16) ? 4 : (W == 32) ? 5 : 6;
    cpx<T> step[M];
    cpx<T> stage[NB > 0 ? NB : 1];
    __device__ __forceinline__ void load(const cpx<T>* tw, int l) {
#pragma unroll
        for (int s = 0; s < M; ++s) step[s] = tw[(l * s) % L];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int h = 1 << b;
            stage[b] = tw[(l % h) * (L / (2 * h))];
        }
    }
};

template <int DIR, typename T>
__device__ __forceinline__ cpx<T> twmul(cpx<T> v, cpx<T> w) {
    if (DIR > 0) w.y = -w.y;
    return cmul(v, w);
}

// natural -> scrambled, direction DIR, on x[M] of one lane
template <int DIR, int M, int W, typename T>
__device__ __forceinline__ void wave_fft_nat2scr(cpx<T>* x, int l, const WaveTwiddles<T, M, W>& tw) {
    RegDFT<M, DIR, cpx<T>>::run(x);
#pragma unroll
    for (int s = 1; s < M; ++s) x[s] = twmul<DIR, T>(x[s], tw.step[s]);
#pragma unroll
    for (int b = WaveTwiddles<T, M, W>::NB - 1; b >= 0; --b) {
        const int h = 1 << b;
        const bool upper = (l & h) != 0;
#pragma unroll
        for (int s = 0; s < M; ++s) {
            const cpx<T> o = shfl_xor_c<T>(x[s], h);
            x[s] = upper ? twmul<DIR, T>(csub(o, x[s]), tw.stage[b]) : cadd(x[s], o);
        }
    }
}

// scrambled -> natural, direction DIR
template <int DIR, int M, int W, typename T>
__device__ __forceinline__ void wave_fft_scr2nat(cpx<T>* x, int l, const WaveTwiddles<T, M, W>& tw) {
#pragma unroll
    for (int b = 0; b < WaveTwiddles<T, M, W>::NB; ++b) {
        const int h = 1 << b;
        const bool upper = (l & h) != 0;
#pragma unroll
        for (int s = 0; s < M; ++s) {
            const cpx<T> o = shfl_xor_c<T>(x[s], h);
            x[s] = upper ? csub(o, twmul<DIR, T>(x[s], tw.stage[b])) : cadd(x[s], twmul<DIR, T>(o, tw.stage[b]));
        }
    }
#pragma unroll
    for (int s = 1; s < M; ++s) x[s] = twmul<DIR, T>(x[s], tw.step[s]);
    RegDFT<M, DIR, cpx<T>>::run(x);
}

}  // namespace combo
