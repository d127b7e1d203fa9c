// Register-resident DFTs and a two-stage column FFT with a single LDS exchange.
//
// Length L = P * Q.  With input index j = j1 + P j2 and output index
// k = k1 + Q k2 (j1, k2 < P; j2, k1 < Q):
//   X[k1 + Q k2] = sum_j1 W_L^{j1 k1} W_P^{j1 k2} sum_j2 x[j1 + P j2] W_Q^{j2 k1}.
// Stage A: each work item (column, j1) loads the Q elements x[j1 + P j2],
// applies a size-Q DFT and the twiddles W_L^{j1 k1}, and writes them to LDS.
// Stage B: each work item (column, k1) reads the P values of its k1, applies a
// size-P DFT and owns the outputs X[k1 + Q k2].  Small DFTs recurse over the
// same factorisation with compile-time twiddles, so every array index is a
// constant and the data stay in registers.
#pragma once

#include "common.h"

namespace combo {

// ---- compile-time trigonometry (Taylor series after reduction to [-pi/4, pi/4]) ----
namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double sin_t(double x) {
    double t = x, s = x;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        s += t;
    }
    return s;
}
constexpr double cos_t(double x) {
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}
// cos and sin of 2 pi m / n for integers (exact octant reduction)
constexpr double cos2pi(long m, long n) {
    m %= n;
    if (m < 0) m += n;
    // angle = 2 pi m / n in [0, 2 pi); reduce with the octant of 8m/n
    const long oct = (8 * m + n / 2) / n;   // nearest multiple of pi/4 (0..8)
    const double r = 2.0 * kPi * (double)m / (double)n - (double)oct * (kPi / 4.0);
    const double c = cos_t(r), s = sin_t(r);
    const double h = 0.70710678118654752440084436210485;
    switch (oct % 8) {
        case 0: return c;
        case 1: return h * (c - s);
        case 2: return -s;
        case 3: return -h * (c + s);
        case 4: return -c;
        case 5: return -h * (c - s);
        case 6: return s;
        default: return h * (c + s);
    }
}
constexpr double sin2pi(long m, long n) { return cos2pi(4 * m - n, 4 * n); }   // sin x = cos(x - pi/2)
}  // namespace ct

template <int N, int DIR, typename C>
struct RegDFT;

template <int DIR, typename C>
struct RegDFT<1, DIR, C> {
    __device__ __forceinline__ static void run(C*) {}
};

template <int DIR, typename C>
struct RegDFT<2, DIR, C> {
    __device__ __forceinline__ static void run(C* x) {
        C t = x[0];
        x[0] = cadd(t, x[1]);
        x[1] = csub(t, x[1]);
    }
};

template <int DIR, typename C>
struct RegDFT<3, DIR, C> {
    __device__ __forceinline__ static void run(C* x) {
        using T = decltype(x[0].x);
        const T s1 = T(DIR) * T(0.86602540378443864676);
        C s = cadd(x[1], x[2]);
        C d = csub(x[1], x[2]);
        C x0 = cadd(x[0], s);
        C m;
        m.x = x[0].x - T(0.5) * s.x;
        m.y = x[0].y - T(0.5) * s.y;
        C t;
        t.x = -s1 * d.y;
        t.y = s1 * d.x;
        x[0] = x0;
        x[1] = cadd(m, t);
        x[2] = csub(m, t);
    }
};

template <int DIR, typename C>
struct RegDFT<4, DIR, C> {
    __device__ __forceinline__ static void run(C* x) {
        C t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]), t2 = cadd(x[1], x[3]), t3 = csub(x[1], x[3]);
        C it3 = cmul_i<DIR>(t3);
        x[0] = cadd(t0, t2);
        x[2] = csub(t0, t2);
        x[1] = cadd(t1, it3);
        x[3] = csub(t1, it3);
    }
};

constexpr int first_factor(int n) { return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : 3; }

// multiply by W_N^m = exp(DIR 2 pi i m / N) with compile-time constants
template <int N, int M, int DIR, typename C>
__device__ __forceinline__ C twc(C v) {
    using T = decltype(v.x);
    constexpr int m = M % N;
    if constexpr (m == 0) {
        return v;
    } else if constexpr (4 * m == N) {
        return cmul_i<DIR>(v);
    } else if constexpr (2 * m == N) {
        C r;
        r.x = -v.x;
        r.y = -v.y;
        return r;
    } else if constexpr (4 * m == 3 * N) {
        return cmul_i<-DIR>(v);
    } else {
        constexpr double c = ct::cos2pi(m, N);
        constexpr double s = DIR * ct::sin2pi(m, N);
        C w;
        w.x = T(c);
        w.y = T(s);
        return cmul(v, w);
    }
}

template <int N, int DIR, typename C, int J1 = 0>
__device__ __forceinline__ void reg_dft_inner(C (&y)[first_factor(N)][N / first_factor(N)], C* x) {
    constexpr int P = first_factor(N), Q = N / P;
    if constexpr (J1 < P) {
#pragma unroll
        for (int j2 = 0; j2 < Q; ++j2) y[J1][j2] = x[J1 + P * j2];
        RegDFT<Q, DIR, C>::run(y[J1]);
        reg_dft_inner<N, DIR, C, J1 + 1>(y, x);
    }
}

template <int N, int DIR, typename C, int J1, int K1>
__device__ __forceinline__ void reg_twiddle(C (&y)[first_factor(N)][N / first_factor(N)]) {
    constexpr int P = first_factor(N), Q = N / P;
    if constexpr (J1 < P) {
        if constexpr (K1 < Q) {
            y[J1][K1] = twc<N, J1 * K1, DIR>(y[J1][K1]);
            reg_twiddle<N, DIR, C, J1, K1 + 1>(y);
        } else {
            reg_twiddle<N, DIR, C, J1 + 1, 0>(y);
        }
    }
}

template <int N, int DIR, typename C>
struct RegDFT {
    __device__ __forceinline__ static void run(C* x) {
        constexpr int P = first_factor(N), Q = N / P;
        C y[P][Q];
        reg_dft_inner<N, DIR, C>(y, x);
        reg_twiddle<N, DIR, C, 1, 1>(y);
#pragma unroll
        for (int k1 = 0; k1 < Q; ++k1) {
            C z[P];
#pragma unroll
            for (int j1 = 0; j1 < P; ++j1) z[j1] = y[j1][k1];
            RegDFT<P, DIR, C>::run(z);
#pragma unroll
            for (int k2 = 0; k2 < P; ++k2) x[k1 + Q * k2] = z[k2];
        }
    }
};

// ---- two-stage column FFT ------------------------------------------------------
// TX columns of length L = P*Q.  Stage A work items (t, j1) = (it % TX, it / TX),
// it < TX*P; stage B work items (t, k1), it < TX*Q.  LDS exchange layout:
// ex[(j1*Q + k1)*TXP + t] (TXP = TX padded by one to spread banks).
template <int P, int Q, int TX>
struct Fft2 {
    static constexpr int L = P * Q;
    static constexpr int TXP = TX + ((TX % 2 == 0) ? 1 : 0);
    static constexpr int NA = TX * P;       // stage A items
    static constexpr int NB = TX * Q;       // stage B items
    static constexpr int exch_elems() { return P * Q * TXP; }
};

// Stage A for one item: x[j2] holds the loaded inputs x[j1 + P j2]; transforms,
// twiddles with W_L^{j1 k1} from the table tw (forward table of length L) and
// writes the exchange buffer.
template <int P, int Q, int TX, int DIR, typename T>
__device__ __forceinline__ void fft2_stageA(cpx<T>* x, int t, int j1, cpx<T>* ex, const cpx<T>* tw) {
    using C = cpx<T>;
    constexpr int L = P * Q;
    constexpr int TXP = Fft2<P, Q, TX>::TXP;
    RegDFT<Q, DIR, C>::run(x);
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) {
        C v = x[k1];
        if (P > 1 && k1 > 0) {
            C w = tw[j1 * k1];   // j1 k1 < L
            if (DIR > 0) w.y = -w.y;
            v = cmul(v, w);
        }
        ex[(j1 * Q + k1) * TXP + t] = v;
    }
}

// Stage B for one item: reads the P values of column t, index k1, transforms;
// y[k2] = X[k1 + Q k2].
template <int P, int Q, int TX, int DIR, typename T>
__device__ __forceinline__ void fft2_stageB(cpx<T>* y, int t, int k1, const cpx<T>* ex) {
    constexpr int TXP = Fft2<P, Q, TX>::TXP;
#pragma unroll
    for (int j1 = 0; j1 < P; ++j1) y[j1] = ex[(j1 * Q + k1) * TXP + t];
    RegDFT<P, DIR, cpx<T>>::run(y);
}

}  // namespace combo
