// Batched complex FFTs on data staged in LDS (Stockham autosort, mixed radix
// 2/3/4/8/16), executed cooperatively by one 256-thread workgroup.
//
// Layout in LDS: COLMAJOR = false: element (index l along the transform,
// column t) at buf[l*TX + t] (columns interleaved, as tiles of a strided axis
// arrive from global memory); COLMAJOR = true: at buf[t*L + l] (each column
// contiguous, as rows of the unit-stride axis arrive).  Consecutive threads
// take consecutive columns (row-major) or consecutive butterflies of one column
// (column-major), so LDS accesses stay unit-stride in both cases.  TX columns
// are transformed at once.  A pass of radix R with Ns = product of
// the earlier radices reads x[j + r L/R] (r < R) for butterfly j, multiplies by
// W_{Ns R}^{r (j mod Ns)}, applies the size-R DFT and writes to
// (j div Ns) Ns R + (j mod Ns) + r Ns, so the result lands in natural order.
// Each pass stages its inputs in registers, synchronises, then writes back in
// place.  DIR = -1: forward exp(-2 pi i jk/L); DIR = +1: inverse (unnormalised).
#pragma once

#include "common.h"

namespace combo {

template <int DIR, typename C>
__device__ __forceinline__ void dft2(C& a, C& b) {
    C t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int DIR, typename C>
__device__ __forceinline__ void dft3(C& a, C& b, C& c) {
    using T = decltype(a.x);
    const T s1 = T(DIR) * T(0.86602540378443864676);   // DIR sin(2 pi / 3)
    C s = cadd(b, c);
    C d = csub(b, c);
    C x0 = cadd(a, s);
    C m;
    m.x = a.x - T(0.5) * s.x;
    m.y = a.y - T(0.5) * s.y;
    C t;
    t.x = -s1 * d.y;
    t.y = s1 * d.x;
    a = x0;
    b = cadd(m, t);
    c = csub(m, t);
}

template <int DIR, typename C>
__device__ __forceinline__ void dft4(C& a, C& b, C& c, C& d) {
    C t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
    C it3 = cmul_i<DIR>(t3);
    a = cadd(t0, t2);
    c = csub(t0, t2);
    b = cadd(t1, it3);
    d = csub(t1, it3);
}

// multiply by W_8^m = exp(DIR 2 pi i m / 8), m = 1..3
template <int DIR, int M, typename C>
__device__ __forceinline__ C w8(C x) {
    using T = decltype(x.x);
    const T h = T(0.70710678118654752440);
    if (M == 0) return x;
    if (M == 2) return cmul_i<DIR>(x);
    C r;
    if (M == 1) {  // (1 + DIR i) h
        r.x = h * (x.x - T(DIR) * x.y);
        r.y = h * (x.y + T(DIR) * x.x);
    } else {       // (-1 + DIR i) h
        r.x = h * (-x.x - T(DIR) * x.y);
        r.y = h * (-x.y + T(DIR) * x.x);
    }
    return r;
}

// size-8 DFT as 2 x 4: inner size-4 DFTs over x[j1 + 2 j2], twiddle W_8^{j1 k1},
// outer size-2 DFTs; X[k1 + 4 k2].
template <int DIR, typename C>
__device__ __forceinline__ void dft8(C* x) {
    C y0[4] = {x[0], x[2], x[4], x[6]};
    C y1[4] = {x[1], x[3], x[5], x[7]};
    dft4<DIR>(y0[0], y0[1], y0[2], y0[3]);
    dft4<DIR>(y1[0], y1[1], y1[2], y1[3]);
    y1[1] = w8<DIR, 1>(y1[1]);
    y1[2] = w8<DIR, 2>(y1[2]);
    y1[3] = w8<DIR, 3>(y1[3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C a = y0[k1], b = y1[k1];
        dft2<DIR>(a, b);
        x[k1] = a;
        x[k1 + 4] = b;
    }
}

// multiply by W_16^m = exp(DIR 2 pi i m / 16)
template <int DIR, typename C>
__device__ __forceinline__ C w16(C x, int m) {
    using T = decltype(x.x);
    const T cs[10] = {T(1.0), T(0.92387953251128675613), T(0.70710678118654752440), T(0.38268343236508977173),
                      T(0.0), T(-0.38268343236508977173), T(-0.70710678118654752440), T(-0.92387953251128675613),
                      T(-1.0), T(-0.92387953251128675613)};
    const T sn[10] = {T(0.0), T(0.38268343236508977173), T(0.70710678118654752440), T(0.92387953251128675613),
                      T(1.0), T(0.92387953251128675613), T(0.70710678118654752440), T(0.38268343236508977173),
                      T(0.0), T(-0.38268343236508977173)};
    C w;
    w.x = cs[m];
    w.y = T(DIR) * sn[m];
    return cmul(x, w);
}

// size-16 DFT as 4 x 4: inner size-4 DFTs over x[j1 + 4 j2], twiddle W_16^{j1 k1},
// outer size-4 DFTs over j1; X[k1 + 4 k2].
template <int DIR, typename C>
__device__ __forceinline__ void dft16(C* x) {
    C y[4][4];
#pragma unroll
    for (int j1 = 0; j1 < 4; ++j1) {
        y[j1][0] = x[j1];
        y[j1][1] = x[j1 + 4];
        y[j1][2] = x[j1 + 8];
        y[j1][3] = x[j1 + 12];
        dft4<DIR>(y[j1][0], y[j1][1], y[j1][2], y[j1][3]);
    }
#pragma unroll
    for (int j1 = 1; j1 < 4; ++j1)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) y[j1][k1] = w16<DIR>(y[j1][k1], j1 * k1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C a = y[0][k1], b = y[1][k1], c = y[2][k1], d = y[3][k1];
        dft4<DIR>(a, b, c, d);
        x[k1] = a;
        x[k1 + 4] = b;
        x[k1 + 8] = c;
        x[k1 + 12] = d;
    }
}

template <int R, int DIR, typename C>
__device__ __forceinline__ void dftR(C* v) {
    if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
    else if constexpr (R == 3) dft3<DIR>(v[0], v[1], v[2]);
    else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<DIR>(v);
    else dft16<DIR>(v);
}

// CAP: most elements (L TX) a call may hold; it sets the butterflies each thread keeps in flight.
template <int R, int DIR, bool COLMAJOR, typename T, int CAP>
__device__ __forceinline__ void stockham_pass(cpx<T>* buf, int L, int TX, int Ns, const cpx<T>* tw) {
    constexpr int NB = (CAP / R + kBlock - 1) / kBlock;
    const int tid = threadIdx.x;
    const int LR = L / R;
    const int nbf = LR * TX;
    const int tws = L / (Ns * R);
    cpx<T> v[NB][R];
    int jj[NB], tt[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int b = tid + q * kBlock;
        jj[q] = 0;
        tt[q] = 0;
        if (b < nbf) {
            int t, j;
            if (COLMAJOR) { t = b / LR; j = b - t * LR; }
            else { j = b / TX; t = b - j * TX; }
            const int k = j % Ns;
            jj[q] = j;
            tt[q] = t;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int l = j + r * LR;
                cpx<T> x = COLMAJOR ? buf[t * L + l] : buf[l * TX + t];
                if (r > 0 && k > 0) {
                    cpx<T> w = tw[r * k * tws];
                    if (DIR > 0) w.y = -w.y;
                    x = cmul(x, w);
                }
                v[q][r] = x;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int b = tid + q * kBlock;
        if (b < nbf) {
            dftR<R, DIR>(v[q]);
            const int j = jj[q];
            const int k = j % Ns;
            const int base = (j / Ns) * Ns * R + k;
            const int t = tt[q];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int l = base + r * Ns;
                if (COLMAJOR) buf[t * L + l] = v[q][r];
                else buf[l * TX + t] = v[q][r];
            }
        }
    }
    __syncthreads();
}

// Transform TX columns of length plan.L held in buf; tw = forward twiddles of plan.L.
// plan.L * TX must not exceed CAP (callers size their tiles for it).
template <int DIR, bool COLMAJOR, typename T, int CAP = max_elems<T>()>
__device__ __forceinline__ void fft_lds(cpx<T>* buf, const AxisPlan& plan, int TX, const cpx<T>* tw) {
    int Ns = 1;
    for (int p = 0; p < plan.npass; ++p) {
        const int R = plan.radix[p];
        switch (R) {
            case 2: stockham_pass<2, DIR, COLMAJOR, T, CAP>(buf, plan.L, TX, Ns, tw); break;
            case 3: stockham_pass<3, DIR, COLMAJOR, T, CAP>(buf, plan.L, TX, Ns, tw); break;
            case 4: stockham_pass<4, DIR, COLMAJOR, T, CAP>(buf, plan.L, TX, Ns, tw); break;
            case 8: stockham_pass<8, DIR, COLMAJOR, T, CAP>(buf, plan.L, TX, Ns, tw); break;
            default: stockham_pass<16, DIR, COLMAJOR, T, CAP>(buf, plan.L, TX, Ns, tw); break;
        }
        Ns *= R;
    }
}

// Copy the forward twiddle table of length L from global memory into LDS.
template <typename T>
__device__ __forceinline__ void load_twiddles(cpx<T>* sh_tw, const cpx<T>* g_tw, int L) {
    for (int i = threadIdx.x; i < L; i += blockDim.x) sh_tw[i] = g_tw[i];
}

}  // namespace combo
