// FFT passes of the Lippmann-Schwinger operator on gfx950.
//
// A compatible field F = Fbar + Grad u is represented by the displacement
// coefficients u_hat (3 complex numbers per frequency): FFT(F - Fbar) = u_hat (x) xi
// (unnormalised FFT, xi_d = 2 pi k_d / l_d).  The Green operator of the paper
// (Sec. 3, eq. Gamma0) is then  Gamma0_hat tau_hat = (K^{-1} tau_hat xi) (x) xi  with the
// acoustic tensor K = mu0 |xi|^2 I + kappa0 xi (x) xi of the reference medium, so
// only the three components of tau_hat xi are ever needed.  The three grid axes
// are transformed in separate passes and the xi_J factors are applied axis by
// axis, which shrinks the spectral data between passes:
//
//   forward  x: 9 real comps -> R2C, comps (i,1) times xi_1           9 complex
//            y: FFT, a_i = (xi_1 tau_i1)^ + xi_2 tau_i2^               9 -> 6
//            z: FFT, v_i = a_i + xi_3 tau_i3^, then K^{-1} v          6 -> 3
//   inverse  z: u_i and xi_3 u_i, IFFT                                3 -> 6
//            y: IFFT of u_i, xi_2 u_i, xi_3 u_i                       6 -> 9
//            x: comps (i,1) times xi_1, C2R                           9 real comps
//
// In the CG operator the x inverse pass, the tangent action and the x forward
// pass are one kernel, so the real-space field never reaches HBM.  Frequencies
// on a Nyquist plane of an even axis and the zero frequency are projected out;
// the x Nyquist bin is not stored at all (half spectrum of n1/2 values).
//
// Real transforms along x pack two real components into one complex FFT:
// z = a + i b, A_k = (Z_k + conj Z_{n-k})/2, B_k = (Z_k - conj Z_{n-k})/(2i).
#include <algorithm>

#include <type_traits>

#include "fft_lds.h"
#include "fft_reg.h"
#include "kernels.h"
#include "wave_fft.h"

// The build compiles this file once per part (COMBO_PART = 1..6, in parallel);
// kernel templates are instantiated only by the launchers of their part.
// Without COMBO_PART everything is compiled in one unit.
#ifndef COMBO_PART
#define COMBO_PART 0
#endif
#define COMBO_IN_PART(k) (COMBO_PART == 0 || COMBO_PART == (k))
#define COMBO_PART_XF 1   // x pass, float
#define COMBO_PART_XD 2   // x pass, double
#define COMBO_PART_Y 3    // y passes
#define COMBO_PART_ZF 4   // z passes, float
#define COMBO_PART_ZD 5   // z passes with double transforms
#define COMBO_PART_CG 6   // CG vector kernels, finalisers, host helpers

namespace combo {

// ------------------------------------------------------------------------------
// block reduction of one double per thread; result valid in thread 0
// ------------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) r += sh[w];
    }
    return r;
}

// ------------------------------------------------------------------------------
// tangent action tau = A : p
// ------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void tangent_apply(const TangentState<T>& ts, long long sidx, const T* p, T* tau) {
    const int slot = ts.slot[sidx];
    if (slot >= 0) {
        const T* A = ts.Acomp + (long long)slot * 45;
        T a[45];
#pragma unroll
        for (int i = 0; i < 45; ++i) a[i] = A[i];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            T acc = T(0);
#pragma unroll
            for (int s = 0; s < 9; ++s) {
                const int lo = r < s ? r : s, hi = r < s ? s : r;
                acc += a[lo * 9 - (lo * (lo - 1)) / 2 + (hi - lo)] * p[s];
            }
            tau[r] = acc;
        }
        return;
    }
    const int ph = (slot == -1) ? 0 : 1;
    const T mu = ts.mu[ph], lam = ts.lam[ph];
    T fi[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) fi[c] = ts.Sinv[c * ts.n + sidx];
    const T m = ts.sm[sidx];
    // B = F^{-1} p, C = B F^{-1};  tau_iJ = mu p_iJ + lam tr(B) Finv_Ji + m C_Ji
    T B[9];
#pragma unroll
    for (int J = 0; J < 3; ++J)
#pragma unroll
        for (int L = 0; L < 3; ++L) B[3 * J + L] = fi[3 * J + 0] * p[0 + L] + fi[3 * J + 1] * p[3 + L] + fi[3 * J + 2] * p[6 + L];
    const T tr = B[0] + B[4] + B[8];
    T C[9];
#pragma unroll
    for (int J = 0; J < 3; ++J)
#pragma unroll
        for (int i = 0; i < 3; ++i) C[3 * J + i] = B[3 * J + 0] * fi[0 + i] + B[3 * J + 1] * fi[3 + i] + B[3 * J + 2] * fi[6 + i];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int J = 0; J < 3; ++J) tau[3 * i + J] = mu * p[3 * i + J] + lam * tr * fi[3 * J + i] + m * C[3 * J + i];
}

// the same with the pure-voxel state (slot, F^{-1}, mu - lambda ln J) already loaded
template <typename T>
__device__ __forceinline__ void tangent_apply_loaded(const TangentState<T>& ts, int slot, const T* fi, T m,
                                                     const T* p, T* tau) {
    if (slot >= 0) {
        const T* A = ts.Acomp + (long long)slot * 45;
        T a[45];
#pragma unroll
        for (int i = 0; i < 45; ++i) a[i] = A[i];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            T acc = T(0);
#pragma unroll
            for (int s = 0; s < 9; ++s) {
                const int lo = r < s ? r : s, hi = r < s ? s : r;
                acc += a[lo * 9 - (lo * (lo - 1)) / 2 + (hi - lo)] * p[s];
            }
            tau[r] = acc;
        }
        return;
    }
    const int ph = (slot == -1) ? 0 : 1;
    const T mu = ts.mu[ph], lam = ts.lam[ph];
    T B[9];
#pragma unroll
    for (int J = 0; J < 3; ++J)
#pragma unroll
        for (int L = 0; L < 3; ++L) B[3 * J + L] = fi[3 * J + 0] * p[0 + L] + fi[3 * J + 1] * p[3 + L] + fi[3 * J + 2] * p[6 + L];
    const T tr = B[0] + B[4] + B[8];
    T C[9];
#pragma unroll
    for (int J = 0; J < 3; ++J)
#pragma unroll
        for (int i = 0; i < 3; ++i) C[3 * J + i] = B[3 * J + 0] * fi[0 + i] + B[3 * J + 1] * fi[3 + i] + B[3 * J + 2] * fi[6 + i];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int J = 0; J < 3; ++J) tau[3 * i + J] = mu * p[3 * i + J] + lam * tr * fi[3 * J + i] + m * C[3 * J + i];
}

// ------------------------------------------------------------------------------
// x pass
// ------------------------------------------------------------------------------
// Sequences s = 0..4 pack components (2s, 2s+1), the last one component 8 alone.
__device__ __forceinline__ bool xi1_comp(int c) { return c == 0 || c == 3 || c == 6; }

template <typename T, int MODE>
__device__ __forceinline__ void k_xpass_body(const XArgs<T>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    if (MODE == X_CG && a.st->done) return;
    if (MODE != X_CG && a.skip_done && a.st->done) return;
    extern __shared__ char smem_raw[];
    const int L = a.g.n1, nh = a.g.nh, nk = a.g.nkx, R = a.R;   // row stride, stored bins
    C* tw = reinterpret_cast<C*>(smem_raw);
    C* buf = tw + L;                   // [5R][L], column-major (each sequence contiguous)
    __shared__ double red[16];
    const long long nrows = (long long)a.g.n2 * a.g.n3;
    const long long row0 = (long long)tile_ * R;
    const int tid = threadIdx.x;
    const T xs1 = T(a.g.xs1);
    load_twiddles<T>(tw, a.tw, L);

    constexpr bool HAS_INV = (MODE == X_CG || MODE == X_AVG || MODE == X_INV_REAL);
    constexpr bool HAS_FWD = (MODE == X_CG || MODE == X_RHS_E || MODE == X_FWD_REAL);

    if (HAS_INV) {
        // unpack half spectra into full-length sequences
        const int items = 5 * R * nk;
        for (int it = tid; it < items; it += kBlock) {
            const int k = it % nk;
            const int sr = it / nk;
            const int rr = sr % R, s = sr / R;
            const long long row = row0 + rr;
            C ha = mk<T>(0, 0), hb = mk<T>(0, 0);
            if (row < nrows) {
                const long long off = row * nh + k;
                const int ca = 2 * s, cb = 2 * s + 1;
                ha = a.in[ca * a.g.nspec + off];
                if (s < 4) hb = a.in[cb * a.g.nspec + off];
                if (a.g.disc == 2) {
                    const C f1 = fst1<T>(a.g, k);
                    if (xi1_comp(ca)) ha = cmul(ha, f1);
                    if (s < 4 && xi1_comp(cb)) hb = cmul(hb, f1);
                } else if (a.g.disc) {
                    const T d1 = T(fac_d1(a.g, k)), a1 = T(fac_a1(a.g, k));
                    ha = cscale(ha, xi1_comp(ca) ? d1 : a1);
                    if (s < 4) hb = cscale(hb, xi1_comp(cb) ? d1 : a1);
                } else {
                    const T x1 = xs1 * T(k);
                    if (xi1_comp(ca)) ha = cscale(ha, x1);
                    if (s < 4 && xi1_comp(cb)) hb = cscale(hb, x1);
                }
            }
            C* col = buf + (s * R + rr) * L;
            if (k == 0 || 2 * k == L) {   // self-conjugate bins (x Nyquist only where it is stored)
                col[k] = mk<T>(ha.x, hb.x);
            } else {
                col[k] = mk<T>(ha.x - hb.y, ha.y + hb.x);
                col[L - k] = mk<T>(ha.x + hb.y, hb.x - ha.y);
            }
            if (2 * nk == L && k == nk - 1 && L > 1) col[L / 2] = mk<T>(0, 0);
        }
        __syncthreads();
        fft_lds<+1, true, T, xpass_cap<T>()>(buf, a.plan, 5 * R, tw);
    }

    // pointwise stage
    double acc[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] = 0.0;
    {
        const int items = R * L;
        for (int it = tid; it < items; it += kBlock) {
            const int x = it % L, rr = it / L;
            const long long row = row0 + rr;
            if (row >= nrows) {
                if (HAS_FWD) {
#pragma unroll
                    for (int s = 0; s < 5; ++s) buf[(s * R + rr) * L + x] = mk<T>(0, 0);
                }
                continue;
            }
            const long long vox = row * L + x;
            T p[9];
            if (MODE == X_RHS_E) {
#pragma unroll
                for (int c = 0; c < 9; ++c) p[c] = T(a.E[c]);
            } else if (MODE == X_FWD_REAL) {
                if (a.real_in_t) {
#pragma unroll
                    for (int c = 0; c < 9; ++c) p[c] = a.real_in_t[c * a.g.n + vox];
                } else {
#pragma unroll
                    for (int c = 0; c < 9; ++c) p[c] = T(a.real_in[c * a.g.n + vox]);
                }
            } else {
#pragma unroll
                for (int s = 0; s < 5; ++s) {
                    const C z = buf[(s * R + rr) * L + x];
                    p[2 * s] = z.x;
                    if (s < 4) p[2 * s + 1] = z.y;
                }
            }
            if (MODE == X_INV_REAL) {
                if (a.real_out_t) {
#pragma unroll
                    for (int c = 0; c < 9; ++c) a.real_out_t[c * a.g.n + vox] = T(double(p[c]) * a.scale);
                } else {
#pragma unroll
                    for (int c = 0; c < 9; ++c) a.real_out[c * a.g.n + vox] = double(p[c]) * a.scale;
                }
                continue;
            }
            if (MODE == X_AVG) {
#pragma unroll
                for (int c = 0; c < 9; ++c) p[c] = T(double(p[c]) * a.scale + a.E[c]);
            }
            T tau[9];
            if (MODE == X_FWD_REAL) {
#pragma unroll
                for (int c = 0; c < 9; ++c) tau[c] = p[c];
            } else {
                tangent_apply<T>(a.ts, state_pos(vox, a.g.n1, a.g.xm, a.g.xwbits), p, tau);
            }
            if (MODE == X_AVG) {
#pragma unroll
                for (int c = 0; c < 9; ++c) acc[c] += double(tau[c]);
                continue;
            }
#pragma unroll
            for (int s = 0; s < 5; ++s) buf[(s * R + rr) * L + x] = mk<T>(tau[2 * s], s < 4 ? tau[2 * s + 1] : T(0));
        }
    }
    if (MODE == X_AVG) {
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const double t = block_sum(acc[c], red);
            if (tid == 0) a.partials[(long long)tile_ * 9 + c] = t;
        }
        return;
    }
    if (!HAS_FWD) return;
    __syncthreads();
    fft_lds<-1, true, T, xpass_cap<T>()>(buf, a.plan, 5 * R, tw);
    // pack: half spectra of both real components of every sequence
    const int items = 5 * R * nh;
    for (int it = tid; it < items; it += kBlock) {
        const int k = it % nh;
        const int sr = it / nh;
        const int rr = sr % R, s = sr / R;
        const long long row = row0 + rr;
        if (row >= nrows) continue;
        const C* col = buf + (s * R + rr) * L;
        const C zk = col[k];
        const C zm = col[(L - k) % L];
        C ha = mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));
        C hb = mk<T>(T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x));
        const long long off = row * nh + k;
        const int ca = 2 * s, cb = 2 * s + 1;
        if (k >= nk) {   // row padding: zero modes
            ha = hb = mk<T>(0, 0);
        } else if (a.g.disc == 2) {
            const C f1c = cconj(fst1<T>(a.g, k));
            if (xi1_comp(ca)) ha = cmul(ha, f1c);
            if (xi1_comp(cb)) hb = cmul(hb, f1c);
        } else if (a.g.disc) {
            const T d1 = T(fac_d1(a.g, k)), a1 = T(fac_a1(a.g, k));
            ha = cscale(ha, xi1_comp(ca) ? d1 : a1);
            hb = cscale(hb, xi1_comp(cb) ? d1 : a1);
        } else {
            const T x1 = xs1 * T(k);
            if (xi1_comp(ca)) ha = cscale(ha, x1);
            if (xi1_comp(cb)) hb = cscale(hb, x1);
        }
        a.out[ca * a.g.nspec + off] = ha;
        if (s < 4) a.out[cb * a.g.nspec + off] = hb;
    }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_xpass(XArgs<T> a) {
    k_xpass_body<T, MODE>(a, blockIdx.x, gridDim.x);
}

template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_xpass_b(const XArgs<T>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_xpass_body<T, MODE>(as[e.rve], e.tile, e.ntiles);
}

// ------------------------------------------------------------------------------
// x pass, wavefront version: one grid row (y, z) per group of W lanes, m = n1/W
// values per lane and sequence, all five packed sequences in registers, no LDS
// and no barriers (wave_fft.h).  The inverse transform leaves voxel
// x = s + m bitrev(l) in lane l, slot s, which is where the tangent is applied;
// the forward transform returns to the natural layout for the store.
// ------------------------------------------------------------------------------
template <typename T, int MODE, int M, int W>
__device__ __forceinline__ void k_xwave_body(const XArgs<T>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    constexpr int L = M * W;
    constexpr int G = 256 / W;   // rows per workgroup
    if (MODE == X_CG && a.st->done) return;
    __shared__ double red[16];
    const int lane = threadIdx.x % W;
    const long long nrows = (long long)a.g.n2 * a.g.n3;
    const long long row = (long long)tile_ * G + threadIdx.x / W;
    const bool live = row < nrows;
    const int nh = a.g.nh;
    const T xs1 = T(a.g.xs1);
    WaveTwiddles<T, M, W> tw;
    tw.load(a.tw, lane);
    constexpr bool HAS_INV = (MODE == X_CG || MODE == X_AVG || MODE == X_INV_REAL);
    constexpr bool HAS_FWD = (MODE == X_CG || MODE == X_RHS_E || MODE == X_FWD_REAL);
    C z[5][M];
    const int xbase = M * bitrev_lane<W>(lane);   // voxel of slot s is xbase + s

    if (HAS_INV) {
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            const int ca = 2 * s, cb = 2 * s + 1;
#pragma unroll
            for (int r = 0; r < M; ++r) {
                const int k = lane + W * r;
                C ha = mk<T>(0, 0), hb = mk<T>(0, 0);
                bool conj = false;
                int kk = k;
                if (k >= nh) {
                    kk = L - k;
                    conj = true;
                }
                const bool valid = live && !(k >= nh && kk >= nh);   // kk = nh only at the even-n1 Nyquist bin
                if (valid) {
                    const long long off = row * nh + kk;
                    ha = a.in[ca * a.g.nspec + off];
                    if (s < 4) hb = a.in[cb * a.g.nspec + off];
                    const T x1 = xs1 * T(kk);
                    if (xi1_comp(ca)) ha = cscale(ha, x1);
                    if (s < 4 && xi1_comp(cb)) hb = cscale(hb, x1);
                }
                if (k == 0) {
                    z[s][r] = mk<T>(ha.x, hb.x);
                } else if (!conj) {
                    z[s][r] = mk<T>(ha.x - hb.y, ha.y + hb.x);
                } else {
                    z[s][r] = mk<T>(ha.x + hb.y, hb.x - ha.y);
                }
            }
            wave_fft_nat2scr<+1, M, W, T>(z[s], lane, tw);
        }
    }

    double acc[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] = 0.0;
#pragma unroll
    for (int sl = 0; sl < M; ++sl) {
        const long long vox = row * L + xbase + sl;
        T p[9];
        if (MODE == X_RHS_E) {
#pragma unroll
            for (int c = 0; c < 9; ++c) p[c] = T(a.E[c]);
        } else if (MODE == X_FWD_REAL) {
#pragma unroll
            for (int c = 0; c < 9; ++c) p[c] = live ? T(a.real_in[c * a.g.n + vox]) : T(0);
        } else {
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                p[2 * s] = z[s][sl].x;
                if (s < 4) p[2 * s + 1] = z[s][sl].y;
            }
        }
        if (MODE == X_INV_REAL) {
            if (live)
#pragma unroll
                for (int c = 0; c < 9; ++c) a.real_out[c * a.g.n + vox] = double(p[c]) * a.scale;
            continue;
        }
        if (MODE == X_AVG) {
#pragma unroll
            for (int c = 0; c < 9; ++c) p[c] = T(double(p[c]) * a.scale + a.E[c]);
        }
        T tau[9];
        if (MODE == X_FWD_REAL || !live) {
#pragma unroll
            for (int c = 0; c < 9; ++c) tau[c] = p[c];
        } else {
            tangent_apply<T>(a.ts, a.g.xwbits >= 0 ? row * L + lane + W * sl : vox, p, tau);
        }
        if (MODE == X_AVG) {
            if (live)
#pragma unroll
                for (int c = 0; c < 9; ++c) acc[c] += double(tau[c]);
            continue;
        }
#pragma unroll
        for (int s = 0; s < 5; ++s) z[s][sl] = mk<T>(tau[2 * s], s < 4 ? tau[2 * s + 1] : T(0));
    }
    if (MODE == X_AVG) {
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const double t = block_sum(acc[c], red);
            if (threadIdx.x == 0) a.partials[(long long)tile_ * 9 + c] = t;
        }
        return;
    }
    if (!HAS_FWD) return;
    const int src = (W - lane) & (W - 1);
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        wave_fft_scr2nat<-1, M, W, T>(z[s], lane, tw);
        const int ca = 2 * s, cb = 2 * s + 1;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            if (W * r >= nh) break;                       // no lane of this slot stores
            const C zk = z[s][r];
            C zm = shfl_c<W, T>(z[s][M - 1 - r], src);       // index L - k for lanes l >= 1
            if (lane == 0) zm = z[s][(M - r) % M];        // index L - W r for lane 0
            const int k = lane + W * r;
            if (!live || k >= nh) continue;
            C ha = mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));
            C hb = mk<T>(T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x));
            const T x1 = xs1 * T(k);
            if (xi1_comp(ca)) ha = cscale(ha, x1);
            if (xi1_comp(cb)) hb = cscale(hb, x1);
            const long long off = row * nh + k;
            a.out[ca * a.g.nspec + off] = ha;
            if (s < 4) a.out[cb * a.g.nspec + off] = hb;
        }
    }
}

template <typename T, int MODE, int M, int W>
__global__ void __launch_bounds__(256) k_xwave(XArgs<T> a) {
    k_xwave_body<T, MODE, M, W>(a, blockIdx.x, gridDim.x);
}

template <typename T, int MODE, int M, int W>
__global__ void __launch_bounds__(256) k_xwave_b(const XArgs<T>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_xwave_body<T, MODE, M, W>(as[e.rve], e.tile, e.ntiles);
}

// (M, W) of the wavefront x pass for a row length n1, or M = 0 if unsupported
// ------------------------------------------------------------------------------
// x pass, two-stage version (CG operator and averaged tangent): a workgroup takes
// R rows; the five packed sequences of its rows are 5R "columns" of an
// L = P * Q two-stage transform (size-Q DFT in registers, twiddles, one LDS
// exchange, size-P DFT in registers; fft_reg.h).  Between the inverse and the
// forward transform the real rows sit in LDS, where the tangent acts voxel by
// voxel with the state read in natural order.  Column t = s R + r (sequence s,
// row r); a stage-A item (t, j1) holds x[j1 + P j2], a stage-B item (t, k1)
// holds X[k1 + Q k2], and the forward stage A starts from the LDS rows.
// ------------------------------------------------------------------------------
template <int P, int Q, int RR = 0>
struct XLdsShape {
    static constexpr int L = P * Q;
    static constexpr int NT = P > Q ? P : Q;                     // threads per column
    static constexpr int R = RR > 0 ? RR : 256 / (5 * NT);       // rows per workgroup
    static constexpr int TX = 5 * R;                             // columns
    static constexpr int NTH = (TX * NT + 63) / 64 * 64;         // threads per workgroup
    static constexpr int QP = Q + 1;            // padded stage-A row (LDS banks)
    static constexpr int LP = L + 1;            // padded natural row
    static constexpr int EXA = TX * P * QP;     // complex elements of the exchange
    static constexpr int EXN = TX * LP;         // complex elements of the natural rows
};

constexpr int cmax3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }

template <typename T, int MODE, int P, int Q, int RR, int DISC>
__device__ __forceinline__ void k_xlds_body(const XArgs<T>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    using S = XLdsShape<P, Q, RR>;
    constexpr int L = S::L, R = S::R, TX = S::TX, QP = S::QP, LP = S::LP;
    constexpr int FLD = (10 * R * L * (int)sizeof(T) + (int)sizeof(C) - 1) / (int)sizeof(C);
    constexpr int BUFC = cmax3(S::EXA, S::EXN, FLD);
    if (MODE == X_CG && a.st->done) return;
    if (MODE != X_CG && a.skip_done && a.st->done) return;
    __shared__ C buf[BUFC];   // exchange, natural rows and real rows in turn
    // stored x frequencies: the Nyquist bin is dropped (Moulinec-Suquet) or kept (rotated
    // scheme, whose rows may be padded: row stride ld >= nh)
    constexpr int nh = DISC ? L / 2 + 1 : L / 2;
    const int ld = DISC ? a.g.nh : nh;
    __shared__ C tw[L];
    __shared__ T fx[DISC ? 2 * nh : 1];   // rotated scheme: D1[nh] A1[nh]
    __shared__ double red[16];
    T* fld = reinterpret_cast<T*>(buf);   // real rows [9][R][L] and a sink row block
    const int tid = threadIdx.x;
    static_assert(L % 2 == 0, "two-stage x pass rows have even length");
    const long long nspec = a.g.nspec;
    const long long nrows = (long long)a.g.n2 * a.g.n3;
    const long long row0 = (long long)tile_ * R;
    const T xs1 = T(a.g.xs1);
    for (int i = tid; i < L; i += blockDim.x) tw[i] = a.tw[i];
    if constexpr (DISC) {
        stage_factors<T>(fx, a.g.ftab, nh, tid, blockDim.x);
        stage_factors<T>(fx + nh, a.g.ftab + ld, nh, tid, blockDim.x);
    }
    const int t = tid / S::NT, j = tid % S::NT;   // column and item index of this thread
    const bool col_ok = t < TX;
    const int s = col_ok ? t / R : 0, r = col_ok ? t % R : 0;
    const long long row = row0 + r;
    const bool live = col_ok && row < nrows;
    const int ca = 2 * s, cb = 2 * s + 1;
    __syncthreads();

    // ---- inverse: half spectra -> packed complex rows z = a + i b -> real rows.
    // Branch-free so that all loads of an item are in flight together: the fifth
    // sequence (one component) reads its component twice and scales the copy by
    // 0, and invalid bins read bin 0 of the row and scale it by 0.
    T* fa = fld + (ca * R + r) * L;
    T* fb = fld + ((s < 4 ? cb : 9) * R + r) * L;   // row 9 of fld is a write-only sink
    C y[P];
    if constexpr (MODE != X_FWD_REAL) {
    if (col_ok && j < P) {
        const long long rowc = live ? row : 0;
        const C* pa = a.in + ca * nspec + rowc * ld;
        const C* pb = a.in + (s < 4 ? cb : ca) * nspec + rowc * ld;
        const bool sa = xi1_comp(ca), sb = xi1_comp(cb);
        const T mb0 = s < 4 ? T(1) : T(0);
        C ha[Q], hb[Q];
#pragma unroll
        for (int j2 = 0; j2 < Q; ++j2) {
            const int k = j + P * j2;
            const int kk = k > L / 2 ? L - k : (k == L / 2 && !DISC ? 0 : k);
            const int kc = kk < nh ? kk : 0;
            ha[j2] = pa[kc];
            hb[j2] = pb[kc];
        }
        C x[Q];
#pragma unroll
        for (int j2 = 0; j2 < Q; ++j2) {
            const int k = j + P * j2;
            const bool conj = k > L / 2;
            const int kk = conj ? L - k : k;
            const T m = (live && kk < nh) ? T(1) : T(0);
            T ma, mb;
            C A, B;
            if constexpr (DISC == 2) {   // staggered grid: components (i, 1) times f_1
                const C f1 = mk<T>(fx[kk], fx[nh + kk]);
                A = cscale(sa ? cmul(ha[j2], f1) : ha[j2], m);
                B = cscale(sb ? cmul(hb[j2], f1) : hb[j2], mb0 * m);
            } else {
                if constexpr (DISC) {
                    const T d1 = fx[kk], a1 = fx[nh + kk];
                    ma = m * (sa ? d1 : a1);
                    mb = mb0 * m * (sb ? d1 : a1);
                } else {
                    const T x1 = xs1 * T(kk);
                    ma = sa ? m * x1 : m;
                    mb = sb ? mb0 * m * x1 : mb0 * m;
                }
                A = cscale(ha[j2], ma);
                B = cscale(hb[j2], mb);
            }
            const C zc = conj ? mk<T>(A.x + B.y, B.x - A.y) : mk<T>(A.x - B.y, A.y + B.x);
            x[j2] = (k == 0 || 2 * k == L) ? mk<T>(A.x, B.x) : zc;   // self-conjugate bins (L/2: zero unless stored)
        }
        RegDFT<Q, +1, C>::run(x);
#pragma unroll
        for (int k1 = 0; k1 < Q; ++k1) {
            C v = x[k1];
            if (k1 > 0) {
                C w = tw[j * k1];
                w.y = -w.y;
                v = cmul(v, w);
            }
            buf[(t * P + j) * QP + k1] = v;
        }
    }
    __syncthreads();
    if (col_ok && j < Q) {
#pragma unroll
        for (int j1 = 0; j1 < P; ++j1) y[j1] = buf[(t * P + j1) * QP + j];
        RegDFT<P, +1, C>::run(y);   // y[k2] = z at voxel j + Q k2
    }
    __syncthreads();
    if (col_ok && j < Q) {
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) {
            fa[j + Q * k2] = y[k2].x;
            fb[j + Q * k2] = y[k2].y;
        }
    }
    __syncthreads();
    }   // MODE != X_FWD_REAL

    // ---- real fields in the precision of the pass (staggered-grid CG operator)
    if constexpr (MODE == X_INV_REAL) {
        const T sc = T(a.scale);
        for (int v = tid; v < R * L; v += blockDim.x) {
            const int rr = v / L, xx = v - rr * L;
            const long long rw = row0 + rr;
            if (rw >= nrows) continue;
#pragma unroll
            for (int c = 0; c < 9; ++c) a.real_out_t[c * a.g.n + rw * L + xx] = fld[(c * R + rr) * L + xx] * sc;
        }
        return;
    }
    if constexpr (MODE == X_FWD_REAL) {
        for (int v = tid; v < R * L; v += blockDim.x) {
            const int rr = v / L, xx = v - rr * L;
            const long long rw = row0 + rr;
#pragma unroll
            for (int c = 0; c < 9; ++c) fld[(c * R + rr) * L + xx] = rw < nrows ? a.real_in_t[c * a.g.n + rw * L + xx] : T(0);
        }
        __syncthreads();
    }

    // ---- tangent action per voxel (X_AVG: averaged instead of stored).  Moulinec-Suquet:
    // the state of all of a thread's voxels is requested first (slot, F^{-1} and
    // mu - lambda ln J, read for every voxel: in bounds, unused for composites), so
    // that one memory round trip serves them all instead of two dependent ones per voxel.
    double acc[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] = 0.0;
    if constexpr ((MODE == X_CG || MODE == X_AVG) && DISC == 0) {
        constexpr int NTH = S::NTH;
        constexpr int VPT = (R * L + NTH - 1) / NTH;   // voxels per thread
        int sl[VPT];
        T fis[VPT][9], mss[VPT];
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int v = tid + q * NTH;
            const int rr = v / L, xx = v - rr * L;
            const bool ok = v < R * L && row0 + rr < nrows;
            const long long sidx = ok ? (row0 + rr) * L + xx : 0;
            sl[q] = a.ts.slot[sidx];
#pragma unroll
            for (int c = 0; c < 9; ++c) fis[q][c] = a.ts.Sinv[c * a.ts.n + sidx];
            mss[q] = a.ts.sm[sidx];
        }
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int v = tid + q * NTH;
            const int rr = v / L, xx = v - rr * L;
            if (v >= R * L || row0 + rr >= nrows) continue;
            T p[9], tau[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) p[c] = fld[(c * R + rr) * L + xx];
            if (MODE == X_AVG) {
#pragma unroll
                for (int c = 0; c < 9; ++c) p[c] = T(double(p[c]) * a.scale + a.E[c]);
            }
            tangent_apply_loaded<T>(a.ts, sl[q], fis[q], mss[q], p, tau);
            if (MODE == X_AVG) {
#pragma unroll
                for (int c = 0; c < 9; ++c) acc[c] += double(tau[c]);
            } else {
#pragma unroll
                for (int c = 0; c < 9; ++c) fld[(c * R + rr) * L + xx] = tau[c];
            }
        }
    } else {
        // rotated scheme: voxel by voxel (its x pass has fewer registers to spare)
        for (int v = (MODE == X_FWD_REAL) ? R * L : tid; v < R * L; v += blockDim.x) {
            const int rr = v / L, xx = v - rr * L;
            const long long rw = row0 + rr;
            if (rw >= nrows) continue;
            T p[9], tau[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) p[c] = fld[(c * R + rr) * L + xx];
            if (MODE == X_AVG) {
#pragma unroll
                for (int c = 0; c < 9; ++c) p[c] = T(double(p[c]) * a.scale + a.E[c]);
            }
            tangent_apply<T>(a.ts, rw * L + xx, p, tau);
            if (MODE == X_AVG) {
#pragma unroll
                for (int c = 0; c < 9; ++c) acc[c] += double(tau[c]);
            } else {
#pragma unroll
                for (int c = 0; c < 9; ++c) fld[(c * R + rr) * L + xx] = tau[c];
            }
        }
    }
    if (MODE == X_AVG) {
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const double tt = block_sum(acc[c], red);
            if (tid == 0) a.partials[(long long)tile_ * 9 + c] = tt;
        }
        return;
    }
    if (MODE != X_FWD_REAL) __syncthreads();

    // ---- forward: real rows -> packed complex rows -> half spectra
    C x2[Q];
    if (col_ok && j < P) {
        const T* gb = fld + ((s < 4 ? cb : ca) * R + r) * L;
        const T mb0 = s < 4 ? T(1) : T(0);
#pragma unroll
        for (int j2 = 0; j2 < Q; ++j2) {
            const int xx = j + P * j2;
            x2[j2] = mk<T>(fa[xx], mb0 * gb[xx]);
        }
    }
    __syncthreads();
    if (col_ok && j < P) {
        RegDFT<Q, -1, C>::run(x2);
#pragma unroll
        for (int k1 = 0; k1 < Q; ++k1) {
            C v = x2[k1];
            if (k1 > 0) v = cmul(v, tw[j * k1]);
            buf[(t * P + j) * QP + k1] = v;
        }
    }
    __syncthreads();
    if (col_ok && j < Q) {
#pragma unroll
        for (int j1 = 0; j1 < P; ++j1) y[j1] = buf[(t * P + j1) * QP + j];
        RegDFT<P, -1, C>::run(y);   // y[k2] = Z[j + Q k2]
    }
    __syncthreads();
    if (col_ok && j < Q) {
#pragma unroll
        for (int k2 = 0; k2 < P; ++k2) buf[t * LP + j + Q * k2] = y[k2];
    }
    __syncthreads();
    for (int i = tid; i < TX * ld; i += blockDim.x) {
        const int tt = i / ld, k = i - tt * ld;
        const int ss = tt / R, rr = tt - ss * R;
        const long long rw = row0 + rr;
        if (rw >= nrows) continue;
        const C zk = buf[tt * LP + k];
        const C zm = buf[tt * LP + (k == 0 ? 0 : L - k)];
        C ha = mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));
        C hb = mk<T>(T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x));
        const int c1 = 2 * ss, c2 = 2 * ss + 1;
        if constexpr (DISC == 2) {   // staggered grid: components (i, 1) times conj(f_1)
            const bool pad = k >= nh;
            const C f1c = pad ? mk<T>(0, 0) : mk<T>(fx[k], -fx[nh + k]);
            ha = xi1_comp(c1) ? cmul(ha, f1c) : (pad ? mk<T>(0, 0) : ha);
            hb = xi1_comp(c2) ? cmul(hb, f1c) : (pad ? mk<T>(0, 0) : hb);
        } else if constexpr (DISC) {
            const bool pad = k >= nh;   // row padding: zero modes
            const T d1 = pad ? T(0) : fx[k], a1 = pad ? T(0) : fx[nh + k];
            ha = cscale(ha, xi1_comp(c1) ? d1 : a1);
            hb = cscale(hb, xi1_comp(c2) ? d1 : a1);
        } else {
            const T x1 = xs1 * T(k);
            if (xi1_comp(c1)) ha = cscale(ha, x1);
            if (xi1_comp(c2)) hb = cscale(hb, x1);
        }
        const long long off = rw * ld + k;
        a.out[c1 * nspec + off] = ha;
        if (ss < 4) a.out[c2 * nspec + off] = hb;
    }
}

template <typename T, int MODE, int P, int Q, int RR, int DISC>
__global__ void __launch_bounds__((XLdsShape<P, Q, RR>::NTH)) k_xlds(XArgs<T> a) {
    k_xlds_body<T, MODE, P, Q, RR, DISC>(a, blockIdx.x, gridDim.x);
}

template <typename T, int MODE, int P, int Q, int RR, int DISC>
__global__ void __launch_bounds__((XLdsShape<P, Q, RR>::NTH)) k_xlds_b(const XArgs<T>* __restrict__ as,
                                                                         const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_xlds_body<T, MODE, P, Q, RR, DISC>(as[e.rve], e.tile, e.ntiles);
}

// row lengths with a two-stage x pass (CG operator, averaged tangent):
// L, P, Q, rows per workgroup (0 = as many as fit 256 threads), variant.
// Variants above 0 are autotuner candidates, built for float only.
#define COMBO_XLDS_CONFIGS(X) \
    X(256, 16, 16, 0, 0)      \
    X(256, 16, 16, 2, 1)      \
    X(128, 8, 16, 0, 0)       \
    X(128, 16, 8, 0, 1)       \
    X(384, 16, 24, 0, 0)      \
    X(384, 24, 16, 0, 1)      \
    X(192, 16, 12, 0, 0)      \
    X(192, 12, 16, 0, 1)      \
    X(96, 8, 12, 0, 0)        \
    X(96, 12, 8, 0, 1)        \
    X(64, 8, 8, 0, 0)         \
    X(64, 8, 8, 3, 1)         \
    X(48, 8, 6, 0, 0)         \
    X(48, 6, 8, 0, 1)         \
    X(32, 4, 8, 0, 0)         \
    X(32, 8, 4, 0, 1)

#define COMBO_XWAVE_CONFIGS(X) \
    X(256, 4, 64)              \
    X(128, 2, 64)              \
    X(64, 1, 64)               \
    X(384, 6, 64)              \
    X(192, 3, 64)              \
    X(96, 3, 32)               \
    X(48, 3, 16)               \
    X(32, 1, 32)               \
    X(16, 1, 16)

// ------------------------------------------------------------------------------
// y passes: tile = TX consecutive x frequencies of one z plane, all y
// ------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void y_load(const YArgs<T>& a, cpx<T>* buf, int comp, int z, int kx0, int TX) {
    const int n2 = a.g.n2, nh = a.g.nh;
    const int items = n2 * TX;
    for (int e = threadIdx.x; e < items; e += kBlock) {
        const int y = e / TX, t = e - y * TX;
        const int kx = kx0 + t;
        buf[e] = (kx < nh) ? a.in[comp * a.g.nspec + ((long long)z * n2 + y) * nh + kx] : mk<T>(0, 0);
    }
}

template <typename T>
__device__ __forceinline__ void y_store(const YArgs<T>& a, const cpx<T>* buf, int comp, int z, int kx0, int TX) {
    const int n2 = a.g.n2, nh = a.g.nh;
    const int items = n2 * TX;
    for (int e = threadIdx.x; e < items; e += kBlock) {
        const int y = e / TX, t = e - y * TX;
        const int kx = kx0 + t;
        if (kx < nh) a.out[comp * a.g.nspec + ((long long)z * n2 + y) * nh + kx] = buf[e];
    }
}

// forward: in 9 comps (row-major (i,J), comps (i,1) already times xi_1) -> out 6:
// out_i = FFT(in_i1) + xi_2 FFT(in_i2), out_{3+i} = FFT(in_i3)   (1-based J in the comments)
template <typename T, int DISC>
__device__ __forceinline__ void k_ypass_fwd_body(const YArgs<T>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    if (a.st && a.st->done) return;
    extern __shared__ char smem_raw[];
    const int L = a.g.n2, TX = a.TX;
    C* tw = reinterpret_cast<C*>(smem_raw);
    C* buf = tw + L;
    const int z = tile_ / a.ntile;
    const int kx0 = (tile_ % a.ntile) * TX;
    load_twiddles<T>(tw, a.tw, L);
    constexpr int Q = max_elems<T>() / kBlock;
    C acc[Q];
    const int items = L * TX;
    const T xs2 = T(a.g.xs2);
    for (int i = 0; i < 3; ++i) {
        y_load(a, buf, 3 * i + 0, z, kx0, TX);
        __syncthreads();
        fft_lds<-1, false, T>(buf, a.plan, TX, tw);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + q * kBlock;
            if (e < items) acc[q] = buf[e];
        }
        __syncthreads();
        y_load(a, buf, 3 * i + 1, z, kx0, TX);
        __syncthreads();
        fft_lds<-1, false, T>(buf, a.plan, TX, tw);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + q * kBlock;
            if (e < items) {
                const int y = e / TX, t = e - y * TX;
                C v;
                if (DISC == 2) {
                    v = cadd(acc[q], cmul(buf[e], cconj(fst2<T>(a.g, y))));
                } else {
                    const T x2 = DISC ? T(fac_d2(a.g, y)) : xs2 * T(freq_of(y, L));
                    const C a0 = DISC ? cscale(acc[q], T(fac_a2(a.g, y))) : acc[q];
                    v = cadd(a0, cscale(buf[e], x2));
                }
                const int kx = kx0 + t;
                if (kx < a.g.nh) a.out[i * a.g.nspec + ((long long)z * L + y) * a.g.nh + kx] = v;
            }
        }
        __syncthreads();
        y_load(a, buf, 3 * i + 2, z, kx0, TX);
        __syncthreads();
        fft_lds<-1, false, T>(buf, a.plan, TX, tw);
        if (DISC == 1) {
            for (int e = threadIdx.x; e < items; e += kBlock) buf[e] = cscale(buf[e], T(fac_a2(a.g, e / TX)));
            __syncthreads();
        }
        y_store(a, buf, 3 + i, z, kx0, TX);
        __syncthreads();
    }
}

template <typename T, int DISC>
__global__ void __launch_bounds__(kBlock) k_ypass_fwd(YArgs<T> a) {
    k_ypass_fwd_body<T, DISC>(a, blockIdx.x, gridDim.x);
}

template <typename T, int DISC>
__global__ void __launch_bounds__(kBlock) k_ypass_fwd_b(const YArgs<T>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_ypass_fwd_body<T, DISC>(as[e.rve], e.tile, e.ntiles);
}

// inverse: in 6 comps [A_i, B_i] -> out 9: (i,1) = IFFT(A_i), (i,2) = IFFT(xi_2 A_i), (i,3) = IFFT(B_i)
template <typename T, int DISC>
__device__ __forceinline__ void k_ypass_inv_body(const YArgs<T>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    if (a.st && a.st->done) return;
    extern __shared__ char smem_raw[];
    const int L = a.g.n2, TX = a.TX;
    C* tw = reinterpret_cast<C*>(smem_raw);
    C* buf = tw + L;
    const int z = tile_ / a.ntile;
    const int kx0 = (tile_ % a.ntile) * TX;
    load_twiddles<T>(tw, a.tw, L);
    constexpr int Q = max_elems<T>() / kBlock;
    C av[Q];
    const int items = L * TX;
    const T xs2 = T(a.g.xs2);
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + q * kBlock;
            if (e < items) {
                const int y = e / TX, t = e - y * TX;
                const int kx = kx0 + t;
                av[q] = (kx < a.g.nh) ? a.in[i * a.g.nspec + ((long long)z * L + y) * a.g.nh + kx] : mk<T>(0, 0);
                buf[e] = (DISC == 1) ? cscale(av[q], T(fac_a2(a.g, y))) : av[q];
            }
        }
        __syncthreads();
        fft_lds<+1, false, T>(buf, a.plan, TX, tw);
        y_store(a, buf, 3 * i + 0, z, kx0, TX);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + q * kBlock;
            if (e < items) {
                const int y = e / TX;
                buf[e] = (DISC == 2) ? cmul(av[q], fst2<T>(a.g, y))
                                     : cscale(av[q], DISC ? T(fac_d2(a.g, y)) : xs2 * T(freq_of(y, L)));
            }
        }
        __syncthreads();
        fft_lds<+1, false, T>(buf, a.plan, TX, tw);
        y_store(a, buf, 3 * i + 1, z, kx0, TX);
        __syncthreads();
        y_load(a, buf, 3 + i, z, kx0, TX);
        __syncthreads();
        if (DISC == 1) {
            for (int e = threadIdx.x; e < items; e += kBlock) buf[e] = cscale(buf[e], T(fac_a2(a.g, e / TX)));
            __syncthreads();
        }
        fft_lds<+1, false, T>(buf, a.plan, TX, tw);
        y_store(a, buf, 3 * i + 2, z, kx0, TX);
        __syncthreads();
    }
}

template <typename T, int DISC>
__global__ void __launch_bounds__(kBlock) k_ypass_inv(YArgs<T> a) {
    k_ypass_inv_body<T, DISC>(a, blockIdx.x, gridDim.x);
}

template <typename T, int DISC>
__global__ void __launch_bounds__(kBlock) k_ypass_inv_b(const YArgs<T>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_ypass_inv_body<T, DISC>(as[e.rve], e.tile, e.ntiles);
}

// ------------------------------------------------------------------------------
// z passes: tile = TX consecutive elements m of the (y, x) frequency plane, all z
// ------------------------------------------------------------------------------
struct Freq {
    double x1, x2, x3, s;   // xi and |xi|^2
    bool zero;              // zero mode or Nyquist plane: projected out
    double w;               // Parseval weight of the half spectrum (1 or 2)
};

// frequency data of one (y, x) column m = ky nh + kx of the half spectrum
// (m < 2^31 for every supported grid: 32-bit index arithmetic)
struct ColFreq {
    double x1, x2, s12;     // xi_1, xi_2, xi_1^2 + xi_2^2 (rotated scheme: D1 A2, A1 D2, unused)
    double c3;              // rotated scheme: A1 A2
    double w;               // Parseval weight (1 on the kx = 0 plane, else 2)
    int kx, ky;
    bool zero12;            // kx = 0 and ky = 0
    bool nyq2;              // Nyquist plane of y
};

// column data of the rotated scheme (what col_freq_k computes when g.disc is set)
__device__ __forceinline__ ColFreq col_freq_rot(const Grid& g, int ky, int kx) {
    ColFreq c;
    c.ky = ky;
    c.kx = kx;
    const double d1 = fac_d1(g, kx), a1 = fac_a1(g, kx), d2 = fac_d2(g, ky), a2 = fac_a2(g, ky);
    c.x1 = d1 * a2;
    c.x2 = a1 * d2;
    c.c3 = a1 * a2;
    c.s12 = 0.0;
    c.w = (kx == 0 || 2 * kx == g.n1) ? 1.0 : 2.0;
    c.zero12 = false;
    c.nyq2 = false;
    return c;
}

__device__ __forceinline__ ColFreq col_freq_k(const Grid& g, int ky, int kx) {
    ColFreq c;
    c.ky = ky;
    c.kx = kx;
    if (g.disc) {
        const double d1 = fac_d1(g, kx), a1 = fac_a1(g, kx), d2 = fac_d2(g, ky), a2 = fac_a2(g, ky);
        c.x1 = d1 * a2;
        c.x2 = a1 * d2;
        c.c3 = a1 * a2;
        c.s12 = 0.0;
        c.w = (kx == 0 || 2 * kx == g.n1) ? 1.0 : 2.0;
        c.zero12 = false;
        c.nyq2 = false;
        return c;
    }
    c.c3 = 1.0;
    const int fy = freq_of(c.ky, g.n2);
    c.x1 = g.xs1 * c.kx;
    c.x2 = g.xs2 * fy;
    c.s12 = c.x1 * c.x1 + c.x2 * c.x2;
    c.w = (c.kx == 0) ? 1.0 : 2.0;
    c.zero12 = (c.kx == 0 && fy == 0);
    c.nyq2 = is_nyquist(c.ky, g.n2);
    return c;
}

__device__ __forceinline__ ColFreq col_freq(const Grid& g, int m) {
    const int ky = m / g.nh;
    return col_freq_k(g, ky, m - ky * g.nh);
}

// rotated scheme: the column's factors times the z factors a3 = A3(z), d3 = D3(z) (what
// freq_z computes when g.disc is set, with the factors passed in)
__device__ __forceinline__ Freq freq_z_rot(const ColFreq& c, double a3, double d3) {
    Freq f;
    f.x1 = c.x1 * a3;
    f.x2 = c.x2 * a3;
    f.x3 = c.c3 * d3;
    f.s = f.x1 * f.x1 + f.x2 * f.x2 + f.x3 * f.x3;
    f.zero = !(f.s > 0.0);   // the mean and modes on two or more Nyquist planes
    f.w = c.w;
    return f;
}

__device__ __forceinline__ Freq freq_z(const Grid& g, const ColFreq& c, int z) {
    Freq f;
    if (g.disc) {
        const double a3 = fac_a3(g, z);
        f.x1 = c.x1 * a3;
        f.x2 = c.x2 * a3;
        f.x3 = c.c3 * fac_d3(g, z);
        f.s = f.x1 * f.x1 + f.x2 * f.x2 + f.x3 * f.x3;
        f.zero = !(f.s > 0.0);   // the mean and modes on two or more Nyquist planes
        f.w = c.w;
        return f;
    }
    const int fz = freq_of(z, g.n3);
    f.x1 = c.x1;
    f.x2 = c.x2;
    f.x3 = g.xs3 * fz;
    f.s = c.s12 + f.x3 * f.x3;
    f.zero = (c.zero12 && fz == 0) || c.nyq2 || is_nyquist(z, g.n3);
    f.w = c.w;
    return f;
}

__device__ __forceinline__ Freq freq_at(const Grid& g, long long m, int z) {
    return freq_z(g, col_freq(g, (int)m), z);
}

// w = K^{-1} v with K = mu0 |xi|^2 I + kappa0 xi (x) xi
template <typename C, typename T>
__device__ __forceinline__ void kinv(const Freq& f, T mu0, T kappa0, const C* v, C* w) {
    const T x1 = T(f.x1), x2 = T(f.x2), x3 = T(f.x3), s = T(f.s);
    const T theta = kappa0 / (mu0 + kappa0);
    C xv;
    xv.x = x1 * v[0].x + x2 * v[1].x + x3 * v[2].x;
    xv.y = x1 * v[0].y + x2 * v[1].y + x3 * v[2].y;
    const T inv = T(1) / (mu0 * s);
    const T t = theta / s;
    const T xx[3] = {x1, x2, x3};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        w[i].x = (v[i].x - t * xx[i] * xv.x) * inv;
        w[i].y = (v[i].y - t * xx[i] * xv.y) * inv;
    }
}

// K u for a CG vector u (used in the C0 inner products)
template <typename C>
__device__ __forceinline__ void kmul(const Freq& f, double mu0, double kappa0, const C* u, double* kr, double* ki) {
    const double xu_r = f.x1 * double(u[0].x) + f.x2 * double(u[1].x) + f.x3 * double(u[2].x);
    const double xu_i = f.x1 * double(u[0].y) + f.x2 * double(u[1].y) + f.x3 * double(u[2].y);
    const double xx[3] = {f.x1, f.x2, f.x3};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        kr[i] = mu0 * f.s * double(u[i].x) + kappa0 * xx[i] * xu_r;
        ki[i] = mu0 * f.s * double(u[i].y) + kappa0 * xx[i] * xu_i;
    }
}

// Staggered grid (disc 2): the complex forward-difference symbols f = (f1, f2, f3)
// of one stored mode.  The displacement coefficients u of a compatible field give
// its gradient in the shifted layout as H_hat_iJ = f_J u_i, and the reference
// medium's acoustic tensor is K_ab = mu0 |f|^2 d_ab + kappa0 conj(f_a) f_b.
struct FreqC {
    double fr[3], fi[3];    // Re and Im of f_d
    double s;               // |f|^2
    bool zero;              // the mean, the only mode with f = 0: projected out
    double w;               // Parseval weight of the half spectrum (1 or 2)
};

__device__ __forceinline__ FreqC freqc_k(const Grid& g, int ky, int kx, int z) {
    FreqC f;
    f.fr[0] = g.ftab[kx];
    f.fi[0] = g.ftab[g.nh + kx];
    f.fr[1] = g.ftab[2 * g.nh + ky];
    f.fi[1] = g.ftab[2 * g.nh + g.n2 + ky];
    f.fr[2] = g.ftab[2 * g.nh + 2 * g.n2 + z];
    f.fi[2] = g.ftab[2 * g.nh + 2 * g.n2 + g.n3 + z];
    f.s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) f.s += f.fr[d] * f.fr[d] + f.fi[d] * f.fi[d];
    f.zero = !(f.s > 0.0);
    f.w = (kx == 0 || 2 * kx == g.n1) ? 1.0 : 2.0;
    return f;
}

__device__ __forceinline__ FreqC freqc_at(const Grid& g, long long m, int z) {
    const int ky = (int)(m / g.nh);
    return freqc_k(g, ky, (int)(m - (long long)ky * g.nh), z);
}

// w = K^{-1} v:  w = (v - theta conj(f) (f . v) / |f|^2) / (mu0 |f|^2), theta = kappa0 / (mu0 + kappa0)
template <typename C, typename T>
__device__ __forceinline__ void kinv_stag(const FreqC& f, T mu0, T kappa0, const C* v, C* w) {
    T fvr = T(0), fvi = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        fvr += T(f.fr[b]) * v[b].x - T(f.fi[b]) * v[b].y;
        fvi += T(f.fr[b]) * v[b].y + T(f.fi[b]) * v[b].x;
    }
    const T s = T(f.s);
    const T t = (kappa0 / (mu0 + kappa0)) / s;
    const T inv = T(1) / (mu0 * s);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T cr = T(f.fr[a]) * fvr + T(f.fi[a]) * fvi;    // conj(f_a) (f . v)
        const T ci = T(f.fr[a]) * fvi - T(f.fi[a]) * fvr;
        w[a].x = (v[a].x - t * cr) * inv;
        w[a].y = (v[a].y - t * ci) * inv;
    }
}

// K u (FP64), for the C0 inner products
template <typename C>
__device__ __forceinline__ void kmul_stag(const FreqC& f, double mu0, double kappa0, const C* u, double* kr,
                                          double* ki) {
    double fur = 0.0, fui = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        fur += f.fr[b] * double(u[b].x) - f.fi[b] * double(u[b].y);
        fui += f.fr[b] * double(u[b].y) + f.fi[b] * double(u[b].x);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        kr[a] = mu0 * f.s * double(u[a].x) + kappa0 * (f.fr[a] * fur + f.fi[a] * fui);
        ki[a] = mu0 * f.s * double(u[a].y) + kappa0 * (f.fr[a] * fui - f.fi[a] * fur);
    }
}

// Per-frequency end of the forward z pass: given v = tau_hat xi at the frequency f
// stored at idx (z M + m),
//   Z_CG:   q = K^{-1} v / n, accumulate <p, q>_K = w Re(p^H v)/n
//   Z_RHS:  r = b = -K^{-1} v, x = 0, accumulate <b, b>_K and |G P|^2 = |v|^2/|xi|^2
//   Z_PROJ: x = K^{-1} v
template <typename T, typename TU, int MODE>
__device__ __forceinline__ void z_epilogue(const ZArgs<T, TU>& a, const Freq& f, long long idx, const cpx<T>* vv,
                                           double& s1, double& s2) {
    using C = cpx<T>;
    using CU = cpx<TU>;
    C w[3];
    if (f.zero) {
        w[0] = w[1] = w[2] = mk<T>(0, 0);
    } else {
        kinv(f, T(a.mu0), T(a.kappa0), vv, w);
    }
    if (MODE == Z_CG) {
        const T sc = T(a.inv_n);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            CU qi;
            qi.x = TU(w[i].x * sc);
            qi.y = TU(w[i].y * sc);
            a.q[i * a.g.nspec + idx] = qi;
            if (!f.zero) {
                const CU pi = a.p[i * a.g.nspec + idx];
                s1 += f.w * (double(pi.x) * double(vv[i].x) + double(pi.y) * double(vv[i].y)) * a.inv_n;
            }
        }
    } else if (MODE == Z_RHS) {
        CU b[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            b[i].x = TU(-w[i].x);
            b[i].y = TU(-w[i].y);
            a.r[i * a.g.nspec + idx] = b[i];
            a.x[i * a.g.nspec + idx] = CU{TU(0), TU(0)};
        }
        if (!f.zero) {
            double kr[3], ki[3];
            kmul(f, a.mu0, a.kappa0, b, kr, ki);
            double bb = 0.0, vv2 = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                bb += double(b[i].x) * kr[i] + double(b[i].y) * ki[i];
                vv2 += double(vv[i].x) * double(vv[i].x) + double(vv[i].y) * double(vv[i].y);
            }
            s1 += f.w * bb;
            s2 += f.w * vv2 / f.s;
        }
    } else {  // Z_PROJ
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            CU o;
            o.x = TU(w[i].x);
            o.y = TU(w[i].y);
            a.x[i * a.g.nspec + idx] = o;
        }
    }
}

// z_epilogue at column m, frequency index z of the Moulinec-Suquet spectrum (frequency
// from the column data)
template <typename T, typename TU, int MODE>
__device__ __forceinline__ void z_epilogue_at(const ZArgs<T, TU>& a, const ColFreq& cf, long long m, int z,
                                              const cpx<T>* vv, double& s1, double& s2) {
    const long long M = (long long)a.g.n2 * a.g.nh;
    z_epilogue<T, TU, MODE>(a, freq_z(a.g, cf, z), (long long)z * M + m, vv, s1, s2);
}

// z_epilogue of the staggered grid: the same modes with the complex acoustic tensor
template <typename T, typename TU, int MODE>
__device__ __forceinline__ void z_epilogue_stag(const ZArgs<T, TU>& a, const FreqC& f, long long idx,
                                                const cpx<T>* vv, double& s1, double& s2) {
    using C = cpx<T>;
    using CU = cpx<TU>;
    C w[3];
    if (f.zero) {
        w[0] = w[1] = w[2] = mk<T>(0, 0);
    } else {
        kinv_stag(f, T(a.mu0), T(a.kappa0), vv, w);
    }
    if (MODE == Z_CG) {
        const T sc = T(a.inv_n);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            CU qi;
            qi.x = TU(w[i].x * sc);
            qi.y = TU(w[i].y * sc);
            a.q[i * a.g.nspec + idx] = qi;
            if (!f.zero) {
                const CU pi = a.p[i * a.g.nspec + idx];
                s1 += f.w * (double(pi.x) * double(vv[i].x) + double(pi.y) * double(vv[i].y)) * a.inv_n;
            }
        }
    } else if (MODE == Z_RHS) {
        CU b[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            b[i].x = TU(-w[i].x);
            b[i].y = TU(-w[i].y);
            a.r[i * a.g.nspec + idx] = b[i];
            a.x[i * a.g.nspec + idx] = CU{TU(0), TU(0)};
        }
        if (!f.zero) {
            double kr[3], ki[3];
            kmul_stag(f, a.mu0, a.kappa0, b, kr, ki);
            double bb = 0.0, vv2 = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                bb += double(b[i].x) * kr[i] + double(b[i].y) * ki[i];
                vv2 += double(vv[i].x) * double(vv[i].x) + double(vv[i].y) * double(vv[i].y);
            }
            s1 += f.w * bb;
            s2 += f.w * vv2 / f.s;
        }
    } else {  // Z_PROJ
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            CU o;
            o.x = TU(w[i].x);
            o.y = TU(w[i].y);
            a.x[i * a.g.nspec + idx] = o;
        }
    }
}

template <typename T>
__device__ __forceinline__ void z_load(const cpx<T>* in, const Grid& g, cpx<T>* buf, int comp, long long m0, int TX) {
    const long long M = (long long)g.n2 * g.nh;
    const int items = g.n3 * TX;
    for (int e = threadIdx.x; e < items; e += kBlock) {
        const int z = e / TX, t = e - z * TX;
        const long long m = m0 + t;
        buf[e] = (m < M) ? in[comp * g.nspec + (long long)z * M + m] : mk<T>(0, 0);
    }
}

template <typename T>
__device__ __forceinline__ void z_store(cpx<T>* out, const Grid& g, const cpx<T>* buf, int comp, long long m0, int TX) {
    const long long M = (long long)g.n2 * g.nh;
    const int items = g.n3 * TX;
    for (int e = threadIdx.x; e < items; e += kBlock) {
        const int z = e / TX, t = e - z * TX;
        const long long m = m0 + t;
        if (m < M) out[comp * g.nspec + (long long)z * M + m] = buf[e];
    }
}

// forward z pass: v_i = FFT(in_i) + xi_3 FFT(in_{3+i}) and then, by mode,
//   Z_CG:   q = K^{-1} v / n, partial sum of <p, q>_K = sum w Re(p^H v)/n
//   Z_RHS:  r = b = -K^{-1} v, x = 0, partials of <b, b>_K and of |G P|^2 = |v|^2/|xi|^2
//   Z_PROJ: x = K^{-1} v
template <typename T, typename TU, int MODE, int DISC>
__device__ __forceinline__ void k_zpass_fwd_body(const ZArgs<T, TU>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    using CU = cpx<TU>;
    if (MODE == Z_CG && a.st->done) return;
    extern __shared__ char smem_raw[];
    __shared__ double red[16];
    const int L = a.g.n3, TX = a.TX;
    C* tw = reinterpret_cast<C*>(smem_raw);
    C* buf = tw + L;
    const long long m0 = (long long)tile_ * TX;
    const long long M = (long long)a.g.n2 * a.g.nh;
    load_twiddles<T>(tw, a.tw, L);
    constexpr int Q = max_elems<T>() / kBlock;
    C v[3][Q];
    const int items = L * TX;
    const T xs3 = T(a.g.xs3);
    for (int i = 0; i < 3; ++i) {
        z_load<T>(a.in, a.g, buf, i, m0, TX);
        __syncthreads();
        fft_lds<-1, false, T>(buf, a.plan, TX, tw);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + q * kBlock;
            if (e < items) v[i][q] = (DISC == 1) ? cscale(buf[e], T(fac_a3(a.g, e / TX))) : buf[e];
        }
        __syncthreads();
        z_load<T>(a.in, a.g, buf, 3 + i, m0, TX);
        __syncthreads();
        fft_lds<-1, false, T>(buf, a.plan, TX, tw);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + q * kBlock;
            if (e < items) {
                const int z = e / TX;
                v[i][q] = (DISC == 2)
                              ? cadd(v[i][q], cmul(buf[e], cconj(fst3<T>(a.g, z))))
                              : cadd(v[i][q], cscale(buf[e], DISC ? T(fac_d3(a.g, z)) : xs3 * T(freq_of(z, L))));
            }
        }
        __syncthreads();
    }
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int e = threadIdx.x + q * kBlock;
        if (e >= items) continue;
        const int z = e / TX, t = e - z * TX;
        const long long m = m0 + t;
        if (m >= M) continue;
        C vv[3] = {v[0][q], v[1][q], v[2][q]};
        if (DISC == 2)
            z_epilogue_stag<T, TU, MODE>(a, freqc_at(a.g, m, z), (long long)z * M + m, vv, s1, s2);
        else
            z_epilogue<T, TU, MODE>(a, freq_at(a.g, m, z), (long long)z * M + m, vv, s1, s2);
    }
    if (MODE == Z_CG || MODE == Z_RHS) {
        const double t1 = block_sum(s1, red);
        if (threadIdx.x == 0) a.partials[tile_] = t1;
    }
    if (MODE == Z_RHS) {
        const double t2 = block_sum(s2, red);
        if (threadIdx.x == 0) a.partials2[tile_] = t2;
    }
}

template <typename T, typename TU, int MODE, int DISC>
__global__ void __launch_bounds__(kBlock) k_zpass_fwd(ZArgs<T, TU> a) {
    k_zpass_fwd_body<T, TU, MODE, DISC>(a, blockIdx.x, gridDim.x);
}

template <typename T, typename TU, int MODE, int DISC>
__global__ void __launch_bounds__(kBlock) k_zpass_fwd_b(const ZArgs<T, TU>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_zpass_fwd_body<T, TU, MODE, DISC>(as[e.rve], e.tile, e.ntiles);
}

// inverse z pass: source vector u (Z_INV_CG: p = r + beta p first, p = r on the
// first iteration; Z_INV_PLAIN: u = x), out_i = IFFT(u_i), out_{3+i} = IFFT(xi_3 u_i)
template <typename T, typename TU, int MODE, int DISC>
__device__ __forceinline__ void k_zpass_inv_body(const ZArgs<T, TU>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    using CU = cpx<TU>;
    if (MODE == Z_INV_CG && a.st->done) return;
    extern __shared__ char smem_raw[];
    const int L = a.g.n3, TX = a.TX;
    C* tw = reinterpret_cast<C*>(smem_raw);
    C* buf = tw + L;
    const long long m0 = (long long)tile_ * TX;
    const long long M = (long long)a.g.n2 * a.g.nh;
    load_twiddles<T>(tw, a.tw, L);
    constexpr int Q = max_elems<T>() / kBlock;
    const int items = L * TX;
    const T xs3 = T(a.g.xs3);
    double beta = 0.0;
    bool first = true;
    if (MODE == Z_INV_CG) {
        beta = a.st->beta;
        first = (a.st->iter == 0);
    }
    for (int i = 0; i < 3; ++i) {
        C u[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + q * kBlock;
            u[q] = mk<T>(0, 0);
            if (e < items) {
                const int z = e / TX, t = e - z * TX;
                const long long m = m0 + t;
                if (m < M) {
                    const long long idx = i * a.g.nspec + (long long)z * M + m;
                    if (MODE == Z_INV_CG) {
                        const CU ri = a.r[idx];
                        CU pn;
                        if (first) {
                            pn = ri;
                        } else {
                            const CU pi = a.p[idx];
                            pn.x = ri.x + TU(beta) * pi.x;
                            pn.y = ri.y + TU(beta) * pi.y;
                        }
                        a.p[idx] = pn;
                        u[q] = mk<T>(T(pn.x), T(pn.y));
                    } else {
                        const CU xi = a.x[idx];
                        u[q] = mk<T>(T(xi.x), T(xi.y));
                    }
                }
                buf[e] = (DISC == 1) ? cscale(u[q], T(fac_a3(a.g, e / TX))) : u[q];
            }
        }
        __syncthreads();
        fft_lds<+1, false, T>(buf, a.plan, TX, tw);
        z_store<T>(a.out, a.g, buf, i, m0, TX);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int e = threadIdx.x + q * kBlock;
            if (e < items) {
                const int z = e / TX;
                buf[e] = (DISC == 2) ? cmul(u[q], fst3<T>(a.g, z))
                                     : cscale(u[q], DISC ? T(fac_d3(a.g, z)) : xs3 * T(freq_of(z, L)));
            }
        }
        __syncthreads();
        fft_lds<+1, false, T>(buf, a.plan, TX, tw);
        z_store<T>(a.out, a.g, buf, 3 + i, m0, TX);
        __syncthreads();
    }
}

template <typename T, typename TU, int MODE, int DISC>
__global__ void __launch_bounds__(kBlock) k_zpass_inv(ZArgs<T, TU> a) {
    k_zpass_inv_body<T, TU, MODE, DISC>(a, blockIdx.x, gridDim.x);
}

template <typename T, typename TU, int MODE, int DISC>
__global__ void __launch_bounds__(kBlock) k_zpass_inv_b(const ZArgs<T, TU>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_zpass_inv_body<T, TU, MODE, DISC>(as[e.rve], e.tile, e.ntiles);
}

// ------------------------------------------------------------------------------
// CG update: x += alpha p, r -= alpha q, partial <r, r>_K
//
// On the stored half spectrum the x = 0 frequency plane holds both members of
// each conjugate pair (0, ky, kz) / (0, -ky, -kz).  A displacement coefficient
// field of a real deformation is anti-Hermitian there, u(-k) = -conj(u(k)); its
// Hermitian part is discarded by the real inverse transform along x and is
// therefore a null space of the CG operator.  Round-off would feed it and CG
// would grow it once the right-hand side is small, so r is projected back on
// the anti-Hermitian part in that plane; the thread owning the lower index of a
// pair updates both members.
// ------------------------------------------------------------------------------
__device__ __forceinline__ long long kx0_partner(const Grid& g, long long M, int z, int ky) {
    const int z2 = (g.n3 - z) % g.n3, ky2 = (g.n2 - ky) % g.n2;
    return (long long)z2 * M + (long long)ky2 * g.nh;
}

template <typename CU>
__device__ __forceinline__ void antiherm_pair(CU& a, CU& b) {
    // a <- (a - conj b)/2, b <- -conj(a_new)
    using TU = decltype(a.x);
    const double ax = 0.5 * (double(a.x) - double(b.x));
    const double ay = 0.5 * (double(a.y) + double(b.y));
    a.x = TU(ax);
    a.y = TU(ay);
    b.x = TU(-ax);
    b.y = TU(ay);
}

// Self-conjugate planes of the stored half spectrum: kx = 0, and kx = n1/2 where the
// rotated scheme stores it.  There a coefficient of a real field satisfies
// w(-k) = sigma conj(w(k)): sigma = -1 (anti-Hermitian) where k' changes sign with k,
// sigma = +1 (Hermitian) where it does not, i.e. (rotated scheme only) on the kx = n1/2
// plane and, on the kx = 0 plane, at modes with exactly one Nyquist index among ky, kz.
__device__ __forceinline__ bool selfconj_plane(const Grid& g, int kx) { return kx == 0 || (g.disc && 2 * kx == g.n1); }

__device__ __forceinline__ bool herm_mode(const Grid& g, int kx, int ky, int z) {
    if (!g.disc) return false;
    if (g.disc == 2) return true;   // staggered grid: coefficients of real fields, no phase carried
    if (kx != 0) return true;
    return is_nyquist(ky, g.n2) != is_nyquist(z, g.n3);
}

template <typename CU>
__device__ __forceinline__ void herm_pair(CU& a, CU& b) {
    // a <- (a + conj b)/2, b <- conj(a_new)
    using TU = decltype(a.x);
    const double ax = 0.5 * (double(a.x) + double(b.x));
    const double ay = 0.5 * (double(a.y) - double(b.y));
    a.x = TU(ax);
    a.y = TU(ay);
    b.x = TU(ax);
    b.y = TU(-ay);
}

template <typename TU>
__device__ __forceinline__ double cg_update_one(const UArgs<TU>& a, long long idx, double alpha, cpx<TU>* rr) {
    using CU = cpx<TU>;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const long long o = i * a.g.nspec + idx;
        CU xi = a.x[o];
        const CU pi = a.p[o];
        CU ri = a.r[o];
        const CU qi = a.q[o];
        const TU al = TU(alpha);   // vector arithmetic in the precision of the CG vectors
        xi.x += al * pi.x;
        xi.y += al * pi.y;
        ri.x -= al * qi.x;
        ri.y -= al * qi.y;
        a.x[o] = xi;
        rr[i] = ri;
    }
    return 0.0;
}

// w Re(r^H K r) at one frequency
template <typename TU>
__device__ __forceinline__ double rkr(const UArgs<TU>& a, const cpx<TU>* rr, const Freq& f) {
    if (f.zero) return 0.0;
    double kr[3], ki[3];
    kmul(f, a.mu0, a.kappa0, rr, kr, ki);
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) t += double(rr[i].x) * kr[i] + double(rr[i].y) * ki[i];
    return f.w * t;
}

// w Re(r^H K r) at one frequency of the staggered grid
template <typename TU>
__device__ __forceinline__ double rkr_stag(const UArgs<TU>& a, const cpx<TU>* rr, const FreqC& f) {
    if (f.zero) return 0.0;
    double kr[3], ki[3];
    kmul_stag(f, a.mu0, a.kappa0, rr, kr, ki);
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) t += double(rr[i].x) * kr[i] + double(rr[i].y) * ki[i];
    return f.w * t;
}

// element e of the half spectrum (e < 2^31): row = z n2 + ky, kx
__device__ __forceinline__ void split_index(const Grid& g, int e, int& z, int& ky, int& kx) {
    const int row = e / g.nh;
    kx = e - row * g.nh;
    z = row / g.n2;
    ky = row - z * g.n2;
}

template <typename TU>
__device__ __forceinline__ void k_cg_update_body(const UArgs<TU>& a, int tile_, int ntiles_) {
    using CU = cpx<TU>;
    if (a.st->done) return;
    __shared__ double red[16];
    const double alpha = a.st->alpha;
    const long long M = (long long)a.g.n2 * a.g.nh;
    const int nspec = (int)a.g.nspec;
    double s = 0.0;
    for (int idx = tile_ * (int)blockDim.x + (int)threadIdx.x; idx < nspec; idx += ntiles_ * (int)blockDim.x) {
        int z, ky, kx;
        split_index(a.g, idx, z, ky, kx);
        const ColFreq cf = col_freq_k(a.g, ky, kx);
        CU r1[3];
        if (!selfconj_plane(a.g, kx)) {
            cg_update_one(a, idx, alpha, r1);
#pragma unroll
            for (int i = 0; i < 3; ++i) a.r[i * a.g.nspec + idx] = r1[i];
            s += (a.g.disc == 2) ? rkr_stag(a, r1, freqc_k(a.g, ky, kx, z)) : rkr(a, r1, freq_z(a.g, cf, z));
            continue;
        }
        const long long idx2 = kx0_partner(a.g, M, z, ky) + kx;
        if (idx2 < idx) continue;   // the partner's thread owns this pair
        const bool herm = herm_mode(a.g, kx, ky, z);
        cg_update_one(a, idx, alpha, r1);
        if (idx2 == idx) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {   // self-conjugate: purely imaginary (anti-Hermitian) or real
                if (herm) r1[i].y = TU(0);
                else r1[i].x = TU(0);
            }
        } else {
            CU r2[3];
            cg_update_one(a, idx2, alpha, r2);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (herm) herm_pair(r1[i], r2[i]);
                else antiherm_pair(r1[i], r2[i]);
                a.r[i * a.g.nspec + idx2] = r2[i];
            }
            const int z2 = (a.g.n3 - z) % a.g.n3, ky2 = (a.g.n2 - ky) % a.g.n2;
            s += (a.g.disc == 2) ? rkr_stag(a, r2, freqc_k(a.g, ky2, kx, z2))
                                 : rkr(a, r2, freq_z(a.g, col_freq_k(a.g, ky2, kx), z2));
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) a.r[i * a.g.nspec + idx] = r1[i];
        s += (a.g.disc == 2) ? rkr_stag(a, r1, freqc_k(a.g, ky, kx, z)) : rkr(a, r1, freq_z(a.g, cf, z));
    }
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) a.partials[tile_] = tot;
}

template <typename TU>
__global__ void __launch_bounds__(kBlock) k_cg_update(UArgs<TU> a) {
    k_cg_update_body<TU>(a, blockIdx.x, gridDim.x);
}

template <typename TU>
__global__ void __launch_bounds__(kBlock) k_cg_update_b(const UArgs<TU>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_cg_update_body<TU>(as[e.rve], e.tile, e.ntiles);
}

// anti-Hermitian projection of the x = 0 plane of the CG vector a.r (right-hand sides)
template <typename TU>
__device__ __forceinline__ void k_antiherm_body(const UArgs<TU>& a, int tile_, int ntiles_) {
    const Grid& g = a.g;
    cpx<TU>* u = a.r;
    const long long M = (long long)g.n2 * g.nh;
    const long long npl = (long long)g.n2 * g.n3;
    const int nplanes = (g.disc && g.n1 > 1 && 2 * (g.nkx - 1) == g.n1) ? 2 : 1;
    for (long long t = (long long)tile_ * blockDim.x + threadIdx.x; t < npl * nplanes;
         t += (long long)ntiles_ * blockDim.x) {
        const int plane = (int)(t / npl);
        const long long tp = t - plane * npl;
        const int kx = plane ? g.nkx - 1 : 0;
        const int z = (int)(tp / g.n2), ky = (int)(tp - (long long)z * g.n2);
        const long long idx = (long long)z * M + (long long)ky * g.nh + kx;
        const long long idx2 = kx0_partner(g, M, z, ky) + kx;
        if (idx2 < idx) continue;
        const bool herm = herm_mode(g, kx, ky, z);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cpx<TU> v = u[i * g.nspec + idx];
            if (idx2 == idx) {
                if (herm) v.y = TU(0);
                else v.x = TU(0);
            } else {
                cpx<TU> w = u[i * g.nspec + idx2];
                if (herm) herm_pair(v, w);
                else antiherm_pair(v, w);
                u[i * g.nspec + idx2] = w;
            }
            u[i * g.nspec + idx] = v;
        }
    }
}

template <typename TU>
__global__ void __launch_bounds__(kBlock) k_antiherm(UArgs<TU> a) {
    k_antiherm_body<TU>(a, blockIdx.x, gridDim.x);
}

template <typename TU>
__global__ void __launch_bounds__(kBlock) k_antiherm_b(const UArgs<TU>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_antiherm_body<TU>(as[e.rve], e.tile, e.ntiles);
}

#if COMBO_IN_PART(COMBO_PART_CG)
// ------------------------------------------------------------------------------
// finalisers: one workgroup, fixed summation order (deterministic)
// ------------------------------------------------------------------------------
__device__ __forceinline__ double ordered_sum(const double* p, int count, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) s += p[i];
    return block_sum(s, sh);
}

__device__ __forceinline__ void finalize_body(int mode, const FinArgs& f) {
    __shared__ double red[16];
    CGState* st = f.st;
    if (mode != FIN_RHS && st->done) return;
    const double s1 = ordered_sum(f.partials, f.count, red);
    double s2 = 0.0;
    if (mode == FIN_RHS) s2 = ordered_sum(f.partials2, f.count, red);
    if (threadIdx.x != 0) return;
    if (mode == FIN_RHS) {
        st->rho0 = s1;
        st->rho = s1;
        st->tol2 = f.tol2;
        st->maxit = f.maxit;
        st->eta2 = s2;
        st->iter = 0;
        st->beta = 0.0;
        st->alpha = 0.0;
        st->status = 0;
        st->done = (s1 > 0.0) ? 0 : 1;
    } else if (mode == FIN_ALPHA) {
        if (s1 != s1) {
            st->status = 1;
            st->done = 1;
        } else if (!(s1 > 0.0)) {   // negative curvature: x keeps the last iterate
            st->status = 3;
            st->done = 1;
        } else {
            st->alpha = st->rho / s1;
        }
    } else {  // FIN_BETA
        st->iter += 1;
        if (!(s1 == s1)) {
            st->status = 1;
            st->done = 1;
        } else if (s1 <= st->tol2 * st->rho0) {
            st->done = 1;
        } else if (st->iter >= st->maxit) {
            st->status = 2;
            st->done = 1;
        }
        st->beta = s1 / st->rho;
        st->rho = s1;
    }
}

__global__ void __launch_bounds__(kBlock) k_finalize(int mode, FinArgs f) { finalize_body(mode, f); }

__global__ void __launch_bounds__(kBlock) k_finalize_b(int mode, const FinArgs* __restrict__ fs) {
    finalize_body(mode, fs[blockIdx.x]);
}

__global__ void __launch_bounds__(kBlock) k_reduce_columns(const double* partials, int rows, int cols, double* out) {
    __shared__ double red[16];
    for (int c = 0; c < cols; ++c) {
        double s = 0.0;
        for (int r = threadIdx.x; r < rows; r += blockDim.x) s += partials[(long long)r * cols + c];
        const double t = block_sum(s, red);
        if (threadIdx.x == 0) out[c] = t;
    }
}
#endif

// ------------------------------------------------------------------------------
// Two-stage register FFT versions of the y and z passes (fft_reg.h): each 1D
// transform is one size-Q DFT per thread straight from global memory, one LDS
// exchange and one size-P DFT per thread, so a component costs two barriers.
// ------------------------------------------------------------------------------
template <int P, int Q, int TX>
constexpr int fft2_threads() { return TX * (P > Q ? P : Q); }

template <int P, int Q, int TX, typename T, int DISC>
__device__ __forceinline__ void k_y2_fwd_body(const YArgs<T>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    using F = Fft2<P, Q, TX>;
    constexpr int L = P * Q;
    if (a.st && a.st->done) return;
    __shared__ C ex[F::exch_elems()];
    __shared__ C tw[L];
    __shared__ T fy[DISC ? 2 * L : 1];   // rotated scheme: D2[L] A2[L]
    const int tid = threadIdx.x;
    const int z = tile_ / a.ntile, kx0 = (tile_ % a.ntile) * TX;
    const int nh = a.g.nh;
    const long long zoff = (long long)z * L * nh;
    for (int i = tid; i < L; i += blockDim.x) tw[i] = a.tw[i];
    if constexpr (DISC) stage_factors<T>(fy, a.g.ftab + 2 * a.g.nh, 2 * L, tid, blockDim.x);
    const bool hasA = tid < F::NA, hasB = tid < F::NB;
    const int tA = tid % TX, j1 = tid / TX, tB = tid % TX, k1 = tid / TX;
    const bool colA = kx0 + tA < nh, colB = kx0 + tB < nh;
    const T xs2 = T(a.g.xs2);
    __syncthreads();
    C acc[P];
    // component c's column, loaded one step ahead so that its loads are in flight
    // during the previous component's transform
    C nx[Q];
    auto load = [&](int c) {
        const C* src = a.in + c * a.g.nspec + zoff + kx0;   // uniform
#pragma unroll
        for (int j2 = 0; j2 < Q; ++j2) nx[j2] = (hasA && colA) ? src[tA + (j1 + P * j2) * nh] : mk<T>(0, 0);
    };
    load(0);
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
#pragma unroll 1
        for (int sub = 0; sub < 3; ++sub) {
            const int c = 3 * i + sub;
            C x[Q];
#pragma unroll
            for (int j2 = 0; j2 < Q; ++j2) x[j2] = nx[j2];
            if (c + 1 < 9) load(c + 1);
            if (hasA) fft2_stageA<P, Q, TX, -1, T>(x, tA, j1, ex, tw);
            __syncthreads();
            if (hasB) {
                C y[P];
                fft2_stageB<P, Q, TX, -1, T>(y, tB, k1, ex);
                if (sub == 0) {
#pragma unroll
                    for (int k2 = 0; k2 < P; ++k2)
                        acc[k2] = (DISC == 1) ? cscale(y[k2], fy[L + k1 + Q * k2]) : y[k2];
                } else if (colB) {
                    const int oc = (sub == 1) ? i : 3 + i;
                    C* dst = a.out + oc * a.g.nspec + zoff + kx0;   // uniform
#pragma unroll
                    for (int k2 = 0; k2 < P; ++k2) {
                        const int ky = k1 + Q * k2;
                        C v = y[k2];
                        if (DISC == 2) {   // staggered grid: times conj(f_2)
                            if (sub == 1) v = cadd(acc[k2], cmul(v, mk<T>(fy[ky], -fy[L + ky])));
                        } else {
                            if (sub == 1) v = cadd(acc[k2], cscale(v, DISC ? fy[ky] : xs2 * T(freq_of(ky, L))));
                            else if (DISC) v = cscale(v, fy[L + ky]);
                        }
                        dst[tB + ky * nh] = v;
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <int P, int Q, int TX, typename T, int DISC>
__global__ void __launch_bounds__((fft2_threads<P, Q, TX>())) k_y2_fwd(YArgs<T> a) {
    k_y2_fwd_body<P, Q, TX, T, DISC>(a, blockIdx.x, gridDim.x);
}

template <int P, int Q, int TX, typename T, int DISC>
__global__ void __launch_bounds__((fft2_threads<P, Q, TX>())) k_y2_fwd_b(const YArgs<T>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_y2_fwd_body<P, Q, TX, T, DISC>(as[e.rve], e.tile, e.ntiles);
}

template <int P, int Q, int TX, typename T, int DISC>
__device__ __forceinline__ void k_y2_inv_body(const YArgs<T>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    using F = Fft2<P, Q, TX>;
    constexpr int L = P * Q;
    if (a.st && a.st->done) return;
    __shared__ C ex[F::exch_elems()];
    __shared__ C tw[L];
    __shared__ T fy[DISC ? 2 * L : 1];   // rotated scheme: D2[L] A2[L]
    const int tid = threadIdx.x;
    const int z = tile_ / a.ntile, kx0 = (tile_ % a.ntile) * TX;
    const int nh = a.g.nh;
    const long long zoff = (long long)z * L * nh;
    for (int i = tid; i < L; i += blockDim.x) tw[i] = a.tw[i];
    if constexpr (DISC) stage_factors<T>(fy, a.g.ftab + 2 * a.g.nh, 2 * L, tid, blockDim.x);
    const bool hasA = tid < F::NA, hasB = tid < F::NB;
    const int tA = tid % TX, j1 = tid / TX, tB = tid % TX, k1 = tid / TX;
    const bool colA = kx0 + tA < nh, colB = kx0 + tB < nh;
    const T xs2 = T(a.g.xs2);
    __syncthreads();
    // step 3 i + sub reads component (sub == 2 ? 3 + i : i), one step ahead
    C nx[Q];
    auto load = [&](int step) {
        const int i = step / 3, sub = step - 3 * i;
        const C* src = a.in + (sub == 2 ? 3 + i : i) * a.g.nspec + zoff + kx0;   // uniform
#pragma unroll
        for (int j2 = 0; j2 < Q; ++j2) nx[j2] = (hasA && colA) ? src[tA + (j1 + P * j2) * nh] : mk<T>(0, 0);
    };
    load(0);
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
#pragma unroll 1
        for (int sub = 0; sub < 3; ++sub) {
            // sub 0: A_i, sub 1: xi_2 A_i (A_i re-read, normally from L2), sub 2: B_i
            C x[Q];
#pragma unroll
            for (int j2 = 0; j2 < Q; ++j2) {
                const int y = j1 + P * j2;
                if (DISC == 2) x[j2] = (sub == 1) ? cmul(nx[j2], mk<T>(fy[y], fy[L + y])) : nx[j2];
                else if (DISC) x[j2] = cscale(nx[j2], fy[sub == 1 ? y : L + y]);
                else x[j2] = (sub == 1) ? cscale(nx[j2], xs2 * T(freq_of(y, L))) : nx[j2];
            }
            if (3 * i + sub + 1 < 9) load(3 * i + sub + 1);
            if (hasA) fft2_stageA<P, Q, TX, +1, T>(x, tA, j1, ex, tw);
            __syncthreads();
            if (hasB && colB) {
                C y[P];
                fft2_stageB<P, Q, TX, +1, T>(y, tB, k1, ex);
                C* dst = a.out + (3 * i + sub) * a.g.nspec + zoff + kx0;   // uniform
#pragma unroll
                for (int k2 = 0; k2 < P; ++k2) dst[tB + (k1 + Q * k2) * nh] = y[k2];
            }
            __syncthreads();
        }
    }
}

template <int P, int Q, int TX, typename T, int DISC>
__global__ void __launch_bounds__((fft2_threads<P, Q, TX>())) k_y2_inv(YArgs<T> a) {
    k_y2_inv_body<P, Q, TX, T, DISC>(a, blockIdx.x, gridDim.x);
}

template <int P, int Q, int TX, typename T, int DISC>
__global__ void __launch_bounds__((fft2_threads<P, Q, TX>())) k_y2_inv_b(const YArgs<T>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_y2_inv_body<P, Q, TX, T, DISC>(as[e.rve], e.tile, e.ntiles);
}

template <int P, int Q, int TX, typename T, typename TU, int MODE, int DISC>
__device__ __forceinline__ void k_z2_fwd_body(const ZArgs<T, TU>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    using F = Fft2<P, Q, TX>;
    constexpr int L = P * Q;
    if (MODE == Z_CG && a.st->done) return;
    __shared__ C ex[F::exch_elems()];
    __shared__ C tw[L];
    __shared__ T fz[DISC ? 2 * L : 1];   // rotated scheme: D3[L] A3[L]
    __shared__ double red[16];
    const int tid = threadIdx.x;
    const long long M = (long long)a.g.n2 * a.g.nh;
    const long long m0 = (long long)tile_ * TX;
    for (int i = tid; i < L; i += blockDim.x) tw[i] = a.tw[i];
    if constexpr (DISC) stage_factors<T>(fz, a.g.ftab + 2 * a.g.nh + 2 * a.g.n2, 2 * L, tid, blockDim.x);
    const bool hasA = tid < F::NA, hasB = tid < F::NB;
    const int tA = tid % TX, j1 = tid / TX, tB = tid % TX, k1 = tid / TX;
    const bool colA = m0 + tA < M, colB = m0 + tB < M;
    const T xs3 = T(a.g.xs3);
    __syncthreads();
    C v[3][P];
    // step 2 i + sub reads component (sub ? 3 + i : i), one step ahead
    C nx[Q];
    auto load = [&](int step) {
        const int c = (step & 1) ? 3 + (step >> 1) : (step >> 1);
        const C* src = a.in + c * a.g.nspec + m0;   // uniform
        const int Mi = (int)M;
#pragma unroll
        for (int j2 = 0; j2 < Q; ++j2) nx[j2] = (hasA && colA) ? src[tA + (j1 + P * j2) * Mi] : mk<T>(0, 0);
    };
    load(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll 1
        for (int sub = 0; sub < 2; ++sub) {
            C x[Q];
#pragma unroll
            for (int j2 = 0; j2 < Q; ++j2) x[j2] = nx[j2];
            if (2 * i + sub + 1 < 6) load(2 * i + sub + 1);
            if (hasA) fft2_stageA<P, Q, TX, -1, T>(x, tA, j1, ex, tw);
            __syncthreads();
            if (hasB) {
                C y[P];
                fft2_stageB<P, Q, TX, -1, T>(y, tB, k1, ex);
#pragma unroll
                for (int k2 = 0; k2 < P; ++k2) {
                    const int zz = k1 + Q * k2;
                    if constexpr (DISC == 2) {   // staggered grid: times conj(f_3)
                        if (sub == 0) v[i][k2] = y[k2];
                        else v[i][k2] = cadd(v[i][k2], cmul(y[k2], mk<T>(fz[zz], -fz[L + zz])));
                    } else if constexpr (DISC) {
                        if (sub == 0) v[i][k2] = cscale(y[k2], fz[L + zz]);
                        else v[i][k2] = cadd(v[i][k2], cscale(y[k2], fz[zz]));
                    } else {
                        if (sub == 0) v[i][k2] = y[k2];
                        else v[i][k2] = cadd(v[i][k2], cscale(y[k2], xs3 * T(freq_of(zz, L))));
                    }
                }
            }
            __syncthreads();
        }
    }
    double s1 = 0.0, s2 = 0.0;
    if (hasB && colB) {
        if constexpr (DISC == 2) {
            const int m = (int)(m0 + tB), ky = m / a.g.nh, kx = m - ky * a.g.nh;   // one column per thread
#pragma unroll
            for (int k2 = 0; k2 < P; ++k2) {
                const int zz = k1 + Q * k2;
                C vv[3] = {v[0][k2], v[1][k2], v[2][k2]};
                z_epilogue_stag<T, TU, MODE>(a, freqc_k(a.g, ky, kx, zz), (long long)zz * M + m, vv, s1, s2);
            }
        } else if constexpr (DISC) {
            const int m = (int)(m0 + tB), ky = m / a.g.nh, kx = m - ky * a.g.nh;   // one column per thread
            const ColFreq cf = col_freq_rot(a.g, ky, kx);
#pragma unroll
            for (int k2 = 0; k2 < P; ++k2) {
                const int zz = k1 + Q * k2;
                C vv[3] = {v[0][k2], v[1][k2], v[2][k2]};
                const Freq f = freq_z_rot(cf, double(fz[L + zz]), double(fz[zz]));
                z_epilogue<T, TU, MODE>(a, f, (long long)zz * M + m, vv, s1, s2);
            }
        } else {
            const ColFreq cf = col_freq(a.g, (int)(m0 + tB));   // one column per thread
#pragma unroll
            for (int k2 = 0; k2 < P; ++k2) {
                C vv[3] = {v[0][k2], v[1][k2], v[2][k2]};
                z_epilogue_at<T, TU, MODE>(a, cf, m0 + tB, k1 + Q * k2, vv, s1, s2);
            }
        }
    }
    if (MODE == Z_CG || MODE == Z_RHS) {
        const double t1 = block_sum(s1, red);
        if (tid == 0) a.partials[tile_] = t1;
    }
    if (MODE == Z_RHS) {
        const double t2 = block_sum(s2, red);
        if (tid == 0) a.partials2[tile_] = t2;
    }
}

template <int P, int Q, int TX, typename T, typename TU, int MODE, int DISC>
__global__ void __launch_bounds__((fft2_threads<P, Q, TX>())) k_z2_fwd(ZArgs<T, TU> a) {
    k_z2_fwd_body<P, Q, TX, T, TU, MODE, DISC>(a, blockIdx.x, gridDim.x);
}

template <int P, int Q, int TX, typename T, typename TU, int MODE, int DISC>
__global__ void __launch_bounds__((fft2_threads<P, Q, TX>())) k_z2_fwd_b(const ZArgs<T, TU>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_z2_fwd_body<P, Q, TX, T, TU, MODE, DISC>(as[e.rve], e.tile, e.ntiles);
}

template <int P, int Q, int TX, typename T, typename TU, int MODE, int DISC>
__device__ __forceinline__ void k_z2_inv_body(const ZArgs<T, TU>& a, int tile_, int ntiles_) {
    using C = cpx<T>;
    using CU = cpx<TU>;
    using F = Fft2<P, Q, TX>;
    constexpr int L = P * Q;
    if (MODE == Z_INV_CG && a.st->done) return;
    __shared__ C ex[F::exch_elems()];
    __shared__ C tw[L];
    __shared__ T fz[DISC ? 2 * L : 1];   // rotated scheme: D3[L] A3[L]
    const int tid = threadIdx.x;
    const long long M = (long long)a.g.n2 * a.g.nh;
    const long long m0 = (long long)tile_ * TX;
    for (int i = tid; i < L; i += blockDim.x) tw[i] = a.tw[i];
    if constexpr (DISC) stage_factors<T>(fz, a.g.ftab + 2 * a.g.nh + 2 * a.g.n2, 2 * L, tid, blockDim.x);
    const bool hasA = tid < F::NA, hasB = tid < F::NB;
    const int tA = tid % TX, j1 = tid / TX, tB = tid % TX, k1 = tid / TX;
    const bool colA = m0 + tA < M, colB = m0 + tB < M;
    const T xs3 = T(a.g.xs3);
    double beta = 0.0;
    bool first = true;
    if (MODE == Z_INV_CG) {
        beta = a.st->beta;
        first = (a.st->iter == 0);
    }
    __syncthreads();
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
        // u_i is read once (CG mode: p = r + beta p, written back) and kept for the xi_3 u_i transform
        C u[Q];
        if (hasA) {
            const long long base = i * a.g.nspec + m0;   // uniform
            CU* pb = a.p + base;
            const CU* rb = a.r + base;
            const CU* xb = a.x + base;
            const int Mi = (int)M;
#pragma unroll
            for (int j2 = 0; j2 < Q; ++j2) {
                u[j2] = mk<T>(0, 0);
                if (!colA) continue;
                const int off = tA + (j1 + P * j2) * Mi;
                if (MODE == Z_INV_CG) {
                    const CU ri = rb[off];
                    CU pn;
                    if (first) {
                        pn = ri;
                    } else {
                        const CU pi = pb[off];
                        pn.x = ri.x + TU(beta) * pi.x;
                        pn.y = ri.y + TU(beta) * pi.y;
                    }
                    pb[off] = pn;
                    u[j2] = mk<T>(T(pn.x), T(pn.y));
                } else {
                    const CU xi = xb[off];
                    u[j2] = mk<T>(T(xi.x), T(xi.y));
                }
            }
        }
#pragma unroll 1
        for (int sub = 0; sub < 2; ++sub) {
            if (hasA) {
                C x[Q];
#pragma unroll
                for (int j2 = 0; j2 < Q; ++j2) {
                    const int zz = j1 + P * j2;
                    if (DISC == 2) x[j2] = sub ? cmul(u[j2], mk<T>(fz[zz], fz[L + zz])) : u[j2];
                    else if (DISC) x[j2] = cscale(u[j2], fz[sub ? zz : L + zz]);
                    else x[j2] = sub ? cscale(u[j2], xs3 * T(freq_of(zz, L))) : u[j2];
                }
                fft2_stageA<P, Q, TX, +1, T>(x, tA, j1, ex, tw);
            }
            __syncthreads();
            if (hasB && colB) {
                C y[P];
                fft2_stageB<P, Q, TX, +1, T>(y, tB, k1, ex);
                C* dst = a.out + (sub ? 3 + i : i) * a.g.nspec + m0;   // uniform
                const int Mi = (int)M;
#pragma unroll
                for (int k2 = 0; k2 < P; ++k2) dst[tB + (k1 + Q * k2) * Mi] = y[k2];
            }
            __syncthreads();
        }
    }
}

template <int P, int Q, int TX, typename T, typename TU, int MODE, int DISC>
__global__ void __launch_bounds__((fft2_threads<P, Q, TX>())) k_z2_inv(ZArgs<T, TU> a) {
    k_z2_inv_body<P, Q, TX, T, TU, MODE, DISC>(a, blockIdx.x, gridDim.x);
}

template <int P, int Q, int TX, typename T, typename TU, int MODE, int DISC>
__global__ void __launch_bounds__((fft2_threads<P, Q, TX>())) k_z2_inv_b(const ZArgs<T, TU>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_z2_inv_body<P, Q, TX, T, TU, MODE, DISC>(as[e.rve], e.tile, e.ntiles);
}

// Supported fast-path lengths: (P, Q, TX) per precision; TX keeps the exchange
// buffer near 35 KB so four workgroups fit in the 160 KB LDS of a CU.
// two-stage y/z configurations: element type, length, P, Q, tile width TX, variant.
// Variant 0 is the default; the others are candidates of the autotuner (float,
// the precision of the CG passes in mixed mode).
#define COMBO_FFT2_CONFIGS(X)           \
    X(float, 256, 16, 16, 16, 0)        \
    X(float, 256, 16, 16, 8, 1)         \
    X(float, 192, 16, 12, 16, 0)        \
    X(float, 192, 12, 16, 16, 1)        \
    X(float, 128, 8, 16, 16, 0)         \
    X(float, 128, 16, 8, 16, 1)         \
    X(float, 96, 8, 12, 16, 0)          \
    X(float, 96, 12, 8, 16, 1)          \
    X(float, 64, 8, 8, 32, 0)           \
    X(float, 64, 8, 8, 16, 1)           \
    X(float, 48, 8, 6, 24, 0)           \
    X(float, 48, 6, 8, 24, 1)           \
    X(float, 32, 4, 8, 32, 0)           \
    X(float, 32, 8, 4, 32, 1)           \
    X(double, 256, 16, 16, 8, 0)        \
    X(double, 192, 16, 12, 8, 0)        \
    X(double, 128, 8, 16, 8, 0)         \
    X(double, 96, 8, 12, 16, 0)         \
    X(double, 64, 8, 8, 16, 0)          \
    X(double, 48, 8, 6, 24, 0)          \
    X(double, 32, 4, 8, 16, 0)

// variants of the two-stage y/z pass for rows of L (0: none, slow LDS path)
template <typename T>
int fft2_variants(int L) {
    int n = 0;
#define COMBO_NV_CASE(TT, LL, PP, QQ, TXX, VV) \
    if (std::is_same<T, TT>::value && L == LL) ++n;
    COMBO_FFT2_CONFIGS(COMBO_NV_CASE)
#undef COMBO_NV_CASE
    return n;
}

// the variant that runs for a requested one (unknown variants fall back to 0)
template <typename T>
int fft2_pick(int L, int v) { return (v > 0 && v < fft2_variants<T>(L)) ? v : 0; }

template <typename T>
int fft2_tx(int L, int v) {
    const int vv = fft2_pick<T>(L, v);
#define COMBO_TX_CASE(TT, LL, PP, QQ, TXX, VV) \
    if (std::is_same<T, TT>::value && L == LL && vv == VV) return TXX;
    COMBO_FFT2_CONFIGS(COMBO_TX_CASE)
#undef COMBO_TX_CASE
    return 0;
}

template <typename T>
int y_tile(const Grid& g) {
    const int tx = fft2_tx<T>(g.n2, g.yv);
    if (tx) return tx;
    return std::max(1, std::min(g.nh, max_elems<T>() / g.n2));
}

template <typename T>
int z_tile(const Grid& g) {
    const int tx = fft2_tx<T>(g.n3, g.zv);
    if (tx) return tx;
    return (int)std::max<long long>(1, std::min<long long>((long long)g.n2 * g.nh, max_elems<T>() / g.n3));
}

#if COMBO_IN_PART(COMBO_PART_CG)
template int y_tile<float>(const Grid&);
template int y_tile<double>(const Grid&);
template int z_tile<float>(const Grid&);
template int z_tile<double>(const Grid&);
template int fft2_variants<float>(int);
template int fft2_variants<double>(int);

// ------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------
void xpass_wave_shape(int n1, int& m, int& w) {
    m = w = 0;
#define COMBO_XS_CASE(LL, MM, WW) \
    if (n1 == LL) {                \
        m = MM;                    \
        w = WW;                    \
        return;                    \
    }
    COMBO_XWAVE_CONFIGS(COMBO_XS_CASE)
#undef COMBO_XS_CASE
}

int xpass_lds_variants(int n1) {
    int n = 0;
#define COMBO_XNV_CASE(LL, PP, QQ, RR, VV) \
    if (n1 == LL) ++n;
    COMBO_XLDS_CONFIGS(COMBO_XNV_CASE)
#undef COMBO_XNV_CASE
    return n;
}

// variant that runs for a requested one: double has variant 0 only
int xpass_lds_pick(int n1, int v, bool is_float) {
    return (is_float && v > 0 && v < xpass_lds_variants(n1)) ? v : 0;
}

int xpass_lds_rows(int n1, int v, bool is_float) {
    const int vv = xpass_lds_pick(n1, v, is_float);
#define COMBO_XLR_CASE(LL, PP, QQ, RR, VV) \
    if (n1 == LL && vv == VV) return XLdsShape<PP, QQ, RR>::R;
    COMBO_XLDS_CONFIGS(COMBO_XLR_CASE)
#undef COMBO_XLR_CASE
    return 0;
}

int blocks_x(const Grid& g, int R, int mode, bool is_float) {
    const long long nrows = (long long)g.n2 * g.n3;
    if (mode == X_CG || mode == X_AVG) {
        const int rows = xpass_lds_rows(g.n1, g.xv, is_float);
        if (rows > 0) return (int)((nrows + rows - 1) / rows);
    }
    if (g.disc) return (int)((nrows + R - 1) / R);   // the rotated scheme has no wavefront x pass
#define COMBO_XB_CASE(LL, MM, WW) \
    if (g.n1 == LL) return (int)((nrows + (256 / WW) - 1) / (256 / WW));
    COMBO_XWAVE_CONFIGS(COMBO_XB_CASE)
#undef COMBO_XB_CASE
    return (int)((nrows + R - 1) / R);
}
int blocks_y(const Grid& g, int TX) { return g.n3 * ((g.nh + TX - 1) / TX); }
int blocks_z(const Grid& g, int TX) { return (int)(((long long)g.n2 * g.nh + TX - 1) / TX); }
int blocks_u(const Grid& g) {
    long long b = (g.nspec + kBlock - 1) / kBlock;
    return (int)(b < 4096 ? b : 4096);
}

#endif  // host helpers

#define COMBO_UNPAREN(...) __VA_ARGS__
// launch KNAME<TARGS> with the argument block `a`, or its batched twin KNAME_b<TARGS>
// over the tile map of `b` (KARGS_T: the argument block type, one token)
#define COMBO_LAUNCH(KNAME, TARGS, KARGS_T, GRID, BLOCK, LDS)                                                    \
    do {                                                                                                      \
        if (b) {                                                                                              \
            hipLaunchKernelGGL((KNAME##_b<COMBO_UNPAREN TARGS>), dim3(b->nblocks), dim3(BLOCK), LDS, s,       \
                               static_cast<const KARGS_T*>(b->args), b->map);                                 \
        } else {                                                                                              \
            hipLaunchKernelGGL((KNAME<COMBO_UNPAREN TARGS>), dim3(GRID), dim3(BLOCK), LDS, s, a);             \
        }                                                                                                     \
    } while (0)

#if COMBO_IN_PART(COMBO_PART_XF) || COMBO_IN_PART(COMBO_PART_XD)
template <typename T>
hipError_t launch_x(int mode, const XArgs<T>& a, hipStream_t s, int* nb, const BatchLaunch* b) {
    using XA = XArgs<T>;
    const long long nrows = (long long)a.g.n2 * a.g.n3;
    // the staggered grid transforms real fields only (its tangent action is a separate stencil)
    if (a.g.disc == 2 && mode != X_FWD_REAL && mode != X_INV_REAL) return hipErrorInvalidValue;
    if (a.g.disc == 2 && (a.real_in_t || a.real_out_t)) {   // real fields in the pass's precision: two-stage kernel
#define COMBO_XS_CASE(LL, PP, QQ, RR, VV)                                                                    \
        if constexpr (VV == 0) {                                                                             \
            if (a.g.n1 == LL) {                                                                              \
                using SH = XLdsShape<PP, QQ, RR>;                                                            \
                const int nblk = (int)((nrows + SH::R - 1) / SH::R);                                         \
                if (nb) *nb = nblk;                                                                          \
                if (mode == X_INV_REAL) COMBO_LAUNCH(k_xlds, (T, X_INV_REAL, PP, QQ, RR, 2), XA, nblk, SH::NTH, 0); \
                else COMBO_LAUNCH(k_xlds, (T, X_FWD_REAL, PP, QQ, RR, 2), XA, nblk, SH::NTH, 0);             \
                return hipGetLastError();                                                                    \
            }                                                                                                \
        }
        COMBO_XLDS_CONFIGS(COMBO_XS_CASE)
#undef COMBO_XS_CASE
    }
    if (a.g.disc != 2 && (mode == X_CG || mode == X_AVG)) {
        const int vv = xpass_lds_pick(a.g.n1, a.g.xv, std::is_same<T, float>::value);
#define COMBO_XL_CASE(LL, PP, QQ, RR, VV)                                                                    \
        if constexpr (VV == 0 || std::is_same<T, float>::value) {                                            \
            if (a.g.n1 == LL && vv == VV) {                                                                  \
                using SH = XLdsShape<PP, QQ, RR>;                                                            \
                const int nblk = (int)((nrows + SH::R - 1) / SH::R);                                         \
                if (nb) *nb = nblk;                                                                          \
                if (a.g.disc) {                                                                              \
                    if (mode == X_CG) COMBO_LAUNCH(k_xlds, (T, X_CG, PP, QQ, RR, 1), XA, nblk, SH::NTH, 0);  \
                    else COMBO_LAUNCH(k_xlds, (T, X_AVG, PP, QQ, RR, 1), XA, nblk, SH::NTH, 0);              \
                } else {                                                                                     \
                    if (mode == X_CG) COMBO_LAUNCH(k_xlds, (T, X_CG, PP, QQ, RR, 0), XA, nblk, SH::NTH, 0);  \
                    else COMBO_LAUNCH(k_xlds, (T, X_AVG, PP, QQ, RR, 0), XA, nblk, SH::NTH, 0);              \
                }                                                                                            \
                return hipGetLastError();                                                                    \
            }                                                                                                \
        }
        COMBO_XLDS_CONFIGS(COMBO_XL_CASE)
#undef COMBO_XL_CASE
    }
#define COMBO_XW_CASE(LL, MM, WW)                                                                             \
    if (!a.g.disc && a.g.n1 == LL) {                                                                        \
        const int nblk = (int)((nrows + (256 / WW) - 1) / (256 / WW));                                       \
        if (nb) *nb = nblk;                                                                                  \
        switch (mode) {                                                                                      \
            case X_CG: COMBO_LAUNCH(k_xwave, (T, X_CG, MM, WW), XA, nblk, 256, 0); break;               \
            case X_RHS_E: COMBO_LAUNCH(k_xwave, (T, X_RHS_E, MM, WW), XA, nblk, 256, 0); break;         \
            case X_AVG: COMBO_LAUNCH(k_xwave, (T, X_AVG, MM, WW), XA, nblk, 256, 0); break;             \
            case X_FWD_REAL: COMBO_LAUNCH(k_xwave, (T, X_FWD_REAL, MM, WW), XA, nblk, 256, 0); break;   \
            default: COMBO_LAUNCH(k_xwave, (T, X_INV_REAL, MM, WW), XA, nblk, 256, 0); break;           \
        }                                                                                                    \
        return hipGetLastError();                                                                            \
    }
    COMBO_XWAVE_CONFIGS(COMBO_XW_CASE)
#undef COMBO_XW_CASE
    if ((long long)5 * a.R * a.g.n1 > xpass_cap<T>()) return hipErrorInvalidValue;   // rows beyond the pass's capacity
    const int nblk = blocks_x(a.g, a.R, X_FWD_REAL, std::is_same<T, float>::value);
    if (nb) *nb = nblk;
    const size_t lds = sizeof(cpx<T>) * ((size_t)a.g.n1 + (size_t)5 * a.R * a.g.n1);
    switch (mode) {
        case X_CG: COMBO_LAUNCH(k_xpass, (T, X_CG), XA, nblk, kBlock, lds); break;
        case X_RHS_E: COMBO_LAUNCH(k_xpass, (T, X_RHS_E), XA, nblk, kBlock, lds); break;
        case X_AVG: COMBO_LAUNCH(k_xpass, (T, X_AVG), XA, nblk, kBlock, lds); break;
        case X_FWD_REAL: COMBO_LAUNCH(k_xpass, (T, X_FWD_REAL), XA, nblk, kBlock, lds); break;
        default: COMBO_LAUNCH(k_xpass, (T, X_INV_REAL), XA, nblk, kBlock, lds); break;
    }
    return hipGetLastError();
}

#endif

#if COMBO_IN_PART(COMBO_PART_Y)
// y and z launchers: the caller's TX/ntile are replaced by the tile width of the
// kernel that runs (two-stage fast path or LDS Stockham)
template <typename T>
void y_fill_tiles(YArgs<T>& a) {
    a.TX = y_tile<T>(a.g);
    a.ntile = (a.g.nh + a.TX - 1) / a.TX;
}

template <typename T>
hipError_t launch_y(int dir, const YArgs<T>& a0, hipStream_t s, const BatchLaunch* b) {
    using YA = YArgs<T>;
    YArgs<T> a = a0;
    y_fill_tiles(a);
    const int nblk = a.g.n3 * a.ntile;
    const int vv = fft2_pick<T>(a.g.n2, a.g.yv);
#define COMBO_Y_CASE(TT, LL, PP, QQ, TXX, VV)                                                                   \
    if constexpr (std::is_same<T, TT>::value) {                                                               \
        if (a.g.n2 == LL && vv == VV) {                                                                        \
            constexpr int nt = fft2_threads<PP, QQ, TXX>();                                                    \
            if (dir < 0 && a.g.disc == 2) COMBO_LAUNCH(k_y2_fwd, (PP, QQ, TXX, T, 2), YA, nblk, nt, 0);  \
            else if (dir > 0 && a.g.disc == 2) COMBO_LAUNCH(k_y2_inv, (PP, QQ, TXX, T, 2), YA, nblk, nt, 0); \
            else if (dir < 0 && a.g.disc) COMBO_LAUNCH(k_y2_fwd, (PP, QQ, TXX, T, 1), YA, nblk, nt, 0);  \
            else if (dir < 0) COMBO_LAUNCH(k_y2_fwd, (PP, QQ, TXX, T, 0), YA, nblk, nt, 0);              \
            else if (a.g.disc) COMBO_LAUNCH(k_y2_inv, (PP, QQ, TXX, T, 1), YA, nblk, nt, 0);             \
            else COMBO_LAUNCH(k_y2_inv, (PP, QQ, TXX, T, 0), YA, nblk, nt, 0);                           \
            return hipGetLastError();                                                                          \
        }                                                                                                      \
    }
    COMBO_FFT2_CONFIGS(COMBO_Y_CASE)
#undef COMBO_Y_CASE
    const size_t lds = sizeof(cpx<T>) * ((size_t)a.g.n2 + (size_t)a.g.n2 * a.TX);
    if (a.g.disc == 2) {   // staggered grid without a two-stage pass: LDS Stockham with complex multipliers
        if (dir < 0) COMBO_LAUNCH(k_ypass_fwd, (T, 2), YA, nblk, kBlock, lds);
        else COMBO_LAUNCH(k_ypass_inv, (T, 2), YA, nblk, kBlock, lds);
        return hipGetLastError();
    }
    if (dir < 0 && a.g.disc) COMBO_LAUNCH(k_ypass_fwd, (T, 1), YA, nblk, kBlock, lds);
    else if (dir < 0) COMBO_LAUNCH(k_ypass_fwd, (T, 0), YA, nblk, kBlock, lds);
    else if (a.g.disc) COMBO_LAUNCH(k_ypass_inv, (T, 1), YA, nblk, kBlock, lds);
    else COMBO_LAUNCH(k_ypass_inv, (T, 0), YA, nblk, kBlock, lds);
    return hipGetLastError();
}

#endif

#if COMBO_IN_PART(COMBO_PART_ZF) || COMBO_IN_PART(COMBO_PART_ZD)
template <typename T, typename TU>
hipError_t launch_z(int mode, const ZArgs<T, TU>& a0, hipStream_t s, int* nb, const BatchLaunch* b) {
    using ZA = ZArgs<T, TU>;
    ZArgs<T, TU> a = a0;
    a.TX = z_tile<T>(a.g);
    const int nblk = blocks_z(a.g, a.TX);
    if (nb) *nb = nblk;
    const int vv = fft2_pick<T>(a.g.n3, a.g.zv);
#define COMBO_Z_CASE(TT, LL, PP, QQ, TXX, VV)                                                                  \
    if constexpr (std::is_same<T, TT>::value) {                                                              \
        if (a.g.n3 == LL && vv == VV) {                                                                       \
            constexpr int nt = fft2_threads<PP, QQ, TXX>();                                                   \
            switch (mode) {                                                                                   \
                case Z_CG:                                                                                    \
                    if (a.g.disc == 2) COMBO_LAUNCH(k_z2_fwd, (PP, QQ, TXX, T, TU, Z_CG, 2), ZA, nblk, nt, 0);  \
                    else if (a.g.disc) COMBO_LAUNCH(k_z2_fwd, (PP, QQ, TXX, T, TU, Z_CG, 1), ZA, nblk, nt, 0);     \
                    else COMBO_LAUNCH(k_z2_fwd, (PP, QQ, TXX, T, TU, Z_CG, 0), ZA, nblk, nt, 0);              \
                    break;                                                                                    \
                case Z_RHS:                                                                                   \
                    if (a.g.disc == 2) COMBO_LAUNCH(k_z2_fwd, (PP, QQ, TXX, T, TU, Z_RHS, 2), ZA, nblk, nt, 0);  \
                    else if (a.g.disc) COMBO_LAUNCH(k_z2_fwd, (PP, QQ, TXX, T, TU, Z_RHS, 1), ZA, nblk, nt, 0);    \
                    else COMBO_LAUNCH(k_z2_fwd, (PP, QQ, TXX, T, TU, Z_RHS, 0), ZA, nblk, nt, 0);             \
                    break;                                                                                    \
                case Z_PROJ:                                                                                  \
                    if (a.g.disc == 2) COMBO_LAUNCH(k_z2_fwd, (PP, QQ, TXX, T, TU, Z_PROJ, 2), ZA, nblk, nt, 0);  \
                    else if (a.g.disc) COMBO_LAUNCH(k_z2_fwd, (PP, QQ, TXX, T, TU, Z_PROJ, 1), ZA, nblk, nt, 0);   \
                    else COMBO_LAUNCH(k_z2_fwd, (PP, QQ, TXX, T, TU, Z_PROJ, 0), ZA, nblk, nt, 0);            \
                    break;                                                                                    \
                case Z_INV_CG:                                                                                \
                    if (a.g.disc == 2) COMBO_LAUNCH(k_z2_inv, (PP, QQ, TXX, T, TU, Z_INV_CG, 2), ZA, nblk, nt, 0);  \
                    else if (a.g.disc) COMBO_LAUNCH(k_z2_inv, (PP, QQ, TXX, T, TU, Z_INV_CG, 1), ZA, nblk, nt, 0); \
                    else COMBO_LAUNCH(k_z2_inv, (PP, QQ, TXX, T, TU, Z_INV_CG, 0), ZA, nblk, nt, 0);          \
                    break;                                                                                    \
                default:                                                                                      \
                    if (a.g.disc == 2) COMBO_LAUNCH(k_z2_inv, (PP, QQ, TXX, T, TU, Z_INV_PLAIN, 2), ZA, nblk, nt, 0);  \
                    else if (a.g.disc) COMBO_LAUNCH(k_z2_inv, (PP, QQ, TXX, T, TU, Z_INV_PLAIN, 1), ZA, nblk, nt, 0); \
                    else COMBO_LAUNCH(k_z2_inv, (PP, QQ, TXX, T, TU, Z_INV_PLAIN, 0), ZA, nblk, nt, 0);       \
                    break;                                                                                    \
            }                                                                                                 \
            return hipGetLastError();                                                                         \
        }                                                                                                     \
    }
    COMBO_FFT2_CONFIGS(COMBO_Z_CASE)
#undef COMBO_Z_CASE
    const size_t lds = sizeof(cpx<T>) * ((size_t)a.g.n3 + (size_t)a.g.n3 * a.TX);
    if (a.g.disc == 2) {   // staggered grid without a two-stage pass: LDS Stockham with complex multipliers
        switch (mode) {
            case Z_CG: COMBO_LAUNCH(k_zpass_fwd, (T, TU, Z_CG, 2), ZA, nblk, kBlock, lds); break;
            case Z_RHS: COMBO_LAUNCH(k_zpass_fwd, (T, TU, Z_RHS, 2), ZA, nblk, kBlock, lds); break;
            case Z_PROJ: COMBO_LAUNCH(k_zpass_fwd, (T, TU, Z_PROJ, 2), ZA, nblk, kBlock, lds); break;
            case Z_INV_CG: COMBO_LAUNCH(k_zpass_inv, (T, TU, Z_INV_CG, 2), ZA, nblk, kBlock, lds); break;
            default: COMBO_LAUNCH(k_zpass_inv, (T, TU, Z_INV_PLAIN, 2), ZA, nblk, kBlock, lds); break;
        }
        return hipGetLastError();
    }
    if (a.g.disc) {
        switch (mode) {
            case Z_CG: COMBO_LAUNCH(k_zpass_fwd, (T, TU, Z_CG, 1), ZA, nblk, kBlock, lds); break;
            case Z_RHS: COMBO_LAUNCH(k_zpass_fwd, (T, TU, Z_RHS, 1), ZA, nblk, kBlock, lds); break;
            case Z_PROJ: COMBO_LAUNCH(k_zpass_fwd, (T, TU, Z_PROJ, 1), ZA, nblk, kBlock, lds); break;
            case Z_INV_CG: COMBO_LAUNCH(k_zpass_inv, (T, TU, Z_INV_CG, 1), ZA, nblk, kBlock, lds); break;
            default: COMBO_LAUNCH(k_zpass_inv, (T, TU, Z_INV_PLAIN, 1), ZA, nblk, kBlock, lds); break;
        }
        return hipGetLastError();
    }
    switch (mode) {
        case Z_CG: COMBO_LAUNCH(k_zpass_fwd, (T, TU, Z_CG, 0), ZA, nblk, kBlock, lds); break;
        case Z_RHS: COMBO_LAUNCH(k_zpass_fwd, (T, TU, Z_RHS, 0), ZA, nblk, kBlock, lds); break;
        case Z_PROJ: COMBO_LAUNCH(k_zpass_fwd, (T, TU, Z_PROJ, 0), ZA, nblk, kBlock, lds); break;
        case Z_INV_CG: COMBO_LAUNCH(k_zpass_inv, (T, TU, Z_INV_CG, 0), ZA, nblk, kBlock, lds); break;
        default: COMBO_LAUNCH(k_zpass_inv, (T, TU, Z_INV_PLAIN, 0), ZA, nblk, kBlock, lds); break;
    }
    return hipGetLastError();
}

#endif

#if COMBO_IN_PART(COMBO_PART_CG)
template <typename TU>
hipError_t launch_update(const UArgs<TU>& a, hipStream_t s, int* nb, const BatchLaunch* b) {
    using UA = UArgs<TU>;
    const int nblk = blocks_u(a.g);
    if (nb) *nb = nblk;
    COMBO_LAUNCH(k_cg_update, (TU), UA, nblk, kBlock, 0);
    return hipGetLastError();
}

int blocks_antiherm(const Grid& g) {
    const long long npl = 2LL * g.n2 * g.n3;
    return (int)std::min<long long>((npl + kBlock - 1) / kBlock, 1024);
}

template <typename TU>
hipError_t launch_antiherm(const UArgs<TU>& a, hipStream_t s, const BatchLaunch* b) {
    using UA = UArgs<TU>;
    COMBO_LAUNCH(k_antiherm, (TU), UA, blocks_antiherm(a.g), kBlock, 0);
    return hipGetLastError();
}

hipError_t launch_finalize(int mode, const FinArgs& f, hipStream_t s, const FinArgs* dev_batch, int nrve) {
    if (dev_batch) hipLaunchKernelGGL(k_finalize_b, dim3(nrve), dim3(kBlock), 0, s, mode, dev_batch);
    else hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, mode, f);
    return hipGetLastError();
}

hipError_t launch_reduce_columns(const double* partials, int rows, int cols, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_columns, dim3(1), dim3(kBlock), 0, s, partials, rows, cols, out);
    return hipGetLastError();
}

#endif

#if COMBO_IN_PART(COMBO_PART_XF)
template hipError_t launch_x<float>(int, const XArgs<float>&, hipStream_t, int*, const BatchLaunch*);
#endif
#if COMBO_IN_PART(COMBO_PART_XD)
template hipError_t launch_x<double>(int, const XArgs<double>&, hipStream_t, int*, const BatchLaunch*);
#endif
#if COMBO_IN_PART(COMBO_PART_Y)
template hipError_t launch_y<float>(int, const YArgs<float>&, hipStream_t, const BatchLaunch*);
template hipError_t launch_y<double>(int, const YArgs<double>&, hipStream_t, const BatchLaunch*);
#endif
#if COMBO_IN_PART(COMBO_PART_ZF)
template hipError_t launch_z<float, float>(int, const ZArgs<float, float>&, hipStream_t, int*, const BatchLaunch*);
#endif
#if COMBO_IN_PART(COMBO_PART_ZD)
template hipError_t launch_z<double, double>(int, const ZArgs<double, double>&, hipStream_t, int*, const BatchLaunch*);
template hipError_t launch_z<double, float>(int, const ZArgs<double, float>&, hipStream_t, int*, const BatchLaunch*);
#endif
#if COMBO_IN_PART(COMBO_PART_CG)
template hipError_t launch_update<float>(const UArgs<float>&, hipStream_t, int*, const BatchLaunch*);
template hipError_t launch_update<double>(const UArgs<double>&, hipStream_t, int*, const BatchLaunch*);
template hipError_t launch_antiherm<float>(const UArgs<float>&, hipStream_t, const BatchLaunch*);
template hipError_t launch_antiherm<double>(const UArgs<double>&, hipStream_t, const BatchLaunch*);
#endif

}  // namespace combo
