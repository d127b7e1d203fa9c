// Doubly-fine material grid (DFMG) law on the staggered grid (paper App. A,
// eq. constitutive_law), its tangent action and the staggered layout shifts, on
// gfx950.  Layout and conventions: dfmg.h.  Pure doubly-fine cells take the
// compressible Neo-Hooke law (Sec. 6.1), those of composite cells the rank-one
// laminate of Sec. 4 (laminate_point.h), one solve per doubly-fine cell.
#include <hip/hip_runtime.h>

#include "dfmg.h"
#include "laminate_point.h"
#include "material.h"

namespace combo {

namespace {

struct CellIdx {
    int i, j, k;
};

__device__ __forceinline__ CellIdx cell_of(long long cell, int n1, int n2) {
    CellIdx c;
    c.i = (int)(cell % n1);
    const long long t = cell / n1;
    c.j = (int)(t % n2);
    c.k = (int)(t / n2);
    return c;
}

__device__ __forceinline__ int wrap(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// index of cell c + (di, dj, dk), periodic (|d| <= 1)
__device__ __forceinline__ long long cell_at(const CellIdx& c, int di, int dj, int dk, int n1, int n2, int n3) {
    return ((long long)wrap(c.k + dk, n3) * n2 + wrap(c.j + dj, n2)) * n1 + wrap(c.i + di, n1);
}

// the deformation of doubly-fine cell (c, l) from a field H in the shifted layout:
// F_aa = H_aa[c], F_ab = H_ab[c + l_a e_a + l_b e_b - e_b]
template <typename TF, typename TH>
__device__ __forceinline__ void gather_dfc(const TH* H, long long n, const CellIdx& c, int l, int n1, int n2,
                                           int n3, TF* Fd) {
    const int lb[3] = {l & 1, (l >> 1) & 1, (l >> 2) & 1};
    const long long self = ((long long)c.k * n2 + c.j) * n1 + c.i;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            long long idx = self;
            if (a != b) {
                int d[3] = {0, 0, 0};
                d[a] += lb[a];
                d[b] += lb[b] - 1;
                idx = cell_at(c, d[0], d[1], d[2], n1, n2, n3);
            }
            Fd[3 * a + b] = TF(H[(long long)(3 * a + b) * n + idx]);
        }
}

template <typename T>
__device__ __forceinline__ void block_sums(double* v, int nv, double* sh, double* out_row) {
    // nv <= 31 values per thread; sums over the block into out_row (thread 0 writes)
    for (int c = 0; c < nv; ++c) {
        double x = v[c];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) t += sh[w];
            out_row[c] = t;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_dfmg_update(DfmgArgs<T> a) {
    const long long total = 9 * a.n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(e / a.n);
        double f = a.F_old[e] + a.dFbar[c];
        if (a.dF) f += a.s * a.dF[e];
        a.F_new[e] = f;
    }
}

// pure cells: thread per cell, its eight doubly-fine cells; sums as the per-voxel
// law's pure kernel (P of matrix / inclusion cells, weight 1/8; det F <= 0 count)
template <typename T>
__global__ void __launch_bounds__(256) k_dfmg_pure(DfmgArgs<T> a) {
    __shared__ double sh[4];
    double sums[19];
#pragma unroll
    for (int c = 0; c < 19; ++c) sums[c] = 0.0;
    for (long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x; cell < a.n;
         cell += (long long)gridDim.x * blockDim.x) {
        const int slot = a.slot[cell];
        if (slot >= 0) continue;
        const int ph = (slot == -1) ? 0 : 1;
        const double mu = a.mu[ph], lam = a.lam[ph];
        const CellIdx ci = cell_of(cell, a.n1, a.n2);
        for (int l = 0; l < 8; ++l) {
            double F[9];
            gather_dfc<double>(a.F_new, a.n, ci, l, a.n1, a.n2, a.n3, F);
            const double J = det3(F);
            double P[9], Finv[9], m = 0.0;
            if (!(J > 0.0)) {
                sums[18] += 1.0;
#pragma unroll
                for (int c = 0; c < 9; ++c) P[c] = Finv[c] = 0.0;
            } else {
                nh_stress(F, J, mu, lam, Finv, P, m);
            }
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                a.Pd[(long long)(c * 8 + l) * a.n + cell] = P[c];
                sums[9 * ph + c] += 0.125 * P[c];
            }
        }
    }
    block_sums<T>(sums, 19, sh, a.partials + (long long)blockIdx.x * 19);
}

// composite cells: thread per (composite, l); sums as the per-voxel laminate kernel
template <typename T>
__global__ void __launch_bounds__(128) k_dfmg_laminate(DfmgArgs<T> a) {
    __shared__ double sh[2];
    double sums[31];
#pragma unroll
    for (int c = 0; c < 31; ++c) sums[c] = 0.0;
    const long long total = 8LL * a.nc;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const int ic = (int)(t >> 3), l = (int)(t & 7);
        const long long cell = a.comp_vox[ic];
        const CellIdx ci = cell_of(cell, a.n1, a.n2);
        double Fb[9];
        gather_dfc<double>(a.F_new, a.n, ci, l, a.n1, a.n2, a.n3, Fb);
        const double cp = a.cc[ic], cm = 1.0 - cp;
        double N[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) N[d] = a.NN[(long long)d * a.nc + ic];
        const double mats[4] = {a.mu[0], a.lam[0], a.mu[1], a.lam[1]};
        double ainit[3];
        if (a.warm) {
#pragma unroll
            for (int i = 0; i < 3; ++i) ainit[i] = a.a_prev[(long long)(i * 8 + l) * a.nc + ic];
        }
        LamPoint o;
        laminate_point(Fb, cp, N, mats, kLawNeoHooke, a.maxit, a.warm ? ainit : nullptr, o);
        const bool ok = o.status == 0;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const double pb = ok ? cp * o.Pp[c] + cm * o.Pm[c] : 0.0;
            a.Pd[(long long)(c * 8 + l) * a.n + cell] = pb;
            sums[c] += 0.125 * pb;
            sums[9 + c] += ok ? 0.125 * cp * o.Pp[c] : 0.0;
            sums[18 + c] += ok ? 0.125 * cm * o.Pm[c] : 0.0;
        }
        sums[27] += ok ? 0.0 : 1.0;
        sums[28] += o.iters;
        sums[29] += o.nbp;
        sums[30] = fmax(sums[30], (double)o.iters);
#pragma unroll
        for (int i = 0; i < 3; ++i) a.a_out[(long long)(i * 8 + l) * a.nc + ic] = o.a[i];
        if (a.Ad) {
            T* dst = a.Ad + ((long long)ic * 8 + l) * 45;
            if (ok) {
                laminate_tangent<T>(o, cp, N, mats, dst, nullptr, 0);
            } else {
                for (int r = 0; r < 45; ++r) dst[r] = T(0);
            }
        }
    }
    // 30 sums and one max, as the per-voxel laminate kernel
    {
        double mx = sums[30];
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
        sums[30] = mx;
    }
    __shared__ double shm[2];
    if ((threadIdx.x & 63) == 0) shm[threadIdx.x >> 6] = sums[30];
    double* row = a.partials2 + (long long)blockIdx.x * 31;
    block_sums<T>(sums, 30, sh, row);
    if (threadIdx.x == 0) row[30] = fmax(shm[0], blockDim.x > 64 ? shm[1] : 0.0);
}

// reductions of the two kernels' partials into the kSumsLen layout (fixed order)
__global__ void __launch_bounds__(256) k_dfmg_reduce(const double* pp, int nbp, const double* pl, int nbl,
                                                     double* out) {
    __shared__ double sh[4];
    for (int c = 0; c < 19 + 31; ++c) {
        const bool lam = c >= 19;
        const int cc = lam ? c - 19 : c;
        const int rows = lam ? nbl : nbp;
        const int cols = lam ? 31 : 19;
        const double* src = lam ? pl : pp;
        const bool is_max = lam && cc == 30;
        double s = 0.0;
        for (int r = threadIdx.x; r < rows; r += blockDim.x) {
            const double v = src[(long long)r * cols + cc];
            s = is_max ? fmax(s, v) : s + v;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_down(s, off, 64);
            s = is_max ? fmax(s, o) : s + o;
        }
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) t = is_max ? fmax(t, sh[w]) : t + sh[w];
            out[c] = t;
        }
        __syncthreads();
    }
}

// The 27 staggered values of one component set that a cell's eight doubly-fine cells
// use: the diagonal (a, a) at the cell (slot a), and for each ordered pair p = (a, b)
// of the order of dfmg.h the value at cell + l_a e_a + (l_b - 1) e_b (slot
// 3 + 4 p + 2 l_a + l_b), read from the shifted layout.
__device__ __forceinline__ constexpr int pair_a(int p) { return p / 2; }
__device__ __forceinline__ constexpr int pair_b(int p) { return (p % 2 == 0) ? (p / 2 == 0 ? 1 : 0) : (p / 2 == 2 ? 1 : 2); }

template <typename TV, typename TH>
__device__ __forceinline__ void load27(const TH* H, long long n, const CellIdx& c, int n1, int n2, int n3, TV* v) {
    const long long self = ((long long)c.k * n2 + c.j) * n1 + c.i;
#pragma unroll
    for (int a0 = 0; a0 < 3; ++a0) v[a0] = TV(H[(long long)(4 * a0) * n + self]);
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int aa = pair_a(p), bb = pair_b(p);
#pragma unroll
        for (int la = 0; la < 2; ++la)
#pragma unroll
            for (int lb = 0; lb < 2; ++lb) {
                int d[3] = {0, 0, 0};
                d[aa] += la;
                d[bb] += lb - 1;
                v[3 + 4 * p + 2 * la + lb] = TV(H[(long long)(3 * aa + bb) * n + cell_at(c, d[0], d[1], d[2], n1, n2, n3)]);
            }
    }
}

// the deformation of doubly-fine cell l from the 27 values
template <typename TV, int L>
__device__ __forceinline__ void dfc_from27(const TV* v, TV* Fd) {
    constexpr int lb[3] = {L & 1, (L >> 1) & 1, (L >> 2) & 1};
#pragma unroll
    for (int a0 = 0; a0 < 3; ++a0) Fd[4 * a0] = v[a0];
#pragma unroll
    for (int p = 0; p < 6; ++p) {
        const int aa = pair_a(p), bb = pair_b(p);
        Fd[3 * aa + bb] = v[3 + 4 * p + 2 * lb[aa] + lb[bb]];
    }
}

template <typename T, int L>
__device__ __forceinline__ void action_dfc(const DfmgActArgs<T>& a, int slot, double mu, double lam, const double* Fv,
                                           const T* hv, T* own, T* part) {
    constexpr int lb[3] = {L & 1, (L >> 1) & 1, (L >> 2) & 1};
    T p[9], tau[9];
    dfc_from27<T, L>(hv, p);
    if (slot >= 0) {
        const T* A = a.Ad + ((long long)slot * 8 + L) * 45;
        T s[45];
#pragma unroll
        for (int r = 0; r < 45; ++r) s[r] = A[r];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int lo = r < q ? r : q, hi = r < q ? q : r;
                acc += s[lo * 9 - (lo * (lo - 1)) / 2 + (hi - lo)] * p[q];
            }
            tau[r] = acc;
        }
    } else {
        // Neo-Hooke tangent at the doubly-fine deformation: F^{-1} and m = mu - lambda ln J in FP64
        double F[9], Fi[9];
        dfc_from27<double, L>(Fv, F);
        const double J = det3(F);
        adj3(F, Fi);
        double m = 0.0, iJ = 0.0;
        if (J > 0.0) {
            iJ = 1.0 / J;
            m = mu - lam * log(J);
        }
        T fi[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) fi[c] = T(Fi[c] * iJ);
        const T mt = T(m), mut = T(mu), lamt = T(lam);
        // B = F^{-1} p, C = B F^{-1};  tau_iJ = mu p_iJ + lam tr(B) Finv_Ji + m C_Ji
        T B[9];
#pragma unroll
        for (int J2 = 0; J2 < 3; ++J2)
#pragma unroll
            for (int Lc = 0; Lc < 3; ++Lc)
                B[3 * J2 + Lc] = fi[3 * J2 + 0] * p[0 + Lc] + fi[3 * J2 + 1] * p[3 + Lc] + fi[3 * J2 + 2] * p[6 + Lc];
        const T tr = B[0] + B[4] + B[8];
        T C[9];
#pragma unroll
        for (int J2 = 0; J2 < 3; ++J2)
#pragma unroll
            for (int i = 0; i < 3; ++i)
                C[3 * J2 + i] = B[3 * J2 + 0] * fi[0 + i] + B[3 * J2 + 1] * fi[3 + i] + B[3 * J2 + 2] * fi[6 + i];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int J2 = 0; J2 < 3; ++J2)
                tau[3 * i + J2] = mut * p[3 * i + J2] + lamt * tr * fi[3 * J2 + i] + mt * C[3 * J2 + i];
    }
    // destinations: diagonal -> own; (a, b) -> offset l_a e_a + (l_b - 1) e_b
#pragma unroll
    for (int a0 = 0; a0 < 3; ++a0) own[4 * a0] += T(0.125) * tau[4 * a0];
#pragma unroll
    for (int pr = 0; pr < 6; ++pr) {
        const int aa = pair_a(pr), bb = pair_b(pr);
        const T v = T(0.125) * tau[3 * aa + bb];
        if (lb[aa] == 0 && lb[bb] == 1) own[3 * aa + bb] += v;       // offset 0
        else if (lb[aa] == 1 && lb[bb] == 1) part[3 * pr + 0] += v;  // +e_a
        else if (lb[aa] == 0) part[3 * pr + 1] += v;                 // -e_b
        else part[3 * pr + 2] += v;                                  // e_a - e_b
    }
}

// tangent action per cell, summed per destination (thread per cell; dfmg.h).  The
// 27 values of the deformation and of dH that the cell's doubly-fine cells use are
// loaded once, then the eight doubly-fine cells are evaluated from registers.
template <typename T>
__global__ void __launch_bounds__(256) k_dfmg_action(DfmgActArgs<T> a) {
    if (a.st && a.st->done) return;
    for (long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x; cell < a.n;
         cell += (long long)gridDim.x * blockDim.x) {
        const int slot = a.slot[cell];
        const CellIdx ci = cell_of(cell, a.n1, a.n2);
        T hv[27];
        double Fv[27];
        load27<T>(a.dH, a.n, ci, a.n1, a.n2, a.n3, hv);
        if (slot < 0) {
            load27<double>(a.F, a.n, ci, a.n1, a.n2, a.n3, Fv);
        } else {
#pragma unroll
            for (int c = 0; c < 27; ++c) Fv[c] = 0.0;
        }
        const int ph = (slot == -1) ? 0 : 1;
        const double mu = a.mu[ph], lam = a.lam[ph];
        T own[9], part[18];
#pragma unroll
        for (int c = 0; c < 9; ++c) own[c] = T(0);
#pragma unroll
        for (int c = 0; c < 18; ++c) part[c] = T(0);
        action_dfc<T, 0>(a, slot, mu, lam, Fv, hv, own, part);
        action_dfc<T, 1>(a, slot, mu, lam, Fv, hv, own, part);
        action_dfc<T, 2>(a, slot, mu, lam, Fv, hv, own, part);
        action_dfc<T, 3>(a, slot, mu, lam, Fv, hv, own, part);
        action_dfc<T, 4>(a, slot, mu, lam, Fv, hv, own, part);
        action_dfc<T, 5>(a, slot, mu, lam, Fv, hv, own, part);
        action_dfc<T, 6>(a, slot, mu, lam, Fv, hv, own, part);
        action_dfc<T, 7>(a, slot, mu, lam, Fv, hv, own, part);
#pragma unroll
        for (int c = 0; c < 9; ++c) a.own[(long long)c * a.n + cell] = own[c];
#pragma unroll
        for (int c = 0; c < 18; ++c) a.part[(long long)c * a.n + cell] = part[c];
    }
}

// Q = own + neighbours' parts (thread per cell)
template <typename T>
__global__ void __launch_bounds__(256) k_dfmg_sum(DfmgSumArgs<T> a) {
    if (a.st && a.st->done) return;
    for (long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x; cell < a.n;
         cell += (long long)gridDim.x * blockDim.x) {
        const CellIdx ci = cell_of(cell, a.n1, a.n2);
#pragma unroll
        for (int a0 = 0; a0 < 3; ++a0) a.Q[(long long)(4 * a0) * a.n + cell] = a.own[(long long)(4 * a0) * a.n + cell];
#pragma unroll
        for (int pr = 0; pr < 6; ++pr) {
            const int aa = pr / 2, bb = (pr % 2 == 0) ? (aa == 0 ? 1 : 0) : (aa == 2 ? 1 : 2);
            const int c = 3 * aa + bb;
            // contributions written at cell - offset by the cells that own them
            int d0[3] = {0, 0, 0}, d1[3] = {0, 0, 0}, d2[3] = {0, 0, 0};
            d0[aa] = -1;             // written with offset +e_a at cell - e_a
            d1[bb] = +1;             // offset -e_b at cell + e_b
            d2[aa] = -1;
            d2[bb] = +1;             // offset e_a - e_b at cell - e_a + e_b
            T v = a.own[(long long)c * a.n + cell];
            v += a.part[(long long)(3 * pr + 0) * a.n + cell_at(ci, d0[0], d0[1], d0[2], a.n1, a.n2, a.n3)];
            v += a.part[(long long)(3 * pr + 1) * a.n + cell_at(ci, d1[0], d1[1], d1[2], a.n1, a.n2, a.n3)];
            v += a.part[(long long)(3 * pr + 2) * a.n + cell_at(ci, d2[0], d2[1], d2[2], a.n1, a.n2, a.n3)];
            a.Q[(long long)c * a.n + cell] = v;
        }
    }
}

// DFMG sum into the shifted layout (thread per cell)
template <typename TI>
__global__ void __launch_bounds__(256) k_dfmg_gather(DfmgGatherArgs<TI> a) {
    if (a.st && a.st->done) return;
    for (long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x; cell < a.n;
         cell += (long long)gridDim.x * blockDim.x) {
        const CellIdx ci = cell_of(cell, a.n1, a.n2);
#pragma unroll
        for (int a0 = 0; a0 < 3; ++a0)
#pragma unroll
            for (int b0 = 0; b0 < 3; ++b0) {
                const int c = 3 * a0 + b0;
                double acc = 0.0;
                for (int l = 0; l < 8; ++l) {
                    long long idx = cell;
                    if (a0 != b0) {
                        // P_ab at the edge xi + e_b: doubly-fine cell (xi + e_b - l_a e_a - l_b e_b, l)
                        const int lb[3] = {l & 1, (l >> 1) & 1, (l >> 2) & 1};
                        int d[3] = {0, 0, 0};
                        d[a0] -= lb[a0];
                        d[b0] += 1 - lb[b0];
                        idx = cell_at(ci, d[0], d[1], d[2], a.n1, a.n2, a.n3);
                    }
                    acc += double(a.Pd[(long long)(c * 8 + l) * a.n + idx]);
                }
                a.Q[(long long)c * a.n + cell] = 0.125 * acc;
            }
    }
}

__global__ void __launch_bounds__(256) k_stag_shift(const double* in, double* out, int n1, int n2, int n3, int dir) {
    const long long n = (long long)n1 * n2 * n3;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < 9 * n;
         e += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(e / n);
        const long long cell = e - (long long)c * n;
        const int a = c / 3, J = c % 3;
        long long src = cell;
        if (a != J) {
            const CellIdx ci = cell_of(cell, n1, n2);
            int d[3] = {0, 0, 0};
            d[J] = dir;
            src = cell_at(ci, d[0], d[1], d[2], n1, n2, n3);
        }
        out[e] = in[(long long)c * n + src];
    }
}

// f[c][v] = E_c (add = 0) or f[c][v] += E_c (add = 1): a uniform tensor field, the same in
// the natural and the shifted layout
template <typename T>
__global__ void __launch_bounds__(256) k_stag_uniform(T* f, long long n, UniformE E, int add) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < 9 * n;
         e += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(e / n);
        f[e] = add ? T(double(f[e]) + E.v[c]) : T(E.v[c]);
    }
}

// per-workgroup sums of the nine components of a [9][n] field, in FP64 and a fixed order
template <typename T>
__global__ void __launch_bounds__(256) k_stag_field_sums(const T* f, long long n, double* partials) {
    __shared__ double red[4];
    for (int c = 0; c < 9; ++c) {
        double acc = 0.0;
        for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
             v += (long long)gridDim.x * blockDim.x)
            acc += double(f[(long long)c * n + v]);
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) partials[(long long)blockIdx.x * 9 + c] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

unsigned grid_for(long long items) {
    const long long b = (items + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

int dfmg_blocks_pure(long long n) {
    const long long b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

int dfmg_blocks_laminate(int nc) {
    const long long b = (8LL * nc + 127) / 128;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

template <typename T>
hipError_t launch_dfmg_update(const DfmgArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_dfmg_update<T>, dim3(grid_for(9 * a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dfmg_law(const DfmgArgs<T>& a, double* sums_out, hipStream_t s) {
    const int nbp = dfmg_blocks_pure(a.n), nbl = dfmg_blocks_laminate(a.nc);
    hipLaunchKernelGGL(k_dfmg_pure<T>, dim3(nbp), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.nc > 0) {
        hipLaunchKernelGGL(k_dfmg_laminate<T>, dim3(nbl), dim3(128), 0, s, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_dfmg_reduce, dim3(1), dim3(256), 0, s, a.partials, nbp, a.partials2, a.nc > 0 ? nbl : 0,
                       sums_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dfmg_action(const DfmgActArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_dfmg_action<T>, dim3(grid_for(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dfmg_sum(const DfmgSumArgs<T>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_dfmg_sum<T>, dim3(grid_for(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <typename TI>
hipError_t launch_dfmg_gather(const DfmgGatherArgs<TI>& a, hipStream_t s) {
    hipLaunchKernelGGL(k_dfmg_gather<TI>, dim3(grid_for(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stag_shift(const double* in, double* out, int n1, int n2, int n3, int dir, hipStream_t s) {
    const long long n = (long long)n1 * n2 * n3;
    hipLaunchKernelGGL(k_stag_shift, dim3(grid_for(9 * n)), dim3(256), 0, s, in, out, n1, n2, n3, dir);
    return hipGetLastError();
}

template hipError_t launch_dfmg_update<float>(const DfmgArgs<float>&, hipStream_t);
template hipError_t launch_dfmg_update<double>(const DfmgArgs<double>&, hipStream_t);
template hipError_t launch_dfmg_law<float>(const DfmgArgs<float>&, double*, hipStream_t);
template hipError_t launch_dfmg_law<double>(const DfmgArgs<double>&, double*, hipStream_t);
template hipError_t launch_dfmg_action<float>(const DfmgActArgs<float>&, hipStream_t);
template hipError_t launch_dfmg_action<double>(const DfmgActArgs<double>&, hipStream_t);
template hipError_t launch_dfmg_sum<float>(const DfmgSumArgs<float>&, hipStream_t);
template hipError_t launch_dfmg_sum<double>(const DfmgSumArgs<double>&, hipStream_t);
template hipError_t launch_dfmg_gather<double>(const DfmgGatherArgs<double>&, hipStream_t);

template <typename T>
hipError_t launch_stag_uniform(T* f, long long n, const double E[9], int add, hipStream_t s) {
    UniformE u;
    for (int c = 0; c < 9; ++c) u.v[c] = E[c];
    hipLaunchKernelGGL(k_stag_uniform<T>, dim3(grid_for(9 * n)), dim3(256), 0, s, f, n, u, add);
    return hipGetLastError();
}

int stag_sum_blocks(long long n) {
    const long long b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

template <typename T>
hipError_t launch_stag_field_sums(const T* f, long long n, double* partials, hipStream_t s) {
    hipLaunchKernelGGL(k_stag_field_sums<T>, dim3(stag_sum_blocks(n)), dim3(256), 0, s, f, n, partials);
    return hipGetLastError();
}

template hipError_t launch_stag_uniform<float>(float*, long long, const double*, int, hipStream_t);
template hipError_t launch_stag_uniform<double>(double*, long long, const double*, int, hipStream_t);
template hipError_t launch_stag_field_sums<float>(const float*, long long, double*, hipStream_t);
template hipError_t launch_stag_field_sums<double>(const double*, long long, double*, hipStream_t);

}  // namespace combo
