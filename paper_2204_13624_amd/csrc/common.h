// Shared device/host definitions of the ComBo HIP path (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace combo {

constexpr int kBlock = 256;          // threads per workgroup of the FFT passes
// complex elements held in LDS by one FFT workgroup (32 KiB of data either way)
template <typename T> __host__ __device__ constexpr int max_elems() { return sizeof(T) == 4 ? 4096 : 2048; }
constexpr int kMaxAxis = 512;        // largest supported grid axis
// elements the generic x pass holds in LDS: five packed sequences of a row of up to kMaxAxis
template <typename T> __host__ __device__ constexpr int xpass_cap() {
    return 5 * kMaxAxis > max_elems<T>() ? 5 * kMaxAxis : max_elems<T>();
}
constexpr int kMaxPasses = 8;

template <typename T> struct cpx_t;
template <> struct cpx_t<float> { using type = float2; };
template <> struct cpx_t<double> { using type = double2; };
template <typename T> using cpx = typename cpx_t<T>::type;

template <typename T> __host__ __device__ inline cpx<T> mk(T x, T y) { cpx<T> r; r.x = x; r.y = y; return r; }
template <typename C> __host__ __device__ inline C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __host__ __device__ inline C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __host__ __device__ inline C cmul(C a, C b) {
    C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
template <typename C> __host__ __device__ inline C cconj(C a) { C r; r.x = a.x; r.y = -a.y; return r; }
template <typename C, typename T> __host__ __device__ inline C cscale(C a, T s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }
// multiply by +i (s = +1) or -i (s = -1)
template <int S, typename C> __host__ __device__ inline C cmul_i(C a) {
    C r;
    if (S > 0) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
    return r;
}

// Radix plan of one axis: L = prod(radix[0..npass)).  Twiddles W_L^m = exp(-2 pi i m / L)
// are read from a table of L entries (forward); the inverse uses their conjugates.
struct AxisPlan {
    int L;
    int npass;
    int radix[kMaxPasses];
};

// Geometry of one RVE as the kernels see it.
struct Grid {
    int n1, n2, n3;       // voxels per axis
    int nh;               // row stride of the half spectrum (complex values; >= nkx)
    int nkx;              // stored x frequencies: n1/2 (even n1, Nyquist dropped) or (n1+1)/2;
                          // rotated scheme: n1/2 + 1, rows padded to nh with zero modes
    long long n;          // n1*n2*n3
    long long nspec;      // nh*n2*n3 (complex values per spectral component, padding included)
    double xs1, xs2, xs3; // 2 pi / l_d: xi_d(k) = xs_d * k
    int xm, xwbits;       // wavefront x pass: m values per lane, log2 of lanes per row (-1: none)
    int xv, yv, zv;       // schedule: variant of the x, y and z FFT passes (0 = default)
    int disc;             // 0: Moulinec-Suquet frequencies, 1: Willot's rotated scheme, 2: staggered grid
    const double* ftab;   // disc 1: device table D1[nh] A1[nh] D2[n2] A2[n2] D3[n3] A3[n3]
                          // (D1 = A1 = 0 on the padding x >= nkx: every padded mode is a zero mode);
                          // disc 2: the same slots hold Re f_d and Im f_d of the forward-difference
                          // symbol f_d = (e^{i theta} - 1) / h_d (0 on the padding)
};

// Position of voxel `vox` in the tangent-state arrays.  With the wavefront x
// pass, voxel x of a row sits in lane bitrev(x / m), slot x mod m after the
// inverse transform, so the state is stored at lane + W slot within the row and
// the x pass reads it unit-stride; otherwise the natural order is kept.
__host__ __device__ inline long long state_pos(long long vox, int n1, int xm, int xwbits) {
    if (xwbits < 0) return vox;
    const long long row = vox / n1;
    const int x = (int)(vox - row * n1);
    const int s = x % xm, t = x / xm;
    int l = 0;
    for (int b = 0; b < xwbits; ++b) l |= ((t >> b) & 1) << (xwbits - 1 - b);
    return row * n1 + l + (1 << xwbits) * s;
}

// One workgroup of a batched launch: which RVE, which of its tiles, and how many
// tiles that RVE has in this launch (grid-stride kernels stride by it).
struct TileMap {
    int rve;
    int tile;
    int ntiles;
};

// Device-side description of a batched launch: per-RVE argument blocks and the
// workgroup -> (RVE, tile) map (nblocks entries).  Null pointer = single launch.
struct BatchLaunch {
    const void* args;
    const TileMap* map;
    int nblocks;
};

__host__ __device__ inline int freq_of(int j, int n) { return (j < (n + 1) / 2) ? j : j - n; }

// Gradient factors per axis at a stored index: the gradient of a CG coefficient
// field w_hat is F_hat_iJ = k'_J w_hat_i with k' = (D1 A2 A3, A1 D2 A3, A1 A2 D3).
// Moulinec-Suquet: D_d = xi_d, A_d = 1.  Willot's rotated scheme: D = (2/h) sin(theta/2),
// A = cos(theta/2) (the common phase of the corner-to-centre stencil is carried by w_hat).
__device__ inline double fac_d1(const Grid& g, int k) { return g.disc ? g.ftab[k] : g.xs1 * k; }
__device__ inline double fac_a1(const Grid& g, int k) { return g.disc ? g.ftab[g.nh + k] : 1.0; }
__device__ inline double fac_d2(const Grid& g, int j) { return g.disc ? g.ftab[2 * g.nh + j] : g.xs2 * freq_of(j, g.n2); }
__device__ inline double fac_a2(const Grid& g, int j) { return g.disc ? g.ftab[2 * g.nh + g.n2 + j] : 1.0; }
__device__ inline double fac_d3(const Grid& g, int j) {
    return g.disc ? g.ftab[2 * g.nh + 2 * g.n2 + j] : g.xs3 * freq_of(j, g.n3);
}
__device__ inline double fac_a3(const Grid& g, int j) { return g.disc ? g.ftab[2 * g.nh + 2 * g.n2 + g.n3 + j] : 1.0; }
// Copies count factors of the table (e.g. one axis's D[len] A[len], contiguous: count =
// 2 len) into LDS in the precision of the pass, so that the transforms read them from
// LDS instead of keeping per-element double loads from the table in flight.
template <typename T>
__device__ inline void stage_factors(T* dst, const double* src, int count, int tid, int nthreads) {
    for (int i = tid; i < count; i += nthreads) dst[i] = T(src[i]);
}
// Staggered grid (disc 2): forward-difference symbol of each axis at a stored index
// (x: 0 <= k < nh, y and z: array index), complex, in the precision of the pass.
template <typename T> __device__ inline cpx<T> fst1(const Grid& g, int k) {
    return mk<T>(T(g.ftab[k]), T(g.ftab[g.nh + k]));
}
template <typename T> __device__ inline cpx<T> fst2(const Grid& g, int j) {
    return mk<T>(T(g.ftab[2 * g.nh + j]), T(g.ftab[2 * g.nh + g.n2 + j]));
}
template <typename T> __device__ inline cpx<T> fst3(const Grid& g, int j) {
    return mk<T>(T(g.ftab[2 * g.nh + 2 * g.n2 + j]), T(g.ftab[2 * g.nh + 2 * g.n2 + g.n3 + j]));
}
// true if index j is the Nyquist index of an even axis of length n
__host__ __device__ inline bool is_nyquist(int j, int n) { return (n % 2 == 0) && (j == n / 2) && n > 1; }

}  // namespace combo
