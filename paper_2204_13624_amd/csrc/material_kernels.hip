// Pointwise constitutive update on gfx950, FP64 throughout.
//
// Pure voxels: compressible Neo-Hooke (paper Sec. 6.1),
//   W = lambda/2 (ln J)^2 - mu ln J + mu/2 (tr F^T F - 3),
//   P = mu F - m F^{-T} with m = mu - lambda ln J,
//   A_iJkL = mu d_ik d_JL + lambda Finv_Ji Finv_Lk + m Finv_Jk Finv_Li.
// The tangent state kept for the linear solves is {F^{-1}, m} (10 numbers).
//
// Composite voxels: the rank-one laminate of paper Sec. 4 with
//   F+- = F_box +- a (x) N / c+-                                  (eq. Fpm)
//   f(a) = (P+ - P-) N                                            (eq. tractionbalance)
//   Delta = sum_+- (mu I + (lambda + m) g (x) g) / c,  g = F^{-T} N  (eq. hessian,
//           written out for Neo-Hooke: N_J A_iJkL N_L = mu d_ik + (lambda + m) g_i g_k)
//   J+- = (1 +- a.v / c+-) J_box, v = F_box^{-T} N                (eq. Jpm)
// Newton-Raphson (Alg. 1) with the selective back-projection of Alg. 2 on the
// admissible interval beta_c^+ < a.m < beta_c^- (eq. matrixlemma), then
//   P_box = c+ P+ + c- P-                                         (eq. Peff:Seff)
//   A_box = c+ A+ + c- A- - dA D Delta^{-1} D^T dA,  with (D^T dA)_{k,pq} = dB_{k,pq},
//   B_{k,pq} = sum_J N_J A_kJpq = mu d_kp N_q + lambda g_k Finv_qp + m g_p Finv_qk.
// Small-strain law (law == kLawLinear, appendix cheat sheet, infinitesimal column):
//   sigma = lambda tr(eps) I + 2 mu eps, eps = sym(F - I), whose stiffness is the
//   Neo-Hooke tangent at F = I (state {I, mu}); the laminate jump is the closed form
//   a = -Delta^{-1} f(0) with f(0) = (sigma+(eps_box) - sigma-(eps_box)) N and g = N in
//   Delta, after which the stress and tangent formulas above apply unchanged.
// Stopping rule: |f| <= 1e-12 max(|P+ N|, |P- N|, 1e-3 max mu, 1e-2 max lambda)
// (the last term keeps the test above the round-off of lambda ln J) or a Newton
// correction |Delta^{-1} f| <= 1e-13 max(|a|, 1e-3) (round-off stagnation);
// at most max_laminate updates.  One thread per composite voxel.
#include <hip/hip_runtime.h>

#include "common.h"
#include "laminate_point.h"
#include "material.h"

namespace combo {

// per-block reduction of NV doubles per thread into out[0..NV) (thread 0 writes)
template <int NV>
__device__ __forceinline__ void block_sum_n(double* v, double* sh, double* out) {
#pragma unroll
    for (int c = 0; c < NV; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_down(v[c], off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) sh[wid * NV + c] = v[c];
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[w * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// ------------------------------------------------------------------------------
// pure voxels (and the deformation update of every voxel)
// ------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void k_material_pure_body(const MatArgs<T>& a, int tile_, int ntiles_) {
    __shared__ double sh[4 * 19];
    double sums[19];
#pragma unroll
    for (int c = 0; c < 19; ++c) sums[c] = 0.0;
    for (long long vox = (long long)tile_ * blockDim.x + threadIdx.x; vox < a.n;
         vox += (long long)ntiles_ * blockDim.x) {
        double F[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            double f = a.F_old[c * a.n + vox] + a.dFbar[c];
            if (a.dF) f += a.s * a.dF[c * a.n + vox];
            F[c] = f;
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) a.F_new[c * a.n + vox] = F[c];
        const int slot = a.slot[vox];
        if (slot >= 0) continue;
        const int ph = (slot == -1) ? 0 : 1;
        const double mu = a.mu[ph], lam = a.lam[ph];
        double Finv[9], P[9], m;
        if (a.law == kLawLinear) {
            lin_stress(F, mu, lam, Finv, P, m);
        } else {
            const double J = det3(F);
            if (!(J > 0.0)) {
                sums[18] += 1.0;
#pragma unroll
                for (int c = 0; c < 9; ++c) a.P[c * a.n + vox] = 0.0;
                continue;
            }
            nh_stress(F, J, mu, lam, Finv, P, m);
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            a.P[c * a.n + vox] = P[c];
            sums[9 * ph + c] += P[c];
        }
        if (a.Sinv) {
            const long long sp = state_pos(vox, a.n1, a.xm, a.xwbits);
#pragma unroll
            for (int c = 0; c < 9; ++c) a.Sinv[c * a.n + sp] = T(Finv[c]);
            a.sm[sp] = T(m);
        }
        if (a.A_full) {
            for (int r = 0; r < 81; ++r)
                a.A_full[(long long)r * a.n + vox] = nh_tangent(Finv, mu, lam, m, r / 27, (r / 9) % 3, (r % 9) / 3, r % 3);
        }
        if (a.a_full) {
#pragma unroll
            for (int c = 0; c < 3; ++c) a.a_full[c * a.n + vox] = 0.0;
        }
        if (a.iters_full) a.iters_full[vox] = 0;
    }
    double out[19];
    block_sum_n<19>(sums, sh, out);
    if (threadIdx.x < 19) a.partials[(long long)tile_ * 19 + threadIdx.x] = out[threadIdx.x];
}

template <typename T>
__global__ void __launch_bounds__(256) k_material_pure(MatArgs<T> a) {
    k_material_pure_body<T>(a, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_material_pure_b(const MatArgs<T>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_material_pure_body<T>(as[e.rve], e.tile, e.ntiles);
}

// ------------------------------------------------------------------------------
// composite voxels
// ------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void k_material_laminate_body(const MatArgs<T>& a, int tile_, int ntiles_) {
    __shared__ double sh[2 * 31];
    double sums[31];   // P_box (9), c P+ (9), (1-c) P- (9), fails, iters, backprojections, max iters
#pragma unroll
    for (int c = 0; c < 31; ++c) sums[c] = 0.0;
    for (int ic = tile_ * blockDim.x + threadIdx.x; ic < a.nc; ic += ntiles_ * blockDim.x) {
        const long long vox = a.comp_vox[ic];
        double Fb[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) Fb[c] = a.F_new[c * a.n + vox];
        const double cp = a.cc[ic], cm = 1.0 - cp;
        double N[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) N[d] = a.NN[(long long)d * a.nc + ic];
        const double mats[4] = {a.mu[0], a.lam[0], a.mu[1], a.lam[1]};
        double ainit[3];
        if (a.warm) {
#pragma unroll
            for (int i = 0; i < 3; ++i) ainit[i] = a.a_prev[(long long)i * a.nc + ic];
        }
        LamPoint o;
        laminate_point(Fb, cp, N, mats, a.law, a.maxit, a.warm ? ainit : nullptr, o);
        const int status = o.status;
        double Pb[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) Pb[c] = (status == 0) ? cp * o.Pp[c] + cm * o.Pm[c] : 0.0;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            a.P[c * a.n + vox] = Pb[c];
            sums[c] += Pb[c];
            sums[9 + c] += (status == 0) ? cp * o.Pp[c] : 0.0;
            sums[18 + c] += (status == 0) ? cm * o.Pm[c] : 0.0;
        }
        sums[27] += (status == 0) ? 0.0 : 1.0;
        sums[28] += o.iters;
        sums[29] += o.nbp;
        sums[30] = fmax(sums[30], (double)o.iters);
#pragma unroll
        for (int i = 0; i < 3; ++i) a.a_out[(long long)i * a.nc + ic] = o.a[i];
        if (a.a_full)
#pragma unroll
            for (int i = 0; i < 3; ++i) a.a_full[i * a.n + vox] = o.a[i];
        if (a.iters_full) a.iters_full[vox] = o.iters;

        // consistent tangent at the converged jump
        const bool want_state = (a.Acomp != nullptr) || (a.A_full != nullptr);
        if (!want_state) continue;
        if (status != 0) {
            if (a.Acomp)
                for (int r = 0; r < 45; ++r) a.Acomp[(long long)ic * 45 + r] = T(0);
            if (a.A_full)
                for (int r = 0; r < 81; ++r) a.A_full[(long long)r * a.n + vox] = 0.0;
            continue;
        }
        laminate_tangent<T>(o, cp, N, mats, a.Acomp ? a.Acomp + (long long)ic * 45 : nullptr,
                            a.A_full ? a.A_full + vox : nullptr, a.n);
    }
    // block reduction: sums 0..29 added, 30 = max
    double out[31];
    {
        double mx = sums[30];
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
        sums[30] = mx;
    }
    block_sum_n<30>(sums, sh, out);
    // max over the waves of the block
    __shared__ double shm[4];
    if ((threadIdx.x & 63) == 0) shm[threadIdx.x >> 6] = sums[30];
    __syncthreads();
    if (threadIdx.x < 30) a.partials2[(long long)tile_ * 31 + threadIdx.x] = out[threadIdx.x];
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) mx = fmax(mx, shm[w]);
        a.partials2[(long long)tile_ * 31 + 30] = mx;
    }
}

template <typename T>
__global__ void __launch_bounds__(128) k_material_laminate(MatArgs<T> a) {
    k_material_laminate_body<T>(a, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(128) k_material_laminate_b(const MatArgs<T>* __restrict__ as, const TileMap* __restrict__ map) {
    const TileMap e = map[blockIdx.x];
    k_material_laminate_body<T>(as[e.rve], e.tile, e.ntiles);
}

// ------------------------------------------------------------------------------
// reductions of the per-block material sums (fixed order)
// ------------------------------------------------------------------------------
// column c of the sums: out[0..19) over pure blocks, out[19..50) over laminate blocks (49 = max)
__device__ __forceinline__ void material_reduce_body(const double* pp, int nbp, const double* pl, int nbl,
                                                     double* out, int c) {
    __shared__ double sh[4];
    {
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

// one workgroup per column of the sums
__global__ void __launch_bounds__(256) k_material_reduce(const double* pp, int nbp, const double* pl, int nbl,
                                                         double* out) {
    material_reduce_body(pp, nbp, pl, nbl, out, blockIdx.x);
}

// one workgroup per RVE and column
__global__ void __launch_bounds__(256) k_material_reduce_b(const MatReduceArgs* __restrict__ red) {
    const MatReduceArgs r = red[blockIdx.x];
    material_reduce_body(r.pp, r.nbp, r.pl, r.nbl, r.out, blockIdx.y);
}

int material_blocks_pure(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}
int material_blocks_laminate(int nc) {
    int b = (nc + 127) / 128;
    return b < 1 ? 1 : (b < 4096 ? b : 4096);
}

// The laminate kernel reads F at its composites from the pure kernel's output, so the two run
// in order; the reduction takes one workgroup per column of the sums.
template <typename T>
hipError_t launch_material(const MatArgs<T>& a, int nbp, int nbl, double* sums_out, hipStream_t s) {
    hipLaunchKernelGGL(k_material_pure<T>, dim3(nbp), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.nc > 0) {
        hipLaunchKernelGGL(k_material_laminate<T>, dim3(nbl), dim3(128), 0, s, a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_material_reduce, dim3(19 + 31), dim3(256), 0, s, a.partials, nbp, a.partials2,
                       a.nc > 0 ? nbl : 0, sums_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_material_batch(const MatArgs<T>* dev_args, const BatchLaunch& pure, const BatchLaunch& lam,
                                 const MatReduceArgs* dev_red, int nrve, hipStream_t s) {
    if (pure.nblocks > 0) {
        hipLaunchKernelGGL(k_material_pure_b<T>, dim3(pure.nblocks), dim3(256), 0, s, dev_args, pure.map);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (lam.nblocks > 0) {
        hipLaunchKernelGGL(k_material_laminate_b<T>, dim3(lam.nblocks), dim3(128), 0, s, dev_args, lam.map);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_material_reduce_b, dim3(nrve, 19 + 31), dim3(256), 0, s, dev_red);
    return hipGetLastError();
}

template hipError_t launch_material<float>(const MatArgs<float>&, int, int, double*, hipStream_t);
template hipError_t launch_material<double>(const MatArgs<double>&, int, int, double*, hipStream_t);
template hipError_t launch_material_batch<float>(const MatArgs<float>*, const BatchLaunch&, const BatchLaunch&,
                                                 const MatReduceArgs*, int, hipStream_t);
template hipError_t launch_material_batch<double>(const MatArgs<double>*, const BatchLaunch&, const BatchLaunch&,
                                                  const MatReduceArgs*, int, hipStream_t);

}  // namespace combo
