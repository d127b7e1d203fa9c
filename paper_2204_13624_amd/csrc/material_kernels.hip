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
#include "material.h"

namespace combo {

__device__ __forceinline__ double det3(const double* F) {
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) + F[2] * (F[3] * F[7] - F[4] * F[6]);
}

// adjugate: F^{-1} = adj(F) / det F
__device__ __forceinline__ void adj3(const double* F, double* A) {
    A[0] = F[4] * F[8] - F[5] * F[7];
    A[1] = F[2] * F[7] - F[1] * F[8];
    A[2] = F[1] * F[5] - F[2] * F[4];
    A[3] = F[5] * F[6] - F[3] * F[8];
    A[4] = F[0] * F[8] - F[2] * F[6];
    A[5] = F[2] * F[3] - F[0] * F[5];
    A[6] = F[3] * F[7] - F[4] * F[6];
    A[7] = F[1] * F[6] - F[0] * F[7];
    A[8] = F[0] * F[4] - F[1] * F[3];
}

// Neo-Hooke stress at F with a known J > 0: Finv, P and m = mu - lambda ln J
__device__ __forceinline__ void nh_stress(const double* F, double J, double mu, double lam, double* Finv, double* P,
                                          double& m) {
    adj3(F, Finv);
    const double iJ = 1.0 / J;
#pragma unroll
    for (int i = 0; i < 9; ++i) Finv[i] *= iJ;
    m = mu - lam * log(J);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int J2 = 0; J2 < 3; ++J2) P[3 * i + J2] = mu * F[3 * i + J2] - m * Finv[3 * J2 + i];
}

// small-strain isotropic stress of the displacement gradient F - I; Finv = I and
// m = mu make the Neo-Hooke tangent formulas give the isotropic stiffness
__device__ __forceinline__ void lin_stress(const double* F, double mu, double lam, double* Finv, double* P,
                                           double& m) {
    const double tr = F[0] + F[4] + F[8] - 3.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int J = 0; J < 3; ++J) {
            const double e = 0.5 * (F[3 * i + J] + F[3 * J + i]) - (i == J ? 1.0 : 0.0);
            P[3 * i + J] = 2.0 * mu * e + (i == J ? lam * tr : 0.0);
            Finv[3 * i + J] = (i == J) ? 1.0 : 0.0;
        }
    m = mu;
}

// full tangent entry A_(iJ)(kL) of Neo-Hooke
__device__ __forceinline__ double nh_tangent(const double* Finv, double mu, double lam, double m, int i, int J, int k,
                                             int L) {
    return ((i == k && J == L) ? mu : 0.0) + lam * Finv[3 * J + i] * Finv[3 * L + k] + m * Finv[3 * J + k] * Finv[3 * L + i];
}

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
        const double mup = a.mu[1], lamp = a.lam[1], mum = a.mu[0], lamm = a.lam[0];
        const double floor_t = fmax(1e-3 * fmax(mup, mum), 1e-2 * fmax(lamp, lamm));

        int status = 1;   // 0 ok, 1 iteration limit, 2 bad F_box, 3 inadmissible
        int iters = 0, nbp = 0;
        double a3[3] = {0.0, 0.0, 0.0};
        double Pp[9], Pm[9], Fip[9], Fim[9], mp = 0.0, mm = 0.0;
        const double Jb = det3(Fb);
        double v[3] = {0, 0, 0}, mb[3] = {0, 0, 0}, bp = 0.0, bm = 0.0;
        if (a.law == kLawLinear) {
            // closed form: one exact Newton step from a = 0 (the traction jump is linear in a)
            lin_stress(Fb, mup, lamp, Fip, Pp, mp);
            lin_stress(Fb, mum, lamm, Fim, Pm, mm);
            double f[3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                f[i] = (Pp[3 * i] - Pm[3 * i]) * N[0] + (Pp[3 * i + 1] - Pm[3 * i + 1]) * N[1] +
                       (Pp[3 * i + 2] - Pm[3 * i + 2]) * N[2];
            const double kp = (lamp + mup) / cp, km = (lamm + mum) / cm, d0 = mup / cp + mum / cm;
            double D[6];
            D[0] = d0 + (kp + km) * N[0] * N[0];
            D[1] = (kp + km) * N[0] * N[1];
            D[2] = (kp + km) * N[0] * N[2];
            D[3] = d0 + (kp + km) * N[1] * N[1];
            D[4] = (kp + km) * N[1] * N[2];
            D[5] = d0 + (kp + km) * N[2] * N[2];
            double Di[6], da[3];
            sym3_inv(D, Di);
            sym3_mul(Di, f, da);
            double Fp[9], Fm[9];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                a3[i] = -da[i];
#pragma unroll
                for (int J = 0; J < 3; ++J) {
                    const double aN = -da[i] * N[J];
                    Fp[3 * i + J] = Fb[3 * i + J] + aN / cp;
                    Fm[3 * i + J] = Fb[3 * i + J] - aN / cm;
                }
            }
            lin_stress(Fp, mup, lamp, Fip, Pp, mp);
            lin_stress(Fm, mum, lamm, Fim, Pm, mm);
            status = 0;
        } else if (!(Jb > 0.0)) {
            status = 2;
        } else {
            double adjb[9];
            adj3(Fb, adjb);
#pragma unroll
            for (int i = 0; i < 3; ++i) v[i] = (adjb[0 + i] * N[0] + adjb[3 + i] * N[1] + adjb[6 + i] * N[2]) / Jb;
            const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
            for (int i = 0; i < 3; ++i) mb[i] = v[i] / nv;
            bp = -cp / nv;
            bm = cm / nv;
            if (a.warm) {
#pragma unroll
                for (int i = 0; i < 3; ++i) a3[i] = a.a_prev[(long long)i * a.nc + ic];
                const double b0 = a3[0] * mb[0] + a3[1] * mb[1] + a3[2] * mb[2];
                if (!(bp < b0 && b0 < bm)) a3[0] = a3[1] = a3[2] = 0.0;
            }
            for (;;) {
                const double av = a3[0] * v[0] + a3[1] * v[1] + a3[2] * v[2];
                const double Jp = (1.0 + av / cp) * Jb, Jm = (1.0 - av / cm) * Jb;
                if (!(Jp > 0.0 && Jm > 0.0)) {
                    status = 3;
                    break;
                }
                double Fp[9], Fm[9];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int J = 0; J < 3; ++J) {
                        const double aN = a3[i] * N[J];
                        Fp[3 * i + J] = Fb[3 * i + J] + aN / cp;
                        Fm[3 * i + J] = Fb[3 * i + J] - aN / cm;
                    }
                nh_stress(Fp, Jp, mup, lamp, Fip, Pp, mp);
                nh_stress(Fm, Jm, mum, lamm, Fim, Pm, mm);
                double tp[3], tm[3], f[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    tp[i] = Pp[3 * i] * N[0] + Pp[3 * i + 1] * N[1] + Pp[3 * i + 2] * N[2];
                    tm[i] = Pm[3 * i] * N[0] + Pm[3 * i + 1] * N[1] + Pm[3 * i + 2] * N[2];
                    f[i] = tp[i] - tm[i];
                }
                const double err = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
                const double ntp = sqrt(tp[0] * tp[0] + tp[1] * tp[1] + tp[2] * tp[2]);
                const double ntm = sqrt(tm[0] * tm[0] + tm[1] * tm[1] + tm[2] * tm[2]);
                if (!(err == err)) {
                    status = 3;
                    break;
                }
                if (err <= 1e-12 * fmax(fmax(ntp, ntm), floor_t)) {
                    status = 0;
                    break;
                }
                double gp[3], gm[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    gp[i] = Fip[i] * N[0] + Fip[3 + i] * N[1] + Fip[6 + i] * N[2];
                    gm[i] = Fim[i] * N[0] + Fim[3 + i] * N[1] + Fim[6 + i] * N[2];
                }
                const double kp = (lamp + mp) / cp, km = (lamm + mm) / cm, d0 = mup / cp + mum / cm;
                double D[6];   // symmetric: 00 01 02 11 12 22
                D[0] = d0 + kp * gp[0] * gp[0] + km * gm[0] * gm[0];
                D[1] = kp * gp[0] * gp[1] + km * gm[0] * gm[1];
                D[2] = kp * gp[0] * gp[2] + km * gm[0] * gm[2];
                D[3] = d0 + kp * gp[1] * gp[1] + km * gm[1] * gm[1];
                D[4] = kp * gp[1] * gp[2] + km * gm[1] * gm[2];
                D[5] = d0 + kp * gp[2] * gp[2] + km * gm[2] * gm[2];
                double Di[6];
                sym3_inv(D, Di);
                double da[3];
                sym3_mul(Di, f, da);
                const double nda = sqrt(da[0] * da[0] + da[1] * da[1] + da[2] * da[2]);
                const double na = sqrt(a3[0] * a3[0] + a3[1] * a3[1] + a3[2] * a3[2]);
                if (nda <= 1e-13 * fmax(na, 1e-3)) {
                    status = 0;
                    break;
                }
                if (iters >= a.maxit) break;
                double a1[3] = {a3[0] - da[0], a3[1] - da[1], a3[2] - da[2]};
                const double b1 = a1[0] * mb[0] + a1[1] * mb[1] + a1[2] * mb[2];
                if (!(bp < b1 && b1 < bm)) {
                    const double b0 = a3[0] * mb[0] + a3[1] * mb[1] + a3[2] * mb[2];
                    const double bc = (b1 <= bp) ? bp : bm;
                    const double bs = 0.5 * (b0 + bc);
#pragma unroll
                    for (int i = 0; i < 3; ++i) a1[i] += (bs - b1) * mb[i];
                    ++nbp;
                }
#pragma unroll
                for (int i = 0; i < 3; ++i) a3[i] = a1[i];
                ++iters;
            }
        }
        double Pb[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) Pb[c] = (status == 0) ? cp * Pp[c] + cm * Pm[c] : 0.0;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            a.P[c * a.n + vox] = Pb[c];
            sums[c] += Pb[c];
            sums[9 + c] += (status == 0) ? cp * Pp[c] : 0.0;
            sums[18 + c] += (status == 0) ? cm * Pm[c] : 0.0;
        }
        sums[27] += (status == 0) ? 0.0 : 1.0;
        sums[28] += iters;
        sums[29] += nbp;
        sums[30] = fmax(sums[30], (double)iters);
#pragma unroll
        for (int i = 0; i < 3; ++i) a.a_out[(long long)i * a.nc + ic] = a3[i];
        if (a.a_full)
#pragma unroll
            for (int i = 0; i < 3; ++i) a.a_full[i * a.n + vox] = a3[i];
        if (a.iters_full) a.iters_full[vox] = iters;

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
        double gp[3], gm[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            gp[i] = Fip[i] * N[0] + Fip[3 + i] * N[1] + Fip[6 + i] * N[2];
            gm[i] = Fim[i] * N[0] + Fim[3 + i] * N[1] + Fim[6 + i] * N[2];
        }
        const double kp = (lamp + mp) / cp, km = (lamm + mm) / cm, d0 = mup / cp + mum / cm;
        double D[6];
        D[0] = d0 + kp * gp[0] * gp[0] + km * gm[0] * gm[0];
        D[1] = kp * gp[0] * gp[1] + km * gm[0] * gm[1];
        D[2] = kp * gp[0] * gp[2] + km * gm[0] * gm[2];
        D[3] = d0 + kp * gp[1] * gp[1] + km * gm[1] * gm[1];
        D[4] = kp * gp[1] * gp[2] + km * gm[1] * gm[2];
        D[5] = d0 + kp * gp[2] * gp[2] + km * gm[2] * gm[2];
        double Di[6];
        sym3_inv(D, Di);
        // dB_{k,(pq)} = B+_{k,(pq)} - B-_{k,(pq)}
        double dB[27];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const double bpl = (k == p ? mup * N[q] : 0.0) + lamp * gp[k] * Fip[3 * q + p] + mp * gp[p] * Fip[3 * q + k];
                    const double bmi = (k == p ? mum * N[q] : 0.0) + lamm * gm[k] * Fim[3 * q + p] + mm * gm[p] * Fim[3 * q + k];
                    dB[9 * k + 3 * p + q] = bpl - bmi;
                }
        // W_{l,(pq)} = sum_k Dinv_lk dB_{k,(pq)}
        double W[27];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const double b0 = dB[r], b1 = dB[9 + r], b2 = dB[18 + r];
            W[r] = Di[0] * b0 + Di[1] * b1 + Di[2] * b2;
            W[9 + r] = Di[1] * b0 + Di[3] * b1 + Di[4] * b2;
            W[18 + r] = Di[2] * b0 + Di[4] * b1 + Di[5] * b2;
        }
        int idx = 0;
        for (int r = 0; r < 9; ++r) {
            const int i = r / 3, J = r % 3;
            for (int s = (a.A_full ? 0 : r); s < 9; ++s) {
                const int k = s / 3, L = s % 3;
                const double corr = dB[r] * W[s] + dB[9 + r] * W[9 + s] + dB[18 + r] * W[18 + s];
                const double val = cp * nh_tangent(Fip, mup, lamp, mp, i, J, k, L) +
                                   cm * nh_tangent(Fim, mum, lamm, mm, i, J, k, L) - corr;
                if (a.A_full) a.A_full[(long long)(9 * r + s) * a.n + vox] = val;
                if (a.Acomp && s >= r) a.Acomp[(long long)ic * 45 + idx++] = T(val);
            }
        }
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
__device__ __forceinline__ void material_reduce_body(const double* pp, int nbp, const double* pl, int nbl,
                                                     double* out) {
    // out[0..19) = sums over pure blocks, out[19..50) = sums over laminate blocks (index 49 = max)
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

__global__ void __launch_bounds__(256) k_material_reduce(const double* pp, int nbp, const double* pl, int nbl,
                                                         double* out) {
    material_reduce_body(pp, nbp, pl, nbl, out);
}

// one workgroup per RVE
__global__ void __launch_bounds__(256) k_material_reduce_b(const MatReduceArgs* __restrict__ red) {
    const MatReduceArgs r = red[blockIdx.x];
    material_reduce_body(r.pp, r.nbp, r.pl, r.nbl, r.out);
}

int material_blocks_pure(long long n) {
    long long b = (n + 255) / 256;
    return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}
int material_blocks_laminate(int nc) {
    int b = (nc + 127) / 128;
    return b < 1 ? 1 : (b < 4096 ? b : 4096);
}

template <typename T>
hipError_t launch_material(const MatArgs<T>& a, int nbp, int nbl, double* sums_out, hipStream_t s) {
    hipLaunchKernelGGL(k_material_pure<T>, dim3(nbp), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.nc > 0) {
        hipLaunchKernelGGL(k_material_laminate<T>, dim3(nbl), dim3(128), 0, s, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_material_reduce, dim3(1), dim3(256), 0, s, a.partials, nbp, a.partials2,
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
    hipLaunchKernelGGL(k_material_reduce_b, dim3(nrve), dim3(256), 0, s, dev_red);
    return hipGetLastError();
}

template hipError_t launch_material<float>(const MatArgs<float>&, int, int, double*, hipStream_t);
template hipError_t launch_material<double>(const MatArgs<double>&, int, int, double*, hipStream_t);
template hipError_t launch_material_batch<float>(const MatArgs<float>*, const BatchLaunch&, const BatchLaunch&,
                                                 const MatReduceArgs*, int, hipStream_t);
template hipError_t launch_material_batch<double>(const MatArgs<double>*, const BatchLaunch&, const BatchLaunch&,
                                                  const MatReduceArgs*, int, hipStream_t);

}  // namespace combo
