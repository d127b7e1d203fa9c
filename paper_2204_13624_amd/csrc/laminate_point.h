// The rank-one laminate of one composite point (paper Sec. 4), shared by the
// per-voxel law (material_kernels.hip) and the doubly-fine material grid law of
// the staggered grid (dfmg_kernels.hip).  FP64 throughout.
//
//   F+- = F_box +- a (x) N / c+-                                  (eq. Fpm)
//   f(a) = (P+ - P-) N                                            (eq. tractionbalance)
//   Delta = sum_+- (mu I + (lambda + m) g (x) g) / c,  g = F^{-T} N  (eq. hessian)
//   J+- = (1 +- a.v / c+-) J_box, v = F_box^{-T} N                (eq. Jpm)
// Newton-Raphson (Alg. 1) with the selective back-projection of Alg. 2 on the
// admissible interval beta_c^+ < a.m < beta_c^- (eq. matrixlemma); stress
// P_box = c+ P+ + c- P- (eq. Peff:Seff) and the consistent tangent
//   A_box = c+ A+ + c- A- - dB^T Delta^{-1} dB,
//   B_{k,pq} = sum_J N_J A_kJpq = mu d_kp N_q + lambda g_k Finv_qp + m g_p Finv_qk.
// The small-strain law (kLawLinear) takes the closed-form jump a = -Delta^{-1} f(0).
// Stopping rule: |f| <= 1e-12 max(|P+ N|, |P- N|, 1e-3 max mu, 1e-2 max lambda) or a
// Newton correction |Delta^{-1} f| <= 1e-13 max(|a|, 1e-3); at most maxit updates.
#pragma once

#include <hip/hip_runtime.h>

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

// Result of one laminate solve.
struct LamPoint {
    int status;              // 0 ok, 1 iteration limit, 2 bad F_box, 3 inadmissible
    int iters, nbp;          // Newton updates, back-projections
    double a[3];             // jump vector
    double Pp[9], Pm[9];     // phase stresses
    double Fip[9], Fim[9];   // phase inverse deformations
    double mp, mm;           // mu - lambda ln J of the phases
};

// Laminate of one point at F_box = Fb with inclusion fraction cp and normal N.
// mats = {mu-, lambda-, mu+, lambda+}.  a_init (may be null) is a warm start,
// dropped if it is not admissible at Fb.
__device__ __forceinline__ void laminate_point(const double* Fb, double cp, const double* N, const double* mats,
                                               int law, int maxit, const double* a_init, LamPoint& o) {
    const double cm = 1.0 - cp;
    const double mum = mats[0], lamm = mats[1], mup = mats[2], lamp = mats[3];
    const double floor_t = fmax(1e-3 * fmax(mup, mum), 1e-2 * fmax(lamp, lamm));
    o.status = 1;
    o.iters = 0;
    o.nbp = 0;
    o.a[0] = o.a[1] = o.a[2] = 0.0;
    o.mp = o.mm = 0.0;
    const double Jb = det3(Fb);
    double v[3] = {0, 0, 0}, mb[3] = {0, 0, 0}, bp = 0.0, bm = 0.0;
    if (law == kLawLinear) {
        // closed form: one exact Newton step from a = 0 (the traction jump is linear in a)
        lin_stress(Fb, mup, lamp, o.Fip, o.Pp, o.mp);
        lin_stress(Fb, mum, lamm, o.Fim, o.Pm, o.mm);
        double f[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            f[i] = (o.Pp[3 * i] - o.Pm[3 * i]) * N[0] + (o.Pp[3 * i + 1] - o.Pm[3 * i + 1]) * N[1] +
                   (o.Pp[3 * i + 2] - o.Pm[3 * i + 2]) * N[2];
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
            o.a[i] = -da[i];
#pragma unroll
            for (int J = 0; J < 3; ++J) {
                const double aN = -da[i] * N[J];
                Fp[3 * i + J] = Fb[3 * i + J] + aN / cp;
                Fm[3 * i + J] = Fb[3 * i + J] - aN / cm;
            }
        }
        lin_stress(Fp, mup, lamp, o.Fip, o.Pp, o.mp);
        lin_stress(Fm, mum, lamm, o.Fim, o.Pm, o.mm);
        o.status = 0;
        return;
    }
    if (!(Jb > 0.0)) {
        o.status = 2;
        return;
    }
    double adjb[9];
    adj3(Fb, adjb);
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] = (adjb[0 + i] * N[0] + adjb[3 + i] * N[1] + adjb[6 + i] * N[2]) / Jb;
    const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) mb[i] = v[i] / nv;
    bp = -cp / nv;
    bm = cm / nv;
    double* a3 = o.a;
    if (a_init) {
#pragma unroll
        for (int i = 0; i < 3; ++i) a3[i] = a_init[i];
        const double b0 = a3[0] * mb[0] + a3[1] * mb[1] + a3[2] * mb[2];
        if (!(bp < b0 && b0 < bm)) a3[0] = a3[1] = a3[2] = 0.0;
    }
    for (;;) {
        const double av = a3[0] * v[0] + a3[1] * v[1] + a3[2] * v[2];
        const double Jp = (1.0 + av / cp) * Jb, Jm = (1.0 - av / cm) * Jb;
        if (!(Jp > 0.0 && Jm > 0.0)) {
            o.status = 3;
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
        nh_stress(Fp, Jp, mup, lamp, o.Fip, o.Pp, o.mp);
        nh_stress(Fm, Jm, mum, lamm, o.Fim, o.Pm, o.mm);
        double tp[3], tm[3], f[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            tp[i] = o.Pp[3 * i] * N[0] + o.Pp[3 * i + 1] * N[1] + o.Pp[3 * i + 2] * N[2];
            tm[i] = o.Pm[3 * i] * N[0] + o.Pm[3 * i + 1] * N[1] + o.Pm[3 * i + 2] * N[2];
            f[i] = tp[i] - tm[i];
        }
        const double err = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        const double ntp = sqrt(tp[0] * tp[0] + tp[1] * tp[1] + tp[2] * tp[2]);
        const double ntm = sqrt(tm[0] * tm[0] + tm[1] * tm[1] + tm[2] * tm[2]);
        if (!(err == err)) {
            o.status = 3;
            break;
        }
        if (err <= 1e-12 * fmax(fmax(ntp, ntm), floor_t)) {
            o.status = 0;
            break;
        }
        double gp[3], gm[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            gp[i] = o.Fip[i] * N[0] + o.Fip[3 + i] * N[1] + o.Fip[6 + i] * N[2];
            gm[i] = o.Fim[i] * N[0] + o.Fim[3 + i] * N[1] + o.Fim[6 + i] * N[2];
        }
        const double kp = (lamp + o.mp) / cp, km = (lamm + o.mm) / cm, d0 = mup / cp + mum / cm;
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
            o.status = 0;
            break;
        }
        if (o.iters >= maxit) break;
        double a1[3] = {a3[0] - da[0], a3[1] - da[1], a3[2] - da[2]};
        const double b1 = a1[0] * mb[0] + a1[1] * mb[1] + a1[2] * mb[2];
        if (!(bp < b1 && b1 < bm)) {
            const double b0 = a3[0] * mb[0] + a3[1] * mb[1] + a3[2] * mb[2];
            const double bc = (b1 <= bp) ? bp : bm;
            const double bs = 0.5 * (b0 + bc);
#pragma unroll
            for (int i = 0; i < 3; ++i) a1[i] += (bs - b1) * mb[i];
            ++o.nbp;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) a3[i] = a1[i];
        ++o.iters;
    }
}

// Consistent tangent of a converged laminate point (status 0).  Writes the packed
// upper triangle (45 values, row-major r <= s) to `packed` (may be null) and, if
// `full` is not null, every entry (9 r + s) to full[(9 r + s) * fstride].
template <typename T>
__device__ __forceinline__ void laminate_tangent(const LamPoint& o, double cp, const double* N, const double* mats,
                                                 T* packed, double* full, long long fstride) {
    const double cm = 1.0 - cp;
    const double mum = mats[0], lamm = mats[1], mup = mats[2], lamp = mats[3];
    double gp[3], gm[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gp[i] = o.Fip[i] * N[0] + o.Fip[3 + i] * N[1] + o.Fip[6 + i] * N[2];
        gm[i] = o.Fim[i] * N[0] + o.Fim[3 + i] * N[1] + o.Fim[6 + i] * N[2];
    }
    const double kp = (lamp + o.mp) / cp, km = (lamm + o.mm) / cm, d0 = mup / cp + mum / cm;
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
                const double bpl = (k == p ? mup * N[q] : 0.0) + lamp * gp[k] * o.Fip[3 * q + p] + o.mp * gp[p] * o.Fip[3 * q + k];
                const double bmi = (k == p ? mum * N[q] : 0.0) + lamm * gm[k] * o.Fim[3 * q + p] + o.mm * gm[p] * o.Fim[3 * q + k];
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
        for (int s = (full ? 0 : r); s < 9; ++s) {
            const int k = s / 3, L = s % 3;
            const double corr = dB[r] * W[s] + dB[9 + r] * W[9 + s] + dB[18 + r] * W[18 + s];
            const double val = cp * nh_tangent(o.Fip, mup, lamp, o.mp, i, J, k, L) +
                               cm * nh_tangent(o.Fim, mum, lamm, o.mm, i, J, k, L) - corr;
            if (full) full[(long long)(9 * r + s) * fstride] = val;
            if (packed && s >= r) packed[idx++] = T(val);
        }
    }
}

}  // namespace combo
