// Argument block and launcher of the pointwise constitutive update.
#pragma once

#include "common.h"

namespace combo {

template <typename T>
struct MatArgs {
    long long n;            // voxels
    int nc;                 // composite voxels
    const double* F_old;    // [9][n]
    const double* dF;       // [9][n] or null
    double s;               // step length applied to dF
    double dFbar[9];        // homogeneous increment added to every voxel
    double* F_new;          // [9][n] receives F_old + s dF + dFbar
    double* P;              // [9][n]
    const int* slot;        // [n]: -1 matrix, -2 inclusion, >= 0 composite index
    double mu[2], lam[2];   // phase 0 = matrix, 1 = inclusion
    const int* comp_vox;    // [nc] voxel of each composite
    const double* cc;       // [nc] inclusion fraction c+
    const double* NN;       // [3][nc] unit normal out of the inclusion
    const double* a_prev;   // [3][nc] warm start of the jump vector
    double* a_out;          // [3][nc]
    int warm;
    int maxit;
    int law;                // kLawNeoHooke or kLawLinear
    T* Sinv;                // [9][n] tangent state at state_pos(voxel) (null: not wanted)
    T* sm;                  // [n]
    int n1, xm, xwbits;     // state layout (see state_pos)
    T* Acomp;               // [nc][45]
    double* A_full;         // [81][n] full FP64 tangent (diagnostics) or null
    double* a_full;         // [3][n] jump vector per voxel (diagnostics) or null
    int* iters_full;        // [n] laminate updates per voxel (diagnostics) or null
    double* partials;       // [blocks_pure][19]
    double* partials2;      // [blocks_laminate][31]
};

// Constitutive laws: finite-strain Neo-Hooke with the Newton-Raphson laminate, or
// small-strain isotropic elasticity with the closed-form laminate.
constexpr int kLawNeoHooke = 0;
constexpr int kLawLinear = 1;

// Layout of the reduced sums written by launch_material (50 doubles):
//   [0, 9)   sum of P over matrix voxels       [9, 18)  over inclusion voxels
//   [18]     pure voxels with det F <= 0
//   [19, 28) sum of P_box over composites      [28, 37) sum of c+ P+     [37, 46) sum of c- P-
//   [46]     failed laminates   [47] laminate updates   [48] back-projections   [49] max updates
constexpr int kSumsLen = 50;

__host__ __device__ inline void sym3_inv(const double* D, double* Di) {
    const double c00 = D[3] * D[5] - D[4] * D[4];
    const double c01 = D[2] * D[4] - D[1] * D[5];
    const double c02 = D[1] * D[4] - D[2] * D[3];
    const double c11 = D[0] * D[5] - D[2] * D[2];
    const double c12 = D[1] * D[2] - D[0] * D[4];
    const double c22 = D[0] * D[3] - D[1] * D[1];
    const double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
    const double id = 1.0 / det;
    Di[0] = c00 * id;
    Di[1] = c01 * id;
    Di[2] = c02 * id;
    Di[3] = c11 * id;
    Di[4] = c12 * id;
    Di[5] = c22 * id;
}

__host__ __device__ inline void sym3_mul(const double* S, const double* x, double* y) {
    y[0] = S[0] * x[0] + S[1] * x[1] + S[2] * x[2];
    y[1] = S[1] * x[0] + S[3] * x[1] + S[4] * x[2];
    y[2] = S[2] * x[0] + S[4] * x[1] + S[5] * x[2];
}

int material_blocks_pure(long long n);
int material_blocks_laminate(int nc);
template <typename T>
hipError_t launch_material(const MatArgs<T>& a, int nbp, int nbl, double* sums_out, hipStream_t s);

// Batched material update: per-RVE MatArgs and tile maps for the pure and the
// laminate kernels, then one reduction workgroup per RVE (red[i] describes RVE i).
struct MatReduceArgs {
    const double* pp;   // pure partials [nbp][19]
    int nbp;
    const double* pl;   // laminate partials [nbl][31]
    int nbl;
    double* out;        // [kSumsLen]
};
template <typename T>
hipError_t launch_material_batch(const MatArgs<T>* dev_args, const BatchLaunch& pure, const BatchLaunch& lam,
                                 const MatReduceArgs* dev_red, int nrve, hipStream_t s);

}  // namespace combo
