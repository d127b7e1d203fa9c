// Argument blocks and launchers of the ComBo HIP kernels.
#pragma once

#include "common.h"

namespace combo {

// Scalars of one conjugate-gradient solve, kept on the device so that a CG
// iteration needs no host round trip.
struct CGState {
    double rho;     // <r, r>_K of the current residual
    double rho0;    // <b, b>_K
    double alpha;
    double beta;
    double tol2;    // tol_cg^2
    double eta2;    // residual kernels: sum over frequencies of |G P|^2 (times n)
    int iter;
    int maxit;
    int done;       // 1 once converged or failed: every later kernel of the solve returns at once
    int status;     // 0 ok, 1 breakdown (NaN), 2 iteration limit, 3 negative curvature (<p, Ap> <= 0)
};

// Tangent state of the pointwise law in the precision T of the linear solves.
template <typename T>
struct TangentState {
    // all three arrays are indexed by state_pos(voxel)
    const int* slot;    // [n]: -1 matrix, -2 inclusion, >= 0 index of a composite voxel
    const T* Sinv;      // [9][n] F^{-1} of pure voxels (row-major)
    const T* sm;        // [n] mu - lambda ln J of pure voxels
    const T* Acomp;     // [nc][45] packed upper triangle of the 9x9 composite tangent
    T mu[2], lam[2];
    long long n;
};

enum XMode {
    X_CG = 0,        // spectrum -> C2R -> A:(.) -> R2C -> spectrum      (CG operator)
    X_RHS_E = 1,     // constant E -> A:E -> R2C -> spectrum               (tangent right-hand side)
    X_AVG = 2,       // spectrum -> C2R/n + E -> A:(.) -> row sums          (tangent column average)
    X_FWD_REAL = 3,  // real FP64 field -> R2C -> spectrum                  (residual)
    X_INV_REAL = 4   // spectrum -> C2R/n -> real FP64 field                (Newton update)
};

template <typename T>
struct XArgs {
    Grid g;
    AxisPlan plan;
    int R;                      // rows (y, z pairs) per workgroup
    const cpx<T>* tw;           // twiddles of n1
    const cpx<T>* in;           // [9][n3*n2][nh]
    cpx<T>* out;                // [9][n3*n2][nh]
    const double* real_in;      // [9][n]
    double* real_out;           // [9][n]
    const T* real_in_t;         // [9][n] in the pass's precision (used instead of real_in if set)
    T* real_out_t;              // [9][n] in the pass's precision (used instead of real_out if set)
    double scale;               // 1/n for X_AVG and X_INV_REAL
    TangentState<T> ts;
    double E[9];
    double* partials;           // X_AVG: [gridDim.x][9]
    const CGState* st;          // X_CG: skip when st->done
    int skip_done;              // other modes: skip as well when st->done (CG operator of the staggered grid)
};

template <typename T>
struct YArgs {
    Grid g;
    AxisPlan plan;
    int TX;                     // x frequencies per tile
    int ntile;                  // tiles per z plane
    const cpx<T>* tw;           // twiddles of n2
    const cpx<T>* in;
    cpx<T>* out;
    const CGState* st;          // skip when non-null and st->done
};

// Z passes: T = precision of the spectra, TU = precision of the CG vectors.
template <typename T, typename TU>
struct ZArgs {
    Grid g;
    AxisPlan plan;
    int TX;                     // elements of the (y, x) frequency plane per tile
    const cpx<T>* tw;           // twiddles of n3
    const cpx<T>* in;           // [6][n3][n2*nh]
    cpx<T>* out;                // [6][n3][n2*nh]
    cpx<TU>* x;                 // CG vectors [3][n3][n2*nh]
    cpx<TU>* r;
    cpx<TU>* p;
    cpx<TU>* q;
    double mu0, kappa0, inv_n;
    double* partials;           // per-workgroup partial sums
    double* partials2;
    CGState* st;
};

template <typename TU>
struct UArgs {
    Grid g;
    cpx<TU>* x;
    cpx<TU>* r;
    const cpx<TU>* p;
    const cpx<TU>* q;
    double mu0, kappa0;
    double* partials;
    const CGState* st;
};

// Tile geometry chosen on the host.
struct PassShape {
    int xR;     // rows per x-pass workgroup
    int yTX;    // tile width of the y passes
    int zTX;    // tile width of the z passes
};

// Launchers (fft_kernels.hip).  All enqueue on `s` and return hipError_t.
// Launchers (fft_kernels.hip).  All enqueue on `s` and return hipError_t.  With
// a BatchLaunch, `a` only selects the kernel variant (all RVEs of the batch share
// its grid) and the per-RVE arguments come from b->args.
template <typename T> hipError_t launch_x(int mode, const XArgs<T>& a, hipStream_t s, int* nblocks_out = nullptr,
                                          const BatchLaunch* b = nullptr);
template <typename T> hipError_t launch_y(int dir, const YArgs<T>& a, hipStream_t s, const BatchLaunch* b = nullptr);
// z modes
enum ZMode { Z_CG = 0, Z_RHS = 1, Z_INV_CG = 2, Z_INV_PLAIN = 3, Z_PROJ = 4 };
template <typename T, typename TU> hipError_t launch_z(int mode, const ZArgs<T, TU>& a, hipStream_t s,
                                                       int* nblocks_out = nullptr, const BatchLaunch* b = nullptr);
template <typename TU> hipError_t launch_update(const UArgs<TU>& a, hipStream_t s, int* nblocks_out = nullptr,
                                               const BatchLaunch* b = nullptr);
// anti-Hermitian projection of the x = 0 frequency plane of the CG vector a.r
template <typename TU> hipError_t launch_antiherm(const UArgs<TU>& a, hipStream_t s, const BatchLaunch* b = nullptr);
int blocks_antiherm(const Grid& g);
// finalisers (one workgroup per RVE): reduce `count` partials in fixed order
enum FinMode { FIN_ALPHA = 0, FIN_BETA = 1, FIN_RHS = 2 };
struct FinArgs {
    CGState* st;
    const double* partials;
    const double* partials2;
    int count;
    double tol2;
    int maxit;
};
// single: one FinArgs by value; batched: nrve FinArgs in device memory
hipError_t launch_finalize(int mode, const FinArgs& f, hipStream_t s, const FinArgs* dev_batch = nullptr, int nrve = 1);
hipError_t launch_reduce_columns(const double* partials, int rows, int cols, double* out, hipStream_t s);

// tile widths the y and z launchers use (two-stage fast path or LDS Stockham)
template <typename T> int y_tile(const Grid& g);
template <typename T> int z_tile(const Grid& g);

// (m, W) of the wavefront x pass for a row length n1; m = W = 0 if it has none
void xpass_wave_shape(int n1, int& m, int& w);

// workgroups of an x pass in `mode` (the two-stage kernel serves X_CG and X_AVG)
int blocks_x(const Grid& g, int R, int mode, bool is_float);
// two-stage x pass for rows of n1: number of variants (0: there is none, and the
// tangent state keeps the wavefront kernel's lane order, see state_pos), and rows
// per workgroup of the variant that runs for variant v
int xpass_lds_variants(int n1);
int xpass_lds_rows(int n1, int v, bool is_float);
int xpass_lds_pick(int n1, int v, bool is_float);   // the variant that runs for variant v
// variants of the two-stage y/z passes for rows of L (0: none)
template <typename T> int fft2_variants(int L);
int blocks_y(const Grid& g, int TX);
int blocks_z(const Grid& g, int TX);
int blocks_u(const Grid& g);

}  // namespace combo
