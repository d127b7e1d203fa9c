// Staggered grid with the doubly-fine material grid (DFMG) law (paper App. A):
// argument blocks and launchers.
//
// Storage ("shifted" layout of the staggered fields): the gradient of the
// displacement is kept as forward differences H_aJ = D_J^+ U_a in every
// component, so that a single Fourier multiplier per axis serves all nine
// components.  The staggered value itself is F_aJ[xi] = H_aJ[xi] on the diagonal
// and F_aJ[xi] = D_J^- U_a[xi] = H_aJ[xi - e_J] off it (a backward difference at
// xi is the forward difference at xi - e_J); stresses are kept the same way,
// Q_aJ[xi] = P_aJ[xi + e_J] off the diagonal.
//
// Doubly-fine cells: cell xi has eight, (xi, l) with l in {0, 1}^3.  The one at l
// holds the diagonal F_aa[xi] and, for a != b, F_ab[xi + l_a e_a + l_b e_b] (the
// edge value of F_ab on its boundary); its law is that of cell xi.  The DFMG
// stress is P_aa[xi] = 1/8 sum_l P(xi, l)_aa and, for a != b,
// P_ab[p] = 1/8 sum_l P(p - l_a e_a - l_b e_b, l)_ab: every doubly-fine cell
// touching the edge p.  This is the sum of eq. constitutive_law with every term
// named by the doubly-fine cell it evaluates.
#pragma once

#include "kernels.h"

namespace combo {

template <typename T>
struct DfmgArgs {
    int n1, n2, n3;
    long long n;             // cells
    int nc;                  // composite cells
    const double* F_old;     // [9][n] shifted layout
    const double* dF;        // [9][n] or null
    double s;                // step length applied to dF
    double dFbar[9];         // homogeneous increment
    double* F_new;           // [9][n] F_old + s dF + dFbar
    const int* slot;         // [n]: -1 matrix, -2 inclusion, >= 0 composite index
    const int* comp_vox;     // [nc]
    const double* cc;        // [nc] c+
    const double* NN;        // [3][nc]
    const double* a_prev;    // [3][8][nc] warm starts of the doubly-fine laminates (index (i 8 + l) nc + ic)
    double* a_out;           // [3][8][nc]
    int warm, maxit;
    double mu[2], lam[2];
    double* Pd;              // [9][8][n] stress of every doubly-fine cell (index (c 8 + l) n + cell)
    T* Ad;                   // [nc][8][45] packed tangent of composite doubly-fine cells
    double* partials;        // pure kernel: [blocks][19]
    double* partials2;       // laminate kernel: [blocks][31]
};

// F_new = F_old + s dF + dFbar over 9 n values
template <typename T> hipError_t launch_dfmg_update(const DfmgArgs<T>& a, hipStream_t s);
// law of every doubly-fine cell, then the reductions into sums_out (kSumsLen layout of
// material.h, stresses weighted 1/8); stresses in a.Pd
int dfmg_blocks_pure(long long n);
int dfmg_blocks_laminate(int nc);
template <typename T> hipError_t launch_dfmg_law(const DfmgArgs<T>& a, double* sums_out, hipStream_t s);

// Tangent action on a field dH in the shifted layout, summed per destination.
// Each doubly-fine cell (c, l) gives dP(c, l) = A(c, l) : dF(c, l).  Its diagonal
// components belong to cell c; its component (a, b), a != b, to the edge stored
// at Q_ab[c + l_a e_a + (l_b - 1) e_b] (shifted layout).  The kernel adds the
// contributions that land on cell c itself into own[9][c] (weight 1/8) and the
// rest, summed over l_d of the third axis d, into part[18][c]: for the ordered
// pair p = (a, b) (order (0,1) (0,2) (1,0) (1,2) (2,0) (2,1)) the offsets
// e_a, -e_b and e_a - e_b in part[3 p + k], k = 0, 1, 2.  Pure cells evaluate the
// Neo-Hooke tangent from the deformation F of the last law evaluation (FP64 det F
// and ln J); composite cells read their doubly-fine laminate tangents Ad.
template <typename T>
struct DfmgActArgs {
    int n1, n2, n3;
    long long n;
    const T* dH;             // [9][n] shifted layout
    const double* F;         // [9][n] shifted layout, the deformation the law was evaluated at
    T* own;                  // [9][n]
    T* part;                 // [18][n]
    const int* slot;
    const T* Ad;             // [nc][8][45]
    double mu[2], lam[2];
    const CGState* st;       // skip when st->done (null: always run)
};
template <typename T> hipError_t launch_dfmg_action(const DfmgActArgs<T>& a, hipStream_t s);

// Q = own + the neighbours' parts (see DfmgActArgs): the DFMG sum of the action.
template <typename T>
struct DfmgSumArgs {
    int n1, n2, n3;
    long long n;
    const T* own;
    const T* part;
    T* Q;                    // [9][n] shifted layout
    const CGState* st;
};
template <typename T> hipError_t launch_dfmg_sum(const DfmgSumArgs<T>& a, hipStream_t s);

// DFMG sum of doubly-fine cell stresses into a field in the shifted layout:
// Q_aa[xi] = 1/8 sum_l Pd_aa(xi, l), Q_ab[xi] = P_ab[xi + e_b] (a != b).
template <typename TI>
struct DfmgGatherArgs {
    int n1, n2, n3;
    long long n;
    const TI* Pd;            // [9][8][n]
    double* Q;               // [9][n]
    const CGState* st;       // skip when st->done (null: always run)
};
template <typename TI> hipError_t launch_dfmg_gather(const DfmgGatherArgs<TI>& a, hipStream_t s);

// A uniform tensor E as a [9][n] field (add = 1: added to f); the same in both layouts.
struct UniformE {
    double v[9];
};
template <typename T> hipError_t launch_stag_uniform(T* f, long long n, const double E[9], int add, hipStream_t s);
// Per-workgroup FP64 sums of the nine components of a [9][n] field: partials [stag_sum_blocks(n)][9].
int stag_sum_blocks(long long n);
template <typename T> hipError_t launch_stag_field_sums(const T* f, long long n, double* partials, hipStream_t s);

// Natural staggered layout <-> shifted layout of a [9][n] field:
// dir = +1: out_aJ[xi] = in_aJ[xi + e_J] (natural -> shifted), dir = -1 the inverse;
// diagonal components are copied.  in and out must not overlap.
hipError_t launch_stag_shift(const double* in, double* out, int n1, int n2, int n3, int dir, hipStream_t s);

}  // namespace combo
