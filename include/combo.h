/*
 * combo.h -- C-ABI of libcombo: FFT-based finite-strain homogenization with
 * composite boxels (ComBo) on one AMD Instinct MI355X (gfx950).
 *
 * The library solves the periodic homogenization problem of the paper
 * (Keshav, Fritzen, Kabel: "FFT-based homogenization at finite strains using
 * composite boxels", Sec. 2 eqs. Pbar, hom:start, equilibrium): given the
 * macroscopic deformation gradient Fbar, find the deformation gradient field
 * F = Fbar + Grad(periodic fluctuation) with Div P(F) = 0, where P is the
 * compressible Neo-Hookean law (Sec. 6.1) in pure voxels and the rank-one
 * laminate law of Sec. 4 (Alg. 1 Newton-Raphson for the jump vector with the
 * selective back-projection of Alg. 2, stress eq. Peff:Seff and the
 * consistent tangent that follows it) in composite voxels.  The equation
 * solved is the Lippmann-Schwinger equation (Sec. 3, eq. nonlinearLSE) by
 * Newton's method with a conjugate-gradient linear solver on the spectral
 * (Moulinec-Suquet) discretization.
 *
 * Conventions
 *   - Tensors are 3x3, stored row-major: component (i, J) at index 3*i + J
 *     (paper Sec. 1.5).  4th-order tangents are 9x9 row-major (row 3i+J,
 *     column 3k+L).
 *   - Grids are n1 x n2 x n3 voxels of a box l1 x l2 x l3 (boxels allowed);
 *     fields are structure-of-arrays [9][n3][n2][n1] (x fastest); scalar
 *     fields [n3][n2][n1]; normals [3][n3][n2][n1].
 *   - phase: 0 = matrix ("-"), 1 = inclusion ("+"), 2 = composite boxel.
 *     c = inclusion volume fraction c+ of a composite boxel, 0 < c < 1.
 *     N = unit interface normal pointing out of the inclusion (Sec. 2, 5.1).
 *     c and N are read only where phase == 2.
 *   - Materials: index 0 = matrix, 1 = inclusion, each (mu, lambda).
 *   - Every grid axis must be 1 or a product of 2s and 3s, at most 512
 *     (COMBO_E_SIZE otherwise).
 *
 * Ownership: the caller owns every pointer it passes.  set_* calls copy their
 * inputs; no caller pointer is kept after a call returns.  Output buffers are
 * written in place.  mem_kind tells whether caller pointers are host memory
 * (COMBO_MEM_HOST) or device memory of the context's GPU (COMBO_MEM_DEVICE).
 * The context owns all device memory it allocates; combo_destroy frees it.
 *
 * Errors: every call returns a status (COMBO_OK or a negative COMBO_E_*); no
 * exception crosses the ABI.  combo_last_error() gives a message.  Inputs are
 * validated on the host before any GPU work.  After a failed solve the output
 * buffers are unspecified, but stats (if given) is filled.
 *
 * Streams and threads: all GPU work of a context runs on its stream; calls
 * block until their results are ready.  A context is not thread-safe;
 * different contexts may be used from different threads.
 */
#ifndef COMBO_H
#define COMBO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COMBO_ABI_VERSION 7

typedef struct combo_ctx combo_ctx;
typedef struct combo_batch combo_batch;

enum combo_status {
    COMBO_OK = 0,
    COMBO_E_INVAL = -1,        /* invalid argument (null pointer, bad value) */
    COMBO_E_NOMEM = -2,        /* device or host allocation failed */
    COMBO_E_HIP = -3,          /* HIP runtime error / no usable GPU */
    COMBO_E_SIZE = -4,         /* grid size not supported */
    COMBO_E_NOCONV = -5,       /* Newton, CG or laminate did not converge */
    COMBO_E_INADMISSIBLE = -6, /* det F <= 0 (macroscopic or unrecoverable local) */
    COMBO_E_NUMERIC = -7,      /* NaN/Inf input or CG breakdown */
    COMBO_E_STATE = -8         /* call out of order (e.g. solve before set_grid) */
};

enum combo_mem { COMBO_MEM_HOST = 0, COMBO_MEM_DEVICE = 1 };

/* Precision of the conjugate-gradient linear solves (FFT, Green operator,
 * tangent action, CG vectors).  The material law, the laminate Newton, the
 * deformation and stress fields and the Newton residual are always FP64. */
enum combo_precision { COMBO_FP64 = 0, COMBO_MIXED = 1 };

enum combo_green { COMBO_GREEN_GAMMA0 = 0, COMBO_GREEN_G = 1 };

typedef struct {
    double mu;
    double lambda;
} combo_material;

/* Constitutive laws (combo_options.law).
 * COMBO_LAW_NEO_HOOKE: finite strain.  Pure voxels: compressible Neo-Hooke
 *   (paper Sec. 6.1); composite voxels: the rank-one laminate solved by
 *   Newton-Raphson with selective back-projection (Sec. 4, Alg. 1 and 2).
 * COMBO_LAW_LINEAR: infinitesimal strain (appendix cheat sheet, right column).
 *   F is read as I + grad u and P as the stress of eps = sym(F - I).  Pure voxels:
 *   sigma = lambda tr(eps) I + 2 mu eps; composite voxels: the laminate jump in
 *   closed form, a = Delta^{-1} N.(C- - C+) eps_box, with stress and tangent of
 *   the same table.  The problem is linear: one Newton step solves it up to the
 *   CG tolerance, and no det F or admissibility condition applies. */
#define COMBO_LAW_NEO_HOOKE 0
#define COMBO_LAW_LINEAR 1

typedef struct {
    int precision;            /* COMBO_FP64 or COMBO_MIXED */
    double tol_newton;        /* eta = |G[P]|_2 / (sqrt(n) |Pbar|_F) <= tol_newton */
    double tol_cg;            /* |r|_C0 / |b|_C0 <= tol_cg (mixed mode: at least 1e-5) */
    int max_newton;           /* Newton iterations per increment */
    int max_cg;               /* CG iterations per linear solve */
    int max_laminate;         /* laminate Newton updates per voxel (<= 64) */
    int n_increments;         /* load increments from <F_init> (or I) to Fbar */
    double mu0, kappa0;       /* reference medium C0 = mu0 Id + kappa0 I(x)I; <= 0: default */
    int warm_start_laminate;  /* start each laminate solve from the last accepted a */
    int want_tangent;         /* compute the effective tangent Abar */
    int max_step_halvings;    /* Newton step control */
    int max_cutbacks;         /* increment halvings */
    int graph_chunk;          /* CG iterations per captured HIP graph replay; 0 = plain launches */
    int autotune;             /* 1: pick the FFT schedule of the grid by timing (combo_autotune) before solving */
    int line_search;          /* 1 (default): a Newton step F + s dF is taken only if the residual decreases,
                                 eta(s) <= (1 - 1e-4 s) eta, halving s otherwise (max_step_halvings) */
    int law;                  /* COMBO_LAW_NEO_HOOKE (default) or COMBO_LAW_LINEAR */
    int batch_streams;        /* batches: at most this many lanes (streams), 0 = 8, at most 16; see combo_batch_solve */
} combo_options;

typedef struct {
    int status;
    int newton_iters;
    int cg_iters_total;       /* Newton solves only */
    int cg_iters_tangent;     /* effective-tangent solves */
    int increments_done;
    int step_halvings;
    int cutbacks;
    int laminate_iters_max;
    long long laminate_iters_total;
    long long laminate_backprojections;
    long long laminate_failures;
    double eta_final;
    double time_ms_total;
    double time_ms_cg;
    double time_ms_material;
    double time_ms_residual;
    double time_ms_tangent;
    int cg_truncations;       /* Newton steps whose CG stopped at negative curvature (truncated Newton) */
} combo_stats;

/* Library identification and messages ------------------------------------ */
int combo_abi_version(void);
const char* combo_strerror(int status);
/* Fill opt with the defaults: FP64, tol_newton 1e-8, tol_cg 1e-10, max_newton 30,
 * max_cg 5000, max_laminate 50, 1 increment, default C0, warm start on,
 * no tangent, 10 step halvings, 5 cutbacks, graph_chunk 0, no autotuning,
 * line search on, Neo-Hooke law, batch_streams 0 (8 lanes). */
void combo_default_options(combo_options* opt);

/* Host-only validation of a microstructure (no GPU needed).  Checks phase ids,
 * 0 < c < 1 and |N| = 1 (within 1e-6) where phase == 2, finite values.
 * Host pointers only.  Returns COMBO_OK or COMBO_E_INVAL; msg (may be NULL,
 * msg_len bytes) receives a description of the first problem. */
int combo_validate_microstructure(int n1, int n2, int n3, const uint8_t* phase, const double* c,
                                  const double* N, char* msg, int msg_len);
/* Returns COMBO_OK if n is 1 or a product of 2s and 3s not above 512. */
int combo_check_size(int n);

/* Context ------------------------------------------------------------------ */
/* Create a context on GPU `device` using `hip_stream` (a hipStream_t; NULL =
 * a stream the context creates and owns, non-blocking).  COMBO_E_HIP if no
 * usable GPU.  Device buffers given to any call are read and written on that
 * stream: work on other streams that produces them must be complete (or
 * ordered before the call) when the call is made.  Calls return after their
 * device outputs are written. */
int combo_create(combo_ctx** out, int device, void* hip_stream);
int combo_destroy(combo_ctx* ctx);
/* Message of the last failed call on ctx; owned by ctx, valid until the next call. */
const char* combo_last_error(const combo_ctx* ctx);

/* Grid and box (paper Sec. 2: the RVE [-l1/2, l1/2] x ...).  Resets the microstructure. */
int combo_set_grid(combo_ctx* ctx, int n1, int n2, int n3, double l1, double l2, double l3);
/* Discretization of the gradient (paper Sec. 3 compares several; the default is
 * the Fourier-polynomial scheme of Moulinec and Suquet).
 * COMBO_DISC_MS: grad_J -> i xi_J, xi_d = 2 pi k_d / l_d; the mean and every
 *   Nyquist plane of an even axis are projected out.
 * COMBO_DISC_WILLOT: Willot's rotated (HEX8R) scheme, the discretization of the
 *   paper's reference solutions: the displacement lives at voxel corners and the
 *   gradient at a voxel centre is the mean of the four edge differences per axis,
 *   grad_J -> k_J = (e^{i th_J} - 1)/h_J prod_{m != J} (1 + e^{i th_m})/2,
 *   th_d = 2 pi k_d / n_d.  Only the mean and modes on two or more Nyquist planes
 *   are projected out; an even n1 keeps its x-Nyquist plane.  Runs the same FFT
 *   passes with the rotated factors; combo_autotune tunes and caches its schedules
 *   separately ("mixed-willot" / "fp64-willot").  Batches: combo_batch_set_discretization.
 * COMBO_DISC_STAGGERED: the staggered grid of the paper's appendix (App. A): the
 *   displacement component U_a lives on the cell faces normal to e_a; F_aa (and P_aa)
 *   at the cell centre from forward differences, F_ab (a != b) on the cell edge at the
 *   lower corner in a and b from backward differences (eq. gradient_operator); the
 *   material law is the doubly-fine material grid average (eq. constitutive_law):
 *   each cell's eight doubly-fine cells evaluate the law of the cell (Neo-Hooke, or
 *   the laminate with one solve per doubly-fine cell) at the deformation assembled
 *   from the staggered values on their boundary.  Only the mean mode is projected
 *   out.  Fields passed in or out (F_init, F_out, P_out, combo_eval_law,
 *   combo_apply_green, combo_apply_operator) hold the staggered values: component
 *   (a, b) at index xi is the value at cell xi's own position of that component.
 *   Finite-strain law only, no batches.  The effective tangent (want_tangent) is the
 *   derivative of <P> with P the DFMG stress: nine CG solves with the DFMG tangent.
 * Rebuilds the grid's frequency data like combo_set_grid and therefore resets the
 * microstructure: call after combo_set_grid, before combo_set_microstructure. */
#define COMBO_DISC_MS 0
#define COMBO_DISC_WILLOT 1
#define COMBO_DISC_STAGGERED 2
int combo_set_discretization(combo_ctx* ctx, int disc);
/* The grid and box set by combo_set_grid (host only; COMBO_E_STATE before it). */
int combo_get_grid(const combo_ctx* ctx, int* n1, int* n2, int* n3, double* l1, double* l2, double* l3);
/* Materials (mu, lambda) for phase 0 (matrix) and 1 (inclusion); mu > 0, lambda >= 0. */
int combo_set_materials(combo_ctx* ctx, const combo_material mats[2]);
/* Per-voxel ComBo data (paper Sec. 4: volume fraction and laminate normal).
 * phase [n], c [n], N [3][n] in the layout above; mem_kind as documented. */
int combo_set_microstructure(combo_ctx* ctx, const uint8_t* phase, const double* c, const double* N,
                             int mem_kind);

/* Composite boxels from a fine binary image (paper Sec. 5).
 * chi: [n3 s3][n2 s2][n1 s1] bytes, x fastest, 1 = inclusion, 0 = matrix; the grid
 * (n1, n2, n3) and box (l1, l2, l3) are the context's (combo_set_grid), so a fine
 * voxel measures h_m = l_m / (n_m s_m).  Boxel (i, j, k) holds the fine voxels
 * [i s1, (i+1) s1) x [j s2, (j+1) s2) x [k s3, (k+1) s3).  Outputs, in the layout
 * of combo_set_microstructure: phase [n3][n2][n1] (0 matrix, 1 inclusion,
 * 2 composite), c [n3][n2][n1] = inclusion fraction of the boxel, N [3][n3][n2][n1]
 * = unit normal out of the inclusion for composite boxels, 0 elsewhere.
 * method COMBO_NORMALS_LAPLACE: interface weights w = |S * chi| of the periodic
 *   per-axis 3-point Laplacian weighted by r_m = h_i h_j / h_m (Sec. 5.2, [N.1]),
 *   second moment of w about the weighted barycentre of the interface and its
 *   smallest eigenvector ([N.2]), oriented by eq. normal:flip;
 * method COMBO_NORMALS_BARYCENTRE: N = (c- - c+) / |c- - c+| of the phase
 *   barycentres (eq. normal:kabel); (1, 0, 0) where the two coincide.
 * All of chi, phase, c and N are host or all device pointers (mem_kind); the
 * caller owns them.  Runs on the context's stream and returns when the outputs
 * are written.  COMBO_E_STATE without a grid, COMBO_E_INVAL for s_m < 1, a
 * method out of range, null pointers or an image value other than 0 and 1. */
#define COMBO_NORMALS_LAPLACE 0
#define COMBO_NORMALS_BARYCENTRE 1
int combo_image_to_boxels(combo_ctx* ctx, const uint8_t* chi, int s1, int s2, int s3, int method, uint8_t* phase,
                          double* c, double* N, int mem_kind);
/* combo_image_to_boxels followed by combo_set_microstructure with its outputs,
 * kept on the device. */
int combo_set_microstructure_from_image(combo_ctx* ctx, const uint8_t* chi, int s1, int s2, int s3, int method,
                                        int mem_kind);
/* combo_image_to_boxels for callers that cannot allocate device memory (tight
 * serving loops, code that must not call hipMalloc): the same kernels and
 * outputs, with every intermediate buffer (counters, block offsets, composite
 * list, packed fine words, moments) in one static device array of 64 MiB per
 * GPU, held from the library's first use on that GPU until the process ends.
 * No device or host memory is allocated by this call.  chi, phase, c and N are
 * device pointers of the context's GPU (layouts as combo_image_to_boxels).
 * Limits: 12 bytes per boxel (+ 8 more with s = (4, s2, s3), s2 s3 <= 16) plus
 * 104 bytes per composite boxel must fit in the 64 MiB; a grid that does not
 * fit is refused with COMBO_E_SIZE before any GPU work, and a composite count
 * that does not fit with COMBO_E_SIZE after phase and c are written (N is then
 * unspecified).  Every call on one GPU uses the same array and leaves its
 * contents behind: calls that overlap in time on one GPU (from several host
 * threads, or on several streams) race and must be serialised by the caller.
 * Returns after the outputs are written (one host wait in the middle for the
 * composite count). */
int combo_image_to_boxels_static(combo_ctx* ctx, const uint8_t* chi, int s1, int s2, int s3, int method,
                                 uint8_t* phase, double* c, double* N);
int combo_set_options(combo_ctx* ctx, const combo_options* opt);

/* Solve HOM for the macroscopic deformation gradient Fbar (host, 9 doubles,
 * det > 0).  Starts from F_init ([9][n], or NULL for F = I) and follows
 * n_increments load steps to Fbar.  Outputs (each may be NULL): F_out and
 * P_out [9][n] in mem_kind memory; Pbar (host, 9) = <P> (eq. Pbar); Abar
 * (host, 81) = dPbar/dFbar when opt.want_tangent; Pbar_phase (host, 18) =
 * volume averages of P over the inclusion (first 9) and matrix (last 9),
 * counting c+ P+ and c- P- inside composite voxels; stats (host). */
int combo_solve(combo_ctx* ctx, const double Fbar[9], const double* F_init, double* F_out, double* P_out,
                double Pbar[9], double Abar[81], double Pbar_phase[18], combo_stats* stats, int mem_kind);

/* Diagnostics used by the test-suite ------------------------------------- */
/* Evaluate the pointwise law (Sec. 6.1 in pure voxels, Sec. 4 Alg. 1 + 2 in
 * composite voxels, cold start a = 0) at the field F [9][n] (staggered grid: the
 * DFMG law; A, a and iters must then be NULL).  Writes P [9][n]
 * (may be NULL), the tangent dP/dF A [81][n] (may be NULL; FP64), the jump
 * vector a [3][n] (may be NULL; 0 in pure voxels) and laminate updates
 * iters [n] (may be NULL; int32, 0 in pure voxels).  Also leaves the tangent
 * state of the current precision in the context for combo_apply_operator.
 * Returns COMBO_E_INADMISSIBLE if any voxel has det F <= 0 or a laminate
 * fails (outputs still written). */
int combo_eval_law(combo_ctx* ctx, const double* F, double* P, double* A, double* a, int* iters, int mem_kind);
/* out = Gamma0[tau] (which = COMBO_GREEN_GAMMA0, reference medium of the
 * options) or G[tau] (COMBO_GREEN_G) for a real field tau [9][n] (Sec. 3,
 * eq. Gamma0; zero mean and Nyquist modes), computed in `precision`. */
int combo_apply_green(combo_ctx* ctx, int which, int precision, const double* tau, double* out, int mem_kind);
/* q = Gamma0[A : p] with the tangent state of the last combo_eval_law, for a
 * compatible zero-mean field p [9][n]; the linear operator of each Newton step. */
int combo_apply_operator(combo_ctx* ctx, int precision, const double* p, double* q, int mem_kind);

/* FFT schedules and the autotuner ---------------------------------------------
 * Each CG pass (x: inverse transform, tangent action, forward transform; y and z
 * transform pairs with the Green projection) has compiled variants that differ
 * in radix order, tile width and rows per workgroup; all compute the same
 * operator (Sec. 3, eq. Gamma0) up to rounding.  The schedule of a context is
 * one variant per axis (0 = default).  combo_autotune times every variant of
 * each pass on this context's grid and buffers in `precision` and keeps the
 * fastest (FP64 passes have variant 0 only).  Results are kept per process and,
 * when the environment variable COMBO_TUNE_CACHE names a file, appended to it as
 * text lines "arch n1 n2 n3 precision xv yv zv" and reused by later processes.
 * Needs grid, materials and microstructure; xv, yv, zv (may be NULL) receive
 * the schedule.  The timing writes the context's work buffers only. */
int combo_autotune(combo_ctx* ctx, int precision, int* xv, int* yv, int* zv);
/* Set the schedule directly; a variant that does not exist for an axis length
 * runs variant 0.  COMBO_E_INVAL for negative values. */
int combo_set_schedule(combo_ctx* ctx, int xv, int yv, int zv);
/* Current schedule and the number of variants per axis of the grid (any may be NULL). */
int combo_get_schedule(const combo_ctx* ctx, int* xv, int* yv, int* zv, int* nxv, int* nyv, int* nzv);

/* Per-kernel timing ---------------------------------------------------------
 * With profiling on, the context records a HIP event pair on its stream around
 * every launch of the kernel classes below (the CG iterations then run as
 * plain launches, not as captured graphs) and accumulates the elapsed time.
 * Reading does not reset; combo_profile_enable(ctx, 1) resets the counters. */
enum combo_kernel {
    COMBO_K_XPASS_CG = 0,     /* x pass of the CG operator: C2R, tangent action, R2C */
    COMBO_K_YPASS_INV = 1,    /* y pass, inverse (6 -> 9 components) */
    COMBO_K_YPASS_FWD = 2,    /* y pass, forward (9 -> 6 components) */
    COMBO_K_ZPASS_INV = 3,    /* z pass, inverse, with the search-direction update */
    COMBO_K_ZPASS_FWD = 4,    /* z pass, forward, with the Green projection and <p, A p> */
    COMBO_K_CG_UPDATE = 5,    /* x += alpha p, r -= alpha q, <r, r> */
    COMBO_K_CG_FINALIZE = 6,  /* the two one-workgroup scalar reductions of a CG iteration */
    COMBO_K_MATERIAL = 7,     /* pure-voxel law + laminate law + their reductions */
    COMBO_K_RESIDUAL = 8,     /* FP64 x, y, z forward passes of P, residual norm, right-hand side */
    COMBO_K_NEWTON_DIR = 9,   /* FP64 inverse passes giving dF */
    COMBO_K_BOXEL_COUNT = 10, /* image -> boxels, pass 1: volume fractions, phases, composite list */
    COMBO_K_BOXEL_NORMALS = 11, /* image -> boxels, pass 2: interface weights, moments, normals */
    COMBO_K_COUNT = 12
};
int combo_profile_enable(combo_ctx* ctx, int enable);
/* Which classes profiling times: bit (1u << kernel) set = timed (default: all).
 * Each timed launch adds an event pair to the stream, a few microseconds per
 * launch; timing only the class of interest keeps a measured solve close to an
 * untimed one.  Takes effect for launches made after the call. */
int combo_profile_select(combo_ctx* ctx, unsigned mask);
/* Accumulated milliseconds and number of timed launches of one kernel class.
 * CG iterations run in chunks (8, or graph_chunk) between host checks; the
 * launches of a chunk's iterations after the one that finished the CG find it
 * done and return at once.  Those are not counted here, so that ms_total /
 * launches is the time of a launch that did its work. */
int combo_profile_read(combo_ctx* ctx, int kernel, double* ms_total, long long* launches);
/* The launches combo_profile_read leaves out: chunk iterations after the CG had
 * finished (each returns at once). */
int combo_profile_read_idle(combo_ctx* ctx, int kernel, double* ms_total, long long* launches);

/* Batches of RVEs -----------------------------------------------------------
 * Many independent RVEs, each with its own grid, box, materials and
 * microstructure, solved together on one GPU (the many-RVE workloads of
 * multiscale FE^2-type use, paper Sec. 1).  The members are split into lanes
 * (at most options.batch_streams, default 8): members of one grid shape share a
 * lane, lanes hold contiguous ranges of grid sizes (with fewer shapes than
 * lanes, the most populated shapes are split), and each lane runs on a
 * stream of its own (lane 0 on the batch's stream, the others on streams the
 * batch creates and owns).  Within a lane every pass runs as one launch over
 * all members that share its kernel shape (axis length), each workgroup
 * reading its member's arguments from a device table.  Lanes advance
 * independently, so a small RVE with a long Newton-CG chain runs beside the
 * launches of larger ones instead of waiting for them.  Every member keeps its
 * own Newton, step-control and CG progress, and a member whose CG has finished
 * leaves the launches of the others at once.  Member i solved in a batch
 * follows the steps of combo_solve on a context with the
 * same data and options, F_init = NULL and n_increments[i] increments; the
 * batched kernels are separately compiled instances of the same code, so the
 * results agree to rounding (the compiler may fuse multiply-adds differently). */
/* Create an empty batch on GPU `device` using `hip_stream` (NULL = a stream the
 * batch creates and owns).  COMBO_E_HIP if no usable GPU. */
int combo_batch_create(combo_batch** out, int device, void* hip_stream);
/* Frees every member and all device memory of the batch. */
int combo_batch_destroy(combo_batch* b);
/* Message of the last failed call on b (member failures name the member). */
const char* combo_batch_last_error(const combo_batch* b);
/* Options of every member (validated as combo_set_options).  graph_chunk > 0:
 * the CG iterations of the members in CG run in chunks of that many, captured
 * once as a HIP graph and replayed while the same members stay in CG. */
int combo_batch_set_options(combo_batch* b, const combo_options* opt);
/* Discretization (COMBO_DISC_MS or COMBO_DISC_WILLOT, see combo_set_discretization)
 * of the members added after this call; members of either kind can share a batch. */
int combo_batch_set_discretization(combo_batch* b, int disc);
/* Append one RVE: grid and box as combo_set_grid, materials as
 * combo_set_materials, microstructure as combo_set_microstructure (pointers of
 * mem_kind, copied).  *index (may be NULL) receives the member's position.
 * On failure nothing is appended. */
int combo_batch_add(combo_batch* b, int n1, int n2, int n3, double l1, double l2, double l3,
                    const combo_material mats[2], const uint8_t* phase, const double* c, const double* N,
                    int mem_kind, int* index);
/* Number of members (0 for NULL). */
int combo_batch_size(const combo_batch* b);
/* Solve every member i from F = I to the macroscopic deformation
 * Fbar[9 i .. 9 i + 8] in n_increments[i] load increments (n_increments NULL:
 * the options' value).  Host arrays over the members, each may be NULL except
 * Fbar: Pbar [m][9], Abar [m][81] (written when options.want_tangent),
 * Pbar_phase [m][18] (as combo_solve), stats [m] (time_ms_total is the
 * batch's wall time; per-phase times are 0).  Returns COMBO_OK if every member
 * converged, else the status of the first failing member; every member's own
 * status is in stats[i].status and the outputs of converged members are
 * written either way. */
int combo_batch_solve(combo_batch* b, const double* Fbar, const int* n_increments, double* Pbar, double* Abar,
                      double* Pbar_phase, combo_stats* stats);
/* Fields of member i after combo_batch_solve: F and P, [9][n_i] each (either
 * may be NULL), in memory of mem_kind. */
int combo_batch_fields(combo_batch* b, int i, double* F, double* P, int mem_kind);

#ifdef __cplusplus
}
#endif

#endif /* COMBO_H */
