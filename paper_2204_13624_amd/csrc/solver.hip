// Host driver of the ComBo Lippmann-Schwinger Newton-CG solve and the C-ABI.
//
// Newton-Raphson on the Lippmann-Schwinger equation (paper Sec. 3, eq.
// nonlinearLSE) at fixed macroscopic deformation: with F - Fbar compatible and
// zero-mean, each Newton step solves  Gamma0[A : dF] = -Gamma0[P]  by conjugate
// gradients in the C0 inner product.  On the GPU the unknown dF = Grad du is
// carried by its displacement coefficients du_hat (see fft_kernels.hip); the
// inner product <x, y>_C0 = sum mu0 x:y + kappa0 tr x tr y becomes
// sum_xi u^H K(xi) v by Parseval, so the CG iterates are those of the
// field formulation.
//
// Readings of the paper used here (where it is silent):
//   - reference medium C0 = mu0 Id + kappa0 I(x)I, default mu0 = sqrt(mu_min mu_max),
//     kappa0 = sqrt((lambda+mu)_min (lambda+mu)_max);
//   - Newton test eta = |G[P]|_2 / (sqrt(n) |Pbar|_F) <= tol_newton;
//   - CG test |r|_C0 <= tol_cg |b|_C0 (at least 1e-5 in mixed precision);
//   - load path Fbar_k = Fbar_0 + (k/K)(Fbar - Fbar_0) with the homogeneous
//     predictor F += Fbar_k - Fbar_{k-1};
//   - step control: F + s dF, s halved while any voxel has det F <= 0 or a
//     laminate fails; then the increment is halved;
//   - Nyquist planes of even axes and the zero mode are projected out;
//   - effective tangent column kL: solve Gamma0[A:dF] = -Gamma0[A:E_kL] and
//     average A:(E_kL + dF).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "combo.h"
#include "boxels.h"
#include "setup.h"
#include "context.h"
#include "dfmg.h"

using namespace combo;

namespace {

// internal (positive) return of cg_solve: CG stopped at a direction of
// non-positive curvature; x holds the iterate reached before it
constexpr int kNegCurv = 1;

// sufficient decrease of the Newton line search: eta(s) <= (1 - kArmijo s) eta
constexpr double kArmijo = 1e-4;

int set_err(combo_ctx* ctx, int status, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return status;
}

#define HIP_OR_FAIL(...)                                                                                    \
    do {                                                                                                    \
        hipError_t e__ = (__VA_ARGS__);                                                                     \
        if (e__ != hipSuccess)                                                                              \
            return set_err(ctx, e__ == hipErrorOutOfMemory ? COMBO_E_NOMEM : COMBO_E_HIP,                   \
                           std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e__));                      \
    } while (0)

// COMBO_VERBOSE=1 in the environment traces Newton and CG progress on stderr.
bool verbose() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("COMBO_VERBOSE");
        v = (e && e[0] && e[0] != '0') ? 1 : 0;
    }
    return v == 1;
}

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); }

bool size_ok(int n) {
    if (n < 1 || n > kMaxAxis) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

AxisPlan make_plan(int L) {
    AxisPlan p{};
    p.L = L;
    p.npass = 0;
    int m = L;
    while (m % 16 == 0) { p.radix[p.npass++] = 16; m /= 16; }
    while (m % 8 == 0) { p.radix[p.npass++] = 8; m /= 8; }
    while (m % 4 == 0) { p.radix[p.npass++] = 4; m /= 4; }
    while (m % 2 == 0) { p.radix[p.npass++] = 2; m /= 2; }
    while (m % 3 == 0) { p.radix[p.npass++] = 3; m /= 3; }
    return p;
}

template <typename T> const cpx<T>* twid(const combo_ctx* c, int axis) {
    return sizeof(T) == 4 ? static_cast<const cpx<T>*>(c->tw32[axis].p) : static_cast<const cpx<T>*>(c->tw64[axis].p);
}

template <typename T> PassShape shape_for(const combo_ctx* c) {
    const int maxE = max_elems<T>();
    PassShape s;
    s.xR = std::max(1, maxE / (5 * c->g.n1));
    s.xR = (int)std::min<long long>(s.xR, (long long)c->g.n2 * c->g.n3);
    s.yTX = y_tile<T>(c->g);
    s.zTX = z_tile<T>(c->g);
    return s;
}

void mean_field_host(const double* F, long long n, double out[9]) {
    for (int c = 0; c < 9; ++c) {
        long double s = 0;
        for (long long v = 0; v < n; ++v) s += F[c * n + v];
        out[c] = (double)(s / n);
    }
}

__global__ void k_fill_identity(double* F, long long n) {
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x)
        for (int c = 0; c < 9; ++c) F[c * n + v] = (c % 4 == 0) ? 1.0 : 0.0;
}

__global__ void k_colsum9(const double* F, long long n, double* partials) {
    __shared__ double sh[4];
    for (int c = 0; c < 9; ++c) {
        double s = 0.0;
        for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
             v += (long long)gridDim.x * blockDim.x)
            s += F[c * n + v];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) partials[blockIdx.x * 9 + c] = sh[0] + sh[1] + sh[2] + sh[3];
        __syncthreads();
    }
}

__global__ void k_zero_state(CGState* st) {
    if (threadIdx.x == 0) {
        st->rho = st->rho0 = st->alpha = st->beta = st->tol2 = st->eta2 = 0.0;
        st->iter = st->maxit = st->done = st->status = 0;
    }
}

double frob9(const double* a) {
    double s = 0;
    for (int i = 0; i < 9; ++i) s += a[i] * a[i];
    return std::sqrt(s);
}

// ------------------------------------------------------------------------------
// per-kernel event timing (no-ops unless profiling is on)
// ------------------------------------------------------------------------------
hipEvent_t prof_event(combo_ctx* ctx) {
    if (!ctx->prof_pool.empty()) {
        hipEvent_t e = ctx->prof_pool.back();
        ctx->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int prof_begin(combo_ctx* ctx, int kernel) {
    if (!ctx->profile || !((ctx->prof_mask >> kernel) & 1u)) return -1;
    combo_ctx::ProfRec r{kernel, prof_event(ctx), prof_event(ctx), ctx->prof_iter};
    if (!r.start || !r.stop) return -1;
    (void)hipEventRecord(r.start, ctx->stream);
    ctx->prof_pending.push_back(r);
    return (int)ctx->prof_pending.size() - 1;
}

void prof_end(combo_ctx* ctx, int idx) {
    if (idx < 0) return;
    (void)hipEventRecord(ctx->prof_pending[idx].stop, ctx->stream);
}

// call after the stream has been synchronised; launches of a CG chunk's
// iterations at positions >= work_iters found the CG finished and did no work
void prof_harvest(combo_ctx* ctx, int work_iters = 1 << 30) {
    for (auto& r : ctx->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            if (r.iter >= work_iters) {
                ctx->prof_idle_ms[r.kernel] += ms;
                ctx->prof_idle_n[r.kernel] += 1;
            } else {
                ctx->prof_ms[r.kernel] += ms;
                ctx->prof_n[r.kernel] += 1;
            }
        }
        ctx->prof_pool.push_back(r.start);
        ctx->prof_pool.push_back(r.stop);
    }
    ctx->prof_pending.clear();
}

struct ProfScope {
    combo_ctx* ctx;
    int idx;
    ProfScope(combo_ctx* c, int k) : ctx(c), idx(prof_begin(c, k)) {}
    ~ProfScope() { prof_end(ctx, idx); }
};

// ------------------------------------------------------------------------------
// work buffers
// ------------------------------------------------------------------------------
// laminate points (warm-start slots): one per composite voxel, eight per composite cell
// on the staggered grid (its doubly-fine cells)
size_t lam_points(const combo_ctx* ctx) {
    return (ctx->g.disc == COMBO_DISC_STAGGERED ? 8 : 1) * (size_t)std::max(ctx->nc, 1);
}

// staggered grid: fields at the caller's boundary hold the staggered values at each
// cell's own positions; inside, off-diagonal components are shifted (dfmg.h)
int to_shifted(combo_ctx* ctx, const double* src, double* dst) {
    HIP_OR_FAIL(launch_stag_shift(src, dst, ctx->g.n1, ctx->g.n2, ctx->g.n3, +1, ctx->stream));
    return COMBO_OK;
}
int to_natural(combo_ctx* ctx, const double* src, double* dst) {
    HIP_OR_FAIL(launch_stag_shift(src, dst, ctx->g.n1, ctx->g.n2, ctx->g.n3, -1, ctx->stream));
    return COMBO_OK;
}
bool staggered(const combo_ctx* ctx) { return ctx->g.disc == COMBO_DISC_STAGGERED; }

int ensure_work(combo_ctx* ctx) {
    const long long n = ctx->g.n, ns = ctx->g.nspec;
    const size_t f9 = sizeof(double) * 9 * (size_t)n;
    HIP_OR_FAIL(ctx->F_cur.ensure(f9));
    HIP_OR_FAIL(ctx->F_trial.ensure(f9));
    HIP_OR_FAIL(ctx->F_save.ensure(f9));
    HIP_OR_FAIL(ctx->dF.ensure(f9));
    HIP_OR_FAIL(ctx->P.ensure(f9));
    HIP_OR_FAIL(ctx->specA.ensure(sizeof(double2) * 9 * (size_t)ns));
    HIP_OR_FAIL(ctx->specB.ensure(sizeof(double2) * 9 * (size_t)ns));
    const size_t u3 = sizeof(double2) * 3 * (size_t)ns;
    HIP_OR_FAIL(ctx->ux.ensure(u3));
    HIP_OR_FAIL(ctx->ur.ensure(u3));
    HIP_OR_FAIL(ctx->up.ensure(u3));
    HIP_OR_FAIL(ctx->uq.ensure(u3));
    HIP_OR_FAIL(ctx->Sinv.ensure(sizeof(double) * 9 * (size_t)n));
    HIP_OR_FAIL(ctx->sm.ensure(sizeof(double) * (size_t)n));
    HIP_OR_FAIL(ctx->Acomp.ensure(sizeof(double) * 45 * (size_t)std::max(ctx->nc, 1)));
    HIP_OR_FAIL(ctx->a_prev.ensure(sizeof(double) * 3 * lam_points(ctx)));
    HIP_OR_FAIL(ctx->a_trial.ensure(sizeof(double) * 3 * lam_points(ctx)));
    if (ctx->g.disc == COMBO_DISC_STAGGERED) {
        const size_t n8 = 8 * (size_t)n;
        HIP_OR_FAIL(ctx->dfmg_Pd.ensure(sizeof(double) * 9 * n8));
        HIP_OR_FAIL(ctx->dfmg_Ad.ensure(sizeof(double) * 45 * 8 * (size_t)std::max(ctx->nc, 1)));
        HIP_OR_FAIL(ctx->dfmg_act.ensure(sizeof(double) * 27 * (size_t)n));   // own [9][n] + parts [18][n]
        HIP_OR_FAIL(ctx->dfmg_dH.ensure(f9));
        HIP_OR_FAIL(ctx->dfmg_dQ.ensure(f9));
        HIP_OR_FAIL(ctx->stag_tmp.ensure(f9));
    }
    // partial sums: the largest consumer over all kernels
    size_t np = 0;
    for (int prec = 0; prec < 2; ++prec) {
        // every schedule variant the autotuner may pick
        const bool f = prec == 1;
        PassShape s = f ? shape_for<float>(ctx) : shape_for<double>(ctx);
        Grid g = ctx->g;
        const int nxv = std::max(1, xpass_lds_variants(g.n1));
        const int nzv = std::max(1, f ? fft2_variants<float>(g.n3) : fft2_variants<double>(g.n3));
        for (int v = 0; v < nxv; ++v) {
            g.xv = v;
            np = std::max(np, (size_t)blocks_x(g, s.xR, X_AVG, f) * 9);
        }
        np = std::max(np, (size_t)blocks_x(g, s.xR, X_FWD_REAL, f) * 9);
        for (int v = 0; v < nzv; ++v) {
            g.zv = v;
            np = std::max(np, (size_t)blocks_z(g, f ? z_tile<float>(g) : z_tile<double>(g)));
        }
    }
    np = std::max(np, (size_t)blocks_u(ctx->g));
    np = std::max(np, (size_t)material_blocks_pure(n) * 19);
    np = std::max(np, (size_t)material_blocks_laminate(ctx->nc) * 31);
    np = std::max(np, (size_t)dfmg_blocks_pure(n) * 19);
    np = std::max(np, (size_t)dfmg_blocks_laminate(ctx->nc) * 31);
    np = std::max(np, (size_t)2048 * 9);
    HIP_OR_FAIL(ctx->part1.ensure(sizeof(double) * np));
    HIP_OR_FAIL(ctx->part2.ensure(sizeof(double) * np));
    HIP_OR_FAIL(ctx->sums.ensure(sizeof(double) * (kSumsLen + 16)));
    HIP_OR_FAIL(ctx->cgst.ensure(sizeof(CGState)));
    if (!ctx->hs) {
        HIP_OR_FAIL(hipHostMalloc((void**)&ctx->hs, sizeof(HostScalars), hipHostMallocDefault));
        memset(ctx->hs, 0, sizeof(HostScalars));
    }
    return COMBO_OK;
}

void reference_medium(const combo_ctx* ctx, double& mu0, double& kappa0) {
    const double mu_m = ctx->mats[0].mu, mu_p = ctx->mats[1].mu;
    const double k_m = ctx->mats[0].lambda + mu_m, k_p = ctx->mats[1].lambda + mu_p;
    mu0 = ctx->opt.mu0 > 0 ? ctx->opt.mu0 : std::sqrt(mu_m * mu_p);
    kappa0 = ctx->opt.kappa0 > 0 ? ctx->opt.kappa0 : std::sqrt(k_m * k_p);
}

// ------------------------------------------------------------------------------
// building blocks
// ------------------------------------------------------------------------------
template <typename T>
TangentState<T> tangent_state(const combo_ctx* ctx) {
    TangentState<T> ts{};
    ts.slot = ctx->slot_s.as<int>();
    ts.Sinv = ctx->Sinv.as<T>();
    ts.sm = ctx->sm.as<T>();
    ts.Acomp = ctx->Acomp.as<T>();
    for (int p = 0; p < 2; ++p) {
        ts.mu[p] = T(ctx->mats[p].mu);
        ts.lam[p] = T(ctx->mats[p].lambda);
    }
    ts.n = ctx->g.n;
    return ts;
}

template <typename T>
XArgs<T> xargs(const combo_ctx* ctx) {
    XArgs<T> a{};
    a.g = ctx->g;
    a.plan = ctx->plan[0];
    a.R = shape_for<T>(ctx).xR;
    a.tw = twid<T>(ctx, 0);
    a.ts = tangent_state<T>(ctx);
    a.scale = 1.0 / (double)ctx->g.n;
    a.partials = ctx->part1.as<double>();
    a.st = ctx->cgst.as<CGState>();
    return a;
}

template <typename T>
YArgs<T> yargs(const combo_ctx* ctx, const void* in, void* out, bool use_state) {
    YArgs<T> a{};
    a.g = ctx->g;
    a.plan = ctx->plan[1];
    a.TX = shape_for<T>(ctx).yTX;
    a.ntile = (ctx->g.nh + a.TX - 1) / a.TX;
    a.tw = twid<T>(ctx, 1);
    a.in = static_cast<const cpx<T>*>(in);
    a.out = static_cast<cpx<T>*>(out);
    a.st = use_state ? ctx->cgst.as<CGState>() : nullptr;
    return a;
}

template <typename T, typename TU>
ZArgs<T, TU> zargs(const combo_ctx* ctx, double mu0, double kappa0) {
    ZArgs<T, TU> a{};
    a.g = ctx->g;
    a.plan = ctx->plan[2];
    a.TX = shape_for<T>(ctx).zTX;
    a.tw = twid<T>(ctx, 2);
    a.x = ctx->ux.as<cpx<TU>>();
    a.r = ctx->ur.as<cpx<TU>>();
    a.p = ctx->up.as<cpx<TU>>();
    a.q = ctx->uq.as<cpx<TU>>();
    a.mu0 = mu0;
    a.kappa0 = kappa0;
    a.inv_n = 1.0 / (double)ctx->g.n;
    a.partials = ctx->part1.as<double>();
    a.partials2 = ctx->part2.as<double>();
    a.st = ctx->cgst.as<CGState>();
    return a;
}

template <typename TU>
UArgs<TU> uargs(const combo_ctx* ctx, double mu0, double kappa0) {
    UArgs<TU> ua{};
    ua.g = ctx->g;
    ua.x = ctx->ux.as<cpx<TU>>();
    ua.r = ctx->ur.as<cpx<TU>>();
    ua.p = ctx->up.as<cpx<TU>>();
    ua.q = ctx->uq.as<cpx<TU>>();
    ua.mu0 = mu0;
    ua.kappa0 = kappa0;
    ua.partials = ctx->part2.as<double>();
    ua.st = ctx->cgst.as<CGState>();
    return ua;
}

FinArgs finargs(const combo_ctx* ctx, const double* p1, const double* p2, int count, double tol2 = 0.0, int maxit = 0) {
    FinArgs f{};
    f.st = ctx->cgst.as<CGState>();
    f.partials = p1;
    f.partials2 = p2;
    f.count = count;
    f.tol2 = tol2;
    f.maxit = maxit;
    return f;
}

// Staggered grid: the DFMG law at F = F_old + s dF + dFbar (shifted layout) -> F_new,
// P (shifted layout), the doubly-fine tangent states (precision T), a_trial; sums as material().
template <typename T>
int material_dfmg(combo_ctx* ctx, const double* F_old, const double* dF, double s, const double dFbar[9],
                  double* F_new, bool cold) {
    DfmgArgs<T> d{};
    d.n1 = ctx->g.n1;
    d.n2 = ctx->g.n2;
    d.n3 = ctx->g.n3;
    d.n = ctx->g.n;
    d.nc = ctx->nc;
    d.F_old = F_old;
    d.dF = dF;
    d.s = s;
    for (int c = 0; c < 9; ++c) d.dFbar[c] = dFbar ? dFbar[c] : 0.0;
    d.F_new = F_new;
    d.slot = ctx->slot.as<int>();
    d.comp_vox = ctx->comp_vox.as<int>();
    d.cc = ctx->comp_c.as<double>();
    d.NN = ctx->comp_N.as<double>();
    d.a_prev = ctx->a_prev.as<double>();
    d.a_out = ctx->a_trial.as<double>();
    d.warm = (!cold && ctx->opt.warm_start_laminate) ? 1 : 0;
    d.maxit = ctx->opt.max_laminate;
    for (int p = 0; p < 2; ++p) {
        d.mu[p] = ctx->mats[p].mu;
        d.lam[p] = ctx->mats[p].lambda;
    }
    d.Pd = ctx->dfmg_Pd.as<double>();
    d.Ad = ctx->dfmg_Ad.as<T>();
    d.partials = ctx->part1.as<double>();
    d.partials2 = ctx->part2.as<double>();
    {
        ProfScope ps(ctx, COMBO_K_MATERIAL);
        HIP_OR_FAIL(launch_dfmg_update<T>(d, ctx->stream));
        HIP_OR_FAIL(launch_dfmg_law<T>(d, ctx->sums.as<double>(), ctx->stream));
        DfmgGatherArgs<double> ga{ctx->g.n1, ctx->g.n2, ctx->g.n3, ctx->g.n, d.Pd, ctx->P.as<double>(), nullptr};
        HIP_OR_FAIL(launch_dfmg_gather<double>(ga, ctx->stream));
    }
    HIP_OR_FAIL(hipMemcpyAsync(ctx->hs->sums, ctx->sums.p, sizeof(double) * kSumsLen, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx);
    ctx->state_prec = sizeof(T) == 4 ? COMBO_MIXED : COMBO_FP64;
    ctx->dfmg_Feval = F_new;   // pure doubly-fine tangents are recomputed from it
    return COMBO_OK;
}

// material law at F = F_old + s dF + dFbar -> F_trial, P, tangent state (precision T), a_trial.
template <typename T>
int material(combo_ctx* ctx, const double* F_old, const double* dF, double s, const double dFbar[9], double* F_new,
             bool cold, double* A_full, double* a_full, int* it_full) {
    if (ctx->g.disc == COMBO_DISC_STAGGERED) return material_dfmg<T>(ctx, F_old, dF, s, dFbar, F_new, cold);
    MatArgs<T> m{};
    m.n = ctx->g.n;
    m.nc = ctx->nc;
    m.F_old = F_old;
    m.dF = dF;
    m.s = s;
    for (int c = 0; c < 9; ++c) m.dFbar[c] = dFbar ? dFbar[c] : 0.0;
    m.F_new = F_new;
    m.P = ctx->P.as<double>();
    m.slot = ctx->slot.as<int>();
    for (int p = 0; p < 2; ++p) {
        m.mu[p] = ctx->mats[p].mu;
        m.lam[p] = ctx->mats[p].lambda;
    }
    m.comp_vox = ctx->comp_vox.as<int>();
    m.cc = ctx->comp_c.as<double>();
    m.NN = ctx->comp_N.as<double>();
    m.a_prev = ctx->a_prev.as<double>();
    m.a_out = ctx->a_trial.as<double>();
    m.warm = (!cold && ctx->opt.warm_start_laminate) ? 1 : 0;
    m.maxit = ctx->opt.max_laminate;
    m.law = ctx->opt.law;
    m.Sinv = ctx->Sinv.as<T>();
    m.sm = ctx->sm.as<T>();
    m.n1 = ctx->g.n1;
    m.xm = ctx->g.xm;
    m.xwbits = ctx->g.xwbits;
    m.Acomp = ctx->Acomp.as<T>();
    m.A_full = A_full;
    m.a_full = a_full;
    m.iters_full = it_full;
    m.partials = ctx->part1.as<double>();
    m.partials2 = ctx->part2.as<double>();
    const int nbp = material_blocks_pure(m.n), nbl = material_blocks_laminate(m.nc);
    {
        ProfScope ps(ctx, COMBO_K_MATERIAL);
        HIP_OR_FAIL(launch_material<T>(m, nbp, nbl, ctx->sums.as<double>(), ctx->stream));
    }
    HIP_OR_FAIL(hipMemcpyAsync(ctx->hs->sums, ctx->sums.p, sizeof(double) * kSumsLen, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx);
    ctx->state_prec = sizeof(T) == 4 ? COMBO_MIXED : COMBO_FP64;
    return COMBO_OK;
}

double material_failures(const combo_ctx* ctx) { return ctx->hs->sums[18] + ctx->hs->sums[46]; }

void material_pbar(const combo_ctx* ctx, double Pbar[9]) {
    const double* s = ctx->hs->sums;
    for (int c = 0; c < 9; ++c) Pbar[c] = (s[c] + s[9 + c] + s[19 + c]) / (double)ctx->g.n;
}

// forward x and y passes of a real FP64 field into specB (6 components)
template <typename T>
int forward_xy_real(combo_ctx* ctx, const double* field) {
    XArgs<T> xa = xargs<T>(ctx);
    xa.real_in = field;
    xa.out = ctx->specA.as<cpx<T>>();
    HIP_OR_FAIL(launch_x<T>(X_FWD_REAL, xa, ctx->stream));
    HIP_OR_FAIL(launch_y<T>(-1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, false), ctx->stream));
    return COMBO_OK;
}

// residual of P (FP64): eta, and the right-hand side r = b = -K^{-1}(P_hat xi), x = 0 (precision TU)
template <typename TU>
int residual(combo_ctx* ctx, double mu0, double kappa0, double tol_cg, double& eta) {
    {
        ProfScope ps(ctx, COMBO_K_RESIDUAL);
        int st = forward_xy_real<double>(ctx, ctx->P.as<double>());
        if (st) return st;
        ZArgs<double, TU> za = zargs<double, TU>(ctx, mu0, kappa0);
        za.in = ctx->specB.as<double2>();
        int nb = 0;
        HIP_OR_FAIL(launch_z<double, TU>(Z_RHS, za, ctx->stream, &nb));
        HIP_OR_FAIL(launch_antiherm<TU>(uargs<TU>(ctx, mu0, kappa0), ctx->stream));
        HIP_OR_FAIL(launch_finalize(FIN_RHS, finargs(ctx, ctx->part1.as<double>(), ctx->part2.as<double>(), nb,
                                                     tol_cg * tol_cg, ctx->opt.max_cg), ctx->stream));
    }
    HIP_OR_FAIL(hipMemcpyAsync(&ctx->hs->cg, ctx->cgst.p, sizeof(CGState), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx);
    double Pbar[9];
    material_pbar(ctx, Pbar);
    const double den = (double)ctx->g.n * std::max(frob9(Pbar), 1e-300);
    eta = std::sqrt(std::max(ctx->hs->cg.eta2, 0.0)) / den;
    return COMBO_OK;
}

// The tangent action of the staggered grid on the spectrum in specB (after the y
// inverse pass): inverse x pass to the shifted-layout field dH, per doubly-fine
// cell A : dF summed per destination, the DFMG sum dQ, forward x pass into specA;
// real fields in the precision of the CG.  Kernels skip once the CG state says done.
// dQ = the DFMG sum of A : dH per doubly-fine cell (dH and dQ in the shifted layout, in
// the precision T); st: skip once the CG state says done (null: always run)
template <typename T>
int stag_action_sum(combo_ctx* ctx, hipStream_t s, const CGState* st) {
    const long long n = ctx->g.n;
    DfmgActArgs<T> act{};
    act.n1 = ctx->g.n1;
    act.n2 = ctx->g.n2;
    act.n3 = ctx->g.n3;
    act.n = n;
    act.dH = ctx->dfmg_dH.as<T>();
    act.F = ctx->dfmg_Feval;
    act.own = ctx->dfmg_act.as<T>();
    act.part = ctx->dfmg_act.as<T>() + 9 * n;
    act.slot = ctx->slot.as<int>();
    act.Ad = ctx->dfmg_Ad.as<T>();
    for (int p = 0; p < 2; ++p) {
        act.mu[p] = ctx->mats[p].mu;
        act.lam[p] = ctx->mats[p].lambda;
    }
    act.st = st;
    HIP_OR_FAIL(launch_dfmg_action<T>(act, s));
    DfmgSumArgs<T> sm{ctx->g.n1, ctx->g.n2, ctx->g.n3, n, act.own, act.part, ctx->dfmg_dQ.as<T>(), st};
    HIP_OR_FAIL(launch_dfmg_sum<T>(sm, s));
    return COMBO_OK;
}

template <typename T>
int stag_tangent_x(combo_ctx* ctx, hipStream_t s) {
    XArgs<T> xi = xargs<T>(ctx);
    xi.in = ctx->specB.as<cpx<T>>();
    xi.real_out_t = ctx->dfmg_dH.as<T>();
    xi.scale = 1.0;   // the 1/n of the operator is applied by the z pass
    xi.skip_done = 1;
    HIP_OR_FAIL(launch_x<T>(X_INV_REAL, xi, s));
    const int st = stag_action_sum<T>(ctx, s, ctx->cgst.as<CGState>());
    if (st) return st;
    XArgs<T> xf = xargs<T>(ctx);
    xf.real_in_t = ctx->dfmg_dQ.as<T>();
    xf.out = ctx->specA.as<cpx<T>>();
    xf.skip_done = 1;
    HIP_OR_FAIL(launch_x<T>(X_FWD_REAL, xf, s));
    return COMBO_OK;
}

// one CG iteration (8 launches; 11 on the staggered grid)
template <typename T>
int cg_iteration(combo_ctx* ctx, double mu0, double kappa0) {
    hipStream_t s = ctx->stream;
    ZArgs<T, T> za = zargs<T, T>(ctx, mu0, kappa0);
    za.out = ctx->specA.as<cpx<T>>();
    {
        ProfScope ps(ctx, COMBO_K_ZPASS_INV);
        HIP_OR_FAIL(launch_z<T, T>(Z_INV_CG, za, s));
    }
    {
        ProfScope ps(ctx, COMBO_K_YPASS_INV);
        HIP_OR_FAIL(launch_y<T>(+1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, true), s));
    }
    if (ctx->g.disc == COMBO_DISC_STAGGERED) {
        ProfScope ps(ctx, COMBO_K_XPASS_CG);
        const int st = stag_tangent_x<T>(ctx, s);
        if (st) return st;
    } else {
        XArgs<T> xa = xargs<T>(ctx);
        xa.in = ctx->specB.as<cpx<T>>();
        xa.out = ctx->specA.as<cpx<T>>();
        ProfScope ps(ctx, COMBO_K_XPASS_CG);
        HIP_OR_FAIL(launch_x<T>(X_CG, xa, s));
    }
    {
        ProfScope ps(ctx, COMBO_K_YPASS_FWD);
        HIP_OR_FAIL(launch_y<T>(-1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, true), s));
    }
    za.in = ctx->specB.as<cpx<T>>();
    za.out = nullptr;
    int nbz = 0;
    {
        ProfScope ps(ctx, COMBO_K_ZPASS_FWD);
        HIP_OR_FAIL(launch_z<T, T>(Z_CG, za, s, &nbz));
    }
    {
        ProfScope ps(ctx, COMBO_K_CG_FINALIZE);
        HIP_OR_FAIL(launch_finalize(FIN_ALPHA, finargs(ctx, ctx->part1.as<double>(), nullptr, nbz), s));
    }
    const UArgs<T> ua = uargs<T>(ctx, mu0, kappa0);
    int nbu = 0;
    {
        ProfScope ps(ctx, COMBO_K_CG_UPDATE);
        HIP_OR_FAIL(launch_update<T>(ua, s, &nbu));
    }
    {
        ProfScope ps(ctx, COMBO_K_CG_FINALIZE);
        HIP_OR_FAIL(launch_finalize(FIN_BETA, finargs(ctx, ctx->part2.as<double>(), nullptr, nbu), s));
    }
    return COMBO_OK;
}

// CG solve on the right-hand side already in r (x = 0, FIN_RHS done); returns iterations
template <typename T>
int cg_solve(combo_ctx* ctx, double mu0, double kappa0, int& iters) {
    const int chunk = ctx->opt.graph_chunk > 0 ? ctx->opt.graph_chunk : 8;
    const bool use_graph = ctx->opt.graph_chunk > 0 && !ctx->profile;
    CGGraph& gr = ctx->graph[sizeof(T) == 4 ? 1 : 0];
    if (use_graph && (!gr.exec || gr.iters != chunk)) {
        gr.reset();
        HIP_OR_FAIL(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        int st = COMBO_OK;
        for (int k = 0; k < chunk && st == COMBO_OK; ++k) st = cg_iteration<T>(ctx, mu0, kappa0);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->stream, &g);
        if (st) return st;
        HIP_OR_FAIL(e);
        gr.graph = g;
        HIP_OR_FAIL(hipGraphInstantiate(&gr.exec, g, nullptr, nullptr, 0));
        gr.iters = chunk;
    }
    const int max_rounds = ctx->opt.max_cg / chunk + 2;
    int iter_before = -1;   // CG iterations done before the pending chunk (-1: no chunk pending)
    for (int round = 0; round < max_rounds; ++round) {
        HIP_OR_FAIL(hipMemcpyAsync(&ctx->hs->cg, ctx->cgst.p, sizeof(CGState), hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
        prof_harvest(ctx, iter_before < 0 ? (1 << 30) : ctx->hs->cg.iter - iter_before);
        iter_before = ctx->hs->cg.iter;
        if (verbose())
            fprintf(stderr, "[combo] cg iter %d  |r|/|b| %.3e  alpha %.3e  beta %.3e  done %d  status %d\n",
                    ctx->hs->cg.iter, std::sqrt(std::max(ctx->hs->cg.rho, 0.0) / std::max(ctx->hs->cg.rho0, 1e-300)),
                    ctx->hs->cg.alpha, ctx->hs->cg.beta, ctx->hs->cg.done, ctx->hs->cg.status);
        if (ctx->hs->cg.done) break;
        if (use_graph) {
            HIP_OR_FAIL(hipGraphLaunch(gr.exec, ctx->stream));
        } else {
            for (int k = 0; k < chunk; ++k) {
                ctx->prof_iter = k;
                int st = cg_iteration<T>(ctx, mu0, kappa0);
                ctx->prof_iter = -1;
                if (st) return st;
            }
        }
    }
    iters = ctx->hs->cg.iter;
    if (!ctx->hs->cg.done)
        return set_err(ctx, COMBO_E_NOCONV, "CG did not terminate");
    if (ctx->hs->cg.status == 1)
        return set_err(ctx, COMBO_E_NUMERIC, "CG breakdown (<p, A p> is NaN)");
    if (ctx->hs->cg.status == 3) {
        set_err(ctx, COMBO_E_NUMERIC, "CG met negative curvature (<p, A p> <= 0)");
        return kNegCurv;
    }
    if (ctx->hs->cg.status == 2)
        return set_err(ctx, COMBO_E_NOCONV, "CG did not converge in max_cg iterations");
    return COMBO_OK;
}

// ------------------------------------------------------------------------------
// autotuner: the schedule (variant of the x, y and z passes) of a CG iteration
// ------------------------------------------------------------------------------
struct Schedule {
    int xv = 0, yv = 0, zv = 0;
};

std::mutex g_tune_mu;
std::map<std::string, Schedule> g_tune;   // per process: "arch n1 n2 n3 precision"
bool g_tune_file_read = false;

std::string tune_key(const combo_ctx* ctx, int precision) {
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
        arch = prop.gcnArchName;
        for (char& c : arch)
            if (c == ' ') c = '_';
    }
    // the rotated scheme has schedules of its own (its passes are separate instances)
    return arch + " " + std::to_string(ctx->g.n1) + " " + std::to_string(ctx->g.n2) + " " +
           std::to_string(ctx->g.n3) + " " + (precision == COMBO_MIXED ? "mixed" : "fp64") +
           (ctx->g.disc == COMBO_DISC_WILLOT ? "-willot" : "");
}

// COMBO_TUNE_CACHE names a text file: one line "arch n1 n2 n3 precision xv yv zv" per tuned grid
void tune_file_read_locked() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char* path = getenv("COMBO_TUNE_CACHE");
    if (!path || !path[0]) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char arch[128], prec[16];
    int n1, n2, n3;
    Schedule sc;
    while (fscanf(f, "%127s %d %d %d %15s %d %d %d", arch, &n1, &n2, &n3, prec, &sc.xv, &sc.yv, &sc.zv) == 8) {
        const std::string key = std::string(arch) + " " + std::to_string(n1) + " " + std::to_string(n2) + " " +
                                std::to_string(n3) + " " + prec;
        g_tune[key] = sc;
    }
    fclose(f);
}

void tune_file_append_locked(const std::string& key, const Schedule& sc) {
    const char* path = getenv("COMBO_TUNE_CACHE");
    if (!path || !path[0]) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d\n", key.c_str(), sc.xv, sc.yv, sc.zv);
    fclose(f);
}

// average milliseconds of `launch` (enqueues one pass) on the context's stream
int time_pass(combo_ctx* ctx, const std::function<hipError_t()>& launch, int reps, double& ms) {
    hipEvent_t e0 = prof_event(ctx), e1 = prof_event(ctx);
    if (!e0 || !e1) return set_err(ctx, COMBO_E_HIP, "event creation failed");
    for (int k = 0; k < 2; ++k) HIP_OR_FAIL(launch());
    HIP_OR_FAIL(hipEventRecord(e0, ctx->stream));
    for (int k = 0; k < reps; ++k) HIP_OR_FAIL(launch());
    HIP_OR_FAIL(hipEventRecord(e1, ctx->stream));
    HIP_OR_FAIL(hipEventSynchronize(e1));
    float t = 0.f;
    HIP_OR_FAIL(hipEventElapsedTime(&t, e0, e1));
    ms = double(t) / reps;
    ctx->prof_pool.push_back(e0);
    ctx->prof_pool.push_back(e1);
    return COMBO_OK;
}

// Times every compiled variant of each CG pass (x operator pass; y inverse +
// forward; z inverse + forward) on the context's buffers and keeps the fastest.
// The data in the buffers is whatever they hold: only the timing matters, and
// every index the kernels use (slot map, composites) is valid.
template <typename T>
int autotune_impl(combo_ctx* ctx, Schedule& best) {
    double mu0, kappa0;
    reference_medium(ctx, mu0, kappa0);
    hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(64), 0, ctx->stream, ctx->cgst.as<CGState>());
    HIP_OR_FAIL(hipGetLastError());
    const Grid g0 = ctx->g;
    const bool f = sizeof(T) == 4;
    const int nxv = f ? std::max(1, xpass_lds_variants(g0.n1)) : 1;
    const int nyv = std::max(1, fft2_variants<T>(g0.n2));
    const int nzv = std::max(1, fft2_variants<T>(g0.n3));
    const int reps = (int)std::min<long long>(100, std::max<long long>(5, 30000000LL / std::max(1LL, g0.n)));
    double bx = 1e30, by = 1e30, bz = 1e30, ms = 0.0;
    int st = COMBO_OK;
    for (int v = 0; v < nxv && !st; ++v) {
        ctx->g = g0;
        ctx->g.xv = v;
        XArgs<T> xa = xargs<T>(ctx);
        xa.in = ctx->specB.as<cpx<T>>();
        xa.out = ctx->specA.as<cpx<T>>();
        st = time_pass(ctx, [&]() { return launch_x<T>(X_CG, xa, ctx->stream); }, reps, ms);
        if (!st && ms < bx) bx = ms, best.xv = v;
    }
    for (int v = 0; v < nyv && !st; ++v) {
        ctx->g = g0;
        ctx->g.yv = v;
        const YArgs<T> yi = yargs<T>(ctx, ctx->specA.p, ctx->specB.p, true);
        const YArgs<T> yf = yargs<T>(ctx, ctx->specA.p, ctx->specB.p, true);
        st = time_pass(ctx, [&]() {
            hipError_t e = launch_y<T>(+1, yi, ctx->stream);
            return e != hipSuccess ? e : launch_y<T>(-1, yf, ctx->stream);
        }, reps, ms);
        if (!st && ms < by) by = ms, best.yv = v;
    }
    for (int v = 0; v < nzv && !st; ++v) {
        ctx->g = g0;
        ctx->g.zv = v;
        ZArgs<T, T> zi = zargs<T, T>(ctx, mu0, kappa0);
        zi.out = ctx->specA.as<cpx<T>>();
        ZArgs<T, T> zf = zargs<T, T>(ctx, mu0, kappa0);
        zf.in = ctx->specB.as<cpx<T>>();
        zf.out = nullptr;
        st = time_pass(ctx, [&]() {
            hipError_t e = launch_z<T, T>(Z_INV_CG, zi, ctx->stream);
            return e != hipSuccess ? e : launch_z<T, T>(Z_CG, zf, ctx->stream);
        }, reps, ms);
        if (!st && ms < bz) bz = ms, best.zv = v;
    }
    ctx->g = g0;
    if (st) return st;
    if (verbose())
        fprintf(stderr, "[combo] autotune %dx%dx%d %s: x %d (%.1f us) y %d (%.1f us) z %d (%.1f us)\n", g0.n1, g0.n2,
                g0.n3, f ? "mixed" : "fp64", best.xv, bx * 1e3, best.yv, by * 1e3, best.zv, bz * 1e3);
    return COMBO_OK;
}

void apply_schedule(combo_ctx* ctx, const Schedule& sc) {
    ctx->g.xv = sc.xv;
    ctx->g.yv = sc.yv;
    ctx->g.zv = sc.zv;
    for (auto& gr : ctx->graph) gr.reset();
}

int autotune(combo_ctx* ctx, int precision) {
    if (ctx->g.disc == COMBO_DISC_STAGGERED) {   // one schedule: the LDS Stockham passes
        apply_schedule(ctx, Schedule{});
        return COMBO_OK;
    }
    const std::string key = tune_key(ctx, precision);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_file_read_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            apply_schedule(ctx, it->second);
            return COMBO_OK;
        }
    }
    Schedule sc;
    int st = precision == COMBO_MIXED ? autotune_impl<float>(ctx, sc) : autotune_impl<double>(ctx, sc);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!g_tune.count(key)) {
            g_tune[key] = sc;
            tune_file_append_locked(key, sc);
        }
    }
    apply_schedule(ctx, sc);
    return COMBO_OK;
}

// dF (FP64 field) from the CG solution x (precision TU)
template <typename TU>
int newton_direction(combo_ctx* ctx) {
    ProfScope ps(ctx, COMBO_K_NEWTON_DIR);
    ZArgs<double, TU> za = zargs<double, TU>(ctx, 1.0, 0.0);
    za.out = ctx->specA.as<double2>();
    HIP_OR_FAIL(launch_z<double, TU>(Z_INV_PLAIN, za, ctx->stream));
    HIP_OR_FAIL(launch_y<double>(+1, yargs<double>(ctx, ctx->specA.p, ctx->specB.p, false), ctx->stream));
    XArgs<double> xa = xargs<double>(ctx);
    xa.in = ctx->specB.as<double2>();
    xa.real_out = ctx->dF.as<double>();
    HIP_OR_FAIL(launch_x<double>(X_INV_REAL, xa, ctx->stream));
    return COMBO_OK;
}

// effective tangent column by column (precision T of the linear solves)
// Effective tangent on the staggered grid (same steps as below): for E = e_kL, the
// right-hand side -Gamma0[A : E] from the DFMG action of the uniform field E, the CG
// solve, then <A : (E + dF)> as the mean of the DFMG action of E + dF.
template <typename T>
int effective_tangent_stag(combo_ctx* ctx, double mu0, double kappa0, double tol_cg, double Abar[81],
                           int& cg_total) {
    const long long n = ctx->g.n;
    hipStream_t s = ctx->stream;
    T* dH = ctx->dfmg_dH.as<T>();
    cg_total = 0;
    for (int kL = 0; kL < 9; ++kL) {
        double E[9];
        for (int c = 0; c < 9; ++c) E[c] = (c == kL) ? 1.0 : 0.0;
        HIP_OR_FAIL(launch_stag_uniform<T>(dH, n, E, 0, s));
        int st = stag_action_sum<T>(ctx, s, nullptr);
        if (st) return st;
        XArgs<T> xf = xargs<T>(ctx);
        xf.real_in_t = ctx->dfmg_dQ.as<T>();
        xf.out = ctx->specA.as<cpx<T>>();
        HIP_OR_FAIL(launch_x<T>(X_FWD_REAL, xf, s));
        HIP_OR_FAIL(launch_y<T>(-1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, false), s));
        ZArgs<T, T> za = zargs<T, T>(ctx, mu0, kappa0);
        za.in = ctx->specB.as<cpx<T>>();
        int nb = 0;
        HIP_OR_FAIL(launch_z<T, T>(Z_RHS, za, s, &nb));
        HIP_OR_FAIL(launch_antiherm<T>(uargs<T>(ctx, mu0, kappa0), s));
        HIP_OR_FAIL(launch_finalize(FIN_RHS, finargs(ctx, ctx->part1.as<double>(), ctx->part2.as<double>(), nb,
                                                     tol_cg * tol_cg, ctx->opt.max_cg), s));
        int it = 0;
        st = cg_solve<T>(ctx, mu0, kappa0, it);
        if (st == kNegCurv) return COMBO_E_NUMERIC;   // message set by cg_solve
        if (st) return st;
        cg_total += it;
        ZArgs<T, T> zi = zargs<T, T>(ctx, mu0, kappa0);
        zi.out = ctx->specA.as<cpx<T>>();
        HIP_OR_FAIL(launch_z<T, T>(Z_INV_PLAIN, zi, s));
        HIP_OR_FAIL(launch_y<T>(+1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, false), s));
        XArgs<T> xi = xargs<T>(ctx);   // scale 1/n: the inverse transforms are unnormalised
        xi.in = ctx->specB.as<cpx<T>>();
        xi.real_out_t = dH;
        HIP_OR_FAIL(launch_x<T>(X_INV_REAL, xi, s));
        HIP_OR_FAIL(launch_stag_uniform<T>(dH, n, E, 1, s));
        st = stag_action_sum<T>(ctx, s, nullptr);
        if (st) return st;
        HIP_OR_FAIL(launch_stag_field_sums<T>(ctx->dfmg_dQ.as<T>(), n, ctx->part1.as<double>(), s));
        double* col = ctx->sums.as<double>() + kSumsLen;
        HIP_OR_FAIL(launch_reduce_columns(ctx->part1.as<double>(), stag_sum_blocks(n), 9, col, s));
        double h[9];
        HIP_OR_FAIL(hipMemcpyAsync(h, col, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        for (int r = 0; r < 9; ++r) Abar[9 * r + kL] = h[r] / (double)n;
    }
    return COMBO_OK;
}

template <typename T>
int effective_tangent(combo_ctx* ctx, double mu0, double kappa0, double tol_cg, double Abar[81], int& cg_total) {
    if (staggered(ctx)) return effective_tangent_stag<T>(ctx, mu0, kappa0, tol_cg, Abar, cg_total);
    cg_total = 0;
    for (int kL = 0; kL < 9; ++kL) {
        XArgs<T> xa = xargs<T>(ctx);
        for (int c = 0; c < 9; ++c) xa.E[c] = (c == kL) ? 1.0 : 0.0;
        xa.out = ctx->specA.as<cpx<T>>();
        HIP_OR_FAIL(launch_x<T>(X_RHS_E, xa, ctx->stream));
        HIP_OR_FAIL(launch_y<T>(-1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, false), ctx->stream));
        ZArgs<T, T> za = zargs<T, T>(ctx, mu0, kappa0);
        za.in = ctx->specB.as<cpx<T>>();
        int nb = 0;
        HIP_OR_FAIL(launch_z<T, T>(Z_RHS, za, ctx->stream, &nb));
        HIP_OR_FAIL(launch_antiherm<T>(uargs<T>(ctx, mu0, kappa0), ctx->stream));
        HIP_OR_FAIL(launch_finalize(FIN_RHS, finargs(ctx, ctx->part1.as<double>(), ctx->part2.as<double>(), nb,
                                                     tol_cg * tol_cg, ctx->opt.max_cg), ctx->stream));
        int it = 0;
        int st = cg_solve<T>(ctx, mu0, kappa0, it);
        if (st == kNegCurv) return COMBO_E_NUMERIC;   // message set by cg_solve
        if (st) return st;
        cg_total += it;
        ZArgs<T, T> zi = zargs<T, T>(ctx, mu0, kappa0);
        zi.out = ctx->specA.as<cpx<T>>();
        HIP_OR_FAIL(launch_z<T, T>(Z_INV_PLAIN, zi, ctx->stream));
        HIP_OR_FAIL(launch_y<T>(+1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, false), ctx->stream));
        XArgs<T> xv = xargs<T>(ctx);
        for (int c = 0; c < 9; ++c) xv.E[c] = (c == kL) ? 1.0 : 0.0;
        xv.in = ctx->specB.as<cpx<T>>();
        int nbx = 0;
        HIP_OR_FAIL(launch_x<T>(X_AVG, xv, ctx->stream, &nbx));
        double* col = ctx->sums.as<double>() + kSumsLen;
        HIP_OR_FAIL(launch_reduce_columns(ctx->part1.as<double>(), nbx, 9, col, ctx->stream));
        double h[9];
        HIP_OR_FAIL(hipMemcpyAsync(h, col, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
        for (int r = 0; r < 9; ++r) Abar[9 * r + kL] = h[r] / (double)ctx->g.n;
    }
    return COMBO_OK;
}

// ------------------------------------------------------------------------------
// the full solve
// ------------------------------------------------------------------------------
struct SolveOut {
    combo_stats st{};
    double Pbar[9]{};
    double Pp[9]{}, Pm[9]{};
    double Abar_store[81]{};
};

template <typename T>
int solve_impl(combo_ctx* ctx, const double Fbar[9], const double Fbar0[9], SolveOut& out, double Abar[81]) {
    const auto t_start = clk::now();
    combo_stats& S = out.st;
    double mu0, kappa0;
    reference_medium(ctx, mu0, kappa0);
    double tol_cg = ctx->opt.tol_cg;
    if (sizeof(T) == 4) tol_cg = std::max(tol_cg, 1e-5);
    const int K = std::max(1, ctx->opt.n_increments);
    HIP_OR_FAIL(hipMemsetAsync(ctx->a_prev.p, 0, sizeof(double) * 3 * lam_points(ctx), ctx->stream));
    auto load = [&](double t, int c) { return Fbar0[c] + t * (Fbar[c] - Fbar0[c]); };
    double* Fc = ctx->F_cur.as<double>();
    double* Ft = ctx->F_trial.as<double>();
    const size_t f9 = sizeof(double) * 9 * (size_t)ctx->g.n;
    double eta = 0.0;
    for (int k = 1; k <= K; ++k) {
        const double t0 = double(k - 1) / K, t1 = double(k) / K;
        double dt = t1 - t0, t = t0;
        int depth = 0;
        while (t < t1 - 1e-15) {
            const double tn = std::min(t1, t + dt);
            double dFbar[9];
            for (int c = 0; c < 9; ++c) dFbar[c] = load(tn, c) - load(t, c);
            HIP_OR_FAIL(hipMemcpyAsync(ctx->F_save.p, Fc, f9, hipMemcpyDeviceToDevice, ctx->stream));
            bool converged = false;
            auto tm = clk::now();
            int st = material<T>(ctx, Fc, nullptr, 0.0, dFbar, Ft, false, nullptr, nullptr, nullptr);
            S.time_ms_material += ms_since(tm);
            if (st) return st;
            if (material_failures(ctx) == 0.0) {
                std::swap(ctx->F_cur.p, ctx->F_trial.p);
                std::swap(ctx->a_prev.p, ctx->a_trial.p);
                Fc = ctx->F_cur.as<double>();
                Ft = ctx->F_trial.as<double>();
                bool have_eta = false;   // the line search left the residual of the accepted step
                for (int it_n = 0; it_n <= ctx->opt.max_newton; ++it_n) {
                    if (!have_eta) {
                        auto tr = clk::now();
                        st = residual<T>(ctx, mu0, kappa0, tol_cg, eta);
                        S.time_ms_residual += ms_since(tr);
                        if (st) return st;
                    }
                    have_eta = false;
                    if (verbose())
                        fprintf(stderr, "[combo] increment %d t=%.4f newton %d eta %.3e rho0 %.3e fails %g\n", k, tn,
                                it_n, eta, ctx->hs->cg.rho0, material_failures(ctx));
                    if (!(eta == eta)) return set_err(ctx, COMBO_E_NUMERIC, "NaN in the equilibrium residual");
                    if (eta <= ctx->opt.tol_newton) {
                        converged = true;
                        break;
                    }
                    if (it_n == ctx->opt.max_newton) break;
                    auto tc = clk::now();
                    int cgit = 0;
                    st = cg_solve<T>(ctx, mu0, kappa0, cgit);
                    S.time_ms_cg += ms_since(tc);
                    S.cg_iters_total += cgit;
                    if (st == kNegCurv) {
                        // truncated Newton: step along the iterate reached so far, or
                        // halve the increment if there is none
                        S.cg_truncations += 1;
                        st = COMBO_OK;
                        if (cgit == 0) break;
                    }
                    if (st) {
                        S.eta_final = eta;
                        return st;
                    }
                    S.newton_iters += 1;
                    st = newton_direction<T>(ctx);
                    if (st) return st;
                    // step control: admissible law everywhere and, with the line search,
                    // sufficient decrease of the residual, eta(s) <= (1 - 1e-4 s) eta
                    double s = 1.0;
                    bool ok = false;
                    for (int h = 0; h <= ctx->opt.max_step_halvings; ++h) {
                        tm = clk::now();
                        st = material<T>(ctx, Fc, ctx->dF.as<double>(), s, nullptr, Ft, false, nullptr, nullptr,
                                         nullptr);
                        S.time_ms_material += ms_since(tm);
                        if (st) return st;
                        if (material_failures(ctx) == 0.0) {
                            if (!ctx->opt.line_search) {
                                ok = true;
                                break;
                            }
                            double eta_t = 0.0;
                            auto tr = clk::now();
                            st = residual<T>(ctx, mu0, kappa0, tol_cg, eta_t);
                            S.time_ms_residual += ms_since(tr);
                            if (st) return st;
                            if (eta_t <= (1.0 - kArmijo * s) * eta) {
                                eta = eta_t;
                                have_eta = true;
                                ok = true;
                                break;
                            }
                        }
                        s *= 0.5;
                        S.step_halvings += 1;
                    }
                    if (!ok) break;
                    std::swap(ctx->F_cur.p, ctx->F_trial.p);
                    std::swap(ctx->a_prev.p, ctx->a_trial.p);
                    Fc = ctx->F_cur.as<double>();
                    Ft = ctx->F_trial.as<double>();
                }
            }
            if (converged) {
                const double* sm = ctx->hs->sums;
                S.laminate_iters_total += (long long)sm[47];
                S.laminate_backprojections += (long long)sm[48];
                S.laminate_iters_max = std::max(S.laminate_iters_max, (int)sm[49]);
                S.increments_done += 1;
                t = tn;
            } else {
                HIP_OR_FAIL(hipMemcpyAsync(Fc, ctx->F_save.p, f9, hipMemcpyDeviceToDevice, ctx->stream));
                S.laminate_failures += (long long)(ctx->hs->sums[46]);
                depth += 1;
                S.cutbacks += 1;
                if (depth > ctx->opt.max_cutbacks) {
                    S.eta_final = eta;
                    return set_err(ctx, COMBO_E_NOCONV, "load increment " + std::to_string(k) + " failed after " +
                                                            std::to_string(ctx->opt.max_cutbacks) + " cutbacks");
                }
                dt *= 0.5;
            }
        }
    }
    S.eta_final = eta;
    // effective stress and phase averages from the last (accepted) evaluation
    const double* sm = ctx->hs->sums;
    for (int c = 0; c < 9; ++c) {
        out.Pbar[c] = (sm[c] + sm[9 + c] + sm[19 + c]) / (double)ctx->g.n;
        const double vp = ctx->n_incl + ctx->sum_c, vm = ctx->n_mat + ((double)ctx->nc - ctx->sum_c);
        out.Pp[c] = vp > 0 ? (sm[9 + c] + sm[28 + c]) / vp : 0.0;
        out.Pm[c] = vm > 0 ? (sm[c] + sm[37 + c]) / vm : 0.0;
    }
    if (Abar) {
        auto tt = clk::now();
        int it = 0;
        int st = effective_tangent<T>(ctx, mu0, kappa0, tol_cg, Abar, it);
        S.time_ms_tangent += ms_since(tt);
        S.cg_iters_tangent = it;
        if (st) return st;
    }
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx);
    S.time_ms_total = ms_since(t_start);
    return COMBO_OK;
}

// ------------------------------------------------------------------------------
// batched solve: many RVEs, one launch per pass and kernel shape
// ------------------------------------------------------------------------------
int bset_err(combo_batch* b, int status, const std::string& msg) {
    if (b) b->err = msg;
    return status;
}

#define BHIP_OR_FAIL(...)                                                                                   \
    do {                                                                                                    \
        hipError_t e__ = (__VA_ARGS__);                                                                     \
        if (e__ != hipSuccess)                                                                              \
            return bset_err(B, e__ == hipErrorOutOfMemory ? COMBO_E_NOMEM : COMBO_E_HIP,                    \
                            std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e__));                     \
    } while (0)

// Argument tables and tile maps of a set of batched launches, built on the host,
// uploaded in one copy, then launched in order.
struct LaunchPlan {
    std::vector<char> host;
    std::vector<std::function<hipError_t(char*)>> ops;
    DevBuf dev;
    char* pinned = nullptr;   // staging for asynchronous uploads
    size_t pinned_cap = 0;
    LaunchPlan() = default;
    LaunchPlan(const LaunchPlan&) = delete;
    LaunchPlan& operator=(const LaunchPlan&) = delete;
    ~LaunchPlan() {
        if (pinned) (void)hipHostFree(pinned);
    }
    size_t put(const void* src, size_t bytes) {
        const size_t off = (host.size() + 255) & ~(size_t)255;
        host.resize(off + bytes);
        if (bytes) memcpy(host.data() + off, src, bytes);
        return off;
    }
    void clear() {
        host.clear();
        ops.clear();
    }
    // Copies the tables to the device, in stream order.  Nothing may be in flight on
    // the stream that reads `dev` or `pinned` (the batch synchronises every tick).
    hipError_t upload(hipStream_t s) {
        if (host.empty()) return hipSuccess;
        hipError_t e = dev.ensure(host.size());
        if (e != hipSuccess) return e;
        if (pinned_cap < host.size()) {
            if (pinned) (void)hipHostFree(pinned);
            pinned = nullptr;
            pinned_cap = 0;
            e = hipHostMalloc((void**)&pinned, host.size() * 2, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            pinned_cap = host.size() * 2;
        }
        memcpy(pinned, host.data(), host.size());
        return hipMemcpyAsync(dev.p, pinned, host.size(), hipMemcpyHostToDevice, s);
    }
    hipError_t run() const {
        for (const auto& op : ops) {
            hipError_t e = op(static_cast<char*>(dev.p));
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
};

// One pass over the members whose argument blocks are `args`: one launch per
// distinct key (the kernel shape), over the nblk[i] tiles of each member i.
template <class A, class F>
void plan_pass(LaunchPlan& lp, const std::vector<A>& args, const std::vector<long long>& key,
               const std::vector<int>& nblk, F launch) {
    if (args.empty()) return;
    const size_t aoff = lp.put(args.data(), sizeof(A) * args.size());
    std::vector<int> idx(args.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return key[a] < key[b]; });
    for (size_t g0 = 0; g0 < idx.size();) {
        size_t g1 = g0;
        while (g1 < idx.size() && key[idx[g1]] == key[idx[g0]]) ++g1;
        std::vector<TileMap> map;
        for (size_t k = g0; k < g1; ++k) {
            const int i = idx[k];
            for (int t = 0; t < nblk[i]; ++t) map.push_back(TileMap{i, t, nblk[i]});
        }
        const size_t moff = lp.put(map.data(), sizeof(TileMap) * map.size());
        const A rep = args[idx[g0]];
        const int nb = (int)map.size();
        lp.ops.push_back([=](char* base) -> hipError_t {
            BatchLaunch bl{base + aoff, reinterpret_cast<const TileMap*>(base + moff), nb};
            return launch(rep, &bl);
        });
        g0 = g1;
    }
}

void plan_finalize(LaunchPlan& lp, int mode, const std::vector<FinArgs>& f, hipStream_t s) {
    if (f.empty()) return;
    const size_t off = lp.put(f.data(), sizeof(FinArgs) * f.size());
    const int cnt = (int)f.size();
    const FinArgs rep = f[0];
    lp.ops.push_back([=](char* base) -> hipError_t {
        return launch_finalize(mode, rep, s, reinterpret_cast<const FinArgs*>(base + off), cnt);
    });
}

// launch-group key: axis length, schedule variant and discretization, tile width or rows
long long key2(long long len, long long tile, int variant = 0) { return (len << 40) | ((long long)variant << 32) | tile; }
// the discretization selects other kernel instances: members that differ in it never share a launch
int vkey(const Grid& g, int variant) { return variant + 64 * g.disc; }

enum MemberPhase { PH_INC = 0, PH_RES, PH_CG, PH_STEP, PH_LSRES, PH_DONE, PH_FAIL };

struct Member {
    combo_ctx* ctx = nullptr;
    int index = 0;
    size_t slot = 0;   // position of the member's CG state and sums in the batch's scalar array
    double Fbar[9]{}, Fbar0[9]{};
    int K = 1;
    double mu0 = 0, kappa0 = 0, tol_cg = 0;
    int phase = PH_INC;
    int k = 1, depth = 0, it_n = 0, h = 0, cg_rounds = 0;
    double t = 0, t1 = 0, dt = 0, tn = 0, s = 1.0, eta = 0.0;
    double dFbar[9]{};
    SolveOut out;
    int status = COMBO_OK;
    double load(double tt, int c) const { return Fbar0[c] + tt * (Fbar[c] - Fbar0[c]); }
};

void member_fail(Member& m, int status, const std::string& msg) {
    m.status = status;
    m.ctx->err = msg;
    m.phase = PH_FAIL;
    m.out.st.eta_final = m.eta;
}

void member_begin_substep(Member& m) {
    m.tn = std::min(m.t1, m.t + m.dt);
    for (int c = 0; c < 9; ++c) m.dFbar[c] = m.load(m.tn, c) - m.load(m.t, c);
    m.phase = PH_INC;
}

void member_begin_increment(Member& m) {
    const double t0 = double(m.k - 1) / m.K;
    m.t1 = double(m.k) / m.K;
    m.dt = m.t1 - t0;
    m.t = t0;
    m.depth = 0;
    member_begin_substep(m);
}

// the load step did not converge: restore F, halve the increment
int member_cutback(Member& m) {
    combo_ctx* ctx = m.ctx;
    HIP_OR_FAIL(hipMemcpyAsync(ctx->F_cur.p, ctx->F_save.p, sizeof(double) * 9 * (size_t)ctx->g.n,
                               hipMemcpyDeviceToDevice, ctx->stream));
    m.out.st.laminate_failures += (long long)(ctx->hs->sums[46]);
    m.depth += 1;
    m.out.st.cutbacks += 1;
    if (m.depth > ctx->opt.max_cutbacks) {
        member_fail(m, COMBO_E_NOCONV, "load increment " + std::to_string(m.k) + " failed after " +
                                           std::to_string(ctx->opt.max_cutbacks) + " cutbacks");
        return COMBO_OK;
    }
    m.dt *= 0.5;
    member_begin_substep(m);
    return COMBO_OK;
}

void member_accept_swap(Member& m) {
    std::swap(m.ctx->F_cur.p, m.ctx->F_trial.p);
    std::swap(m.ctx->a_prev.p, m.ctx->a_trial.p);
}

void member_finish(Member& m) {
    combo_ctx* ctx = m.ctx;
    const double* sm = ctx->hs->sums;
    m.out.st.eta_final = m.eta;
    for (int c = 0; c < 9; ++c) {
        m.out.Pbar[c] = (sm[c] + sm[9 + c] + sm[19 + c]) / (double)ctx->g.n;
        const double vp = ctx->n_incl + ctx->sum_c, vm = ctx->n_mat + ((double)ctx->nc - ctx->sum_c);
        m.out.Pp[c] = vp > 0 ? (sm[9 + c] + sm[28 + c]) / vp : 0.0;
        m.out.Pm[c] = vm > 0 ? (sm[c] + sm[37 + c]) / vm : 0.0;
    }
    m.phase = PH_DONE;
}

// eta of the member's last residual evaluation
double member_eta(const Member& m) {
    const combo_ctx* ctx = m.ctx;
    double Pbar[9];
    material_pbar(ctx, Pbar);
    const double den = (double)ctx->g.n * std::max(frob9(Pbar), 1e-300);
    return std::sqrt(std::max(ctx->hs->cg.eta2, 0.0)) / den;
}

// Newton test after a residual at the current F (m.eta set)
int member_after_residual(Member& m) {
    combo_ctx* ctx = m.ctx;
    combo_stats& S = m.out.st;
    if (verbose())
        fprintf(stderr, "[combo] member %d increment %d t=%.4f newton %d eta %.3e\n", m.index, m.k, m.tn, m.it_n,
                m.eta);
    if (!(m.eta == m.eta)) {
        member_fail(m, COMBO_E_NUMERIC, "NaN in the equilibrium residual");
        return COMBO_OK;
    }
    if (m.eta <= ctx->opt.tol_newton) {
        const double* sm = ctx->hs->sums;
        S.laminate_iters_total += (long long)sm[47];
        S.laminate_backprojections += (long long)sm[48];
        S.laminate_iters_max = std::max(S.laminate_iters_max, (int)sm[49]);
        S.increments_done += 1;
        m.t = m.tn;
        if (m.t < m.t1 - 1e-15) {
            member_begin_substep(m);
        } else if (m.k < m.K) {
            m.k += 1;
            member_begin_increment(m);
        } else {
            member_finish(m);
        }
        return COMBO_OK;
    }
    if (m.it_n == ctx->opt.max_newton) return member_cutback(m);
    m.cg_rounds = 0;
    m.phase = PH_CG;
    return COMBO_OK;
}

// the trial step was rejected: halve it, or give up the increment
int member_halve_step(Member& m) {
    m.s *= 0.5;
    m.out.st.step_halvings += 1;
    m.h += 1;
    if (m.h > m.ctx->opt.max_step_halvings) return member_cutback(m);
    m.phase = PH_STEP;
    return COMBO_OK;
}

// host decision after the tick's scalars have been read back
int member_advance(Member& m) {
    combo_ctx* ctx = m.ctx;
    combo_stats& S = m.out.st;
    switch (m.phase) {
        case PH_INC:
            if (material_failures(ctx) == 0.0) {
                member_accept_swap(m);
                m.it_n = 0;
                m.phase = PH_RES;
                return COMBO_OK;
            }
            return member_cutback(m);
        case PH_RES:
            m.eta = member_eta(m);
            return member_after_residual(m);
        case PH_CG: {
            const CGState& cg = ctx->hs->cg;
            if (!cg.done) {
                m.cg_rounds += 1;
                if (m.cg_rounds > ctx->opt.max_cg / 8 + 2) member_fail(m, COMBO_E_NOCONV, "CG did not terminate");
                return COMBO_OK;
            }
            S.cg_iters_total += cg.iter;
            if (cg.status == 1) {
                member_fail(m, COMBO_E_NUMERIC, "CG breakdown (<p, A p> is NaN)");
                return COMBO_OK;
            }
            if (cg.status == 3) {
                // truncated Newton, as in the single solve
                S.cg_truncations += 1;
                if (cg.iter == 0) return member_cutback(m);
            }
            if (cg.status == 2) {
                member_fail(m, COMBO_E_NOCONV, "CG did not converge in max_cg iterations");
                return COMBO_OK;
            }
            S.newton_iters += 1;
            m.s = 1.0;
            m.h = 0;
            m.phase = PH_STEP;
            return COMBO_OK;
        }
        case PH_STEP:
            if (material_failures(ctx) == 0.0) {
                if (ctx->opt.line_search) {
                    m.phase = PH_LSRES;   // residual of the trial before it is taken
                    return COMBO_OK;
                }
                member_accept_swap(m);
                m.it_n += 1;
                m.phase = PH_RES;
                return COMBO_OK;
            }
            return member_halve_step(m);
        case PH_LSRES: {
            const double eta_t = member_eta(m);
            if (eta_t <= (1.0 - kArmijo * m.s) * m.eta) {
                member_accept_swap(m);
                m.it_n += 1;
                m.eta = eta_t;
                return member_after_residual(m);
            }
            m.phase = PH_STEP;
            return member_halve_step(m);
        }
        default: return COMBO_OK;
    }
}

template <typename T>
MatArgs<T> member_matargs(const Member& m) {
    combo_ctx* ctx = m.ctx;
    MatArgs<T> a{};
    a.n = ctx->g.n;
    a.nc = ctx->nc;
    a.F_old = ctx->F_cur.as<double>();
    if (m.phase == PH_INC) {
        a.dF = nullptr;
        a.s = 0.0;
        for (int c = 0; c < 9; ++c) a.dFbar[c] = m.dFbar[c];
    } else {
        a.dF = ctx->dF.as<double>();
        a.s = m.s;
    }
    a.F_new = ctx->F_trial.as<double>();
    a.P = ctx->P.as<double>();
    a.slot = ctx->slot.as<int>();
    for (int p = 0; p < 2; ++p) {
        a.mu[p] = ctx->mats[p].mu;
        a.lam[p] = ctx->mats[p].lambda;
    }
    a.comp_vox = ctx->comp_vox.as<int>();
    a.cc = ctx->comp_c.as<double>();
    a.NN = ctx->comp_N.as<double>();
    a.a_prev = ctx->a_prev.as<double>();
    a.a_out = ctx->a_trial.as<double>();
    a.warm = ctx->opt.warm_start_laminate ? 1 : 0;
    a.maxit = ctx->opt.max_laminate;
    a.law = ctx->opt.law;
    a.Sinv = ctx->Sinv.as<T>();
    a.sm = ctx->sm.as<T>();
    a.n1 = ctx->g.n1;
    a.xm = ctx->g.xm;
    a.xwbits = ctx->g.xwbits;
    a.Acomp = ctx->Acomp.as<T>();
    a.partials = ctx->part1.as<double>();
    a.partials2 = ctx->part2.as<double>();
    return a;
}

// the launches of one tick: increment starts, Newton directions, material
// updates, residuals (the CG chunk has its own cached plan)
template <typename T>
void plan_tick(std::vector<Member>& ms, const std::vector<int>& list, LaunchPlan& lp, hipStream_t s) {
    lp.clear();
    // F_save <- F at the start of a (sub)increment
    for (int mi : list) {
        Member& m = ms[mi];
        if (m.phase != PH_INC) continue;
        combo_ctx* ctx = m.ctx;
        void* dst = ctx->F_save.p;
        const void* src = ctx->F_cur.p;
        const size_t bytes = sizeof(double) * 9 * (size_t)ctx->g.n;
        lp.ops.push_back([=](char*) { return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s); });
    }
    // Newton directions dF from the CG solutions (first trial of a step only)
    {
        std::vector<ZArgs<double, T>> za;
        std::vector<YArgs<double>> ya;
        std::vector<XArgs<double>> xa;
        std::vector<long long> kz, ky, kx;
        std::vector<int> nz, ny, nx;
        for (int mi : list) {
            Member& m = ms[mi];
            if (m.phase != PH_STEP || m.h != 0) continue;
            combo_ctx* ctx = m.ctx;
            ZArgs<double, T> z = zargs<double, T>(ctx, 1.0, 0.0);
            z.out = ctx->specA.as<double2>();
            za.push_back(z);
            kz.push_back(key2(ctx->g.n3, z.TX, vkey(ctx->g, ctx->g.zv)));
            nz.push_back(blocks_z(ctx->g, z.TX));
            YArgs<double> y = yargs<double>(ctx, ctx->specA.p, ctx->specB.p, false);
            ya.push_back(y);
            ky.push_back(key2(ctx->g.n2, y.TX, vkey(ctx->g, ctx->g.yv)));
            ny.push_back(blocks_y(ctx->g, y.TX));
            XArgs<double> x = xargs<double>(ctx);
            x.in = ctx->specB.as<double2>();
            x.real_out = ctx->dF.as<double>();
            xa.push_back(x);
            kx.push_back(key2(ctx->g.n1, x.R, vkey(ctx->g, ctx->g.xv)));
            nx.push_back(blocks_x(ctx->g, x.R, X_INV_REAL, false));
        }
        plan_pass(lp, za, kz, nz, [=](const ZArgs<double, T>& a, const BatchLaunch* bl) {
            return launch_z<double, T>(Z_INV_PLAIN, a, s, nullptr, bl);
        });
        plan_pass(lp, ya, ky, ny,
                  [=](const YArgs<double>& a, const BatchLaunch* bl) { return launch_y<double>(+1, a, s, bl); });
        plan_pass(lp, xa, kx, nx, [=](const XArgs<double>& a, const BatchLaunch* bl) {
            return launch_x<double>(X_INV_REAL, a, s, nullptr, bl);
        });
    }
    // material law at the trial fields
    {
        std::vector<MatArgs<T>> ma;
        std::vector<MatReduceArgs> red;
        std::vector<TileMap> mp, ml;
        for (int mi : list) {
            Member& m = ms[mi];
            if (m.phase != PH_INC && m.phase != PH_STEP) continue;
            combo_ctx* ctx = m.ctx;
            const int i = (int)ma.size();
            ma.push_back(member_matargs<T>(m));
            const int nbp = material_blocks_pure(ctx->g.n);
            const int nbl = ctx->nc > 0 ? material_blocks_laminate(ctx->nc) : 0;
            for (int t = 0; t < nbp; ++t) mp.push_back(TileMap{i, t, nbp});
            for (int t = 0; t < nbl; ++t) ml.push_back(TileMap{i, t, nbl});
            red.push_back(MatReduceArgs{ctx->part1.as<double>(), nbp, ctx->part2.as<double>(), nbl,
                                        ctx->sums.as<double>()});
            ctx->state_prec = sizeof(T) == 4 ? COMBO_MIXED : COMBO_FP64;
        }
        if (!ma.empty()) {
            const size_t aoff = lp.put(ma.data(), sizeof(MatArgs<T>) * ma.size());
            const size_t poff = lp.put(mp.data(), sizeof(TileMap) * mp.size());
            const size_t loff = lp.put(ml.data(), sizeof(TileMap) * ml.size());
            const size_t roff = lp.put(red.data(), sizeof(MatReduceArgs) * red.size());
            const int np = (int)mp.size(), nl = (int)ml.size(), nr = (int)red.size();
            lp.ops.push_back([=](char* base) -> hipError_t {
                BatchLaunch pure{nullptr, reinterpret_cast<const TileMap*>(base + poff), np};
                BatchLaunch lam{nullptr, reinterpret_cast<const TileMap*>(base + loff), nl};
                return launch_material_batch<T>(reinterpret_cast<const MatArgs<T>*>(base + aoff), pure, lam,
                                                reinterpret_cast<const MatReduceArgs*>(base + roff), nr, s);
            });
        }
    }
    // residuals: FP64 forward passes of P, right-hand sides, eta
    {
        std::vector<XArgs<double>> xa;
        std::vector<YArgs<double>> ya;
        std::vector<ZArgs<double, T>> za;
        std::vector<UArgs<T>> ua;
        std::vector<FinArgs> fa;
        std::vector<long long> kx, ky, kz, ku;
        std::vector<int> nx, ny, nz, nu;
        for (int mi : list) {
            Member& m = ms[mi];
            if (m.phase != PH_RES && m.phase != PH_LSRES) continue;
            combo_ctx* ctx = m.ctx;
            XArgs<double> x = xargs<double>(ctx);
            x.real_in = ctx->P.as<double>();
            x.out = ctx->specA.as<double2>();
            xa.push_back(x);
            kx.push_back(key2(ctx->g.n1, x.R, vkey(ctx->g, ctx->g.xv)));
            nx.push_back(blocks_x(ctx->g, x.R, X_FWD_REAL, false));
            YArgs<double> y = yargs<double>(ctx, ctx->specA.p, ctx->specB.p, false);
            ya.push_back(y);
            ky.push_back(key2(ctx->g.n2, y.TX, vkey(ctx->g, ctx->g.yv)));
            ny.push_back(blocks_y(ctx->g, y.TX));
            ZArgs<double, T> z = zargs<double, T>(ctx, m.mu0, m.kappa0);
            z.in = ctx->specB.as<double2>();
            za.push_back(z);
            kz.push_back(key2(ctx->g.n3, z.TX, vkey(ctx->g, ctx->g.zv)));
            const int nbz = blocks_z(ctx->g, z.TX);
            nz.push_back(nbz);
            ua.push_back(uargs<T>(ctx, m.mu0, m.kappa0));
            ku.push_back(0);
            nu.push_back(blocks_antiherm(ctx->g));
            fa.push_back(finargs(ctx, ctx->part1.as<double>(), ctx->part2.as<double>(), nbz, m.tol_cg * m.tol_cg,
                                 ctx->opt.max_cg));
        }
        plan_pass(lp, xa, kx, nx, [=](const XArgs<double>& a, const BatchLaunch* bl) {
            return launch_x<double>(X_FWD_REAL, a, s, nullptr, bl);
        });
        plan_pass(lp, ya, ky, ny,
                  [=](const YArgs<double>& a, const BatchLaunch* bl) { return launch_y<double>(-1, a, s, bl); });
        plan_pass(lp, za, kz, nz, [=](const ZArgs<double, T>& a, const BatchLaunch* bl) {
            return launch_z<double, T>(Z_RHS, a, s, nullptr, bl);
        });
        plan_pass(lp, ua, ku, nu, [=](const UArgs<T>& a, const BatchLaunch* bl) { return launch_antiherm<T>(a, s, bl); });
        plan_finalize(lp, FIN_RHS, fa, s);
    }
}

// one CG iteration over the members listed (8 launches per kernel shape)
template <typename T>
void plan_cg(std::vector<Member>& ms, const std::vector<int>& list, LaunchPlan& lp, hipStream_t s) {
    lp.clear();
    std::vector<ZArgs<T, T>> zi, zf;
    std::vector<YArgs<T>> yi, yf;
    std::vector<XArgs<T>> xa;
    std::vector<UArgs<T>> ua;
    std::vector<FinArgs> fal, fbe;
    std::vector<long long> kz, ky, kx, ku;
    std::vector<int> nz, ny, nx, nu;
    for (int i : list) {
        Member& m = ms[i];
        combo_ctx* ctx = m.ctx;
        ZArgs<T, T> z = zargs<T, T>(ctx, m.mu0, m.kappa0);
        z.out = ctx->specA.as<cpx<T>>();
        zi.push_back(z);
        z.in = ctx->specB.as<cpx<T>>();
        z.out = nullptr;
        zf.push_back(z);
        kz.push_back(key2(ctx->g.n3, z.TX, vkey(ctx->g, ctx->g.zv)));
        const int nbz = blocks_z(ctx->g, z.TX);
        nz.push_back(nbz);
        YArgs<T> yv = yargs<T>(ctx, ctx->specA.p, ctx->specB.p, true);
        yi.push_back(yv);
        yf.push_back(yv);
        ky.push_back(key2(ctx->g.n2, yv.TX, vkey(ctx->g, ctx->g.yv)));
        ny.push_back(blocks_y(ctx->g, yv.TX));
        XArgs<T> x = xargs<T>(ctx);
        x.in = ctx->specB.as<cpx<T>>();
        x.out = ctx->specA.as<cpx<T>>();
        xa.push_back(x);
        kx.push_back(key2(ctx->g.n1, x.R, vkey(ctx->g, ctx->g.xv)));
        nx.push_back(blocks_x(ctx->g, x.R, X_CG, sizeof(T) == 4));
        ua.push_back(uargs<T>(ctx, m.mu0, m.kappa0));
        ku.push_back(0);
        const int nbu = blocks_u(ctx->g);
        nu.push_back(nbu);
        fal.push_back(finargs(ctx, ctx->part1.as<double>(), nullptr, nbz));
        fbe.push_back(finargs(ctx, ctx->part2.as<double>(), nullptr, nbu));
    }
    plan_pass(lp, zi, kz, nz,
              [=](const ZArgs<T, T>& a, const BatchLaunch* bl) { return launch_z<T, T>(Z_INV_CG, a, s, nullptr, bl); });
    plan_pass(lp, yi, ky, ny, [=](const YArgs<T>& a, const BatchLaunch* bl) { return launch_y<T>(+1, a, s, bl); });
    plan_pass(lp, xa, kx, nx,
              [=](const XArgs<T>& a, const BatchLaunch* bl) { return launch_x<T>(X_CG, a, s, nullptr, bl); });
    plan_pass(lp, yf, ky, ny, [=](const YArgs<T>& a, const BatchLaunch* bl) { return launch_y<T>(-1, a, s, bl); });
    plan_pass(lp, zf, kz, nz,
              [=](const ZArgs<T, T>& a, const BatchLaunch* bl) { return launch_z<T, T>(Z_CG, a, s, nullptr, bl); });
    plan_finalize(lp, FIN_ALPHA, fal, s);
    plan_pass(lp, ua, ku, nu, [=](const UArgs<T>& a, const BatchLaunch* bl) { return launch_update<T>(a, s, nullptr, bl); });
    plan_finalize(lp, FIN_BETA, fbe, s);
}

// A lane: the members whose passes share launches, on a stream of their own.  Lanes
// run their ticks independently (each on a host thread of its own), so members of
// small grids with long Newton-CG chains progress at their own pace beside the
// launches of larger grids instead of waiting for them every iteration.
struct Lane {
    std::vector<int> members;   // indices into the member list; their scalar slots are contiguous
    size_t slot0 = 0;           // first scalar slot of the lane
    hipStream_t stream = nullptr;
    LaunchPlan tick, cgp;
    std::vector<int> cg_list, cg_prev;
    bool cg_valid = false;
    hipGraph_t cg_graph = nullptr;
    hipGraphExec_t cg_exec = nullptr;
    int cg_same = 0;
    int status = COMBO_OK;
    std::string err;
    long long ticks = 0, cg_ticks = 0, graph_ticks = 0, cg_rebuilds = 0;
    double host_ms = 0.0, wait_ms = 0.0, wall_ms = 0.0;
    Lane() = default;
    Lane(const Lane&) = delete;
    Lane& operator=(const Lane&) = delete;
    void drop_graph() {
        if (cg_exec) (void)hipGraphExecDestroy(cg_exec);
        if (cg_graph) (void)hipGraphDestroy(cg_graph);
        cg_exec = nullptr;
        cg_graph = nullptr;
    }
    ~Lane() { drop_graph(); }
};

// Members -> at most L lanes.  Members of one grid shape (n1, n2, n3, discretization)
// share a lane; shapes are ordered by voxel count and cut into contiguous lanes of
// about nm / L members each.  With fewer shapes than L, the most populated shapes are
// split over the spare lanes.  Returns member lists in ascending grid size.
std::vector<std::vector<int>> assign_lanes(const std::vector<combo_ctx*>& mem, int L) {
    const int nm = (int)mem.size();
    std::vector<int> order(nm);
    for (int i = 0; i < nm; ++i) order[i] = i;
    auto key = [&](int i) {
        const Grid& g = mem[i]->g;
        return std::make_tuple(g.n, g.n1, g.n2, g.n3, g.disc);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    std::vector<std::vector<int>> shapes;
    for (int k = 0; k < nm; ++k) {
        if (k == 0 || key(order[k]) != key(order[k - 1])) shapes.emplace_back();
        shapes.back().push_back(order[k]);
    }
    if ((int)shapes.size() <= L) {
        // spare lanes: split the most populated lanes (members dealt alternately), so that a long
        // Newton-CG chain of one member holds up fewer of its shape's members
        while ((int)shapes.size() < L) {
            size_t big = 0;
            for (size_t k = 1; k < shapes.size(); ++k)
                if (shapes[k].size() > shapes[big].size()) big = k;
            if (shapes[big].size() < 2) break;
            std::vector<int> a, b;
            for (size_t k = 0; k < shapes[big].size(); ++k) (k % 2 ? b : a).push_back(shapes[big][k]);
            shapes[big] = a;
            shapes.insert(shapes.begin() + big + 1, b);
        }
        return shapes;
    }
    std::vector<std::vector<int>> lanes;
    const double target = (double)nm / L;
    for (const auto& sh : shapes) {
        if (lanes.empty() || ((double)lanes.back().size() >= target && (int)lanes.size() < L)) lanes.emplace_back();
        for (int i : sh) lanes.back().push_back(i);
    }
    return lanes;
}

// COMBO_BATCH_STATS=1 in the environment prints one line per batch solve: per lane
// its members, ticks, host time, time waiting for its stream and wall time.
bool batch_stats() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("COMBO_BATCH_STATS");
        v = (e && e[0] && e[0] != '0') ? 1 : 0;
    }
    return v == 1;
}

// a HIP failure inside a lane: recorded in the lane (lanes run on threads of their own)
#define LHIP_OR_FAIL(ln, ...)                                                                          \
    do {                                                                                             \
        hipError_t e__ = (__VA_ARGS__);                                                              \
        if (e__ != hipSuccess) {                                                                     \
            (ln).err = std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e__);                    \
            return e__ == hipErrorOutOfMemory ? COMBO_E_NOMEM : COMBO_E_HIP;                         \
        }                                                                                            \
    } while (0)

// Plans and enqueues one tick of a lane: its members' non-CG work, then a CG chunk
// for the members in CG, then the copy of the lane's scalar slots to the host.
template <typename T>
int lane_launch(combo_batch* B, std::vector<Member>& ms, Lane& ln, int chunk, bool use_graph) {
    const size_t stride = combo_batch::kScalStride;
    ++ln.ticks;
    plan_tick<T>(ms, ln.members, ln.tick, ln.stream);
    LHIP_OR_FAIL(ln, ln.tick.upload(ln.stream));
    ln.cg_list.clear();
    for (int i : ln.members)
        if (ms[i].phase == PH_CG) ln.cg_list.push_back(i);
    if (!ln.cg_list.empty() && (!ln.cg_valid || ln.cg_list != ln.cg_prev)) {
        ln.drop_graph();
        ln.cg_same = 0;
        plan_cg<T>(ms, ln.cg_list, ln.cgp, ln.stream);
        LHIP_OR_FAIL(ln, ln.cgp.upload(ln.stream));
        ln.cg_prev = ln.cg_list;
        ln.cg_valid = true;
        ++ln.cg_rebuilds;
    } else if (!ln.cg_list.empty()) {
        ++ln.cg_same;
    }
    LHIP_OR_FAIL(ln, ln.tick.run());
    if (!ln.cg_list.empty()) {
        ++ln.cg_ticks;
        if (use_graph && ln.cg_same >= 1 && !ln.cg_exec) {
            LHIP_OR_FAIL(ln, hipStreamBeginCapture(ln.stream, hipStreamCaptureModeThreadLocal));
            hipError_t ce = hipSuccess;
            for (int k = 0; k < chunk && ce == hipSuccess; ++k) ce = ln.cgp.run();
            hipError_t ee = hipStreamEndCapture(ln.stream, &ln.cg_graph);
            LHIP_OR_FAIL(ln, ce);
            LHIP_OR_FAIL(ln, ee);
            LHIP_OR_FAIL(ln, hipGraphInstantiate(&ln.cg_exec, ln.cg_graph, nullptr, nullptr, 0));
        }
        if (ln.cg_exec) {
            LHIP_OR_FAIL(ln, hipGraphLaunch(ln.cg_exec, ln.stream));
            ++ln.graph_ticks;
        } else {
            for (int k = 0; k < chunk; ++k) LHIP_OR_FAIL(ln, ln.cgp.run());
        }
    }
    LHIP_OR_FAIL(ln, hipMemcpyAsync(B->hscal + ln.slot0 * stride, static_cast<char*>(B->scal.p) + ln.slot0 * stride,
                                    stride * ln.members.size(), hipMemcpyDeviceToHost, ln.stream));
    return COMBO_OK;
}

// host decisions of a lane whose tick has completed
void lane_advance(combo_batch* B, std::vector<Member>& ms, Lane& ln) {
    const size_t stride = combo_batch::kScalStride;
    for (int i : ln.members) {
        Member& m = ms[i];
        if (m.phase == PH_DONE || m.phase == PH_FAIL) continue;
        const char* src = B->hscal + m.slot * stride;
        memcpy(&m.ctx->hs->cg, src, sizeof(CGState));
        memcpy(m.ctx->hs->sums, src + combo_batch::kScalSums, sizeof(double) * kSumsLen);
        int st = member_advance(m);
        if (st) member_fail(m, st, m.ctx->err);
    }
}

bool lane_active(const std::vector<Member>& ms, const Lane& ln) {
    for (int i : ln.members)
        if (ms[i].phase != PH_DONE && ms[i].phase != PH_FAIL) return true;
    return false;
}

// One lane from start to finish: tick, wait for it on the lane's stream, decide,
// until every member of the lane is done or failed.  Lanes share no member and
// write disjoint ranges of the scalar arrays, so each runs on a host thread of
// its own.
template <typename T>
int lane_run(combo_batch* B, std::vector<Member>& ms, Lane& ln, int chunk, bool use_graph) {
    const auto t_begin = clk::now();
    while (lane_active(ms, ln)) {
        const auto t0 = clk::now();
        const int st = lane_launch<T>(B, ms, ln, chunk, use_graph);
        if (st) {
            ln.status = st;
            break;
        }
        const auto t1 = clk::now();
        ln.host_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
        const hipError_t e = hipStreamSynchronize(ln.stream);
        const auto t2 = clk::now();
        ln.wait_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
        if (e != hipSuccess) {
            ln.err = std::string("batch lane: ") + hipGetErrorString(e);
            ln.status = COMBO_E_HIP;
            break;
        }
        lane_advance(B, ms, ln);
        ln.host_ms += ms_since(t2);
    }
    (void)hipStreamSynchronize(ln.stream);   // nothing of the lane is left in flight, on error as on success
    ln.drop_graph();
    ln.wall_ms = ms_since(t_begin);
    return ln.status;
}

template <typename T>
int batch_solve_impl(combo_batch* B, std::vector<Member>& ms, std::vector<Lane>& lanes) {
    const size_t nm = ms.size();
    // graph_chunk > 0: CG chunks of that many iterations, captured as a hipGraph once
    // the set of a lane's members in CG has stayed the same for a tick, and replayed until it changes
    const bool use_graph = B->opt.graph_chunk > 0;
    const int chunk = use_graph ? B->opt.graph_chunk : 8;
    const bool stats = batch_stats();
    (void)verbose();   // initialise the environment switches before the lanes' threads read them
    const auto t_begin = clk::now();
    const int dev = B->device;
    std::vector<std::thread> threads;
    for (size_t l = 1; l < lanes.size(); ++l) {
        try {
            threads.emplace_back([&, l]() {
                if (hipSetDevice(dev) != hipSuccess) {
                    lanes[l].status = COMBO_E_HIP;
                    lanes[l].err = "hipSetDevice failed in a batch lane";
                    return;
                }
                lane_run<T>(B, ms, lanes[l], chunk, use_graph);
            });
        } catch (...) {
            lanes[l].status = COMBO_E_HIP;
            lanes[l].err = "could not start the host thread of a batch lane";
        }
    }
    if (!lanes.empty()) lane_run<T>(B, ms, lanes[0], chunk, use_graph);
    for (std::thread& t : threads) t.join();
    for (Lane& ln : lanes)
        if (ln.status) return bset_err(B, ln.status, ln.err);
    if (stats) {
        long long ticks = 0, cg_ticks = 0, graph_ticks = 0, rebuilds = 0;
        std::string per;
        char buf[128];
        for (const Lane& ln : lanes) {
            ticks += ln.ticks;
            cg_ticks += ln.cg_ticks;
            graph_ticks += ln.graph_ticks;
            rebuilds += ln.cg_rebuilds;
            snprintf(buf, sizeof(buf), " [%zu members, %lld ticks, host %.0f ms, wait %.0f ms, wall %.0f ms]",
                     ln.members.size(), ln.ticks, ln.host_ms, ln.wait_ms, ln.wall_ms);
            per += buf;
        }
        fprintf(stderr, "[combo] batch: %zu members in %zu lanes%s; %lld ticks (%lld with CG, %lld from a graph, %lld CG "
                        "plan rebuilds), wall %.1f ms\n",
                nm, lanes.size(), per.c_str(), ticks, cg_ticks, graph_ticks, rebuilds, ms_since(t_begin));
    }
    return COMBO_OK;
}

const char* options_error(const combo_options* o) {
    if (o->precision != COMBO_FP64 && o->precision != COMBO_MIXED) return "precision must be COMBO_FP64 or COMBO_MIXED";
    if (!(o->tol_newton > 0) || !(o->tol_cg > 0) || o->max_newton < 0 || o->max_cg < 1 || o->max_laminate < 0 ||
        o->max_laminate > 64 || o->n_increments < 1 || o->max_step_halvings < 0 || o->max_cutbacks < 0 ||
        o->graph_chunk < 0 || o->graph_chunk > 256 || o->autotune < 0 || o->autotune > 1 ||
        o->line_search < 0 || o->line_search > 1 || (o->law != COMBO_LAW_NEO_HOOKE && o->law != COMBO_LAW_LINEAR) ||
        o->batch_streams < 0 || o->batch_streams > 16)
        return "option out of range";
    return nullptr;
}

int require_ready(combo_ctx* ctx) {
    if (!ctx) return COMBO_E_INVAL;
    if (!ctx->has_grid) return set_err(ctx, COMBO_E_STATE, "combo_set_grid has not been called");
    if (!ctx->has_mats) return set_err(ctx, COMBO_E_STATE, "combo_set_materials has not been called");
    if (!ctx->has_ms) return set_err(ctx, COMBO_E_STATE, "combo_set_microstructure has not been called");
    return COMBO_OK;
}

int copy_in(combo_ctx* ctx, void* dst, const void* src, size_t bytes, int mem_kind) {
    HIP_OR_FAIL(hipMemcpyAsync(dst, src, bytes, mem_kind == COMBO_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                                             : hipMemcpyHostToDevice,
                               ctx->stream));
    return COMBO_OK;
}

int copy_out(combo_ctx* ctx, void* dst, const void* src, size_t bytes, int mem_kind) {
    HIP_OR_FAIL(hipMemcpyAsync(dst, src, bytes, mem_kind == COMBO_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                                             : hipMemcpyDeviceToHost,
                               ctx->stream));
    return COMBO_OK;
}

bool finite9(const double* a) {
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

double det9(const double* F) {
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) + F[2] * (F[3] * F[7] - F[4] * F[6]);
}

}  // namespace

// ==============================================================================
// Static device scratch of combo_image_to_boxels_static.  Each GPU holds its own
// copy of the array from the library's first use on it until the process ends.
// In host code `scratch` only names the symbol: its device address on a GPU is
// looked up once per device (static_scratch_setup, called by combo_create with
// that device current) and only that address is passed to kernels.
// ==============================================================================
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on `device` (the current device); 0 or a HIP error code
hipError_t static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void* static_scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

// ==============================================================================
// C-ABI
// ==============================================================================
extern "C" {

int combo_abi_version(void) { return COMBO_ABI_VERSION; }

const char* combo_strerror(int status) {
    switch (status) {
        case COMBO_OK: return "ok";
        case COMBO_E_INVAL: return "invalid argument";
        case COMBO_E_NOMEM: return "out of memory";
        case COMBO_E_HIP: return "HIP runtime error";
        case COMBO_E_SIZE: return "unsupported grid size";
        case COMBO_E_NOCONV: return "no convergence";
        case COMBO_E_INADMISSIBLE: return "inadmissible deformation (det F <= 0)";
        case COMBO_E_NUMERIC: return "numerical failure";
        case COMBO_E_STATE: return "call out of order";
        default: return "unknown status";
    }
}

void combo_default_options(combo_options* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->precision = COMBO_FP64;
    o->tol_newton = 1e-8;
    o->tol_cg = 1e-10;
    o->max_newton = 30;
    o->max_cg = 5000;
    o->max_laminate = 50;
    o->n_increments = 1;
    o->mu0 = 0.0;
    o->kappa0 = 0.0;
    o->warm_start_laminate = 1;
    o->want_tangent = 0;
    o->max_step_halvings = 10;
    o->max_cutbacks = 5;
    o->graph_chunk = 0;
    o->autotune = 0;
    o->line_search = 1;
    o->law = COMBO_LAW_NEO_HOOKE;
    o->batch_streams = 0;
}

int combo_check_size(int n) { return size_ok(n) ? COMBO_OK : COMBO_E_SIZE; }

}  // extern "C"

namespace {
// The problem with one voxel's values, or an empty string.
std::string voxel_problem(long long v, int ph, double cv, double a, double b, double d) {
    if (ph > 2) return "phase id " + std::to_string(ph) + " at voxel " + std::to_string(v) + " (must be 0, 1, 2)";
    if (ph != 2) return std::string();
    if (!(cv > 0.0 && cv < 1.0)) return "composite voxel " + std::to_string(v) + " has c outside (0, 1)";
    if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(d))
        return "composite voxel " + std::to_string(v) + " has a non-finite normal";
    const double nn = std::sqrt(a * a + b * b + d * d);
    if (std::fabs(nn - 1.0) > 1e-6) return "composite voxel " + std::to_string(v) + " normal is not unit length";
    return std::string();
}
}  // namespace

extern "C" {

int combo_validate_microstructure(int n1, int n2, int n3, const uint8_t* phase, const double* c, const double* N,
                                  char* msg, int msg_len) {
    auto say = [&](const std::string& s) {
        if (msg && msg_len > 0) {
            strncpy(msg, s.c_str(), (size_t)msg_len - 1);
            msg[msg_len - 1] = 0;
        }
        return COMBO_E_INVAL;
    };
    if (n1 < 1 || n2 < 1 || n3 < 1) return say("grid dimensions must be positive");
    if (!phase || !c || !N) return say("null microstructure pointer");
    const long long n = (long long)n1 * n2 * n3;
    for (long long v = 0; v < n; ++v) {
        const int ph = phase[v];
        if (ph < 2) continue;
        const std::string e = ph == 2 ? voxel_problem(v, ph, c[v], N[v], N[n + v], N[2 * n + v])
                                      : voxel_problem(v, ph, 0.0, 0.0, 0.0, 0.0);
        if (!e.empty()) return say(e);
    }
    if (msg && msg_len > 0) msg[0] = 0;
    return COMBO_OK;
}

int combo_create(combo_ctx** out, int device, void* stream) {
    if (!out) return COMBO_E_INVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return COMBO_E_HIP;
    if (device < 0 || device >= count) return COMBO_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return COMBO_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return COMBO_E_HIP;
    if (std::string(prop.gcnArchName).find("gfx950") == std::string::npos) return COMBO_E_HIP;
    if (static_scratch_setup(device) != hipSuccess) return COMBO_E_HIP;
    combo_ctx* ctx = new combo_ctx();
    ctx->device = device;
    ctx->lds_limit = prop.sharedMemPerBlock;
    if (stream) {
        ctx->stream = static_cast<hipStream_t>(stream);
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return COMBO_E_HIP;
        }
        ctx->own_stream = true;
    }
    combo_default_options(&ctx->opt);
    *out = ctx;
    return COMBO_OK;
}

int combo_destroy(combo_ctx* ctx) {
    if (!ctx) return COMBO_E_INVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& g : ctx->graph) g.reset();
    prof_harvest(ctx);
    for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
    if (ctx->hs) (void)hipHostFree(ctx->hs);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return COMBO_OK;
}

const char* combo_last_error(const combo_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int combo_set_grid(combo_ctx* ctx, int n1, int n2, int n3, double l1, double l2, double l3) {
    if (!ctx) return COMBO_E_INVAL;
    if (!size_ok(n1) || !size_ok(n2) || !size_ok(n3))
        return set_err(ctx, COMBO_E_SIZE, "each grid axis must be 1 or 2^a 3^b <= 512");
    if (!(l1 > 0 && l2 > 0 && l3 > 0) || !std::isfinite(l1) || !std::isfinite(l2) || !std::isfinite(l3))
        return set_err(ctx, COMBO_E_INVAL, "box lengths must be positive and finite");
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    ctx->g.n1 = n1;
    ctx->g.n2 = n2;
    ctx->g.n3 = n3;
    ctx->g.xv = ctx->g.yv = ctx->g.zv = 0;
    ctx->g.disc = COMBO_DISC_MS;
    ctx->g.ftab = nullptr;
    ctx->g.nh = (n1 % 2 == 0) ? n1 / 2 : (n1 + 1) / 2;
    ctx->g.nkx = ctx->g.nh;
    ctx->g.n = (long long)n1 * n2 * n3;
    ctx->g.nspec = (long long)ctx->g.nh * n2 * n3;
    const double twopi = 6.283185307179586476925286766559;
    ctx->g.xs1 = twopi / l1;
    ctx->g.xs2 = twopi / l2;
    ctx->g.xs3 = twopi / l3;
    int xm = 0, xw = 0;
    xpass_wave_shape(n1, xm, xw);
    ctx->g.xm = xm;
    ctx->g.xwbits = -1;
    if (xw > 0 && xpass_lds_variants(n1) == 0) {
        int b = 0;
        while ((1 << b) < xw) ++b;
        ctx->g.xwbits = b;
    }
    ctx->l[0] = l1;
    ctx->l[1] = l2;
    ctx->l[2] = l3;
    const int ns[3] = {n1, n2, n3};
    for (int d = 0; d < 3; ++d) {
        ctx->plan[d] = make_plan(ns[d]);
        const int L = ns[d];
        std::vector<double2> w64(L);
        std::vector<float2> w32(L);
        for (int m = 0; m < L; ++m) {
            const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)L;
            w64[m].x = (double)cosl(ang);
            w64[m].y = (double)sinl(ang);
            w32[m].x = (float)w64[m].x;
            w32[m].y = (float)w64[m].y;
        }
        HIP_OR_FAIL(ctx->tw64[d].ensure(sizeof(double2) * L));
        HIP_OR_FAIL(ctx->tw32[d].ensure(sizeof(float2) * L));
        HIP_OR_FAIL(hipMemcpy(ctx->tw64[d].p, w64.data(), sizeof(double2) * L, hipMemcpyHostToDevice));
        HIP_OR_FAIL(hipMemcpy(ctx->tw32[d].p, w32.data(), sizeof(float2) * L, hipMemcpyHostToDevice));
    }
    for (auto& gr : ctx->graph) gr.reset();
    ctx->has_grid = true;
    ctx->has_ms = false;
    return COMBO_OK;
}

int combo_set_discretization(combo_ctx* ctx, int disc) {
    if (!ctx) return COMBO_E_INVAL;
    if (!ctx->has_grid) return set_err(ctx, COMBO_E_STATE, "combo_set_grid has not been called");
    if (disc != COMBO_DISC_MS && disc != COMBO_DISC_WILLOT && disc != COMBO_DISC_STAGGERED)
        return set_err(ctx, COMBO_E_INVAL, "disc must be COMBO_DISC_MS, COMBO_DISC_WILLOT or COMBO_DISC_STAGGERED");
    const int n1 = ctx->g.n1, n2 = ctx->g.n2, n3 = ctx->g.n3;
    int st = combo_set_grid(ctx, n1, n2, n3, ctx->l[0], ctx->l[1], ctx->l[2]);
    if (st != COMBO_OK || disc == COMBO_DISC_MS) return st;
    Grid& g = ctx->g;
    g.disc = disc;
    g.nkx = n1 / 2 + 1;   // x frequencies 0 .. floor(n1/2): an even n1 keeps its Nyquist bin
    // Rows of nkx = 16 m + 1 values would start off the 128-byte lines that the y pass
    // reads in tiles of 16 columns; pad them to a multiple of 16 where that adds at
    // most a quarter of zero modes (e.g. 256: 129 -> 144, 112: 57 -> 64; 64: none).
    const int padded = (g.nkx + 15) / 16 * 16;
    g.nh = (4 * (padded - g.nkx) <= g.nkx) ? padded : g.nkx;
    g.nspec = (long long)g.nh * n2 * n3;
    g.xwbits = -1;       // natural state order: the rotated scheme has no wavefront x pass
    // Rotated scheme: D = (2/h) sin(theta/2), A = cos(theta/2); x: theta = 2 pi k / n1 (k >= 0),
    // y and z: theta = 2 pi freq / n with freq in [-n/2, n/2); A = 0 exactly at |theta| = pi.
    // Staggered grid: D = Re f, A = Im f of f = (e^{i theta} - 1) / h = (cos theta - 1 + i sin theta) / h,
    // written as -2 sin^2(theta/2) / h + i sin(theta) / h (sin theta = 0 exactly at |theta| = pi)
    const int ns[3] = {n1, n2, n3};
    const int len[3] = {g.nh, n2, n3};
    std::vector<double> tab;
    for (int d = 0; d < 3; ++d) {
        const long double h = (long double)ctx->l[d] / ns[d];
        std::vector<double> D(len[d]), A(len[d]);
        for (int j = 0; j < len[d]; ++j) {
            const int f = (d == 0) ? j : freq_of(j, ns[d]);
            const long double half = 3.14159265358979323846264338327950288L * (long double)f / (long double)ns[d];
            const bool nyq = (2 * f == ns[d] || 2 * f == -ns[d]);
            if (disc == COMBO_DISC_STAGGERED) {
                const long double sh = sinl(half);
                D[j] = (double)(-2.0L * sh * sh / h);
                A[j] = nyq ? 0.0 : (double)(sinl(2.0L * half) / h);
            } else {
                D[j] = (double)(2.0L / h * sinl(half));
                A[j] = nyq ? 0.0 : (double)cosl(half);
            }
            if (d == 0 && j >= g.nkx) D[j] = A[j] = 0.0;   // row padding: zero modes
        }
        tab.insert(tab.end(), D.begin(), D.end());
        tab.insert(tab.end(), A.begin(), A.end());
    }
    HIP_OR_FAIL(ctx->ftab.ensure(sizeof(double) * tab.size()));
    HIP_OR_FAIL(hipMemcpy(ctx->ftab.p, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice));
    g.ftab = static_cast<const double*>(ctx->ftab.p);
    return COMBO_OK;
}

int combo_set_materials(combo_ctx* ctx, const combo_material mats[2]) {
    if (!ctx || !mats) return COMBO_E_INVAL;
    for (int p = 0; p < 2; ++p)
        if (!(mats[p].mu > 0.0) || !(mats[p].lambda >= 0.0) || !std::isfinite(mats[p].mu) ||
            !std::isfinite(mats[p].lambda))
            return set_err(ctx, COMBO_E_INVAL, "materials need mu > 0 and lambda >= 0");
    ctx->mats[0] = mats[0];
    ctx->mats[1] = mats[1];
    ctx->has_mats = true;
    for (auto& gr : ctx->graph) gr.reset();
    return COMBO_OK;
}

int combo_set_options(combo_ctx* ctx, const combo_options* o) {
    if (!ctx || !o) return COMBO_E_INVAL;
    const char* bad = options_error(o);
    if (bad) return set_err(ctx, COMBO_E_INVAL, bad);
    ctx->opt = *o;
    for (auto& gr : ctx->graph) gr.reset();
    return COMBO_OK;
}

int combo_get_grid(const combo_ctx* ctx, int* n1, int* n2, int* n3, double* l1, double* l2, double* l3) {
    if (!ctx || !n1 || !n2 || !n3 || !l1 || !l2 || !l3) return COMBO_E_INVAL;
    if (!ctx->has_grid) return COMBO_E_STATE;
    *n1 = ctx->g.n1;
    *n2 = ctx->g.n2;
    *n3 = ctx->g.n3;
    *l1 = ctx->l[0];
    *l2 = ctx->l[1];
    *l3 = ctx->l[2];
    return COMBO_OK;
}

}  // extern "C"

namespace {

// checks shared by the image -> boxels entry points
int boxel_check(combo_ctx* ctx, const void* chi, const void* phase, const void* c, const void* N, int s1, int s2,
                int s3, int method) {
    if (!ctx->has_grid) return set_err(ctx, COMBO_E_STATE, "combo_set_grid has not been called");
    if (!chi || !phase || !c || !N) return set_err(ctx, COMBO_E_INVAL, "null image or output pointer");
    if (s1 < 1 || s2 < 1 || s3 < 1 || s1 > 4096 || s2 > 4096 || s3 > 4096)
        return set_err(ctx, COMBO_E_INVAL, "fine voxels per boxel must be in [1, 4096]");
    if (method != COMBO_NORMALS_LAPLACE && method != COMBO_NORMALS_BARYCENTRE)
        return set_err(ctx, COMBO_E_INVAL, "method must be COMBO_NORMALS_LAPLACE or COMBO_NORMALS_BARYCENTRE");
    const Grid& g = ctx->g;
    const long long N1 = (long long)g.n1 * s1, N2 = (long long)g.n2 * s2, N3 = (long long)g.n3 * s3;
    if ((double)N1 * (double)N2 * (double)N3 > 1.0e12 || (long long)s1 * s2 * s3 > (1LL << 30))
        return set_err(ctx, COMBO_E_INVAL, "image too large");
    return COMBO_OK;
}

// argument block of the boxel kernels for device image and outputs (packed and counter left null)
BoxelArgs boxel_args(const combo_ctx* ctx, const uint8_t* chi_d, int s1, int s2, int s3, int method, uint8_t* phase_d,
                     double* c_d, double* N_d) {
    const Grid& g = ctx->g;
    BoxelArgs a{};
    a.chi = chi_d;
    a.N1 = (long long)g.n1 * s1;
    a.N2 = (long long)g.n2 * s2;
    a.N3 = (long long)g.n3 * s3;
    a.n1 = g.n1;
    a.n2 = g.n2;
    a.n3 = g.n3;
    a.s1 = s1;
    a.s2 = s2;
    a.s3 = s3;
    a.h[0] = ctx->l[0] / (double)a.N1;
    a.h[1] = ctx->l[1] / (double)a.N2;
    a.h[2] = ctx->l[2] / (double)a.N3;
    a.r[0] = a.h[1] * a.h[2] / a.h[0];
    a.r[1] = a.h[0] * a.h[2] / a.h[1];
    a.r[2] = a.h[0] * a.h[1] / a.h[2];
    a.method = method;
    a.vec4 = (s1 % 4 == 0) && (a.N1 % 4 == 0) && (reinterpret_cast<uintptr_t>(chi_d) % 4 == 0);
    a.vec16 = (s1 == 4) && (g.n1 % 4 == 0) && (a.N1 % 16 == 0) && (reinterpret_cast<uintptr_t>(chi_d) % 16 == 0) &&
              (reinterpret_cast<uintptr_t>(phase_d) % 4 == 0) && (reinterpret_cast<uintptr_t>(c_d) % 16 == 0);
    a.phase = phase_d;
    a.c = c_d;
    a.N = N_d;
    a.packed = nullptr;
    a.counter = nullptr;
    return a;
}

// pass 1 (counts, phases) needs packed fine words: the four-boxel path with s2 s3 <= 16
bool boxel_wants_packed(const BoxelArgs& a) { return a.vec16 && (long long)a.s2 * a.s3 <= 16; }

}  // namespace

extern "C" {

int combo_image_to_boxels(combo_ctx* ctx, const uint8_t* chi, int s1, int s2, int s3, int method, uint8_t* phase,
                          double* c, double* N, int mem_kind) {
    if (!ctx) return COMBO_E_INVAL;
    if (mem_kind != COMBO_MEM_HOST && mem_kind != COMBO_MEM_DEVICE) return set_err(ctx, COMBO_E_INVAL, "bad mem_kind");
    const int chk = boxel_check(ctx, chi, phase, c, N, s1, s2, s3, method);
    if (chk != COMBO_OK) return chk;
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    const Grid& g = ctx->g;
    const long long nb = g.n;
    const size_t img_bytes = (size_t)((long long)g.n1 * s1 * (long long)g.n2 * s2 * (long long)g.n3 * s3);
    DevBuf dchi, dphase, dc, dN;
    DevBuf& bx = ctx->bx_scratch;   // kept by the context: repeated calls allocate nothing new
    const uint8_t* chi_d = chi;
    uint8_t* phase_d = phase;
    double* c_d = c;
    double* N_d = N;
    if (mem_kind == COMBO_MEM_HOST) {
        HIP_OR_FAIL(dchi.ensure(img_bytes + 4));
        HIP_OR_FAIL(hipMemcpyAsync(dchi.p, chi, img_bytes, hipMemcpyHostToDevice, ctx->stream));
        HIP_OR_FAIL(dphase.ensure((size_t)nb));
        HIP_OR_FAIL(dc.ensure(sizeof(double) * nb));
        HIP_OR_FAIL(dN.ensure(sizeof(double) * 3 * nb));
        chi_d = static_cast<const uint8_t*>(dchi.p);
        phase_d = static_cast<uint8_t*>(dphase.p);
        c_d = static_cast<double*>(dc.p);
        N_d = static_cast<double*>(dN.p);
    }
    HIP_OR_FAIL(bx.ensure(sizeof(int) * (2 + (size_t)boxel_blocks(nb) + (size_t)nb)));
    BoxelArgs a = boxel_args(ctx, chi_d, s1, s2, s3, method, phase_d, c_d, N_d);
    if (boxel_wants_packed(a)) {
        HIP_OR_FAIL(ctx->bx_packed.ensure(sizeof(uint64_t) * (size_t)nb));
        a.packed = static_cast<uint64_t*>(ctx->bx_packed.p);
    }
    a.counter = static_cast<int*>(bx.p);
    HIP_OR_FAIL(hipMemsetAsync(a.counter, 0, 2 * sizeof(int), ctx->stream));
    {
        ProfScope ps(ctx, COMBO_K_BOXEL_COUNT);
        HIP_OR_FAIL(launch_boxel_count(a, ctx->stream));
    }
    int* blockcnt = a.counter + 2;
    int* list = blockcnt + boxel_blocks(nb);
    int hcnt[2] = {0, 0};
    DevBuf& mom = ctx->bx_mom;
    {
        ProfScope ps(ctx, COMBO_K_BOXEL_NORMALS);
        HIP_OR_FAIL(launch_boxel_list(a, blockcnt, list, ctx->stream));
        HIP_OR_FAIL(hipMemcpyAsync(hcnt, a.counter, sizeof(hcnt), hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
        HIP_OR_FAIL(mom.ensure(sizeof(double) * 13 * (size_t)std::max(hcnt[0], 1)));
        HIP_OR_FAIL(launch_boxel_normals(a, list, static_cast<double*>(mom.p), hcnt[0], ctx->stream));
    }
    if (mem_kind == COMBO_MEM_HOST) {
        HIP_OR_FAIL(hipMemcpyAsync(phase, phase_d, (size_t)nb, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(hipMemcpyAsync(c, c_d, sizeof(double) * nb, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OR_FAIL(hipMemcpyAsync(N, N_d, sizeof(double) * 3 * nb, hipMemcpyDeviceToHost, ctx->stream));
    }
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx);
    if (hcnt[1]) return set_err(ctx, COMBO_E_INVAL, "image values must be 0 or 1");
    return COMBO_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------
// image -> boxels without allocation: the counters, block offsets, composite
// list, packed fine words and moments live in one static device array per GPU
// ------------------------------------------------------------------------------
namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// byte offsets of the pieces of the static scratch for nb boxels
struct StaticBoxelLayout {
    size_t blockcnt, list, packed, mom;
};

StaticBoxelLayout static_boxel_layout(long long nb, bool packed) {
    StaticBoxelLayout L{};
    L.blockcnt = 256;   // the two counters sit at offset 0
    L.list = align256(L.blockcnt + sizeof(int) * (size_t)boxel_blocks(nb));
    L.packed = align256(L.list + sizeof(int) * (size_t)nb);
    L.mom = align256(L.packed + (packed ? sizeof(uint64_t) * (size_t)nb : 0));
    return L;
}

}  // namespace

extern "C" {

int combo_image_to_boxels_static(combo_ctx* ctx, const uint8_t* chi, int s1, int s2, int s3, int method,
                                 uint8_t* phase, double* c, double* N) {
    if (!ctx) return COMBO_E_INVAL;
    const int chk = boxel_check(ctx, chi, phase, c, N, s1, s2, s3, method);
    if (chk != COMBO_OK) return chk;
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    char* base = static_cast<char*>(static_scratch_ptr(ctx->device));
    if (!base) return set_err(ctx, COMBO_E_STATE, "the static scratch of this device was not set up");
    const long long nb = ctx->g.n;
    BoxelArgs a = boxel_args(ctx, chi, s1, s2, s3, method, phase, c, N);
    const bool packed = boxel_wants_packed(a);
    const StaticBoxelLayout L = static_boxel_layout(nb, packed);
    if (L.mom > kStaticScratchBytes)
        return set_err(ctx, COMBO_E_SIZE,
                       "grid of " + std::to_string(nb) + " boxels needs " + std::to_string(L.mom) +
                           " bytes of scratch before the moments; the static scratch holds " +
                           std::to_string(kStaticScratchBytes));
    a.counter = reinterpret_cast<int*>(base);
    a.packed = packed ? reinterpret_cast<uint64_t*>(base + L.packed) : nullptr;
    int* blockcnt = reinterpret_cast<int*>(base + L.blockcnt);
    int* list = reinterpret_cast<int*>(base + L.list);
    double* mom = reinterpret_cast<double*>(base + L.mom);
    HIP_OR_FAIL(launch_boxel_zero(a.counter, 2, ctx->stream));
    HIP_OR_FAIL(launch_boxel_count(a, ctx->stream));
    HIP_OR_FAIL(launch_boxel_list(a, blockcnt, list, ctx->stream));
    int hcnt[2] = {0, 0};
    HIP_OR_FAIL(hipMemcpyAsync(hcnt, a.counter, sizeof(hcnt), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    if (hcnt[1]) return set_err(ctx, COMBO_E_INVAL, "image values must be 0 or 1");
    const size_t need = L.mom + sizeof(double) * 13 * (size_t)hcnt[0];
    if (need > kStaticScratchBytes)
        return set_err(ctx, COMBO_E_SIZE,
                       std::to_string(hcnt[0]) + " composite boxels need " + std::to_string(need) +
                           " bytes of scratch with their moments; the static scratch holds " +
                           std::to_string(kStaticScratchBytes) + " (phase and c are written, N is not)");
    HIP_OR_FAIL(launch_boxel_normals(a, list, mom, hcnt[0], ctx->stream));
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    return COMBO_OK;
}

int combo_set_microstructure_from_image(combo_ctx* ctx, const uint8_t* chi, int s1, int s2, int s3, int method,
                                        int mem_kind) {
    if (!ctx) return COMBO_E_INVAL;
    if (!ctx->has_grid) return set_err(ctx, COMBO_E_STATE, "combo_set_grid has not been called");
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    const long long nb = ctx->g.n;
    DevBuf dphase, dc, dN, dchi;
    HIP_OR_FAIL(dphase.ensure((size_t)nb));
    HIP_OR_FAIL(dc.ensure(sizeof(double) * nb));
    HIP_OR_FAIL(dN.ensure(sizeof(double) * 3 * nb));
    const uint8_t* chi_d = chi;
    if (mem_kind == COMBO_MEM_HOST && chi) {
        if (s1 < 1 || s2 < 1 || s3 < 1 || s1 > 4096 || s2 > 4096 || s3 > 4096)
            return set_err(ctx, COMBO_E_INVAL, "fine voxels per boxel must be in [1, 4096]");
        const double img = (double)ctx->g.n1 * s1 * (double)ctx->g.n2 * s2 * (double)ctx->g.n3 * s3;
        if (img > 1.0e12) return set_err(ctx, COMBO_E_INVAL, "image too large");
        HIP_OR_FAIL(dchi.ensure((size_t)img + 4));
        HIP_OR_FAIL(hipMemcpy(dchi.p, chi, (size_t)img, hipMemcpyHostToDevice));
        chi_d = static_cast<const uint8_t*>(dchi.p);
    } else if (mem_kind != COMBO_MEM_DEVICE && mem_kind != COMBO_MEM_HOST) {
        return set_err(ctx, COMBO_E_INVAL, "bad mem_kind");
    }
    int st = combo_image_to_boxels(ctx, chi_d, s1, s2, s3, method, static_cast<uint8_t*>(dphase.p),
                                   static_cast<double*>(dc.p), static_cast<double*>(dN.p), COMBO_MEM_DEVICE);
    if (st != COMBO_OK) return st;
    return combo_set_microstructure(ctx, static_cast<const uint8_t*>(dphase.p), static_cast<const double*>(dc.p),
                                    static_cast<const double*>(dN.p), COMBO_MEM_DEVICE);
}

int combo_set_microstructure(combo_ctx* ctx, const uint8_t* phase, const double* c, const double* N, int mem_kind) {
    if (!ctx) return COMBO_E_INVAL;
    if (!ctx->has_grid) return set_err(ctx, COMBO_E_STATE, "combo_set_grid has not been called");
    if (!phase || !c || !N) return set_err(ctx, COMBO_E_INVAL, "null microstructure pointer");
    if (mem_kind != COMBO_MEM_HOST && mem_kind != COMBO_MEM_DEVICE) return set_err(ctx, COMBO_E_INVAL, "bad mem_kind");
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const long long n = ctx->g.n;
    // host fields are uploaded once; everything below runs on the device
    DevBuf up;
    const uint8_t* P = phase;
    const double* C = c;
    const double* NN = N;
    if (mem_kind == COMBO_MEM_HOST) {
        HIP_OR_FAIL(up.ensure(sizeof(double) * 4 * n + (size_t)n));   // c, N, then the phase bytes
        double* cd = static_cast<double*>(up.p);
        HIP_OR_FAIL(hipMemcpyAsync(cd, c, sizeof(double) * n, hipMemcpyHostToDevice, s));
        HIP_OR_FAIL(hipMemcpyAsync(cd + n, N, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
        HIP_OR_FAIL(hipMemcpyAsync(cd + 4 * n, phase, n, hipMemcpyHostToDevice, s));
        C = cd;
        NN = cd + n;
        P = reinterpret_cast<const uint8_t*>(cd + 4 * n);
    }
    const int nblk = setup_blocks(n);
    DevBuf wk;   // cnt2[nblk] cnt01[2 nblk] flags[2] | sumc[nblk]
    const size_t ints = (size_t)3 * nblk + 2, off_d = (ints * sizeof(int) + 255) / 256 * 256;
    HIP_OR_FAIL(wk.ensure(off_d + sizeof(double) * nblk));
    SetupArgs a{};
    a.phase = P;
    a.c = C;
    a.N = NN;
    a.n = n;
    a.cnt2 = static_cast<int*>(wk.p);
    a.cnt01 = a.cnt2 + nblk;
    a.flags = a.cnt2 + 3 * nblk;
    a.sumc = reinterpret_cast<double*>(static_cast<char*>(wk.p) + off_d);
    HIP_OR_FAIL(launch_setup_reset(a.flags, s));
    HIP_OR_FAIL(launch_setup_count(a, s));
    int fl[2];
    std::vector<int> c01((size_t)2 * nblk);
    std::vector<double> sc(nblk);
    HIP_OR_FAIL(hipMemcpyAsync(fl, a.flags, sizeof(fl), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipMemcpyAsync(c01.data(), a.cnt01, sizeof(int) * 2 * nblk, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipMemcpyAsync(sc.data(), a.sumc, sizeof(double) * nblk, hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    if (fl[0] != INT_MAX) {   // the first invalid voxel: its values make the message
        const long long v = fl[0];
        uint8_t ph = 0;
        double vals[4] = {0, 0, 0, 0};
        HIP_OR_FAIL(hipMemcpy(&ph, P + v, 1, hipMemcpyDeviceToHost));
        if (ph == 2) {
            HIP_OR_FAIL(hipMemcpy(&vals[0], C + v, sizeof(double), hipMemcpyDeviceToHost));
            for (int d = 0; d < 3; ++d)
                HIP_OR_FAIL(hipMemcpy(&vals[1 + d], NN + d * n + v, sizeof(double), hipMemcpyDeviceToHost));
        }
        std::string e = voxel_problem(v, ph, vals[0], vals[1], vals[2], vals[3]);
        if (e.empty()) e = "voxel " + std::to_string(v) + " failed validation";
        return set_err(ctx, COMBO_E_INVAL, e);
    }
    double nm = 0, ni = 0, sumc = 0;
    for (int b = 0; b < nblk; ++b) {
        nm += c01[2 * (size_t)b];
        ni += c01[2 * (size_t)b + 1];
        sumc += sc[b];
    }
    const int nc = fl[1];
    HIP_OR_FAIL(ctx->slot_s.ensure(sizeof(int) * n));
    HIP_OR_FAIL(ctx->slot.ensure(sizeof(int) * n));
    HIP_OR_FAIL(ctx->comp_vox.ensure(sizeof(int) * std::max(nc, 1)));
    HIP_OR_FAIL(ctx->comp_c.ensure(sizeof(double) * std::max(nc, 1)));
    HIP_OR_FAIL(ctx->comp_N.ensure(sizeof(double) * 3 * std::max(nc, 1)));
    a.n1 = ctx->g.n1;
    a.xm = ctx->g.xm;
    a.xwbits = ctx->g.xwbits;
    a.nc = nc;
    a.slot = ctx->slot.as<int>();
    a.slot_s = ctx->slot_s.as<int>();
    a.comp_vox = ctx->comp_vox.as<int>();
    a.comp_c = ctx->comp_c.as<double>();
    a.comp_N = ctx->comp_N.as<double>();
    HIP_OR_FAIL(launch_setup_compact(a, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));   // the uploads and work buffers are freed on return
    ctx->nc = nc;
    ctx->n_mat = nm;
    ctx->n_incl = ni;
    ctx->sum_c = sumc;
    int st = ensure_work(ctx);
    if (st) return st;
    for (auto& gr : ctx->graph) gr.reset();
    ctx->state_prec = -1;
    ctx->has_ms = true;
    return COMBO_OK;
}

int combo_solve(combo_ctx* ctx, const double Fbar[9], const double* F_init, double* F_out, double* P_out,
                double Pbar[9], double Abar[81], double Pbar_phase[18], combo_stats* stats, int mem_kind) {
    int st = require_ready(ctx);
    if (st) return st;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (!Fbar) return set_err(ctx, COMBO_E_INVAL, "Fbar is null");
    if (mem_kind != COMBO_MEM_HOST && mem_kind != COMBO_MEM_DEVICE) return set_err(ctx, COMBO_E_INVAL, "bad mem_kind");
    if (!finite9(Fbar)) {
        if (stats) stats->status = COMBO_E_NUMERIC;
        return set_err(ctx, COMBO_E_NUMERIC, "Fbar is not finite");
    }
    if (ctx->opt.law != COMBO_LAW_LINEAR && !(det9(Fbar) > 0.0)) {
        if (stats) stats->status = COMBO_E_INADMISSIBLE;
        return set_err(ctx, COMBO_E_INADMISSIBLE, "det Fbar <= 0");
    }
    if (staggered(ctx) && ctx->opt.law != COMBO_LAW_NEO_HOOKE)
        return set_err(ctx, COMBO_E_INVAL, "the staggered grid takes the finite-strain law");
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    const long long n = ctx->g.n;
    const size_t f9 = sizeof(double) * 9 * (size_t)n;
    double Fbar0[9];
    if (F_init) {
        if (mem_kind == COMBO_MEM_HOST) {
            for (long long v = 0; v < 9 * n; ++v)
                if (!std::isfinite(F_init[v])) {
                    if (stats) stats->status = COMBO_E_NUMERIC;
                    return set_err(ctx, COMBO_E_NUMERIC, "F_init is not finite");
                }
            mean_field_host(F_init, n, Fbar0);
        }
        if (staggered(ctx)) {
            st = copy_in(ctx, ctx->stag_tmp.p, F_init, f9, mem_kind);
            if (st || (st = to_shifted(ctx, ctx->stag_tmp.as<double>(), ctx->F_cur.as<double>()))) return st;
        } else {
            st = copy_in(ctx, ctx->F_cur.p, F_init, f9, mem_kind);
            if (st) return st;
        }
        if (mem_kind == COMBO_MEM_DEVICE) {
            const int nb = 1024;
            hipLaunchKernelGGL(k_colsum9, dim3(nb), dim3(256), 0, ctx->stream, ctx->F_cur.as<double>(), n,
                               ctx->part1.as<double>());
            HIP_OR_FAIL(hipGetLastError());
            HIP_OR_FAIL(launch_reduce_columns(ctx->part1.as<double>(), nb, 9, ctx->sums.as<double>() + kSumsLen,
                                              ctx->stream));
            HIP_OR_FAIL(hipMemcpyAsync(Fbar0, ctx->sums.as<double>() + kSumsLen, sizeof(Fbar0), hipMemcpyDeviceToHost,
                                       ctx->stream));
            HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
            for (int c = 0; c < 9; ++c) Fbar0[c] /= (double)n;
            if (!finite9(Fbar0)) {
                if (stats) stats->status = COMBO_E_NUMERIC;
                return set_err(ctx, COMBO_E_NUMERIC, "F_init is not finite");
            }
        }
    } else {
        hipLaunchKernelGGL(k_fill_identity, dim3(1024), dim3(256), 0, ctx->stream, ctx->F_cur.as<double>(), n);
        HIP_OR_FAIL(hipGetLastError());
        for (int c = 0; c < 9; ++c) Fbar0[c] = (c % 4 == 0) ? 1.0 : 0.0;
    }
    if (ctx->opt.autotune) {
        st = autotune(ctx, ctx->opt.precision);
        if (st) return st;
    }
    hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(64), 0, ctx->stream, ctx->cgst.as<CGState>());
    SolveOut so;
    double Atmp[81];
    double* Aptr = (ctx->opt.want_tangent && Abar) ? Atmp : nullptr;
    if (ctx->opt.precision == COMBO_MIXED) st = solve_impl<float>(ctx, Fbar, Fbar0, so, Aptr);
    else st = solve_impl<double>(ctx, Fbar, Fbar0, so, Aptr);
    so.st.status = st;
    if (stats) *stats = so.st;
    if (st) return st;
    if (Pbar) memcpy(Pbar, so.Pbar, sizeof(so.Pbar));
    if (Pbar_phase) {
        memcpy(Pbar_phase, so.Pp, sizeof(so.Pp));
        memcpy(Pbar_phase + 9, so.Pm, sizeof(so.Pm));
    }
    if (Aptr) memcpy(Abar, Atmp, sizeof(Atmp));
    if (F_out) {
        const void* src = ctx->F_cur.p;
        if (staggered(ctx)) {
            if ((st = to_natural(ctx, ctx->F_cur.as<double>(), ctx->stag_tmp.as<double>()))) return st;
            src = ctx->stag_tmp.p;
        }
        st = copy_out(ctx, F_out, src, f9, mem_kind);
        if (st) return st;
    }
    if (P_out) {
        const void* src = ctx->P.p;
        if (staggered(ctx)) {
            // stream order: the copy of F_out above has read stag_tmp before it is rewritten
            if ((st = to_natural(ctx, ctx->P.as<double>(), ctx->stag_tmp.as<double>()))) return st;
            src = ctx->stag_tmp.p;
        }
        st = copy_out(ctx, P_out, src, f9, mem_kind);
        if (st) return st;
    }
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    return COMBO_OK;
}

int combo_eval_law(combo_ctx* ctx, const double* F, double* Pout, double* A, double* a, int* iters, int mem_kind) {
    int st = require_ready(ctx);
    if (st) return st;
    if (!F) return set_err(ctx, COMBO_E_INVAL, "F is null");
    if (mem_kind != COMBO_MEM_HOST && mem_kind != COMBO_MEM_DEVICE) return set_err(ctx, COMBO_E_INVAL, "bad mem_kind");
    if (staggered(ctx) && (A || a || iters))
        return set_err(ctx, COMBO_E_INVAL, "the staggered grid's law returns P only (A, a and iters must be NULL)");
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    const long long n = ctx->g.n;
    const size_t f9 = sizeof(double) * 9 * (size_t)n;
    if (staggered(ctx)) {
        st = copy_in(ctx, ctx->stag_tmp.p, F, f9, mem_kind);
        if (st || (st = to_shifted(ctx, ctx->stag_tmp.as<double>(), ctx->F_save.as<double>()))) return st;
    } else {
        st = copy_in(ctx, ctx->F_save.p, F, f9, mem_kind);
        if (st) return st;
    }
    DevBuf dA, da, dit;
    if (A) HIP_OR_FAIL(dA.ensure(sizeof(double) * 81 * (size_t)n));
    if (a) HIP_OR_FAIL(da.ensure(sizeof(double) * 3 * (size_t)n));
    if (iters) HIP_OR_FAIL(dit.ensure(sizeof(int) * (size_t)n));
    if (ctx->opt.precision == COMBO_MIXED)
        st = material<float>(ctx, ctx->F_save.as<double>(), nullptr, 0.0, nullptr, ctx->F_trial.as<double>(), true,
                             dA.as<double>(), da.as<double>(), dit.as<int>());
    else
        st = material<double>(ctx, ctx->F_save.as<double>(), nullptr, 0.0, nullptr, ctx->F_trial.as<double>(), true,
                              dA.as<double>(), da.as<double>(), dit.as<int>());
    if (st) return st;
    if (Pout && staggered(ctx)) {
        if ((st = to_natural(ctx, ctx->P.as<double>(), ctx->stag_tmp.as<double>()))) return st;
        if ((st = copy_out(ctx, Pout, ctx->stag_tmp.p, f9, mem_kind))) return st;
    } else if (Pout && (st = copy_out(ctx, Pout, ctx->P.p, f9, mem_kind))) {
        return st;
    }
    if (A && (st = copy_out(ctx, A, dA.p, sizeof(double) * 81 * (size_t)n, mem_kind))) return st;
    if (a && (st = copy_out(ctx, a, da.p, sizeof(double) * 3 * (size_t)n, mem_kind))) return st;
    if (iters && (st = copy_out(ctx, iters, dit.p, sizeof(int) * (size_t)n, mem_kind))) return st;
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    if (material_failures(ctx) > 0.0)
        return set_err(ctx, COMBO_E_INADMISSIBLE, "det F <= 0 or a laminate failed in some voxel");
    return COMBO_OK;
}

}  // extern "C"

namespace {
template <typename T>
int apply_green_impl(combo_ctx* ctx, int which, const double* tau_dev, double* out_dev) {
    double mu0 = 1.0, kappa0 = 0.0;
    if (which == COMBO_GREEN_GAMMA0) reference_medium(ctx, mu0, kappa0);
    int st = forward_xy_real<T>(ctx, tau_dev);
    if (st) return st;
    ZArgs<T, T> za = zargs<T, T>(ctx, mu0, kappa0);
    za.in = ctx->specB.as<cpx<T>>();
    HIP_OR_FAIL(launch_z<T, T>(Z_PROJ, za, ctx->stream));
    ZArgs<T, T> zi = zargs<T, T>(ctx, mu0, kappa0);
    zi.out = ctx->specA.as<cpx<T>>();
    HIP_OR_FAIL(launch_z<T, T>(Z_INV_PLAIN, zi, ctx->stream));
    HIP_OR_FAIL(launch_y<T>(+1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, false), ctx->stream));
    XArgs<T> xa = xargs<T>(ctx);
    xa.in = ctx->specB.as<cpx<T>>();
    xa.real_out = out_dev;
    HIP_OR_FAIL(launch_x<T>(X_INV_REAL, xa, ctx->stream));
    return COMBO_OK;
}

template <typename T>
int apply_operator_impl(combo_ctx* ctx, const double* p_dev, double* q_dev) {
    double mu0, kappa0;
    reference_medium(ctx, mu0, kappa0);
    // displacement coefficients of p: u = (p_hat xi) / |xi|^2 (exact for compatible p)
    int st = forward_xy_real<T>(ctx, p_dev);
    if (st) return st;
    ZArgs<T, T> za = zargs<T, T>(ctx, 1.0, 0.0);
    za.in = ctx->specB.as<cpx<T>>();
    HIP_OR_FAIL(launch_z<T, T>(Z_PROJ, za, ctx->stream));
    // one application of the CG operator: x -> q
    hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(64), 0, ctx->stream, ctx->cgst.as<CGState>());
    HIP_OR_FAIL(hipGetLastError());
    ZArgs<T, T> zi = zargs<T, T>(ctx, mu0, kappa0);
    zi.out = ctx->specA.as<cpx<T>>();
    HIP_OR_FAIL(launch_z<T, T>(Z_INV_PLAIN, zi, ctx->stream));
    HIP_OR_FAIL(launch_y<T>(+1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, true), ctx->stream));
    if (staggered(ctx)) {
        st = stag_tangent_x<T>(ctx, ctx->stream);
        if (st) return st;
    } else {
        XArgs<T> xa = xargs<T>(ctx);
        xa.in = ctx->specB.as<cpx<T>>();
        xa.out = ctx->specA.as<cpx<T>>();
        HIP_OR_FAIL(launch_x<T>(X_CG, xa, ctx->stream));
    }
    HIP_OR_FAIL(launch_y<T>(-1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, true), ctx->stream));
    ZArgs<T, T> zc = zargs<T, T>(ctx, mu0, kappa0);
    zc.in = ctx->specB.as<cpx<T>>();
    zc.p = zc.x;
    HIP_OR_FAIL(launch_z<T, T>(Z_CG, zc, ctx->stream));
    // q -> field
    ZArgs<T, T> zq = zargs<T, T>(ctx, mu0, kappa0);
    zq.x = zq.q;
    zq.out = ctx->specA.as<cpx<T>>();
    HIP_OR_FAIL(launch_z<T, T>(Z_INV_PLAIN, zq, ctx->stream));
    HIP_OR_FAIL(launch_y<T>(+1, yargs<T>(ctx, ctx->specA.p, ctx->specB.p, false), ctx->stream));
    XArgs<T> xo = xargs<T>(ctx);
    xo.in = ctx->specB.as<cpx<T>>();
    xo.real_out = q_dev;
    HIP_OR_FAIL(launch_x<T>(X_INV_REAL, xo, ctx->stream));
    return COMBO_OK;
}
}  // namespace

extern "C" {

int combo_apply_green(combo_ctx* ctx, int which, int precision, const double* tau, double* out, int mem_kind) {
    if (!ctx) return COMBO_E_INVAL;
    if (!ctx->has_grid) return set_err(ctx, COMBO_E_STATE, "combo_set_grid has not been called");
    if (which != COMBO_GREEN_GAMMA0 && which != COMBO_GREEN_G) return set_err(ctx, COMBO_E_INVAL, "bad operator id");
    if (which == COMBO_GREEN_GAMMA0 && !ctx->has_mats && (ctx->opt.mu0 <= 0 || ctx->opt.kappa0 <= 0))
        return set_err(ctx, COMBO_E_STATE, "Gamma0 needs materials or an explicit reference medium");
    if (precision != COMBO_FP64 && precision != COMBO_MIXED) return set_err(ctx, COMBO_E_INVAL, "bad precision");
    if (!tau || !out) return set_err(ctx, COMBO_E_INVAL, "null field");
    if (mem_kind != COMBO_MEM_HOST && mem_kind != COMBO_MEM_DEVICE) return set_err(ctx, COMBO_E_INVAL, "bad mem_kind");
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    if (!ctx->has_ms) {
        ctx->nc = 0;
        int st = ensure_work(ctx);
        if (st) return st;
    }
    const size_t f9 = sizeof(double) * 9 * (size_t)ctx->g.n;
    int st = copy_in(ctx, ctx->F_save.p, tau, f9, mem_kind);
    if (st) return st;
    const double* in_dev = ctx->F_save.as<double>();
    if (staggered(ctx)) {
        if ((st = to_shifted(ctx, ctx->F_save.as<double>(), ctx->stag_tmp.as<double>()))) return st;
        in_dev = ctx->stag_tmp.as<double>();
    }
    if (precision == COMBO_MIXED) st = apply_green_impl<float>(ctx, which, in_dev, ctx->dF.as<double>());
    else st = apply_green_impl<double>(ctx, which, in_dev, ctx->dF.as<double>());
    if (st) return st;
    const void* res = ctx->dF.p;
    if (staggered(ctx)) {
        if ((st = to_natural(ctx, ctx->dF.as<double>(), ctx->stag_tmp.as<double>()))) return st;
        res = ctx->stag_tmp.p;
    }
    st = copy_out(ctx, out, res, f9, mem_kind);
    if (st) return st;
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    return COMBO_OK;
}

int combo_apply_operator(combo_ctx* ctx, int precision, const double* p, double* q, int mem_kind) {
    int st = require_ready(ctx);
    if (st) return st;
    if (precision != COMBO_FP64 && precision != COMBO_MIXED) return set_err(ctx, COMBO_E_INVAL, "bad precision");
    if (ctx->state_prec != precision)
        return set_err(ctx, COMBO_E_STATE, "no tangent state of this precision: call combo_eval_law first");
    if (!p || !q) return set_err(ctx, COMBO_E_INVAL, "null field");
    if (mem_kind != COMBO_MEM_HOST && mem_kind != COMBO_MEM_DEVICE) return set_err(ctx, COMBO_E_INVAL, "bad mem_kind");
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    const size_t f9 = sizeof(double) * 9 * (size_t)ctx->g.n;
    st = copy_in(ctx, ctx->F_save.p, p, f9, mem_kind);
    if (st) return st;
    const double* in_dev = ctx->F_save.as<double>();
    if (staggered(ctx)) {
        if ((st = to_shifted(ctx, ctx->F_save.as<double>(), ctx->stag_tmp.as<double>()))) return st;
        in_dev = ctx->stag_tmp.as<double>();
    }
    if (precision == COMBO_MIXED) st = apply_operator_impl<float>(ctx, in_dev, ctx->dF.as<double>());
    else st = apply_operator_impl<double>(ctx, in_dev, ctx->dF.as<double>());
    if (st) return st;
    const void* res = ctx->dF.p;
    if (staggered(ctx)) {
        if ((st = to_natural(ctx, ctx->dF.as<double>(), ctx->stag_tmp.as<double>()))) return st;
        res = ctx->stag_tmp.p;
    }
    st = copy_out(ctx, q, res, f9, mem_kind);
    if (st) return st;
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    return COMBO_OK;
}

int combo_autotune(combo_ctx* ctx, int precision, int* xv, int* yv, int* zv) {
    int st = require_ready(ctx);
    if (st) return st;
    if (precision != COMBO_FP64 && precision != COMBO_MIXED) return set_err(ctx, COMBO_E_INVAL, "bad precision");
    HIP_OR_FAIL(hipSetDevice(ctx->device));
    st = autotune(ctx, precision);
    if (st) return st;
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    if (xv) *xv = ctx->g.xv;
    if (yv) *yv = ctx->g.yv;
    if (zv) *zv = ctx->g.zv;
    return COMBO_OK;
}

int combo_set_schedule(combo_ctx* ctx, int xv, int yv, int zv) {
    if (!ctx) return COMBO_E_INVAL;
    if (!ctx->has_grid) return set_err(ctx, COMBO_E_STATE, "combo_set_grid has not been called");
    if (xv < 0 || yv < 0 || zv < 0) return set_err(ctx, COMBO_E_INVAL, "schedule variants must be >= 0");
    Schedule sc;
    sc.xv = xv;
    sc.yv = yv;
    sc.zv = zv;
    apply_schedule(ctx, sc);
    return COMBO_OK;
}

int combo_get_schedule(const combo_ctx* ctx, int* xv, int* yv, int* zv, int* nxv, int* nyv, int* nzv) {
    if (!ctx) return COMBO_E_INVAL;
    if (xv) *xv = ctx->g.xv;
    if (yv) *yv = ctx->g.yv;
    if (zv) *zv = ctx->g.zv;
    if (nxv) *nxv = std::max(1, xpass_lds_variants(ctx->g.n1));
    if (nyv) *nyv = std::max(1, fft2_variants<float>(ctx->g.n2));
    if (nzv) *nzv = std::max(1, fft2_variants<float>(ctx->g.n3));
    return COMBO_OK;
}

int combo_profile_enable(combo_ctx* ctx, int enable) {
    if (!ctx) return COMBO_E_INVAL;
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx);
    ctx->profile = enable != 0;
    for (int k = 0; k < COMBO_K_COUNT; ++k) {
        ctx->prof_ms[k] = 0.0;
        ctx->prof_n[k] = 0;
        ctx->prof_idle_ms[k] = 0.0;
        ctx->prof_idle_n[k] = 0;
    }
    return COMBO_OK;
}

int combo_profile_select(combo_ctx* ctx, unsigned mask) {
    if (!ctx) return COMBO_E_INVAL;
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx);
    ctx->prof_mask = mask;
    return COMBO_OK;
}

int combo_profile_read(combo_ctx* ctx, int kernel, double* ms_total, long long* launches) {
    if (!ctx || kernel < 0 || kernel >= COMBO_K_COUNT) return COMBO_E_INVAL;
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx);
    if (ms_total) *ms_total = ctx->prof_ms[kernel];
    if (launches) *launches = ctx->prof_n[kernel];
    return COMBO_OK;
}

int combo_profile_read_idle(combo_ctx* ctx, int kernel, double* ms_total, long long* launches) {
    if (!ctx || kernel < 0 || kernel >= COMBO_K_COUNT) return COMBO_E_INVAL;
    HIP_OR_FAIL(hipStreamSynchronize(ctx->stream));
    prof_harvest(ctx);
    if (ms_total) *ms_total = ctx->prof_idle_ms[kernel];
    if (launches) *launches = ctx->prof_idle_n[kernel];
    return COMBO_OK;
}

// ---- batches ------------------------------------------------------------------
int combo_batch_create(combo_batch** out, int device, void* stream) {
    if (!out) return COMBO_E_INVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return COMBO_E_HIP;
    if (device < 0 || device >= count) return COMBO_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return COMBO_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return COMBO_E_HIP;
    if (std::string(prop.gcnArchName).find("gfx950") == std::string::npos) return COMBO_E_HIP;
    combo_batch* b = new combo_batch();
    b->device = device;
    if (stream) {
        b->stream = static_cast<hipStream_t>(stream);
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return COMBO_E_HIP;
        }
        b->own_stream = true;
    }
    combo_default_options(&b->opt);
    *out = b;
    return COMBO_OK;
}

int combo_batch_destroy(combo_batch* b) {
    if (!b) return COMBO_E_INVAL;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    for (hipStream_t ls : b->lane_streams) (void)hipStreamSynchronize(ls);
    for (combo_ctx* m : b->members) combo_destroy(m);
    b->members.clear();
    for (hipStream_t ls : b->lane_streams) (void)hipStreamDestroy(ls);
    b->lane_streams.clear();
    b->scal.release();
    if (b->hscal) (void)hipHostFree(b->hscal);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return COMBO_OK;
}

const char* combo_batch_last_error(const combo_batch* b) { return b ? b->err.c_str() : "null batch"; }

int combo_batch_size(const combo_batch* b) { return b ? (int)b->members.size() : 0; }

int combo_batch_set_options(combo_batch* b, const combo_options* o) {
    if (!b || !o) return COMBO_E_INVAL;
    const char* bad = options_error(o);
    if (bad) return bset_err(b, COMBO_E_INVAL, bad);
    b->opt = *o;
    for (combo_ctx* m : b->members) combo_set_options(m, o);
    return COMBO_OK;
}

int combo_batch_set_discretization(combo_batch* b, int disc) {
    if (!b) return COMBO_E_INVAL;
    if (disc != COMBO_DISC_MS && disc != COMBO_DISC_WILLOT)
        return bset_err(b, COMBO_E_INVAL, "batches take COMBO_DISC_MS or COMBO_DISC_WILLOT members");
    b->disc = disc;
    return COMBO_OK;
}

int combo_batch_add(combo_batch* b, int n1, int n2, int n3, double l1, double l2, double l3,
                    const combo_material mats[2], const uint8_t* phase, const double* c, const double* N, int mem_kind,
                    int* index) {
    if (!b) return COMBO_E_INVAL;
    if (!mats) return bset_err(b, COMBO_E_INVAL, "materials are null");
    combo_ctx* m = nullptr;
    int st = combo_create(&m, b->device, b->stream);
    if (st) return bset_err(b, st, "member context creation failed");
    st = combo_set_grid(m, n1, n2, n3, l1, l2, l3);
    if (!st && b->disc != COMBO_DISC_MS) st = combo_set_discretization(m, b->disc);
    if (!st) st = combo_set_materials(m, mats);
    if (!st) st = combo_set_options(m, &b->opt);
    if (!st) st = combo_set_microstructure(m, phase, c, N, mem_kind);
    if (st) {
        bset_err(b, st, "member " + std::to_string(b->members.size()) + ": " + m->err);
        combo_destroy(m);
        return st;
    }
    if (index) *index = (int)b->members.size();
    b->members.push_back(m);
    return COMBO_OK;
}

int combo_batch_solve(combo_batch* B, const double* Fbar, const int* n_increments, double* Pbar, double* Abar,
                      double* Pbar_phase, combo_stats* stats) {
    if (!B) return COMBO_E_INVAL;
    const size_t nm = B->members.size();
    if (stats) memset(stats, 0, sizeof(combo_stats) * nm);
    if (nm == 0) return bset_err(B, COMBO_E_STATE, "the batch has no members");
    if (!Fbar) return bset_err(B, COMBO_E_INVAL, "Fbar is null");
    for (size_t i = 0; i < nm; ++i) {
        const std::string who = "member " + std::to_string(i) + ": ";
        if (!finite9(Fbar + 9 * i)) return bset_err(B, COMBO_E_NUMERIC, who + "Fbar is not finite");
        if (B->opt.law != COMBO_LAW_LINEAR && !(det9(Fbar + 9 * i) > 0.0)) return bset_err(B, COMBO_E_INADMISSIBLE, who + "det Fbar <= 0");
        if (n_increments && n_increments[i] < 1) return bset_err(B, COMBO_E_INVAL, who + "n_increments < 1");
    }
    BHIP_OR_FAIL(hipSetDevice(B->device));
    const auto t_start = clk::now();
    const size_t stride = combo_batch::kScalStride;
    if (B->scal.bytes < stride * nm) {
        BHIP_OR_FAIL(B->scal.ensure(stride * nm));
        if (B->hscal) (void)hipHostFree(B->hscal);
        B->hscal = nullptr;
        BHIP_OR_FAIL(hipHostMalloc((void**)&B->hscal, stride * nm, hipHostMallocDefault));
        B->hscal_bytes = stride * nm;
    }
    if (B->opt.autotune) {
        for (size_t i = 0; i < nm; ++i) {
            combo_ctx* ctx = B->members[i];
            ctx->cgst.borrow(static_cast<char*>(B->scal.p) + i * stride, sizeof(CGState));
            const int st = autotune(ctx, B->opt.precision);
            if (st) return bset_err(B, st, "member " + std::to_string(i) + ": " + ctx->err);
        }
    }
    // lanes: members of similar grid size share launches on a stream of their own
    const int nlanes_max = B->opt.batch_streams > 0 ? B->opt.batch_streams : 8;
    const std::vector<std::vector<int>> lane_members = assign_lanes(B->members, nlanes_max);
    while (B->lane_streams.size() + 1 < lane_members.size()) {
        hipStream_t ls = nullptr;
        BHIP_OR_FAIL(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking));
        B->lane_streams.push_back(ls);
    }
    std::vector<Lane> lanes(lane_members.size());
    std::vector<size_t> slot_of(nm);
    {
        size_t next = 0;
        for (size_t l = 0; l < lanes.size(); ++l) {
            lanes[l].members = lane_members[l];
            lanes[l].slot0 = next;
            lanes[l].stream = l == 0 ? B->stream : B->lane_streams[l - 1];
            for (int i : lane_members[l]) slot_of[i] = next++;
        }
    }
    std::vector<Member> ms(nm);
    for (size_t i = 0; i < nm; ++i) {
        Member& m = ms[i];
        combo_ctx* ctx = B->members[i];
        m.ctx = ctx;
        m.index = (int)i;
        m.slot = slot_of[i];
        char* base = static_cast<char*>(B->scal.p) + m.slot * stride;
        ctx->cgst.borrow(base, sizeof(CGState));
        ctx->sums.borrow(base + combo_batch::kScalSums, sizeof(double) * (kSumsLen + 16));
        for (int c = 0; c < 9; ++c) {
            m.Fbar[c] = Fbar[9 * i + c];
            m.Fbar0[c] = (c % 4 == 0) ? 1.0 : 0.0;
        }
        m.K = n_increments ? n_increments[i] : std::max(1, ctx->opt.n_increments);
        reference_medium(ctx, m.mu0, m.kappa0);
        m.tol_cg = ctx->opt.tol_cg;
        if (ctx->opt.precision == COMBO_MIXED) m.tol_cg = std::max(m.tol_cg, 1e-5);
        const long long n = ctx->g.n;
        hipLaunchKernelGGL(k_fill_identity, dim3(1024), dim3(256), 0, B->stream, ctx->F_cur.as<double>(), n);
        BHIP_OR_FAIL(hipGetLastError());
        BHIP_OR_FAIL(hipMemsetAsync(ctx->a_prev.p, 0, sizeof(double) * 3 * std::max(ctx->nc, 1), B->stream));
        hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(64), 0, B->stream, ctx->cgst.as<CGState>());
        BHIP_OR_FAIL(hipGetLastError());
        m.k = 1;
        member_begin_increment(m);
    }
    // the set-up above runs on the batch stream; the lanes start after it
    BHIP_OR_FAIL(hipStreamSynchronize(B->stream));
    for (size_t l = 0; l < lanes.size(); ++l)
        for (int i : lanes[l].members) B->members[i]->stream = lanes[l].stream;
    int st = B->opt.precision == COMBO_MIXED ? batch_solve_impl<float>(B, ms, lanes)
                                             : batch_solve_impl<double>(B, ms, lanes);
    for (combo_ctx* ctx : B->members) ctx->stream = B->stream;
    if (st) return st;
    // effective tangents, member by member
    for (Member& m : ms) {
        if (m.phase != PH_DONE || !B->opt.want_tangent || !Abar) continue;
        int it = 0;
        auto tt = clk::now();
        int s2 = B->opt.precision == COMBO_MIXED
                     ? effective_tangent<float>(m.ctx, m.mu0, m.kappa0, m.tol_cg, m.out.Abar_store, it)
                     : effective_tangent<double>(m.ctx, m.mu0, m.kappa0, m.tol_cg, m.out.Abar_store, it);
        m.out.st.time_ms_tangent = ms_since(tt);
        m.out.st.cg_iters_tangent = it;
        if (s2) member_fail(m, s2, m.ctx->err);
    }
    BHIP_OR_FAIL(hipStreamSynchronize(B->stream));
    const double wall = ms_since(t_start);
    int first = COMBO_OK;
    for (size_t i = 0; i < nm; ++i) {
        Member& m = ms[i];
        m.out.st.status = m.phase == PH_DONE ? COMBO_OK : m.status;
        m.out.st.time_ms_total = wall;
        if (stats) stats[i] = m.out.st;
        if (m.phase != PH_DONE) {
            if (first == COMBO_OK) {
                first = m.status;
                B->err = "member " + std::to_string(i) + ": " + m.ctx->err;
            }
            continue;
        }
        if (Pbar) memcpy(Pbar + 9 * i, m.out.Pbar, sizeof(m.out.Pbar));
        if (Pbar_phase) {
            memcpy(Pbar_phase + 18 * i, m.out.Pp, sizeof(m.out.Pp));
            memcpy(Pbar_phase + 18 * i + 9, m.out.Pm, sizeof(m.out.Pm));
        }
        if (Abar && B->opt.want_tangent) memcpy(Abar + 81 * i, m.out.Abar_store, sizeof(m.out.Abar_store));
    }
    return first;
}

int combo_batch_fields(combo_batch* B, int i, double* F, double* P, int mem_kind) {
    if (!B) return COMBO_E_INVAL;
    if (i < 0 || i >= (int)B->members.size()) return bset_err(B, COMBO_E_INVAL, "member index out of range");
    if (mem_kind != COMBO_MEM_HOST && mem_kind != COMBO_MEM_DEVICE) return bset_err(B, COMBO_E_INVAL, "bad mem_kind");
    combo_ctx* ctx = B->members[i];
    BHIP_OR_FAIL(hipSetDevice(B->device));
    const size_t f9 = sizeof(double) * 9 * (size_t)ctx->g.n;
    int st = COMBO_OK;
    if (F && (st = copy_out(ctx, F, ctx->F_cur.p, f9, mem_kind))) return bset_err(B, st, ctx->err);
    if (P && (st = copy_out(ctx, P, ctx->P.p, f9, mem_kind))) return bset_err(B, st, ctx->err);
    BHIP_OR_FAIL(hipStreamSynchronize(B->stream));
    return COMBO_OK;
}

}  // extern "C"
