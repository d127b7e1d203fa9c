// Internal state of a libcombo context (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "combo.h"
#include "common.h"
#include "kernels.h"
#include "material.h"

namespace combo {

// Owning device allocation that only grows.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool own = true;   // false: a view of memory owned elsewhere (never freed here)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p && own) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        own = true;
    }
    void borrow(void* q, size_t nbytes) {
        release();
        p = q;
        bytes = nbytes;
        own = false;
    }
    hipError_t ensure(size_t nbytes) {
        if (nbytes <= bytes && p) return hipSuccess;
        release();
        if (nbytes == 0) nbytes = 16;
        hipError_t e = hipMalloc(&p, nbytes);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = nbytes;
        return hipSuccess;
    }
    template <typename X> X* as() const { return static_cast<X*>(p); }
};

// Host-visible scalars copied back once per material / residual evaluation.
struct HostScalars {
    CGState cg;
    double sums[kSumsLen];
};

// Captured CG iteration chunk (one per precision).
struct CGGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int iters = 0;
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        iters = 0;
    }
};

}  // namespace combo

struct combo_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    size_t lds_limit = 65536;

    // grid
    bool has_grid = false;
    combo::Grid g{};
    double l[3] = {1, 1, 1};
    combo::AxisPlan plan[3]{};
    combo::DevBuf tw32[3], tw64[3];
    combo::DevBuf ftab;                   // gradient factor table of the rotated scheme
    combo::DevBuf bx_scratch, bx_mom;     // image -> boxels: counters, block offsets, list; moments
    combo::DevBuf bx_packed;              // image -> boxels: one 64-bit word of fine values per boxel

    // materials and options
    bool has_mats = false;
    combo_material mats[2]{};
    combo_options opt{};

    // microstructure
    bool has_ms = false;
    int nc = 0;
    double n_mat = 0, n_incl = 0, sum_c = 0;
    combo::DevBuf slot, slot_s, comp_vox, comp_c, comp_N, a_prev, a_trial;   // slot: natural order, slot_s: state_pos order
    // staggered grid with the DFMG law: stresses, tangent states and stress increments of the
    // doubly-fine cells, the shifted-layout fields of the CG operator and a layout scratch field
    combo::DevBuf dfmg_Pd, dfmg_Ad, dfmg_act, dfmg_dH, dfmg_dQ, stag_tmp;
    const double* dfmg_Feval = nullptr;   // F (shifted layout) of the last law evaluation, for the tangent action

    // fields (FP64) and work buffers
    combo::DevBuf F_cur, F_trial, F_save, dF, P;
    combo::DevBuf specA, specB;           // spectra, sized for FP64
    combo::DevBuf ux, ur, up, uq;         // CG vectors, sized for FP64
    combo::DevBuf Sinv, sm, Acomp;        // tangent state, sized for FP64
    int state_prec = -1;                  // precision the tangent state was written in
    combo::DevBuf part1, part2, sums, cgst;
    combo::HostScalars* hs = nullptr;     // pinned host copy of the device scalars
    combo::CGGraph graph[2];

    // per-kernel event timing
    bool profile = false;
    unsigned prof_mask = ~0u;   // kernel classes timed while profiling (bit k: class k)
    // iter: position of the launch's CG iteration in its chunk (-1 outside a chunk);
    // launches of iterations after the one that finished the CG return at once and
    // are counted apart (prof_idle_*), so the averages cover launches that did work
    struct ProfRec { int kernel; hipEvent_t start, stop; int iter; };
    std::vector<ProfRec> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    int prof_iter = -1;
    double prof_ms[COMBO_K_COUNT] = {};
    long long prof_n[COMBO_K_COUNT] = {};
    double prof_idle_ms[COMBO_K_COUNT] = {};
    long long prof_idle_n[COMBO_K_COUNT] = {};
};

// A batch of independent RVEs solved together (each member is a full context
// sharing the batch's stream; its CG state and sums live in one device array
// so that one copy brings every member's scalars to the host).
struct combo_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    combo_options opt{};
    int disc = COMBO_DISC_MS;           // discretization of members added from now on
    std::vector<combo_ctx*> members;
    std::vector<hipStream_t> lane_streams;   // streams of lanes 1.. (lane 0 runs on `stream`); owned
    combo::DevBuf scal;                 // [members] x kScalStride bytes: CGState at 0, sums at kScalSums
    char* hscal = nullptr;              // pinned host copy of scal
    size_t hscal_bytes = 0;
    static constexpr size_t kScalStride = 1024;
    static constexpr size_t kScalSums = 128;
    static_assert(sizeof(combo::CGState) <= kScalSums, "a member's CG state overlaps its sums");
};

