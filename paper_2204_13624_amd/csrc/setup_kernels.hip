// Microstructure setup on gfx950: validation, counts and the ordered composite list
// from device-resident fields, so that a microstructure made on the device (e.g. by
// the boxel kernels) never crosses to the host.
//
// Pass 1, blocks of kSetupBlock voxels: matrix / inclusion / composite counts, the
// sum of c over the composites (fixed reduction order: the result does not depend
// on scheduling) and the smallest invalid voxel index (atomicMin; the host turns it
// into a message).  The composite counts are scanned in one workgroup.  Pass 2
// writes each voxel's slot (composite index, -1 matrix, -2 inclusion) in natural
// and in state order, and the composites' voxel, c and normalised N, ascending.
#include <hip/hip_runtime.h>

#include <climits>

#include "boxels.h"
#include "common.h"
#include "setup.h"

namespace combo {

namespace {

constexpr int kSetupBlock = 1024;   // voxels per workgroup (256 threads x 4)

// Same conditions as the host validation: composite voxels need 0 < c < 1 and a finite
// unit normal (within 1e-6); phase ids above 2 are invalid.
__device__ inline bool voxel_invalid(const SetupArgs& a, long long v, int ph) {
    if (ph > 2) return true;
    if (ph != 2) return false;
    const double cv = a.c[v];
    if (!(cv > 0.0 && cv < 1.0)) return true;
    const double x = a.N[v], y = a.N[a.n + v], z = a.N[2 * a.n + v];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return true;
    return fabs(sqrt(x * x + y * y + z * z) - 1.0) > 1e-6;
}

__global__ void __launch_bounds__(256) k_setup_count(SetupArgs a) {
    __shared__ int r0[4], r1[4], r2[4], rb[4];
    __shared__ double rc[4];
    int c0 = 0, c1 = 0, c2 = 0, bad = INT_MAX;
    double sc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const long long v = (long long)blockIdx.x * kSetupBlock + q * 256 + threadIdx.x;
        if (v >= a.n) continue;
        const int ph = a.phase[v];
        if (ph == 0) ++c0;
        else if (ph == 1) ++c1;
        else if (ph == 2) {
            ++c2;
            sc += a.c[v];
        }
        if (voxel_invalid(a, v, ph)) bad = min(bad, (int)v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        c0 += __shfl_down(c0, off, 64);
        c1 += __shfl_down(c1, off, 64);
        c2 += __shfl_down(c2, off, 64);
        sc += __shfl_down(sc, off, 64);
        bad = min(bad, __shfl_down(bad, off, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        r0[w] = c0;
        r1[w] = c1;
        r2[w] = c2;
        rc[w] = sc;
        rb[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int b = blockIdx.x;
        a.cnt2[b] = r2[0] + r2[1] + r2[2] + r2[3];
        a.cnt01[2 * b] = r0[0] + r0[1] + r0[2] + r0[3];
        a.cnt01[2 * b + 1] = r1[0] + r1[1] + r1[2] + r1[3];
        a.sumc[b] = (rc[0] + rc[1]) + (rc[2] + rc[3]);
        const int bb = min(min(rb[0], rb[1]), min(rb[2], rb[3]));
        if (bb != INT_MAX) atomicMin(a.flags, bb);
    }
}

__global__ void k_setup_reset(int* flags) {
    if (threadIdx.x == 0) {
        flags[0] = INT_MAX;
        flags[1] = 0;
    }
}

__global__ void __launch_bounds__(256) k_setup_compact(SetupArgs a) {
    __shared__ int wsum[4][4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long masks[4];
    int ph[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const long long v = (long long)blockIdx.x * kSetupBlock + q * 256 + threadIdx.x;
        ph[q] = v < a.n ? a.phase[v] : 0;
        masks[q] = __ballot(v < a.n && ph[q] == 2);
        if (lane == 0) wsum[q][w] = __popcll(masks[q]);
    }
    __syncthreads();
    int base = a.cnt2[blockIdx.x];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int before = 0;
        for (int ww = 0; ww < w; ++ww) before += wsum[q][ww];
        const long long v = (long long)blockIdx.x * kSetupBlock + q * 256 + threadIdx.x;
        if (v < a.n) {
            int sl = ph[q] == 0 ? -1 : -2;
            if (ph[q] == 2) {
                sl = base + before + __popcll(masks[q] & below);
                const double x = a.N[v], y = a.N[a.n + v], z = a.N[2 * a.n + v];
                const double s = 1.0 / sqrt(x * x + y * y + z * z);
                a.comp_vox[sl] = (int)v;
                a.comp_c[sl] = a.c[v];
                a.comp_N[sl] = x * s;
                a.comp_N[a.nc + sl] = y * s;
                a.comp_N[2 * (long long)a.nc + sl] = z * s;
            }
            a.slot[v] = sl;
            a.slot_s[state_pos(v, a.n1, a.xm, a.xwbits)] = sl;
        }
        base += wsum[q][0] + wsum[q][1] + wsum[q][2] + wsum[q][3];
    }
}

}  // namespace

int setup_blocks(long long n) { return (int)((n + kSetupBlock - 1) / kSetupBlock); }

hipError_t launch_setup_reset(int* flags, hipStream_t s) {
    hipLaunchKernelGGL(k_setup_reset, dim3(1), dim3(64), 0, s, flags);
    return hipGetLastError();
}

hipError_t launch_setup_count(const SetupArgs& a, hipStream_t s) {
    const int nblk = setup_blocks(a.n);
    hipLaunchKernelGGL(k_setup_count, dim3(nblk), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_block_scan(a.cnt2, nblk, a.flags + 1, s);
}

hipError_t launch_setup_compact(const SetupArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_setup_compact, dim3(setup_blocks(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace combo
