// Composite boxels from a fine binary image (paper Sec. 5): argument block and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace combo {

struct BoxelArgs {
    const uint8_t* chi;         // [N3][N2][N1] fine image, 1 = inclusion, 0 = matrix
    long long N1, N2, N3;       // fine voxels per axis (N_m = n_m s_m)
    int n1, n2, n3;             // boxels per axis
    int s1, s2, s3;             // fine voxels per boxel and axis
    double h[3];                // fine voxel size
    double r[3];                // stencil ratios r_m = h_i h_j / h_m
    int method;                 // 0: Laplacian moments (Sec. 5.2), 1: barycentres (eq. normal:kabel)
    int vec4;                   // rows start 4-byte aligned and s1 % 4 == 0: pass 1 reads dwords
    int vec16;                  // s1 == 4, n1 % 4 == 0, rows 16-byte aligned, phase and c 16-byte
                                // aligned: pass 1 takes four boxels per thread with 16-byte loads
    uint8_t* phase;             // [nb] out
    double* c;                  // [nb] out
    double* N;                  // [3][nb] out
    uint64_t* packed;           // [nb] or null: pass 1 (four-boxel path, s1 = 4, s2 s3 <= 16) stores each
                                // boxel's fine values as bits x + 4 (y + s2 z) for pass 2
    int* counter;               // [2] scratch, zero before pass 1: [0] composites (pass 2a), [1] nonzero if a
                                // value is not 0/1
};

// Zero n ints (the counters before pass 1) with a kernel rather than a memset.
hipError_t launch_boxel_zero(int* p, int n, hipStream_t s);
// Pass 1, one thread per boxel: volume fraction and phase.
hipError_t launch_boxel_count(const BoxelArgs& a, hipStream_t s);
// Pass 2a: N = 0 for pure boxels, the ordered list of composite boxels (blockcnt: boxel_blocks(nb)
// ints, list: nb ints; the count goes to counter[0]).
int boxel_blocks(long long nb);
hipError_t launch_boxel_list(const BoxelArgs& a, int* blockcnt, int* list, hipStream_t s);
// Exclusive prefix of nblk ints in place (one workgroup); the total goes to total[0].
hipError_t launch_block_scan(int* cnt, int nblk, int* total, hipStream_t s);
// Pass 2b: moments and normals of the ncomp entries.  Packed words: one lane per entry, mom unused;
// byte path: 16 lanes per entry through mom (13 doubles per entry).
hipError_t launch_boxel_normals(const BoxelArgs& a, const int* list, double* mom, int ncomp, hipStream_t s);

}  // namespace combo
