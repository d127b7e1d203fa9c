// Microstructure setup on the device: validation, phase counts and the ordered list
// of composite voxels (paper Sec. 4: composite voxels carry c and N, pure voxels
// only a phase id), computed from device-resident phase, c and N fields.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace combo {

struct SetupArgs {
    const uint8_t* phase;       // [n] 0 matrix, 1 inclusion, 2 composite
    const double* c;            // [n] inclusion volume fraction (read for composites only)
    const double* N;            // [3][n] normal (read for composites only)
    long long n;                // voxels (< 2^31)
    int* cnt2;                  // [nblk] composites per block; scanned in place to offsets
    int* cnt01;                 // [2 nblk] matrix and inclusion voxels per block
    double* sumc;               // [nblk] sum of c over each block's composites
    int* flags;                 // [2]: [0] smallest invalid voxel (INT_MAX: none), [1] composites in total
    // compaction (second launch)
    int n1, xm, xwbits;         // state order of the tangent arrays (state_pos)
    int nc;                     // composites in total
    int* slot;                  // [n] composite index, -1 matrix, -2 inclusion
    int* slot_s;                // [n] the same in state order
    int* comp_vox;              // [nc] voxel of each composite, ascending
    double* comp_c;             // [nc]
    double* comp_N;             // [3][nc] normalised
};

int setup_blocks(long long n);
// Pass 1: per-block counts, composite c sums and the first invalid voxel (flags[0] must hold
// INT_MAX: launch_setup_reset), then the exclusive scan of the composite counts (total in flags[1]).
hipError_t launch_setup_reset(int* flags, hipStream_t s);
hipError_t launch_setup_count(const SetupArgs& a, hipStream_t s);
// Pass 2 (after the host has read flags and sized the lists): slots and the composite lists.
hipError_t launch_setup_compact(const SetupArgs& a, hipStream_t s);

}  // namespace combo
