// Composite boxels from a fine binary image on gfx950 (paper Sec. 5).
//
// Per boxel of s1 x s2 x s3 fine voxels (fine voxel size h):
//   c+ = mean of chi, phase 0 / 1 / 2 for c+ = 0 / 1 / between;
//   barycentre normal (eq. normal:kabel): N~ ~ c- - c+; with xi the fine voxel
//     centre in half-voxel units from the boxel centre (xi_m = 2 x_m + 1 - s_m) the
//     xi of the whole boxel sum to zero, so c- - c+ ~ -h (.) sum_{chi=1} xi;
//   interface weights [N.1]: w = |sum_m r_m (chi(-e_m) - 2 chi + chi(+e_m))| with
//     r_m = h_i h_j / h_m.  At a fine voxel all three second differences have the
//     sign of (1 - 2 chi) (the neighbours are 0 or 1), so w = sum_m r_m |a_m| with
//     integer a_m in {0, 1, 2};
//   [N.2]: M = sum w x (x) x with x taken from the weighted barycentre of the
//     interface, i.e. the centred moment sum w xi xi^T - (sum w xi)(sum w xi)^T / sum w
//     scaled by h_d h_e / 4; N = eigenvector of its smallest eigenvalue (cyclic
//     Jacobi in FP64), flipped unless N~ . N > 0 (eq. normal:flip).
// Pass 1 (one thread per boxel) streams the image once with dword loads and
// popcounts and writes c and phase; pass 2 (one wave per 64 boxels) writes N = 0
// for pure boxels and revisits the composite ones, four at a time with 16 lanes
// each, with their one-voxel periodic halo.
#include <hip/hip_runtime.h>

#include "boxels.h"

namespace combo {

namespace {

constexpr int kTeam = 16;

__global__ void __launch_bounds__(256) k_boxel_count(BoxelArgs a) {
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int i = (int)(b % a.n1);
    const long long t = b / a.n1;
    const int j = (int)(t % a.n2), k = (int)(t / a.n2);
    const long long V = (long long)a.s1 * a.s2 * a.s3;
    const int rows = a.s2 * a.s3;
    const uint8_t* base = a.chi + ((long long)k * a.s3 * a.N2 + (long long)j * a.s2) * a.N1 + (long long)i * a.s1;
    long long cnt = 0;
    unsigned bad = 0;
    if (a.vec4) {
        const int q = a.s1 / 4;
#pragma unroll 8
        for (int r = 0; r < rows; ++r) {
            const int z = r / a.s2, y = r - z * a.s2;
            const uint32_t* r4 = reinterpret_cast<const uint32_t*>(base + ((long long)z * a.N2 + y) * a.N1);
            for (int x = 0; x < q; ++x) {
                const uint32_t v = r4[x];
                bad |= v & 0xFEFEFEFEu;
                cnt += __popc(v);
            }
        }
    } else {
        for (int r = 0; r < rows; ++r) {
            const int z = r / a.s2, y = r - z * a.s2;
            const uint8_t* row = base + ((long long)z * a.N2 + y) * a.N1;
            for (int x = 0; x < a.s1; ++x) {
                const unsigned v = row[x];
                bad |= v & 0xFEu;
                cnt += v;
            }
        }
    }
    if (bad) atomicOr(&a.counter[1], 1);
    a.c[b] = (double)cnt / (double)V;
    a.phase[b] = (uint8_t)((cnt == 0) ? 0 : (cnt == V ? 1 : 2));
}

// s1 = 4, n1 % 4 == 0, 16-byte aligned rows: one thread per 4 boxels along x,
// one 16-byte load per fine row (lane q of the load is boxel q's row)
__global__ void __launch_bounds__(256) k_boxel_count4(BoxelArgs a) {
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    const long long b4 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (b4 >= nb) return;
    const int i = (int)(b4 % a.n1);
    const long long t = b4 / a.n1;
    const int j = (int)(t % a.n2), k = (int)(t / a.n2);
    const long long V = 4LL * a.s2 * a.s3;
    const int rows = a.s2 * a.s3;
    const uint8_t* base = a.chi + ((long long)k * a.s3 * a.N2 + (long long)j * a.s2) * a.N1 + (long long)i * 4;
    int cnt[4] = {0, 0, 0, 0};
    unsigned bad = 0;
#pragma unroll 8
    for (int r = 0; r < rows; ++r) {
        const int z = r / a.s2, y = r - z * a.s2;
        const uint4 v = *reinterpret_cast<const uint4*>(base + ((long long)z * a.N2 + y) * a.N1);
        bad |= (v.x | v.y | v.z | v.w) & 0xFEFEFEFEu;
        cnt[0] += __popc(v.x);
        cnt[1] += __popc(v.y);
        cnt[2] += __popc(v.z);
        cnt[3] += __popc(v.w);
    }
    if (bad) atomicOr(&a.counter[1], 1);
    double2 c01, c23;
    c01.x = (double)cnt[0] / (double)V;
    c01.y = (double)cnt[1] / (double)V;
    c23.x = (double)cnt[2] / (double)V;
    c23.y = (double)cnt[3] / (double)V;
    *reinterpret_cast<double2*>(a.c + b4) = c01;
    *reinterpret_cast<double2*>(a.c + b4 + 2) = c23;
    uint32_t ph = 0;
    for (int q = 0; q < 4; ++q) ph |= (uint32_t)((cnt[q] == 0) ? 0 : (cnt[q] == V ? 1 : 2)) << (8 * q);
    *reinterpret_cast<uint32_t*>(a.phase + b4) = ph;
}

__device__ __forceinline__ int wrap(long long v, long long n) { return (int)(v < 0 ? v + n : (v >= n ? v - n : v)); }

// eigenvector of the smallest eigenvalue of a symmetric 3x3 matrix (cyclic Jacobi)
__device__ void smallest_eigvec(double A[3][3], double v[3]) {
    double Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 12; ++sweep) {
        // stop once the off-diagonal part is at round-off of the diagonal (|off| <= 1e-16 |diag|)
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (!(off > 1e-32 * dia)) break;
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            const double apq = A[p][q];
            if (!(fabs(apq) > 1e-17 * (fabs(A[p][p]) + fabs(A[q][q])))) continue;
            const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            // A <- J^T A J with J the rotation in the (p, q) plane
            for (int m = 0; m < 3; ++m) {
                const double amp = A[m][p], amq = A[m][q];
                A[m][p] = c * amp - s * amq;
                A[m][q] = s * amp + c * amq;
            }
            for (int m = 0; m < 3; ++m) {
                const double apm = A[p][m], aqm = A[q][m];
                A[p][m] = c * apm - s * aqm;
                A[q][m] = s * apm + c * aqm;
            }
            for (int m = 0; m < 3; ++m) {
                const double qmp = Q[m][p], qmq = Q[m][q];
                Q[m][p] = c * qmp - s * qmq;
                Q[m][q] = s * qmp + c * qmq;
            }
        }
    }
    int imin = 0;
    if (A[1][1] < A[imin][imin]) imin = 1;
    if (A[2][2] < A[imin][imin]) imin = 2;
    const double nv = sqrt(Q[0][imin] * Q[0][imin] + Q[1][imin] * Q[1][imin] + Q[2][imin] * Q[2][imin]);
    for (int m = 0; m < 3; ++m) v[m] = Q[m][imin] / nv;
}

template <typename X>
__device__ __forceinline__ X team_sum(X v) {
#pragma unroll
    for (int m = kTeam / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, kTeam);
    return v;
}

// one wave per 64 consecutive boxels: pure boxels get N = 0; 16-lane teams reduce
// the moments of the composite ones, four at a time, into the wave's LDS slots,
// then every composite lane solves its own 3x3 eigenproblem
constexpr int kMom = 13;   // sw, sw xi (3), sw xi xi^T (6), sum_{chi=1} xi (3)

__global__ void __launch_bounds__(256) k_boxel_normals(BoxelArgs a) {
    __shared__ double mom[256][kMom];
    const int lane = threadIdx.x & 63;
    const int wbase = threadIdx.x - lane;
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    const long long b0 = (long long)blockIdx.x * blockDim.x + wbase;
    const long long bl = b0 + lane;
    const int ph = (bl < nb) ? a.phase[bl] : 0;
    unsigned long long mask = __ballot(ph == 2);
    if (bl < nb && ph != 2) {
        a.N[bl] = 0.0;
        a.N[nb + bl] = 0.0;
        a.N[2 * nb + bl] = 0.0;
    }
    const int s1 = a.s1, s2 = a.s2, s3 = a.s3;
    const long long V = (long long)s1 * s2 * s3;
    const int team = lane / kTeam;
    const int tl = lane % kTeam;
    while (mask) {
        unsigned long long m = mask;
        for (int q = 0; q < team && m; ++q) m &= m - 1;
        for (int q = 0; q < 64 / kTeam && mask; ++q) mask &= mask - 1;
        if (!m) continue;   // uniform over the team
        const int bit = __builtin_ctzll(m);
        const long long b = b0 + bit;
        const int i = (int)(b % a.n1);
        const long long tt = b / a.n1;
        const int j = (int)(tt % a.n2), k = (int)(tt / a.n2);
        double acc[kMom];
#pragma unroll
        for (int q = 0; q < kMom; ++q) acc[q] = 0.0;
        const int V32 = (int)V;
        for (int t = tl; t < V32; t += kTeam) {
            const int u = t / s1;
            const int x = t - u * s1;
            const int z = u / s2;
            const int y = u - z * s2;
            const long long X = (long long)i * s1 + x, Y = (long long)j * s2 + y, Z = (long long)k * s3 + z;
            const uint8_t* plane = a.chi + Z * a.N2 * a.N1;
            const uint8_t* row = plane + Y * a.N1;
            const int c0 = row[X];
            const int xm = row[wrap(X - 1, a.N1)], xp = row[wrap(X + 1, a.N1)];
            const int ym = plane[(long long)wrap(Y - 1, a.N2) * a.N1 + X];
            const int yp = plane[(long long)wrap(Y + 1, a.N2) * a.N1 + X];
            const int zm = a.chi[((long long)wrap(Z - 1, a.N3) * a.N2 + Y) * a.N1 + X];
            const int zp = a.chi[((long long)wrap(Z + 1, a.N3) * a.N2 + Y) * a.N1 + X];
            const int a1 = abs(xm + xp - 2 * c0), a2 = abs(ym + yp - 2 * c0), a3 = abs(zm + zp - 2 * c0);
            const int xi0 = 2 * x + 1 - s1, xi1 = 2 * y + 1 - s2, xi2 = 2 * z + 1 - s3;
            if (c0) {
                acc[10] += xi0;
                acc[11] += xi1;
                acc[12] += xi2;
            }
            if (a1 | a2 | a3) {
                const double w = a.r[0] * a1 + a.r[1] * a2 + a.r[2] * a3;
                const double wx = w * xi0, wy = w * xi1, wz = w * xi2;
                acc[0] += w;
                acc[1] += wx;
                acc[2] += wy;
                acc[3] += wz;
                acc[4] += wx * xi0;
                acc[5] += wx * xi1;
                acc[6] += wx * xi2;
                acc[7] += wy * xi1;
                acc[8] += wy * xi2;
                acc[9] += wz * xi2;
            }
        }
#pragma unroll
        for (int q = 0; q < kMom; ++q) acc[q] = team_sum(acc[q]);
        if (tl == 0)
#pragma unroll
            for (int q = 0; q < kMom; ++q) mom[wbase + bit][q] = acc[q];
    }
    __syncthreads();
    if (ph != 2) return;
    const double* mm = mom[threadIdx.x];
    // sum_{chi=1} xi holds integers (exact in double); N~ ~ -h (.) that sum
    const double nt[3] = {-a.h[0] * mm[10], -a.h[1] * mm[11], -a.h[2] * mm[12]};
    double out[3];
    if (a.method == 1) {
        const double nn = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
        if (nn > 0) {
            for (int q = 0; q < 3; ++q) out[q] = nt[q] / nn;
        } else {
            out[0] = 1.0;
            out[1] = out[2] = 0.0;
        }
    } else {
        const double sw = mm[0];
        const double sx[3] = {mm[1], mm[2], mm[3]};
        const double S[3][3] = {{mm[4], mm[5], mm[6]}, {mm[5], mm[7], mm[8]}, {mm[6], mm[8], mm[9]}};
        double M[3][3];
        for (int d = 0; d < 3; ++d)
            for (int e = 0; e < 3; ++e) M[d][e] = 0.25 * a.h[d] * a.h[e] * (S[d][e] - sx[d] * sx[e] / sw);
        double v[3];
        smallest_eigvec(M, v);
        const double dot = nt[0] * v[0] + nt[1] * v[1] + nt[2] * v[2];
        const double sg = dot > 0 ? 1.0 : -1.0;
        for (int q = 0; q < 3; ++q) out[q] = sg * v[q];
    }
    a.N[bl] = out[0];
    a.N[nb + bl] = out[1];
    a.N[2 * nb + bl] = out[2];
}

}  // namespace

hipError_t launch_boxel_count(const BoxelArgs& a, hipStream_t s) {
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    if (a.vec16) {
        const unsigned blocks = (unsigned)((nb / 4 + 255) / 256);
        hipLaunchKernelGGL(k_boxel_count4, dim3(blocks), dim3(256), 0, s, a);
    } else {
        const unsigned blocks = (unsigned)((nb + 255) / 256);
        hipLaunchKernelGGL(k_boxel_count, dim3(blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_boxel_normals(const BoxelArgs& a, hipStream_t s) {
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    const unsigned blocks = (unsigned)((nb + 255) / 256);
    hipLaunchKernelGGL(k_boxel_normals, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace combo
