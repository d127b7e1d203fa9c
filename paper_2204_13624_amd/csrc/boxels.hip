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
// popcounts, writes c and phase and appends composite boxels to a list; pass 2
// (16 lanes per composite boxel) revisits only those boxels with their one-voxel
// periodic halo.
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
    long long cnt = 0;
    unsigned bad = 0;
    const bool vec = a.vec4 != 0;
    for (int z = 0; z < a.s3; ++z)
        for (int y = 0; y < a.s2; ++y) {
            const uint8_t* row = a.chi + ((long long)(k * a.s3 + z) * a.N2 + (long long)(j * a.s2 + y)) * a.N1 +
                                 (long long)i * a.s1;
            if (vec) {
                const uint32_t* r4 = reinterpret_cast<const uint32_t*>(row);
                for (int x = 0; x < a.s1 / 4; ++x) {
                    const uint32_t v = r4[x];
                    bad |= v & 0xFEFEFEFEu;
                    cnt += __popc(v);
                }
            } else {
                for (int x = 0; x < a.s1; ++x) {
                    const unsigned v = row[x];
                    bad |= v & 0xFEu;
                    cnt += v;
                }
            }
        }
    if (bad) atomicOr(&a.counter[1], 1);
    a.c[b] = (double)cnt / (double)V;
    const int ph = (cnt == 0) ? 0 : (cnt == V ? 1 : 2);
    a.phase[b] = (uint8_t)ph;
    if (ph != 2) {
        a.N[b] = 0.0;
        a.N[nb + b] = 0.0;
        a.N[2 * nb + b] = 0.0;
    } else {
        const int pos = atomicAdd(&a.counter[0], 1);
        a.list[pos] = (int)b;
    }
}

__device__ __forceinline__ int wrap(long long v, long long n) { return (int)(v < 0 ? v + n : (v >= n ? v - n : v)); }

// eigenvector of the smallest eigenvalue of a symmetric 3x3 matrix (cyclic Jacobi)
__device__ void smallest_eigvec(double A[3][3], double v[3]) {
    double Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 12; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (!(off > 1e-34 * dia)) break;
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            const double apq = A[p][q];
            if (apq == 0.0) continue;
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

__global__ void __launch_bounds__(256) k_boxel_normals(BoxelArgs a, long long nteams) {
    const int lane = threadIdx.x % kTeam;
    const long long team = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kTeam;
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    const int ncomp = a.counter[0];
    const int s1 = a.s1, s2 = a.s2, s3 = a.s3;
    const long long V = (long long)s1 * s2 * s3;
    for (long long idx = team; idx < ncomp; idx += nteams) {   // uniform over the team
        const long long b = a.list[idx];
        const int i = (int)(b % a.n1);
        const long long tt = b / a.n1;
        const int j = (int)(tt % a.n2), k = (int)(tt / a.n2);
        double sw = 0, swx0 = 0, swx1 = 0, swx2 = 0;
        double sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
        long long sc0 = 0, sc1 = 0, sc2 = 0;
        for (long long t = lane; t < V; t += kTeam) {
            const int x = (int)(t % s1);
            const long long u = t / s1;
            const int y = (int)(u % s2), z = (int)(u / s2);
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
                sc0 += xi0;
                sc1 += xi1;
                sc2 += xi2;
            }
            if (a1 | a2 | a3) {
                const double w = a.r[0] * a1 + a.r[1] * a2 + a.r[2] * a3;
                const double wx = w * xi0, wy = w * xi1, wz = w * xi2;
                sw += w;
                swx0 += wx;
                swx1 += wy;
                swx2 += wz;
                sxx += wx * xi0;
                sxy += wx * xi1;
                sxz += wx * xi2;
                syy += wy * xi1;
                syz += wy * xi2;
                szz += wz * xi2;
            }
        }
        sw = team_sum(sw);
        swx0 = team_sum(swx0);
        swx1 = team_sum(swx1);
        swx2 = team_sum(swx2);
        sxx = team_sum(sxx);
        sxy = team_sum(sxy);
        sxz = team_sum(sxz);
        syy = team_sum(syy);
        syz = team_sum(syz);
        szz = team_sum(szz);
        sc0 = team_sum(sc0);
        sc1 = team_sum(sc1);
        sc2 = team_sum(sc2);
        if (lane != 0) continue;
        double nt[3] = {-a.h[0] * (double)sc0, -a.h[1] * (double)sc1, -a.h[2] * (double)sc2};
        double out[3];
        if (a.method == 1) {
            const double nn = sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
            if (nn > 0) {
                for (int m = 0; m < 3; ++m) out[m] = nt[m] / nn;
            } else {
                out[0] = 1.0;
                out[1] = out[2] = 0.0;
            }
        } else {
            const double sx[3] = {swx0, swx1, swx2};
            const double S[3][3] = {{sxx, sxy, sxz}, {sxy, syy, syz}, {sxz, syz, szz}};
            double M[3][3];
            for (int d = 0; d < 3; ++d)
                for (int e = 0; e < 3; ++e)
                    M[d][e] = 0.25 * a.h[d] * a.h[e] * (S[d][e] - sx[d] * sx[e] / sw);
            double v[3];
            smallest_eigvec(M, v);
            const double dot = nt[0] * v[0] + nt[1] * v[1] + nt[2] * v[2];
            const double sg = dot > 0 ? 1.0 : -1.0;
            for (int m = 0; m < 3; ++m) out[m] = sg * v[m];
        }
        a.N[b] = out[0];
        a.N[nb + b] = out[1];
        a.N[2 * nb + b] = out[2];
    }
}

}  // namespace

hipError_t launch_boxel_count(const BoxelArgs& a, hipStream_t s) {
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    const unsigned blocks = (unsigned)((nb + 255) / 256);
    hipLaunchKernelGGL(k_boxel_count, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_boxel_normals(const BoxelArgs& a, hipStream_t s) {
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    // at most one team per boxel; teams loop over the composites pass 1 found
    const long long blocks = std::min<long long>((nb * kTeam + 255) / 256, 8192);
    const long long nteams = blocks * 256 / kTeam;
    hipLaunchKernelGGL(k_boxel_normals, dim3((unsigned)blocks), dim3(256), 0, s, a, nteams);
    return hipGetLastError();
}

}  // namespace combo
