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
// Pass 1 (one or four boxels per thread) streams the image once with dword or
// 16-byte loads and popcounts and writes c and phase.  Pass 2 compacts the
// composite boxels into an ordered list (block counts, one-workgroup scan, ordered
// write; N = 0 for the pure ones), then reduces the moments of each list entry
// with 16 lanes over its fine voxels and one-voxel periodic halo, and solves each
// entry's eigenproblem in a thread of its own.
#include <hip/hip_runtime.h>

#include "boxels.h"

namespace combo {

namespace {

constexpr int kTeam = 16;

__global__ void __launch_bounds__(256) k_boxel_zero(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
constexpr int kPer = 4;    // fine voxels per lane and load round in pass 2

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
    uint64_t pk[4] = {0, 0, 0, 0};
    // the four 0/1 bytes of a row dword as four bits
    auto nib = [](uint32_t v) -> uint64_t { return (v & 1u) | ((v >> 7) & 2u) | ((v >> 14) & 4u) | ((v >> 21) & 8u); };
#pragma unroll 8
    for (int r = 0; r < rows; ++r) {
        const int z = r / a.s2, y = r - z * a.s2;
        const uint4 v = *reinterpret_cast<const uint4*>(base + ((long long)z * a.N2 + y) * a.N1);
        bad |= (v.x | v.y | v.z | v.w) & 0xFEFEFEFEu;
        cnt[0] += __popc(v.x);
        cnt[1] += __popc(v.y);
        cnt[2] += __popc(v.z);
        cnt[3] += __popc(v.w);
        if (r < 16) {
            pk[0] |= nib(v.x) << (4 * r);
            pk[1] |= nib(v.y) << (4 * r);
            pk[2] |= nib(v.z) << (4 * r);
            pk[3] |= nib(v.w) << (4 * r);
        }
    }
    if (a.packed) {
        ulonglong2 p01, p23;
        p01.x = pk[0];
        p01.y = pk[1];
        p23.x = pk[2];
        p23.y = pk[3];
        *reinterpret_cast<ulonglong2*>(a.packed + b4) = p01;
        *reinterpret_cast<ulonglong2*>(a.packed + b4 + 2) = p23;
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
#pragma unroll
        for (int pq = 0; pq < 3; ++pq) {   // unrolled: p and q are constants, A and Q stay in registers
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            const double apq = A[p][q];
            if (!(fabs(apq) > 1e-17 * (fabs(A[p][p]) + fabs(A[q][q])))) continue;
            const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            // A <- J^T A J with J the rotation in the (p, q) plane
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double amp = A[m][p], amq = A[m][q];
                A[m][p] = c * amp - s * amq;
                A[m][q] = s * amp + c * amq;
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double apm = A[p][m], aqm = A[q][m];
                A[p][m] = c * apm - s * aqm;
                A[q][m] = s * apm + c * aqm;
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double qmp = Q[m][p], qmq = Q[m][q];
                Q[m][p] = c * qmp - s * qmq;
                Q[m][q] = s * qmp + c * qmq;
            }
        }
    }
    const bool m1 = A[1][1] < A[0][0];
    const double dmin01 = m1 ? A[1][1] : A[0][0];
    const bool m2 = A[2][2] < dmin01;
#pragma unroll
    for (int m = 0; m < 3; ++m) v[m] = m2 ? Q[m][2] : (m1 ? Q[m][1] : Q[m][0]);
    const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
    for (int m = 0; m < 3; ++m) v[m] /= nv;
}

template <typename X>
__device__ __forceinline__ X team_sum(X v) {
#pragma unroll
    for (int m = kTeam / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, kTeam);
    return v;
}

// Pass 2 works on a dense list of the composite boxels so that no lane idles:
//   k_boxel_blockcount: per block of kCompact boxels, the number of composites (and N = 0 for pure boxels);
//   k_boxel_scan:       one workgroup, exclusive prefix of the block counts and the total;
//   k_boxel_compact:    the composites of each block, in ascending order, into list[];
//   k_boxel_moments:    byte path: 16-lane teams per list entry, interface weights and moments -> mom[];
//   k_boxel_eigen:      byte path: one thread per list entry, the normal from its moments;
//   k_boxel_normals_packed: packed words: one lane per list entry, moments and normal together.
constexpr int kCompact = 1024;   // boxels per compaction block (256 threads x 4)
constexpr int kMom = 13;         // sw, sw xi (3), sw xi xi^T (6), sum_{chi=1} xi (3)

__global__ void __launch_bounds__(256) k_boxel_blockcount(BoxelArgs a, int* blockcnt) {
    __shared__ int red[4];
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    int cnt = 0;
    for (int q = 0; q < 4; ++q) {
        const long long b = (long long)blockIdx.x * kCompact + q * 256 + threadIdx.x;
        if (b >= nb) continue;
        if (a.phase[b] == 2) {
            ++cnt;
        } else {
            a.N[b] = 0.0;
            a.N[nb + b] = 0.0;
            a.N[2 * nb + b] = 0.0;
        }
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) blockcnt[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// exclusive prefix of nblk counts in place; total to counter[0]
__global__ void __launch_bounds__(1024) k_boxel_scan(int* blockcnt, int nblk, int* counter) {
    __shared__ int part[1024];
    const int per = (nblk + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(lo + per, nblk);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += blockcnt[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // Hillis-Steele inclusive scan of the 1024 partial sums
        const int v = (threadIdx.x >= off) ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = part[threadIdx.x] - s;             // exclusive start of this thread's range
    for (int i = lo; i < hi; ++i) {
        const int c = blockcnt[i];
        blockcnt[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) counter[0] = part[1023];
}

__global__ void __launch_bounds__(256) k_boxel_compact(BoxelArgs a, const int* blockoff, int* list) {
    __shared__ int wsum[4][4];
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long masks[4];
    for (int q = 0; q < 4; ++q) {
        const long long b = (long long)blockIdx.x * kCompact + q * 256 + threadIdx.x;
        masks[q] = __ballot(b < nb && a.phase[b] == 2);
        if (lane == 0) wsum[q][w] = __popcll(masks[q]);
    }
    __syncthreads();
    int base = blockoff[blockIdx.x];
    for (int q = 0; q < 4; ++q) {
        int before = 0;
        for (int ww = 0; ww < w; ++ww) before += wsum[q][ww];
        const long long b = (long long)blockIdx.x * kCompact + q * 256 + threadIdx.x;
        if ((masks[q] >> lane) & 1ull) list[base + before + __popcll(masks[q] & below)] = (int)b;
        base += wsum[q][0] + wsum[q][1] + wsum[q][2] + wsum[q][3];
    }
}

__global__ void __launch_bounds__(256) k_boxel_moments(BoxelArgs a, const int* list, double* mom, long long nteams) {
    const int tl = threadIdx.x % kTeam;
    const long long team = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kTeam;
    const int ncomp = a.counter[0];
    const int s1 = a.s1, s2 = a.s2, s3 = a.s3;
    const int V32 = s1 * s2 * s3;
    for (long long idx = team; idx < ncomp; idx += nteams) {   // uniform over the team
        const long long b = list[idx];
        const int i = (int)(b % a.n1);
        const long long tt = b / a.n1;
        const int j = (int)(tt % a.n2), k = (int)(tt / a.n2);
        double acc[kMom];
#pragma unroll
        for (int q = 0; q < kMom; ++q) acc[q] = 0.0;
        // kPer voxels per lane and round: all 7 kPer byte loads of a round are issued before
        // any is used, so a round costs one memory latency
        for (int t0 = tl; t0 < V32; t0 += kTeam * kPer) {
            int cv[kPer][7];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int t = t0 + u * kTeam;
                const bool ok = t < V32;
                const int tt2 = ok ? t : 0;
                const int uu = tt2 / s1;
                const int x = tt2 - uu * s1;
                const int z = uu / s2;
                const int y = uu - z * s2;
                const long long X = (long long)i * s1 + x, Y = (long long)j * s2 + y, Z = (long long)k * s3 + z;
                const uint8_t* plane = a.chi + Z * a.N2 * a.N1;
                const uint8_t* row = plane + Y * a.N1;
                cv[u][0] = ok ? row[X] : 0;
                cv[u][1] = ok ? row[wrap(X - 1, a.N1)] : 0;
                cv[u][2] = ok ? row[wrap(X + 1, a.N1)] : 0;
                cv[u][3] = ok ? plane[(long long)wrap(Y - 1, a.N2) * a.N1 + X] : 0;
                cv[u][4] = ok ? plane[(long long)wrap(Y + 1, a.N2) * a.N1 + X] : 0;
                cv[u][5] = ok ? a.chi[((long long)wrap(Z - 1, a.N3) * a.N2 + Y) * a.N1 + X] : 0;
                cv[u][6] = ok ? a.chi[((long long)wrap(Z + 1, a.N3) * a.N2 + Y) * a.N1 + X] : 0;
            }
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int t = t0 + u * kTeam;
                if (t >= V32) continue;
                const int uu = t / s1;
                const int x = t - uu * s1;
                const int z = uu / s2;
                const int y = uu - z * s2;
                const int c0 = cv[u][0];
                const int a1 = abs(cv[u][1] + cv[u][2] - 2 * c0), a2 = abs(cv[u][3] + cv[u][4] - 2 * c0),
                          a3 = abs(cv[u][5] + cv[u][6] - 2 * c0);
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
        }
#pragma unroll
        for (int q = 0; q < kMom; ++q) acc[q] = team_sum(acc[q]);
        // lane q of the team stores moment q
#pragma unroll
        for (int q = 0; q < kMom; ++q)
            if (tl == q) mom[idx * kMom + q] = acc[q];
    }
}

// the normal of a composite boxel from its 13 moments, written to N at boxel b
__device__ __forceinline__ void normal_from_moments(const BoxelArgs& a, long long b, const double* mm) {
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
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
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < 3; ++e) M[d][e] = 0.25 * a.h[d] * a.h[e] * (S[d][e] - sx[d] * sx[e] / sw);
        double v[3];
        smallest_eigvec(M, v);
        const double dot = nt[0] * v[0] + nt[1] * v[1] + nt[2] * v[2];
        const double sg = dot > 0 ? 1.0 : -1.0;
        for (int q = 0; q < 3; ++q) out[q] = sg * v[q];
    }
    a.N[b] = out[0];
    a.N[nb + b] = out[1];
    a.N[2 * nb + b] = out[2];
}

__global__ void __launch_bounds__(256) k_boxel_eigen(BoxelArgs a, const int* list, const double* mom) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.counter[0]) return;
    double mm[kMom];
#pragma unroll
    for (int q = 0; q < kMom; ++q) mm[q] = mom[idx * kMom + q];
    normal_from_moments(a, list[idx], mm);
}

// moments and normal from the packed boxel words (s1 = 4, s2 s3 <= 16), one composite per lane.  Fine
// voxel t = x + 4 (y + s2 z) is bit t of its boxel's word.  The lane reads the composite's word
// and those of its six face neighbours (periodic) and forms, with shifts and masks, the six
// words whose bit t is the neighbour of voxel t along -x, +x, -y, +y, -z, +z.  The stencil
// term of axis m at t is |chi(t - e_m) + chi(t + e_m) - 2 chi(t)|, i.e. the number of the two
// neighbours that differ from chi(t): bit t of (XM ^ W) plus bit t of (XP ^ W).  Only the
// voxels where some term is non-zero carry weight, and the lane visits just those bits.
__device__ __forceinline__ uint64_t shl64(uint64_t w, int k) { return k >= 64 ? 0ull : w << k; }
__device__ __forceinline__ uint64_t shr64(uint64_t w, int k) { return k >= 64 ? 0ull : w >> k; }
__device__ __forceinline__ int bitv(uint64_t w, int i) { return (int)((w >> i) & 1ull); }

__global__ void __launch_bounds__(256) k_boxel_normals_packed(BoxelArgs a, const int* list) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.counter[0]) return;
    const int s2 = a.s2, s3 = a.s3;
    const int V32 = 4 * s2 * s3;
    const int n1 = a.n1, n2 = a.n2, n3 = a.n3;
    const long long b = list[idx];
    const int i = (int)(b % n1);
    const long long tt = b / n1;
    const int j = (int)(tt % n2), k = (int)(tt / n2);
    const long long rowb = (long long)k * n2 + j;
    const uint64_t w0 = a.packed[b];
    const uint64_t wxm = a.packed[rowb * n1 + (i == 0 ? n1 - 1 : i - 1)];
    const uint64_t wxp = a.packed[rowb * n1 + (i == n1 - 1 ? 0 : i + 1)];
    const uint64_t wym = a.packed[((long long)k * n2 + (j == 0 ? n2 - 1 : j - 1)) * n1 + i];
    const uint64_t wyp = a.packed[((long long)k * n2 + (j == n2 - 1 ? 0 : j + 1)) * n1 + i];
    const uint64_t wzm = a.packed[((long long)(k == 0 ? n3 - 1 : k - 1) * n2 + j) * n1 + i];
    const uint64_t wzp = a.packed[((long long)(k == n3 - 1 ? 0 : k + 1) * n2 + j) * n1 + i];
    // masks of the voxels with x = 0, x = 3, y = 0, y = s2 - 1, z = 0, z = s3 - 1
    const uint64_t vm = V32 >= 64 ? ~0ull : ((1ull << V32) - 1ull);
    const uint64_t mx0 = 0x1111111111111111ull & vm, mx3 = mx0 << 3;
    uint64_t my0 = 0;
    for (int z = 0; z < s3; ++z) my0 |= 0xFull << (4 * s2 * z);
    const uint64_t myl = my0 << (4 * (s2 - 1));
    const int pz = 4 * s2;                       // bits per z plane
    const uint64_t mz0 = pz >= 64 ? ~0ull : ((1ull << pz) - 1ull);
    const uint64_t mzl = shl64(mz0, pz * (s3 - 1));
    const uint64_t XM = ((w0 << 1) & ~mx0) | ((wxm >> 3) & mx0);
    const uint64_t XP = ((w0 >> 1) & ~mx3) | ((wxp << 3) & mx3);
    const uint64_t YM = ((w0 << 4) & ~my0) | (shr64(wym, 4 * (s2 - 1)) & my0);
    const uint64_t YP = ((w0 >> 4) & ~myl) | (shl64(wyp, 4 * (s2 - 1)) & myl);
    const uint64_t ZM = (shl64(w0, pz) & ~mz0) | (shr64(wzm, pz * (s3 - 1)) & mz0);
    const uint64_t ZP = (shr64(w0, pz) & ~mzl) | (shl64(wzp, pz * (s3 - 1)) & mzl);
    const uint64_t d1a = XM ^ w0, d1b = XP ^ w0, d2a = YM ^ w0, d2b = YP ^ w0, d3a = ZM ^ w0, d3b = ZP ^ w0;
    const unsigned inv2 = (65536u + (unsigned)s2 - 1u) / (unsigned)s2;   // r / s2 = (r inv2) >> 16 for r < 16
    double acc[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] = 0.0;
    for (uint64_t m = (d1a | d1b | d2a | d2b | d3a | d3b) & vm; m; m &= m - 1ull) {
        const int t = __builtin_ctzll(m);
        const int x = t & 3, r = t >> 2;
        const int z = (int)(((unsigned)r * inv2) >> 16), y = r - z * s2;
        const int a1 = bitv(d1a, t) + bitv(d1b, t), a2 = bitv(d2a, t) + bitv(d2b, t), a3 = bitv(d3a, t) + bitv(d3b, t);
        const double xi0 = 2 * x - 3, xi1 = 2 * y + 1 - s2, xi2 = 2 * z + 1 - s3;
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
    // sums of xi over the inclusion voxels (integers): popcounts of the word under the masks of
    // equal x, equal y and equal z
    const uint64_t win = w0 & vm;
    int c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
    for (int x = 0; x < 4; ++x) c0 += (2 * x - 3) * __popcll(win & (mx0 << x));
    for (int y = 0; y < s2; ++y) c1 += (2 * y + 1 - s2) * __popcll(win & (my0 << (4 * y)));
    for (int z = 0; z < s3; ++z) c2 += (2 * z + 1 - s3) * __popcll(win & shl64(mz0, pz * z));
    double mm[kMom];
#pragma unroll
    for (int q = 0; q < 10; ++q) mm[q] = acc[q];
    mm[10] = c0;
    mm[11] = c1;
    mm[12] = c2;
    normal_from_moments(a, b, mm);
}

}  // namespace

hipError_t launch_boxel_zero(int* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_boxel_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

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

int boxel_blocks(long long nb) { return (int)((nb + kCompact - 1) / kCompact); }

hipError_t launch_boxel_list(const BoxelArgs& a, int* blockcnt, int* list, hipStream_t s) {
    const long long nb = (long long)a.n1 * a.n2 * a.n3;
    const int nblk = boxel_blocks(nb);
    hipLaunchKernelGGL(k_boxel_blockcount, dim3(nblk), dim3(256), 0, s, a, blockcnt);
    hipLaunchKernelGGL(k_boxel_scan, dim3(1), dim3(1024), 0, s, blockcnt, nblk, a.counter);
    hipLaunchKernelGGL(k_boxel_compact, dim3(nblk), dim3(256), 0, s, a, (const int*)blockcnt, list);
    return hipGetLastError();
}

hipError_t launch_block_scan(int* cnt, int nblk, int* total, hipStream_t s) {
    hipLaunchKernelGGL(k_boxel_scan, dim3(1), dim3(1024), 0, s, cnt, nblk, total);
    return hipGetLastError();
}

hipError_t launch_boxel_normals(const BoxelArgs& a, const int* list, double* mom, int ncomp, hipStream_t s) {
    if (ncomp <= 0) return hipSuccess;
    if (a.packed) {
        hipLaunchKernelGGL(k_boxel_normals_packed, dim3((unsigned)((ncomp + 255) / 256)), dim3(256), 0, s, a, list);
        return hipGetLastError();
    }
    const long long blocks = std::min<long long>(((long long)ncomp * kTeam + 255) / 256, 65536);
    const long long nteams = blocks * 256 / kTeam;
    hipLaunchKernelGGL(k_boxel_moments, dim3((unsigned)blocks), dim3(256), 0, s, a, list, mom, nteams);
    hipLaunchKernelGGL(k_boxel_eigen, dim3((unsigned)((ncomp + 255) / 256)), dim3(256), 0, s, a, list,
                       (const double*)mom);
    return hipGetLastError();
}

}  // namespace combo
