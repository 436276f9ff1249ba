// Point-to-point ICP fine registration of two clouds (Sec. 2.3: the clouds
// computed with Eq. 3 are registered by ICP starting from the estimated
// poses).
//
// Target cloud: a spatial hash of cells of edge dmax / 0.99 (counting sort of
// the points by bucket), so every target within dmax of a query lies in the
// 27 cells around the query's cell.  Per iteration:
//   1. correspondences: p' = R p + T and its nearest target within dmax in
//      FP32, every operation rounded on its own in a fixed order (ties to
//      the lowest target index), so the integer decision is reproducible;
//   2. FP64 sums over the accepted pairs (count, sums of p' and q, sum of
//      p' q^T, sum of squared distances), per block in a fixed order and
//      then over the blocks in a fixed order;
//   3. one thread: centroids and cross-covariance H, the optimal rotation by
//      Horn's quaternion method (largest eigenvector of the symmetric 4 x 4
//      matrix built from H, cyclic Jacobi in FP64), translation, composed
//      onto the pose (FP64), rounded to FP32 for the next correspondences.
// An iteration with fewer than 3 pairs leaves the pose unchanged.
#include <hip/hip_runtime.h>

#include "bp_internal.h"

namespace bpk {

constexpr int kIcpBlock = 256;
constexpr int kIcpSums = 17;     // n, sum p'(3), sum q(3), sum p' q^T (9), sum d2

struct IcpGrid {
    const uint32_t *start;       // [T + 1] first sorted slot of each bucket
    const uint32_t *order;       // [m] target indices sorted by bucket
    const float *dst;            // [m][3]
    uint32_t mask;               // T - 1
    float inv_cell;              // 1 / dmax
};

__device__ __forceinline__ uint32_t cell_hash(int ix, int iy, int iz, uint32_t mask)
{
    return (((uint32_t)ix * 73856093u) ^ ((uint32_t)iy * 19349663u) ^ ((uint32_t)iz * 83492791u)) & mask;
}

__device__ __forceinline__ int cell_of(float v, float inv_cell) { return (int)__builtin_floorf(v * inv_cell); }

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *p, uint32_t n, uint32_t v)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_icp_hist(const float *__restrict__ dst, int m, float inv_cell, uint32_t mask,
                                                 uint32_t *__restrict__ count)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const float *q = dst + (int64_t)j * 3;
    const uint32_t b = cell_hash(cell_of(q[0], inv_cell), cell_of(q[1], inv_cell), cell_of(q[2], inv_cell), mask);
    atomicAdd(&count[b], 1u);
}

// Exclusive scan of count[0..T) into start[0..T], one 1024-thread block:
// thread t scans a contiguous chunk, chunk totals are scanned in LDS.
__global__ void __launch_bounds__(1024) k_icp_scan(const uint32_t *__restrict__ count, uint32_t T,
                                                  uint32_t *__restrict__ start)
{
    __shared__ uint32_t tot[1024];
    const uint32_t t = threadIdx.x, per = (T + 1023) / 1024;
    const uint32_t b0 = t * per, b1 = b0 + per < T ? b0 + per : T;
    uint32_t s = 0;
    for (uint32_t b = b0; b < b1; ++b) s += count[b];
    tot[t] = s;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? tot[t - off] : 0u;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    uint32_t run = tot[t] - s;       // exclusive prefix of this chunk
    for (uint32_t b = b0; b < b1; ++b) {
        start[b] = run;
        run += count[b];
    }
    if (t == 1023) start[T] = tot[1023];
}

__global__ void __launch_bounds__(256) k_icp_scatter(const float *__restrict__ dst, int m, float inv_cell,
                                                    uint32_t mask, const uint32_t *__restrict__ start,
                                                    uint32_t *__restrict__ fill, uint32_t *__restrict__ order)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const float *q = dst + (int64_t)j * 3;
    const uint32_t b = cell_hash(cell_of(q[0], inv_cell), cell_of(q[1], inv_cell), cell_of(q[2], inv_cell), mask);
    order[start[b] + atomicAdd(&fill[b], 1u)] = (uint32_t)j;
}

// Correspondences of every source point; block partial sums in FP64.
__global__ void __launch_bounds__(kIcpBlock) k_icp_corr(const float *__restrict__ src, int n, IcpGrid g,
                                                       const float *__restrict__ pose_f, float dmax2,
                                                       int32_t *__restrict__ corr, double *__restrict__ partial)
{
#pragma clang fp contract(off)
    __shared__ double s_sum[kIcpSums][kIcpBlock];
    const int i = blockIdx.x * kIcpBlock + threadIdx.x;
    double acc[kIcpSums];
#pragma unroll
    for (int k = 0; k < kIcpSums; ++k) acc[k] = 0.0;
    if (i < n) {
        const float *p = src + (int64_t)i * 3;
        float q[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            float a = pose_f[r * 3 + 0] * p[0];
            a = a + pose_f[r * 3 + 1] * p[1];
            a = a + pose_f[r * 3 + 2] * p[2];
            q[r] = a + pose_f[9 + r];
        }
        const int cx = cell_of(q[0], g.inv_cell), cy = cell_of(q[1], g.inv_cell), cz = cell_of(q[2], g.inv_cell);
        int best = -1;
        float bd = 0.0f;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const uint32_t b = cell_hash(cx + dx, cy + dy, cz + dz, g.mask);
                    for (uint32_t s = g.start[b]; s < g.start[b + 1]; ++s) {
                        const int j = (int)g.order[s];
                        const float *t = g.dst + (int64_t)j * 3;
                        const float ex = q[0] - t[0], ey = q[1] - t[1], ez = q[2] - t[2];
                        float d = ex * ex;
                        d = d + ey * ey;
                        d = d + ez * ez;
                        if (d <= dmax2 && (best < 0 || d < bd || (d == bd && j < best))) {
                            best = j;
                            bd = d;
                        }
                    }
                }
        corr[i] = best;
        if (best >= 0) {
            const float *t = g.dst + (int64_t)best * 3;
            acc[0] = 1.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                acc[1 + a] = (double)q[a];
                acc[4 + a] = (double)t[a];
#pragma unroll
                for (int b = 0; b < 3; ++b) acc[7 + a * 3 + b] = (double)q[a] * (double)t[b];
            }
            acc[16] = (double)bd;
        }
    }
#pragma unroll
    for (int k = 0; k < kIcpSums; ++k) s_sum[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = kIcpBlock / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int k = 0; k < kIcpSums; ++k) s_sum[k][threadIdx.x] += s_sum[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < kIcpSums) partial[(int64_t)blockIdx.x * kIcpSums + threadIdx.x] = s_sum[threadIdx.x][0];
}

// Eigenvector of the largest eigenvalue of a symmetric 4 x 4 matrix (cyclic Jacobi).
__device__ void jacobi4(double A[4][4], double v[4])
{
    double V[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) off += A[p][q] * A[p][q];
        if (off < 1e-300) break;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) {
                if (A[p][q] == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 4; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 4; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 4; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int best = 0;
    for (int i = 1; i < 4; ++i)
        if (A[i][i] > A[best][best]) best = i;
    for (int k = 0; k < 4; ++k) v[k] = V[k][best];
}

// Sums the block partials (fixed order), solves the rigid update and
// composes it onto the pose.  pose: FP64 [12] (R row-major, T); pose_f: the
// same rounded to FP32.  One 256-thread block.
__global__ void __launch_bounds__(256) k_icp_update(const double *__restrict__ partial, int nblocks,
                                                   double *__restrict__ pose, float *__restrict__ pose_f, int it,
                                                   double *__restrict__ rms, int32_t *__restrict__ pairs)
{
    __shared__ double s[kIcpSums][256];
    double acc[kIcpSums];
    for (int k = 0; k < kIcpSums; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256)
        for (int k = 0; k < kIcpSums; ++k) acc[k] += partial[(int64_t)b * kIcpSums + k];
    for (int k = 0; k < kIcpSums; ++k) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < kIcpSums; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double n = s[0][0];
    if (rms) rms[it] = n > 0.0 ? sqrt(s[16][0] / n) : 0.0;
    if (pairs) pairs[it] = (int32_t)n;
    if (n < 3.0) return;
    double pc[3], qc[3], H[3][3];
    for (int a = 0; a < 3; ++a) {
        pc[a] = s[1 + a][0] / n;
        qc[a] = s[4 + a][0] / n;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) H[a][b] = s[7 + a * 3 + b][0] - n * pc[a] * qc[b];
    // Horn: N = [[tr, D^T], [D, H + H^T - tr I]], D = (H12 - H21, H20 - H02, H01 - H10).
    const double tr = H[0][0] + H[1][1] + H[2][2];
    double N[4][4];
    N[0][0] = tr;
    N[0][1] = N[1][0] = H[1][2] - H[2][1];
    N[0][2] = N[2][0] = H[2][0] - H[0][2];
    N[0][3] = N[3][0] = H[0][1] - H[1][0];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) N[1 + a][1 + b] = H[a][b] + H[b][a] - (a == b ? tr : 0.0);
    double qv[4];
    jacobi4(N, qv);
    const double w = qv[0], x = qv[1], y = qv[2], z = qv[3];
    const double nn = w * w + x * x + y * y + z * z;
    const double Ri[3][3] = {{(w * w + x * x - y * y - z * z) / nn, 2.0 * (x * y - w * z) / nn, 2.0 * (x * z + w * y) / nn},
                             {2.0 * (x * y + w * z) / nn, (w * w - x * x + y * y - z * z) / nn, 2.0 * (y * z - w * x) / nn},
                             {2.0 * (x * z - w * y) / nn, 2.0 * (y * z + w * x) / nn, (w * w - x * x - y * y + z * z) / nn}};
    double Ti[3];
    for (int a = 0; a < 3; ++a) Ti[a] = qc[a] - (Ri[a][0] * pc[0] + Ri[a][1] * pc[1] + Ri[a][2] * pc[2]);
    double R[3][3], T[3], Rn[3][3], Tn[3];
    for (int a = 0; a < 3; ++a) {
        T[a] = pose[9 + a];
        for (int b = 0; b < 3; ++b) R[a][b] = pose[a * 3 + b];
    }
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) Rn[a][b] = Ri[a][0] * R[0][b] + Ri[a][1] * R[1][b] + Ri[a][2] * R[2][b];
        Tn[a] = Ri[a][0] * T[0] + Ri[a][1] * T[1] + Ri[a][2] * T[2] + Ti[a];
    }
    for (int a = 0; a < 3; ++a) {
        pose[9 + a] = Tn[a];
        pose_f[9 + a] = (float)Tn[a];
        for (int b = 0; b < 3; ++b) {
            pose[a * 3 + b] = Rn[a][b];
            pose_f[a * 3 + b] = (float)Rn[a][b];
        }
    }
}

__global__ void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst, int n)
{
    const int k = threadIdx.x;
    if (k < n) dst[k] = src[k];
}

__global__ void k_icp_init(const double *__restrict__ pose_in, double *__restrict__ pose, float *__restrict__ pose_f)
{
    const int k = threadIdx.x;
    if (k < 12) {
        pose[k] = pose_in[k];
        pose_f[k] = (float)pose_in[k];
    }
}

static uint32_t icp_buckets(int m)
{
    uint32_t T = 1024;
    while (T < 2u * (uint32_t)m) T <<= 1;
    return T;
}

size_t icp_workspace_bytes(int n, int m)
{
    const uint32_t T = icp_buckets(m);
    const size_t nb = (size_t)((n + kIcpBlock - 1) / kIcpBlock);
    return align_up((size_t)(T + 1) * 4) * 2 + align_up((size_t)m * 4) + align_up(nb * kIcpSums * 8 + 8) +
           align_up(12 * 8) + align_up(12 * 4) + align_up((size_t)n * 4);
}

bp_status launch_icp(const float *src, int n, const float *dst, int m, const double *pose_in, int iters, float dmax,
                     double *pose_out, double *rms, int32_t *pairs, int32_t *corr_out, uint8_t *ws, hipStream_t st)
{
    const uint32_t T = icp_buckets(m);
    const int nb = (n + kIcpBlock - 1) / kIcpBlock;
    uint8_t *p = ws;
    uint32_t *count = (uint32_t *)p;
    p += align_up((size_t)(T + 1) * 4);
    uint32_t *start = (uint32_t *)p;
    p += align_up((size_t)(T + 1) * 4);
    uint32_t *order = (uint32_t *)p;
    p += align_up((size_t)m * 4);
    double *partial = (double *)p;
    p += align_up((size_t)nb * kIcpSums * 8 + 8);
    double *pose = (double *)p;
    p += align_up(12 * 8);
    float *pose_f = (float *)p;
    p += align_up(12 * 4);
    int32_t *corr = corr_out ? corr_out : (int32_t *)p;
    // Cells slightly larger than dmax (edge dmax / 0.99): a target within dmax
    // of a query then lies in the 27 cells around the query's cell despite the
    // rounding of the cell coordinates, for coordinates within about 8e4
    // cells of the origin.
    const float inv_cell = 0.99f / dmax;
    const float dmax2 = dmax * dmax;
    const unsigned gm = (unsigned)((m + 255) / 256);
    k_fill_u32<<<(T + 1 + 255) / 256, 256, 0, st>>>(count, T + 1, 0u);
    if (m > 0) k_icp_hist<<<gm, 256, 0, st>>>(dst, m, inv_cell, T - 1, count);
    k_icp_scan<<<1, 1024, 0, st>>>(count, T, start);
    k_fill_u32<<<(T + 1 + 255) / 256, 256, 0, st>>>(count, T + 1, 0u);
    if (m > 0) k_icp_scatter<<<gm, 256, 0, st>>>(dst, m, inv_cell, T - 1, start, count, order);
    k_icp_init<<<1, 64, 0, st>>>(pose_in, pose, pose_f);
    bp_status s = launch_status();
    const IcpGrid g{start, order, dst, T - 1, inv_cell};
    for (int it = 0; it < iters && s == BP_OK; ++it) {
        if (n > 0) k_icp_corr<<<nb, kIcpBlock, 0, st>>>(src, n, g, pose_f, dmax2, corr, partial);
        k_icp_update<<<1, 256, 0, st>>>(partial, n > 0 ? nb : 0, pose, pose_f, it, rms, pairs);
        s = launch_status();
    }
    if (s == BP_OK) {
        k_copy_f64<<<1, 64, 0, st>>>(pose, pose_out, 12);
        s = launch_status();
    }
    return s;
}

}  // namespace bpk
