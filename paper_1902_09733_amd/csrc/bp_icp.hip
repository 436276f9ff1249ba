// Point-to-point ICP fine registration of two clouds (Sec. 2.3: the clouds
// computed with Eq. 3 are registered by ICP starting from the estimated
// poses).
//
// Both clouds are counting-sorted by the cell (edge dmax / 0.99) they fall
// in, into float4 records {x, y, z, index}, so every target within dmax of a
// query lies in the 27 cells around the query's cell.  Buckets are cell
// coordinates relative to the target's bounding box, wrapped to the bits a
// table of T buckets allows, with z fastest, then x, then y: the three
// z-neighbours of a column are adjacent buckets (for terrain, a column holds
// all its points) and queries taken in bucket order sweep the surface in
// raster order, so neighbouring wavefronts share cells in cache.  Cells that
// wrap onto the same bucket only add candidates.  Per iteration:
//   1. correspondences (queries in sorted order): p' = R p + T and its
//      nearest target within dmax in FP32, every operation rounded on its own
//      in a fixed order (ties to the lowest target index).  A neighbour cell
//      is skipped when a lower bound of its distance, reduced by a margin
//      that covers every rounding involved, already exceeds the best squared
//      distance found (or dmax^2), so the pairing equals the exhaustive one;
//   2. FP64 sums over the accepted pairs (count, sums of p' and q, sum of
//      p' q^T, sum of squared distances) in source-index order: per block in
//      a fixed shuffle tree, then over the blocks in a fixed order, so the
//      sums do not depend on the order the sort produced;
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

// Bucket of a cell: ((z - oz) & mz) | ((x - ox) & mx) << sx | ((y - oy) & my) << sy.
struct IcpHash {
    int ox, oy, oz;
    uint32_t mx, my, mz, sx, sy;
};

struct IcpGrid {
    const uint32_t *start;       // [T + 1] first record of each bucket
    const float4 *rec;           // [m] targets {x, y, z, index bits} sorted by bucket
    const IcpHash *hash;
    float inv_cell;              // 0.99 / dmax
    float cell;                  // 1 / inv_cell
};

__device__ __forceinline__ uint32_t cell_bucket(const IcpHash &h, int ix, int iy, int iz)
{
    return (((uint32_t)iz - (uint32_t)h.oz) & h.mz) | ((((uint32_t)ix - (uint32_t)h.ox) & h.mx) << h.sx) |
           ((((uint32_t)iy - (uint32_t)h.oy) & h.my) << h.sy);
}

// Integer cell of a floored coordinate, clamped to +-2^30 so that huge or
// non-finite coordinates (NaN clamps to -2^30) still convert to a defined
// integer; such points never pair anyway (their distances are not <= dmax^2).
__device__ __forceinline__ int cell_index(float fl)
{
    return (int)__builtin_fminf(__builtin_fmaxf(fl, -0x1p30f), 0x1p30f);
}

__device__ __forceinline__ int cell_of(float v, float inv_cell) { return cell_index(__builtin_floorf(v * inv_cell)); }

__device__ __forceinline__ uint32_t bucket_of(const IcpHash &h, float x, float y, float z, float inv_cell)
{
    return cell_bucket(h, cell_of(x, inv_cell), cell_of(y, inv_cell), cell_of(z, inv_cell));
}

// p' = R p + T in FP32, each product and sum rounded on its own, in row order.
__device__ __forceinline__ void icp_move(const float *__restrict__ P, float x, float y, float z, float q[3])
{
#pragma clang fp contract(off)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        float a = P[r * 3 + 0] * x;
        a = a + P[r * 3 + 1] * y;
        a = a + P[r * 3 + 2] * z;
        q[r] = a + P[9 + r];
    }
}

__device__ __forceinline__ float icp_dist2(const float q[3], float tx, float ty, float tz)
{
#pragma clang fp contract(off)
    const float ex = q[0] - tx, ey = q[1] - ty, ez = q[2] - tz;
    float d = ex * ex;
    d = d + ey * ey;
    return d + ez * ez;
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *p, uint32_t n, uint32_t v)
{
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// Bounding box of the cells of pts, per block: part[block][0..2] min,
// part[block][3..5] max (INT_MAX / INT_MIN for a block without points).
constexpr int kBoxBlocks = 256;

__global__ void __launch_bounds__(256) k_icp_bbox(const float *__restrict__ pts, int m, float inv_cell,
                                                 int *__restrict__ part)
{
    __shared__ int s_box[4][6];
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
    for (int j = blockIdx.x * 256 + threadIdx.x; j < m; j += gridDim.x * 256) {
        const float *q = pts + (int64_t)j * 3;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int v = cell_of(q[a], inv_cell);
            lo[a] = min(lo[a], v);
            hi[a] = max(hi[a], v);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = max(hi[a], __shfl_xor(hi[a], o, 64));
        }
    const int w = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            s_box[w][a] = lo[a];
            s_box[w][3 + a] = hi[a];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        int v = s_box[0][threadIdx.x];
        for (int k = 1; k < 4; ++k) v = threadIdx.x < 3 ? min(v, s_box[k][threadIdx.x]) : max(v, s_box[k][threadIdx.x]);
        part[blockIdx.x * 6 + threadIdx.x] = v;
    }
}

__host__ __device__ static inline uint32_t ceil_log2(uint64_t v)
{
    uint32_t b = 0;
    while (((uint64_t)1 << b) < v) ++b;
    return b;
}

// Bucket mapping from the bounding box: one cell of margin on each side, as
// many bits per axis as the extent needs while they fit in log2(T), the
// widest axes cut first when they do not.
__global__ void __launch_bounds__(64) k_icp_hash(const int *__restrict__ part, int nparts, uint32_t log2T,
                                                IcpHash *__restrict__ h)
{
    int box[6];
    for (int a = 0; a < 6; ++a) {
        int v = a < 3 ? INT_MAX : INT_MIN;
        for (int b = threadIdx.x; b < nparts; b += 64) v = a < 3 ? min(v, part[b * 6 + a]) : max(v, part[b * 6 + a]);
        for (int o = 32; o >= 1; o >>= 1) v = a < 3 ? min(v, __shfl_xor(v, o, 64)) : max(v, __shfl_xor(v, o, 64));
        box[a] = v;
    }
    if (threadIdx.x != 0) return;
    int64_t org[3] = {0, 0, 0};
    uint32_t bits[3] = {log2T / 2, log2T - log2T / 2, 0};          // x, y, z for an empty cloud
    if (box[0] <= box[3]) {
        for (int a = 0; a < 3; ++a) {
            org[a] = (int64_t)box[a] - 1;
            bits[a] = ceil_log2((uint64_t)((int64_t)box[3 + a] - (int64_t)box[a] + 3));
        }
        while (bits[0] + bits[1] + bits[2] > log2T) {
            int w = 2;
            if (bits[0] > bits[w]) w = 0;
            if (bits[1] > bits[w]) w = 1;
            --bits[w];
        }
    }
    IcpHash r;
    r.ox = (int)(uint32_t)org[0];
    r.oy = (int)(uint32_t)org[1];
    r.oz = (int)(uint32_t)org[2];
    r.mx = (1u << bits[0]) - 1u;
    r.my = (1u << bits[1]) - 1u;
    r.mz = (1u << bits[2]) - 1u;
    r.sx = bits[2];
    r.sy = bits[2] + bits[0];
    *h = r;
}

__global__ void __launch_bounds__(256) k_icp_hist(const float *__restrict__ pts, int m, float inv_cell,
                                                 const IcpHash *__restrict__ hp, uint32_t *__restrict__ count)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const IcpHash h = *hp;
    const float *q = pts + (int64_t)j * 3;
    atomicAdd(&count[bucket_of(h, q[0], q[1], q[2], inv_cell)], 1u);
}

// Exclusive scan of count[0..T) into start[0..T] (T a power of two >= 1024)
// in three passes: 1024-entry tiles scanned in LDS with their totals in
// tile[], the tile totals scanned by one block, the tile offsets added.
__device__ __forceinline__ uint32_t block_scan_256(uint32_t v, uint32_t *lds)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t u = t >= off ? lds[t - off] : 0u;
        __syncthreads();
        lds[t] += u;
        __syncthreads();
    }
    return lds[t];              // inclusive
}

__global__ void __launch_bounds__(256) k_icp_scan_tiles(const uint32_t *__restrict__ count,
                                                       uint32_t *__restrict__ start, uint32_t *__restrict__ tile)
{
    __shared__ uint32_t lds[256];
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x * 4;
    const uint4 c = *(const uint4 *)(count + base);
    const uint32_t own = c.x + c.y + c.z + c.w;
    const uint32_t incl = block_scan_256(own, lds);
    uint32_t run = incl - own;
    *(uint4 *)(start + base) = make_uint4(run, run + c.x, run + c.x + c.y, run + c.x + c.y + c.z);
    if (threadIdx.x == 255) tile[blockIdx.x] = incl;
}

// Exclusive scan of tile[0..nt) in place, 256 entries per round; total -> *total.
__global__ void __launch_bounds__(256) k_icp_scan_top(uint32_t *__restrict__ tile, uint32_t nt,
                                                     uint32_t *__restrict__ total)
{
    __shared__ uint32_t lds[256];
    uint32_t carry = 0;
    for (uint32_t r = 0; r < nt; r += 256) {
        const uint32_t i = r + threadIdx.x;
        const uint32_t v = i < nt ? tile[i] : 0u;
        const uint32_t incl = block_scan_256(v, lds);
        if (i < nt) tile[i] = carry + incl - v;
        carry += lds[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(256) k_icp_scan_add(uint32_t *__restrict__ start, const uint32_t *__restrict__ tile)
{
    const size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x * 4;
    uint4 v = *(uint4 *)(start + base);
    const uint32_t o = tile[blockIdx.x];
    *(uint4 *)(start + base) = make_uint4(v.x + o, v.y + o, v.z + o, v.w + o);
}

// Records in bucket order (the order inside a bucket is whatever the atomics
// give; nothing computed from the records depends on it).
__global__ void __launch_bounds__(256) k_icp_scatter(const float *__restrict__ pts, int m, float inv_cell,
                                                    const IcpHash *__restrict__ hp, const uint32_t *__restrict__ start,
                                                    uint32_t *__restrict__ fill, float4 *__restrict__ rec)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const IcpHash h = *hp;
    const float *q = pts + (int64_t)j * 3;
    const uint32_t b = bucket_of(h, q[0], q[1], q[2], inv_cell);
    rec[start[b] + atomicAdd(&fill[b], 1u)] = make_float4(q[0], q[1], q[2], __int_as_float(j));
}

// Nearest target within dmax of every source point, queries taken in the
// sorted record order; corr is written at the source index.
__global__ void __launch_bounds__(kIcpBlock) k_icp_corr(const float4 *__restrict__ qrec, int n, IcpGrid g,
                                                       const float *__restrict__ pose_f, float dmax2,
                                                       int32_t *__restrict__ corr)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kIcpBlock + threadIdx.x;
    if (i >= n) return;
    const float4 r = qrec[i];
    float q[3];
    icp_move(pose_f, r.x, r.y, r.z, q);
    // Cell coordinates and, per axis, lower bounds of the distance to the
    // cells below (lo) and above (hi).  frac(v * inv) is exact; the margin
    // covers the rounding of v * inv on both sides of a cell boundary, of
    // cell vs 1 / inv, and of the products below (relative 2^-22 per cell
    // of coordinate magnitude, against errors of at most about 2^-24).
    int c[3];
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float sv = q[a] * g.inv_cell;
        const float fl = __builtin_floorf(sv);
        const float fr = sv - fl;
        c[a] = cell_index(fl);
        const float margin = (__builtin_fabsf(fl) + 4.0f) * (g.cell * 0x1p-22f);
        lo[a] = __builtin_fmaxf(fr * g.cell - margin, 0.0f);
        hi[a] = __builtin_fmaxf((1.0f - fr) * g.cell - margin, 0.0f);
    }
    const IcpHash h = *g.hash;
    int best = -1;
    float bd = 0.0f;
    auto test = [&](const float4 t) {
        const float d = icp_dist2(q, t.x, t.y, t.z);
        const int j = __float_as_int(t.w);
        if (d <= dmax2 && (best < 0 || d < bd || (d == bd && j < best))) {
            best = j;
            bd = d;
        }
    };
    // Records [s, e) in groups of four independent loads; in the last group
    // the loads past e re-read record e - 1 and stand for an infinitely far
    // point (never accepted).
    auto scan = [&](uint32_t s, uint32_t e) {
        const float4 far = make_float4(__builtin_inff(), __builtin_inff(), __builtin_inff(), 0.0f);
        for (; s < e; s += 4) {
            const uint32_t l = e - 1;
            float4 t[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) t[u] = g.rec[s + u < e ? s + u : l];
#pragma unroll
            for (int u = 0; u < 4; ++u) test(s + u < e ? t[u] : far);
        }
    };
    const float shrink = 1.0f - 0x1p-19f;
    // Columns (x, y offsets), own one first so the best distance shrinks
    // early.  The three z cells of a column are adjacent buckets unless the z
    // coordinate wraps; then they are one record range, trimmed at either end
    // when that z neighbour is out of reach.
#pragma unroll 1
    for (int k = 0; k < 9; ++k) {
        const int oy = k / 3, ox = k % 3;                             // 0, 1, 2 -> offsets 0, -1, +1
        const float lx = ox == 0 ? 0.0f : (ox == 1 ? lo[0] : hi[0]);
        const float ly = oy == 0 ? 0.0f : (oy == 1 ? lo[1] : hi[1]);
        float lxy = lx * lx;
        lxy = lxy + ly * ly;
        if (lxy * shrink > (best < 0 ? dmax2 : bd)) continue;
        const int x = c[0] + (ox == 2 ? 1 : -(ox == 1)), y = c[1] + (oy == 2 ? 1 : -(oy == 1));
        const uint32_t b0 = cell_bucket(h, x, y, c[2]), bm = cell_bucket(h, x, y, c[2] - 1),
                       bp = cell_bucket(h, x, y, c[2] + 1);
        const float lbm = (lxy + lo[2] * lo[2]) * shrink, lbp = (lxy + hi[2] * hi[2]) * shrink;
        if (bm + 1 == b0 && b0 + 1 == bp) {
            const uint32_t a0 = g.start[bm], a1 = g.start[b0], a2 = g.start[bp], a3 = g.start[bp + 1];
            const float thr = best < 0 ? dmax2 : bd;
            scan(lbm > thr ? a1 : a0, lbp > thr ? a2 : a3);
        } else {
            scan(g.start[b0], g.start[b0 + 1]);
            // Wrapped z cells may share a bucket (with one z bit or none): scan each bucket once.
            bool did_m = false;
            if (bm != b0 && !(lbm > (best < 0 ? dmax2 : bd))) {
                scan(g.start[bm], g.start[bm + 1]);
                did_m = true;
            }
            if (bp != b0 && !(bp == bm && did_m) && !(lbp > (best < 0 ? dmax2 : bd)))
                scan(g.start[bp], g.start[bp + 1]);
        }
    }
    corr[__float_as_int(r.w)] = best;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kSumsPerThread = 4;
constexpr int kSumsChunk = kIcpBlock * kSumsPerThread;   // source points per block of k_icp_sums

// Block-wide FP64 sum of one value per thread in a fixed order (shuffle tree
// per wavefront, then the four wavefront sums in order); valid in thread 0.
__device__ __forceinline__ void block_sums(const double (&acc)[kIcpSums], double (*lds)[kIcpSums],
                                           double (&out)[kIcpSums])
{
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int k = 0; k < kIcpSums; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) lds[w][k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kIcpSums; ++k) {
        double v = lds[0][k];
#pragma unroll
        for (int q = 1; q < kIcpBlock / 64; ++q) v += lds[q][k];
        out[k] = v;
    }
}

__device__ void icp_solve(const double (&s)[kIcpSums], double *pose, float *pose_f, int it, double *rms,
                          int32_t *pairs);

// Sums of the partials of nblocks blocks (fixed order: thread t takes blocks
// t, t + 256, ..., then the block tree), then the rigid update by thread 0.
__device__ void icp_finish(const double *partial, int nblocks, double (*lds)[kIcpSums], double *pose, float *pose_f,
                           int it, double *rms, int32_t *pairs)
{
    double acc[kIcpSums], tot[kIcpSums];
#pragma unroll
    for (int k = 0; k < kIcpSums; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kIcpBlock)
#pragma unroll
        for (int k = 0; k < kIcpSums; ++k)
            acc[k] += partial[(int64_t)b * kIcpSums + k];
    __syncthreads();
    block_sums(acc, lds, tot);
    if (threadIdx.x == 0) icp_solve(tot, pose, pose_f, it, rms, pairs);
}

// FP64 sums over the pairs in source-index order, kSumsPerThread points per
// thread, one partial per block.
__global__ void __launch_bounds__(kIcpBlock) k_icp_sums(const float *__restrict__ src, int n,
                                                       const float *__restrict__ dst, const int32_t *__restrict__ corr,
                                                       const float *__restrict__ pose_f, double *__restrict__ partial)
{
    __shared__ double lds[kIcpBlock / 64][kIcpSums];
    double acc[kIcpSums];
#pragma unroll
    for (int k = 0; k < kIcpSums; ++k) acc[k] = 0.0;
    float P[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) P[k] = pose_f[k];
#pragma unroll
    for (int u = 0; u < kSumsPerThread; ++u) {
        const int i = blockIdx.x * kSumsChunk + u * kIcpBlock + threadIdx.x;
        const int j = i < n ? corr[i] : -1;
        if (j >= 0) {
            const float *p = src + (int64_t)i * 3;
            const float *t = dst + (int64_t)j * 3;
            float q[3];
            icp_move(P, p[0], p[1], p[2], q);
            const float t0 = t[0], t1 = t[1], t2 = t[2];
            const double tq[3] = {(double)t0, (double)t1, (double)t2};
            acc[0] += 1.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                acc[1 + a] += (double)q[a];
                acc[4 + a] += tq[a];
#pragma unroll
                for (int b = 0; b < 3; ++b) acc[7 + a * 3 + b] += (double)q[a] * tq[b];
            }
            acc[16] += (double)icp_dist2(q, t0, t1, t2);
        }
    }
    double tot[kIcpSums];
    block_sums(acc, lds, tot);
    if (threadIdx.x < kIcpSums) partial[(int64_t)blockIdx.x * kIcpSums + threadIdx.x] = tot[threadIdx.x];
}

// Eigenvector of the largest eigenvalue of a symmetric 4 x 4 matrix (cyclic Jacobi).
__device__ void jacobi4(double A[4][4], double v[4])
{
    double V[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < 4; ++p) {
            diag += A[p][p] * A[p][p];
            for (int q = p + 1; q < 4; ++q) off += A[p][q] * A[p][q];
        }
        // Off-diagonal entries below 1e-17 of the matrix norm: converged.
        if (off <= 1e-34 * (diag + off)) break;
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

__device__ __forceinline__ double det3(double a, double b, double c, double d, double e, double f, double g, double h,
                                       double i)
{
    return a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
}

// Determinant of M without row r and column c.
__device__ __forceinline__ double minor4(const double M[4][4], int r, int c)
{
    double m[9];
    int k = 0;
    for (int i = 0; i < 4; ++i)
        if (i != r)
            for (int j = 0; j < 4; ++j)
                if (j != c) m[k++] = M[i][j];
    return det3(m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7], m[8]);
}

// Eigenvector of the largest eigenvalue of Horn's traceless symmetric 4 x 4
// matrix N built from H.  Its characteristic polynomial is
// x^4 + c2 x^2 + c1 x + c0 with c2 = -tr(N^2) / 2, c1 = -8 det(H), c0 =
// det(N); Newton's method from the upper bound sqrt(3 tr(N^2) / 4) (at
// least the sum of the singular values of H) descends monotonically onto the
// largest root, where the polynomial is convex.  The eigenvector is then the
// row of adj(N - x I) through its largest diagonal entry.  When that entry is
// tiny against |N|^3 (a repeated or nearly repeated top eigenvalue), cyclic
// Jacobi takes over.
__device__ void horn_eigvec(double N[4][4], const double H[3][3], double v[4])
{
    double p2 = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) p2 += N[i][j] * N[i][j];
    if (p2 > 0.0) {
        const double c2 = -0.5 * p2;
        const double c1 = -8.0 * det3(H[0][0], H[0][1], H[0][2], H[1][0], H[1][1], H[1][2], H[2][0], H[2][1], H[2][2]);
        const double c0 = N[0][0] * minor4(N, 0, 0) - N[0][1] * minor4(N, 0, 1) + N[0][2] * minor4(N, 0, 2) -
                          N[0][3] * minor4(N, 0, 3);
        double x = sqrt(0.75 * p2);
        for (int k = 0; k < 100; ++k) {
            const double P = ((x * x + c2) * x + c1) * x + c0;
            const double dP = (4.0 * x * x + 2.0 * c2) * x + c1;
            if (!(dP > 0.0)) break;
            const double step = P / dP;
            x -= step;
            if (fabs(step) <= 1e-15 * fabs(x)) break;
        }
        double M[4][4];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) M[i][j] = N[i][j] - (i == j ? x : 0.0);
        int r = 0;
        double cr = fabs(minor4(M, 0, 0));
        for (int i = 1; i < 4; ++i) {
            const double ci = fabs(minor4(M, i, i));
            if (ci > cr) {
                cr = ci;
                r = i;
            }
        }
        if (cr > 1e-6 * p2 * sqrt(p2)) {
            for (int j = 0; j < 4; ++j) v[j] = ((r + j) & 1 ? -1.0 : 1.0) * minor4(M, r, j);
            return;
        }
    }
    jacobi4(N, v);
}

// The rigid update from the pair sums s, composed onto the pose.  pose:
// FP64 [12] (R row-major, T); pose_f: the same rounded to FP32.  One thread.
__device__ void icp_solve(const double (&s)[kIcpSums], double *pose, float *pose_f, int it, double *rms,
                          int32_t *pairs)
{
    const double n = s[0];
    if (rms) rms[it] = n > 0.0 ? sqrt(s[16] / n) : 0.0;
    if (pairs) pairs[it] = (int32_t)n;
    if (n < 3.0) return;
    double pc[3], qc[3], H[3][3];
    for (int a = 0; a < 3; ++a) {
        pc[a] = s[1 + a] / n;
        qc[a] = s[4 + a] / n;
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) H[a][b] = s[7 + a * 3 + b] - n * pc[a] * qc[b];
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
    horn_eigvec(N, H, qv);
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

// Adds up the block partials and updates the pose (one block).
__global__ void __launch_bounds__(kIcpBlock) k_icp_update(const double *__restrict__ partial, int nblocks,
                                                         double *__restrict__ pose, float *__restrict__ pose_f, int it,
                                                         double *__restrict__ rms, int32_t *__restrict__ pairs)
{
    __shared__ double lds[kIcpBlock / 64][kIcpSums];
    icp_finish(partial, nblocks, lds, pose, pose_f, it, rms, pairs);
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
    const uint32_t T = icp_buckets(n > m ? n : m);
    const size_t nb = (size_t)((n + kIcpBlock - 1) / kIcpBlock);
    return align_up((size_t)(T + 1) * 4) * 2 + align_up((size_t)(T / 1024) * 4) + align_up((size_t)m * 16) +
           align_up((size_t)n * 16) +
           align_up(nb * kIcpSums * 8 + 8) + align_up(12 * 8) + align_up(12 * 4) + align_up(kBoxBlocks * 6 * 4) +
           align_up(sizeof(IcpHash)) + align_up((size_t)n * 4);
}

// Counting sort of pts into bucket-ordered records; start[0..T] is left with
// the bucket offsets.
static void icp_sort(const float *pts, int k, float inv_cell, const IcpHash *hash, uint32_t T, uint32_t *count,
                     uint32_t *start, uint32_t *tile, float4 *rec, hipStream_t st)
{
    const unsigned gk = (unsigned)((k + 255) / 256), gt = (T + 1 + 255) / 256;
    k_fill_u32<<<gt, 256, 0, st>>>(count, T + 1, 0u);
    if (k > 0) k_icp_hist<<<gk, 256, 0, st>>>(pts, k, inv_cell, hash, count);
    k_icp_scan_tiles<<<T / 1024, 256, 0, st>>>(count, start, tile);
    k_icp_scan_top<<<1, 256, 0, st>>>(tile, T / 1024, start + T);
    k_icp_scan_add<<<T / 1024, 256, 0, st>>>(start, tile);
    k_fill_u32<<<gt, 256, 0, st>>>(count, T + 1, 0u);
    if (k > 0) k_icp_scatter<<<gk, 256, 0, st>>>(pts, k, inv_cell, hash, start, count, rec);
}

bp_status launch_icp(const float *src, int n, const float *dst, int m, const double *pose_in, int iters, float dmax,
                     double *pose_out, double *rms, int32_t *pairs, int32_t *corr_out, uint8_t *ws, hipStream_t st)
{
    const uint32_t T = icp_buckets(n > m ? n : m);
    const int nb = (n + kIcpBlock - 1) / kIcpBlock;
    uint8_t *p = ws;
    uint32_t *count = (uint32_t *)p;
    p += align_up((size_t)(T + 1) * 4);
    uint32_t *start = (uint32_t *)p;
    p += align_up((size_t)(T + 1) * 4);
    uint32_t *tile = (uint32_t *)p;
    p += align_up((size_t)(T / 1024) * 4);
    float4 *rec_dst = (float4 *)p;
    p += align_up((size_t)m * 16);
    float4 *rec_src = (float4 *)p;
    p += align_up((size_t)n * 16);
    double *partial = (double *)p;
    p += align_up((size_t)nb * kIcpSums * 8 + 8);
    double *pose = (double *)p;
    p += align_up(12 * 8);
    float *pose_f = (float *)p;
    p += align_up(12 * 4);
    int *box = (int *)p;
    p += align_up(kBoxBlocks * 6 * 4);
    IcpHash *hash = (IcpHash *)p;
    p += align_up(sizeof(IcpHash));
    int32_t *corr = corr_out ? corr_out : (int32_t *)p;
    // Cells slightly larger than dmax (edge dmax / 0.99): a target within dmax
    // of a query then lies in the 27 cells around the query's cell despite the
    // rounding of the cell coordinates, for coordinates within about 8e4
    // cells of the origin.
    const float inv_cell = 0.99f / dmax;
    const float dmax2 = dmax * dmax;
    // The source order only serves locality; the target offsets must be the
    // ones left in start, so the source is sorted first.
    uint32_t log2T = 0;
    while ((1u << log2T) < T) ++log2T;
    const int nparts = m > 0 ? std::min(kBoxBlocks, (m + 255) / 256) : 0;
    if (m > 0) k_icp_bbox<<<nparts, 256, 0, st>>>(dst, m, inv_cell, box);
    k_icp_hash<<<1, 64, 0, st>>>(box, nparts, log2T, hash);
    icp_sort(src, n, inv_cell, hash, T, count, start, tile, rec_src, st);
    icp_sort(dst, m, inv_cell, hash, T, count, start, tile, rec_dst, st);
    k_icp_init<<<1, 64, 0, st>>>(pose_in, pose, pose_f);
    bp_status s = launch_status();
    const IcpGrid g{start, rec_dst, hash, inv_cell, 1.0f / inv_cell};
    const int ns = (n + kSumsChunk - 1) / kSumsChunk;
    for (int it = 0; it < iters && s == BP_OK; ++it) {
        if (n > 0) {
            k_icp_corr<<<nb, kIcpBlock, 0, st>>>(rec_src, n, g, pose_f, dmax2, corr);
            k_icp_sums<<<ns, kIcpBlock, 0, st>>>(src, n, dst, corr, pose_f, partial);
        }
        k_icp_update<<<1, kIcpBlock, 0, st>>>(partial, ns, pose, pose_f, it, rms, pairs);
        s = launch_status();
    }
    if (s == BP_OK) {
        k_copy_f64<<<1, 64, 0, st>>>(pose, pose_out, 12);
        s = launch_status();
    }
    return s;
}

}  // namespace bpk
