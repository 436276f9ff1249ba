// a1 + a2 on gfx950: optional s x s block-mean downsampling of the rectified
// pair fused with the truncated absolute-difference data term of Eq. 1.
//
// bp_cost_volume: one 256-thread block produces one output row segment of 256
// pixels for all labels: the downsampled left pixels of the segment and the
// right pixels it can match (segment start - (L-1) .. end) are computed once
// into LDS, then every label plane is written with coalesced 1 KB row stores.
//
// bp_run from a pair: the downsampled pair is first packed (one 32-bit word
// per pixel) into the workspace, then the data term is written straight into
// the finest level's colour-split layout (pixel-major or label-major), so the
// planar volume never exists.
#include <hip/hip_runtime.h>

#include "bp_internal.h"
#include "bp_levels.h"

namespace bpk {

// s x s block mean of channel `ch` at output pixel (x, y), rounded half up.
template <int C>
__device__ __forceinline__ uint32_t pixel_ds(const uint8_t *__restrict__ img, int64_t stride, int x, int y, int s)
{
    uint32_t out = 0;
#pragma unroll
    for (int ch = 0; ch < C; ++ch) {
        uint32_t sum = 0;
        for (int j = 0; j < s; ++j) {
            const uint8_t *row = img + (int64_t)(s * y + j) * stride + (int64_t)(s * x) * C + ch;
            for (int i = 0; i < s; ++i) sum += row[i * C];
        }
        const uint32_t n = (uint32_t)(s * s);
        out |= ((sum + n / 2) / n) << (8 * ch);
    }
    return out;
}

constexpr int kSeg = 256;

// Data term of Eq. 1 for packed left/right pixels lv, rv (label d with x - d >= 0).
template <int C>
__device__ __forceinline__ float ad_cost(uint32_t lv, uint32_t rv, int rgb_mode, float trunc)
{
    float a;
    if constexpr (C == 1) {
        a = (float)abs((int)lv - (int)rv);
    } else {
        int sum = 0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
            sum += abs((int)((lv >> (8 * ch)) & 0xffu) - (int)((rv >> (8 * ch)) & 0xffu));
        a = rgb_mode == 0 ? (float)((sum + 1) / 3) : (float)sum / 3.0f;
    }
    return fminf(a, trunc);
}

template <int C>
__global__ void __launch_bounds__(256) k_cost(const uint8_t *__restrict__ left, const uint8_t *__restrict__ right,
                                             int64_t stride, int s, int wo, int ho, int L, float trunc, int rgb_mode,
                                             float *__restrict__ cost)
{
    extern __shared__ uint32_t lds[];
    uint32_t *lpx = lds;               // [kSeg]
    uint32_t *rpx = lds + kSeg;        // [kSeg + L - 1]
    const int y = blockIdx.y;
    const int x0 = blockIdx.x * kSeg;
    const int tid = threadIdx.x;
    {
        const int x = x0 + tid;
        lpx[tid] = x < wo ? pixel_ds<C>(left, stride, x, y, s) : 0u;
    }
    for (int i = tid; i < kSeg + L - 1; i += 256) {
        const int x = x0 - (L - 1) + i;
        rpx[i] = (x >= 0 && x < wo) ? pixel_ds<C>(right, stride, x, y, s) : 0u;
    }
    __syncthreads();
    const int x = x0 + tid;
    if (x >= wo) return;
    const uint32_t lv = lpx[tid];
    const int64_t plane = (int64_t)wo * ho;
    float *out = cost + (int64_t)y * wo + x;
    for (int d = 0; d < L; ++d) {
        const float v = x - d >= 0 ? ad_cost<C>(lv, rpx[tid + (L - 1) - d], rgb_mode, trunc) : trunc;
        out[(int64_t)d * plane] = v;
    }
}

bp_status launch_cost_volume(const uint8_t *left, const uint8_t *right, int w, int h, int ch, int64_t stride,
                             int ds, int L, float trunc, int rgb_mode, float *cost, hipStream_t s)
{
    const int wo = w / ds, ho = h / ds;
    dim3 grid((wo + kSeg - 1) / kSeg, ho);
    const size_t lds = sizeof(uint32_t) * (2 * kSeg + L - 1);
    if (ch == 1)
        k_cost<1><<<grid, 256, lds, s>>>(left, right, stride, ds, wo, ho, L, trunc, rgb_mode, cost);
    else
        k_cost<3><<<grid, 256, lds, s>>>(left, right, stride, ds, wo, ho, L, trunc, rgb_mode, cost);
    return launch_status();
}

template <int C>
__global__ void __launch_bounds__(256) k_downsample(const uint8_t *__restrict__ in, int64_t stride, int s, int wo,
                                                   int ho, uint8_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)wo * ho) return;
    const int x = (int)(i % wo), y = (int)(i / wo);
    const uint32_t v = pixel_ds<C>(in, stride, x, y, s);
#pragma unroll
    for (int ch = 0; ch < C; ++ch) out[i * C + ch] = (uint8_t)(v >> (8 * ch));
}

bp_status launch_downsample(const uint8_t *in, int w, int h, int ch, int64_t stride, int ds, uint8_t *out,
                            hipStream_t s)
{
    const int wo = w / ds, ho = h / ds;
    const int64_t n = (int64_t)wo * ho;
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (ch == 1) k_downsample<1><<<grid, 256, 0, s>>>(in, stride, ds, wo, ho, out);
    else k_downsample<3><<<grid, 256, 0, s>>>(in, stride, ds, wo, ho, out);
    return launch_status();
}

// ------------------------------------------------------------------------
// Finest-level data term computed from a pair (bp_problem.pair)
// ------------------------------------------------------------------------

// s x s block mean of an interleaved row chunk read as 32-bit words (s a
// multiple of 4, word-aligned rows): the bytes of channel c in word i are
// selected by a 0/1 byte mask and summed with one 4 x u8 dot product.  Byte b
// of a pixel block's row has channel b % C; the mask pattern repeats every C
// words.  Same rounding as pixel_ds.
template <int C, int S>
__device__ __forceinline__ uint32_t pixel_ds_words(const uint8_t *__restrict__ img, int64_t stride, int x, int y,
                                                   int s_rt)
{
    // S > 0: the scale fixed at compile time (the row chunk's words then load
    // as one vector); S = 0: s_rt.
    const int s = S > 0 ? S : s_rt;
    const int nw = s * C / 4;
    uint32_t acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0;
    for (int j = 0; j < s; ++j) {
        const uint32_t *row = (const uint32_t *)(img + (int64_t)(s * y + j) * stride + (int64_t)s * x * C);
        for (int i = 0; i < nw; ++i) {
            const uint32_t d = row[i];
            if constexpr (C == 1) {
                acc[0] = __builtin_amdgcn_udot4(d, 0x01010101u, acc[0], false);
            } else {
                // Word phase i % 3: byte channels (0,1,2,0), (1,2,0,1), (2,0,1,2).
                const int ph = i % 3;
                const uint32_t m0 = ph == 0 ? 0x01000001u : ph == 1 ? 0x00010000u : 0x00000100u;
                const uint32_t m1 = ph == 0 ? 0x00000100u : ph == 1 ? 0x01000001u : 0x00010000u;
                const uint32_t m2 = ph == 0 ? 0x00010000u : ph == 1 ? 0x00000100u : 0x01000001u;
                acc[0] = __builtin_amdgcn_udot4(d, m0, acc[0], false);
                acc[1] = __builtin_amdgcn_udot4(d, m1, acc[1], false);
                acc[2] = __builtin_amdgcn_udot4(d, m2, acc[2], false);
            }
        }
    }
    const uint32_t n = (uint32_t)(s * s);
    uint32_t out = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) out |= ((acc[c] + n / 2) / n) << (8 * c);
    return out;
}

// Both images of the pair, downsampled and packed: out[z][y][x], z = 0 left.
// Block (bx, by, z) of a (ceil(wo / 256), gy, 2) block grid packs pixels
// [256 bx, 256 bx + 256) of rows by, by + gy, ...
template <int C, bool WORDS, int S>
__device__ __forceinline__ void pack_block(const uint8_t *__restrict__ left, const uint8_t *__restrict__ right,
                                           int64_t stride, int s, int wo, int ho, uint32_t *__restrict__ out, int bx,
                                           int by, int z, int gy)
{
    const int x = bx * 256 + threadIdx.x;
    if (x >= wo) return;
    const uint8_t *img = z ? right : left;
    uint32_t *o = out + (int64_t)z * wo * ho;
    for (int y = by; y < ho; y += gy) {
        if constexpr (WORDS) o[(int64_t)y * wo + x] = pixel_ds_words<C, S>(img, stride, x, y, s);
        else o[(int64_t)y * wo + x] = pixel_ds<C>(img, stride, x, y, s);
    }
}

// The packing followed, in the same launch, by the message initialisation
// (the two touch disjoint memory): a flat grid whose first gx * gy * 2 blocks
// are the packing's (gx, gy, 2) grid and whose next ix * (levels + 1) blocks
// are the initialisation's (ix, levels + 1) grid.
template <int C, bool WORDS, int S>
__global__ void __launch_bounds__(256) k_pack_pair(const uint8_t *__restrict__ left, const uint8_t *__restrict__ right,
                                                  int64_t stride, int s, int wo, int ho, uint32_t *__restrict__ out,
                                                  int gx, int gy, const InitArgs ia, int ix)
{
    const int b = blockIdx.x, np = gx * gy * 2;
    if (b < np) {
        const int z = b / (gx * gy), r = b - z * (gx * gy), by = r / gx;
        pack_block<C, WORDS, S>(left, right, stride, s, wo, ho, out, r - by * gx, by, z, gy);
    } else {
        const int l = (b - np) / ix;
        init_msgs_block(ia, b - np - l * ix, l);
    }
}

// One block owns row y, pixels [x0, x0 + xb) (x0 even): the packed left
// pixels and the right pixels they can match are staged in LDS, then the
// cost of every (pixel, label) is stored at its colour-split address
// c * blk + label * ls + j * ps, j = y * wh + x / 2, c = (x + y) & 1.
// Pixel-major levels (PM): consecutive lanes take consecutive labels of a
// pixel (lp2 = L rounded up to a power of two lanes per pixel); label-major
// levels: consecutive lanes take consecutive same-colour pixels of a label.
template <int C, bool PM>
__global__ void __launch_bounds__(256) k_cost_level0(const uint32_t *__restrict__ packed, int w, int h, int L,
                                                    float trunc, int rgb_mode, int xb, int lp2, int wh, int64_t blk,
                                                    int64_t ls, int64_t ps, float *__restrict__ out)
{
    extern __shared__ uint32_t lds[];
    const int y = blockIdx.y, x0 = blockIdx.x * xb;
    const int nx = min(xb, w - x0);
    uint32_t *lpx = lds;             // [xb]
    uint32_t *rpx = lds + xb;        // [xb + L - 1], rpx[i] = right pixel x0 - (L - 1) + i
    const uint32_t *lrow = packed + (int64_t)y * w;
    const uint32_t *rrow = packed + (int64_t)w * h + (int64_t)y * w;
    for (int i = threadIdx.x; i < nx; i += 256) lpx[i] = lrow[x0 + i];
    for (int i = threadIdx.x; i < nx + L - 1; i += 256) {
        const int x = x0 - (L - 1) + i;
        rpx[i] = x >= 0 ? rrow[x] : 0u;
    }
    __syncthreads();
    // Pixels of colour 0 first, then colour 1; n0 of colour 0 in the segment.
    const int off0 = y & 1;                       // first x (relative to x0) of colour 0
    const int n0 = (nx - off0 + 1) / 2, n1 = (nx - (off0 ^ 1) + 1) / 2;
    const int np = n0 + n1;
    auto pixel = [&](int p, int &xl, int64_t &base) {
        const int c = p < n0 ? 0 : 1;
        const int i = c ? p - n0 : p;
        xl = 2 * i + (c ? off0 ^ 1 : off0);
        const int x = x0 + xl;
        base = (int64_t)c * blk + (int64_t)(y * wh + (x >> 1)) * ps;
    };
    if constexpr (PM) {
        const int f = (int)threadIdx.x % lp2;
        const int step = 256 / lp2;
        if (f >= L) return;
        for (int p = (int)threadIdx.x / lp2; p < np; p += step) {
            int xl;
            int64_t base;
            pixel(p, xl, base);
            const float v = x0 + xl - f >= 0 ? ad_cost<C>(lpx[xl], rpx[xl + (L - 1) - f], rgb_mode, trunc) : trunc;
            out[base + (int64_t)f * ls] = v;
        }
    } else {
        for (int f = 0; f < L; ++f)
            for (int p = threadIdx.x; p < np; p += 256) {
                int xl;
                int64_t base;
                pixel(p, xl, base);
                const float v = x0 + xl - f >= 0 ? ad_cost<C>(lpx[xl], rpx[xl + (L - 1) - f], rgb_mode, trunc) : trunc;
                out[base + (int64_t)f * ls] = v;
            }
    }
}

// Pixel-major levels 0 and 1 together: one block owns level-1 row Y, pixels
// [X0, X0 + xb1), i.e. level-0 rows 2Y and 2Y + 1 (if present) and pixels
// [2 X0, 2 X0 + 2 xb1).  A lane takes four consecutive labels of one level-1
// pixel (q4 lanes per pixel, q4 = ceil(L/4) rounded up to a power of two),
// computes the (up to four) level-0 children, stores each as one 16-byte
// vector, and stores their sum, added in the order (0,0), (1,0), (0,1), (1,1)
// as the separate pyramid step does.  Labels past L (inside the level's
// padded row) get the truncation value; no kernel reads them.
// CF: level 0's storage, FP32, FP16 (four labels in one 8-byte store) or bytes
// (one 4-byte store); the plan chooses the narrow ones only where every value
// is exact in them.
template <int C, int CF>
__global__ void __launch_bounds__(256) k_cost_level01(const uint32_t *__restrict__ packed, int w, int h, int L,
                                                     float trunc, int rgb_mode, int xb1, int q4, int wh0,
                                                     int64_t blk0, int64_t ps0, void *__restrict__ out0, int w1,
                                                     int wh1, int64_t blk1, int64_t ps1, float *__restrict__ out1)
{
    extern __shared__ uint32_t lds[];
    const int Y = blockIdx.y, X0 = blockIdx.x * xb1;
    const int nX = min(xb1, w1 - X0);
    const int x0 = 2 * X0, nx = min(2 * xb1, w - x0);
    const int span = 2 * xb1 + L - 1;
    const int rows = min(2, h - 2 * Y);
    // Row r of the block: lpx at lds[r * (2 xb1 + span)], rpx after it
    // (rpx[i] = right pixel x0 - (L - 1) + i).
    for (int r = 0; r < rows; ++r) {
        uint32_t *lpx = lds + r * (2 * xb1 + span);
        uint32_t *rpx = lpx + 2 * xb1;
        const int y = 2 * Y + r;
        const uint32_t *lrow = packed + (int64_t)y * w;
        const uint32_t *rrow = packed + (int64_t)w * h + (int64_t)y * w;
        for (int i = threadIdx.x; i < nx; i += 256) lpx[i] = lrow[x0 + i];
        for (int i = threadIdx.x; i < nx + L - 1; i += 256) {
            const int x = x0 - (L - 1) + i;
            rpx[i] = x >= 0 ? rrow[x] : 0u;
        }
    }
    __syncthreads();
    const int q = (int)threadIdx.x % q4;
    const int f0 = 4 * q;
    if (f0 >= L) return;
    const int step = 256 / q4;
    for (int X = (int)threadIdx.x / q4; X < nX; X += step) {
        float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int ii = 0; ii < 2; ++ii) {
                const int xl = 2 * X + ii, x = x0 + xl, y = 2 * Y + jj;
                if (xl >= nx || jj >= rows) continue;
                const uint32_t *lpx = lds + jj * (2 * xb1 + span);
                const uint32_t *rpx = lpx + 2 * xb1;
                const uint32_t lv = lpx[xl];
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int f = f0 + e;
                    v[e] = (f < L && x - f >= 0) ? ad_cost<C>(lv, rpx[xl + (L - 1) - f], rgb_mode, trunc) : trunc;
                }
                const int64_t e0 = (int64_t)((x + y) & 1) * blk0 + (int64_t)(y * wh0 + (x >> 1)) * ps0 + f0;
                if constexpr (CF == COST_F16) {
                    typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
                    const h4_t hv = {(_Float16)v[0], (_Float16)v[1], (_Float16)v[2], (_Float16)v[3]};
                    *(h4_t *)((_Float16 *)out0 + e0) = hv;
                } else if constexpr (CF == COST_U8) {
                    *(uint32_t *)((uint8_t *)out0 + e0) = (uint32_t)v[0] | ((uint32_t)v[1] << 8) |
                                                          ((uint32_t)v[2] << 16) | ((uint32_t)v[3] << 24);
                } else {
                    *(float4 *)((float *)out0 + e0) = make_float4(v[0], v[1], v[2], v[3]);
                }
                acc.x += v[0];
                acc.y += v[1];
                acc.z += v[2];
                acc.w += v[3];
            }
        const int Xg = X0 + X;
        *(float4 *)(out1 + (int64_t)((Xg + Y) & 1) * blk1 + (int64_t)(Y * wh1 + (Xg >> 1)) * ps1 + f0) = acc;
    }
}

bp_status launch_pair_cost(const bp_pair &pr, const Plan &p, uint8_t *ws, hipStream_t st, int *levels_done)
{
    // The message initialisation runs in the packing's launch.
    const Level &v = p.lv[0];
    const int w = v.w, h = v.h, L = p.L;
    uint32_t *packed = (uint32_t *)(ws + p.pair_off);
    const int gx = (w + 255) / 256, gy = h < 4096 ? h : 4096;
    unsigned ix;
    const InitArgs ia = init_args(p, ws, &ix);
    const unsigned g1 = (unsigned)(gx * gy * 2) + ix * (unsigned)(p.levels + 1);
    // Word loads when every pixel block's row chunk is word-aligned.
    const bool words = pr.downsample % 4 == 0 && pr.row_stride_bytes % 4 == 0 && ((uintptr_t)pr.left % 4) == 0 &&
                       ((uintptr_t)pr.right % 4) == 0;
#define BP_PACK_S(CV, WV, SV) \
    k_pack_pair<CV, WV, SV><<<g1, 256, 0, st>>>(pr.left, pr.right, pr.row_stride_bytes, pr.downsample, w, h, packed, \
                                                gx, gy, ia, (int)ix)
#define BP_PACK(CV, WV) BP_PACK_S(CV, WV, 0)
    if (pr.channels == 1) {
        if (words) BP_PACK(1, true);
        else BP_PACK(1, false);
    } else {
        if (words && pr.downsample == 4) BP_PACK_S(3, true, 4);
        else if (words) BP_PACK(3, true);
        else BP_PACK(3, false);
    }
#undef BP_PACK_S
#undef BP_PACK
    int lp2 = 1;
    while (lp2 < L) lp2 <<= 1;
    if (p.levels >= 2 && v.layout == PIXEL_MAJOR && p.lv[1].layout == PIXEL_MAJOR) {
        const Level &v1 = p.lv[1];
        // 16-byte stores need every pixel's row (lp labels) to be a multiple of 4.
        int q4 = 1;
        while (4 * q4 < L) q4 <<= 1;
        const int xb1 = 16;   // 16: 19.0 us at 676x380x64, against 19.9 (32) and 20.5 (64)
        const dim3 grid1((unsigned)((v1.w + xb1 - 1) / xb1), (unsigned)v1.h);
        const size_t lds1 = sizeof(uint32_t) * (size_t)2 * (2 * xb1 + 2 * xb1 + L - 1);
        void *out0 = ws + v.cost_off;
        float *out1 = (float *)(ws + v1.cost_off);
#define BP_COST01(CV, HV)                                                                                   \
    k_cost_level01<CV, HV><<<grid1, 256, lds1, st>>>(packed, w, h, L, pr.data_trunc, pr.rgb_mode, xb1, q4, v.wh, \
                                                     v.blk, v.ps, out0, v1.w, v1.wh, v1.blk, v1.ps, out1)
        if (pr.channels == 1) {
            if (v.cost_fmt == COST_F16) BP_COST01(1, COST_F16);
            else if (v.cost_fmt == COST_U8) BP_COST01(1, COST_U8);
            else BP_COST01(1, COST_F32);
        } else {
            if (v.cost_fmt == COST_F16) BP_COST01(3, COST_F16);
            else if (v.cost_fmt == COST_U8) BP_COST01(3, COST_U8);
            else BP_COST01(3, COST_F32);
        }
#undef BP_COST01
        *levels_done = 2;
        return launch_status();
    }
    *levels_done = 1;
    // Row segments of at most 256 pixels, balanced, even width.
    const int nseg = (w + 255) / 256;
    int xb = (w + nseg - 1) / nseg;
    xb += xb & 1;
    const dim3 grid((unsigned)((w + xb - 1) / xb), (unsigned)h);
    const size_t lds = sizeof(uint32_t) * (size_t)(2 * xb + L - 1);
    float *out = (float *)(ws + v.cost_off);
    const bool pm = v.layout == PIXEL_MAJOR;
#define BP_COST0(CV, PMV)                                                                                    \
    k_cost_level0<CV, PMV><<<grid, 256, lds, st>>>(packed, w, h, L, pr.data_trunc, pr.rgb_mode, xb, lp2, v.wh, \
                                                   v.blk, v.ls, v.ps, out)
    if (pr.channels == 1) {
        if (pm) BP_COST0(1, true);
        else BP_COST0(1, false);
    } else {
        if (pm) BP_COST0(3, true);
        else BP_COST0(3, false);
    }
#undef BP_COST0
    return launch_status();
}

}  // namespace bpk
