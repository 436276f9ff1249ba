// a1 + a2 on gfx950: optional s x s block-mean downsampling of the rectified
// pair fused with the truncated absolute-difference data term of Eq. 1.
//
// One 256-thread block produces one output row segment of 256 pixels for all
// labels: the downsampled left pixels of the segment and the right pixels it
// can match (segment start - (L-1) .. end) are computed once into LDS, then
// every label plane is written with coalesced 1 KB row stores.
#include <hip/hip_runtime.h>

#include "bp_internal.h"

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
        float v = trunc;
        if (x - d >= 0) {
            const uint32_t rv = rpx[tid + (L - 1) - d];
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
            v = fminf(a, trunc);
        }
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

}  // namespace bpk
