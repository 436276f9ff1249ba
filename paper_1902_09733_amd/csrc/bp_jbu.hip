// a7 on gfx950: joint bilateral upsampling of the disparity (Eq. 2), with an
// optional fused triangulation of every output pixel (Eq. 3).
//
// A 256-thread block owns 16 x 16 full-resolution pixels.  The low-resolution
// taps every pixel of the block can reach (disparity and the guide sample
// I_q at scale*q + scale/2, packed RGB, with |I_q|^2) are staged once in LDS.
// The weight of a tap is one exp2 of a sum of exponents: the spatial part is
// separable and depends only on the pixel's sub-pixel phase, so it is a
// per-thread table of 2R+1 values per axis; the range part is |I_p - I_q|^2
// scaled by log2(e) / (2 sigma_r^2), with the squared distance formed exactly
// in integers as |I_p|^2 + |I_q|^2 - 2 I_p.I_q (one 4 x u8 dot product per
// tap).  Weights are evaluated relative to the smallest exponent of the window
// (a common factor that cancels in K_p), so no pixel can lose all its weights
// to underflow.  ALU/transcendental bound: about (2R+1)^2 exp2 and a dozen
// other vector operations per output pixel and tap.
#include <hip/hip_runtime.h>

#include "bp_internal.h"

namespace bpk {

constexpr int kTile = 16;
constexpr int kMaxTap = kTile + 1 + 2 * 8;   // low-res tile width for scale >= 1, R <= 8

template <int C>
__device__ __forceinline__ uint32_t guide_px(const uint8_t *__restrict__ g, int64_t stride, int x, int y)
{
    const uint8_t *p = g + (int64_t)y * stride + (int64_t)x * C;
    if constexpr (C == 1) return p[0];
    else return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
}

// Eq. 3 epilogue: the camera-frame point of a full-resolution pixel (u, v)
// with disparity d = s * D_p pixels is (B / d) [u - u0, (v - v0) dv / du, f / du]
// (the last entry from Eq. 3's projection, d = f B / (z du)); NaN where d <= 0.
struct PointArgs {
    float *xyz;                 // [hh][wh][3], or NULL
    float baseline, f_du, dv_du, u0, v0;
};

template <int R, int C, bool PTS>
__global__ void __launch_bounds__(256) k_jbu(const int32_t *__restrict__ disp, int wl, int hl,
                                            const uint8_t *__restrict__ guide, int wh, int hh, int64_t stride,
                                            int s, float ksp, float krg, float *__restrict__ out, PointArgs pa)
{
    __shared__ float t_d[kMaxTap * kMaxTap];
    // Per tap: packed guide colour and |I_q|^2 (+inf outside the grid, which
    // gives the tap zero weight).
    __shared__ uint2 t_g[kMaxTap * kMaxTap];
    constexpr int NT = 2 * R + 1;
    const int bx0 = blockIdx.x * kTile, by0 = blockIdx.y * kTile;
    const int qx0 = bx0 / s - R, qy0 = by0 / s - R;
    const int tw = (bx0 + kTile - 1) / s - bx0 / s + 1 + 2 * R;
    const int th = (by0 + kTile - 1) / s - by0 / s + 1 + 2 * R;
    for (int i = threadIdx.x; i < tw * th; i += 256) {
        const int ty = i / tw, tx = i - ty * tw;
        const int qx = qx0 + tx, qy = qy0 + ty;
        float d = 0.0f;
        uint32_t g = 0u;
        float n = __builtin_huge_valf();
        if (qx >= 0 && qx < wl && qy >= 0 && qy < hl) {
            d = (float)disp[(int64_t)qy * wl + qx];
            g = guide_px<C>(guide, stride, s * qx + s / 2, s * qy + s / 2);
            n = (float)__builtin_amdgcn_udot4(g, g, 0u, false);
        }
        t_d[ty * kMaxTap + tx] = d;
        t_g[ty * kMaxTap + tx] = make_uint2(g, __float_as_uint(n));
    }
    __syncthreads();
    const int px = bx0 + (int)(threadIdx.x % kTile), py = by0 + (int)(threadIdx.x / kTile);
    if (px >= wh || py >= hh) return;
    const uint32_t ip = guide_px<C>(guide, stride, px, py);
    const int np = (int)__builtin_amdgcn_udot4(ip, ip, 0u, false);
    const int cx = px / s, cy = py / s;
    const int ox = cx - R - qx0, oy = cy - R - qy0;   // tile coordinates of the window corner
    // Separable spatial exponents: s * (p_lo - q) = phase + 0.5 - s/2 - s*dq.
    float ex[NT], ey[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const float tx = (float)(px - s * cx) + 0.5f - 0.5f * (float)s - (float)(s * (i - R));
        const float ty = (float)(py - s * cy) + 0.5f - 0.5f * (float)s - (float)(s * (i - R));
        ex[i] = tx * tx * ksp;
        ey[i] = ty * ty * ksp;
    }
    constexpr bool KEEP = NT * NT <= 81;
    float e[KEEP ? NT * NT : 1];
    // Exponent of tap (dx, dy); |I_p - I_q|^2 = (|I_p|^2 - 2 I_p.I_q) + |I_q|^2
    // is an integer below 2^24, so every step is exact.
    auto expo = [&](int dx, int dy) {
        const uint2 g = t_g[(oy + dy) * kMaxTap + ox + dx];
        const int dot = (int)__builtin_amdgcn_udot4(ip, g.x, 0u, false);
        const float r2 = (float)(np - 2 * dot) + __uint_as_float(g.y);
        return fmaf(r2, krg, ex[dx] + ey[dy]);
    };
    float emin = __builtin_huge_valf();
#pragma unroll
    for (int dy = 0; dy < NT; ++dy)
#pragma unroll
        for (int dx = 0; dx < NT; ++dx) {
            const float v = expo(dx, dy);
            if constexpr (KEEP) e[dy * NT + dx] = v;
            emin = fminf(emin, v);
        }
    float num = 0.0f, den = 0.0f;
#pragma unroll
    for (int dy = 0; dy < NT; ++dy)
#pragma unroll
        for (int dx = 0; dx < NT; ++dx) {
            float v;
            if constexpr (KEEP) v = e[dy * NT + dx];
            else v = expo(dx, dy);
            const float w = __builtin_amdgcn_exp2f(emin - v);
            num = fmaf(w, t_d[(oy + dy) * kMaxTap + ox + dx], num);
            den += w;
        }
    const float dp = num / den;
    if (out) out[(int64_t)py * wh + px] = dp;
    if constexpr (PTS) {
        const float d = (float)s * dp;
        float x = __builtin_nanf(""), y = x, z = x;
        if (d > 0.0f) {
            const float k = pa.baseline / d;
            x = k * ((float)px - pa.u0);
            y = k * ((float)py - pa.v0) * pa.dv_du;
            z = k * pa.f_du;
        }
        float *o = pa.xyz + ((int64_t)py * wh + px) * 3;
        o[0] = x;
        o[1] = y;
        o[2] = z;
    }
}

bp_status launch_upsample(const int32_t *disp_lo, int wl, int hl, const uint8_t *guide, int wh, int hh, int ch,
                          int64_t stride, float sigma_s, float sigma_r, int radius, float *out, const bp_camera *cam,
                          float *xyz, hipStream_t st)
{
    const int s = wh / wl;
    const float log2e = 1.4426950408889634f;
    const float ksp = log2e / (2.0f * sigma_s * sigma_s);
    const float krg = log2e / (2.0f * sigma_r * sigma_r);
    PointArgs pa{xyz, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (cam) {
        pa.baseline = cam->baseline;
        pa.f_du = cam->focal / cam->du;
        pa.dv_du = cam->dv / cam->du;
        pa.u0 = cam->u0;
        pa.v0 = cam->v0;
    }
    const bool pts = xyz != nullptr;
    dim3 grid((wh + kTile - 1) / kTile, (hh + kTile - 1) / kTile);
#define BP_JBU_CASE(RV)                                                                                       \
    case RV:                                                                                                  \
        if (ch == 1) {                                                                                        \
            if (pts) k_jbu<RV, 1, true><<<grid, 256, 0, st>>>(disp_lo, wl, hl, guide, wh, hh, stride, s, ksp, krg, out, pa); \
            else k_jbu<RV, 1, false><<<grid, 256, 0, st>>>(disp_lo, wl, hl, guide, wh, hh, stride, s, ksp, krg, out, pa);    \
        } else {                                                                                              \
            if (pts) k_jbu<RV, 3, true><<<grid, 256, 0, st>>>(disp_lo, wl, hl, guide, wh, hh, stride, s, ksp, krg, out, pa); \
            else k_jbu<RV, 3, false><<<grid, 256, 0, st>>>(disp_lo, wl, hl, guide, wh, hh, stride, s, ksp, krg, out, pa);    \
        }                                                                                                     \
        break;
    switch (radius) {
        BP_JBU_CASE(0)
        BP_JBU_CASE(1)
        BP_JBU_CASE(2)
        BP_JBU_CASE(3)
        BP_JBU_CASE(4)
        BP_JBU_CASE(5)
        BP_JBU_CASE(6)
        BP_JBU_CASE(7)
        BP_JBU_CASE(8)
    default: return BP_ERR_UNSUPPORTED;
    }
#undef BP_JBU_CASE
    return launch_status();
}

}  // namespace bpk
