// a7 on gfx950: joint bilateral upsampling of the disparity (Eq. 2), with an
// optional fused triangulation of every output pixel (Eq. 3).
//
// A 256-thread block owns 16 x 16 full-resolution pixels.  The low-resolution
// taps every pixel of the block can reach are staged once in LDS, one 16-byte
// record each: the guide sample I_q at scale*q + scale/2 as FP16 channel pairs
// (exact for 8-bit values), -|I_q|^2 and the tap's disparity as floats.  The
// weight of a tap is exp2 of a non-positive exponent, spatial + range: the
// spatial part is separable and depends only on the pixel's sub-pixel phase,
// so a per-block LDS table holds, for each of the block's 16 columns, the
// 2R+1 x exponents (each thread copies its column's row into registers) and,
// for each of its 16 rows, the 2R+1 exp2 factors of the y part, applied once
// per window row to that row's sums; the range part is
// -|I_p - I_q|^2 scaled by log2(e) / (2 sigma_r^2).  The squared distance is
// formed exactly by FP16 dot products accumulating in FP32 (every term is an
// integer below 2^24): 2 I_p.I_q - |I_q|^2 - 256 floor(|I_p|^2 / 256), the
// remaining low byte of |I_p|^2 entering through the x table.  Weights are
// taken relative to exponent 0; a pixel whose weights sum below 2^-60 (a guide
// colour far from every tap in its window) is evaluated again relative to its
// largest exponent, so no pixel loses its weights to underflow.
// ALU/transcendental bound: per output pixel and tap one or two dot products,
// one exp2 and three other vector operations.
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

typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t h2_bits(float a, float b)
{
    const h2_t v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ h2_t bits_h2(uint32_t u) { return __builtin_bit_cast(h2_t, u); }

// floor(a / b) for 0 <= a < 2^20 and b >= 1 from a reciprocal rb of b within
// one ulp: (a + 0.5) / b lies at least 0.5 / b, four ulps of the quotient,
// from an integer, beyond the error of the product.
__device__ __forceinline__ int div_small(int a, float rb) { return (int)(((float)a + 0.5f) * rb); }

template <int R, int C, bool PTS>
__global__ void __launch_bounds__(256) k_jbu(const int32_t *__restrict__ disp, int wl, int hl,
                                            const uint8_t *__restrict__ guide, int wh, int hh, int64_t stride,
                                            int s, float rs, float ksp, float krg, float *__restrict__ out,
                                            PointArgs pa)
{
    // Per tap: FP16 (I_R, I_G), (I_B, 256) (grey: (I, 256), unused),
    // -|I_q|^2 and the disparity.  Outside the grid -|I_q|^2 is -inf, which
    // gives the tap zero weight.
    __shared__ uint4 t_q[kMaxTap * kMaxTap];
    constexpr int NT = 2 * R + 1;
    // Separable spatial terms of the block's 16 columns and 16 rows, per
    // window column / row: the x exponent, and exp2 of the y exponent.
    __shared__ float t_sx[kTile * NT], t_wy[kTile * NT];
    const int bx0 = blockIdx.x * kTile, by0 = blockIdx.y * kTile;
    const int qx0 = bx0 / s - R, qy0 = by0 / s - R;
    const int tw = (bx0 + kTile - 1) / s - bx0 / s + 1 + 2 * R;
    const int th = (by0 + kTile - 1) / s - by0 / s + 1 + 2 * R;
    const float rtw = __builtin_amdgcn_rcpf((float)tw);
    for (int i = threadIdx.x; i < tw * th; i += 256) {
        const int ty = div_small(i, rtw), tx = i - ty * tw;
        const int qx = qx0 + tx, qy = qy0 + ty;
        uint4 r = make_uint4(0u, 0u, __float_as_uint(-__builtin_huge_valf()), 0u);
        if (qx >= 0 && qx < wl && qy >= 0 && qy < hl) {
            const uint32_t g = guide_px<C>(guide, stride, s * qx + s / 2, s * qy + s / 2);
            const int n = (int)__builtin_amdgcn_udot4(g, g, 0u, false);
            if constexpr (C == 3) {
                r.x = h2_bits((float)(g & 255u), (float)((g >> 8) & 255u));
                r.y = h2_bits((float)(g >> 16), 256.0f);
            } else {
                r.x = h2_bits((float)g, 256.0f);
            }
            r.z = __float_as_uint(-(float)n);
            r.w = __float_as_uint((float)disp[(int64_t)qy * wl + qx]);
        }
        t_q[ty * kMaxTap + tx] = r;
    }
    // s * (p_lo - q) = phase + 0.5 - s/2 - s*dq for window offset dq = i - R.
    for (int i = threadIdx.x; i < 2 * kTile * NT; i += 256) {
        const int y = i >= kTile * NT, e = i - y * (kTile * NT), c = e / NT, k = e - c * NT;
        const int p = (y ? by0 : bx0) + c;
        const float t = (float)(p - s * div_small(p, rs)) + 0.5f - 0.5f * (float)s - (float)(s * (k - R));
        const float v = -(t * t * ksp);
        if (y) t_wy[e] = __builtin_amdgcn_exp2f(v);
        else t_sx[e] = v;
    }
    __syncthreads();
    const int col = (int)(threadIdx.x % kTile), rowi = (int)(threadIdx.x / kTile);
    const int px = bx0 + col, py = by0 + rowi;
    if (px >= wh || py >= hh) return;
    const uint32_t ip = guide_px<C>(guide, stride, px, py);
    const int np = (int)__builtin_amdgcn_udot4(ip, ip, 0u, false);
    // Pixel side of the dot products: 2 I_p (exact in FP16 up to 510) and
    // -floor(|I_p|^2 / 256) (at most 762) against the tap's 256.
    h2_t pa2, pb2;
    if constexpr (C == 3) {
        pa2 = bits_h2(h2_bits(2.0f * (float)(ip & 255u), 2.0f * (float)((ip >> 8) & 255u)));
        pb2 = bits_h2(h2_bits(2.0f * (float)(ip >> 16), -(float)(np >> 8)));
    } else {
        pa2 = bits_h2(h2_bits(2.0f * (float)ip, -(float)(np >> 8)));
        pb2 = pa2;
    }
    const float np_lo = krg * (float)(np & 255);
    const int cx = div_small(px, rs), cy = div_small(py, rs);
    const int ox = cx - R - qx0, oy = cy - R - qy0;   // tile coordinates of the window corner
    // Separable spatial exponents: s * (p_lo - q) = phase + 0.5 - s/2 - s*dq.
    const float fx = (float)(px - s * cx) + 0.5f - 0.5f * (float)s;
    const float fy = (float)(py - s * cy) + 0.5f - 0.5f * (float)s;
    // Range part of a tap's exponent before scaling, from its record:
    // 2 I_p.I_q - |I_q|^2 - 256 floor(|I_p|^2 / 256), an exact integer (-inf
    // outside the grid).
    auto range = [&](const uint4 &q) {
        float r = __builtin_amdgcn_fdot2(pa2, bits_h2(q.x), __uint_as_float(q.z), false);
        if constexpr (C == 3) r = __builtin_amdgcn_fdot2(pb2, bits_h2(q.y), r, false);
        return r;
    };
    // x term of the exponent: spatial x exponent less krg * the low byte of |I_p|^2.
    float ex[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) ex[i] = t_sx[col * NT + i] - np_lo;
    float num = 0.0f, den = 0.0f;
#pragma unroll
    for (int dy = 0; dy < NT; ++dy) {
        const float wy = t_wy[rowi * NT + dy];
        float rn = 0.0f, rd = 0.0f;
#pragma unroll
        for (int dx = 0; dx < NT; ++dx) {
            const uint4 q = t_q[(oy + dy) * kMaxTap + ox + dx];
            const float w = __builtin_amdgcn_exp2f(fmaf(range(q), krg, ex[dx]));
            rn = fmaf(w, __uint_as_float(q.w), rn);
            rd += w;
        }
        num = fmaf(wy, rn, num);
        den = fmaf(wy, rd, den);
    }
    if (!(den >= 0x1p-60f)) {
        // Every weight is tiny: the same sums relative to the tap of largest
        // exponent (finite, since the pixel's own cell is in the grid), with
        // the range difference to it taken exactly before scaling so that
        // exponents far below zero keep their precision.
        float emax = -__builtin_huge_valf(), rm = 0.0f, sm = 0.0f;
#pragma unroll 1
        for (int dy = 0; dy < NT; ++dy) {
            const float ty = fy - (float)(s * (dy - R)), sy = -(ty * ty * ksp);
#pragma unroll 1
            for (int dx = 0; dx < NT; ++dx) {
                const float tx = fx - (float)(s * (dx - R)), sp = sy - tx * tx * ksp;
                const float r = range(t_q[(oy + dy) * kMaxTap + ox + dx]), e = fmaf(r, krg, sp);
                if (e > emax) {
                    emax = e;
                    rm = r;
                    sm = sp;
                }
            }
        }
        num = 0.0f;
        den = 0.0f;
#pragma unroll 1
        for (int dy = 0; dy < NT; ++dy) {
            const float ty = fy - (float)(s * (dy - R)), sy = -(ty * ty * ksp);
#pragma unroll 1
            for (int dx = 0; dx < NT; ++dx) {
                const float tx = fx - (float)(s * (dx - R)), sp = sy - tx * tx * ksp;
                const uint4 q = t_q[(oy + dy) * kMaxTap + ox + dx];
                const float w = __builtin_amdgcn_exp2f(fmaf(range(q) - rm, krg, sp - sm));
                num = fmaf(w, __uint_as_float(q.w), num);
                den += w;
            }
        }
    }
    // den >= 2^-60 here (>= 1 after the second pass): a normal number.
    const float dp = num * __builtin_amdgcn_rcpf(den);
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
    const float rs = 1.0f / (float)s;
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
            if (pts) k_jbu<RV, 1, true><<<grid, 256, 0, st>>>(disp_lo, wl, hl, guide, wh, hh, stride, s, rs, ksp, krg, out, pa); \
            else k_jbu<RV, 1, false><<<grid, 256, 0, st>>>(disp_lo, wl, hl, guide, wh, hh, stride, s, rs, ksp, krg, out, pa);    \
        } else {                                                                                              \
            if (pts) k_jbu<RV, 3, true><<<grid, 256, 0, st>>>(disp_lo, wl, hl, guide, wh, hh, stride, s, rs, ksp, krg, out, pa); \
            else k_jbu<RV, 3, false><<<grid, 256, 0, st>>>(disp_lo, wl, hl, guide, wh, hh, stride, s, rs, ksp, krg, out, pa);    \
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
