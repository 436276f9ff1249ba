// Undistortion of a frame under a radial-only lens model (Sec. 2.1: the
// calibrated intrinsics with radial distortion only; every frame is
// undistorted and remapped before matching).
//
// Output pixel (u, v) samples the distorted frame at
//   xn = (u - cx) / fx, yn = (v - cy) / fy, r2 = xn^2 + yn^2,
//   g = 1 + r2 (k1 + r2 (k2 + r2 k3)),  (us, vs) = (cx + (u - cx) g, cy + (v - cy) g)
// (the pinhole projection of the radially scaled normalised point, written so
// that g = 1 maps each pixel onto itself), with bilinear interpolation per
// channel rounded half up to u8, and 0 where (us, vs) leaves [0, W-1] x [0, H-1].
// The source position is computed per pixel, so no map is stored or read.
// Every operation is rounded on its own (no contraction into fused
// multiply-adds): the u8 result is decided in FP32 by a fixed sequence of
// operations.  HBM-bound: about C bytes read and C written per pixel.
#include <hip/hip_runtime.h>

#include "bp_device.h"
#include "bp_internal.h"

namespace bpk {

// Source samples (x0, y), (x1, y) of every channel.  RGB rows with a
// word-aligned start and stride (WORDS) are read as three 32-bit buffer loads
// realigned with v_alignbyte (loads past the image return 0 and are not
// used); otherwise byte loads.
template <int C, bool WORDS>
__device__ __forceinline__ void sample_row(const uint8_t *__restrict__ in, __amdgpu_buffer_rsrc_t rs, int64_t in_stride,
                                           int y, int x0, int x1, float (&p0)[C], float (&p1)[C])
{
    if constexpr (WORDS && C == 3) {
        const uint32_t off = (uint32_t)((int64_t)y * in_stride + (int64_t)x0 * 3);
        const uint32_t a = off & ~3u, sh = off & 3u;
        const uint32_t w0 = __builtin_amdgcn_raw_buffer_load_b32(rs, a, 0, 0);
        const uint32_t w1 = __builtin_amdgcn_raw_buffer_load_b32(rs, a + 4u, 0, 0);
        const uint32_t w2 = __builtin_amdgcn_raw_buffer_load_b32(rs, a + 8u, 0, 0);
        const uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, sh);
        const uint32_t hi = __builtin_amdgcn_alignbyte(w2, w1, sh);
        p0[0] = (float)(lo & 0xffu);
        p0[1] = (float)((lo >> 8) & 0xffu);
        p0[2] = (float)((lo >> 16) & 0xffu);
        if (x1 != x0) {
            p1[0] = (float)(lo >> 24);
            p1[1] = (float)(hi & 0xffu);
            p1[2] = (float)((hi >> 8) & 0xffu);
        } else {
            p1[0] = p0[0];
            p1[1] = p0[1];
            p1[2] = p0[2];
        }
    } else {
        const uint8_t *r = in + (int64_t)y * in_stride;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            p0[c] = r[x0 * C + c];
            p1[c] = r[x1 * C + c];
        }
    }
}

template <int C, bool WORDS>
__global__ void __launch_bounds__(256) k_undistort(const uint8_t *__restrict__ in, int w, int h, int64_t in_stride,
                                                  float fx_inv, float fy_inv, float cx, float cy, float k1, float k2,
                                                  float k3, uint8_t *__restrict__ out, int64_t out_stride)
{
#pragma clang fp contract(off)
    const int u = blockIdx.x * 64 + (int)(threadIdx.x & 63);
    const int v = blockIdx.y * 4 + (int)(threadIdx.x >> 6);
    if (u >= w || v >= h) return;
    const float du = (float)u - cx, dv = (float)v - cy;
    const float xn = du * fx_inv, yn = dv * fy_inv;
    const float r2 = xn * xn + yn * yn;
    const float g = 1.0f + r2 * (k1 + r2 * (k2 + r2 * k3));
    const float us = cx + du * g, vs = cy + dv * g;
    uint8_t *o = out + (int64_t)v * out_stride + (int64_t)u * C;
    if (!(us >= 0.0f && vs >= 0.0f && us <= (float)(w - 1) && vs <= (float)(h - 1))) {
#pragma unroll
        for (int c = 0; c < C; ++c) o[c] = 0;
        return;
    }
    const int x0 = (int)__builtin_floorf(us), y0 = (int)__builtin_floorf(vs);
    const int x1 = x0 + 1 < w ? x0 + 1 : x0, y1 = y0 + 1 < h ? y0 + 1 : y0;
    const float ax = us - (float)x0, ay = vs - (float)y0;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(in, (uint32_t)((int64_t)h * in_stride));
    float p00[C], p10[C], p01[C], p11[C];
    sample_row<C, WORDS>(in, rs, in_stride, y0, x0, x1, p00, p10);
    sample_row<C, WORDS>(in, rs, in_stride, y1, x0, x1, p01, p11);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const float top = p00[c] + ax * (p10[c] - p00[c]);
        const float bot = p01[c] + ax * (p11[c] - p01[c]);
        const float val = top + ay * (bot - top);
        const float rr = __builtin_floorf(val + 0.5f);
        o[c] = (uint8_t)(rr > 255.0f ? 255.0f : rr);
    }
}

bp_status launch_undistort(const uint8_t *in, int w, int h, int ch, int64_t in_stride, const bp_intrinsics &K,
                           uint8_t *out, int64_t out_stride, hipStream_t st)
{
    const float fx_inv = 1.0f / K.fx, fy_inv = 1.0f / K.fy;
    const dim3 grid((unsigned)((w + 63) / 64), (unsigned)((h + 3) / 4));
    const bool words = ((uintptr_t)in % 4) == 0 && in_stride % 4 == 0 && (int64_t)h * in_stride < (1ll << 32);
    if (ch == 1)
        k_undistort<1, false><<<grid, 256, 0, st>>>(in, w, h, in_stride, fx_inv, fy_inv, K.cx, K.cy, K.k1, K.k2, K.k3,
                                                   out, out_stride);
    else if (words)
        k_undistort<3, true><<<grid, 256, 0, st>>>(in, w, h, in_stride, fx_inv, fy_inv, K.cx, K.cy, K.k1, K.k2, K.k3,
                                                  out, out_stride);
    else
        k_undistort<3, false><<<grid, 256, 0, st>>>(in, w, h, in_stride, fx_inv, fy_inv, K.cx, K.cy, K.k1, K.k2, K.k3,
                                                   out, out_stride);
    return launch_status();
}

}  // namespace bpk
