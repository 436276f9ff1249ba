/*
 * FP32 CPU oracle for undistortion of a frame under a radial-only lens
 * model (Sec. 2.1: intrinsic calibration with radial distortion only, then
 * undistort-and-remap of every frame before matching).
 *
 * TEST INFRASTRUCTURE ONLY (same rules as bp_oracle.c): only the test suite
 * may load it, and it shares no code with the GPU library.
 *
 * The paper names the operation, not its arithmetic; the model and the
 * sampling rule used here:
 *  - output pixel (u, v) of the undistorted frame looks at the distorted
 *    frame at
 *      xn = (u - cx) / fx, yn = (v - cy) / fy, r2 = xn^2 + yn^2,
 *      g  = 1 + r2 (k1 + r2 (k2 + r2 k3)),
 *      us = cx + (u - cx) g,  vs = cy + (v - cy) g
 *    (the pinhole projection of the radially scaled normalised point,
 *    fx xn g + cx, written so that g = 1 maps every pixel onto itself);
 *  - bilinear interpolation of each channel between the 2 x 2 pixels around
 *    (us, vs), rounded half up to u8; a source point outside
 *    [0, W-1] x [0, H-1] gives 0.
 * The result is an integer decided by floating point, so the oracle takes
 * that decision in the same precision as the kernel: FP32, every operation
 * rounded on its own (no fused multiply-add), in the order written.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define BPO_OK 0
#define BPO_EINVAL (-1)

int bpo_undistort(const uint8_t *in, int w, int h, int C, const float *K, uint8_t *out)
{
    if (!in || !out || !K || w <= 0 || h <= 0 || (C != 1 && C != 3)) return BPO_EINVAL;
    const float fx = K[0], fy = K[1], cx = K[2], cy = K[3], k1 = K[4], k2 = K[5], k3 = K[6];
    if (!(fx > 0.0f) || !(fy > 0.0f)) return BPO_EINVAL;
    const float ifx = 1.0f / fx, ify = 1.0f / fy;
    for (int v = 0; v < h; ++v)
        for (int u = 0; u < w; ++u) {
            const float du = (float)u - cx, dv = (float)v - cy;
            const float xn = du * ifx, yn = dv * ify;
            const float r2 = xn * xn + yn * yn;
            const float g = 1.0f + r2 * (k1 + r2 * (k2 + r2 * k3));
            const float us = cx + du * g, vs = cy + dv * g;
            uint8_t *o = out + ((size_t)v * w + u) * C;
            if (!(us >= 0.0f && vs >= 0.0f && us <= (float)(w - 1) && vs <= (float)(h - 1))) {
                for (int c = 0; c < C; ++c) o[c] = 0;
                continue;
            }
            const int x0 = (int)floorf(us), y0 = (int)floorf(vs);
            const int x1 = x0 + 1 < w ? x0 + 1 : x0, y1 = y0 + 1 < h ? y0 + 1 : y0;
            const float ax = us - (float)x0, ay = vs - (float)y0;
            for (int c = 0; c < C; ++c) {
                const float p00 = in[((size_t)y0 * w + x0) * C + c], p10 = in[((size_t)y0 * w + x1) * C + c];
                const float p01 = in[((size_t)y1 * w + x0) * C + c], p11 = in[((size_t)y1 * w + x1) * C + c];
                const float top = p00 + ax * (p10 - p00);
                const float bot = p01 + ax * (p11 - p01);
                const float val = top + ay * (bot - top);
                const float r = floorf(val + 0.5f);
                o[c] = (uint8_t)(r > 255.0f ? 255.0f : r);
            }
        }
    return BPO_OK;
}
