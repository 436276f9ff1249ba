// The pose front end's data-parallel part (Sec. 2.3): Harris response
// (Eq. 4-5), per-cell corner selection (a g x g grid of cells with a hard
// threshold, as in the experiments), and ZSSD patch matching within a search
// range.  Everything is exact integer arithmetic:
//   A = I(x+1, y) - I(x-1, y), B = I(x, y+1) - I(x, y-1)   (central differences)
//   M = sum w [A^2, AB; AB, B^2], w = (1 4 6 4 1)^T (1 4 6 4 1)   (binomial window)
//   25 R = 25 det M - tr(M)^2   (Eq. 5 with k = 1/25), 0 within 3 of the border
//   n ZSSD = n sum (a - b)^2 - (sum a - sum b)^2   (n patch pixels)
// so selections (largest response, smallest cost) are decided without
// rounding.  Ties: first in row-major order.
#include <hip/hip_runtime.h>

#include "bp_internal.h"

namespace bpk {

constexpr int kHT = 16;                  // response tile (16 x 16 outputs per block)
constexpr int kHI = kHT + 6;             // image tile (halo 3)
constexpr int kHD = kHT + 4;             // derivative tile (halo 2)

__global__ void __launch_bounds__(256) k_harris_response(const uint8_t *__restrict__ img, int w, int h, int64_t stride,
                                                        int64_t *__restrict__ r25)
{
    __shared__ int16_t s_img[kHI][kHI];
    __shared__ int32_t s_a[kHD][kHD], s_b[kHD][kHD];
    __shared__ int32_t s_h[3][kHD][kHT];     // horizontal window sums of A^2, B^2, AB
    const int bx = blockIdx.x * kHT, by = blockIdx.y * kHT;
    const int t = threadIdx.x;
    for (int i = t; i < kHI * kHI; i += 256) {
        const int ty = i / kHI, tx = i - ty * kHI;
        const int x = bx - 3 + tx, y = by - 3 + ty;
        s_img[ty][tx] = (x >= 0 && y >= 0 && x < w && y < h) ? (int16_t)img[(int64_t)y * stride + x] : (int16_t)0;
    }
    __syncthreads();
    for (int i = t; i < kHD * kHD; i += 256) {
        const int ty = i / kHD, tx = i - ty * kHD;
        s_a[ty][tx] = s_img[ty + 1][tx + 2] - s_img[ty + 1][tx];
        s_b[ty][tx] = s_img[ty + 2][tx + 1] - s_img[ty][tx + 1];
    }
    __syncthreads();
    const int wt[5] = {1, 4, 6, 4, 1};
    for (int i = t; i < kHD * kHT; i += 256) {
        const int ty = i / kHT, tx = i - ty * kHT;
        int32_t xx = 0, yy = 0, xy = 0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int32_t a = s_a[ty][tx + k], b = s_b[ty][tx + k];
            xx += wt[k] * a * a;
            yy += wt[k] * b * b;
            xy += wt[k] * a * b;
        }
        s_h[0][ty][tx] = xx;
        s_h[1][ty][tx] = yy;
        s_h[2][ty][tx] = xy;
    }
    __syncthreads();
    const int tx = t % kHT, ty = t / kHT;
    const int x = bx + tx, y = by + ty;
    if (x >= w || y >= h) return;
    int64_t v = 0;
    if (x >= 3 && y >= 3 && x <= w - 4 && y <= h - 4) {
        int64_t sxx = 0, syy = 0, sxy = 0;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            sxx += wt[k] * s_h[0][ty + k][tx];
            syy += wt[k] * s_h[1][ty + k][tx];
            sxy += wt[k] * s_h[2][ty + k][tx];
        }
        const int64_t det = sxx * syy - sxy * sxy, tr = sxx + syy;
        v = 25 * det - tr * tr;
    }
    r25[(int64_t)y * w + x] = v;
}

// One block per cell: the largest response above the threshold among the
// cell's 3 x 3 local maxima, first in row-major order on ties.  The cell is
// taken in strips of rows whose responses, with a one-pixel border, are
// staged in LDS by coalesced loads (outside the frame: INT64_MIN, never
// larger); cells wider than the staging row fall back to global loads.
constexpr int kSelTile = 4096;          // int64 responses staged per strip

__device__ __forceinline__ void take_best(int64_t v, int64_t idx, int64_t &bv, int64_t &bi)
{
    if (bi < 0 || v > bv || (v == bv && idx < bi)) {
        bv = v;
        bi = idx;
    }
}

__global__ void __launch_bounds__(256) k_harris_select(const int64_t *__restrict__ r25, int w, int h, int g,
                                                      int64_t thr, bp_corner *__restrict__ out)
{
    __shared__ int64_t s_t[kSelTile];
    __shared__ int64_t s_v[256];
    __shared__ int64_t s_i[256];
    const int ci = blockIdx.x / g, cj = blockIdx.x - ci * g;
    const int x0 = (int)((int64_t)cj * w / g), x1 = (int)((int64_t)(cj + 1) * w / g);
    const int y0 = (int)((int64_t)ci * h / g), y1 = (int)((int64_t)(ci + 1) * h / g);
    const int cw = x1 - x0, ch = y1 - y0;
    int64_t bv = 0, bi = -1;       // best value and row-major index of its pixel
    const int tw = cw + 2;
    const int sr = kSelTile / tw - 2; // rows per strip
    if (sr >= 1) {
        for (int ys = y0; ys < y1; ys += sr) {
            const int ye = ys + sr < y1 ? ys + sr : y1, th = ye - ys + 2;
            for (int k = threadIdx.x; k < th * tw; k += 256) {
                const int ty = k / tw, tx = k - ty * tw;
                const int y = ys - 1 + ty, x = x0 - 1 + tx;
                s_t[k] = (x >= 0 && y >= 0 && x < w && y < h) ? r25[(int64_t)y * w + x] : INT64_MIN;
            }
            __syncthreads();
            for (int k = threadIdx.x; k < (ye - ys) * cw; k += 256) {
                const int py = k / cw, px = k - py * cw;
                const int t = (py + 1) * tw + px + 1;
                const int64_t v = s_t[t];
                if (v <= thr) continue;
                const bool peak = s_t[t - tw - 1] <= v && s_t[t - tw] <= v && s_t[t - tw + 1] <= v && s_t[t - 1] <= v &&
                                  s_t[t + 1] <= v && s_t[t + tw - 1] <= v && s_t[t + tw] <= v && s_t[t + tw + 1] <= v;
                if (peak) take_best(v, (int64_t)(ys + py) * w + (x0 + px), bv, bi);
            }
            __syncthreads();
        }
    } else {
        for (int k = threadIdx.x; k < cw * ch; k += 256) {
            const int y = y0 + k / cw, x = x0 + k % cw;
            const int64_t v = r25[(int64_t)y * w + x];
            if (v <= thr) continue;
            bool peak = true;
            for (int j = -1; j <= 1; ++j)
                for (int i = -1; i <= 1; ++i) {
                    const int nx = x + i, ny = y + j;
                    if ((i || j) && nx >= 0 && ny >= 0 && nx < w && ny < h && r25[(int64_t)ny * w + nx] > v)
                        peak = false;
                }
            if (peak) take_best(v, (int64_t)y * w + x, bv, bi);
        }
    }
    s_v[threadIdx.x] = bv;
    s_i[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const int64_t ov = s_v[threadIdx.x + s], oi = s_i[threadIdx.x + s];
            const int64_t mv = s_v[threadIdx.x], mi = s_i[threadIdx.x];
            if (oi >= 0 && (mi < 0 || ov > mv || (ov == mv && oi < mi))) {
                s_v[threadIdx.x] = ov;
                s_i[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bp_corner c;
        c.x = s_i[0] < 0 ? -1 : (int32_t)(s_i[0] % w);
        c.y = s_i[0] < 0 ? -1 : (int32_t)(s_i[0] / w);
        c.response = s_i[0] < 0 ? 0 : s_v[0];
        out[blockIdx.x] = c;
    }
}

constexpr int kMaxPatchRadius = 15, kMaxSearchRadius = 32;
constexpr int kMaxRegion = 2 * (kMaxPatchRadius + kMaxSearchRadius) + 1;

// One block per corner: every shift in [-sr, sr]^2 whose patch lies inside
// frame b; the patch of frame a and the search region of frame b are staged
// in LDS.  The smallest n ZSSD wins, the first shift in row-major order on ties.
__global__ void __launch_bounds__(256) k_zssd(const uint8_t *__restrict__ a, const uint8_t *__restrict__ b, int w,
                                             int h, int64_t stride, const bp_corner *__restrict__ corners, int pr,
                                             int sr, bp_match *__restrict__ out)
{
    __shared__ uint8_t s_a[2 * kMaxPatchRadius + 1][2 * kMaxPatchRadius + 1];
    __shared__ uint8_t s_b[kMaxRegion][kMaxRegion];
    __shared__ int64_t s_c[256];
    __shared__ int32_t s_k[256];
    const bp_corner c = corners[blockIdx.x];
    const int P = 2 * pr + 1, S = 2 * sr + 1, G = P + 2 * sr;
    const bool ok = c.x >= pr && c.y >= pr && c.x + pr < w && c.y + pr < h;
    if (!ok) {
        if (threadIdx.x == 0) out[blockIdx.x] = bp_match{-1, -1, 0};
        return;
    }
    for (int i = threadIdx.x; i < P * P; i += 256) {
        const int j = i / P, k = i - j * P;
        s_a[j][k] = a[(int64_t)(c.y - pr + j) * stride + (c.x - pr + k)];
    }
    for (int i = threadIdx.x; i < G * G; i += 256) {
        const int j = i / G, k = i - j * G;
        const int x = c.x - sr - pr + k, y = c.y - sr - pr + j;
        s_b[j][k] = (x >= 0 && y >= 0 && x < w && y < h) ? b[(int64_t)y * stride + x] : (uint8_t)0;
    }
    __syncthreads();
    int64_t sa = 0;
    for (int j = 0; j < P; ++j)
        for (int k = 0; k < P; ++k) sa += s_a[j][k];
    const int64_t np = (int64_t)P * P;
    int64_t best = -1;
    int bk = -1;
    for (int s = threadIdx.x; s < S * S; s += 256) {
        const int dy = s / S - sr, dx = s % S - sr;
        const int qx = c.x + dx, qy = c.y + dy;
        if (qx < pr || qy < pr || qx + pr >= w || qy + pr >= h) continue;
        // 32-bit sums: at most 31^2 pixels, so sum (a - b)^2 <= 961 * 255^2 < 2^26.
        int32_t sd = 0, sb = 0;
        for (int j = 0; j < P; ++j)
            for (int k = 0; k < P; ++k) {
                const int32_t va = s_a[j][k], vb = s_b[dy + sr + j][dx + sr + k];
                sd += (va - vb) * (va - vb);
                sb += vb;
            }
        const int64_t cost = np * (int64_t)sd - (sa - (int64_t)sb) * (sa - (int64_t)sb);
        if (bk < 0 || cost < best) {       // s increases per thread: the first shift wins ties
            best = cost;
            bk = s;
        }
    }
    s_c[threadIdx.x] = best;
    s_k[threadIdx.x] = bk;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const int64_t oc = s_c[threadIdx.x + st];
            const int ok2 = s_k[threadIdx.x + st];
            const int64_t mc = s_c[threadIdx.x];
            const int mk = s_k[threadIdx.x];
            if (ok2 >= 0 && (mk < 0 || oc < mc || (oc == mc && ok2 < mk))) {
                s_c[threadIdx.x] = oc;
                s_k[threadIdx.x] = ok2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int k = s_k[0];
        out[blockIdx.x] = k < 0 ? bp_match{-1, -1, 0} : bp_match{c.x + (k % S - sr), c.y + (k / S - sr), s_c[0]};
    }
}

bp_status launch_harris(const uint8_t *img, int w, int h, int64_t stride, int g, int64_t thr, int64_t *r25,
                        bp_corner *corners, hipStream_t st)
{
    k_harris_response<<<dim3((unsigned)((w + kHT - 1) / kHT), (unsigned)((h + kHT - 1) / kHT)), 256, 0, st>>>(
        img, w, h, stride, r25);
    bp_status s = launch_status();
    if (s != BP_OK) return s;
    k_harris_select<<<(unsigned)(g * g), 256, 0, st>>>(r25, w, h, g, thr, corners);
    return launch_status();
}

bp_status launch_zssd(const uint8_t *a, const uint8_t *b, int w, int h, int64_t stride, const bp_corner *corners,
                      int n, int pr, int sr, bp_match *out, hipStream_t st)
{
    if (n == 0) return BP_OK;
    k_zssd<<<(unsigned)n, 256, 0, st>>>(a, b, w, h, stride, corners, pr, sr, out);
    return launch_status();
}

}  // namespace bpk
