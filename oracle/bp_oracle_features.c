/*
 * CPU oracle for the pose front end's data-parallel part (Sec. 2.3): the
 * Harris response (Eq. 4-5), the per-cell corner selection of the
 * experiments (a 30 x 30 grid of cells with a hard threshold), ZSSD patch
 * matching within a search range (all in exact integers), and the
 * correspondence step of ICP fine registration (FP32, see bpo_icp_correspond).
 *
 * TEST INFRASTRUCTURE ONLY (same rules as bp_oracle.c).
 *
 * Readings (the paper names the operations, not their discretisation):
 *  - first derivatives A, B of Eq. 4 are central differences without the
 *    1/2: A = I(x+1, y) - I(x-1, y), B = I(x, y+1) - I(x, y-1);
 *  - the Gaussian window w is the 5 x 5 binomial kernel (1 4 6 4 1)^T (1 4 6 4 1),
 *    the integer discrete Gaussian of variance 1;
 *  - M = sum w [A^2, AB; AB, B^2] and Eq. 5 with k = 1/25 (0.04, the usual
 *    Harris constant): the response is kept as the integer 25 R = 25 det M -
 *    tr(M)^2, so every quantity is exact in int64 and the selections below
 *    are decided without rounding; pixels closer than 3 to the border have
 *    response 0 (their window leaves the image);
 *  - cell (i, j) of a g x g grid covers columns [floor(j W / g), floor((j+1) W / g))
 *    and rows likewise; its corner is the pixel of largest response among
 *    those above the threshold that are 3 x 3 local maxima (no neighbour
 *    larger), the first in row-major order on ties, or none;
 *  - ZSSD between an n-pixel patch a of the first frame (centred on the
 *    corner) and a patch b of the second: sum((a - mean a) - (b - mean b))^2,
 *    kept as the integer n ZSSD = n sum (a - b)^2 - (sum a - sum b)^2; the
 *    match is the shift (dx, dy) in [-r, r]^2 whose patch lies inside the
 *    second frame with the smallest cost, the first in row-major (dy, dx)
 *    order on ties; none when the corner's own patch leaves the first frame.
 */
#include <stdint.h>
#include <stddef.h>

#define BPO_OK 0
#define BPO_EINVAL (-1)

static const int64_t kBin[5] = {1, 4, 6, 4, 1};

int bpo_harris_response(const uint8_t *img, int w, int h, int64_t *r25)
{
    if (!img || !r25 || w <= 0 || h <= 0) return BPO_EINVAL;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int64_t *o = r25 + (size_t)y * w + x;
            if (x < 3 || y < 3 || x > w - 4 || y > h - 4) {
                *o = 0;
                continue;
            }
            int64_t sxx = 0, syy = 0, sxy = 0;
            for (int j = -2; j <= 2; ++j)
                for (int i = -2; i <= 2; ++i) {
                    const int px = x + i, py = y + j;
                    const int64_t a = (int64_t)img[(size_t)py * w + px + 1] - img[(size_t)py * w + px - 1];
                    const int64_t b = (int64_t)img[(size_t)(py + 1) * w + px] - img[(size_t)(py - 1) * w + px];
                    const int64_t wt = kBin[i + 2] * kBin[j + 2];
                    sxx += wt * a * a;
                    syy += wt * b * b;
                    sxy += wt * a * b;
                }
            const int64_t det = sxx * syy - sxy * sxy, tr = sxx + syy;
            *o = 25 * det - tr * tr;
        }
    return BPO_OK;
}

/* corners: [g*g][3] int64 (x, y, 25 R), x = -1 for a cell without a corner. */
int bpo_harris_cells(const int64_t *r25, int w, int h, int g, int64_t threshold, int64_t *corners)
{
    if (!r25 || !corners || w <= 0 || h <= 0 || g <= 0) return BPO_EINVAL;
    for (int ci = 0; ci < g; ++ci)
        for (int cj = 0; cj < g; ++cj) {
            const int x0 = (int)((int64_t)cj * w / g), x1 = (int)((int64_t)(cj + 1) * w / g);
            const int y0 = (int)((int64_t)ci * h / g), y1 = (int)((int64_t)(ci + 1) * h / g);
            int bx = -1, by = -1;
            int64_t best = 0;
            for (int y = y0; y < y1; ++y)
                for (int x = x0; x < x1; ++x) {
                    const int64_t v = r25[(size_t)y * w + x];
                    if (v <= threshold) continue;
                    int peak = 1;
                    for (int j = -1; j <= 1 && peak; ++j)
                        for (int i = -1; i <= 1; ++i) {
                            const int nx = x + i, ny = y + j;
                            if ((i || j) && nx >= 0 && ny >= 0 && nx < w && ny < h && r25[(size_t)ny * w + nx] > v) {
                                peak = 0;
                                break;
                            }
                        }
                    if (peak && (bx < 0 || v > best)) {
                        best = v;
                        bx = x;
                        by = y;
                    }
                }
            int64_t *o = corners + ((size_t)ci * g + cj) * 3;
            o[0] = bx;
            o[1] = by;
            o[2] = bx < 0 ? 0 : best;
        }
    return BPO_OK;
}

/* matches: [n][3] int64 (x2, y2, n_pix * ZSSD), x2 = -1 when there is none. */
int bpo_zssd_match(const uint8_t *a, const uint8_t *b, int w, int h, const int64_t *corners, int n, int pr, int sr,
                   int64_t *matches)
{
    if (!a || !b || !corners || !matches || w <= 0 || h <= 0 || n < 0 || pr < 0 || sr < 0) return BPO_EINVAL;
    const int64_t np = (int64_t)(2 * pr + 1) * (2 * pr + 1);
    for (int k = 0; k < n; ++k) {
        const int64_t cx = corners[(size_t)k * 3], cy = corners[(size_t)k * 3 + 1];
        int64_t *o = matches + (size_t)k * 3;
        o[0] = -1;
        o[1] = -1;
        o[2] = 0;
        if (cx < pr || cy < pr || cx + pr >= w || cy + pr >= h) continue;
        int64_t best = -1;
        for (int dy = -sr; dy <= sr; ++dy)
            for (int dx = -sr; dx <= sr; ++dx) {
                const int64_t qx = cx + dx, qy = cy + dy;
                if (qx < pr || qy < pr || qx + pr >= w || qy + pr >= h) continue;
                int64_t sd = 0, sa = 0, sb = 0;
                for (int j = -pr; j <= pr; ++j)
                    for (int i = -pr; i <= pr; ++i) {
                        const int64_t va = a[(size_t)(cy + j) * w + (cx + i)];
                        const int64_t vb = b[(size_t)(qy + j) * w + (qx + i)];
                        sd += (va - vb) * (va - vb);
                        sa += va;
                        sb += vb;
                    }
                const int64_t cost = np * sd - (sa - sb) * (sa - sb);
                if (best < 0 || cost < best) {
                    best = cost;
                    o[0] = qx;
                    o[1] = qy;
                    o[2] = cost;
                }
            }
    }
    return BPO_OK;
}

/* ------------------------------------------------------------------ */
/* ICP correspondences (Sec. 2.3: ICP fine registration of the clouds). */
/* ------------------------------------------------------------------ */

/* One correspondence step of point-to-point ICP, decided in FP32 (the GPU
 * kernel's precision; every operation rounded on its own, in this order):
 *   p' = R p + T  (R row-major 3 x 3, T; p'_i = ((R_i0 p_0 + R_i1 p_1) + R_i2 p_2) + T_i)
 *   nearest target q_j by d2 = (dx dx + dy dy) + dz dz, dx = p'_x - q_x, ...,
 *   accepted when d2 <= dmax2; ties to the lowest j.  Brute force.
 * moved: [n][3] p'; corr: [n] index or -1; d2: [n]. */
int bpo_icp_correspond(const float *src, int n, const float *dst, int m, const float *R, const float *T, float dmax2,
                       float *moved, int32_t *corr, float *d2)
{
    if (!src || !dst || !R || !T || !moved || !corr || !d2 || n < 0 || m < 0) return BPO_EINVAL;
    for (int i = 0; i < n; ++i) {
        const float *p = src + (size_t)i * 3;
        float q[3];
        for (int r = 0; r < 3; ++r) {
            float acc = R[r * 3 + 0] * p[0];
            acc = acc + R[r * 3 + 1] * p[1];
            acc = acc + R[r * 3 + 2] * p[2];
            q[r] = acc + T[r];
        }
        moved[(size_t)i * 3] = q[0];
        moved[(size_t)i * 3 + 1] = q[1];
        moved[(size_t)i * 3 + 2] = q[2];
        int best = -1;
        float bd = 0.0f;
        for (int j = 0; j < m; ++j) {
            const float *t = dst + (size_t)j * 3;
            const float dx = q[0] - t[0], dy = q[1] - t[1], dz = q[2] - t[2];
            float d = dx * dx;
            d = d + dy * dy;
            d = d + dz * dz;
            if (d <= dmax2 && (best < 0 || d < bd)) {
                best = j;
                bd = d;
            }
        }
        corr[i] = best;
        d2[i] = best < 0 ? 0.0f : bd;
    }
    return BPO_OK;
}
