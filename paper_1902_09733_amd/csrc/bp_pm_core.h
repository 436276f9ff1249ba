// The per-message arithmetic of a pixel-major half-sweep, shared by the
// one-half-sweep kernels (bp_iter_pm.hip) and the fused pair of half-sweeps
// (bp_iter_pm2_impl.h): the distance transform of h over a message's SEG lanes
// (R labels per lane), truncation and normalisation, and the readout of a
// belief (argmin and soft-argmin, also used by the readout pass).  The identities behind the split scans are in bp_iter_pm.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "bp_device.h"

namespace bpk {

// out(f) = min(min_g h(g) + lambda |f - g|, min h + lt) - min h for the
// labels [s R, s R + R) of lane s of its segment; labels at or past L must
// hold +inf in h unless EXACT (L == SEG * R).
//
// The minimum over g splits by where g lies: in the lane itself (the two
// lane-local passes), in a lower lane (the exclusive prefix scan of the local
// forward values, entering at label s R - 1) or in a higher lane (the
// exclusive suffix scan of the local backward values, entering at label
// s R + R); the three candidates meet in one three-way minimum per label.  The
// two scans and the segment minimum of h are independent, so they run
// interleaved.
//
// Every product is rounded before it is added (no multiply-add contraction):
// the compiler would otherwise fuse or not depending on what it hoists out of
// the calling kernel's loops, and two kernels running this transform on the
// same data (one half-sweep per launch, or two) must agree bit for bit.
//
// With a truncation of at most 1 + W labels (W = 1 for tau <= 2, W = 2 for
// tau <= 3) a label g more than W labels from f costs
// h(g) + lambda min(|f - g|, tau) = h(g) + lambda tau >= min h + lt, never less
// than the truncation cap, so only the labels within W of f remain:
//   out(f) = min(min_{|g - f| <= W} h(g) + lambda |f - g|, min h + lt) - min h,
// the same function without the passes and scans (pm_transform_near).
// Calls f with std::integral_constant<int, W> for a uniform run-time W (0 for
// the two-pass transform): a loop over a pixel's four messages is then
// compiled once per form of the transform (a branch inside it would keep the
// messages' code apart).  The five-label form (W = 2) is used with four labels
// per lane; with more, its extra rows of h + 2 lambda cost registers and
// occupancy (at 128 labels, eight per lane, it was slower than the scans), so
// those lanes keep the scans.
template <int R, typename F>
__device__ __forceinline__ void with_near(int w, F &&f)
{
    if (w == 1) {
        f(std::integral_constant<int, 1>{});
    } else {
        if constexpr (R <= 4) {
            if (w == 2) {
                f(std::integral_constant<int, 2>{});
                return;
            }
        }
        f(std::integral_constant<int, 0>{});
    }
}

template <int SEG, int R, bool EXACT, int W>
__device__ __forceinline__ void pm_transform_near(float (&h)[R], int s, int f0, int L, float lam, float lt,
                                                  float (&out)[R])
{
#pragma clang fp contract(off)
    static_assert(W == 1 || W == 2, "window of one or two labels");
    static_assert(R >= 2 * W, "a lane holds at least 2W labels");
    const float inf = __builtin_huge_valf();
    float hmin = inf;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!EXACT && f0 + r >= L) h[r] = inf;
        hmin = fminf(hmin, h[r]);
    }
    float hp[R];   // h + lambda
#pragma unroll
    for (int r = 0; r < R; ++r) hp[r] = h[r] + lam;
    float e[2 * W];   // the lane's first W and last W labels, with the neighbouring lanes' candidates
    if constexpr (W == 1) {
        e[0] = h[0];
        e[1] = h[R - 1];
        seg_near<SEG>(e[0], e[1], hmin, hp[R - 1], hp[0], s);
    }
    float hq[W == 2 ? R : 1];   // h + 2 lambda
    if constexpr (W == 2) {
        const float lam2 = lam + lam;
#pragma unroll
        for (int r = 0; r < R; ++r) hq[r] = h[r] + lam2;
        // The lane below offers its last two labels to this lane's first two,
        // the lane above its first two to this lane's last two.
        e[0] = h[0];
        e[1] = h[1];
        e[2] = h[R - 2];
        e[3] = h[R - 1];
        seg_near2<SEG>(e, hmin, fminf(hp[R - 1], hq[R - 2]), hq[R - 1], fminf(hp[0], hq[1]), hq[0], s);
    }
    const float cap = hmin + lt;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float v = r < W ? e[r] : r >= R - W ? e[2 * W - R + r] : h[r];
        if (r >= 1) v = fminf(v, hp[r - 1]);
        if (r + 1 < R) v = fminf(v, hp[r + 1]);
        if constexpr (W == 2) {
            if (r >= 2) v = fminf(v, hq[r - 2]);
            if (r + 2 < R) v = fminf(v, hq[r + 2]);
        }
        out[r] = fminf(v, cap) - hmin;
    }
}

template <int SEG, int R, bool EXACT, int W>
__device__ __forceinline__ void pm_transform(float (&h)[R], int s, int f0, int L, float lam, float lt, float (&out)[R])
{
#pragma clang fp contract(off)
    if constexpr (W > 0) {
        pm_transform_near<SEG, R, EXACT, W>(h, s, f0, L, lam, lt, out);
        return;
    }
    const float inf = __builtin_huge_valf();
    const float lamR = lam * (float)R;
    float hmin = inf;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!EXACT && f0 + r >= L) h[r] = inf;
        hmin = fminf(hmin, h[r]);
    }
    // Lane-local forward and backward passes.
    float A[R], B[R];
    A[0] = h[0];
#pragma unroll
    for (int r = 1; r < R; ++r) A[r] = fminf(h[r], A[r - 1] + lam);
    B[R - 1] = A[R - 1];
#pragma unroll
    for (int r = R - 2; r >= 0; --r) B[r] = fminf(A[r], B[r + 1] + lam);
    // From the lanes below: min over s' < s of A_s'(last) - lambda R s';
    // from the lanes above: min over s' > s of B_s'(first) + lambda R s'.
    float P = seg_from_lower<SEG, 1>(A[R - 1] - lamR * (float)s, inf, s);
    float Q = seg_from_upper<SEG, 1>(B[0] + lamR * (float)s, inf, s);
    seg_scans<SEG>(P, Q, hmin, s);
    const float lc = P + lamR * (float)(s - 1);
    const float rc = Q - lamR * (float)(s + 1);
    const float cap = hmin + lt;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float t = fminf(fminf(B[r], lc + lam * (float)(r + 1)), rc + lam * (float)(R - r));
        out[r] = fminf(t, cap) - hmin;
    }
}

// h for outgoing message k (to the neighbour on side k): the cost plus the
// incoming rows of the other three slots, added in slot order.
template <int R>
__device__ __forceinline__ void pm_h(const float (&c)[R], const float (&m)[4][R], int k, float (&h)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (k == 0) h[r] = ((c[r] + m[1][r]) + m[2][r]) + m[3][r];
        else if (k == 1) h[r] = ((c[r] + m[0][r]) + m[2][r]) + m[3][r];
        else if (k == 2) h[r] = ((c[r] + m[0][r]) + m[1][r]) + m[3][r];
        else h[r] = ((c[r] + m[0][r]) + m[1][r]) + m[2][r];
    }
}

// The four h rows of pm_h at once, sharing the partial sums cost + m0 and
// cost + m0 + m1 (the same additions in the same order).
template <int R>
__device__ __forceinline__ void pm_h4(const float (&c)[R], const float (&m)[4][R], float (&h)[4][R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float p0 = c[r] + m[0][r];
        const float p01 = p0 + m[1][r];
        h[0][r] = ((c[r] + m[1][r]) + m[2][r]) + m[3][r];
        h[1][r] = (p0 + m[2][r]) + m[3][r];
        h[2][r] = p01 + m[3][r];
        h[3][r] = p01 + m[2][r];
    }
}

// Belief cost + all four incoming rows, in slot order (readout).
template <int R>
__device__ __forceinline__ void pm_belief(const float (&c)[R], const float (&m)[4][R], float (&b)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) b[r] = (((c[r] + m[0][r]) + m[1][r]) + m[2][r]) + m[3][r];
}

// Receiver of message k from (x, y): its coordinates, and whether it is in
// the grid (0 left, 1 right, 2 up, 3 down).
__device__ __forceinline__ bool pm_receiver(int k, int x, int y, int w, int h, int &nx, int &ny)
{
    nx = x;
    ny = y;
    if (k == 0) { nx = x - 1; return x > 0; }
    if (k == 1) { nx = x + 1; return x < w - 1; }
    if (k == 2) { ny = y - 1; return y > 0; }
    ny = y + 1;
    return y < h - 1;
}

// Lowest label minimising the belief over the segment; labels at or past L
// are ignored unless EXACT.
template <int SEG, int R, bool EXACT>
__device__ __forceinline__ int pm_argmin(const float (&bel)[R], int f0, int L)
{
    const float inf = __builtin_huge_valf();
    float bv = inf;
    int bi = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float b = bel[r];
        if (!EXACT && f0 + r >= L) b = inf;
        if (b < bv) {
            bv = b;
            bi = f0 + r;
        }
    }
    seg_argmin<SEG>(bv, bi);
    return bi;
}

// Readout of a pixel from its belief (Eq. 1's minimiser): the lowest label
// minimising it over the segment and, when soft, the soft-argmin
//   sum_f f w(f) / sum_f w(f),  w(f) = exp(-(b(f) - min b) / T)
// (inv_t = 1 / T), both on every lane.  Labels at or past L are ignored
// (there are none when EXACT, L == SEG * R).  Products are rounded before
// they are added, so that every kernel reading out a pixel (the readout pass,
// the fused pair's last phase) agrees bit for bit.
template <int SEG, int R, bool EXACT>
__device__ __forceinline__ void pm_readout(const float (&bel)[R], int f0, int L, bool soft, float inv_t, int &bi,
                                           float &sv)
{
#pragma clang fp contract(off)
    const float inf = __builtin_huge_valf();
    float b[R];
    float bv = inf;
    bi = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        b[r] = (EXACT || f0 + r < L) ? bel[r] : inf;
        if (b[r] < bv) {
            bv = b[r];
            bi = f0 + r;
        }
    }
    seg_argmin<SEG>(bv, bi);
    sv = 0.0f;
    if (soft) {
        float num = 0.0f, den = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (EXACT || f0 + r < L) {
                const float wgt = expf(-(b[r] - bv) * inv_t);
                num += (float)(f0 + r) * wgt;
                den += wgt;
            }
        }
        auto add = [](float p, float q) { return p + q; };
        num = seg_allreduce<SEG>(num, add);
        den = seg_allreduce<SEG>(den, add);
        sv = num / den;
    }
}

}  // namespace bpk
