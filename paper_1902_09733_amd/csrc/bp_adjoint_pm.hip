// a8 on pixel-major states: the reverse half-sweep with the labels of a
// pixel spread over lanes, as in the forward pixel-major kernels (a sender
// pixel owns SEG lanes, R labels per lane, and handles its four outgoing
// messages k in turn, sharing the loads of its cost, incoming rows and
// adjoints and the partial sums of h).
//
// Per message the forward arithmetic is repeated exactly (same sums, same
// lane-local passes and cross-lane carries), now carrying the winner label
// along every minimum:
//   forward pass  A(f) = min(h(f), A(f-1) + lambda), the later label on ties
//                 (larger winner across lanes);
//   backward pass B(f) = min(A(f), B(f+1) + lambda), the current value on
//                 ties (smaller winner across lanes);
//   truncation    applies only when min h + lambda tau < B(f) strictly.
// Given the receiver slot's adjoint mb(f), h-bar(winner(f)) += mb(f) and
// h-bar(gmin) -= mb(f) for untruncated f, with the lambda / tau partials as
// in the label-major reverse step.  The scatter is deterministic in two
// phases through LDS: every lane posts (winner, mb) of its labels, then
// every lane adds, for each of its labels g, the posted mb of the labels f
// with winner g in increasing f.  An untruncated winner lies within tau of f
// (h(g) + lambda |f - g| <= min h + lambda tau), so f only ranges over a
// window of `win` labels around g (all labels when lambda = 0).
#include <hip/hip_runtime.h>

#include "bp_device.h"
#include "bp_internal.h"
#include "bp_pm_core.h"

namespace bpk {

// Level-0 geometry of a pixel-major level, passed by value to kernels.
struct PmDesc {
    int w, h, wh;
    int64_t blk, lp;
};

static PmDesc pm_desc(const Level &v) { return PmDesc{v.w, v.h, v.wh, v.blk, (int64_t)v.lp}; }

struct BwdPmArgs {
    const float *cost;      // level-0 cost, pixel-major
    uint32_t cost_bytes;
    const uint8_t *msg;     // state M_t, pixel-major float32
    uint32_t msg_bytes;
    float *mbar;            // adjoint of the message state, same layout
    uint32_t mbar_bytes;
    float *gcost;           // adjoint of the cost, pixel-major like `cost`
    float *partial;         // per-block (lambda, tau) partial sums
    int w, h, wh;
    uint32_t blk, lp;
    int colour, L, ncomp, win;
    int first;              // 1 for the first reverse step (t = K - 1)
    float lambda, tau, lt;
};

// Value and winner of lane (s - N) of the segment, or (inf, -1) below it.
template <int SEG, int N>
__device__ __forceinline__ void pair_from_lower(float v, int i, int s, float &ov, int &oi)
{
    ov = dpp_f<0x110 + N>(__builtin_huge_valf(), v);
    oi = dpp_i<0x110 + N>(-1, i);
    if constexpr (SEG < 16) {
        if (s < N) {
            ov = __builtin_huge_valf();
            oi = -1;
        }
    }
}

// Value and winner of lane (s + N) of the segment, or (inf, -1) above it.
template <int SEG, int N>
__device__ __forceinline__ void pair_from_upper(float v, int i, int s, float &ov, int &oi)
{
    ov = dpp_f<0x100 + N>(__builtin_huge_valf(), v);
    oi = dpp_i<0x100 + N>(-1, i);
    if constexpr (SEG < 16) {
        if (s + N >= SEG) {
            ov = __builtin_huge_valf();
            oi = -1;
        }
    }
}

// Exclusive prefix minimum over lanes 0..s-1 with its winner (ties: the
// larger winner, i.e. the nearer lane).
template <int SEG>
__device__ __forceinline__ void pair_prefix_excl(float u, int ui, int s, float &pv, int &pi)
{
    pair_from_lower<SEG, 1>(u, ui, s, pv, pi);
    auto step = [&](float ov, int oi) {
        if (ov < pv || (ov == pv && oi > pi)) {
            pv = ov;
            pi = oi;
        }
    };
    float ov;
    int oi;
    if constexpr (SEG > 1) {
        pair_from_lower<SEG, 1>(pv, pi, s, ov, oi);
        step(ov, oi);
    }
    if constexpr (SEG > 2) {
        pair_from_lower<SEG, 2>(pv, pi, s, ov, oi);
        step(ov, oi);
    }
    if constexpr (SEG > 4) {
        pair_from_lower<SEG, 4>(pv, pi, s, ov, oi);
        step(ov, oi);
    }
    if constexpr (SEG > 8) {
        pair_from_lower<SEG, 8>(pv, pi, s, ov, oi);
        step(ov, oi);
    }
}

// Exclusive suffix minimum over lanes s+1..SEG-1 with its winner (ties: the
// smaller winner, i.e. the nearer lane).
template <int SEG>
__device__ __forceinline__ void pair_suffix_excl(float v, int vi, int s, float &qv, int &qi)
{
    pair_from_upper<SEG, 1>(v, vi, s, qv, qi);
    auto step = [&](float ov, int oi) {
        if (ov < qv || (ov == qv && oi >= 0 && (qi < 0 || oi < qi))) {
            qv = ov;
            qi = oi;
        }
    };
    float ov;
    int oi;
    if constexpr (SEG > 1) {
        pair_from_upper<SEG, 1>(qv, qi, s, ov, oi);
        step(ov, oi);
    }
    if constexpr (SEG > 2) {
        pair_from_upper<SEG, 2>(qv, qi, s, ov, oi);
        step(ov, oi);
    }
    if constexpr (SEG > 4) {
        pair_from_upper<SEG, 4>(qv, qi, s, ov, oi);
        step(ov, oi);
    }
    if constexpr (SEG > 8) {
        pair_from_upper<SEG, 8>(qv, qi, s, ov, oi);
        step(ov, oi);
    }
}

template <int SEG, int R>
__device__ __forceinline__ void bwd_step_pm(const BwdPmArgs &a, uint32_t block)
{
    // The forward arithmetic is repeated exactly as the half-sweep kernels
    // do it: products rounded before they are added (bp_pm_core.h).
#pragma clang fp contract(off)
    constexpr int LP = SEG * R;           // labels stored per pixel
    constexpr int PPB = 256 / SEG;        // pixels per block
    // Posted mb and winner (a byte: labels are fewer than 128 here): per
    // pixel its four messages' rows of LP labels, each row preceded and
    // followed by PAD entries that post nothing (winner -1), so that a window
    // of up to PAD labels around a lane's labels needs no clamping at the
    // row's ends.
    static_assert(LP <= kMaxBackwardLabels && kMaxBackwardLabels <= 128, "winners must fit a signed byte");
    constexpr int PAD = 4;
    constexpr int PROW = 4 * (LP + PAD) + PAD;
    __shared__ float s_pv[PPB * PROW];
    __shared__ int8_t s_pw[PPB * PROW];
    __shared__ float s_part[4][2];
    const uint32_t gid = block * 256u + threadIdx.x;
    const int j = (int)(gid / SEG);
    const int s = (int)(gid % SEG);
    const int f0 = s * R;
    const int prow = (int)(threadIdx.x / SEG) * PROW;
    for (int e = (int)threadIdx.x; e < PPB * 5 * PAD; e += 256) {
        const int px = e / (5 * PAD), q = e - px * (5 * PAD);
        const int at = px * PROW + (q / PAD) * (LP + PAD) + q % PAD;
        s_pv[at] = 0.0f;
        s_pw[at] = -1;
    }
    bool live = j < a.ncomp;
    int y = 0, x = 0;
    if (live) {
        y = j / a.wh;
        x = 2 * (j - y * a.wh) + ((y + a.colour) & 1);
        live = x < a.w;
    }
    const uint32_t jj = live ? (uint32_t)j : 0u;
    const bool has[4] = {live && x > 0, live && x < a.w - 1, live && y > 0, live && y < a.h - 1};
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost, a.cost_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(a.msg, a.msg_bytes);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(a.mbar, a.mbar_bytes);
    const __amdgpu_buffer_rsrc_t rg = make_rsrc(a.gcost, a.cost_bytes);
    const float inf = __builtin_huge_valf();
    const float lam = a.lambda;
    const float lamR = lam * (float)R;
    const uint32_t base = jj * a.lp + (uint32_t)f0;

    // The four receiver slots' adjoints (zeros for a missing neighbour), the
    // cost adjoint this pixel accumulates, the cost and the four incoming
    // rows, all loaded before any arithmetic.  The receiver slots are not
    // cleared: every in-grid slot of the receivers' colour is overwritten by
    // the next reverse step's sender side before anything reads it again.
    float mbv[4][R];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t roff = 0;
        if (has[k]) {
            int nx = x, ny = y;
            if (k == 0) nx = x - 1;
            else if (k == 1) nx = x + 1;
            else if (k == 2) ny = y - 1;
            else ny = y + 1;
            const uint32_t dj = (uint32_t)(ny * a.wh + (nx >> 1));
            roff = (((uint32_t)(a.colour ^ 1) * 4u + (uint32_t)(k ^ 1)) * a.blk + dj * a.lp + (uint32_t)f0) * 4u;
        }
        ld_row<StoreF32, R>(rb, roff, mbv[k]);
#pragma unroll
        for (int r = 0; r < R; ++r) mbv[k][r] = has[k] ? mbv[k][r] : 0.0f;
    }
    const uint32_t goff = ((uint32_t)a.colour * a.blk + base) * 4u;
    float gc[R];
    if (live) ld_row<StoreF32, R>(rg, goff, gc);
    // h of the four outgoing messages, summed as in the forward kernels.
    float h[4][R];
    {
        float c[R], m[4][R];
        ld_row<StoreF32, R>(rc, ((uint32_t)a.colour * a.blk + base) * 4u, c);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            ld_row<StoreF32, R>(rm, (((uint32_t)a.colour * 4u + (uint32_t)kk) * a.blk + base) * 4u, m[kk]);
        pm_h4<R>(c, m, h);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (f0 + r >= a.L) h[k][r] = inf;
    }

    // Phase 1, message by message: the transform with winners, then post
    // (winner, mb) of the receiver slot's adjoint.
    float lsum = 0.0f, tsum = 0.0f, nsum[4];
    int gmin[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // Lowest minimiser of h.
        float hmin = inf;
        int gm = 0;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (h[k][r] < hmin) {
                hmin = h[k][r];
                gm = f0 + r;
            }
        seg_argmin<SEG>(hmin, gm);
        gmin[k] = gm;
        // Forward pass with winners.
        float A[R];
        int wa[R];
        A[0] = h[k][0];
        wa[0] = f0;
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const float v = A[r - 1] + lam;
            const bool keep = h[k][r] <= v;
            A[r] = keep ? h[k][r] : v;
            wa[r] = keep ? f0 + r : wa[r - 1];
        }
        {
            float pv;
            int pi;
            pair_prefix_excl<SEG>(A[R - 1] - lamR * (float)s, wa[R - 1], s, pv, pi);
            const float carry = pv + lamR * (float)(s - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float cand = carry + lam * (float)(r + 1);
                if (cand < A[r]) {
                    A[r] = cand;
                    wa[r] = pi;
                }
            }
        }
        // Backward pass with winners.
        float B[R];
        int wb[R];
        B[R - 1] = A[R - 1];
        wb[R - 1] = wa[R - 1];
#pragma unroll
        for (int r = R - 2; r >= 0; --r) {
            const float v = B[r + 1] + lam;
            const bool take = v < A[r];
            B[r] = take ? v : A[r];
            wb[r] = take ? wb[r + 1] : wa[r];
        }
        {
            float qv;
            int qi;
            pair_suffix_excl<SEG>(B[0] + lamR * (float)s, wb[0], s, qv, qi);
            const float carry = qv - lamR * (float)(s + 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float cand = carry + lam * (float)(R - r);
                if (cand < B[r]) {
                    B[r] = cand;
                    wb[r] = qi;
                }
            }
        }
        const float cap = hmin + a.lt;
        float ns = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int f = f0 + r;
            const float mb = f < a.L ? mbv[k][r] : 0.0f;
            int src = -1;
            float post = 0.0f;
            if (cap < B[r]) {
                lsum += mb * a.tau;
                tsum += mb * a.lambda;
            } else {
                src = wb[r];
                post = mb;
                ns += mb;
                lsum += mb * fabsf((float)(f - src));
            }
            s_pv[prow + PAD + k * (LP + PAD) + f] = post;
            s_pw[prow + PAD + k * (LP + PAD) + f] = (int8_t)src;
        }
        nsum[k] = ns;
    }
    __syncthreads();

    // Phase 2: h-bar of this lane's labels for each message.  One pass over
    // the posts that can reach them (winners lie within `win` of their
    // label); every h-bar(g) still adds its posts in increasing f.
    float hb[4][R];
    const int lo = f0 - a.win > 0 ? f0 - a.win : 0;
    const int hi = f0 + R - 1 + a.win < LP - 1 ? f0 + R - 1 + a.win : LP - 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float ntot = seg_allreduce<SEG>(nsum[k], [](float p, float q) { return p + q; });
#pragma unroll
        for (int r = 0; r < R; ++r) hb[k][r] = 0.0f;
        const int row = prow + PAD + k * (LP + PAD);
        if (a.win <= PAD) {
            // Every lane the same count of posts, the pads past the row's
            // ends included (they match no label).
            const int n = R + 2 * a.win, p0 = row + f0 - a.win;
            for (int i = 0; i < n; ++i) {
                const float pv = s_pv[p0 + i];
                const int wv = s_pw[p0 + i];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (wv == f0 + r) hb[k][r] += pv;
            }
        } else {
            for (int f = lo; f <= hi; ++f) {
                const float pv = s_pv[row + f];
                const int d = (int)s_pw[row + f] - f0;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (d == r) hb[k][r] += pv;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (f0 + r == gmin[k]) hb[k][r] -= ntot;
    }

    // Sender side: cost-bar += sum over messages; slot k's adjoint gets the
    // other three messages' h-bar, added to the readout adjoint at the first
    // reverse step and written over the consumed value afterwards.
    float tot[R];
#pragma unroll
    for (int r = 0; r < R; ++r) tot[r] = (hb[0][r] + hb[1][r]) + (hb[2][r] + hb[3][r]);
    if (live) {
#pragma unroll
        for (int r = 0; r < R; ++r) gc[r] += tot[r];
        st_row<StoreF32, R>(rg, goff, gc);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!has[k]) continue;
        const uint32_t moff = (((uint32_t)a.colour * 4u + (uint32_t)k) * a.blk + base) * 4u;
        float cur[R];
        if (a.first) {
            ld_row<StoreF32, R>(rb, moff, cur);
#pragma unroll
            for (int r = 0; r < R; ++r) cur[r] += tot[r] - hb[k][r];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) cur[r] = tot[r] - hb[k][r];
        }
        st_row<StoreF32, R>(rb, moff, cur);
    }

    // Block sums of the lambda and tau partials: per wavefront by shuffles,
    // then the four wavefronts in order.
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lsum += __shfl_xor(lsum, o, 64);
        tsum += __shfl_xor(tsum, o, 64);
    }
    if (threadIdx.x % 64 == 0) {
        s_part[threadIdx.x / 64][0] = lsum;
        s_part[threadIdx.x / 64][1] = tsum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.partial[2 * block] = ((s_part[0][0] + s_part[1][0]) + s_part[2][0]) + s_part[3][0];
        a.partial[2 * block + 1] = ((s_part[0][1] + s_part[1][1]) + s_part[2][1]) + s_part[3][1];
    }
}

struct BwdPmEntry {
    BwdPmArgs a;
    int block0;
    int pad[3];
};
constexpr int kBwdPmChunk = 16;
struct BwdPmChunk {
    BwdPmEntry e[kBwdPmChunk];
    int n;
};

__global__ void k_write_bwd_pm_entries(BwdPmEntry *__restrict__ dst, BwdPmChunk c)
{
    const int i = threadIdx.x;
    if (i < c.n) dst[i] = c.e[i];
}

// The reverse half-sweep of several problems (same lane split) in one
// launch: block b belongs to the last entry whose first block is <= b.
template <int SEG, int R>
__global__ void __launch_bounds__(256) k_bwd_step_pm_batch(const BwdPmEntry *__restrict__ tab, int n)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    bwd_step_pm<SEG, R>(tab[lo].a, blockIdx.x - (uint32_t)tab[lo].block0);
}

// Readout adjoint on pixel-major states: b = cost + the four incoming rows
// (summed as the forward readout sums them), d = sum f p_f with p =
// softmax(-b / T); b-bar(f) = -(g / T) p_f (f - d).  Initialises the cost
// adjoint and every in-grid incoming slot of the message adjoint.  Grid
// (ncomp * SEG / 256, 2 colours).
template <int SEG, int R>
__global__ void __launch_bounds__(256) k_bwd_readout_pm(const float *__restrict__ cost, uint32_t cost_bytes,
                                                       const uint8_t *__restrict__ msg, uint32_t msg_bytes,
                                                       float *__restrict__ mbar, float *__restrict__ gcost,
                                                       const float *__restrict__ grad_soft, PmDesc d, int L,
                                                       float inv_t)
{
    const int c = blockIdx.y;
    const int gid = blockIdx.x * 256 + threadIdx.x;
    const int j = gid / SEG, s = gid % SEG;
    if (j >= d.h * d.wh) return;
    const int y = j / d.wh;
    const int x = 2 * (j - y * d.wh) + ((y + c) & 1);
    if (x >= d.w) return;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(cost, cost_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(msg, msg_bytes);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(mbar, msg_bytes);
    const __amdgpu_buffer_rsrc_t rg = make_rsrc(gcost, cost_bytes);
    const int f0 = s * R;
    const uint32_t lp = (uint32_t)d.lp, blk = (uint32_t)d.blk;
    const uint32_t base = (uint32_t)j * lp + (uint32_t)f0;
    float b[R], m[4][R];
    ld_row<StoreF32, R>(rc, ((uint32_t)c * blk + base) * 4u, b);
#pragma unroll
    for (int k = 0; k < 4; ++k) ld_row<StoreF32, R>(rm, (((uint32_t)c * 4u + (uint32_t)k) * blk + base) * 4u, m[k]);
    const float inf = __builtin_huge_valf();
    float bmin = inf;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        b[r] = (((b[r] + m[0][r]) + m[1][r]) + m[2][r]) + m[3][r];
        if (f0 + r >= L) b[r] = inf;
        bmin = fminf(bmin, b[r]);
    }
    bmin = seg_allreduce<SEG>(bmin, [](float p, float q) { return fminf(p, q); });
    float wgt[R], num = 0.0f, den = 0.0f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        wgt[r] = f0 + r < L ? expf(-(b[r] - bmin) * inv_t) : 0.0f;
        num += (float)(f0 + r) * wgt[r];
        den += wgt[r];
    }
    auto add = [](float p, float q) { return p + q; };
    num = seg_allreduce<SEG>(num, add);
    den = seg_allreduce<SEG>(den, add);
    const float dd = num / den;
    const float g = grad_soft[(int64_t)y * d.w + x];
    float bb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) bb[r] = f0 + r < L ? -g * inv_t * (wgt[r] / den) * ((float)(f0 + r) - dd) : 0.0f;
    st_row<StoreF32, R>(rg, ((uint32_t)c * blk + base) * 4u, bb);
    const bool has[4] = {x > 0, x < d.w - 1, y > 0, y < d.h - 1};
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (has[k]) st_row<StoreF32, R>(rb, (((uint32_t)c * 4u + (uint32_t)k) * blk + base) * 4u, bb);
}

// Pixel-major cost adjoint -> planar [L][h][w] output, through an LDS tile
// of 32 consecutive pixels of one row (their rows of both colours read as
// contiguous runs, labels written as 128-byte runs of x).  Rows padded by
// one word against bank conflicts.  grid (ceil(w / 32), h).
template <int LP>
__global__ void __launch_bounds__(256) k_gcost_to_planar(const float *__restrict__ gcost, PmDesc d, int L,
                                                        float *__restrict__ out)
{
    __shared__ float tile[32][LP + 1];
    const int x0 = blockIdx.x * 32, y = blockIdx.y;
    // Load: 32 pixels x LP labels; pixel p of the tile is x0 + p.
    for (int e = threadIdx.x; e < 32 * LP; e += 256) {
        const int p = e / LP, f = e - p * LP;
        const int x = x0 + p;
        if (x < d.w) {
            const int c = (x + y) & 1;
            tile[p][f] = gcost[(int64_t)c * d.blk + ((int64_t)y * d.wh + (x >> 1)) * d.lp + f];
        }
    }
    __syncthreads();
    const int64_t plane = (int64_t)d.h * d.w;
    for (int e = threadIdx.x; e < 32 * L; e += 256) {
        const int f = e / 32, p = e - f * 32;
        const int x = x0 + p;
        if (x < d.w) out[(int64_t)f * plane + (int64_t)y * d.w + x] = tile[p][f];
    }
}

// The same transpose with 16-byte accesses both ways (w % 4 == 0, 16-byte
// aligned output): a block moves 64 pixels of one row x 64 labels through
// LDS, loading four consecutive labels of one pixel per lane (a pixel's
// labels are contiguous) and storing four consecutive pixels of one label.
// grid (w / 64, h, L / 64).
__global__ void __launch_bounds__(256) k_gcost_to_planar4(const float *__restrict__ gcost, PmDesc d, int L,
                                                         float *__restrict__ out)
{
    __shared__ float tile[64][65];
    const int x0 = blockIdx.x * 64, y = blockIdx.y, f0 = blockIdx.z * 64;
    const int t = threadIdx.x, q = t & 15, r = t >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int xl = r + 16 * i, x = x0 + xl, f = f0 + 4 * q;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (x < d.w && f < L) {
            const int c = (x + y) & 1;
            v = *(const float4 *)(gcost + (int64_t)c * d.blk + ((int64_t)y * d.wh + (x >> 1)) * d.lp + f);
        }
        tile[4 * q][xl] = v.x;
        tile[4 * q + 1][xl] = v.y;
        tile[4 * q + 2][xl] = v.z;
        tile[4 * q + 3][xl] = v.w;
    }
    __syncthreads();
    const int64_t plane = (int64_t)d.h * d.w;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int fl = r + 16 * i, f = f0 + fl, x = x0 + 4 * q;
        if (f < L && x < d.w)
            *(float4 *)(out + f * plane + (int64_t)y * d.w + x) =
                make_float4(tile[fl][4 * q], tile[fl][4 * q + 1], tile[fl][4 * q + 2], tile[fl][4 * q + 3]);
    }
}

int bwd_pm_blocks(const Plan &p)
{
    int S, R;
    pm_split(p.L, &S, &R);
    return (int)(((int64_t)p.lv[0].h * p.lv[0].wh * S + 255) / 256);
}

bp_status launch_bwd_readout_pm(const Plan &p, const uint8_t *msg, float *mbar, float *gcost, const float *grad_soft,
                                float temperature, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[0];
    const int64_t ncomp = (int64_t)v.h * v.wh;
    int S, R;
    pm_split(p.L, &S, &R);
    const float *cost = (const float *)(ws + v.cost_off);
    const float inv_t = 1.0f / temperature;
#define BP_RPM(SV, RV)                                                                                             \
    if (S == SV && R == RV) {                                                                                      \
        k_bwd_readout_pm<SV, RV><<<dim3((unsigned)((ncomp * SV + 255) / 256), 2), 256, 0, s>>>(                    \
            cost, (uint32_t)v.cost_bytes, msg, (uint32_t)v.msg_bytes, mbar, gcost, grad_soft, pm_desc(v), p.L, inv_t); \
        return launch_status();                                                                                    \
    }
    BP_RPM(4, 4) BP_RPM(8, 4) BP_RPM(16, 4) BP_RPM(16, 6) BP_RPM(16, 8)
#undef BP_RPM
    return BP_ERR_UNSUPPORTED;
}

bp_status launch_gcost_to_planar(const Plan &p, const float *gcost, float *grad_cost, hipStream_t s)
{
    const Level &v = p.lv[0];
    if (v.w % 4 == 0 && ((uintptr_t)grad_cost % 16) == 0) {
        k_gcost_to_planar4<<<dim3((unsigned)((v.w + 63) / 64), (unsigned)v.h, (unsigned)((p.L + 63) / 64)), 256, 0, s>>>(
            gcost, pm_desc(v), p.L, grad_cost);
        return launch_status();
    }
    const dim3 grid((unsigned)((v.w + 31) / 32), (unsigned)v.h);
    switch (v.lp) {
    case 16: k_gcost_to_planar<16><<<grid, 256, 0, s>>>(gcost, pm_desc(v), p.L, grad_cost); break;
    case 32: k_gcost_to_planar<32><<<grid, 256, 0, s>>>(gcost, pm_desc(v), p.L, grad_cost); break;
    case 64: k_gcost_to_planar<64><<<grid, 256, 0, s>>>(gcost, pm_desc(v), p.L, grad_cost); break;
    case 96: k_gcost_to_planar<96><<<grid, 256, 0, s>>>(gcost, pm_desc(v), p.L, grad_cost); break;
    case 128: k_gcost_to_planar<128><<<grid, 256, 0, s>>>(gcost, pm_desc(v), p.L, grad_cost); break;
    default: return BP_ERR_UNSUPPORTED;
    }
    return launch_status();
}

size_t bwd_pm_table_bytes(int count) { return align_up((size_t)count * sizeof(BwdPmEntry)); }

bp_status launch_bwd_step_pm_batch(const BwdPmProblem *probs, int count, int t, bool first_step, float lambda,
                                   float tau, uint8_t *table, hipStream_t s)
{
    BwdPmEntry *dev = (BwdPmEntry *)table;
    bool *done = new bool[count]();
    BwdPmEntry *host = new BwdPmEntry[count];
    bp_status st = BP_OK;
    int used = 0;
    // One launch per lane split (the kernel's template arguments).
    for (int i = 0; i < count && st == BP_OK; ++i) {
        if (done[i]) continue;
        int S, R;
        pm_split(probs[i].plan->L, &S, &R);
        const int first = used;
        int blocks = 0;
        for (int k = i; k < count; ++k) {
            int Sk, Rk;
            pm_split(probs[k].plan->L, &Sk, &Rk);
            if (done[k] || Sk != S || Rk != R) continue;
            done[k] = true;
            const Plan &p = *probs[k].plan;
            const Level &v = p.lv[0];
            BwdPmEntry &e = host[used++];
            BwdPmArgs &a = e.a;
            a.cost = (const float *)(probs[k].ws + v.cost_off);
            a.cost_bytes = (uint32_t)v.cost_bytes;
            a.msg = probs[k].state;
            a.msg_bytes = (uint32_t)v.msg_bytes;
            a.mbar = probs[k].mbar;
            a.mbar_bytes = (uint32_t)v.msg_bytes;
            a.gcost = probs[k].gcost;
            a.partial = probs[k].partial;
            a.w = v.w;
            a.h = v.h;
            a.wh = v.wh;
            a.blk = (uint32_t)v.blk;
            a.lp = (uint32_t)v.lp;
            a.colour = t & 1;
            a.L = p.L;
            a.ncomp = v.h * v.wh;
            // Untruncated winners lie within tau of their label; two labels of
            // margin cover rounding.  Without smoothness any label can win.
            a.win = lambda > 0.0f ? (int)std::min((float)(v.lp - 1), std::floor(tau) + 2.0f) : v.lp - 1;
            a.first = first_step ? 1 : 0;
            a.lambda = lambda;
            a.tau = tau;
            a.lt = lambda * tau;
            e.block0 = blocks;
            blocks += bwd_pm_blocks(p);
        }
        for (int c0 = first; c0 < used && st == BP_OK; c0 += kBwdPmChunk) {
            BwdPmChunk c;
            c.n = used - c0 < kBwdPmChunk ? used - c0 : kBwdPmChunk;
            for (int k = 0; k < c.n; ++k) c.e[k] = host[c0 + k];
            k_write_bwd_pm_entries<<<1, 64, 0, s>>>(dev + c0, c);
            st = launch_status();
        }
        if (st != BP_OK) break;
        const int n = used - first;
        const BwdPmEntry *tab = dev + first;
#define BP_BPM(SV, RV)                                                                                             \
    if (S == SV && R == RV) {                                                                                      \
        k_bwd_step_pm_batch<SV, RV><<<blocks, 256, 0, s>>>(tab, n);                                                \
        st = launch_status();                                                                                      \
        continue;                                                                                                  \
    }
        BP_BPM(4, 4) BP_BPM(8, 4) BP_BPM(16, 4) BP_BPM(16, 6) BP_BPM(16, 8)
#undef BP_BPM
        st = BP_ERR_UNSUPPORTED;
    }
    delete[] done;
    delete[] host;
    return st;
}

}  // namespace bpk
