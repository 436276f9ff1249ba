// a8: reverse-mode derivative of single-level checkerboard BP with a
// soft-argmin readout (the differentiation form).
//
// The forward pass is piecewise linear in the data term, lambda and tau.  For
// the message p -> q at half-sweep t and every output label f:
//   untruncated: m(f) = h(gB) + lambda |f - gB| - h(gmin)
//   truncated:   m(f) = lambda tau
// where gB is the label the two passes of the distance transform carried to
// f and gmin the lowest minimiser of h = cost + incoming messages except q's.
// Given the adjoint of m (accumulated in the receiver's slot), the reverse
// step scatters it to h (gB: +, gmin: -), adds lambda/tau partials, passes
// h's adjoint to the sender's cost and to its other three incoming slots, and
// clears the receiver slot's adjoint (that slot was overwritten at step t).
// Tie rules follow the forward kernels and the oracle: the forward pass keeps
// h(f) when it equals the carried value, the backward pass keeps the current
// value, truncation applies only when min h + lambda tau is strictly smaller.
//
// States M_t are recomputed from checkpoints saved by the forward call, one
// reverse step at a time.  Layout: label-major levels (lanes over pixels, 4
// lanes per pixel = one outgoing message each); the scatter target h-bar(g)
// lives in an LDS row per lane.
#include <hip/hip_runtime.h>

#include "bp_device.h"
#include "bp_internal.h"

namespace bpk {

struct BwdArgs {
    const float *cost;      // colour-split cost of the level (label-major)
    uint32_t cost_bytes;
    const uint8_t *msg;     // state M_t (label-major, float32)
    uint32_t msg_bytes;
    float *mbar;            // adjoint of the message state, same layout
    uint32_t mbar_bytes;
    float *grad_cost;       // planar [L][h][w]
    float *partial;         // per-block (lambda, tau) partial sums
    int w, h, wh;
    uint32_t blk, ls;       // label-major strides (ps = 1)
    int colour, L, ncomp;
    float lambda, tau;
};

// One reverse half-sweep.  64 threads per block: 16 sender pixels x 4
// outgoing messages.  grid = ceil(ncomp / 16).
template <int LP, bool EXACT>
__global__ void __launch_bounds__(64) k_bwd_step(const BwdArgs a)
{
    extern __shared__ float hb_all[];          // [64][LP]
    float *hb = hb_all + threadIdx.x * LP;
    const int nl = EXACT ? LP : a.L;
    const int j = blockIdx.x * 16 + (threadIdx.x >> 2);
    const int q = threadIdx.x & 3;
    const float inf = __builtin_huge_valf();
    float lsum = 0.0f, tsum = 0.0f;
    bool live = j < a.ncomp;
    int y = 0, x = 0;
    if (live) {
        y = j / a.wh;
        x = 2 * (j - y * a.wh) + ((y + a.colour) & 1);
        live = x < a.w;
    }
    bool has[4] = {live && x > 0, live && x < a.w - 1, live && y > 0, live && y < a.h - 1};
    const bool hq = has[q];
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost, a.cost_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(a.msg, a.msg_bytes);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(a.mbar, a.mbar_bytes);
    const uint32_t jj = live ? (uint32_t)j : 0u;
    const uint32_t cls = a.ls * 4u;
    const uint32_t cost_off = ((uint32_t)a.colour * a.blk + jj) * 4u;
    uint32_t moff[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) moff[k] = (((uint32_t)a.colour * 4u + (uint32_t)k) * a.blk + jj) * 4u;

    // Distance transform of h with winners (registers, fully unrolled).
    float A[LP];
    int src[LP];
    float hmin = inf;
    int gmin = 0;
#pragma unroll
    for (int f = 0; f < LP; ++f) {
        float h = inf;
        if (EXACT || f < nl) {
            h = ld_f32(rc, cost_off, (uint32_t)f * cls);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float m = ld_f32(rm, moff[k], (uint32_t)f * cls);
                h += (k == q) ? 0.0f : m;
            }
        }
        if (h < hmin) {
            hmin = h;
            gmin = f;
        }
        if (f == 0) {
            A[0] = h;
            src[0] = 0;
        } else {
            const float v = A[f - 1] + a.lambda;
            const bool keep = h <= v;
            A[f] = keep ? h : v;
            src[f] = keep ? f : src[f - 1];
        }
    }
#pragma unroll
    for (int f = LP - 2; f >= 0; --f) {
        const float v = A[f + 1] + a.lambda;
        if (v < A[f]) {
            A[f] = v;
            src[f] = src[f + 1];
        }
    }
    const float cap = hmin + a.lambda * a.tau;

    // Scatter the receiver slot's adjoint onto h-bar, then clear that slot.
#pragma unroll
    for (int f = 0; f < LP; ++f) hb[f] = 0.0f;
    uint32_t roff = 0;
    if (hq) {
        int nx = x, ny = y;
        if (q == 0) nx = x - 1;
        else if (q == 1) nx = x + 1;
        else if (q == 2) ny = y - 1;
        else ny = y + 1;
        roff = ((uint32_t)((a.colour ^ 1) * 4 + (q ^ 1)) * a.blk + (uint32_t)(ny * a.wh + (nx >> 1))) * 4u;
    }
#pragma unroll
    for (int f = 0; f < LP; ++f) {
        if (!(EXACT || f < nl)) continue;
        if (!hq) continue;
        const float mb = ld_f32(rb, roff, (uint32_t)f * cls);
        if (cap < A[f]) {
            lsum += mb * a.tau;
            tsum += mb * a.lambda;
        } else {
            hb[src[f]] += mb;
            hb[gmin] -= mb;
            lsum += mb * fabsf((float)(f - src[f]));
        }
        st_f32(rb, 0.0f, roff, (uint32_t)f * cls);
    }

    // Sender side: cost-bar += sum_q hbar_q; slot k adjoint += sum_{q != k} hbar_q.
    const int64_t plane = (int64_t)a.h * a.w;
    for (int f = 0; f < nl; ++f) {
        const float hv = hb[f];
        const float tot = group_sum<4>(hv);
        if (live) {
            if (has[q]) {
                const uint32_t so = (uint32_t)f * cls;
                const float cur = ld_f32(rb, moff[q], so);
                st_f32(rb, cur + (tot - hv), moff[q], so);
            }
            if (q == 0) {
                float *gc = a.grad_cost + (int64_t)f * plane + (int64_t)y * a.w + x;
                *gc += tot;
            }
        }
    }

    // Block (one wave) sums of the lambda and tau partials.
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lsum += __shfl_xor(lsum, o, 64);
        tsum += __shfl_xor(tsum, o, 64);
    }
    if (threadIdx.x == 0) {
        a.partial[2 * blockIdx.x] = lsum;
        a.partial[2 * blockIdx.x + 1] = tsum;
    }
}

// Readout adjoint: b = cost + sum of the four incoming messages of M_K,
// d = sum f p_f with p = softmax(-b / T); b-bar(f) = -(g / T) p_f (f - d).
// Initialises grad_cost (planar) and every in-grid slot of the message
// adjoint.  One thread per pixel; grid (ncomp / 256, 2 colours).
__global__ void __launch_bounds__(256) k_bwd_readout(const float *__restrict__ cost, uint32_t cost_bytes,
                                                    const uint8_t *__restrict__ msg, uint32_t msg_bytes,
                                                    float *__restrict__ mbar, uint32_t mbar_bytes,
                                                    const float *__restrict__ grad_soft, float *__restrict__ grad_cost,
                                                    int w, int h, int wh, uint32_t blk, uint32_t ls, int L, float inv_t)
{
    const int c = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= h * wh) return;
    const int y = j / wh;
    const int x = 2 * (j - y * wh) + ((y + c) & 1);
    if (x >= w) return;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(cost, cost_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(msg, msg_bytes);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(mbar, mbar_bytes);
    const uint32_t cls = ls * 4u;
    const uint32_t co = ((uint32_t)c * blk + (uint32_t)j) * 4u;
    uint32_t mo[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) mo[k] = (((uint32_t)c * 4u + (uint32_t)k) * blk + (uint32_t)j) * 4u;
    const bool has[4] = {x > 0, x < w - 1, y > 0, y < h - 1};
    auto belief = [&](int f) {
        float b = ld_f32(rc, co, (uint32_t)f * cls);
#pragma unroll
        for (int k = 0; k < 4; ++k) b += ld_f32(rm, mo[k], (uint32_t)f * cls);
        return b;
    };
    float bmin = __builtin_huge_valf();
    for (int f = 0; f < L; ++f) bmin = fminf(bmin, belief(f));
    float num = 0.0f, den = 0.0f;
    for (int f = 0; f < L; ++f) {
        const float wgt = expf(-(belief(f) - bmin) * inv_t);
        num += (float)f * wgt;
        den += wgt;
    }
    const float d = num / den;
    const float g = grad_soft[(int64_t)y * w + x];
    const int64_t plane = (int64_t)h * w;
    for (int f = 0; f < L; ++f) {
        const float p = expf(-(belief(f) - bmin) * inv_t) / den;
        const float bb = -g * inv_t * p * ((float)f - d);
        grad_cost[(int64_t)f * plane + (int64_t)y * w + x] = bb;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (has[k]) st_f32(rb, bb, mo[k], (uint32_t)f * cls);
    }
}

// Deterministic sum of the per-block partials (fixed order), one thread.
__global__ void k_bwd_finish(const float *__restrict__ partial, int n, float *grad_lambda, float *grad_tau)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double l = 0.0, t = 0.0;
    for (int i = 0; i < n; ++i) {
        l += partial[2 * i];
        t += partial[2 * i + 1];
    }
    *grad_lambda = (float)l;
    *grad_tau = (float)t;
}

// Byte copy with 16-byte words (sizes are multiples of 256).
__global__ void __launch_bounds__(256) k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

bp_status launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return BP_OK;
    k_copy16<<<(unsigned)((n + 255) / 256), 256, 0, s>>>((const uint4 *)src, (uint4 *)dst, n);
    return launch_status();
}

int bwd_step_blocks(const Plan &p) { return (p.lv[0].h * p.lv[0].wh + 15) / 16; }

bp_status launch_bwd_readout(const Plan &p, const uint8_t *msg, float *mbar, const float *grad_soft,
                             float *grad_cost, float temperature, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[0];
    const int64_t ncomp = (int64_t)v.h * v.wh;
    k_bwd_readout<<<dim3((unsigned)((ncomp + 255) / 256), 2), 256, 0, s>>>(
        (const float *)(ws + v.cost_off), (uint32_t)v.cost_bytes, msg, (uint32_t)v.msg_bytes, mbar,
        (uint32_t)v.msg_bytes, grad_soft, grad_cost, v.w, v.h, v.wh, (uint32_t)v.blk, (uint32_t)v.ls, p.L,
        1.0f / temperature);
    return launch_status();
}

bp_status launch_bwd_step(const Plan &p, int t, const uint8_t *msg, float *mbar, float *grad_cost, float *partial,
                          float lambda, float tau, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[0];
    BwdArgs a;
    a.cost = (const float *)(ws + v.cost_off);
    a.cost_bytes = (uint32_t)v.cost_bytes;
    a.msg = msg;
    a.msg_bytes = (uint32_t)v.msg_bytes;
    a.mbar = mbar;
    a.mbar_bytes = (uint32_t)v.msg_bytes;
    a.grad_cost = grad_cost;
    a.partial = partial;
    a.w = v.w;
    a.h = v.h;
    a.wh = v.wh;
    a.blk = (uint32_t)v.blk;
    a.ls = (uint32_t)v.ls;
    a.colour = t & 1;
    a.L = p.L;
    a.ncomp = v.h * v.wh;
    a.lambda = lambda;
    a.tau = tau;
    const unsigned grid = (unsigned)bwd_step_blocks(p);
    const int L = p.L;
#define BP_BWD(LV, EX)                                                             \
    k_bwd_step<LV, EX><<<grid, 64, 64 * LV * sizeof(float), s>>>(a);               \
    return launch_status();
    if (L == 16) { BP_BWD(16, true) }
    if (L == 32) { BP_BWD(32, true) }
    if (L == 64) { BP_BWD(64, true) }
    if (L == 128) { BP_BWD(128, true) }
    if (L < 16) { BP_BWD(16, false) }
    if (L < 32) { BP_BWD(32, false) }
    if (L < 64) { BP_BWD(64, false) }
    if (L < 128) { BP_BWD(128, false) }
#undef BP_BWD
    return BP_ERR_UNSUPPORTED;
}

bp_status launch_bwd_finish(const float *partial, int n, float *grad_lambda, float *grad_tau, hipStream_t s)
{
    k_bwd_finish<<<1, 64, 0, s>>>(partial, n, grad_lambda, grad_tau);
    return launch_status();
}

}  // namespace bpk
