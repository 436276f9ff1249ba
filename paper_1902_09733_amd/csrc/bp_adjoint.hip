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

// One reverse half-sweep of one problem, block `block` of it.  64 threads per
// block: 16 sender pixels x 4 outgoing messages; ceil(ncomp / 16) blocks.
template <int LP>
__device__ __forceinline__ void bwd_step(const BwdArgs &a, uint32_t block)
{
    // h-bar rows in LDS, label-major with the lane fastest ([LP][64]): a lane's
    // entries sit in its own bank whatever label it touches, so neither the
    // label loops nor the data-dependent scatter conflict.
    extern __shared__ float hb_all[];
    float *hb = hb_all + threadIdx.x;
    // Labels past L (up to the register row length LP) are inactive.  The
    // label count stays a runtime value even when it equals LP: that keeps
    // the loads conditional and the register count low.
    const int nl = a.L;
    const int j = (int)block * 16 + (threadIdx.x >> 2);
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

    // Distance transform of h with winners (registers, fully unrolled).  The
    // winner of label f (< 256) is kept as a byte of srcp[f / 4].  Loads are
    // issued in batches (scheduling barriers), which bounds the registers
    // they hold.
    float A[LP];
    uint32_t srcp[LP / 4];
    auto set_src = [&](int f, uint32_t g) {
        const int sh = 8 * (f & 3);
        srcp[f >> 2] = (srcp[f >> 2] & ~(0xffu << sh)) | (g << sh);
    };
    auto get_src = [&](int f) { return (srcp[f >> 2] >> (8 * (f & 3))) & 0xffu; };
#pragma unroll
    for (int i = 0; i < LP / 4; ++i) srcp[i] = 0u;
    float hmin = inf;
    int gmin = 0;
    // Each lane loads the cost and only its own incoming slot q; the four
    // slots' values reach every lane of the pixel's quad by DPP broadcasts, and
    // h is summed in the same order as in the forward kernel.  Loads are
    // issued kB1 labels at a time.
    constexpr int kB1 = LP < 32 ? LP : 32;
#pragma unroll
    for (int f0 = 0; f0 < LP; f0 += kB1) {
        float cv[kB1], mv[kB1];
#pragma unroll
        for (int e = 0; e < kB1; ++e) {
            const int f = f0 + e;
            cv[e] = f < nl ? ld_f32(rc, cost_off, (uint32_t)f * cls) : 0.0f;
            mv[e] = f < nl ? ld_f32(rm, moff[q], (uint32_t)f * cls) : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < kB1; ++e) {
            const int f = f0 + e;
            float h = inf;
            if (f < nl) {
                const float m4[4] = {dpp_f<0x00>(mv[e], mv[e]), dpp_f<0x55>(mv[e], mv[e]), dpp_f<0xAA>(mv[e], mv[e]),
                                     dpp_f<0xFF>(mv[e], mv[e])};
                h = cv[e];
#pragma unroll
                for (int k = 0; k < 4; ++k) h += (k == q) ? 0.0f : m4[k];
            }
            if (h < hmin) {
                hmin = h;
                gmin = f;
            }
            if (f == 0) {
                A[0] = h;
                set_src(0, 0u);
            } else {
                const float v = A[f - 1] + a.lambda;
                const bool keep = h <= v;
                A[f] = keep ? h : v;
                set_src(f, keep ? (uint32_t)f : get_src(f - 1));
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int f = LP - 2; f >= 0; --f) {
        const float v = A[f + 1] + a.lambda;
        if (v < A[f]) {
            A[f] = v;
            set_src(f, get_src(f + 1));
        }
    }
    const float cap = hmin + a.lambda * a.tau;

    // Scatter the receiver slot's adjoint onto h-bar, then clear that slot.
#pragma unroll
    for (int f = 0; f < LP; ++f) hb[f * 64] = 0.0f;
    uint32_t roff = 0;
    if (hq) {
        int nx = x, ny = y;
        if (q == 0) nx = x - 1;
        else if (q == 1) nx = x + 1;
        else if (q == 2) ny = y - 1;
        else ny = y + 1;
        roff = ((uint32_t)((a.colour ^ 1) * 4 + (q ^ 1)) * a.blk + (uint32_t)(ny * a.wh + (nx >> 1))) * 4u;
    }
    if (hq) {
#pragma unroll
        for (int f0 = 0; f0 < LP; f0 += kB1) {
            float mbv[kB1];
#pragma unroll
            for (int e = 0; e < kB1; ++e)
                mbv[e] = (f0 + e < nl) ? ld_f32(rb, roff, (uint32_t)(f0 + e) * cls) : 0.0f;
#pragma unroll
            for (int e = 0; e < kB1; ++e) {
                const int f = f0 + e;
                if (!(f < nl)) continue;
                const float mb = mbv[e];
                if (cap < A[f]) {
                    lsum += mb * a.tau;
                    tsum += mb * a.lambda;
                } else {
                    const int g = (int)get_src(f);
                    hb[g * 64] += mb;
                    hb[gmin * 64] -= mb;
                    lsum += mb * fabsf((float)(f - g));
                }
                st_f32(rb, 0.0f, roff, (uint32_t)f * cls);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // Sender side: cost-bar += sum_q hbar_q; slot k adjoint += sum_{q != k} hbar_q.
    // Read-modify-writes are batched kB3 labels at a time.
    constexpr int kB3 = LP < 16 ? LP : 16;
    const int64_t plane = (int64_t)a.h * a.w;
    float *gc0 = a.grad_cost + (int64_t)y * a.w + x;
#pragma unroll 1
    for (int f0 = 0; f0 < nl; f0 += kB3) {
        float hv[kB3], tot[kB3], cur[kB3], gcv[kB3];
#pragma unroll
        for (int e = 0; e < kB3; ++e) {
            const int f = f0 + e < nl ? f0 + e : nl - 1;
            hv[e] = f0 + e < nl ? hb[f * 64] : 0.0f;
            tot[e] = group_sum<4>(hv[e]);
            cur[e] = (live && has[q] && f0 + e < nl) ? ld_f32(rb, moff[q], (uint32_t)f * cls) : 0.0f;
            gcv[e] = (live && q == 0 && f0 + e < nl) ? gc0[(int64_t)f * plane] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < kB3; ++e) {
            const int f = f0 + e;
            if (!live || f >= nl) continue;
            if (has[q]) st_f32(rb, cur[e] + (tot[e] - hv[e]), moff[q], (uint32_t)f * cls);
            if (q == 0) gc0[(int64_t)f * plane] = gcv[e] + tot[e];
        }
    }

    // Block (one wave) sums of the lambda and tau partials.
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lsum += __shfl_xor(lsum, o, 64);
        tsum += __shfl_xor(tsum, o, 64);
    }
    if (threadIdx.x == 0) {
        a.partial[2 * block] = lsum;
        a.partial[2 * block + 1] = tsum;
    }
}

// The reverse half-sweep of several problems (same label count) in one
// launch: block b belongs to the last entry whose first block is <= b.
struct BwdEntry {
    BwdArgs a;
    int block0;
    int pad[3];
};
constexpr int kBwdChunk = 16;
struct BwdChunk {
    BwdEntry e[kBwdChunk];
    int n;
};

__global__ void k_write_bwd_entries(BwdEntry *__restrict__ dst, BwdChunk c)
{
    const int i = threadIdx.x;
    if (i < c.n) dst[i] = c.e[i];
}

template <int LP>
__global__ void __launch_bounds__(64) k_bwd_step_batch(const BwdEntry *__restrict__ tab, int n)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    bwd_step<LP>(tab[lo].a, blockIdx.x - (uint32_t)tab[lo].block0);
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

// Deterministic sum of the (lambda, tau) partials in two passes.  Pass 1:
// block b of kFinishBlocks takes the contiguous chunk b of the partials;
// thread t adds entries t, t + 256, ... of the chunk in FP64 in that order,
// then a fixed binary tree over the threads.  Pass 2: one block adds the
// block sums with the same tree.  The order depends only on the number of
// partials, so repeated calls give identical bits.
constexpr int kFinishBlocks = 256;

__device__ __forceinline__ void tree_sum_256(double &l, double &t, double *sl, double *st)
{
    const int i = threadIdx.x;
    sl[i] = l;
    st[i] = t;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (i < h) {
            sl[i] += sl[i + h];
            st[i] += st[i + h];
        }
        __syncthreads();
    }
    l = sl[0];
    t = st[0];
}

__global__ void __launch_bounds__(256) k_bwd_finish_part(const float2 *__restrict__ partial, int n, int chunk,
                                                        double2 *__restrict__ out)
{
    __shared__ double sl[256], st[256];
    const int lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double l = 0.0, t = 0.0;
    for (int k = lo + (int)threadIdx.x; k < hi; k += 256) {
        const float2 v = partial[k];
        l += v.x;
        t += v.y;
    }
    tree_sum_256(l, t, sl, st);
    if (threadIdx.x == 0) out[blockIdx.x] = make_double2(l, t);
}

__global__ void __launch_bounds__(256) k_bwd_finish(const double2 *__restrict__ sums, float *grad_lambda,
                                                   float *grad_tau)
{
    __shared__ double sl[256], st[256];
    const double2 v = sums[threadIdx.x];
    double l = v.x, t = v.y;
    tree_sum_256(l, t, sl, st);
    if (threadIdx.x == 0) {
        *grad_lambda = (float)l;
        *grad_tau = (float)t;
    }
}

size_t bwd_finish_bytes() { return align_up((size_t)kFinishBlocks * sizeof(double2)); }

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

// Zero fill with 16-byte words (sizes are multiples of 16).
__global__ void __launch_bounds__(256) k_zero16(uint4 *__restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = make_uint4(0u, 0u, 0u, 0u);
}

bp_status launch_zero(void *dst, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return BP_OK;
    k_zero16<<<(unsigned)((n + 255) / 256), 256, 0, s>>>((uint4 *)dst, n);
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

size_t bwd_table_bytes(int count) { return align_up((size_t)count * sizeof(BwdEntry)); }

bp_status launch_bwd_step_batch(const BwdProblem *probs, int count, int t, float lambda, float tau, uint8_t *table,
                                hipStream_t s)
{
    BwdEntry *dev = (BwdEntry *)table;
    // One launch per label count (the kernel's register row length).
    bool *done = new bool[count]();
    BwdEntry *host = new BwdEntry[count];
    bp_status st = BP_OK;
    int used = 0;
    for (int i = 0; i < count && st == BP_OK; ++i) {
        if (done[i]) continue;
        const int L = probs[i].plan->L;
        const int first = used;
        int blocks = 0;
        for (int k = i; k < count; ++k) {
            if (done[k] || probs[k].plan->L != L) continue;
            done[k] = true;
            const Plan &p = *probs[k].plan;
            const Level &v = p.lv[0];
            BwdEntry &e = host[used++];
            BwdArgs &a = e.a;
            a.cost = (const float *)(probs[k].ws + v.cost_off);
            a.cost_bytes = (uint32_t)v.cost_bytes;
            a.msg = probs[k].state;
            a.msg_bytes = (uint32_t)v.msg_bytes;
            a.mbar = probs[k].mbar;
            a.mbar_bytes = (uint32_t)v.msg_bytes;
            a.grad_cost = probs[k].grad_cost;
            a.partial = probs[k].partial;
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
            e.block0 = blocks;
            blocks += bwd_step_blocks(p);
        }
        // Entries of this group: written by value through kernel arguments.
        for (int c0 = first; c0 < used && st == BP_OK; c0 += kBwdChunk) {
            BwdChunk c;
            c.n = used - c0 < kBwdChunk ? used - c0 : kBwdChunk;
            for (int k = 0; k < c.n; ++k) c.e[k] = host[c0 + k];
            k_write_bwd_entries<<<1, 64, 0, s>>>(dev + c0, c);
            st = launch_status();
        }
        if (st != BP_OK) break;
        const int n = used - first;
        const BwdEntry *tab = dev + first;
#define BP_BWD(LV)                                                                            \
    {                                                                                         \
        k_bwd_step_batch<LV><<<blocks, 64, 64 * LV * sizeof(float), s>>>(tab, n);            \
        st = launch_status();                                                                 \
        continue;                                                                             \
    }
        if (L <= 16) BP_BWD(16)
        if (L <= 32) BP_BWD(32)
        if (L <= 64) BP_BWD(64)
        if (L <= 128) BP_BWD(128)
#undef BP_BWD
        st = BP_ERR_UNSUPPORTED;
    }
    delete[] done;
    delete[] host;
    return st;
}

bp_status launch_bwd_finish(const float *partial, int n, float *grad_lambda, float *grad_tau, uint8_t *scratch,
                            hipStream_t s)
{
    double2 *sums = (double2 *)scratch;
    const int chunk = (n + kFinishBlocks - 1) / kFinishBlocks;
    k_bwd_finish_part<<<kFinishBlocks, 256, 0, s>>>((const float2 *)partial, n, chunk > 0 ? chunk : 1, sums);
    k_bwd_finish<<<1, 256, 0, s>>>(sums, grad_lambda, grad_tau);
    return launch_status();
}

}  // namespace bpk
