// Hierarchical checkerboard min-sum BP on gfx950 (Sec. 2.2, Eq. 1): cost
// pyramid, message initialisation, the half-sweep kernel, readout and the
// message export used by tests.
//
// Data layout (see Level in bp_internal.h): colour-split planes, so that the
// pixels updated by one half-sweep, and each of their four neighbours'
// receiving slots, are contiguous along a row.  Lane mapping of the half-sweep:
// lanes over pixels (coalesced 256-byte accesses per label plane), G lanes per
// pixel each owning 4/G of the outgoing messages; the label recurrence of the
// distance transform runs sequentially in registers, so no cross-lane scan is
// needed and every update costs a handful of VALU operations.
#include <hip/hip_runtime.h>

#include "bp_device.h"
#include "bp_internal.h"

namespace bpk {

// ------------------------------------------------------------------------
// Plans
// ------------------------------------------------------------------------

bool make_plan(int w, int h, int L, int levels, int msg_fmt, size_t base, Plan *p)
{
    p->w = w;
    p->h = h;
    p->L = L;
    p->levels = levels;
    size_t off = base;
    int lw = w, lh = h;
    for (int l = 0; l < levels; ++l) {
        Level &v = p->lv[l];
        v.w = lw;
        v.h = lh;
        v.wh = (lw + 1) / 2;
        v.plane = (int64_t)align_up((size_t)lh * v.wh, 64);
        v.fmt = (l == levels - 1) ? FMT_F32 : msg_fmt;
        v.cost_bytes = align_up((size_t)2 * L * v.plane * sizeof(float));
        v.msg_bytes = align_up((size_t)8 * L * v.plane * fmt_bytes(v.fmt));
        // Buffer offsets inside one level are 32-bit.
        if ((uint64_t)v.cost_bytes >= (1ull << 32) || (uint64_t)v.msg_bytes >= (1ull << 32)) return false;
        v.cost_off = off;
        off += v.cost_bytes;
        v.msg_off = off;
        off += v.msg_bytes;
        lw = (lw + 1) / 2;
        lh = (lh + 1) / 2;
    }
    p->bytes = off - base;
    return true;
}

bp_status launch_status()
{
    return hipGetLastError() == hipSuccess ? BP_OK : BP_ERR_HIP;
}

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ------------------------------------------------------------------------
// a3: colour split of the finest cost and the sum pyramid
// ------------------------------------------------------------------------

// planar [L][h][w] -> colour-split [2][L][plane]
__global__ void __launch_bounds__(256) k_split_cost(const float *__restrict__ planar, float *__restrict__ cs,
                                                   int w, int h, int wh, int64_t plane, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int x = (int)(i % w);
    int64_t r = i / w;
    int y = (int)(r % h);
    int f = (int)(r / h);
    int c = (x + y) & 1;
    int64_t L = n / ((int64_t)w * h);
    cs[((int64_t)c * L + f) * plane + (int64_t)y * wh + (x >> 1)] = planar[i];
}

// level l from level l-1, both colour-split: each coarse pixel sums its
// existing children in the order (0,0), (1,0), (0,1), (1,1).
__global__ void __launch_bounds__(256) k_pyramid(const float *__restrict__ fine, float *__restrict__ coarse,
                                                int wf, int hf, int whf, int64_t pf, int wc, int hc, int whc,
                                                int64_t pc, int L)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t n = (int64_t)L * hc * wc;
    if (i >= n) return;
    int x = (int)(i % wc);
    int64_t r = i / wc;
    int y = (int)(r % hc);
    int f = (int)(r / hc);
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            int fx = 2 * x + k, fy = 2 * y + j;
            if (fx < wf && fy < hf) {
                int c = (fx + fy) & 1;
                s += fine[((int64_t)c * L + f) * pf + (int64_t)fy * whf + (fx >> 1)];
            }
        }
    int cc = (x + y) & 1;
    coarse[((int64_t)cc * L + f) * pc + (int64_t)y * whc + (x >> 1)] = s;
}

bp_status launch_split_cost(const float *planar, const Plan &p, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[0];
    int64_t n = (int64_t)p.L * v.h * v.w;
    k_split_cost<<<blocks_for(n, 256), 256, 0, s>>>(planar, (float *)(ws + v.cost_off), v.w, v.h, v.wh,
                                                   v.plane, n);
    return launch_status();
}

bp_status launch_pyramid_level(const Plan &p, int l, uint8_t *ws, hipStream_t s)
{
    const Level &f = p.lv[l - 1], &c = p.lv[l];
    int64_t n = (int64_t)p.L * c.h * c.w;
    k_pyramid<<<blocks_for(n, 256), 256, 0, s>>>((const float *)(ws + f.cost_off), (float *)(ws + c.cost_off),
                                                f.w, f.h, f.wh, f.plane, c.w, c.h, c.wh, c.plane, p.L);
    return launch_status();
}

// ------------------------------------------------------------------------
// a4: zero out-of-grid slots, explicit parent copy
// ------------------------------------------------------------------------

// Border items: for every label, the pixels of the left column (slot 0), right
// column (slot 1), top row (slot 2) and bottom row (slot 3).
template <typename S>
__global__ void __launch_bounds__(256) k_zero_border(uint8_t *__restrict__ msg, uint32_t msg_bytes, int w, int h,
                                                    int wh, int64_t plane, int L)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t per = 2 * (int64_t)h + 2 * (int64_t)w;
    if (i >= per * L) return;
    int f = (int)(i / per);
    int e = (int)(i % per);
    int x, y, k;
    if (e < h) { x = 0; y = e; k = 0; }
    else if (e < 2 * h) { x = w - 1; y = e - h; k = 1; }
    else if (e < 2 * h + w) { x = e - 2 * h; y = 0; k = 2; }
    else { x = e - 2 * h - w; y = h - 1; k = 3; }
    int c = (x + y) & 1;
    int64_t idx = (((int64_t)c * 4 + k) * L + f) * plane + (int64_t)y * wh + (x >> 1);
    __amdgpu_buffer_rsrc_t r = make_rsrc(msg, msg_bytes);
    S::st(r, 0.0f, (uint32_t)(idx * S::bytes), 0);
}

// Child slot k of pixel (x, y) takes the parent's slot k at (x/2, y/2),
// converted to the child's storage format.
template <typename SP, typename SC>
__global__ void __launch_bounds__(256) k_parent_copy(const uint8_t *__restrict__ pm, uint32_t pm_bytes,
                                                    uint8_t *__restrict__ cm, uint32_t cm_bytes, int wc, int hc,
                                                    int whc, int64_t pc, int whp, int64_t pp, int L)
{
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t n = (int64_t)4 * L * hc * wc;
    if (i >= n) return;
    int x = (int)(i % wc);
    int64_t r = i / wc;
    int y = (int)(r % hc);
    r /= hc;
    int f = (int)(r % L);
    int k = (int)(r / L);
    int px = x >> 1, py = y >> 1;
    int cp = (px + py) & 1, cc = (x + y) & 1;
    int64_t src = (((int64_t)cp * 4 + k) * L + f) * pp + (int64_t)py * whp + (px >> 1);
    int64_t dst = (((int64_t)cc * 4 + k) * L + f) * pc + (int64_t)y * whc + (x >> 1);
    float v = SP::ld(make_rsrc(pm, pm_bytes), (uint32_t)(src * SP::bytes), 0);
    SC::st(make_rsrc(cm, cm_bytes), v, (uint32_t)(dst * SC::bytes), 0);
}

__global__ void __launch_bounds__(256) k_fill_zero(uint32_t *__restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

bp_status launch_zero_level(const Plan &p, int l, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[l];
    const int64_t n = (int64_t)(v.msg_bytes / 4);
    k_fill_zero<<<blocks_for(n, 256), 256, 0, s>>>((uint32_t *)(ws + v.msg_off), n);
    return launch_status();
}

template <typename F>
static bp_status with_store(int fmt, F &&fn)
{
    switch (fmt) {
    case FMT_F16: return fn(StoreF16{});
    case FMT_BF16: return fn(StoreBF16{});
    default: return fn(StoreF32{});
    }
}

bp_status launch_zero_border(const Plan &p, int l, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[l];
    int64_t n = (2 * (int64_t)v.h + 2 * (int64_t)v.w) * p.L;
    return with_store(v.fmt, [&](auto st) {
        using S = decltype(st);
        k_zero_border<S><<<blocks_for(n, 256), 256, 0, s>>>(ws + v.msg_off, (uint32_t)v.msg_bytes, v.w, v.h, v.wh,
                                                           v.plane, p.L);
        return launch_status();
    });
}

bp_status launch_parent_copy(const Plan &p, int l, uint8_t *ws, hipStream_t s)
{
    const Level &c = p.lv[l], &pa = p.lv[l + 1];
    int64_t n = (int64_t)4 * p.L * c.h * c.w;
    return with_store(pa.fmt, [&](auto sp) {
        return with_store(c.fmt, [&](auto sc) {
            using SP = decltype(sp);
            using SC = decltype(sc);
            k_parent_copy<SP, SC><<<blocks_for(n, 256), 256, 0, s>>>(ws + pa.msg_off, (uint32_t)pa.msg_bytes,
                                                                    ws + c.msg_off, (uint32_t)c.msg_bytes, c.w, c.h,
                                                                    c.wh, c.plane, pa.wh, pa.plane, p.L);
            return launch_status();
        });
    });
}

// ------------------------------------------------------------------------
// a5: one checkerboard half-sweep
// ------------------------------------------------------------------------

struct IterArgs {
    const float *cost;     // this level's colour-split cost
    uint32_t cost_bytes;
    uint8_t *msg;          // this level's messages
    uint32_t msg_bytes;
    const uint8_t *src;    // where incoming messages are read (own level or parent)
    uint32_t src_bytes;
    int32_t *disp;         // finest-level argmin output of the senders, or NULL
    int w, h, wh;
    uint32_t plane;        // elements per plane, this level
    uint32_t src_plane;    // elements per plane of `src`
    int src_w, src_h, src_wh;
    int src_mode;          // 0 own slots, 1 parent slots, 2 zero
    int colour;            // sender colour
    int L;                 // label count (runtime, <= LP)
    int ncomp;             // h * wh
    float lambda, lt;      // lambda and lambda * tau
};

// One half-sweep.  Thread group of G lanes = one sender pixel of colour
// `colour`; lane `sub` owns the outgoing messages k = sub*(4/G) .. +4/G-1, the
// message to the neighbour on side k (0 left, 1 right, 2 up, 3 down), which
// excludes what that neighbour sent (incoming slot k):
//   S(f)   = cost(f) + sum_k m_k(f)             (group sum over the G lanes)
//   h_k(f) = S(f) - m_k(f)
//   a(f)   = min(h_k(f), a(f-1) + lambda)       forward pass, kept in registers
//   b(f)   = min(a(f), b(f+1) + lambda, min h_k + lambda*tau)   backward pass
//   out(f) = b(f) - min h_k                     (= b minus its own minimum)
// The truncation folded into the backward pass and the normaliser min h_k are
// exact rewrites of the two-pass transform followed by min(., min h + lambda tau)
// and subtraction of the result's minimum (the result's minimum is min h_k).
// The message lands in the neighbour's slot k^1 (it sees this pixel on the
// opposite side).  Out-of-grid slots hold zero (zeroed per level), so loads
// need no predicate; stores to missing neighbours are masked.
template <int LP, int G, typename S, bool EXACT, bool RO>
__global__ void __launch_bounds__(256) k_iter(const IterArgs a)
{
    constexpr int ND = 4 / G;
    // Labels whose loads are in flight while one label is combined: bounds the
    // registers held by prefetched values (the forward pass itself keeps ND*LP).
    constexpr int PD = LP < 8 ? LP : 8;
    const int nl = EXACT ? LP : a.L;
    const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
    const int j = (int)(gid / G);
    const int sub = (int)(gid % G);
    if (j >= a.ncomp) return;
    const int y = j / a.wh;
    const int x = 2 * (j - y * a.wh) + ((y + a.colour) & 1);
    if (x >= a.w) return;

    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost, a.cost_bytes);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.src, a.src_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(a.msg, a.msg_bytes);

    // Per-lane byte offsets of label 0; label f adds f * plane * bytes (uniform).
    const uint32_t lp_c = (uint32_t)nl * a.plane;          // elements per (colour) block of the cost
    const uint32_t cost_off = ((uint32_t)a.colour * lp_c + (uint32_t)j) * 4u;
    uint32_t src_off[ND];
    uint32_t dst_off[ND];
    bool has[ND];
    {
        int sj = j, sc = a.colour, sx = x, sy = y;
        if (a.src_mode == 1) {
            sx = x >> 1;
            sy = y >> 1;
            sc = (sx + sy) & 1;
            sj = sy * a.src_wh + (sx >> 1);
        }
        const uint32_t lps = (uint32_t)nl * a.src_plane;
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            const int k = sub * ND + i;
            src_off[i] = (((uint32_t)sc * 4u + (uint32_t)k) * lps + (uint32_t)sj) * S::bytes;
            int nx = x, ny = y;
            bool ok;
            if (k == 0) { nx = x - 1; ok = x > 0; }
            else if (k == 1) { nx = x + 1; ok = x < a.w - 1; }
            else if (k == 2) { ny = y - 1; ok = y > 0; }
            else { ny = y + 1; ok = y < a.h - 1; }
            has[i] = ok;
            const uint32_t dj = ok ? (uint32_t)(ny * a.wh + (nx >> 1)) : 0u;
            dst_off[i] = ((((uint32_t)(a.colour ^ 1)) * 4u + (uint32_t)(k ^ 1)) * (uint32_t)nl * a.plane + dj) * S::bytes;
        }
    }
    const float lam = a.lambda;
    const float inf = __builtin_huge_valf();

    // Prefetch ring: cost and owned incoming messages of labels f .. f+PD-1.
    float pc[PD], pm[PD][ND];
    auto issue = [&](int f, int slot) {
        if (EXACT || f < nl) {
            pc[slot] = ld_f32(rc, cost_off, (uint32_t)f * a.plane * 4u);
#pragma unroll
            for (int i = 0; i < ND; ++i) pm[slot][i] = S::ld(rs, src_off[i], (uint32_t)f * a.src_plane * S::bytes);
        }
    };
#pragma unroll
    for (int f = 0; f < PD; ++f) issue(f, f);

    float acc[ND][LP];
    float mn[ND];
    float best = inf;
    int bidx = 0;
#pragma unroll
    for (int f = 0; f < LP; ++f) {
        const int slot = f % PD;
        const bool on = EXACT || f < nl;
        const float c = pc[slot];
        float m[ND];
#pragma unroll
        for (int i = 0; i < ND; ++i) m[i] = pm[slot][i];
        float part = (G == 1 || sub == 0) ? c : 0.0f;
#pragma unroll
        for (int i = 0; i < ND; ++i) part += m[i];
        float tot = group_sum<G>(part);
        if (!on) tot = inf;
        if constexpr (RO) {
            if (tot < best) {
                best = tot;
                bidx = f;
            }
        }
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            const float hv = on ? tot - m[i] : inf;
            if (f == 0) {
                acc[i][0] = hv;
                mn[i] = hv;
            } else {
                acc[i][f] = fminf(hv, acc[i][f - 1] + lam);
                mn[i] = fminf(mn[i], hv);
            }
            // Keep the recurrence at this step: otherwise the compiler sinks it
            // past the loop and holds every label's loaded values at once.
            asm volatile("" : "+v"(acc[i][f]), "+v"(mn[i]));
        }
        if (f + PD < LP) issue(f + PD, slot);
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (RO) {
        if (sub == 0) a.disp[(int64_t)y * a.w + x] = bidx;
    }
    // Backward pass, one outgoing message at a time (border pixels skip the
    // messages that have no receiver without per-label branches).
#pragma unroll
    for (int i = 0; i < ND; ++i) {
        if (!has[i]) continue;
        const float cap = mn[i] + a.lt;
        float b = inf;
#pragma unroll
        for (int f = LP - 1; f >= 0; --f) {
            const float v = fminf(fminf(acc[i][f], b + lam), cap);
            b = v;
            if (EXACT || f < nl) S::st(rm, v - mn[i], dst_off[i], (uint32_t)f * a.plane * S::bytes);
        }
    }
}

// Variant table: lanes per pixel G for a label count.
struct IterVariant {
    int G;
};

int iteration_variants(int L)
{
    if (L <= 32) return 3;   // G = 1, 2, 4
    if (L <= 64) return 2;   // G = 2, 4
    return 1;                // G = 4
}

int iteration_lanes(int L, int variant)
{
    static const int small[3] = {1, 2, 4};
    static const int mid[2] = {2, 4};
    int nv = iteration_variants(L);
    int v = (variant <= 0 || variant > nv) ? 0 : variant - 1;
    if (L <= 32) return small[v];
    if (L <= 64) return mid[v];
    return 4;
}

template <int LP, int G, typename S, bool EXACT>
static void launch_iter_ro(const IterArgs &a, bool ro, unsigned grid, hipStream_t s)
{
    if (ro) k_iter<LP, G, S, EXACT, true><<<grid, 256, 0, s>>>(a);
    else k_iter<LP, G, S, EXACT, false><<<grid, 256, 0, s>>>(a);
}

template <typename S>
static bp_status dispatch_iter(const IterArgs &a, int G, bool ro, hipStream_t s)
{
    const unsigned grid = blocks_for((int64_t)a.ncomp * G, 256);
    const int L = a.L;
#define BP_ITER_CASE(LV, GV, EX)                                  \
    if (G == GV) {                                                \
        launch_iter_ro<LV, GV, S, EX>(a, ro, grid, s);            \
        return launch_status();                                   \
    }
    switch (L) {
    case 16: BP_ITER_CASE(16, 1, true) BP_ITER_CASE(16, 2, true) BP_ITER_CASE(16, 4, true) break;
    case 32: BP_ITER_CASE(32, 1, true) BP_ITER_CASE(32, 2, true) BP_ITER_CASE(32, 4, true) break;
    case 64: BP_ITER_CASE(64, 2, true) BP_ITER_CASE(64, 4, true) break;
    case 96: BP_ITER_CASE(96, 4, true) break;
    case 128: BP_ITER_CASE(128, 4, true) break;
    default: break;
    }
    if (L <= 16) { BP_ITER_CASE(16, 1, false) BP_ITER_CASE(16, 2, false) BP_ITER_CASE(16, 4, false) }
    else if (L <= 32) { BP_ITER_CASE(32, 1, false) BP_ITER_CASE(32, 2, false) BP_ITER_CASE(32, 4, false) }
    else if (L <= 64) { BP_ITER_CASE(64, 2, false) BP_ITER_CASE(64, 4, false) }
    else if (L <= 128) { BP_ITER_CASE(128, 4, false) }
    else { BP_ITER_CASE(256, 4, false) }
#undef BP_ITER_CASE
    return BP_ERR_UNSUPPORTED;
}

bp_status launch_iteration(const Plan &p, int l, int t, int src_mode, float lambda, float tau, int32_t *disp,
                           int variant, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[l];
    IterArgs a;
    a.cost = (const float *)(ws + v.cost_off);
    a.cost_bytes = (uint32_t)v.cost_bytes;
    a.msg = ws + v.msg_off;
    a.msg_bytes = (uint32_t)v.msg_bytes;
    a.disp = disp;
    a.w = v.w;
    a.h = v.h;
    a.wh = v.wh;
    a.plane = (uint32_t)v.plane;
    a.src_mode = src_mode;
    if (src_mode == 1) {
        const Level &pa = p.lv[l + 1];
        a.src = ws + pa.msg_off;
        a.src_bytes = (uint32_t)pa.msg_bytes;
        a.src_plane = (uint32_t)pa.plane;
        a.src_w = pa.w;
        a.src_h = pa.h;
        a.src_wh = pa.wh;
    } else {
        a.src = a.msg;
        a.src_bytes = a.msg_bytes;
        a.src_plane = a.plane;
        a.src_w = v.w;
        a.src_h = v.h;
        a.src_wh = v.wh;
    }
    a.colour = t & 1;
    a.L = p.L;
    a.ncomp = v.h * v.wh;
    a.lambda = lambda;
    a.lt = lambda * tau;
    const int G = iteration_lanes(p.L, variant);
    return with_store(v.fmt, [&](auto st) { return dispatch_iter<decltype(st)>(a, G, disp != nullptr, s); });
}

// ------------------------------------------------------------------------
// a6: readout, message export
// ------------------------------------------------------------------------

// Belief b(f) = cost(f) + m_0 + m_1 + m_2 + m_3 at every pixel of the colours
// in `mask`; lowest-index argmin, and soft-argmin sum f w / sum w with
// w = exp(-(b - min b) / T) accumulated with a running minimum.
template <typename S>
__global__ void __launch_bounds__(256) k_readout(const float *__restrict__ cost, uint32_t cost_bytes,
                                                const uint8_t *__restrict__ msg, uint32_t msg_bytes, int w, int h,
                                                int wh, uint32_t plane, int L, int mask, int32_t *__restrict__ disp,
                                                float *__restrict__ soft, float inv_t)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t ncomp = (int64_t)h * wh;
    if (i >= 2 * ncomp) return;
    const int c = (int)(i / ncomp);
    if (!((mask >> c) & 1)) return;
    const int j = (int)(i - c * ncomp);
    const int y = j / wh;
    const int x = 2 * (j - y * wh) + ((y + c) & 1);
    if (x >= w) return;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(cost, cost_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(msg, msg_bytes);
    const uint32_t lp = (uint32_t)L * plane;
    const uint32_t co = ((uint32_t)c * lp + (uint32_t)j) * 4u;
    uint32_t mo[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) mo[k] = (((uint32_t)c * 4u + (uint32_t)k) * lp + (uint32_t)j) * S::bytes;
    float best = __builtin_huge_valf();
    int bidx = 0;
    float num = 0.0f, den = 0.0f;
    for (int f = 0; f < L; ++f) {
        float b = ld_f32(rc, co, (uint32_t)f * plane * 4u);
#pragma unroll
        for (int k = 0; k < 4; ++k) b += S::ld(rm, mo[k], (uint32_t)f * plane * S::bytes);
        if (b < best) {
            if (soft) {
                const float sc = expf((b - best) * inv_t);
                num *= sc;
                den *= sc;
            }
            best = b;
            bidx = f;
        }
        if (soft) {
            const float wgt = expf(-(b - best) * inv_t);
            num += (float)f * wgt;
            den += wgt;
        }
    }
    const int64_t o = (int64_t)y * w + x;
    if (disp) disp[o] = bidx;
    if (soft) soft[o] = num / den;
}

bp_status launch_readout(const Plan &p, int colour_mask, int32_t *disp, float *soft, float temperature, uint8_t *ws,
                         hipStream_t s)
{
    const Level &v = p.lv[0];
    const int64_t n = 2 * (int64_t)v.h * v.wh;
    const float inv_t = soft ? 1.0f / temperature : 0.0f;
    return with_store(v.fmt, [&](auto st) {
        using S = decltype(st);
        k_readout<S><<<blocks_for(n, 256), 256, 0, s>>>((const float *)(ws + v.cost_off), (uint32_t)v.cost_bytes,
                                                       ws + v.msg_off, (uint32_t)v.msg_bytes, v.w, v.h, v.wh,
                                                       (uint32_t)v.plane, p.L, colour_mask, disp, soft, inv_t);
        return launch_status();
    });
}

// Colour-split messages -> planar float32 [4][L][h][w]; slots without a
// neighbour read as zero.
template <typename S>
__global__ void __launch_bounds__(256) k_export(const uint8_t *__restrict__ msg, uint32_t msg_bytes, int w, int h,
                                               int wh, uint32_t plane, int L, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)4 * L * h * w;
    if (i >= n) return;
    const int x = (int)(i % w);
    int64_t r = i / w;
    const int y = (int)(r % h);
    r /= h;
    const int f = (int)(r % L);
    const int k = (int)(r / L);
    bool ok = (k == 0) ? x > 0 : (k == 1) ? x < w - 1 : (k == 2) ? y > 0 : y < h - 1;
    float v = 0.0f;
    if (ok) {
        const int c = (x + y) & 1;
        const int64_t idx = (((int64_t)c * 4 + k) * L + f) * plane + (int64_t)y * wh + (x >> 1);
        v = S::ld(make_rsrc(msg, msg_bytes), (uint32_t)(idx * S::bytes), 0);
    }
    out[i] = v;
}

bp_status launch_export(const Plan &p, float *out, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[0];
    const int64_t n = (int64_t)4 * p.L * v.h * v.w;
    return with_store(v.fmt, [&](auto st) {
        using S = decltype(st);
        k_export<S><<<blocks_for(n, 256), 256, 0, s>>>(ws + v.msg_off, (uint32_t)v.msg_bytes, v.w, v.h, v.wh,
                                                      (uint32_t)v.plane, p.L, out);
        return launch_status();
    });
}

}  // namespace bpk
