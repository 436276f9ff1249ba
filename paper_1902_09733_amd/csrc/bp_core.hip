// Hierarchical checkerboard min-sum BP on gfx950 (Sec. 2.2, Eq. 1): level
// plans, cost pyramid, message initialisation, readout and message export.
// The half-sweep kernels live in bp_iter_lm.hip (label-major levels) and
// bp_iter_pm.hip (pixel-major levels).
#include <hip/hip_runtime.h>

#include "bp_device.h"
#include "bp_internal.h"
#include "bp_levels.h"
#include "bp_pm_core.h"

namespace bpk {

// ------------------------------------------------------------------------
// Plans
// ------------------------------------------------------------------------

bool make_plan(int w, int h, int L, int levels, int msg_fmt, int pm_from, size_t base, Plan *p)
{
    p->w = w;
    p->h = h;
    p->L = L;
    p->levels = levels;
    p->variant = 0;
    p->pair_off = 0;
    p->pairs = false;
    p->y_off = 0;
    p->zero_coarsest = true;
    size_t off = base;
    int lw = w, lh = h;
    int S, R;
    pm_split(L, &S, &R);
    for (int l = 0; l < levels; ++l) {
        Level &v = p->lv[l];
        v.w = lw;
        v.h = lh;
        v.wh = (lw + 1) / 2;
        v.plane = (int64_t)align_up((size_t)lh * v.wh, 64);
        v.fmt = (l == levels - 1) ? FMT_F32 : msg_fmt;
        v.layout = l >= pm_from ? PIXEL_MAJOR : LABEL_MAJOR;
        v.cost_fmt = COST_F32;
        if (v.layout == PIXEL_MAJOR) {
            v.lp = S * R;
            v.blk = v.plane * v.lp;
            v.ls = 1;
            v.ps = v.lp;
        } else {
            v.lp = L;
            v.blk = (int64_t)L * v.plane;
            v.ls = v.plane;
            v.ps = 1;
        }
        v.cost_bytes = align_up((size_t)2 * v.blk * sizeof(float));
        v.msg_bytes = align_up((size_t)8 * v.blk * fmt_bytes(v.fmt));
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

// The pixel-major lane-split kernel is the faster half-sweep at every level
// size measured on MI355X (676x380x64: 55 vs 70 us per finest-level sweep;
// 1352x760x128: 444 vs 680 us; small levels are latency-bound under the
// lanes-over-pixels kernel's per-lane label chain), so every level defaults to it.
int default_pm_from(int w, int h, int L, int levels, int msg_fmt)
{
    (void)w;
    (void)h;
    (void)L;
    (void)levels;
    (void)msg_fmt;
    return 0;
}

bp_status launch_status()
{
    return hipGetLastError() == hipSuccess ? BP_OK : BP_ERR_HIP;
}

static inline unsigned cdiv(int64_t n, int64_t d) { return (unsigned)((n + d - 1) / d); }

// ------------------------------------------------------------------------
// a3: finest-level cost in the level's layout, and the sum pyramid
// ------------------------------------------------------------------------

// planar [L][h][w] -> label-major colour-split.  grid (w/256, h, L).
__global__ void __launch_bounds__(256) k_split_lm(const float *__restrict__ planar, float *__restrict__ out,
                                                 LevelDesc d)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, f = blockIdx.z;
    if (x >= d.w) return;
    const float v = planar[((int64_t)f * d.h + y) * d.w + x];
    out[cost_idx((x + y) & 1, f, y * d.wh + (x >> 1), d.blk, d.ls, d.ps)] = v;
}

// Cost of one pixel and label at a label-major or planar source level, summed
// over the (up to four) children when SUM (pyramid step), in the order
// (0,0), (1,0), (0,1), (1,1).
template <bool FROM_PLANAR, bool SUM>
__device__ __forceinline__ float gather_cost(const float *__restrict__ src, const LevelDesc &s, int f, int x, int y)
{
    auto at = [&](int fx, int fy) -> float {
        if constexpr (FROM_PLANAR) return src[((int64_t)f * s.h + fy) * s.w + fx];
        else return src[cost_idx((fx + fy) & 1, f, fy * s.wh + (fx >> 1), s.blk, s.ls, s.ps)];
    };
    if constexpr (!SUM) {
        return at(x, y);
    } else {
        float acc = 0.0f;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int ii = 0; ii < 2; ++ii) {
                const int fx = 2 * x + ii, fy = 2 * y + jj;
                if (fx < s.w && fy < s.h) acc += at(fx, fy);
            }
        return acc;
    }
}

// Transposing tile: 64 pixels of one row x 32 labels, read along the row from a
// planar or label-major source and written along the labels into a
// pixel-major level.  grid (w_out/64, h_out, L/32).
template <bool FROM_PLANAR, bool SUM>
__global__ void __launch_bounds__(256) k_to_pm(const float *__restrict__ src, LevelDesc s, float *__restrict__ out,
                                              LevelDesc d, int L)
{
    __shared__ float tile[32][65];
    const int x0 = blockIdx.x * 64, y = blockIdx.y, f0 = blockIdx.z * 32;
    for (int i = threadIdx.x; i < 64 * 32; i += 256) {
        const int fl = i / 64, xl = i % 64;
        const int x = x0 + xl, f = f0 + fl;
        float v = 0.0f;
        if (x < d.w && f < L) v = gather_cost<FROM_PLANAR, SUM>(src, s, f, x, y);
        tile[fl][xl] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * 32; i += 256) {
        const int xl = i / 32, fl = i % 32;
        const int x = x0 + xl, f = f0 + fl;
        if (x < d.w && f < L) out[cost_idx((x + y) & 1, f, y * d.wh + (x >> 1), d.blk, d.ls, d.ps)] = tile[fl][xl];
    }
}

// Planar [L][h][w] -> pixel-major level with 16-byte accesses both ways:
// a block moves 64 pixels of one row x 64 labels through LDS, loading four
// consecutive pixels of one label per lane (256-byte runs along the row) and
// storing four consecutive labels of one pixel per lane (a pixel's labels
// are contiguous).  Needs w % 4 == 0 and a 16-byte aligned source; labels
// from L up to the next multiple of four are stored as zero (they lie inside
// the pixel's padded row, lp being a multiple of four).  grid (w/64, h, L/64).
__global__ void __launch_bounds__(256) k_split_pm4(const float *__restrict__ src, float *__restrict__ out,
                                                  LevelDesc d, int L)
{
    __shared__ float tile[64][65];
    const int x0 = blockIdx.x * 64, y = blockIdx.y, f0 = blockIdx.z * 64;
    const int t = threadIdx.x, q = t & 15, r = t >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int fl = r + 16 * i, f = f0 + fl, x = x0 + 4 * q;
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (f < L && x < d.w) v = *(const float4 *)(src + ((int64_t)f * d.h + y) * d.w + x);
        tile[fl][4 * q] = v.x;
        tile[fl][4 * q + 1] = v.y;
        tile[fl][4 * q + 2] = v.z;
        tile[fl][4 * q + 3] = v.w;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int xl = r + 16 * i, x = x0 + xl, f = f0 + 4 * q;
        if (x < d.w && f < L) {
            const int fl = 4 * q;
            const float4 v = make_float4(tile[fl][xl], tile[fl + 1][xl], tile[fl + 2][xl], tile[fl + 3][xl]);
            *(float4 *)(out + cost_idx((x + y) & 1, f, y * d.wh + (x >> 1), d.blk, d.ls, d.ps)) = v;
        }
    }
}

// label-major -> label-major pyramid step.  grid (wc/256, hc, L).
__global__ void __launch_bounds__(256) k_pyr_lm(const float *__restrict__ fine, LevelDesc s, float *__restrict__ out,
                                               LevelDesc d)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, f = blockIdx.z;
    if (x >= d.w) return;
    out[cost_idx((x + y) & 1, f, y * d.wh + (x >> 1), d.blk, d.ls, d.ps)] = gather_cost<false, true>(fine, s, f, x, y);
}

// pixel-major -> pixel-major pyramid step: threads along (pixel, label) with
// the label fastest.  grid (wc * L / 256, hc).
__global__ void __launch_bounds__(256) k_pyr_pm(const float *__restrict__ fine, LevelDesc s, float *__restrict__ out,
                                               LevelDesc d, int L)
{
    const int i = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (i >= d.w * L) return;
    const int x = i / L, f = i - x * L;
    float acc = 0.0f;
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
            const int fx = 2 * x + ii, fy = 2 * y + jj;
            if (fx < s.w && fy < s.h) acc += fine[cost_idx((fx + fy) & 1, f, fy * s.wh + (fx >> 1), s.blk, s.ls, s.ps)];
        }
    out[cost_idx((x + y) & 1, f, y * d.wh + (x >> 1), d.blk, d.ls, d.ps)] = acc;
}

bp_status launch_split_cost(const float *planar, const Plan &p, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[0];
    float *out = (float *)(ws + v.cost_off);
    LevelDesc d = desc(v);
    if (v.layout == PIXEL_MAJOR && v.w % 4 == 0 && ((uintptr_t)planar % 16) == 0) {
        k_split_pm4<<<dim3(cdiv(v.w, 64), v.h, cdiv(p.L, 64)), 256, 0, s>>>(planar, out, d, p.L);
    } else if (v.layout == PIXEL_MAJOR) {
        LevelDesc src{v.w, v.h, 0, 0, 0, 0};
        k_to_pm<true, false><<<dim3(cdiv(v.w, 64), v.h, cdiv(p.L, 32)), 256, 0, s>>>(planar, src, out, d, p.L);
    } else {
        k_split_lm<<<dim3(cdiv(v.w, 256), v.h, p.L), 256, 0, s>>>(planar, out, d);
    }
    return launch_status();
}

// Up to three pixel-major pyramid levels in one launch: the thread of label f
// of pixel (x, y) of the last level sums its subtree level by level (the
// children of every node added in the order of k_pyr_pm, so every stored
// value is bit-identical to level-by-level launches) and stores every node.
// grid (ceil(w_top * L / 256), h_top).
struct PyrChain {
    const float *src;
    LevelDesc sd;
    float *out[3];
    LevelDesc od[3];
};

// The 4^K source values under node (x, y) of chain level K, loaded before any
// store so that every load is in flight at once; children outside their
// level's grid are skipped (their slots are never read).
template <int K>
__device__ __forceinline__ void pyr_leaves(const PyrChain &a, int x, int y, int f, float *v)
{
    if constexpr (K == 0) {
        v[0] = a.src[cost_idx((x + y) & 1, f, y * a.sd.wh + (x >> 1), a.sd.blk, a.sd.ls, a.sd.ps)];
    } else {
        const LevelDesc &cd = K == 1 ? a.sd : a.od[K - 2];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int ii = 0; ii < 2; ++ii) {
                const int fx = 2 * x + ii, fy = 2 * y + jj;
                if (fx < cd.w && fy < cd.h) pyr_leaves<K - 1>(a, fx, fy, f, v + (2 * jj + ii) * (1 << (2 * (K - 1))));
            }
    }
}

// Sum of node (x, y) of chain level K from its loaded leaves, storing every
// node of the subtree.
template <int K>
__device__ __forceinline__ float pyr_reduce(const PyrChain &a, int x, int y, int f, const float *v)
{
    if constexpr (K == 0) {
        return v[0];
    } else {
        const LevelDesc &cd = K == 1 ? a.sd : a.od[K - 2];
        float acc = 0.0f;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int ii = 0; ii < 2; ++ii) {
                const int fx = 2 * x + ii, fy = 2 * y + jj;
                if (fx < cd.w && fy < cd.h) acc += pyr_reduce<K - 1>(a, fx, fy, f, v + (2 * jj + ii) * (1 << (2 * (K - 1))));
            }
        const LevelDesc &d = a.od[K - 1];
        a.out[K - 1][cost_idx((x + y) & 1, f, y * d.wh + (x >> 1), d.blk, d.ls, d.ps)] = acc;
        return acc;
    }
}

template <int D>
__global__ void __launch_bounds__(256) k_pyr_pm_chain(const PyrChain a, int L)
{
    const int i = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (i >= a.od[D - 1].w * L) return;
    const int x = i / L, f = i - x * L;
    float v[1 << (2 * D)];
    pyr_leaves<D>(a, x, y, f, v);
    pyr_reduce<D>(a, x, y, f, v);
}

bp_status launch_pyramid(const Plan &p, int first, uint8_t *ws, hipStream_t s)
{
    for (int l = first; l < p.levels;) {
        int D = 0;
        while (D < 3 && l + D < p.levels && p.lv[l + D].layout == PIXEL_MAJOR && p.lv[l - 1].layout == PIXEL_MAJOR) ++D;
        if (D < 2) {
            const bp_status st = launch_pyramid_level(p, l, ws, s);
            if (st != BP_OK) return st;
            ++l;
            continue;
        }
        PyrChain a;
        a.src = (const float *)(ws + p.lv[l - 1].cost_off);
        a.sd = desc(p.lv[l - 1]);
        for (int k = 0; k < 3; ++k) {
            const Level &v = p.lv[k < D ? l + k : l];
            a.out[k] = (float *)(ws + v.cost_off);
            a.od[k] = desc(v);
        }
        const Level &top = p.lv[l + D - 1];
        const dim3 grid(cdiv((int64_t)top.w * p.L, 256), top.h);
        if (D == 3) k_pyr_pm_chain<3><<<grid, 256, 0, s>>>(a, p.L);
        else k_pyr_pm_chain<2><<<grid, 256, 0, s>>>(a, p.L);
        const bp_status st = launch_status();
        if (st != BP_OK) return st;
        l += D;
    }
    return BP_OK;
}

bp_status launch_pyramid_level(const Plan &p, int l, uint8_t *ws, hipStream_t s)
{
    const Level &f = p.lv[l - 1], &c = p.lv[l];
    const float *fine = (const float *)(ws + f.cost_off);
    float *out = (float *)(ws + c.cost_off);
    if (c.layout == LABEL_MAJOR) {
        k_pyr_lm<<<dim3(cdiv(c.w, 256), c.h, p.L), 256, 0, s>>>(fine, desc(f), out, desc(c));
    } else if (f.layout == LABEL_MAJOR) {
        k_to_pm<false, true><<<dim3(cdiv(c.w, 64), c.h, cdiv(p.L, 32)), 256, 0, s>>>(fine, desc(f), out, desc(c), p.L);
    } else {
        k_pyr_pm<<<dim3(cdiv((int64_t)c.w * p.L, 256), c.h), 256, 0, s>>>(fine, desc(f), out, desc(c), p.L);
    }
    return launch_status();
}

// ------------------------------------------------------------------------
// a4: message initialisation and explicit parent copy
// ------------------------------------------------------------------------

// grid (blocks, levels + 1): block (x, y) is init_msgs_block(x, y).
__global__ void __launch_bounds__(256) k_init_msgs(InitArgs a) { init_msgs_block(a, blockIdx.x, blockIdx.y); }

bp_status launch_zero_borders(const Plan *plans, uint8_t *const *bases, int count, int n, hipStream_t s)
{
    // Entries (problem, state) in order, up to kMaxLevels per launch and one
    // label count per launch.
    InitArgs a;
    int m = 0;
    int64_t most = 0;
    auto flush = [&]() -> bp_status {
        if (m == 0) return BP_OK;
        a.levels = m;
        a.coarsest_words = 0;
        k_init_msgs<<<dim3((unsigned)((most + 255) / 256), m), 256, 0, s>>>(a);
        m = 0;
        most = 0;
        return launch_status();
    };
    bp_status st = BP_OK;
    for (int i = 0; i < count && st == BP_OK; ++i) {
        const Plan &p = plans[i];
        const Level &v = p.lv[0];
        for (int j = 0; j < n && st == BP_OK; ++j) {
            if (m == kMaxLevels || (m > 0 && a.L != p.L)) st = flush();
            if (st != BP_OK) break;
            a.msg[m] = bases[i] + (size_t)j * v.msg_bytes;
            a.d[m] = desc(v);
            a.bytes[m] = fmt_bytes(v.fmt);
            a.L = p.L;
            const int64_t per = (2 * (int64_t)v.h + 2 * (int64_t)v.w) * p.L;
            if (per > most) most = per;
            ++m;
        }
    }
    return st == BP_OK ? flush() : st;
}

bp_status launch_init_messages(const Plan &p, uint8_t *ws, hipStream_t s)
{
    unsigned blocks;
    const InitArgs a = init_args(p, ws, &blocks);
    k_init_msgs<<<dim3(blocks, p.levels + 1), 256, 0, s>>>(a);
    return launch_status();
}

// Child slot k of pixel (x, y) takes the parent's slot k at (x/2, y/2),
// converted to the child's storage format.  grid (wc/256, hc, 4L).
template <typename SP, typename SC>
__global__ void __launch_bounds__(256) k_parent_copy(const uint8_t *__restrict__ pm, uint32_t pm_bytes, LevelDesc pd,
                                                    uint8_t *__restrict__ cm, uint32_t cm_bytes, LevelDesc cd, int L)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    const int k = blockIdx.z / L, f = blockIdx.z - k * L;
    if (x >= cd.w) return;
    const int px = x >> 1, py = y >> 1;
    const int64_t src = msg_idx((px + py) & 1, k, f, py * pd.wh + (px >> 1), pd.blk, pd.ls, pd.ps);
    const int64_t dst = msg_idx((x + y) & 1, k, f, y * cd.wh + (x >> 1), cd.blk, cd.ls, cd.ps);
    const float v = SP::ld(make_rsrc(pm, pm_bytes), (uint32_t)(src * SP::bytes), 0);
    SC::st(make_rsrc(cm, cm_bytes), v, (uint32_t)(dst * SC::bytes), 0);
}

// Pixel-major levels: lanes along (pixel, label) with the label fastest, so
// both the parent's and the child's label rows are read and written
// contiguously.  grid (w * L / 256, h, 4 slots).
template <typename SP, typename SC>
__global__ void __launch_bounds__(256) k_parent_copy_pm(const uint8_t *__restrict__ pm, uint32_t pm_bytes,
                                                       LevelDesc pd, uint8_t *__restrict__ cm, uint32_t cm_bytes,
                                                       LevelDesc cd, int L)
{
    const int i = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, k = blockIdx.z;
    if (i >= cd.w * L) return;
    const int x = i / L, f = i - x * L;
    const int px = x >> 1, py = y >> 1;
    const int64_t src = msg_idx((px + py) & 1, k, f, py * pd.wh + (px >> 1), pd.blk, pd.ls, pd.ps);
    const int64_t dst = msg_idx((x + y) & 1, k, f, y * cd.wh + (x >> 1), cd.blk, cd.ls, cd.ps);
    const float v = SP::ld(make_rsrc(pm, pm_bytes), (uint32_t)(src * SP::bytes), 0);
    SC::st(make_rsrc(cm, cm_bytes), v, (uint32_t)(dst * SC::bytes), 0);
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

bp_status launch_parent_copy(const Plan &p, int l, uint8_t *ws, hipStream_t s)
{
    const Level &c = p.lv[l], &pa = p.lv[l + 1];
    return with_store(pa.fmt, [&](auto sp) {
        return with_store(c.fmt, [&](auto sc) {
            using SP = decltype(sp);
            using SC = decltype(sc);
            if (c.layout == PIXEL_MAJOR && pa.layout == PIXEL_MAJOR)
                k_parent_copy_pm<SP, SC><<<dim3(cdiv((int64_t)c.w * p.L, 256), c.h, 4), 256, 0, s>>>(
                    ws + pa.msg_off, (uint32_t)pa.msg_bytes, desc(pa), ws + c.msg_off, (uint32_t)c.msg_bytes, desc(c),
                    p.L);
            else
                k_parent_copy<SP, SC><<<dim3(cdiv(c.w, 256), c.h, 4 * p.L), 256, 0, s>>>(
                    ws + pa.msg_off, (uint32_t)pa.msg_bytes, desc(pa), ws + c.msg_off, (uint32_t)c.msg_bytes, desc(c),
                    p.L);
            return launch_status();
        });
    });
}

// ------------------------------------------------------------------------
// a5: half-sweep dispatch
// ------------------------------------------------------------------------

IterArgs make_iter_args(const Plan &p, int l, int t, int src_mode, float lambda, float tau, int32_t *disp,
                        uint8_t *ws)
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
    a.blk = (uint32_t)v.blk;
    a.ls = (uint32_t)v.ls;
    a.ps = (uint32_t)v.ps;
    a.lp = (uint32_t)v.lp;
    const Level &src = src_mode == 1 ? p.lv[l + 1] : v;
    a.src = ws + src.msg_off;
    a.src_bytes = (uint32_t)src.msg_bytes;
    a.sblk = (uint32_t)src.blk;
    a.sls = (uint32_t)src.ls;
    a.sps = (uint32_t)src.ps;
    a.src_wh = src.wh;
    a.src_w = src.w;
    a.src_h = src.h;
    a.src_parent = src_mode == 1;
    a.colour = t & 1;
    a.L = p.L;
    a.ncomp = v.h * v.wh;
    a.lambda = lambda;
    a.lt = lambda * tau;
    a.near = tau <= 2.0f ? 1 : tau <= 3.0f ? 2 : 0;
    return a;
}

bp_status launch_iteration(const Plan &p, int l, int t, int src_mode, float lambda, float tau, int32_t *disp,
                           int variant, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[l];
    const IterArgs a = make_iter_args(p, l, t, src_mode, lambda, tau, disp, ws);
    if (v.layout == PIXEL_MAJOR) {
        int S, R;
        bool xchg;
        pm_split_variant(p.L, variant, &S, &R, &xchg);
        return dispatch_iter_pm(a, v.fmt, S, R, disp != nullptr, xchg, s);
    }
    return dispatch_iter_lm(a, v.fmt, iteration_lanes(p.L, variant), disp != nullptr, s);
}

PairArgs make_pair_args(const Plan &p, int l, int src_kind, size_t src_off, size_t dst_off, bool write_c1,
                        float lambda, float tau, int32_t *disp, uint8_t *ws, uint8_t *ck, bool ck_c1, float *soft,
                        float inv_t)
{
    const Level &v = p.lv[l];
    PairArgs a;
    a.cost = (const float *)(ws + v.cost_off);
    a.cost_bytes = (uint32_t)v.cost_bytes;
    a.msg = ws + v.msg_off;
    a.msg_bytes = (uint32_t)v.msg_bytes;
    const uint32_t half = (uint32_t)((size_t)4 * v.blk * fmt_bytes(v.fmt));
    if (src_kind == PAIR_SRC_PARENT) {
        const Level &pa = p.lv[l + 1];
        a.src = ws + pa.msg_off;
        a.src_bytes = (uint32_t)pa.msg_bytes;
        a.sblk = (uint32_t)pa.blk;
        a.sps = (uint32_t)pa.ps;
        a.src_wh = pa.wh;
    } else {
        a.src = ws + src_off;
        a.src_bytes = half;
        a.sblk = (uint32_t)v.blk;
        a.sps = (uint32_t)v.ps;
        a.src_wh = v.wh;
    }
    a.src_parent = src_kind == PAIR_SRC_PARENT;
    a.src_zero = src_kind == PAIR_SRC_ZERO;
    a.dst = ws + dst_off;
    a.dst_bytes = half;
    a.write_c1 = write_c1;
    a.disp = disp;
    a.soft = soft;
    a.inv_t = inv_t;
    a.w = v.w;
    a.h = v.h;
    a.wh = v.wh;
    a.blk = (uint32_t)v.blk;
    a.lp = (uint32_t)v.lp;
    a.L = p.L;
    a.lambda = lambda;
    a.lt = lambda * tau;
    a.near = tau <= 2.0f ? 1 : tau <= 3.0f ? 2 : 0;
    a.cost_fmt = v.cost_fmt;
    pair_tile(v.lp, fmt_bytes(v.fmt), v.w, v.h, &a.tx, &a.ty);
    a.tiles_x = (v.w + a.tx - 1) / a.tx;
    a.ntiles = a.tiles_x * ((v.h + a.ty - 1) / a.ty);
    a.per_xcd = (a.ntiles + 7) / 8;
    a.ck = ck;
    a.ck_bytes = ck ? (uint32_t)v.msg_bytes : 0u;
    a.ck_c1 = ck != nullptr && ck_c1;
    return a;
}

bp_status launch_iteration_pair(const Plan &p, int l, int src_kind, size_t src_off, size_t dst_off, bool write_c1,
                                float lambda, float tau, int32_t *disp, uint8_t *ws, hipStream_t s, uint8_t *ck,
                                bool ck_c1, float *soft, float inv_t)
{
    const PairArgs a =
        make_pair_args(p, l, src_kind, src_off, dst_off, write_c1, lambda, tau, disp, ws, ck, ck_c1, soft, inv_t);
    int S, R;
    pm_split(p.L, &S, &R);
    return dispatch_iter_pm2(a, p.lv[l].fmt, S, R, disp != nullptr || soft != nullptr, s);
}

bp_status launch_iteration_from(const Plan &p, int t, const uint8_t *src, float lambda, float tau, int variant,
                                uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[0];
    IterArgs a = make_iter_args(p, 0, t, 0, lambda, tau, nullptr, ws);
    a.src = src;
    if (v.layout == PIXEL_MAJOR) {
        int S, R;
        bool xchg;
        pm_split_variant(p.L, variant, &S, &R, &xchg);
        return dispatch_iter_pm(a, v.fmt, S, R, false, xchg, s);
    }
    return dispatch_iter_lm(a, v.fmt, iteration_lanes(p.L, variant), false, s);
}

// ------------------------------------------------------------------------
// a6: readout, message export
// ------------------------------------------------------------------------

// Label-major readout: belief b(f) = cost(f) + m_0 + m_1 + m_2 + m_3 at every
// pixel of colour blockIdx.y (if in `mask`); lowest-index argmin, and
// soft-argmin sum f w / sum w with w = exp(-(b - min b) / T) accumulated with a
// running minimum.  grid (ncomp/256, 2).
template <typename S>
__global__ void __launch_bounds__(256) k_readout_lm(const float *__restrict__ cost, uint32_t cost_bytes,
                                                   const uint8_t *__restrict__ msg, uint32_t msg_bytes, LevelDesc d,
                                                   int L, int mask, int32_t *__restrict__ disp,
                                                   float *__restrict__ soft, float inv_t)
{
    const int c = blockIdx.y;
    if (!((mask >> c) & 1)) return;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= d.h * d.wh) return;
    const int y = j / d.wh;
    const int x = 2 * (j - y * d.wh) + ((y + c) & 1);
    if (x >= d.w) return;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(cost, cost_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(msg, msg_bytes);
    const uint32_t co = (uint32_t)(c * d.blk + j) * 4u;
    uint32_t mo[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) mo[k] = (uint32_t)((c * 4 + k) * d.blk + j) * S::bytes;
    const uint32_t cls = (uint32_t)d.ls * 4u, mls = (uint32_t)d.ls * S::bytes;
    float best = __builtin_huge_valf();
    int bidx = 0;
    float num = 0.0f, den = 0.0f;
#pragma unroll 8
    for (int f = 0; f < L; ++f) {
        float b = ld_f32(rc, co, (uint32_t)f * cls);
#pragma unroll
        for (int k = 0; k < 4; ++k) b += S::ld(rm, mo[k], (uint32_t)f * mls);
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
    const int64_t o = (int64_t)y * d.w + x;
    if (disp) disp[o] = bidx;
    if (soft) soft[o] = num / den;
}

// Pixel-major readout: SEG lanes per pixel, R labels per lane; a block
// covers 256 / SEG pixels of one row of one colour.  grid (ceil(wh * SEG /
// 256), h, colours), colour c0 + blockIdx.z.
template <int SEG, int R, typename S, int CF>
__global__ void __launch_bounds__(256) k_readout_pm(const float *__restrict__ cost, uint32_t cost_bytes,
                                                   const uint8_t *__restrict__ msg, uint32_t msg_bytes, LevelDesc d,
                                                   int lp, int L, int c0, int32_t *__restrict__ disp,
                                                   float *__restrict__ soft, float inv_t)
{
    const int c = c0 + (int)blockIdx.z, y = (int)blockIdx.y;
    const int i = (int)(blockIdx.x * 256 + threadIdx.x) / SEG, s = (int)threadIdx.x % SEG;
    if (i >= d.wh) return;
    const int j = y * d.wh + i;
    const int x = 2 * i + ((y + c) & 1);
    if (x >= d.w) return;
    const __amdgpu_buffer_rsrc_t rc = make_rsrc(cost, cost_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(msg, msg_bytes);
    const int f0 = s * R;
    float b[R], m[R];
    ld_cost<R, CF>(rc, (uint32_t)(c * d.blk) + (uint32_t)j * lp + f0, b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ld_row<S, R>(rm, ((uint32_t)((c * 4 + k) * d.blk) + (uint32_t)j * lp + f0) * S::bytes, m);
#pragma unroll
        for (int r = 0; r < R; ++r) b[r] += m[r];
    }
    int bi;
    float sv;
    pm_readout<SEG, R, false>(b, f0, L, soft != nullptr, inv_t, bi, sv);
    const int64_t o = (int64_t)y * d.w + x;
    if (soft && s == 0) soft[o] = sv;
    if (disp && s == 0) disp[o] = bi;
}

bp_status launch_readout(const Plan &p, int colour_mask, int32_t *disp, float *soft, float temperature, uint8_t *ws,
                         hipStream_t s)
{
    const Level &v = p.lv[0];
    const int64_t ncomp = (int64_t)v.h * v.wh;
    const float inv_t = soft ? 1.0f / temperature : 0.0f;
    return with_store(v.fmt, [&](auto st) {
        using S = decltype(st);
        const float *cost = (const float *)(ws + v.cost_off);
        const uint8_t *msg = ws + v.msg_off;
        if (v.layout == LABEL_MAJOR) {
            k_readout_lm<S><<<dim3(cdiv(ncomp, 256), 2), 256, 0, s>>>(cost, (uint32_t)v.cost_bytes, msg,
                                                                     (uint32_t)v.msg_bytes, desc(v), p.L, colour_mask,
                                                                     disp, soft, inv_t);
            return launch_status();
        }
        int SEGV, R;
        pm_split(p.L, &SEGV, &R);
        // Colours 0 and 1, or just the one the mask names.
        const int c0 = colour_mask == 2 ? 1 : 0, nc = colour_mask == 3 ? 2 : 1;
#define BP_RO_LAUNCH(SV, RV, CFV)                                                                              \
    k_readout_pm<SV, RV, S, CFV><<<dim3(cdiv((int64_t)v.wh * SV, 256), v.h, nc), 256, 0, s>>>(                 \
        cost, (uint32_t)v.cost_bytes, msg, (uint32_t)v.msg_bytes, desc(v), v.lp, p.L, c0, disp, soft, inv_t)
#define BP_RO_CASE(SV, RV)                                                                                      \
    if (SEGV == SV && R == RV) {                                                                                \
        if (v.cost_fmt == COST_F16) BP_RO_LAUNCH(SV, RV, COST_F16);                                             \
        else if (v.cost_fmt == COST_U8) {                                                                       \
            if constexpr (RV % 4 == 0) BP_RO_LAUNCH(SV, RV, COST_U8);                                           \
            else return BP_ERR_UNSUPPORTED;                                                                     \
        } else BP_RO_LAUNCH(SV, RV, COST_F32);                                                                  \
        return launch_status();                                                                                 \
    }
        BP_RO_CASE(4, 4)
        BP_RO_CASE(8, 4)
        BP_RO_CASE(16, 4)
        BP_RO_CASE(16, 6)
        BP_RO_CASE(16, 8)
        BP_RO_CASE(16, 12)
        BP_RO_CASE(16, 16)
#undef BP_RO_CASE
#undef BP_RO_LAUNCH
        return BP_ERR_UNSUPPORTED;
    });
}

// Messages of level 0 -> planar float32 [4][L][h][w]; slots without a
// neighbour read as zero.  grid (w/256, h, 4L).
template <typename S>
__global__ void __launch_bounds__(256) k_export(const uint8_t *__restrict__ msg, uint32_t msg_bytes, LevelDesc d, int L,
                                               float *__restrict__ out)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    const int k = blockIdx.z / L, f = blockIdx.z - k * L;
    if (x >= d.w) return;
    const bool ok = (k == 0) ? x > 0 : (k == 1) ? x < d.w - 1 : (k == 2) ? y > 0 : y < d.h - 1;
    float v = 0.0f;
    if (ok) {
        const int64_t idx = msg_idx((x + y) & 1, k, f, y * d.wh + (x >> 1), d.blk, d.ls, d.ps);
        v = S::ld(make_rsrc(msg, msg_bytes), (uint32_t)(idx * S::bytes), 0);
    }
    out[(((int64_t)k * L + f) * d.h + y) * d.w + x] = v;
}

// Pixel-major level 0: through an LDS tile of 32 consecutive pixels of one
// row (their slot-k rows read as contiguous runs, labels written as 128-byte
// runs of x; rows padded by one word).  grid (ceil(w / 32), h, 4).
template <typename S, int LP>
__global__ void __launch_bounds__(256) k_export_pm(const uint8_t *__restrict__ msg, uint32_t msg_bytes, LevelDesc d,
                                                  int L, float *__restrict__ out)
{
    __shared__ float tile[32][LP + 1];
    const int x0 = blockIdx.x * 32, y = blockIdx.y, k = blockIdx.z;
    const __amdgpu_buffer_rsrc_t r = make_rsrc(msg, msg_bytes);
    for (int e = threadIdx.x; e < 32 * LP; e += 256) {
        const int p = e / LP, f = e - p * LP;
        const int x = x0 + p;
        if (x >= d.w) continue;
        const bool ok = (k == 0) ? x > 0 : (k == 1) ? x < d.w - 1 : (k == 2) ? y > 0 : y < d.h - 1;
        float v = 0.0f;
        if (ok) {
            const int64_t idx = msg_idx((x + y) & 1, k, f, y * d.wh + (x >> 1), d.blk, d.ls, d.ps);
            v = S::ld(r, (uint32_t)(idx * S::bytes), 0);
        }
        tile[p][f] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * L; e += 256) {
        const int f = e / 32, p = e - f * 32;
        const int x = x0 + p;
        if (x < d.w) out[(((int64_t)k * L + f) * d.h + y) * d.w + x] = tile[p][f];
    }
}

bp_status launch_export(const Plan &p, float *out, uint8_t *ws, hipStream_t s)
{
    const Level &v = p.lv[0];
    return with_store(v.fmt, [&](auto st) {
        using S = decltype(st);
        if (v.layout == PIXEL_MAJOR) {
            const dim3 grid(cdiv(v.w, 32), v.h, 4);
            const uint8_t *m = ws + v.msg_off;
            const uint32_t mb = (uint32_t)v.msg_bytes;
            switch (v.lp) {
            case 16: k_export_pm<S, 16><<<grid, 256, 0, s>>>(m, mb, desc(v), p.L, out); break;
            case 32: k_export_pm<S, 32><<<grid, 256, 0, s>>>(m, mb, desc(v), p.L, out); break;
            case 64: k_export_pm<S, 64><<<grid, 256, 0, s>>>(m, mb, desc(v), p.L, out); break;
            case 96: k_export_pm<S, 96><<<grid, 256, 0, s>>>(m, mb, desc(v), p.L, out); break;
            case 128: k_export_pm<S, 128><<<grid, 256, 0, s>>>(m, mb, desc(v), p.L, out); break;
            case 192: k_export_pm<S, 192><<<grid, 256, 0, s>>>(m, mb, desc(v), p.L, out); break;
            case 256: k_export_pm<S, 256><<<grid, 256, 0, s>>>(m, mb, desc(v), p.L, out); break;
            default: return BP_ERR_UNSUPPORTED;
            }
            return launch_status();
        }
        k_export<S><<<dim3(cdiv(v.w, 256), v.h, 4 * p.L), 256, 0, s>>>(ws + v.msg_off, (uint32_t)v.msg_bytes, desc(v),
                                                                        p.L, out);
        return launch_status();
    });
}

}  // namespace bpk
