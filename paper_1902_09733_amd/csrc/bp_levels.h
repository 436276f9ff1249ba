// Level geometry shared by the kernels of bp_core.hip and bp_cost.hip: the
// colour-split cost and message addresses of a level, and the message
// initialisation (out-of-grid slots of every level and the coarsest level's
// whole state start at zero), which the pair route runs in the same launch as
// the pair packing.
#pragma once

#include <hip/hip_runtime.h>

#include "bp_internal.h"

namespace bpk {

__device__ __forceinline__ int64_t cost_idx(int c, int f, int j, int64_t blk, int64_t ls, int64_t ps)
{
    return (int64_t)c * blk + (int64_t)f * ls + (int64_t)j * ps;
}

__device__ __forceinline__ int64_t msg_idx(int c, int k, int f, int j, int64_t blk, int64_t ls, int64_t ps)
{
    return ((int64_t)c * 4 + k) * blk + (int64_t)f * ls + (int64_t)j * ps;
}

// Level geometry passed by value to kernels.
struct LevelDesc {
    int w, h, wh;
    int64_t blk, ls, ps;
};

static inline LevelDesc desc(const Level &v) { return LevelDesc{v.w, v.h, v.wh, v.blk, v.ls, v.ps}; }

struct InitArgs {
    uint8_t *msg[kMaxLevels];
    LevelDesc d[kMaxLevels];
    int bytes[kMaxLevels];     // bytes per stored value
    int L, levels;
    int64_t coarsest_words;    // 32-bit words of the coarsest level's messages
};

// The arguments of the initialisation of plan p and its block count per row
// of the (blocks, levels + 1) block grid.
static inline InitArgs init_args(const Plan &p, uint8_t *ws, unsigned *blocks)
{
    InitArgs a;
    int64_t most = 0;
    for (int l = 0; l < p.levels; ++l) {
        a.msg[l] = ws + p.lv[l].msg_off;
        a.d[l] = desc(p.lv[l]);
        a.bytes[l] = fmt_bytes(p.lv[l].fmt);
        const int64_t n = (2 * (int64_t)p.lv[l].h + 2 * (int64_t)p.lv[l].w) * p.L;
        if (n > most) most = n;
    }
    a.L = p.L;
    a.levels = p.levels;
    a.coarsest_words = p.zero_coarsest ? (int64_t)(p.lv[p.levels - 1].msg_bytes / 4) : 0;
    if (a.coarsest_words / 4 > most) most = a.coarsest_words / 4;
    *blocks = (unsigned)((most + 255) / 256);
    return a;
}

// Block (bx, l) of the initialisation.  l < levels: zero the out-of-grid
// slots of level l (for every label: slot 0 of the left column, 1 of the right
// column, 2 of the top row, 3 of the bottom row).  l == levels: zero every
// message of the coarsest level, where BP starts from zero messages (nothing
// to do when the plan's first fused pair reads zeros instead).
__device__ __forceinline__ void init_msgs_block(const InitArgs &a, int bx, int l)
{
    const int64_t i = (int64_t)bx * 256 + threadIdx.x;
    if (l == a.levels) {
        // The coarsest level's whole state, 16 bytes per thread (its size is
        // a multiple of 256 bytes).
        if (i < a.coarsest_words / 4) ((uint4 *)a.msg[a.levels - 1])[i] = make_uint4(0u, 0u, 0u, 0u);
        return;
    }
    const LevelDesc &d = a.d[l];
    const int per = 2 * d.h + 2 * d.w;
    if (i >= (int64_t)per * a.L) return;
    const int ii = (int)i;
    // Consecutive threads take consecutive labels where a pixel's labels are
    // contiguous (pixel-major), else consecutive border pixels.
    int f, e;
    if (d.ls == 1) {
        e = ii / a.L;
        f = ii - e * a.L;
    } else {
        f = ii / per;
        e = ii - f * per;
    }
    int x, y, k;
    if (e < d.h) { x = 0; y = e; k = 0; }
    else if (e < 2 * d.h) { x = d.w - 1; y = e - d.h; k = 1; }
    else if (e < 2 * d.h + d.w) { x = e - 2 * d.h; y = 0; k = 2; }
    else { x = e - 2 * d.h - d.w; y = d.h - 1; k = 3; }
    const int64_t idx = msg_idx((x + y) & 1, k, f, y * d.wh + (x >> 1), d.blk, d.ls, d.ps);
    if (a.bytes[l] == 4) ((uint32_t *)a.msg[l])[idx] = 0u;
    else ((uint16_t *)a.msg[l])[idx] = 0u;
}

}  // namespace bpk
