// a5, label-major levels: one checkerboard half-sweep with lanes over pixels.
//
// A group of G lanes (1, 2 or 4) serves one sender pixel; lane `sub` owns the
// outgoing messages k = sub*(4/G) .. +4/G-1, the message to the neighbour on
// side k (0 left, 1 right, 2 up, 3 down), which excludes what that neighbour
// sent (incoming slot k):
//   S(f)   = cost(f) + sum_k m_k(f)             (group sum over the G lanes)
//   h_k(f) = S(f) - m_k(f)
//   a(f)   = min(h_k(f), a(f-1) + lambda)       forward pass, kept in registers
//   b(f)   = min(a(f), b(f+1) + lambda, min h_k + lambda*tau)   backward pass
//   out(f) = b(f) - min h_k
// Folding the truncation into the backward pass and normalising by min h_k are
// exact rewrites of "two-pass transform, then min(., min h + lambda*tau), then
// subtract the minimum": addition is monotone, and the transform's minimum is
// min h_k.  The message lands in the neighbour's slot k^1 (it sees this pixel
// on the opposite side).  Every label plane is read and written with one
// coalesced access per wave; per-label offsets are uniform (scalar) buffer
// offsets, and out-of-grid slots hold zero, so loads need no predicate.
#include <hip/hip_runtime.h>

#include "bp_device.h"
#include "bp_internal.h"

namespace bpk {

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

    // Per-lane byte offsets of label 0; label f adds f * ls * bytes (uniform).
    const uint32_t cost_off = ((uint32_t)a.colour * a.blk + (uint32_t)j) * 4u;
    uint32_t src_off[ND];
    uint32_t dst_off[ND];
    bool has[ND];
    {
        int sj = j, sc = a.colour;
        if (a.src_parent) {
            const int sx = x >> 1, sy = y >> 1;
            sc = (sx + sy) & 1;
            sj = sy * a.src_wh + (sx >> 1);
        }
#pragma unroll
        for (int i = 0; i < ND; ++i) {
            const int k = sub * ND + i;
            src_off[i] = (((uint32_t)sc * 4u + (uint32_t)k) * a.sblk + (uint32_t)sj * a.sps) * S::bytes;
            int nx = x, ny = y;
            bool ok;
            if (k == 0) { nx = x - 1; ok = x > 0; }
            else if (k == 1) { nx = x + 1; ok = x < a.w - 1; }
            else if (k == 2) { ny = y - 1; ok = y > 0; }
            else { ny = y + 1; ok = y < a.h - 1; }
            has[i] = ok;
            const uint32_t dj = ok ? (uint32_t)(ny * a.wh + (nx >> 1)) : 0u;
            dst_off[i] = (((uint32_t)(a.colour ^ 1) * 4u + (uint32_t)(k ^ 1)) * a.blk + dj) * S::bytes;
        }
    }
    const float lam = a.lambda;
    const float inf = __builtin_huge_valf();
    const uint32_t cls = a.ls * 4u, sls = a.sls * S::bytes, dls = a.ls * S::bytes;

    // Prefetch ring: cost and owned incoming messages of labels f .. f+PD-1.
    float pc[PD], pm[PD][ND];
    auto issue = [&](int f, int slot) {
        if (EXACT || f < nl) {
            pc[slot] = ld_f32(rc, cost_off, (uint32_t)f * cls);
#pragma unroll
            for (int i = 0; i < ND; ++i) pm[slot][i] = S::ld(rs, src_off[i], (uint32_t)f * sls);
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
            asm volatile("" : "+v"(best), "+v"(bidx));
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
            if (EXACT || f < nl) S::st(rm, v - mn[i], dst_off[i], (uint32_t)f * dls);
        }
    }
}

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
static void launch_ro(const IterArgs &a, bool ro, unsigned grid, hipStream_t s)
{
    if (ro) k_iter<LP, G, S, EXACT, true><<<grid, 256, 0, s>>>(a);
    else k_iter<LP, G, S, EXACT, false><<<grid, 256, 0, s>>>(a);
}

template <typename S>
static bp_status dispatch_lm(const IterArgs &a, int G, bool ro, hipStream_t s)
{
    const unsigned grid = (unsigned)(((int64_t)a.ncomp * G + 255) / 256);
    const int L = a.L;
#define BP_ITER_CASE(LV, GV, EX)                       \
    if (G == GV) {                                     \
        launch_ro<LV, GV, S, EX>(a, ro, grid, s);      \
        return launch_status();                        \
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

bp_status dispatch_iter_lm(const IterArgs &a, int fmt, int G, bool ro, hipStream_t s)
{
    switch (fmt) {
    case FMT_F16: return dispatch_lm<StoreF16>(a, G, ro, s);
    case FMT_BF16: return dispatch_lm<StoreBF16>(a, G, ro, s);
    default: return dispatch_lm<StoreF32>(a, G, ro, s);
    }
}

}  // namespace bpk
