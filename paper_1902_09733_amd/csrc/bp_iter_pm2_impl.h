// a5, pixel-major levels: two consecutive checkerboard half-sweeps (t, t + 1,
// t even) fused into one launch by tiling the level.
//
// Half-sweep t sends from the colour-0 pixels (x + y even) into the incoming
// slots of the colour-1 pixels, and half-sweep t + 1 reads exactly those slots
// and nothing else written at t; afterwards they are dead until half-sweep
// t + 2 overwrites them.  A block owns a TX x TY tile (TX even, tile origin
// even) and runs
//   phase 1: every colour-0 pixel of the tile and of a one-pixel ring around
//            it (the ring pixels belong to neighbouring tiles, which compute
//            them too) reads its cost and four incoming rows and computes
//            its four outgoing messages; those whose receiver is a colour-1
//            pixel of the tile go to LDS (rounded to the storage format),
//            the rest are dropped;
//   phase 2: every colour-1 pixel of the tile reads its cost from memory and
//            its four incoming rows from LDS and sends its four messages to
//            its colour-0 neighbours (inside the tile or on the ring).
// So colour 1's incoming rows never travel to memory, which removes their
// write and re-read: per pixel pair and two half-sweeps the traffic is two
// costs, one colour-0 incoming state read and one written (plus the ring's
// reads), against two costs, both states read and both written.
//
// Phase 1 of one tile reads colour-0 rows of ring pixels that phase 2 of the
// neighbouring tile writes in the same launch, so colour 0's incoming slots
// are double-buffered: phase 1 reads `src` (the level's own state or a
// second buffer of the same layout, or the parent level's final state for
// t = 0) and phase 2 writes `dst`, the other one.  The host alternates them so
// that the level's last pair writes the level's own state.  When the pair
// ends the level (or precedes a last single half-sweep), phase 1 also stores
// colour 1's incoming rows into the level's state, which the next level's
// parent copy and the readout read.
//
// A forward run that saves states for the adjoint passes a checkpoint state
// (`ck`, the level's layout): phase 2's rows are written there too, which
// replaces a copy of the state half, and phase 1's as well for the final
// state (`ck_c1`; the level's own colour-1 block then need not be written
// when nothing else reads it).
//
// The level's cost is read as FP32, or as FP16 or bytes (CF) where the plan
// keeps the finest level's cost narrower (a pair's integer costs, exact there).
//
// Per message the arithmetic is the one-half-sweep kernel's variant 1
// (bp_pm_core.h: h summed in slot order, the same transform), so results
// equal two launches of that kernel bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include "bp_device.h"
#include "bp_internal.h"
#include "bp_pm_core.h"

namespace bpk {

// A pixel owns SEG lanes, lane s holding labels [s R, s R + R) of its cost and
// incoming rows, and computes its four outgoing messages in turn (as the
// one-half-sweep kernel's variant 1).  U pixels per lane group are loaded
// before any is computed, to keep more rows in flight per wave.
template <int SEG, int R, typename S, bool EXACT, bool RO, int NT, int U, int CF>
__device__ __forceinline__ void pm2_tile(const PairArgs &a, int b, uint8_t *lds)
{
    // lds: [tile colour-1 pixel][slot][lp] in the storage format
    constexpr int PPB = NT / SEG;        // lane groups (pixels at a time) per block
    // Tile of block b: blocks b, b + 8, ... run on one XCD of the eight and
    // take a contiguous run of tiles, so a tile's ring comes from its own L2.
    const int tile = (b & 7) * a.per_xcd + (b >> 3);
    if (tile >= a.ntiles) return;
    const int TX = a.tx, TY = a.ty, HX = TX >> 1;
    const int tx0 = (tile % a.tiles_x) * TX, ty0 = (tile / a.tiles_x) * TY;
    const int g = (int)threadIdx.x / SEG, s = (int)threadIdx.x % SEG, f0 = s * R;
    const uint32_t lp = a.lp;

    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost, a.cost_bytes);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.src, a.src_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(a.msg, a.msg_bytes);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(a.dst, a.dst_bytes);
    const __amdgpu_buffer_rsrc_t rk = make_rsrc(a.ck, a.ck_bytes);

    // Phase 1: colour-0 pixels of [tx0 - 1, tx0 + TX] x [ty0 - 1, ty0 + TY]
    // without the corners, HX + 1 per row.
    const int n1 = (TY + 2) * (HX + 1);
    for (int i0 = g; i0 < n1; i0 += PPB * U) {
        int xs[U], ys[U];
        bool live[U];
        float c[U][R], m[U][4][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * PPB;
            const int r = i / (HX + 1), cc = i - r * (HX + 1);
            const int y = ty0 - 1 + r;
            const int x = tx0 - 1 + 2 * cc + ((tx0 - 1 + y) & 1);
            xs[u] = x;
            ys[u] = y;
            live[u] = i < n1 && x >= 0 && x < a.w && y >= 0 && y < a.h &&
                      !((r == 0 || r == TY + 1) && (x < tx0 || x >= tx0 + TX));
            if (!live[u]) continue;
            const int j = y * a.wh + (x >> 1);
            int sj = j, sc = 0;
            if (a.src_parent) {
                const int sx = x >> 1, sy = y >> 1;
                sc = (sx + sy) & 1;
                sj = sy * a.src_wh + (sx >> 1);
            }
            ld_cost<R, CF>(rc, (uint32_t)j * lp + (uint32_t)f0, c[u]);
            const uint32_t base = (uint32_t)sj * a.sps + (uint32_t)f0;
            // Slots from outside the grid are zero; they are not read, since
            // the second buffer never holds them.
            const bool has[4] = {x > 0, x < a.w - 1, y > 0, y < a.h - 1};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                if (!a.src_zero && has[kk]) {
                    ld_row<S, R>(rs, (((uint32_t)sc * 4u + (uint32_t)kk) * a.sblk + base) * S::bytes, m[u][kk]);
                } else {
#pragma unroll
                    for (int q = 0; q < R; ++q) m[u][kk][q] = 0.0f;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!live[u]) continue;
            with_near<R>(a.near, [&](auto near_form) {
                constexpr int NEAR = decltype(near_form)::value;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    int nx, ny;
                    const bool ok = pm_receiver(k, xs[u], ys[u], a.w, a.h, nx, ny);
                    // Only receivers inside the tile (colour 1 by construction);
                    // the same for every lane of the pixel.
                    if (!(ok && nx >= tx0 && nx < tx0 + TX && ny >= ty0 && ny < ty0 + TY)) continue;
                    float h[R], out[R];
                    pm_h<R>(c[u], m[u], k, h);
                    pm_transform<SEG, R, EXACT, NEAR>(h, s, f0, a.L, a.lambda, a.lt, out);
                    const int slot = (ny - ty0) * HX + ((nx - tx0) >> 1);
                    uint8_t *row = lds + (((uint32_t)slot * 4u + (uint32_t)(k ^ 1)) * lp + f0) * S::bytes;
                    if constexpr (S::bytes == 4) {
#pragma unroll
                        for (int q = 0; q < R; ++q) ((float *)row)[q] = out[q];
                    } else {
#pragma unroll
                        for (int q = 0; q < R / 2; ++q)
                            ((uint32_t *)row)[q] = S::pack2(out[2 * q], out[2 * q + 1]);
                    }
                    if (a.write_c1 || a.ck_c1) {
                        const uint32_t dj = (uint32_t)(ny * a.wh + (nx >> 1));
                        const uint32_t off = ((4u + (uint32_t)(k ^ 1)) * a.blk + dj * lp + (uint32_t)f0) * S::bytes;
                        if (a.write_c1) st_row<S, R>(rm, off, out);
                        if (a.ck_c1) st_row<S, R>(rk, off, out);
                    }
                }
            });
        }
    }
    __syncthreads();

    // Phase 2: the tile's colour-1 pixels, HX per row.
    const int n2 = TY * HX;
    for (int i0 = g; i0 < n2; i0 += PPB * U) {
        int xs[U], ys[U];
        bool live[U];
        float c[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * PPB;
            const int r = i / HX, cc = i - r * HX;
            const int y = ty0 + r;
            const int x = tx0 + 2 * cc + ((tx0 + y + 1) & 1);
            xs[u] = x;
            ys[u] = y;
            live[u] = i < n2 && x < a.w && y < a.h;
            if (!live[u]) continue;
            const int j = y * a.wh + (x >> 1);
            ld_cost<R, CF>(rc, (a.blk + (uint32_t)j * lp) + (uint32_t)f0, c[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!live[u]) continue;
            const int i = i0 + u * PPB, x = xs[u], y = ys[u];
            // Slots from outside the grid hold zero (never written above).
            const bool has[4] = {x > 0, x < a.w - 1, y > 0, y < a.h - 1};
            const uint8_t *row = lds + ((uint32_t)i * 4u * lp + f0) * S::bytes;
            float m[4][R];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                if constexpr (S::bytes == 4) {
                    const float *rk = (const float *)row + kk * lp;
#pragma unroll
                    for (int q = 0; q < R; ++q) m[kk][q] = has[kk] ? rk[q] : 0.0f;
                } else {
                    const uint32_t *rk = (const uint32_t *)(row + (size_t)kk * lp * S::bytes);
#pragma unroll
                    for (int q = 0; q < R / 2; ++q) {
                        const uint32_t w = has[kk] ? rk[q] : 0u;
                        m[kk][2 * q] = S::decode((uint16_t)(w & 0xffffu));
                        m[kk][2 * q + 1] = S::decode((uint16_t)(w >> 16));
                    }
                }
            }
            if constexpr (RO) {
                float bel[R], sv;
                int bi;
                pm_belief<R>(c[u], m, bel);
                pm_readout<SEG, R, EXACT>(bel, f0, a.L, a.soft != nullptr, a.inv_t, bi, sv);
                if (s == 0 && a.disp) a.disp[(int64_t)y * a.w + x] = bi;
                if (s == 0 && a.soft) a.soft[(int64_t)y * a.w + x] = sv;
            }
            with_near<R>(a.near, [&](auto near_form) {
                constexpr int NEAR = decltype(near_form)::value;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    int nx, ny;
                    if (!pm_receiver(k, x, y, a.w, a.h, nx, ny)) continue;
                    float h[R], out[R];
                    pm_h<R>(c[u], m, k, h);
                    pm_transform<SEG, R, EXACT, NEAR>(h, s, f0, a.L, a.lambda, a.lt, out);
                    const uint32_t dj = (uint32_t)(ny * a.wh + (nx >> 1));
                    const uint32_t off = ((uint32_t)(k ^ 1) * a.blk + dj * lp + (uint32_t)f0) * S::bytes;
                    st_row<S, R>(rd, off, out);
                    if (a.ck) st_row<S, R>(rk, off, out);
                }
            });
        }
    }
}

template <int SEG, int R, typename S, bool EXACT, bool RO, int NT, int U, int CF>
__global__ void __launch_bounds__(NT) k_iter_pm2(const PairArgs a)
{
    extern __shared__ uint8_t lds[];
    pm2_tile<SEG, R, S, EXACT, RO, NT, U, CF>(a, (int)blockIdx.x, lds);
}

// Batched fused pair: block b belongs to the last table entry whose first
// block is <= b; every entry's first block is a multiple of 8, so the XCD
// grouping of tiles holds within each problem.  EXACT: every entry's label
// count fills its lane split.
template <int SEG, int R, typename S, bool EXACT, bool RO, int NT, int U, int CF>
__global__ void __launch_bounds__(NT) k_iter_pm2_batch(const PairEntry *__restrict__ tab, int n)
{
    extern __shared__ uint8_t lds[];
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const PairArgs a = tab[lo].a;
    pm2_tile<SEG, R, S, EXACT, RO, NT, U, CF>(a, (int)blockIdx.x - tab[lo].block0, lds);
}

constexpr int kPairThreads = 512;

template <int SEG, int R, typename S, bool EXACT, bool RO>
static bp_status launch_pm2(const PairArgs &a, size_t lds, hipStream_t st)
{
    const unsigned grid = (unsigned)pair_blocks(a);
    if (a.cost_fmt == COST_F16) {
        k_iter_pm2<SEG, R, S, EXACT, RO, kPairThreads, 1, COST_F16><<<grid, kPairThreads, lds, st>>>(a);
    } else if (a.cost_fmt == COST_U8) {
        if constexpr (R % 4 == 0) k_iter_pm2<SEG, R, S, EXACT, RO, kPairThreads, 1, COST_U8><<<grid, kPairThreads, lds, st>>>(a);
        else return BP_ERR_UNSUPPORTED;
    } else {
        k_iter_pm2<SEG, R, S, EXACT, RO, kPairThreads, 1, COST_F32><<<grid, kPairThreads, lds, st>>>(a);
    }
    return launch_status();
}

template <typename S, bool EXACT, int CF>
static bp_status dispatch_pm2_batch(const PairEntry *tab, int n, int blocks, size_t lds, int SEGV, int R, bool ro,
                                    hipStream_t st)
{
#define BP_PM2B(SV, RV)                                                                                          \
    if (SEGV == SV && R == RV) {                                                                                 \
        if constexpr (CF == COST_U8 && RV % 4 != 0) return BP_ERR_UNSUPPORTED;                                  \
        else if (ro) k_iter_pm2_batch<SV, RV, S, EXACT, true, kPairThreads, 1, CF><<<blocks, kPairThreads, lds, st>>>(tab, n); \
        else k_iter_pm2_batch<SV, RV, S, EXACT, false, kPairThreads, 1, CF><<<blocks, kPairThreads, lds, st>>>(tab, n);  \
        return launch_status();                                                                                  \
    }
    BP_PM2B(4, 4) BP_PM2B(8, 4) BP_PM2B(16, 4) BP_PM2B(16, 6) BP_PM2B(16, 8) BP_PM2B(16, 12) BP_PM2B(16, 16)
#undef BP_PM2B
    return BP_ERR_UNSUPPORTED;
}

template <typename S>
static bp_status dispatch_pm2_batch_exact(const PairEntry *tab, int n, int blocks, size_t lds, int SEGV, int R,
                                          bool exact, bool ro, int cf, hipStream_t st)
{
    if (cf == COST_F16)
        return exact ? dispatch_pm2_batch<S, true, COST_F16>(tab, n, blocks, lds, SEGV, R, ro, st)
                     : dispatch_pm2_batch<S, false, COST_F16>(tab, n, blocks, lds, SEGV, R, ro, st);
    if (cf == COST_U8)
        return exact ? dispatch_pm2_batch<S, true, COST_U8>(tab, n, blocks, lds, SEGV, R, ro, st)
                     : dispatch_pm2_batch<S, false, COST_U8>(tab, n, blocks, lds, SEGV, R, ro, st);
    return exact ? dispatch_pm2_batch<S, true, COST_F32>(tab, n, blocks, lds, SEGV, R, ro, st)
                 : dispatch_pm2_batch<S, false, COST_F32>(tab, n, blocks, lds, SEGV, R, ro, st);
}

template <int SEG, int R, typename S>
static bp_status launch_pm2_ro(const PairArgs &a, size_t lds, bool ro, hipStream_t st)
{
    const bool exact = a.L == SEG * R;
    if (exact) return ro ? launch_pm2<SEG, R, S, true, true>(a, lds, st) : launch_pm2<SEG, R, S, true, false>(a, lds, st);
    return ro ? launch_pm2<SEG, R, S, false, true>(a, lds, st) : launch_pm2<SEG, R, S, false, false>(a, lds, st);
}

template <typename S>
static bp_status dispatch_pm2(const PairArgs &a, size_t lds, int SEGV, int R, bool ro, hipStream_t st)
{
#define BP_PM2(SV, RV) \
    if (SEGV == SV && R == RV) return launch_pm2_ro<SV, RV, S>(a, lds, ro, st);
    BP_PM2(4, 4) BP_PM2(8, 4) BP_PM2(16, 4) BP_PM2(16, 6) BP_PM2(16, 8) BP_PM2(16, 12) BP_PM2(16, 16)
#undef BP_PM2
    return BP_ERR_UNSUPPORTED;
}

// The entry points of one storage format, explicitly instantiated in
// bp_iter_pm2_<format>.hip (one translation unit per format, so that the
// kernels of the three formats compile in parallel).
template <typename S>
bp_status pm2_single(const PairArgs &a, size_t lds, int SEGV, int R, bool ro, hipStream_t st)
{
    return dispatch_pm2<S>(a, lds, SEGV, R, ro, st);
}

template <typename S>
bp_status pm2_batch(const PairEntry *tab, int n, int blocks, size_t lds, int SEGV, int R, bool exact, bool ro,
                    int cf, hipStream_t st)
{
    return dispatch_pm2_batch_exact<S>(tab, n, blocks, lds, SEGV, R, exact, ro, cf, st);
}

}  // namespace bpk
