// a5, pixel-major levels: host side of the fused pair of half-sweeps (the
// kernels are in bp_iter_pm2_impl.h, compiled per message storage format in
// bp_iter_pm2_f32.hip, bp_iter_pm2_f16.hip and bp_iter_pm2_bf16.hip): tile
// choice, launch shapes, the batched form's entry table, and dispatch by
// storage format.
#include <hip/hip_runtime.h>

#include "bp_device.h"
#include "bp_internal.h"

namespace bpk {

template <typename S>
bp_status pm2_single(const PairArgs &a, size_t lds, int SEGV, int R, bool ro, hipStream_t st);
template <typename S>
bp_status pm2_batch(const PairEntry *tab, int n, int blocks, size_t lds, int SEGV, int R, bool exact, bool ro,
                    int cf, hipStream_t st);

// Table of batch entries written from kernel arguments (capture-safe).
__global__ void k_write_pair_entries(PairEntry *__restrict__ dst, PairChunk c)
{
    const int i = threadIdx.x;
    if (i < c.n) dst[i] = c.e[i];
}

bp_status launch_write_pair_entries(PairEntry *dst, const PairEntry *src, int n, hipStream_t st)
{
    for (int i = 0; i < n; i += kPairChunk) {
        PairChunk c;
        c.n = n - i < kPairChunk ? n - i : kPairChunk;
        for (int k = 0; k < c.n; ++k) c.e[k] = src[i + k];
        k_write_pair_entries<<<1, 64, 0, st>>>(dst + i, c);
        const bp_status s = launch_status();
        if (s != BP_OK) return s;
    }
    return BP_OK;
}

int pair_blocks(const PairArgs &a) { return 8 * a.per_xcd; }

// Tile of a fused pair at a w x h level: the squarest of a few shapes whose
// colour-1 rows fit 32 KiB of LDS (TX x TY / 2 pixels x 4 rows x lp values of
// mb bytes, the storage format), halved (rows first) while the level has
// fewer than 512 tiles, so that small levels still spread over every compute
// unit (down to 4 x 4).  Measured at 64 labels in FP32 (level sums of the
// benchmarked pair's pairs, finest / next level): 8 x 8 tiles (32 KiB, four
// blocks per CU) 315 / 94 us, 16 x 4 313 / 97, 16 x 8 (64 KiB, two blocks)
// 356 / 119, 8 x 4 344 / 94, 32 x 4 369 / 121; a ring of 1.56 colour-0 pixels
// per tile colour-1 pixel costs less than the lower occupancy of larger tiles.
void pair_tile(int lp, int mb, int w, int h, int *tx, int *ty)
{
    const int px = 32768 / (4 * lp * mb);   // colour-1 pixels that fit
    if (px >= 128) { *tx = 16; *ty = 16; }
    else if (px >= 64) { *tx = 16; *ty = 8; }
    else if (px >= 32) { *tx = 8; *ty = 8; }
    else if (px >= 16) { *tx = 8; *ty = 4; }
    else { *tx = 4; *ty = 4; }
    auto tiles = [&](int a, int b) { return (int64_t)((w + a - 1) / a) * ((h + b - 1) / b); };
    while (tiles(*tx, *ty) < 512 && (*tx > 4 || *ty > 4)) {
        if (*ty >= *tx && *ty > 4) *ty /= 2;
        else *tx /= 2;
    }
}

size_t pair_lds_bytes(int tx, int ty, int lp, int mb) { return (size_t)tx * ty / 2 * 4 * lp * mb; }

// Every entry of a launch has the same cost storage (cf).
bp_status launch_iteration_pair_batch(const PairEntry *tab, int n, int blocks, size_t lds, int fmt, int SEGV, int R,
                                      bool exact, bool ro, int cf, hipStream_t st)
{
    if (lds > 65536) return BP_ERR_UNSUPPORTED;
    switch (fmt) {
    case FMT_F16: return pm2_batch<StoreF16>(tab, n, blocks, lds, SEGV, R, exact, ro, cf, st);
    case FMT_BF16: return pm2_batch<StoreBF16>(tab, n, blocks, lds, SEGV, R, exact, ro, cf, st);
    default: return pm2_batch<StoreF32>(tab, n, blocks, lds, SEGV, R, exact, ro, cf, st);
    }
}


bool pair_supported(int SEGV, int R)
{
    return (SEGV == 4 && R == 4) || (SEGV == 8 && R == 4) ||
           (SEGV == 16 && (R == 4 || R == 6 || R == 8 || R == 12 || R == 16));
}

bp_status dispatch_iter_pm2(const PairArgs &a, int fmt, int SEGV, int R, bool ro, hipStream_t st)
{
    const size_t lds = pair_lds_bytes(a.tx, a.ty, (int)a.lp, fmt_bytes(fmt));
    if (lds > 65536 || (a.tx & 1) || a.tx <= 0 || a.ty <= 0) return BP_ERR_UNSUPPORTED;
    switch (fmt) {
    case FMT_F16: return pm2_single<StoreF16>(a, lds, SEGV, R, ro, st);
    case FMT_BF16: return pm2_single<StoreBF16>(a, lds, SEGV, R, ro, st);
    default: return pm2_single<StoreF32>(a, lds, SEGV, R, ro, st);
    }
}

}  // namespace bpk
