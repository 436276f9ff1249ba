// a5, pixel-major levels: one checkerboard half-sweep with the labels of a
// pixel spread over lanes and the distance transform done as wave-level
// min-plus scans.
//
// Lane s of a sender pixel's SEG lanes holds labels [s*R, s*R + R) of its
// cost and of its four incoming slots (16-byte vectors: a pixel's labels are
// contiguous in this layout) and computes, for each outgoing message k (0
// left, 1 right, 2 up, 3 down),
//   h(f) = cost(f) + sum of the incoming messages except slot k   (order 0..3)
// and its transform (variants 1 and 2; variants 3 to 5 give each message its
// own SEG lanes instead, see pm_sweep).  Measured on MI355X, the per-message
// lane split spent 208 VALU instructions per pixel (one wave per pixel at 64
// labels), most of them index arithmetic and h sums repeated by each of the
// four lane groups, and left the finest half-sweep bound by instruction issue;
// the lane holding all four messages spends about 82.
// The transform splits the minimum over g by where g lies:
//   own lane  two lane-local passes over its R labels, forward
//             a(f) = min(h(f), a(f - 1) + lambda) and backward
//             b(f) = min(a(f), b(f + 1) + lambda);
//   below     min_{s'<s} (a_s'(last) - lambda R s') + lambda R (s - 1) is the
//             value entering the lane at label sR - 1 (exclusive DPP
//             prefix-min over the segment);
//   above     min_{s'>s} (b_s'(first) + lambda R s') - lambda R (s + 1) is the
//             value entering at label (s + 1) R (exclusive DPP suffix-min);
//   out(f)    = min(b(f), below + lambda (f - sR + 1), above + lambda (sR + R - f),
//                   min h + lambda tau) - min h   (DPP min-reduction for min h).
// The two scans and the reduction are independent and run interleaved.  When
// tau <= 2 (or tau <= 3 with four labels per lane) the transform reduces to
// its three- (five-) label form (bp_pm_core.h).
// With integer-valued data every step is exact, so the result equals the
// sequential two-pass transform bit for bit.  Labels past L are +inf in h and
// never influence real labels.
#include <hip/hip_runtime.h>

#include "bp_device.h"
#include "bp_internal.h"
#include "bp_pm_core.h"

namespace bpk {

// Variants 1 and 2: a sender pixel owns SEG lanes, lane s holding labels
// [s R, s R + R) of the cost and of all four incoming rows (five 16-byte
// row loads per lane, no load repeated), and computes the four outgoing
// messages of those labels in turn (h in slot order, then the transform).
// Per pixel this is a quarter of the lanes of the four-group split below,
// so the index arithmetic and the h sums are shared by the four messages.
template <int SEG, int R, typename S, bool EXACT, bool RO>
__device__ __forceinline__ void pm_sweep4(const IterArgs &a, uint32_t block)
{
    const uint32_t gid = block * 256u + threadIdx.x;
    const int j = (int)(gid / SEG);
    const int s = (int)(gid % SEG);       // label segment
    if (j >= a.ncomp) return;
    const int y = j / a.wh;
    const int x = 2 * (j - y * a.wh) + ((y + a.colour) & 1);
    if (x >= a.w) return;

    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost, a.cost_bytes);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.src, a.src_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(a.msg, a.msg_bytes);
    const int f0 = s * R;
    int sj = j, sc = a.colour;
    if (a.src_parent) {
        const int sx = x >> 1, sy = y >> 1;
        sc = (sx + sy) & 1;
        sj = sy * a.src_wh + (sx >> 1);
    }
    const uint32_t base = (uint32_t)sj * a.sps + (uint32_t)f0;
    float c[R], m[4][R];
    ld_row<StoreF32, R>(rc, ((uint32_t)a.colour * a.blk + (uint32_t)j * a.lp + (uint32_t)f0) * 4u, c);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
        ld_row<S, R>(rs, (((uint32_t)sc * 4u + (uint32_t)kk) * a.sblk + base) * S::bytes, m[kk]);

    if constexpr (RO) {
        float bel[R];
        pm_belief<R>(c, m, bel);
        const int bi = pm_argmin<SEG, R, EXACT>(bel, f0, a.L);
        if (s == 0 && a.disp) a.disp[(int64_t)y * a.w + x] = bi;
    }
    // All four h rows up front with shared partial sums while they fit the
    // registers comfortably; one at a time for long label rows.
    constexpr bool H4 = R <= 8;
    float h4[H4 ? 4 : 1][R];
    if constexpr (H4) pm_h4<R>(c, m, h4);
    with_near<R>(a.near, [&](auto near_form) {
        constexpr int NEAR = decltype(near_form)::value;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float h[R], out[R];
            if constexpr (H4) {
#pragma unroll
                for (int r = 0; r < R; ++r) h[r] = h4[k][r];
            } else {
                pm_h<R>(c, m, k, h);
            }
            pm_transform<SEG, R, EXACT, NEAR>(h, s, f0, a.L, a.lambda, a.lt, out);
            int nx, ny;
            if (pm_receiver(k, x, y, a.w, a.h, nx, ny)) {
                const uint32_t dj = (uint32_t)(ny * a.wh + (nx >> 1));
                st_row<S, R>(rm, (((uint32_t)(a.colour ^ 1) * 4u + (uint32_t)(k ^ 1)) * a.blk + dj * a.lp +
                                  (uint32_t)f0) * S::bytes,
                             out);
            }
        }
    });
}

// Variants 3 to 5: a sender pixel owns 4 SEG lanes, SEG per outgoing message.
template <int SEG, int R, typename S, bool EXACT, bool RO, bool XCHG>
__device__ __forceinline__ void pm_sweep(const IterArgs &a, uint32_t block)
{
    constexpr int GP = 4 * SEG;           // lanes per pixel
    const uint32_t gid = block * 256u + threadIdx.x;
    const int j = (int)(gid / GP);
    const int lane = (int)(gid % GP);
    const int k = lane / SEG;             // outgoing message / excluded incoming slot
    const int s = lane % SEG;             // label segment
    if (j >= a.ncomp) return;
    const int y = j / a.wh;
    const int x = 2 * (j - y * a.wh) + ((y + a.colour) & 1);
    if (x >= a.w) return;

    const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.cost, a.cost_bytes);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.src, a.src_bytes);
    const __amdgpu_buffer_rsrc_t rm = make_rsrc(a.msg, a.msg_bytes);
    const int f0 = s * R;

    const float inf = __builtin_huge_valf();
    const float lam = a.lambda;
    const float lamR = lam * (float)R;
    int sj = j, sc = a.colour;
    if (a.src_parent) {
        const int sx = x >> 1, sy = y >> 1;
        sc = (sx + sy) & 1;
        sj = sy * a.src_wh + (sx >> 1);
    }
    const uint32_t base = (uint32_t)sj * a.sps + (uint32_t)f0;
    const uint32_t cost_off = ((uint32_t)a.colour * a.blk + (uint32_t)j * a.lp + (uint32_t)f0) * 4u;
    float h[R];
    float bel[R];   // belief cost + sum of the four incoming rows (fused readout)
    if constexpr (!XCHG) {
        // Every lane reads the cost and all four incoming rows of its labels
        // and sums in slot order, adding zero for the excluded slot.
        float c[R], m[4][R];
        ld_row<StoreF32, R>(rc, cost_off, c);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            ld_row<S, R>(rs, (((uint32_t)sc * 4u + (uint32_t)kk) * a.sblk + base) * S::bytes, m[kk]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float v = c[r];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) v += (kk == k) ? 0.0f : m[kk][r];
            h[r] = v;
            if constexpr (RO) bel[r] = (((c[r] + m[0][r]) + m[1][r]) + m[2][r]) + m[3][r];
        }
    } else {
        // Each lane group reads only its own incoming row (group 0 also the
        // cost); the four groups' partial sums are exchanged across lanes
        // (DPP and lane swaps): total = ((cost + m0) + m1) + (m2 + m3),
        // h = total - m_k.
        float own[R], part[R];
        ld_row<S, R>(rs, (((uint32_t)sc * 4u + (uint32_t)k) * a.sblk + base) * S::bytes, own);
        if (k == 0) {
            float c[R];
            ld_row<StoreF32, R>(rc, cost_off, c);
#pragma unroll
            for (int r = 0; r < R; ++r) part[r] = c[r] + own[r];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) part[r] = own[r];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float tot = xor_sum<2 * SEG>(xor_sum<SEG>(part[r]));
            h[r] = tot - own[r];
            if constexpr (RO) bel[r] = tot;
        }
    }

    if constexpr (RO) {
        const int bi = pm_argmin<SEG, R, EXACT>(bel, f0, a.L);
        if (k == 0 && s == 0 && a.disp) a.disp[(int64_t)y * a.w + x] = bi;
    }

    float out[R];
    with_near<R>(a.near, [&](auto near_form) {
        pm_transform<SEG, R, EXACT, decltype(near_form)::value>(h, s, f0, a.L, lam, a.lt, out);
    });

    // Receiver of message k and its slot k^1.
    int nx = x, ny = y;
    bool ok;
    if (k == 0) { nx = x - 1; ok = x > 0; }
    else if (k == 1) { nx = x + 1; ok = x < a.w - 1; }
    else if (k == 2) { ny = y - 1; ok = y > 0; }
    else { ny = y + 1; ok = y < a.h - 1; }
    if (ok) {
        const uint32_t dj = (uint32_t)(ny * a.wh + (nx >> 1));
        st_row<S, R>(rm, (((uint32_t)(a.colour ^ 1) * 4u + (uint32_t)(k ^ 1)) * a.blk + dj * a.lp + (uint32_t)f0) *
                             S::bytes,
                     out);
    }
}

template <int SEG, int R, typename S, bool EXACT, bool RO, bool XCHG>
__global__ void __launch_bounds__(256) k_iter_pm(const IterArgs a)
{
    if constexpr (XCHG) pm_sweep<SEG, R, S, EXACT, RO, true>(a, blockIdx.x);
    else pm_sweep4<SEG, R, S, EXACT, RO>(a, blockIdx.x);
}

// Batched half-sweep: the problems of one launch share the lane split; block
// b belongs to the last table entry whose first block is <= b.
template <int SEG, int R, typename S, bool XCHG, bool RO>
__global__ void __launch_bounds__(256) k_iter_pm_batch(const BatchEntry *__restrict__ tab, int n)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].block0 <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const IterArgs a = tab[lo].a;
    if constexpr (XCHG) pm_sweep<SEG, R, S, false, RO, true>(a, blockIdx.x - (uint32_t)tab[lo].block0);
    else pm_sweep4<SEG, R, S, false, RO>(a, blockIdx.x - (uint32_t)tab[lo].block0);
}

// Table of batch entries written from kernel arguments (capture-safe: no
// host buffer has to outlive the call).
__global__ void k_write_entries(BatchEntry *__restrict__ dst, EntryChunk c)
{
    const int i = threadIdx.x;
    if (i < c.n) dst[i] = c.e[i];
}

bp_status launch_write_entries(BatchEntry *dst, const BatchEntry *src, int n, hipStream_t st)
{
    for (int i = 0; i < n; i += kChunk) {
        EntryChunk c;
        c.n = n - i < kChunk ? n - i : kChunk;
        for (int k = 0; k < c.n; ++k) c.e[k] = src[i + k];
        k_write_entries<<<1, 64, 0, st>>>(dst + i, c);
        const bp_status s = launch_status();
        if (s != BP_OK) return s;
    }
    return BP_OK;
}

template <int SEG, int R, typename S>
static bp_status launch_pm_batch(const BatchEntry *tab, int n, int blocks, bool xchg, bool ro, hipStream_t st)
{
    if (xchg) {
        if (ro) k_iter_pm_batch<SEG, R, S, true, true><<<blocks, 256, 0, st>>>(tab, n);
        else k_iter_pm_batch<SEG, R, S, true, false><<<blocks, 256, 0, st>>>(tab, n);
    } else {
        if (ro) k_iter_pm_batch<SEG, R, S, false, true><<<blocks, 256, 0, st>>>(tab, n);
        else k_iter_pm_batch<SEG, R, S, false, false><<<blocks, 256, 0, st>>>(tab, n);
    }
    return launch_status();
}

template <typename S>
static bp_status dispatch_pm_batch(const BatchEntry *tab, int n, int blocks, int SEGV, int R, bool xchg, bool ro,
                                   hipStream_t st)
{
#define BP_PMB(SV, RV) \
    if (SEGV == SV && R == RV) return launch_pm_batch<SV, RV, S>(tab, n, blocks, xchg, ro, st);
    BP_PMB(4, 4) BP_PMB(8, 4) BP_PMB(16, 4) BP_PMB(16, 6) BP_PMB(16, 8) BP_PMB(16, 12) BP_PMB(16, 16)
    BP_PMB(4, 8) BP_PMB(8, 8) BP_PMB(8, 12) BP_PMB(8, 16)
#undef BP_PMB
#define BP_PMBX(SV, RV)                                                                                            \
    if (SEGV == SV && R == RV) {                                                                                   \
        if (!xchg) return BP_ERR_UNSUPPORTED;                                                                      \
        if (ro) k_iter_pm_batch<SV, RV, S, true, true><<<blocks, 256, 0, st>>>(tab, n);                            \
        else k_iter_pm_batch<SV, RV, S, true, false><<<blocks, 256, 0, st>>>(tab, n);                              \
        return launch_status();                                                                                    \
    }
    BP_PMBX(2, 16) BP_PMBX(4, 16) BP_PMBX(4, 24) BP_PMBX(4, 32)
#undef BP_PMBX
    return BP_ERR_UNSUPPORTED;
}

bp_status launch_iteration_batch(const BatchEntry *tab, int n, int blocks, int fmt, int SEGV, int R, bool xchg,
                                 bool ro, hipStream_t st)
{
    switch (fmt) {
    case FMT_F16: return dispatch_pm_batch<StoreF16>(tab, n, blocks, SEGV, R, xchg, ro, st);
    case FMT_BF16: return dispatch_pm_batch<StoreBF16>(tab, n, blocks, SEGV, R, xchg, ro, st);
    default: return dispatch_pm_batch<StoreF32>(tab, n, blocks, SEGV, R, xchg, ro, st);
    }
}

int pm_blocks(int ncomp, int SEGV) { return (int)(((int64_t)ncomp * 4 * SEGV + 255) / 256); }

// Blocks of a forward half-sweep: SEG lanes per pixel (variants 1, 2) or 4 SEG
// (shuffled-sum variants).
int pm_sweep_blocks(int ncomp, int SEGV, bool xchg) { return (int)(((int64_t)ncomp * (xchg ? 4 : 1) * SEGV + 255) / 256); }

void pm_split(int L, int *S, int *R)
{
    if (L <= 16) { *S = 4; *R = 4; }
    else if (L <= 32) { *S = 8; *R = 4; }
    else if (L <= 64) { *S = 16; *R = 4; }
    else if (L <= 96) { *S = 16; *R = 6; }
    else if (L <= 128) { *S = 16; *R = 8; }
    else if (L <= 192) { *S = 16; *R = 12; }
    else { *S = 16; *R = 16; }
}

static bool pm_can_halve(int L) { return L > 16 && L <= 128; }
static bool pm_can_quarter(int L) { return L > 16 && L <= 128; }

int pm_variants(int L) { return pm_can_quarter(L) ? 5 : (pm_can_halve(L) ? 4 : 2); }

// Measured on MI355X (1352x760 5-level pyramids, 32 to 128 labels): with
// FP32 storage the shuffled-sum split wins above 64 labels; with 16-bit
// storage a quarter of the lanes with shuffled sums wins at 17..64 labels
// (32-byte rows per lane), half the lanes with shuffled sums elsewhere.
int default_variant(int L, int msg_fmt)
{
    if (msg_fmt != FMT_F32) return (pm_can_quarter(L) && L <= 64) ? 5 : (pm_can_halve(L) ? 4 : 3);
    return L > 64 ? 3 : 1;
}

// Pixel-major kernel variants (same storage for all: lp = SEG * R):
//   1 default lane split, every lane reads all five rows of its labels
//   2 half the lanes per message, twice the labels per lane
//   3 default split, each lane group reads only its own row (shuffled sums)
//   4 half lanes and shuffled sums
//   5 a quarter of the lanes (four times the labels per lane) and shuffled sums
//     (17..128 labels)
// Variant 0 means 1.
void pm_split_variant(int L, int variant, int *S, int *R, bool *xchg)
{
    pm_split(L, S, R);
    if (variant <= 0 || variant > pm_variants(L)) variant = 1;
    const bool half = (variant == 2 || variant == 4) && pm_can_halve(L);
    const bool quarter = variant == 5 && pm_can_quarter(L);
    *xchg = variant >= 3;
    if (half) {
        *S /= 2;
        *R *= 2;
    }
    if (quarter) {
        *S /= 4;
        *R *= 4;
    }
}

template <int SEG, int R, typename S, bool XCHG>
static void launch_pm_x(const IterArgs &a, bool ro, unsigned grid, hipStream_t st)
{
    const bool exact = a.L == SEG * R;
    if (exact) {
        if (ro) k_iter_pm<SEG, R, S, true, true, XCHG><<<grid, 256, 0, st>>>(a);
        else k_iter_pm<SEG, R, S, true, false, XCHG><<<grid, 256, 0, st>>>(a);
    } else {
        if (ro) k_iter_pm<SEG, R, S, false, true, XCHG><<<grid, 256, 0, st>>>(a);
        else k_iter_pm<SEG, R, S, false, false, XCHG><<<grid, 256, 0, st>>>(a);
    }
}

template <int SEG, int R, typename S>
static bp_status launch_pm(const IterArgs &a, bool ro, bool xchg, hipStream_t st)
{
    const unsigned grid = (unsigned)pm_sweep_blocks(a.ncomp, SEG, xchg);
    if (xchg) launch_pm_x<SEG, R, S, true>(a, ro, grid, st);
    else launch_pm_x<SEG, R, S, false>(a, ro, grid, st);
    return launch_status();
}

// Splits that only the shuffled-sum form uses.
template <int SEG, int R, typename S>
static bp_status launch_pm_xonly(const IterArgs &a, bool ro, bool xchg, hipStream_t st)
{
    if (!xchg) return BP_ERR_UNSUPPORTED;
    launch_pm_x<SEG, R, S, true>(a, ro, (unsigned)pm_sweep_blocks(a.ncomp, SEG, true), st);
    return launch_status();
}

template <typename S>
static bp_status dispatch_pm(const IterArgs &a, int SEGV, int R, bool ro, bool xchg, hipStream_t st)
{
    if (SEGV == 2 && R == 16) return launch_pm_xonly<2, 16, S>(a, ro, xchg, st);
    if (SEGV == 4 && R == 16) return launch_pm_xonly<4, 16, S>(a, ro, xchg, st);
    if (SEGV == 4 && R == 24) return launch_pm_xonly<4, 24, S>(a, ro, xchg, st);
    if (SEGV == 4 && R == 32) return launch_pm_xonly<4, 32, S>(a, ro, xchg, st);
    if (SEGV == 4 && R == 4) return launch_pm<4, 4, S>(a, ro, xchg, st);
    if (SEGV == 8 && R == 4) return launch_pm<8, 4, S>(a, ro, xchg, st);
    if (SEGV == 16 && R == 4) return launch_pm<16, 4, S>(a, ro, xchg, st);
    if (SEGV == 16 && R == 6) return launch_pm<16, 6, S>(a, ro, xchg, st);
    if (SEGV == 16 && R == 8) return launch_pm<16, 8, S>(a, ro, xchg, st);
    if (SEGV == 16 && R == 12) return launch_pm<16, 12, S>(a, ro, xchg, st);
    if (SEGV == 16 && R == 16) return launch_pm<16, 16, S>(a, ro, xchg, st);
    if (SEGV == 4 && R == 8) return launch_pm<4, 8, S>(a, ro, xchg, st);
    if (SEGV == 8 && R == 8) return launch_pm<8, 8, S>(a, ro, xchg, st);
    if (SEGV == 8 && R == 12) return launch_pm<8, 12, S>(a, ro, xchg, st);
    if (SEGV == 8 && R == 16) return launch_pm<8, 16, S>(a, ro, xchg, st);
    return BP_ERR_UNSUPPORTED;
}

bp_status dispatch_iter_pm(const IterArgs &a, int fmt, int SEGV, int R, bool ro, bool xchg, hipStream_t st)
{
    switch (fmt) {
    case FMT_F16: return dispatch_pm<StoreF16>(a, SEGV, R, ro, xchg, st);
    case FMT_BF16: return dispatch_pm<StoreBF16>(a, SEGV, R, ro, xchg, st);
    default: return dispatch_pm<StoreF32>(a, SEGV, R, ro, xchg, st);
    }
}

}  // namespace bpk
