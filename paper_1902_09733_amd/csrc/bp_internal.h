// Internal declarations of libbpstereo: level geometry, workspace plans and
// kernel launchers.  Not part of the public ABI (see include/bp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "bp.h"

namespace bpk {

constexpr int kMaxLabels = 256;
constexpr int kMaxLevels = 16;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Storage formats of messages (values of bp_msg_dtype).
enum MsgFmt : int { FMT_F32 = 0, FMT_F16 = 1, FMT_BF16 = 2 };
inline int fmt_bytes(int fmt) { return fmt == FMT_F32 ? 4 : 2; }

// Layouts of a level's cost and messages.  Both are colour-split: pixel (x, y)
// has colour c = (x + y) & 1 and compact index j = y * wh + (x >> 1) among its
// colour's `plane` slots (wh = ceil(w / 2), plane >= h * wh).
//  LABEL_MAJOR: [colour][slot][label][plane] -- lanes over pixels read one
//               label plane at a time (coalesced along rows).
//  PIXEL_MAJOR: [colour][slot][plane][lp]    -- a pixel's labels are contiguous
//               (lp = label count padded to the lane split), so the lanes that
//               share one pixel read 16-byte vectors of consecutive labels.
// The cost has the same layout without the slot index.  Element offsets:
//   cost(c, f, j)   = c * blk + f * ls + j * ps
//   msg(c, k, f, j) = (c * 4 + k) * blk + f * ls + j * ps
enum Layout : int { LABEL_MAJOR = 0, PIXEL_MAJOR = 1 };

// Cost storage of a level (Level::cost_fmt): FP32, or, for the finest level of
// a pair whose costs are exact there, FP16 or unsigned bytes.
enum { COST_F32 = 0, COST_F16 = 1, COST_U8 = 2 };

struct Level {
    int w, h, wh;
    int64_t plane;        // compact pixel slots per colour (padded to 64)
    int layout;
    int lp;               // labels stored per pixel (L, or padded for PIXEL_MAJOR)
    int64_t blk, ls, ps;  // element strides: per (colour[, slot]) block, per label, per pixel
    int fmt;              // message storage format at this level
    size_t cost_off;      // byte offset of this level's cost in the workspace
    int cost_fmt;         // cost storage at the same element offsets: COST_F32, or for level 0 of a
                          // pair whose costs it holds exactly COST_F16 or COST_U8
    size_t msg_off;       // byte offset of this level's messages
    size_t cost_bytes, msg_bytes;
};

// Workspace plan of one problem.
struct Plan {
    int w, h, L, levels;
    int variant;          // half-sweep kernel variant (0 = default)
    Level lv[kMaxLevels];
    size_t pair_off;      // byte offset of the packed downsampled pair (cost from a pair)
    bool pairs;           // pixel-major levels run fused pairs of half-sweeps (bp_iter_pm2_impl.h)
    size_t y_off;         // second buffer of colour 0's incoming rows for the fused pairs
                          // (the finest pixel-major level's size; 0 when !pairs)
    bool zero_coarsest;   // the initialisation zeros the coarsest level's whole state
                          // (false when its first fused pair reads zeros in its place)
    size_t bytes;         // total workspace bytes of this problem (aligned)
};

// Pixel-major lane split for L labels: S lanes per message direction (4, 8 or
// 16, a DPP row or part of one), R consecutive labels per lane, lp = S * R.
void pm_split(int L, int *S, int *R);

// Fills `plan` for one problem with its workspace starting at byte `base`.
// Levels >= pm_from are pixel-major.  Returns false when a level does not fit
// the kernels' 32-bit byte offsets.
bool make_plan(int w, int h, int L, int levels, int msg_fmt, int pm_from, size_t base, Plan *plan);

// First pixel-major level the library picks when the caller does not.
int default_pm_from(int w, int h, int L, int levels, int msg_fmt);

bp_status launch_status();

// Fixed scratch of bp_run_noalloc (bp_noalloc.hip): its size, and its device
// address on device `dev` (which must be current), resolved at the first call
// per device; NULL if the runtime cannot resolve it.
constexpr size_t kNoallocScratchBytes = BP_NOALLOC_SCRATCH_BYTES;
void *noalloc_scratch(int dev);

// ---- kernel launchers (each enqueues on `s`, returns BP_OK or BP_ERR_HIP) ----

// a1 + a2: cost volume [L][h/ds][w/ds] from u8 images (optionally downsampled).
bp_status launch_cost_volume(const uint8_t *left, const uint8_t *right, int w, int h, int ch,
                             int64_t stride, int ds, int L, float trunc, int rgb_mode, float *cost,
                             hipStream_t s);
bp_status launch_downsample(const uint8_t *in, int w, int h, int ch, int64_t stride, int ds,
                            uint8_t *out, hipStream_t s);

// a3: level-0 cost in the level's layout, and the sum pyramid.
bp_status launch_split_cost(const float *planar, const Plan &p, uint8_t *ws, hipStream_t s);
// Finest-level cost from a pair: packs the downsampled pair at p.pair_off
// (in the same launch as launch_init_messages' work, which callers therefore
// skip on this route), then writes the data term in the level's layout, and
// level 1's pyramid sum too when both levels are pixel-major
// (*levels_done = 2, else 1).
bp_status launch_pair_cost(const bp_pair &pr, const Plan &p, uint8_t *ws, hipStream_t s, int *levels_done);
bp_status launch_pyramid_level(const Plan &p, int l, uint8_t *ws, hipStream_t s);
// Levels first .. levels - 1 of the pyramid (up to three pixel-major levels
// per launch).
bp_status launch_pyramid(const Plan &p, int first, uint8_t *ws, hipStream_t s);

// a4: zero every level's out-of-grid slots and the coarsest level's
// messages; explicit parent copy.
bp_status launch_init_messages(const Plan &p, uint8_t *ws, hipStream_t s);
bp_status launch_parent_copy(const Plan &p, int l, uint8_t *ws, hipStream_t s);

// a5: one checkerboard half-sweep at level l.  src_mode: 0 read own slots,
// 1 read the parent level's slots (fused parent copy).
// If disp != NULL the senders' argmin labels are written (finest level).
bp_status launch_iteration(const Plan &p, int l, int t, int src_mode, float lambda, float tau,
                           int32_t *disp, int variant, uint8_t *ws, hipStream_t s);
// Half-sweeps t, t + 1 (t even) of pixel-major level l as one fused launch.
// Phase 1 reads colour 0's incoming rows from the colour-0 block at byte
// `src_off` of the workspace (PAIR_SRC_OWN), from the parent level's final
// state (PAIR_SRC_PARENT, t = 0) or as zeros (PAIR_SRC_ZERO, the coarsest
// level at t = 0); phase 2 writes colour 0's incoming rows into the colour-0
// block at `dst_off` (never the block read).  write_c1 also stores colour 1's
// incoming rows into the level's state; disp receives phase 2's senders'
// labels (finest level).
enum { PAIR_SRC_OWN = 0, PAIR_SRC_PARENT = 1, PAIR_SRC_ZERO = 2 };
bp_status launch_iteration_pair(const Plan &p, int l, int src_kind, size_t src_off, size_t dst_off, bool write_c1,
                                float lambda, float tau, int32_t *disp, uint8_t *ws, hipStream_t s,
                                uint8_t *ck = nullptr, bool ck_c1 = false, float *soft = nullptr,
                                float inv_t = 0.0f);

// Half-sweep t of the finest level reading its incoming messages from `src`
// (a saved state in the level's layout) and writing the receivers' slots
// into the level's own message buffer.
bp_status launch_iteration_from(const Plan &p, int t, const uint8_t *src, float lambda, float tau, int variant,
                                uint8_t *ws, hipStream_t s);

// a6: readout of the pixels of `colour_mask` (bit c = colour c) at level 0.
bp_status launch_readout(const Plan &p, int colour_mask, int32_t *disp, float *soft, float temperature,
                         uint8_t *ws, hipStream_t s);
bp_status launch_export(const Plan &p, float *out, uint8_t *ws, hipStream_t s);

// Measurement aid: stream read_bytes from src and write_bytes to dst.
bp_status launch_stream(const void *src, size_t read_bytes, void *dst, size_t write_bytes, hipStream_t s);

// a7: joint bilateral upsampling.
bp_status launch_harris(const uint8_t *img, int w, int h, int64_t stride, int g, int64_t thr, int64_t *r25,
                        bp_corner *corners, hipStream_t s);
bp_status launch_zssd(const uint8_t *a, const uint8_t *b, int w, int h, int64_t stride, const bp_corner *corners,
                      int n, int pr, int sr, bp_match *out, hipStream_t s);
size_t icp_workspace_bytes(int n, int m);
bp_status launch_icp(const float *src, int n, const float *dst, int m, const double *pose_in, int iters, float dmax,
                     double *pose_out, double *rms, int32_t *pairs, int32_t *corr_out, uint8_t *ws, hipStream_t s);
bp_status launch_undistort(const uint8_t *in, int w, int h, int ch, int64_t in_stride, const bp_intrinsics &K,
                           uint8_t *out, int64_t out_stride, hipStream_t s);
bp_status launch_upsample(const int32_t *disp_lo, int wl, int hl, const uint8_t *guide, int wh, int hh, int ch,
                          int64_t stride, float sigma_s, float sigma_r, int radius, float *out, const bp_camera *cam,
                          float *xyz, hipStream_t s);

// Label-major half-sweep variants: count for a label count and the variant's
// lanes per pixel (1, 2 or 4); variant 0 = default.
int iteration_variants(int L);
int iteration_lanes(int L, int variant);

// Label-major half-sweep (bp_iter_lm.hip) and pixel-major half-sweep (bp_iter_pm.hip).
struct IterArgs {
    const float *cost;     // this level's cost
    uint32_t cost_bytes;
    uint8_t *msg;          // this level's messages
    uint32_t msg_bytes;
    const uint8_t *src;    // where incoming messages are read (own level or parent)
    uint32_t src_bytes;
    int32_t *disp;         // finest-level argmin output of the senders, or NULL
    int w, h, wh;
    uint32_t blk, ls, ps, lp;              // this level's element strides (see Level)
    uint32_t sblk, sls, sps;               // element strides of `src`
    int src_wh, src_w, src_h;
    int src_parent;        // 1 when `src` is the parent level
    int colour;            // sender colour
    int L;                 // label count
    int ncomp;             // h * wh
    float lambda, lt;      // lambda and lambda * tau
    int near;              // window of the transform's near form: 1 (tau <= 2), 2 (tau <= 3), 0 (scans)
};
bp_status dispatch_iter_lm(const IterArgs &a, int fmt, int G, bool ro, hipStream_t s);

// a8: adjoint kernels (bp_adjoint.hip).  `msg` is a finest-level message
// state (label-major float32), `mbar` its adjoint, `grad_cost` planar.
bp_status launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
bp_status launch_zero(void *dst, size_t bytes, hipStream_t s);
int bwd_step_blocks(const Plan &p);
bp_status launch_bwd_readout(const Plan &p, const uint8_t *msg, float *mbar, const float *grad_soft,
                             float *grad_cost, float temperature, uint8_t *ws, hipStream_t s);
// One problem's buffers for a reverse half-sweep.
struct BwdProblem {
    const Plan *plan;
    uint8_t *ws;            // workspace holding the plan's cost
    const uint8_t *state;   // message state M_t
    float *mbar;            // message adjoint
    float *grad_cost;       // planar [L][h][w]
    float *partial;         // bwd_step_blocks(plan) (lambda, tau) pairs
};
size_t bwd_table_bytes(int count);
// The reverse step keeps a pixel's message row in registers: up to 128 labels.
constexpr int kMaxBackwardLabels = 128;

// a8 on pixel-major states (bp_adjoint_pm.hip): the same steps with the
// forward kernel's lane split; the cost adjoint is accumulated pixel-major
// (`gcost`, laid out like the level's cost) and written planar at the end.
struct BwdPmProblem {
    const Plan *plan;
    uint8_t *ws;            // workspace holding the plan's cost
    const uint8_t *state;   // message state M_t
    float *mbar;            // message adjoint
    float *gcost;           // cost adjoint, pixel-major
    float *partial;         // bwd_pm_blocks(plan) (lambda, tau) pairs
};
int bwd_pm_blocks(const Plan &p);
size_t bwd_pm_table_bytes(int count);
bp_status launch_bwd_readout_pm(const Plan &p, const uint8_t *msg, float *mbar, float *gcost, const float *grad_soft,
                                float temperature, uint8_t *ws, hipStream_t s);
bp_status launch_bwd_step_pm_batch(const BwdPmProblem *probs, int count, int t, bool first_step, float lambda,
                                   float tau, uint8_t *table, hipStream_t s);
bp_status launch_gcost_to_planar(const Plan &p, const float *gcost, float *grad_cost, hipStream_t s);
// Reverse half-sweep t of every problem, one launch per label count; the
// launch entries are written into `table` (bwd_table_bytes(count) bytes).
bp_status launch_bwd_step_batch(const BwdProblem *probs, int count, int t, float lambda, float tau, uint8_t *table,
                                hipStream_t s);
size_t bwd_finish_bytes();
bp_status launch_bwd_finish(const float *partial, int n, float *grad_lambda, float *grad_tau, uint8_t *scratch,
                            hipStream_t s);
bp_status dispatch_iter_pm(const IterArgs &a, int fmt, int S, int R, bool ro, bool xchg, hipStream_t s);

// Two half-sweeps (t, t + 1, t even) of a pixel-major level in one launch
// (bp_iter_pm2_impl.h).  Phase 1 sends from colour 0, whose incoming rows are
// read from `src` (a colour-0 block [slot][plane][lp] of the level, or the
// parent level's whole state when src_parent, or all zero when src_zero);
// phase 2 sends from colour 1 into `dst`, a colour-0 block of the level.
struct PairArgs {
    const float *cost;     // this level's cost
    uint32_t cost_bytes;
    uint8_t *msg;          // this level's messages (colour 1's block written when write_c1)
    uint32_t msg_bytes;
    const uint8_t *src;
    uint32_t src_bytes;
    uint8_t *dst;
    uint32_t dst_bytes;
    int32_t *disp;         // argmin labels of phase 2's senders, or NULL
    float *soft;           // their soft-argmin disparity (temperature 1 / inv_t), or NULL
    float inv_t;
    int w, h, wh;
    uint32_t blk, lp;      // this level's strides (pixel-major: ls = 1, ps = lp)
    uint32_t sblk, sps;    // strides of `src`
    int src_wh;
    int src_parent, src_zero, write_c1;
    int L;
    float lambda, lt;
    int near;              // window of the transform's near form: 1 (tau <= 2), 2 (tau <= 3), 0 (scans)
    int cost_fmt;          // the level's cost storage (COST_*; selects the kernel)
    int tx, ty;            // tile (tx even)
    int tiles_x, ntiles, per_xcd;
    uint8_t *ck;           // checkpoint state in the level's layout that also receives phase 2's rows,
                           // or NULL
    int ck_c1;             // phase 1's rows also go to ck (the final state)
    uint32_t ck_bytes;
};
void pair_tile(int lp, int mb, int w, int h, int *tx, int *ty);
size_t pair_lds_bytes(int tx, int ty, int lp, int mb);
bp_status dispatch_iter_pm2(const PairArgs &a, int fmt, int S, int R, bool ro, hipStream_t s);
// Whether the fused pair supports a level's lane split.
bool pair_supported(int S, int R);
PairArgs make_pair_args(const Plan &p, int l, int src_kind, size_t src_off, size_t dst_off, bool write_c1,
                        float lambda, float tau, int32_t *disp, uint8_t *ws, uint8_t *ck = nullptr,
                        bool ck_c1 = false, float *soft = nullptr, float inv_t = 0.0f);
// Zero the out-of-grid slots of `n` message states of each of `count`
// problems: problem i's states are laid out like level 0 of plans[i], back to
// back from bases[i] (checkpoint states written by the fused pairs, which
// store in-grid rows only).
bp_status launch_zero_borders(const Plan *plans, uint8_t *const *bases, int count, int n, hipStream_t s);
// Batched fused pairs: one launch over the problems of a lane split; entries
// hold each problem's arguments and its first block (a multiple of 8).
struct PairEntry {
    PairArgs a;
    int block0;
    int pad[3];
};
constexpr int kPairChunk = 12;
struct PairChunk {
    PairEntry e[kPairChunk];
    int n;
};
int pair_blocks(const PairArgs &a);
bp_status launch_write_pair_entries(PairEntry *dst, const PairEntry *src, int n, hipStream_t s);
// exact: every entry's label count equals its lane split's S * R.
bp_status launch_iteration_pair_batch(const PairEntry *tab, int n, int blocks, size_t lds, int fmt, int S, int R,
                                      bool exact, bool ro, int cost_fmt, hipStream_t s);

// Pixel-major kernel variants (1 default split; 2 half the lanes per message,
// twice the labels per lane; 3 and 4 the same with each lane group reading
// only its own incoming row and exchanging sums by lane shuffles).
int pm_variants(int L);
// Variant used when the caller and the tuning table leave the choice open.
int default_variant(int L, int msg_fmt);
void pm_split_variant(int L, int variant, int *S, int *R, bool *xchg);

// Batched pixel-major half-sweep: one launch over several problems that share
// a lane split; table entries hold each problem's arguments and first block.
struct BatchEntry {
    IterArgs a;
    int block0;
    int pad[3];
};
constexpr int kChunk = 16;
struct EntryChunk {
    BatchEntry e[kChunk];
    int n;
};
int pm_blocks(int ncomp, int S);
int pm_sweep_blocks(int ncomp, int S, bool xchg);
bp_status launch_write_entries(BatchEntry *dst, const BatchEntry *src, int n, hipStream_t s);
IterArgs make_iter_args(const Plan &p, int l, int t, int src_mode, float lambda, float tau, int32_t *disp,
                        uint8_t *ws);
// One batched half-sweep over a table of `n` launch entries; `ro` also writes
// each entry's senders' labels (entries with disp == NULL skip that).
bp_status launch_iteration_batch(const BatchEntry *tab, int n, int blocks, int fmt, int S, int R, bool xchg, bool ro,
                                 hipStream_t s);

}  // namespace bpk
