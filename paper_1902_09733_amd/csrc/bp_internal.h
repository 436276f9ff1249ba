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

// One pyramid level of one problem.  Both the cost and the messages are stored
// colour-split: pixel (x, y) has colour (x + y) & 1 and compact index
// j = y * wh + (x >> 1) inside its colour's planes, wh = ceil(w / 2).  A plane
// holds `plane` >= h * wh elements (padded to 64); planes are ordered
//   cost: [colour][label][plane]          (float32)
//   msg:  [colour][slot][label][plane]    (slot k = received from side k:
//                                          0 left, 1 right, 2 up, 3 down)
struct Level {
    int w, h, wh;
    int64_t plane;        // elements per (colour, slot, label) plane
    int fmt;              // message storage format at this level
    size_t cost_off;      // byte offset of this level's cost in the workspace
    size_t msg_off;       // byte offset of this level's messages
    size_t cost_bytes, msg_bytes;
};

// Workspace plan of one problem.
struct Plan {
    int w, h, L, levels;
    Level lv[kMaxLevels];
    size_t bytes;         // total workspace bytes of this problem (aligned)
};

// Fills `plan` for one problem with its workspace starting at byte `base`.
// Returns false when the sizes do not fit the kernels' 32-bit offsets.
bool make_plan(int w, int h, int L, int levels, int msg_fmt, size_t base, Plan *plan);

// Status helpers.
bp_status launch_status();

// ---- kernel launchers (each enqueues on `s`, returns BP_OK or BP_ERR_HIP) ----

// a1 + a2: cost volume [L][h/ds][w/ds] from u8 images (optionally downsampled).
bp_status launch_cost_volume(const uint8_t *left, const uint8_t *right, int w, int h, int ch,
                             int64_t stride, int ds, int L, float trunc, int rgb_mode, float *cost,
                             hipStream_t s);
bp_status launch_downsample(const uint8_t *in, int w, int h, int ch, int64_t stride, int ds,
                            uint8_t *out, hipStream_t s);

// a3: colour-split copy of the finest cost, and the sum pyramid.
bp_status launch_split_cost(const float *planar, const Plan &p, uint8_t *ws, hipStream_t s);
bp_status launch_pyramid_level(const Plan &p, int l, uint8_t *ws, hipStream_t s);

// a4: out-of-grid message slots of a level set to zero; explicit parent copy.
bp_status launch_zero_border(const Plan &p, int l, uint8_t *ws, hipStream_t s);
bp_status launch_parent_copy(const Plan &p, int l, uint8_t *ws, hipStream_t s);
bp_status launch_zero_level(const Plan &p, int l, uint8_t *ws, hipStream_t s);

// a5: one checkerboard half-sweep at level l.  src_mode: 0 read own slots,
// 1 read the parent level's slots (fused parent copy), 2 start from zero.
// If disp != NULL the senders' argmin labels are written (finest level).
bp_status launch_iteration(const Plan &p, int l, int t, int src_mode, float lambda, float tau,
                           int32_t *disp, int variant, uint8_t *ws, hipStream_t s);

// a6: readout of the pixels of `colour_mask` (bit c = colour c) at level 0.
bp_status launch_readout(const Plan &p, int colour_mask, int32_t *disp, float *soft, float temperature,
                         uint8_t *ws, hipStream_t s);
bp_status launch_export(const Plan &p, float *out, uint8_t *ws, hipStream_t s);

// a7: joint bilateral upsampling.
bp_status launch_upsample(const int32_t *disp_lo, int wl, int hl, const uint8_t *guide, int wh, int hh,
                          int ch, int64_t stride, float sigma_s, float sigma_r, int radius, float *out,
                          hipStream_t s);

// Number of iteration-kernel variants for a label count and the variant's
// lanes per pixel (1, 2 or 4); variant 0 = default.
int iteration_variants(int L);
int iteration_lanes(int L, int variant);

}  // namespace bpk
