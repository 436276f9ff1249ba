// C ABI of libbpstereo (include/bp.h): host-side validation, workspace
// planning and the launch sequence of the hierarchical BP path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "bp.h"
#include "bp_internal.h"

using namespace bpk;

namespace {

bool valid_image_args(const void *a, const void *b, int32_t w, int32_t h, int32_t ch, int64_t stride, int32_t ds)
{
    if (!a || !b || w <= 0 || h <= 0 || (ch != 1 && ch != 3) || ds <= 0) return false;
    if (stride < (int64_t)w * ch) return false;
    if (w % ds || h % ds) return false;
    return true;
}

bool valid_params(const bp_params *p)
{
    if (!p) return false;
    if (p->levels < 1 || p->levels > kMaxLevels || p->iters_per_level < 0) return false;
    if (!(p->lambda >= 0.0f) || !std::isfinite(p->lambda)) return false;
    if (!(p->tau > 0.0f) || !std::isfinite(p->tau)) return false;
    if (p->msg_dtype < BP_MSG_F32 || p->msg_dtype > BP_MSG_BF16) return false;
    if (p->checkpoint_every < 0) return false;
    if (p->pm_from < -1 || p->pm_from > p->levels) return false;
    return true;
}

bool valid_pair(const bp_pair *pr, int w, int h)
{
    if (!pr || !pr->left || !pr->right || (pr->channels != 1 && pr->channels != 3) || pr->downsample < 1) return false;
    if ((int64_t)w * pr->downsample > INT32_MAX || (int64_t)h * pr->downsample > INT32_MAX) return false;
    if (pr->row_stride_bytes < (int64_t)w * pr->downsample * pr->channels) return false;
    if (!(pr->data_trunc >= 0.0f) || !std::isfinite(pr->data_trunc)) return false;
    return pr->rgb_mode == 0 || pr->rgb_mode == 1;
}

bool valid_problem(const bp_problem &q, const bp_params &p)
{
    if (q.width <= 0 || q.height <= 0) return false;
    if (!q.cost && !valid_pair(q.pair, q.width, q.height)) return false;
    if (q.soft_disparity && !(p.temperature > 0.0f)) return false;
    // Every level keeps at least one pixel.
    return true;
}

bool supported_labels(int L) { return L >= 2 && L <= kMaxLabels; }

// Launch-shape table written by the autotuner (paper_1902_09733_amd/tune.py):
// text lines "width height labels fmt levels pm_from variant us", read once
// from the file named by BP_TUNE_TABLE.
struct TuneEntry {
    int w, h, L, fmt, levels, pm_from, variant;
};

std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
bool g_tune_init = false;

// Parses a table file; false if it cannot be opened.
bool read_tune_file(const char *path, std::vector<TuneEntry> *out)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        TuneEntry e;
        double us;
        if (std::sscanf(line, "%d %d %d %d %d %d %d %lf", &e.w, &e.h, &e.L, &e.fmt, &e.levels, &e.pm_from,
                        &e.variant, &us) == 8)
            out->push_back(e);
    }
    std::fclose(f);
    return true;
}

// Tuned (pm_from, variant) for a problem, if the table has an entry with the
// same label count, format and level count; the nearest pixel count wins.
bool tuned_choice(int w, int h, int L, int fmt, int levels, int *pm_from, int *variant)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (!g_tune_init) {
        g_tune_init = true;
        const char *path = std::getenv("BP_TUNE_TABLE");
        if (path && *path) read_tune_file(path, &g_tune);
    }
    const TuneEntry *best = nullptr;
    double bd = 0.0;
    for (const TuneEntry &e : g_tune) {
        if (e.L != L || e.fmt != fmt || e.levels != levels) continue;
        const double d = std::fabs(std::log((double)e.w * e.h) - std::log((double)w * h));
        if (!best || d < bd) {
            best = &e;
            bd = d;
        }
    }
    if (!best) return false;
    *pm_from = best->pm_from < 0 ? 0 : (best->pm_from > levels ? levels : best->pm_from);
    *variant = best->variant;
    return true;
}

// The adjoint works on label-major states when the caller asks for them
// (pm_from = levels), otherwise on pixel-major ones.
static bool adjoint_label_major(const bp_params &p) { return p.pm_from == p.levels; }

// Whether level l of a plan runs its half-sweeps as fused pairs.
bool level_pairs(const Plan &pl, int l, int K)
{
    int S, R;
    pm_split(pl.L, &S, &R);
    return pl.pairs && pl.lv[l].layout == PIXEL_MAJOR && K >= 2 && pair_supported(S, R);
}

// Whether a pair's finest-level cost is stored as FP16: its values are the
// integers 0..255 (grey, or the rounded channel mean) and the truncation, all
// exact in FP16 when the truncation is, and the level is written by the fused
// level-0/1 cost kernel (two pixel-major finest levels), whose level 1 and the
// pyramid above it stay FP32.  Every kernel that reads a pixel-major level's
// cost reads either format.
static bool fp16_exact(float t)
{
    if (!(t >= 0.0f) || t > 65504.0f) return false;
    if (t == 0.0f) return true;
    int e;
    std::frexp(t, &e);                       // t = m 2^e, m in [0.5, 1)
    const int lsb = std::max(e - 11, -24);   // 11 significant bits; subnormal step 2^-24
    return std::ldexp(std::nearbyint(std::ldexp(t, -lsb)), lsb) == t;
}

static int pair_cost_fmt(const bp_pair &pr, const Plan &pl, int K)
{
    if (!((pr.channels == 1 || pr.rgb_mode == 0) && fp16_exact(pr.data_trunc) && pl.levels >= 2 &&
          pl.lv[0].layout == PIXEL_MAJOR && pl.lv[1].layout == PIXEL_MAJOR))
        return COST_F32;
    // Only the fused pairs and the readout read it: the finest level runs
    // pairs alone (K even, and no single half-sweeps ahead of the first pair
    // after a materialised parent copy).
    if (!level_pairs(pl, 0, K) || (K & 1)) return COST_F32;
    const Level &c = pl.lv[0], &pa = pl.lv[1];
    const bool fusable = K >= 2 && c.fmt == pa.fmt;
    if (!fusable && ((K / 2) & 1) != 0) return COST_F32;
    // Bytes when the truncation is an integer of at most 255 (then every cost
    // is one) and a lane's labels fill whole words.
    int S, R;
    pm_split(pl.L, &S, &R);
    const float t = pr.data_trunc;
    if (t <= 255.0f && t == std::floor(t) && R % 4 == 0) return COST_U8;
    return COST_F16;
}

// Problem plans laid out back to back in the workspace.  With allow_pairs,
// problems that leave the kernel choice to the library run pixel-major levels
// as fused pairs of half-sweeps, which need a second buffer of colour 0's
// incoming rows (the size of the finest such level's block).
bool plan_all(const bp_problem *probs, int32_t count, const bp_params *p, Plan *plans, size_t *total,
              bool allow_pairs = false, bool tuned_layout_only = false)
{
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        const bp_problem &q = probs[i];
        int pm_from = p->pm_from, tv = 0;
        if (pm_from < 0 && !(p->variant == 0 && tuned_choice(q.width, q.height, q.num_labels, p->msg_dtype,
                                                             p->levels, &pm_from, &tv)))
            pm_from = default_pm_from(q.width, q.height, q.num_labels, p->levels, p->msg_dtype);
        if (tuned_layout_only) tv = 0;
        // A forward call that saves states for the adjoint stores them
        // pixel-major (or label-major when asked with pm_from = levels), the
        // layouts the two adjoints read.
        if (p->checkpoint_every > 0) pm_from = adjoint_label_major(*p) ? p->levels : 0;
        if (!make_plan(q.width, q.height, q.num_labels, p->levels, p->msg_dtype, pm_from, off, &plans[i])) return false;
        if (!q.cost) {
            plans[i].pair_off = off + plans[i].bytes;
            plans[i].bytes += align_up((size_t)2 * q.width * q.height * sizeof(uint32_t));
        }
        plans[i].variant = p->variant != 0 ? p->variant : tv != 0 ? tv : default_variant(q.num_labels, p->msg_dtype);
        // The pixel-major adjoint repeats the sums of the plain-load split.
        if (p->checkpoint_every > 0 && pm_from == 0) plans[i].variant = 1;
        // With checkpoints every `every` half-sweeps the saved halves are
        // colour 0's (after an odd half-sweep, i.e. after a pair) only when
        // `every` is even.
        plans[i].pairs = allow_pairs && p->variant == 0 && tv == 0 && p->checkpoint_every % 2 == 0;
        plans[i].y_off = 0;
        if (plans[i].pairs) {
            size_t yb = 0;
            for (int l = 0; l < plans[i].levels; ++l)
                if (level_pairs(plans[i], l, p->iters_per_level)) {
                    const Level &v = plans[i].lv[l];
                    const size_t b = align_up((size_t)4 * v.blk * fmt_bytes(v.fmt));
                    if (b > yb) yb = b;
                }
            plans[i].pairs = yb > 0;
            plans[i].y_off = off + plans[i].bytes;
            plans[i].bytes += yb;
        }
        // The coarsest level's first half-sweeps run as a fused pair that
        // reads zero messages in place of the state, so only the out-of-grid
        // slots need zeroing there.
        plans[i].zero_coarsest = !level_pairs(plans[i], plans[i].levels - 1, p->iters_per_level);
        plans[i].lv[0].cost_fmt = q.cost ? COST_F32 : pair_cost_fmt(*q.pair, plans[i], p->iters_per_level);
        off += plans[i].bytes;
    }
    *total = align_up(off);
    return true;
}

// Message states a forward call saves for the adjoint: after every
// `every`-th half-sweep t < K, and the final state.
int checkpoint_states(int K, int every) { return (K > 0 ? (K - 1) / every : 0) + 1; }

size_t checkpoint_bytes_of(const Plan &pl, int K, int every)
{
    return (size_t)checkpoint_states(K, every) * pl.lv[0].msg_bytes;
}

bool differentiable(const bp_params &p) { return p.levels == 1 && p.msg_dtype == BP_MSG_F32; }

// Optional timing of the half-sweep kernels (bp_run_profiled): an event pair
// around every launch, or around the K launches of every level.
struct Recorder {
    bp_launch_record *rec;
    hipEvent_t (*ev)[2];
    int cap, n;
    bool per_level;
};

// Algorithmic memory traffic of one half-sweep and of one fused pair at
// level l (bp_launch_record.bytes).
double sweep_bytes(const Plan &pl, int l)
{
    const double nl = (double)pl.lv[l].w * pl.lv[l].h * pl.L;
    return nl * (4.0 + 8.0 * fmt_bytes(pl.lv[l].fmt)) / 2.0;
}

double pair_bytes(const Plan &pl, int l, bool ends)
{
    const double nl = (double)pl.lv[l].w * pl.lv[l].h * pl.L, mb = fmt_bytes(pl.lv[l].fmt);
    const int cf = pl.lv[l].cost_fmt;
    const double cb = cf == COST_U8 ? 1.0 : cf == COST_F16 ? 2.0 : 4.0;   // both colours' costs
    return nl * (cb + 4.0 * mb + (ends ? 2.0 * mb : 0.0));
}

// Runs the whole hierarchical BP of one problem.
bp_status run_one(const bp_problem &q, const Plan &pl, const bp_params &p, uint8_t *ws, hipStream_t s,
                  Recorder *prof = nullptr, uint8_t *ckpt = nullptr)
{
    bp_status st;
    const int n = pl.levels, K = p.iters_per_level;
    // Out-of-grid slots of every level and the coarsest level's messages start
    // at zero (on the pair route, inside the pair packing's launch).
    if (q.cost && (st = launch_init_messages(pl, ws, s)) != BP_OK) return st;
    int done = 1;
    if ((st = q.cost ? launch_split_cost(q.cost, pl, ws, s) : launch_pair_cost(*q.pair, pl, ws, s, &done)) != BP_OK)
        return st;
    if ((st = launch_pyramid(pl, done, ws, s)) != BP_OK) return st;
    // The finest level's last half-sweep also reads out its senders' labels,
    // and their soft-argmin when it runs in a fused pair.
    const bool last_pair = level_pairs(pl, 0, K) && (K & 1) == 0;
    const bool fuse_ro = K >= 1 && (q.soft_disparity ? last_pair : q.disparity != nullptr);
    const float inv_t = q.soft_disparity ? 1.0f / p.temperature : 0.0f;
    for (int l = n - 1; l >= 0; --l) {
        int first_src = 0;
        if (l < n - 1) {
            // Half-sweep 0 reads the parent's slots directly when every slot of
            // this level is rewritten before it is read again (K >= 2) and the
            // storage formats agree; otherwise the copy is materialised.
            const Level &c = pl.lv[l], &pa = pl.lv[l + 1];
            const bool fusable = K >= 2 && c.fmt == pa.fmt && !(c.layout == PIXEL_MAJOR && pa.layout == LABEL_MAJOR);
            if (fusable) first_src = 1;
            else if ((st = launch_parent_copy(pl, l, ws, s)) != BP_OK) return st;
        }
        const bool lrec = prof && prof->per_level && prof->n < prof->cap && K > 0;
        if (lrec && hipEventRecord(prof->ev[prof->n][0], s) != hipSuccess) return BP_ERR_HIP;
        int launches = 0;
        double lbytes = 0.0;   // algorithmic bytes of the level's launches
        int t0 = 0;   // first half-sweep left to the one-half-sweep kernels
        // Single half-sweeps of a level that runs fused pairs sum h in slot
        // order like the pairs do (variant 1).
        const bool lpairs = level_pairs(pl, l, K);
        const int variant = lpairs ? 1 : pl.variant;
        if (lpairs) {
            // Fused pairs over half-sweeps [t0, K - (K & 1)).  Phase 1 of the
            // first pair reads the parent's state, zeros (coarsest level) or the
            // level's own state after a materialised parent copy; pairs
            // alternate between the level's colour-0 block and the second
            // buffer so that the last one writes the level's own block.  When
            // the first pair would have to read and write the own block, two
            // single half-sweeps go first.
            const size_t own = pl.lv[l].msg_off, other = pl.y_off;
            int np = K / 2;
            const bool own_src = l < n - 1 && !first_src;
            if (own_src && (np & 1)) {
                for (; t0 < 2; ++t0, ++launches) {
                    if ((st = launch_iteration(pl, l, t0, 0, p.lambda, p.tau, nullptr, variant, ws, s)) != BP_OK)
                        return st;
                    lbytes += sweep_bytes(pl, l);
                }
                --np;
            }
            size_t src_off = own;
            // Checkpoints (finest level only): out-of-grid slots of every saved
            // state are zeroed once, the pairs write the in-grid rows.
            const size_t ck_state = pl.lv[0].msg_bytes;
            const int ck_n = ckpt ? checkpoint_states(K, p.checkpoint_every) : 0;
            if (ckpt && (st = launch_zero_borders(&pl, &ckpt, 1, ck_n, s)) != BP_OK) return st;
            for (int pi = 0; pi < np; ++pi, t0 += 2, ++launches) {
                const size_t dst_off = ((np - 1 - pi) & 1) ? other : own;
                int kind = PAIR_SRC_OWN;
                if (t0 == 0) kind = l == n - 1 ? PAIR_SRC_ZERO : (first_src ? PAIR_SRC_PARENT : PAIR_SRC_OWN);
                const bool ends = pi == np - 1 && (K & 1) == 0;
                const bool rd = l == 0 && ends && fuse_ro;
                // Colour 1's final rows are stored for the next level's parent
                // copy, the readout and the export; at the finest level with the
                // readout fused here and no export, nothing reads them (the
                // final checkpoint receives them on its own).
                const bool store_c1 = ends && (l > 0 || !rd || q.messages_out);
                // State after the pair: saved (its colour-0 half) every
                // `every` half-sweeps, and whole at the end.
                uint8_t *ck = nullptr;
                if (ckpt) {
                    const int tn = t0 + 2;
                    if (ends) ck = ckpt + (size_t)(ck_n - 1) * ck_state;
                    else if (tn % p.checkpoint_every == 0 && tn < K)
                        ck = ckpt + (size_t)(tn / p.checkpoint_every - 1) * ck_state;
                }
                const bool rec = prof && !prof->per_level && prof->n < prof->cap;
                if (rec && hipEventRecord(prof->ev[prof->n][0], s) != hipSuccess) return BP_ERR_HIP;
                if ((st = launch_iteration_pair(pl, l, kind, src_off, dst_off, store_c1, p.lambda, p.tau,
                                                rd ? q.disparity : nullptr, ws, s, ck, ends,
                                                rd ? q.soft_disparity : nullptr, inv_t)) != BP_OK)
                    return st;
                if (rec) {
                    if (hipEventRecord(prof->ev[prof->n][1], s) != hipSuccess) return BP_ERR_HIP;
                    bp_launch_record &r = prof->rec[prof->n++];
                    r.level = l;
                    r.half_sweep = t0;
                    r.launches = 1;
                    r.readout_fused = rd;
                    r.msg_bytes = fmt_bytes(pl.lv[l].fmt);
                    r.units = 2.0 * pl.lv[l].w * pl.lv[l].h * pl.L;
                    r.ms = 0.0f;
                    r.bytes = pair_bytes(pl, l, store_c1);
                }
                lbytes += pair_bytes(pl, l, store_c1);
                src_off = dst_off;
            }
        }
        for (int t = t0; t < K; ++t) {
            ++launches;
            int32_t *ro = (l == 0 && t == K - 1 && fuse_ro) ? q.disparity : nullptr;
            const bool rec = prof && !prof->per_level && prof->n < prof->cap;
            if (rec && hipEventRecord(prof->ev[prof->n][0], s) != hipSuccess) return BP_ERR_HIP;
            if ((st = launch_iteration(pl, l, t, t == 0 ? first_src : 0, p.lambda, p.tau, ro, variant, ws, s)) != BP_OK)
                return st;
            if (rec) {
                if (hipEventRecord(prof->ev[prof->n][1], s) != hipSuccess) return BP_ERR_HIP;
                bp_launch_record &r = prof->rec[prof->n++];
                r.level = l;
                r.half_sweep = t;
                r.launches = 1;
                r.readout_fused = ro != nullptr;
                r.msg_bytes = fmt_bytes(pl.lv[l].fmt);
                r.units = (double)pl.lv[l].w * pl.lv[l].h * pl.L;
                r.ms = 0.0f;
                r.bytes = sweep_bytes(pl, l);
            }
            lbytes += sweep_bytes(pl, l);
            if (ckpt && (t + 1) % p.checkpoint_every == 0 && t + 1 < K) {
                // The adjoint reads a saved state M_{t+1} only through half-sweep
                // t + 1's senders (the reverse step at t + 1, or the replay from
                // it), i.e. the four slots of colour (t + 1) & 1, which are one
                // contiguous half of the state (out-of-grid slots included).
                const Level &v0 = pl.lv[0];
                const size_t sb = v0.msg_bytes, half = (size_t)4 * v0.blk * fmt_bytes(v0.fmt);
                const size_t at = (size_t)((t + 1) & 1) * half;
                if ((st = launch_copy(ws + v0.msg_off + at, ckpt + (size_t)((t + 1) / p.checkpoint_every - 1) * sb + at,
                                      half, s)) != BP_OK)
                    return st;
            }
        }
        if (lrec) {
            if (hipEventRecord(prof->ev[prof->n][1], s) != hipSuccess) return BP_ERR_HIP;
            bp_launch_record &r = prof->rec[prof->n++];
            r.level = l;
            r.half_sweep = 0;
            r.launches = launches;
            r.readout_fused = (l == 0 && fuse_ro) ? 1 : 0;
            r.msg_bytes = fmt_bytes(pl.lv[l].fmt);
            r.units = (double)K * pl.lv[l].w * pl.lv[l].h * pl.L;
            r.ms = 0.0f;
            r.bytes = lbytes;
        }
    }
    // The final state, unless the last pair has written it.
    if (ckpt && !(level_pairs(pl, 0, K) && (K & 1) == 0)) {
        const size_t sb = pl.lv[0].msg_bytes;
        if ((st = launch_copy(ws + pl.lv[0].msg_off, ckpt + (size_t)(checkpoint_states(K, p.checkpoint_every) - 1) * sb,
                              sb, s)) != BP_OK)
            return st;
    }
    if (q.disparity || q.soft_disparity) {
        // After the fused readout only the last receivers' labels remain.
        const int mask = fuse_ro ? (1 << (K & 1)) : 3;
        if ((st = launch_readout(pl, mask, q.disparity, q.soft_disparity, p.temperature, ws, s)) != BP_OK) return st;
    }
    if (q.messages_out)
        if ((st = launch_export(pl, q.messages_out, ws, s)) != BP_OK) return st;
    return BP_OK;
}

// The batched form: problems whose levels are all pixel-major run each
// (level, half-sweep) as one launch per lane split, over all of them (with
// checkpoints only as fused pairs, see plan_run).
bool batched(const Plan *plans, int32_t count, const bp_params &p)
{
    (void)p;
    if (count < 2) return false;
    for (int i = 0; i < count; ++i)
        for (int l = 0; l < plans[i].levels; ++l)
            if (plans[i].lv[l].layout != PIXEL_MAJOR) return false;
    return true;
}

// The batched form runs fused pairs at every level when the library picks
// the kernels, K is even (no single half-sweeps anywhere) and every level
// whose parent copy cannot be fused into its first pair (16-bit levels under
// the FP32 coarsest level) has an even number of pairs, so that the first
// pair reads the level's own state and writes the second buffer.
bool batch_pairs(const Plan *plans, int32_t count, const bp_params &p)
{
    const int K = p.iters_per_level;
    if (p.variant != 0 || K < 2 || (K & 1)) return false;
    for (int i = 0; i < count; ++i) {
        if (!plans[i].pairs) return false;
        for (int l = 0; l < plans[i].levels; ++l) {
            if (!level_pairs(plans[i], l, K)) return false;
            if (l < plans[i].levels - 1 && plans[i].lv[l].fmt != plans[i].lv[l + 1].fmt && ((K / 2) & 1)) return false;
        }
    }
    return true;
}

// Launch entries of the batched form.  One-half-sweep launches: (level, kind)
// x problems for the kinds {t = 0, odd t, even t > 0}, plus the finest level's
// last half-sweep with its fused readout.  Fused pairs: (level, pair) x
// problems.
size_t batch_table_bytes(int32_t count, int levels, int K, bool pairs)
{
    if (pairs) return align_up((size_t)levels * (K / 2) * count * sizeof(PairEntry));
    return align_up(((size_t)levels * 3 + 1) * count * sizeof(BatchEntry));
}

// Plans of a bp_run call: the batched form when it applies (with fused pairs
// when batch_pairs allows them), otherwise each problem on its own with fused
// pairs of half-sweeps where they apply.  *table: bytes of the batched form's
// launch table (0 when not batched).
bool plan_run(const bp_problem *probs, int32_t count, const bp_params *p, Plan *plans, size_t *total, bool *batch,
              size_t *table = nullptr)
{
    if (table) *table = 0;
    if (!plan_all(probs, count, p, plans, total)) return false;
    *batch = batched(plans, count, *p);
    if (!plan_all(probs, count, p, plans, total, true)) return false;
    if (*batch) {
        bool pairs = batch_pairs(plans, count, *p);
        if (!pairs && p->variant == 0) {
            // A tuned one-half-sweep variant of a single problem would take
            // the whole batch off the fused pairs: inside a batch the table
            // chooses the layouts only.
            if (!plan_all(probs, count, p, plans, total, true, true)) return false;
            pairs = batch_pairs(plans, count, *p);
            if (!pairs && !plan_all(probs, count, p, plans, total, true)) return false;
        }
        // Checkpoints are saved by the fused pairs only; without them each
        // problem runs on its own.
        if (!pairs && p->checkpoint_every > 0) {
            *batch = false;
            return true;
        }
        if (!pairs && !plan_all(probs, count, p, plans, total)) return false;
        if (table) *table = batch_table_bytes(count, p->levels, p->iters_per_level, pairs);
        // A batched launch covers several problems with one kernel, so their
        // finest levels share the cost storage: the narrowest every problem's
        // costs allow (bytes are exact in FP16 too), and FP32 for the
        // one-half-sweep kernels.
        int cf = pairs ? COST_U8 : COST_F32;
        for (int i = 0; i < count; ++i) cf = std::min(cf, plans[i].lv[0].cost_fmt);
        for (int i = 0; i < count; ++i) plans[i].lv[0].cost_fmt = cf;
    }
    return true;
}

// Readout of the colours the last half-sweep did not cover, and the message
// export, problem by problem (those with in_group[i] == g when in_group is
// given).
bp_status finish_batched(const bp_problem *probs, int32_t count, const Plan *plans, const bp_params &p,
                         const bool *fuse, uint8_t *ws, hipStream_t s, const int *in_group = nullptr, int g = 0)
{
    bp_status st = BP_OK;
    const int K = p.iters_per_level;
    for (int i = 0; i < count && st == BP_OK; ++i) {
        if (in_group && in_group[i] != g) continue;
        const bp_problem &q = probs[i];
        if (q.disparity || q.soft_disparity) {
            const int mask = fuse[i] ? (1 << (K & 1)) : 3;
            st = launch_readout(plans[i], mask, q.disparity, q.soft_disparity, p.temperature, ws, s);
        }
        if (st == BP_OK && q.messages_out) st = launch_export(plans[i], q.messages_out, ws, s);
    }
    return st;
}

// Working-set budget of one cache group of the batched fused pairs: well
// inside the 256 MB Infinity Cache that sits between the L2s and HBM, leaving
// room for the streams that pass through it (saved states, the other
// buffers).  Eight 320x240x64 problems (138 MB each at the finest level) run
// 25 us per pair each one after the other, against 29 us each batched
// together, where each pair's state has left the cache before the next pair.
constexpr size_t kPairGroupBytes = (size_t)192 << 20;

// The batched form with fused pairs (batch_pairs): per level, pair and lane
// split one launch over the problems of that split in one cache group
// (kPairGroupBytes), each group's readout and export right after its last
// pair.  Buffers alternate as in run_one, so every level's last pair writes
// the level's own state.  With
// checkpoints (ckpt non-null; problems' saved states back to back) the pairs
// save them as in run_one.
bp_status run_batched_pairs(const bp_problem *probs, int32_t count, const Plan *plans, const bp_params &p,
                            uint8_t *ws, size_t table_off, const bool *fuse, uint8_t *ckpt, hipStream_t s)
{
    const int n = p.levels, K = p.iters_per_level, np = K / 2;
    const int ck_n = ckpt ? checkpoint_states(K, p.checkpoint_every) : 0;
    uint8_t **ck_of = new uint8_t *[count];
    {
        size_t off = 0;
        for (int i = 0; i < count; ++i) {
            ck_of[i] = ckpt ? ckpt + off : nullptr;
            if (ckpt) off += checkpoint_bytes_of(plans[i], K, p.checkpoint_every);
        }
    }
    int cls_S[32], cls_R[32], ncls = 0;
    int *cls_of = new int[count];
    for (int i = 0; i < count; ++i) {
        int S, R;
        pm_split(plans[i].L, &S, &R);
        int c = 0;
        while (c < ncls && !(cls_S[c] == S && cls_R[c] == R)) ++c;
        if (c == ncls) {
            cls_S[c] = S;
            cls_R[c] = R;
            ++ncls;
        }
        cls_of[i] = c;
    }
    // Cache groups: per level, consecutive problems whose working sets at
    // that level (cost, messages, second buffer) add up to at most
    // kPairGroupBytes run all their pairs before the next group starts, so
    // that a group's state stays in the Infinity Cache between its pairs.
    // A problem larger than that is a group of its own: part of its state
    // still survives from one pair to the next (measured on 48 problems of
    // 60 MB to 2 GB: letting all those above the budget share launches was
    // 1-3% slower than one after the other).
    int *grp = new int[(size_t)n * count], ng = 1;
    for (int l = 0; l < n; ++l) {
        int g = 0;
        size_t acc = 0;
        for (int i = 0; i < count; ++i) {
            const Level &v = plans[i].lv[l];
            const size_t wsz = v.cost_bytes + v.msg_bytes + (size_t)4 * v.blk * fmt_bytes(v.fmt);
            if (acc > 0 && acc + wsz > kPairGroupBytes) {
                ++g;
                acc = 0;
            }
            acc += wsz;
            grp[(size_t)l * count + i] = g;
        }
        if (g + 1 > ng) ng = g + 1;
    }
    const size_t nslot = (size_t)n * ng * np * ncls;
    PairEntry *host = new PairEntry[(size_t)n * np * count];
    PairEntry *dev = (PairEntry *)(ws + table_off);
    int *start = new int[nslot], *num = new int[nslot], *blocks = new int[nslot];
    size_t *lds = new size_t[nslot];
    bool *ro = new bool[nslot], *exact = new bool[nslot];
    int e = 0;
    auto slot_of = [&](int l, int g, int q, int c) { return (((size_t)l * ng + g) * np + q) * ncls + c; };
    for (int l = 0; l < n; ++l)
        for (int g = 0; g < ng; ++g)
            for (int q = 0; q < np; ++q)
                for (int c = 0; c < ncls; ++c) {
                    const size_t slot = slot_of(l, g, q, c);
                    start[slot] = e;
                    num[slot] = 0;
                    lds[slot] = 0;
                    ro[slot] = false;
                    exact[slot] = true;
                    int b0 = 0;
                    for (int i = 0; i < count; ++i) {
                        if (cls_of[i] != c || grp[(size_t)l * count + i] != g) continue;
                        const Plan &pl = plans[i];
                        const bool fusable = l == n - 1 || pl.lv[l].fmt == pl.lv[l + 1].fmt;
                        const size_t own = pl.lv[l].msg_off, other = pl.y_off;
                        const size_t dst = ((np - 1 - q) & 1) ? other : own;
                        const size_t src = q == 0 ? own : (((np - q) & 1) ? other : own);
                        const int kind = q > 0 ? PAIR_SRC_OWN
                                               : (l == n - 1 ? PAIR_SRC_ZERO
                                                             : (fusable ? PAIR_SRC_PARENT : PAIR_SRC_OWN));
                        const bool ends = q == np - 1;
                        const bool rd = l == 0 && ends && fuse[i];
                        // State after the pair (finest level): saved every
                        // `every` half-sweeps and at the end.
                        uint8_t *ck = nullptr;
                        if (ck_of[i] && l == 0) {
                            const size_t ck_state = pl.lv[0].msg_bytes;
                            const int tn = 2 * q + 2;
                            if (ends) ck = ck_of[i] + (size_t)(ck_n - 1) * ck_state;
                            else if (tn % p.checkpoint_every == 0 && tn < K)
                                ck = ck_of[i] + (size_t)(tn / p.checkpoint_every - 1) * ck_state;
                        }
                        // Colour 1's final rows: not needed at the finest
                        // level when its readout is fused here and nothing is
                        // exported (the final checkpoint receives them on
                        // its own).
                        const bool store_c1 = ends && (l > 0 || !rd || probs[i].messages_out);
                        PairEntry &pe = host[e++];
                        pe.a = make_pair_args(pl, l, kind, src, dst, store_c1, p.lambda, p.tau,
                                              rd ? probs[i].disparity : nullptr, ws, ck, ends,
                                              rd ? probs[i].soft_disparity : nullptr,
                                              probs[i].soft_disparity ? 1.0f / p.temperature : 0.0f);
                        pe.block0 = b0;
                        b0 += pair_blocks(pe.a);
                        const size_t lb = pair_lds_bytes(pe.a.tx, pe.a.ty, (int)pe.a.lp, fmt_bytes(pl.lv[l].fmt));
                        if (lb > lds[slot]) lds[slot] = lb;
                        if (rd) ro[slot] = true;
                        if (pl.L != cls_S[c] * cls_R[c]) exact[slot] = false;
                        ++num[slot];
                    }
                    blocks[slot] = b0;
                }
    // The device table holds the entries of launches over several problems
    // (runs of consecutive such slots written together); a lone problem's
    // launch takes its arguments directly.
    bp_status st = BP_OK;
    for (size_t slot = 0; slot < nslot && st == BP_OK;) {
        if (num[slot] < 2) {
            ++slot;
            continue;
        }
        const int first = start[slot];
        int n_run = 0;
        for (; slot < nslot && (num[slot] > 1 || num[slot] == 0); ++slot) n_run += num[slot];
        st = launch_write_pair_entries(dev + first, host + first, n_run, s);
    }
    // Out-of-grid slots of every saved state are zeroed once; the pairs write
    // the in-grid rows.
    if (st == BP_OK && ckpt) st = launch_zero_borders(plans, ck_of, count, ck_n, s);
    for (int l = n - 1; l >= 0 && st == BP_OK; --l) {
        const int fmt = plans[0].lv[l].fmt;   // every problem has the same levels
        for (int g = 0; g < ng && st == BP_OK; ++g) {
            if (l < n - 1)
                for (int i = 0; i < count && st == BP_OK; ++i)
                    if (grp[(size_t)l * count + i] == g && plans[i].lv[l].fmt != plans[i].lv[l + 1].fmt)
                        st = launch_parent_copy(plans[i], l, ws, s);
            for (int q = 0; q < np && st == BP_OK; ++q)
                for (int c = 0; c < ncls && st == BP_OK; ++c) {
                    const size_t slot = slot_of(l, g, q, c);
                    if (num[slot] == 0) continue;
                    // A lone problem takes the one-problem kernel (labels
                    // without padding skip the padded-label masks).
                    if (num[slot] == 1)
                        st = dispatch_iter_pm2(host[start[slot]].a, fmt, cls_S[c], cls_R[c], ro[slot], s);
                    else
                        st = launch_iteration_pair_batch(dev + start[slot], num[slot], blocks[slot], lds[slot], fmt,
                                                         cls_S[c], cls_R[c], exact[slot], ro[slot],
                                                         host[start[slot]].a.cost_fmt, s);
                }
            // The group's readout and export while its state is in the cache.
            if (l == 0 && st == BP_OK) st = finish_batched(probs, count, plans, p, fuse, ws, s, grp, g);
        }
    }
    delete[] host;
    delete[] start;
    delete[] num;
    delete[] blocks;
    delete[] lds;
    delete[] ro;
    delete[] exact;
    delete[] cls_of;
    delete[] ck_of;
    delete[] grp;
    return st;
}

bp_status run_batched(const bp_problem *probs, int32_t count, const Plan *plans, const bp_params &p, uint8_t *ws,
                      size_t table_off, uint8_t *ckpt, hipStream_t s)
{
    bp_status st;
    const int n = p.levels, K = p.iters_per_level;
    for (int i = 0; i < count; ++i) {
        if (probs[i].cost && (st = launch_init_messages(plans[i], ws, s)) != BP_OK) return st;
        int done = 1;
        if ((st = probs[i].cost ? launch_split_cost(probs[i].cost, plans[i], ws, s)
                                : launch_pair_cost(*probs[i].pair, plans[i], ws, s, &done)) != BP_OK)
            return st;
        if ((st = launch_pyramid(plans[i], done, ws, s)) != BP_OK) return st;
    }
    if (batch_pairs(plans, count, p)) {
        bool *fz = new bool[count];
        // K is even: the last half-sweep runs in a fused pair, which reads out
        // labels and soft-argmin both.
        for (int i = 0; i < count; ++i) fz[i] = (probs[i].disparity || probs[i].soft_disparity) && K >= 1;
        st = run_batched_pairs(probs, count, plans, p, ws, table_off, fz, ckpt, s);
        delete[] fz;
        return st;
    }
    // Problems grouped by lane split (classes of one launch each).
    int cls_S[32], cls_R[32], ncls = 0;
    bool cls_X[32];
    int *cls_of = new int[count];
    for (int i = 0; i < count; ++i) {
        int S, R;
        bool X;
        pm_split_variant(plans[i].L, plans[i].variant, &S, &R, &X);
        int c = 0;
        while (c < ncls && !(cls_S[c] == S && cls_R[c] == R && cls_X[c] == X)) ++c;
        if (c == ncls) {
            cls_S[c] = S;
            cls_R[c] = R;
            cls_X[c] = X;
            ++ncls;
        }
        cls_of[i] = c;
    }
    // The finest level's last half-sweep also reads out its senders' labels
    // (problems asking for argmin labels only); the readout pass then covers
    // the other colour.
    bool *fuse = new bool[count];
    for (int i = 0; i < count; ++i) fuse[i] = probs[i].disparity && !probs[i].soft_disparity && K >= 1;
    // Entries for every (level, kind), grouped by class; written once.  Kind
    // 3 (level 0 only) is the last half-sweep with the fused readout.
    const size_t nslot = ((size_t)n * 3 + 1) * ncls;
    BatchEntry *host = new BatchEntry[((size_t)n * 3 + 1) * count];
    BatchEntry *dev = (BatchEntry *)(ws + table_off);
    int *start = new int[nslot], *num = new int[nslot], *blocks = new int[nslot];
    int e = 0;
    for (int l = 0; l < n; ++l)
        for (int kind = 0; kind < (l == 0 ? 4 : 3); ++kind) {
            // Half-sweep index the entries stand for (its parity and whether it is 0).
            const int t = kind == 0 ? 0 : kind == 1 ? 1 : kind == 2 ? 2 : (K >= 1 ? K - 1 : 0);
            for (int c = 0; c < ncls; ++c) {
                const int slot = (kind == 3 ? n * 3 : l * 3 + kind) * ncls + c;
                start[slot] = e;
                num[slot] = 0;
                int b0 = 0;
                for (int i = 0; i < count; ++i) {
                    if (cls_of[i] != c) continue;
                    const Plan &pl = plans[i];
                    int src_mode = 0;
                    if (t == 0 && l < n - 1 && K >= 2 && pl.lv[l].fmt == pl.lv[l + 1].fmt) src_mode = 1;
                    int32_t *ro = (kind == 3 && fuse[i]) ? probs[i].disparity : nullptr;
                    BatchEntry &be = host[e++];
                    be.a = make_iter_args(pl, l, t, src_mode, p.lambda, p.tau, ro, ws);
                    be.block0 = b0;
                    b0 += pm_sweep_blocks(be.a.ncomp, cls_S[c], cls_X[c]);
                    ++num[slot];
                }
                blocks[slot] = b0;
            }
        }
    st = launch_write_entries(dev, host, e, s);
    for (int l = n - 1; l >= 0 && st == BP_OK; --l) {
        if (l < n - 1)
            for (int i = 0; i < count && st == BP_OK; ++i) {
                const Level &c = plans[i].lv[l], &pa = plans[i].lv[l + 1];
                if (!(K >= 2 && c.fmt == pa.fmt)) st = launch_parent_copy(plans[i], l, ws, s);
            }
        for (int t = 0; t < K && st == BP_OK; ++t) {
            const bool last = l == 0 && t == K - 1;
            const int kind = last ? 3 : t == 0 ? 0 : (t & 1 ? 1 : 2);
            for (int c = 0; c < ncls && st == BP_OK; ++c) {
                const int slot = (kind == 3 ? n * 3 : l * 3 + kind) * ncls + c;
                if (num[slot] == 0) continue;
                const int fmt = plans[0].lv[l].fmt;   // every problem has the same levels
                st = launch_iteration_batch(dev + start[slot], num[slot], blocks[slot], fmt, cls_S[c], cls_R[c],
                                            cls_X[c], last, s);
            }
        }
    }
    if (st == BP_OK) st = finish_batched(probs, count, plans, p, fuse, ws, s);
    delete[] fuse;
    delete[] host;
    delete[] start;
    delete[] num;
    delete[] blocks;
    delete[] cls_of;
    return st;
}

// The fixed scratch array of bp_run_noalloc on the stream's device: the
// current device, which a non-null stream must belong to.
bp_status noalloc_workspace(hipStream_t stream, void **ws)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BP_ERR_HIP;
    if (stream) {
        int sdev = -1;
        if (hipStreamGetDevice(stream, &sdev) != hipSuccess) return BP_ERR_HIP;
        if (sdev != dev) return BP_ERR_INVALID_ARGUMENT;
    }
    *ws = noalloc_scratch(dev);
    return *ws ? BP_OK : BP_ERR_HIP;
}

// bp_run on a workspace the caller has checked for alignment; a NULL
// workspace selects bp_run_noalloc's fixed array (ws_bytes is then its size),
// resolved only once the call has passed every other check.
bp_status run_checked(const bp_problem *probs, int32_t count, const bp_params *params, void *workspace,
                      size_t ws_bytes, void *checkpoints, size_t ckpt_bytes, hipStream_t stream)
{
    if (!probs || count < 1 || !valid_params(params)) return BP_ERR_INVALID_ARGUMENT;
    for (int i = 0; i < count; ++i) {
        if (!valid_problem(probs[i], *params)) return BP_ERR_INVALID_ARGUMENT;
        if (!supported_labels(probs[i].num_labels)) return BP_ERR_UNSUPPORTED;
    }
    const bool ck = params->checkpoint_every > 0;
    if (ck && !differentiable(*params)) return BP_ERR_UNSUPPORTED;
    if (ck && (!checkpoints || ((uintptr_t)checkpoints % kAlign) != 0)) return BP_ERR_INVALID_ARGUMENT;
    Plan *plans = new Plan[count];
    size_t total = 0, table = 0;
    bool batch = false;
    if (!plan_run(probs, count, params, plans, &total, &batch, &table)) {
        delete[] plans;
        return BP_ERR_UNSUPPORTED;
    }
    size_t ck_total = 0;
    if (ck)
        for (int i = 0; i < count; ++i)
            ck_total += checkpoint_bytes_of(plans[i], params->iters_per_level, params->checkpoint_every);
    const size_t table_off = total;
    total += table;
    if (ws_bytes < total || ckpt_bytes < ck_total) {
        delete[] plans;
        return BP_ERR_WORKSPACE_TOO_SMALL;
    }
    if (!workspace) {
        const bp_status ws = noalloc_workspace(stream, &workspace);
        if (ws != BP_OK) {
            delete[] plans;
            return ws;
        }
    }
    (void)hipGetLastError();
    if (batch) {
        bp_status bs = run_batched(probs, count, plans, *params, (uint8_t *)workspace, table_off,
                                   ck ? (uint8_t *)checkpoints : nullptr, stream);
        delete[] plans;
        return bs;
    }
    bp_status st = BP_OK;
    size_t ck_off = 0;
    for (int i = 0; i < count && st == BP_OK; ++i) {
        uint8_t *cp = ck ? (uint8_t *)checkpoints + ck_off : nullptr;
        st = run_one(probs[i], plans[i], *params, (uint8_t *)workspace, stream, nullptr, cp);
        if (ck) ck_off += checkpoint_bytes_of(plans[i], params->iters_per_level, params->checkpoint_every);
    }
    delete[] plans;
    return st;
}


}  // namespace

extern "C" {

const char *bp_status_string(bp_status status)
{
    switch (status) {
    case BP_OK: return "ok";
    case BP_ERR_INVALID_ARGUMENT: return "invalid argument";
    case BP_ERR_UNSUPPORTED: return "unsupported configuration";
    case BP_ERR_WORKSPACE_TOO_SMALL: return "workspace or checkpoint buffer too small";
    case BP_ERR_HIP: return "HIP runtime error at launch";
    default: return "unknown status";
    }
}

bp_status bp_cost_volume(const uint8_t *left, const uint8_t *right, int32_t width, int32_t height, int32_t channels,
                         int64_t row_stride_bytes, int32_t downsample, int32_t num_labels, float data_trunc,
                         int32_t rgb_mode, float *cost, hipStream_t stream)
{
    if (!valid_image_args(left, right, width, height, channels, row_stride_bytes, downsample) || !cost)
        return BP_ERR_INVALID_ARGUMENT;
    if (num_labels < 1 || num_labels > kMaxLabels || !(data_trunc >= 0.0f) || !std::isfinite(data_trunc))
        return BP_ERR_INVALID_ARGUMENT;
    if (rgb_mode != 0 && rgb_mode != 1) return BP_ERR_INVALID_ARGUMENT;
    if ((int64_t)(width / downsample) * (height / downsample) * num_labels >= (1ll << 40)) return BP_ERR_UNSUPPORTED;
    (void)hipGetLastError();
    return launch_cost_volume(left, right, width, height, channels, row_stride_bytes, downsample, num_labels,
                              data_trunc, rgb_mode, cost, stream);
}

bp_status bp_downsample(const uint8_t *in, int32_t width, int32_t height, int32_t channels, int64_t row_stride_bytes,
                        int32_t downsample, uint8_t *out, hipStream_t stream)
{
    if (!valid_image_args(in, out, width, height, channels, row_stride_bytes, downsample))
        return BP_ERR_INVALID_ARGUMENT;
    (void)hipGetLastError();
    return launch_downsample(in, width, height, channels, row_stride_bytes, downsample, out, stream);
}

size_t bp_workspace_size(const bp_problem *probs, int32_t count, const bp_params *params)
{
    if (!probs || count < 1 || !valid_params(params)) return 0;
    for (int i = 0; i < count; ++i)
        if (probs[i].width <= 0 || probs[i].height <= 0 || !supported_labels(probs[i].num_labels) ||
            (!probs[i].cost && !valid_pair(probs[i].pair, probs[i].width, probs[i].height)))
            return 0;
    Plan *plans = new Plan[count];
    size_t total = 0, table = 0;
    bool batch = false;
    const bool ok = plan_run(probs, count, params, plans, &total, &batch, &table);
    delete[] plans;
    return ok ? total + table : 0;
}

size_t bp_checkpoint_size(const bp_problem *probs, int32_t count, const bp_params *params)
{
    if (!probs || count < 1 || !valid_params(params) || params->checkpoint_every <= 0) return 0;
    if (!differentiable(*params)) return 0;
    for (int i = 0; i < count; ++i)
        if (probs[i].width <= 0 || probs[i].height <= 0 || !supported_labels(probs[i].num_labels)) return 0;
    Plan *plans = new Plan[count];
    size_t total = 0, bytes = 0;
    if (plan_all(probs, count, params, plans, &total))
        for (int i = 0; i < count; ++i) bytes += checkpoint_bytes_of(plans[i], params->iters_per_level, params->checkpoint_every);
    delete[] plans;
    return bytes;
}

bp_status bp_run(const bp_problem *probs, int32_t count, const bp_params *params, void *workspace, size_t ws_bytes,
                 void *checkpoints, size_t ckpt_bytes, hipStream_t stream)
{
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return BP_ERR_INVALID_ARGUMENT;
    return run_checked(probs, count, params, workspace, ws_bytes, checkpoints, ckpt_bytes, stream);
}

bp_status bp_run_noalloc(const bp_problem *probs, int32_t count, const bp_params *params, void *checkpoints,
                         size_t ckpt_bytes, hipStream_t stream)
{
    return run_checked(probs, count, params, nullptr, kNoallocScratchBytes, checkpoints, ckpt_bytes, stream);
}

bp_status bp_run_profiled(const bp_problem *probs, int32_t count, const bp_params *params, void *workspace,
                          size_t ws_bytes, hipStream_t stream, int32_t per_level, bp_launch_record *records,
                          int32_t capacity, int32_t *n_records)
{
    if (!records || capacity < 0 || !n_records || (per_level != 0 && per_level != 1)) return BP_ERR_INVALID_ARGUMENT;
    if (!probs || count != 1 || !valid_params(params)) return BP_ERR_INVALID_ARGUMENT;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return BP_ERR_INVALID_ARGUMENT;
    if (!valid_problem(probs[0], *params)) return BP_ERR_INVALID_ARGUMENT;
    if (!supported_labels(probs[0].num_labels)) return BP_ERR_UNSUPPORTED;
    if (params->checkpoint_every > 0) return BP_ERR_UNSUPPORTED;
    Plan plan;
    size_t total = 0;
    bool batch = false;
    if (!plan_run(probs, 1, params, &plan, &total, &batch)) return BP_ERR_UNSUPPORTED;
    if (ws_bytes < total) return BP_ERR_WORKSPACE_TOO_SMALL;
    (void)hipGetLastError();
    Recorder prof{records, new hipEvent_t[capacity > 0 ? capacity : 1][2], capacity, 0, per_level == 1};
    bp_status st = BP_OK;
    int made = 0;
    for (; made < capacity && st == BP_OK; ++made)
        if (hipEventCreate(&prof.ev[made][0]) != hipSuccess || hipEventCreate(&prof.ev[made][1]) != hipSuccess)
            st = BP_ERR_HIP;
    if (st == BP_OK) st = run_one(probs[0], plan, *params, (uint8_t *)workspace, stream, &prof);
    if (st == BP_OK && hipStreamSynchronize(stream) != hipSuccess) st = BP_ERR_HIP;
    for (int i = 0; st == BP_OK && i < prof.n; ++i)
        if (hipEventElapsedTime(&records[i].ms, prof.ev[i][0], prof.ev[i][1]) != hipSuccess) st = BP_ERR_HIP;
    for (int i = 0; i < made; ++i) {
        (void)hipEventDestroy(prof.ev[i][0]);
        (void)hipEventDestroy(prof.ev[i][1]);
    }
    delete[] prof.ev;
    *n_records = prof.n;
    return st;
}

bp_status bp_stream_probe(const void *src, size_t read_bytes, void *dst, size_t write_bytes, hipStream_t stream)
{
    if ((read_bytes && !src) || (write_bytes && !dst)) return BP_ERR_INVALID_ARGUMENT;
    if ((uintptr_t)src % 16 || (uintptr_t)dst % 16 || read_bytes % 16 || write_bytes % 16)
        return BP_ERR_INVALID_ARGUMENT;
    if (write_bytes < 16) return BP_ERR_INVALID_ARGUMENT;
    (void)hipGetLastError();
    return launch_stream(src, read_bytes, dst, write_bytes, stream);
}

bp_status bp_harris(const uint8_t *img, int32_t width, int32_t height, int64_t stride, int32_t grid, int64_t threshold,
                    int64_t *response, bp_corner *corners, hipStream_t stream)
{
    if (!img || !response || !corners || width <= 0 || height <= 0 || stride < width) return BP_ERR_INVALID_ARGUMENT;
    if (grid < 1 || grid > 1024) return BP_ERR_INVALID_ARGUMENT;
    (void)hipGetLastError();
    return launch_harris(img, width, height, stride, grid, threshold, response, corners, stream);
}

bp_status bp_zssd_match(const uint8_t *a, const uint8_t *b, int32_t width, int32_t height, int64_t stride,
                        const bp_corner *corners, int32_t n, int32_t patch_radius, int32_t search_radius,
                        bp_match *matches, hipStream_t stream)
{
    if (!a || !b || (n > 0 && (!corners || !matches)) || width <= 0 || height <= 0 || stride < width || n < 0)
        return BP_ERR_INVALID_ARGUMENT;
    if (patch_radius < 0 || patch_radius > 15 || search_radius < 0 || search_radius > 32) return BP_ERR_INVALID_ARGUMENT;
    (void)hipGetLastError();
    return launch_zssd(a, b, width, height, stride, corners, n, patch_radius, search_radius, matches, stream);
}

size_t bp_icp_workspace_size(int32_t n, int32_t m)
{
    if (n < 0 || m < 0 || m > (1 << 28)) return 0;
    return icp_workspace_bytes(n, m);
}

bp_status bp_icp(const float *src, int32_t n, const float *dst, int32_t m, const double *pose_in, int32_t iters,
                 float dmax, double *pose_out, double *rms, int32_t *pairs, int32_t *corr, void *workspace,
                 size_t ws_bytes, hipStream_t stream)
{
    if (n < 0 || m < 0 || m > (1 << 28) || iters < 0 || (n > 0 && !src) || (m > 0 && !dst) || !pose_in || !pose_out)
        return BP_ERR_INVALID_ARGUMENT;
    if (!(dmax > 0.0f) || !std::isfinite(dmax)) return BP_ERR_INVALID_ARGUMENT;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return BP_ERR_INVALID_ARGUMENT;
    if (ws_bytes < icp_workspace_bytes(n, m)) return BP_ERR_WORKSPACE_TOO_SMALL;
    (void)hipGetLastError();
    return launch_icp(src, n, dst, m, pose_in, iters, dmax, pose_out, rms, pairs, corr, (uint8_t *)workspace, stream);
}

bp_status bp_undistort(const uint8_t *in, int32_t width, int32_t height, int32_t channels, int64_t in_stride,
                       const bp_intrinsics *intrinsics, uint8_t *out, int64_t out_stride, hipStream_t stream)
{
    if (!in || !out || !intrinsics || width <= 0 || height <= 0 || (channels != 1 && channels != 3))
        return BP_ERR_INVALID_ARGUMENT;
    if (in_stride < (int64_t)width * channels || out_stride < (int64_t)width * channels) return BP_ERR_INVALID_ARGUMENT;
    const bp_intrinsics &K = *intrinsics;
    const float vals[7] = {K.fx, K.fy, K.cx, K.cy, K.k1, K.k2, K.k3};
    for (float x : vals)
        if (!std::isfinite(x)) return BP_ERR_INVALID_ARGUMENT;
    if (!(K.fx > 0.0f) || !(K.fy > 0.0f)) return BP_ERR_INVALID_ARGUMENT;
    (void)hipGetLastError();
    return launch_undistort(in, width, height, channels, in_stride, K, out, out_stride, stream);
}

static bp_status upsample_args(const int32_t *disp_lo, int32_t w_lo, int32_t h_lo, const uint8_t *guide_hi,
                               int32_t w_hi, int32_t h_hi, int32_t channels, int64_t guide_row_stride, float sigma_s,
                               float sigma_r, int32_t radius_lo, int *R)
{
    if (!disp_lo || !guide_hi || w_lo <= 0 || h_lo <= 0 || w_hi <= 0 || h_hi <= 0) return BP_ERR_INVALID_ARGUMENT;
    if ((channels != 1 && channels != 3) || guide_row_stride < (int64_t)w_hi * channels) return BP_ERR_INVALID_ARGUMENT;
    if (w_hi % w_lo || h_hi % h_lo || w_hi / w_lo != h_hi / h_lo) return BP_ERR_INVALID_ARGUMENT;
    if (!(sigma_s > 0.0f) || !(sigma_r > 0.0f) || !std::isfinite(sigma_s) || !std::isfinite(sigma_r))
        return BP_ERR_INVALID_ARGUMENT;
    const int s = w_hi / w_lo;
    *R = radius_lo < 0 ? (int)std::ceil(2.0 * sigma_s / s) : radius_lo;
    if (*R > 8 || w_hi >= (1 << 20) || h_hi >= (1 << 20)) return BP_ERR_UNSUPPORTED;
    return BP_OK;
}

bp_status bp_upsample(const int32_t *disp_lo, int32_t w_lo, int32_t h_lo, const uint8_t *guide_hi, int32_t w_hi,
                      int32_t h_hi, int32_t channels, int64_t guide_row_stride, float sigma_s, float sigma_r,
                      int32_t radius_lo, float *disp_hi, hipStream_t stream)
{
    if (!disp_hi) return BP_ERR_INVALID_ARGUMENT;
    int R = 0;
    const bp_status st = upsample_args(disp_lo, w_lo, h_lo, guide_hi, w_hi, h_hi, channels, guide_row_stride, sigma_s,
                                       sigma_r, radius_lo, &R);
    if (st != BP_OK) return st;
    (void)hipGetLastError();
    return launch_upsample(disp_lo, w_lo, h_lo, guide_hi, w_hi, h_hi, channels, guide_row_stride, sigma_s, sigma_r,
                           R, disp_hi, nullptr, nullptr, stream);
}

bp_status bp_upsample_points(const int32_t *disp_lo, int32_t w_lo, int32_t h_lo, const uint8_t *guide_hi,
                             int32_t w_hi, int32_t h_hi, int32_t channels, int64_t guide_row_stride, float sigma_s,
                             float sigma_r, int32_t radius_lo, const bp_camera *camera, float *disp_hi, float *points,
                             hipStream_t stream)
{
    if (!camera || !points) return BP_ERR_INVALID_ARGUMENT;
    const bp_camera &c = *camera;
    if (!std::isfinite(c.baseline) || !(c.focal > 0.0f) || !(c.du > 0.0f) || !(c.dv > 0.0f) ||
        !std::isfinite(c.focal) || !std::isfinite(c.du) || !std::isfinite(c.dv) || !std::isfinite(c.u0) ||
        !std::isfinite(c.v0))
        return BP_ERR_INVALID_ARGUMENT;
    int R = 0;
    const bp_status st = upsample_args(disp_lo, w_lo, h_lo, guide_hi, w_hi, h_hi, channels, guide_row_stride, sigma_s,
                                       sigma_r, radius_lo, &R);
    if (st != BP_OK) return st;
    (void)hipGetLastError();
    return launch_upsample(disp_lo, w_lo, h_lo, guide_hi, w_hi, h_hi, channels, guide_row_stride, sigma_s, sigma_r,
                           R, disp_hi, camera, points, stream);
}

// Launch tables of the backward call: the reverse steps' entries, or the
// batched rebuild half-sweeps' (one region, rewritten in stream order).
static size_t bwd_tables_bytes(int32_t count)
{
    return std::max(std::max(bwd_table_bytes(count), bwd_pm_table_bytes(count)),
                    align_up((size_t)count * sizeof(BatchEntry)));
}

// One rebuild half-sweep r of every problem's finest level in one launch per
// lane split (pixel-major states): entry i reads srcs[i] (a saved state, the
// zero half, or the problem's own state when NULL) and writes the problem's
// state buffer.
static bp_status rebuild_batched(const Plan *plans, int32_t count, int r, const uint8_t *const *srcs, float lambda,
                                 float tau, uint8_t *ws, uint8_t *table, hipStream_t s)
{
    BatchEntry *host = new BatchEntry[count];
    BatchEntry *dev = (BatchEntry *)table;
    bool *done = new bool[count]();
    bp_status st = BP_OK;
    int used = 0;
    for (int i = 0; i < count && st == BP_OK; ++i) {
        if (done[i]) continue;
        int S, R;
        bool X;
        pm_split_variant(plans[i].L, plans[i].variant, &S, &R, &X);
        const int first = used;
        int blocks = 0;
        for (int k = i; k < count; ++k) {
            int Sk, Rk;
            bool Xk;
            pm_split_variant(plans[k].L, plans[k].variant, &Sk, &Rk, &Xk);
            if (done[k] || Sk != S || Rk != R || Xk != X) continue;
            done[k] = true;
            BatchEntry &e = host[used++];
            e.a = make_iter_args(plans[k], 0, r, 0, lambda, tau, nullptr, ws);
            if (srcs[k]) e.a.src = srcs[k];
            e.block0 = blocks;
            blocks += pm_sweep_blocks(e.a.ncomp, S, X);
        }
        st = launch_write_entries(dev + first, host + first, used - first, s);
        if (st == BP_OK)
            st = launch_iteration_batch(dev + first, used - first, blocks, plans[i].lv[0].fmt, S, R, X, false, s);
    }
    delete[] host;
    delete[] done;
    return st;
}

// Backward workspace: per problem its forward plan (cost + a message state
// rebuilt from checkpoints), the message adjoint and, for pixel-major states,
// the cost adjoint in the cost's layout; then the (lambda, tau) partials of
// every reverse step of every problem, a zero colour half as large as the
// largest problem's (the colour-0 half of the zero state M_0, read in place)
// and the launch table.
static bool backward_layout(const bp_problem *probs, int32_t count, const bp_params *params, Plan *plans,
                            size_t *mbar_off, size_t *gcost_off, size_t *partial_off, int *n_partial,
                            size_t *zero_off, size_t *zero_bytes, size_t *table_off, size_t *total)
{
    const bool lm = adjoint_label_major(*params);
    size_t off = 0, zb = 0;
    int np = 0;
    for (int i = 0; i < count; ++i) {
        const bp_problem &q = probs[i];
        if (!make_plan(q.width, q.height, q.num_labels, 1, BP_MSG_F32, lm ? 1 : 0, off, &plans[i])) return false;
        // Replays write every slot a reverse step reads, and M_0's colour-0
        // half is read from the zero half: the state's out-of-grid slots are
        // all that needs zeroing.
        plans[i].zero_coarsest = false;
        zb = std::max(zb, (size_t)4 * plans[i].lv[0].blk * fmt_bytes(plans[i].lv[0].fmt));
        plans[i].variant = lm ? params->variant : 1;
        off += plans[i].bytes;
        mbar_off[i] = off;
        off += plans[i].lv[0].msg_bytes;
        gcost_off[i] = off;
        if (!lm) off += plans[i].lv[0].cost_bytes;
        np += params->iters_per_level * (lm ? bwd_step_blocks(plans[i]) : bwd_pm_blocks(plans[i]));
    }
    *partial_off = off;
    *n_partial = np;
    off += align_up((size_t)(np > 0 ? np : 1) * 2 * sizeof(float));
    *zero_off = off;
    *zero_bytes = align_up(zb);
    off += align_up(zb);
    *table_off = off;
    off += bwd_tables_bytes(count) + bwd_finish_bytes();
    *total = off;
    return true;
}

static bool valid_backward(const bp_problem *probs, int32_t count, const bp_params *params)
{
    if (!probs || count < 1 || !valid_params(params)) return false;
    if (params->checkpoint_every <= 0 || !differentiable(*params) || !(params->temperature > 0.0f)) return false;
    for (int i = 0; i < count; ++i)
        if (probs[i].width <= 0 || probs[i].height <= 0 || !probs[i].cost || !supported_labels(probs[i].num_labels))
            return false;
    return true;
}

size_t bp_backward_workspace_size(const bp_problem *probs, int32_t count, const bp_params *params)
{
    if (!valid_backward(probs, count, params)) return 0;
    for (int i = 0; i < count; ++i)
        if (probs[i].num_labels > kMaxBackwardLabels) return 0;
    Plan *plans = new Plan[count];
    size_t *mo = new size_t[count], *go = new size_t[count];
    size_t po = 0, zo = 0, zb = 0, to = 0, total = 0;
    int np = 0;
    bool ok = backward_layout(probs, count, params, plans, mo, go, &po, &np, &zo, &zb, &to, &total);
    delete[] plans;
    delete[] mo;
    delete[] go;
    return ok ? total : 0;
}

bp_status bp_backward(const bp_problem *probs, int32_t count, const bp_params *params, const void *checkpoints,
                      size_t ckpt_bytes, const float *grad_soft, float *grad_cost, float *grad_lambda,
                      float *grad_tau, void *workspace, size_t ws_bytes, hipStream_t stream)
{
    if (!probs || count < 1 || !valid_params(params)) return BP_ERR_INVALID_ARGUMENT;
    if (params->checkpoint_every <= 0 || !(params->temperature > 0.0f)) return BP_ERR_INVALID_ARGUMENT;
    if (!differentiable(*params)) return BP_ERR_UNSUPPORTED;
    if (!checkpoints || !grad_soft || !grad_cost || !grad_lambda || !grad_tau || !workspace) return BP_ERR_INVALID_ARGUMENT;
    if (((uintptr_t)workspace % kAlign) != 0 || ((uintptr_t)checkpoints % kAlign) != 0) return BP_ERR_INVALID_ARGUMENT;
    if (!valid_backward(probs, count, params)) return BP_ERR_INVALID_ARGUMENT;
    for (int i = 0; i < count; ++i)
        if (probs[i].num_labels > kMaxBackwardLabels) return BP_ERR_UNSUPPORTED;
    Plan *plans = new Plan[count];
    size_t *mo = new size_t[count], *go = new size_t[count];
    size_t po = 0, zo = 0, zb = 0, to = 0, total = 0;
    int np = 0;
    bp_status st = BP_OK;
    const int K = params->iters_per_level, every = params->checkpoint_every;
    const bool lm = adjoint_label_major(*params);
    if (!backward_layout(probs, count, params, plans, mo, go, &po, &np, &zo, &zb, &to, &total)) st = BP_ERR_UNSUPPORTED;
    size_t ck_total = 0;
    for (int i = 0; st == BP_OK && i < count; ++i) ck_total += checkpoint_bytes_of(plans[i], K, every);
    if (st == BP_OK && (ws_bytes < total || ckpt_bytes < ck_total)) st = BP_ERR_WORKSPACE_TOO_SMALL;
    if (st != BP_OK) {
        delete[] plans;
        delete[] mo;
        delete[] go;
        return st;
    }
    (void)hipGetLastError();
    uint8_t *ws = (uint8_t *)workspace;
    float *partial = (float *)(ws + po);
    const uint8_t *zero_half = ws + zo;
    const int nst = checkpoint_states(K, every);
    st = launch_zero(ws + zo, zb, stream);
    // Per problem: its checkpoints, state buffer, adjoints; the readout adjoint
    // from the final state initialises the message adjoint and the cost adjoint.
    const uint8_t **ck = new const uint8_t *[count];
    BwdProblem *bp = new BwdProblem[count];
    BwdPmProblem *bq = new BwdPmProblem[count];
    {
        const uint8_t *c = (const uint8_t *)checkpoints;
        size_t soft_off = 0, cost_off = 0;
        for (int i = 0; i < count && st == BP_OK; ++i) {
            const Plan &pl = plans[i];
            const size_t sb = pl.lv[0].msg_bytes;
            ck[i] = c;
            c += (size_t)nst * sb;
            float *mbar = (float *)(ws + mo[i]);
            bp[i] = BwdProblem{&pl, ws, ws + pl.lv[0].msg_off, mbar, grad_cost + cost_off, nullptr};
            bq[i] = BwdPmProblem{&pl, ws, ws + pl.lv[0].msg_off, mbar, (float *)(ws + go[i]), nullptr};
            if ((st = launch_split_cost(probs[i].cost, pl, ws, stream)) != BP_OK) break;
            // Out-of-grid slots of the state buffer: zero, and never written
            // afterwards (replays below write only the in-grid slots the
            // reverse steps read).
            if ((st = launch_init_messages(pl, ws, stream)) != BP_OK) break;
            const uint8_t *last = ck[i] + (size_t)(nst - 1) * sb;
            if (lm)
                st = launch_bwd_readout(pl, last, mbar, grad_soft + soft_off, bp[i].grad_cost, params->temperature, ws,
                                        stream);
            else
                st = launch_bwd_readout_pm(pl, last, mbar, bq[i].gcost, grad_soft + soft_off, params->temperature, ws,
                                           stream);
            soft_off += (size_t)probs[i].height * probs[i].width;
            cost_off += (size_t)probs[i].num_labels * probs[i].height * probs[i].width;
        }
    }
    // Reverse half-sweeps, newest first: rebuild every problem's M_t (restore
    // the last saved state at or before t, replay), then one batched step.
    // Pixel-major states of several problems replay in one launch per
    // half-sweep and lane split.
    const bool batch_rebuild = !lm && count > 1;
    const uint8_t **rsrc = new const uint8_t *[count];
    int part = 0;
    for (int t = K - 1; t >= 0 && st == BP_OK; --t) {
        const int t0 = (t / every) * every;
        if (batch_rebuild && t > t0) {
            for (int i = 0; i < count; ++i)
                rsrc[i] = t0 > 0 ? ck[i] + (size_t)(t0 / every - 1) * plans[i].lv[0].msg_bytes : zero_half;
            st = rebuild_batched(plans, count, t0, rsrc, params->lambda, params->tau, ws, ws + to, stream);
            for (int i = 0; i < count; ++i) rsrc[i] = nullptr;
            for (int r = t0 + 1; r < t && st == BP_OK; ++r)
                st = rebuild_batched(plans, count, r, rsrc, params->lambda, params->tau, ws, ws + to, stream);
        }
        for (int i = 0; i < count && st == BP_OK; ++i) {
            const Plan &pl = plans[i];
            const size_t sb = pl.lv[0].msg_bytes;
            uint8_t *state = ws + pl.lv[0].msg_off;
            const uint8_t *saved = t0 > 0 ? ck[i] + (size_t)(t0 / every - 1) * sb : nullptr;
            const uint8_t *mt = state;
            if (saved && t == t0) {
                // M_t is a saved state: the reverse step reads it in place.
                mt = saved;
            } else if (!saved && t == 0) {
                // M_0 is zero and the reverse step at t = 0 reads only its
                // colour-0 half: the zero half, in place.
                mt = zero_half;
            } else if (!batch_rebuild) {
                // Half-sweep r reads the slots of colour r & 1 and writes those of
                // the other colour, and the reverse step at t reads only the slots
                // of colour t & 1: the first replay reads the saved state (or M_0's
                // colour-0 half, the zero half) in place and writes into the state
                // buffer, no copy needed.
                int r = t0;
                st = launch_iteration_from(pl, r, saved ? saved : zero_half, params->lambda, params->tau, pl.variant,
                                           ws, stream);
                ++r;
                for (; r < t && st == BP_OK; ++r)
                    st = launch_iteration(pl, 0, r, 0, params->lambda, params->tau, nullptr, pl.variant, ws, stream);
            }
            bp[i].state = bq[i].state = mt;
            bp[i].partial = bq[i].partial = partial + 2 * part;
            part += lm ? bwd_step_blocks(pl) : bwd_pm_blocks(pl);
        }
        if (st != BP_OK) break;
        if (lm) st = launch_bwd_step_batch(bp, count, t, params->lambda, params->tau, ws + to, stream);
        else st = launch_bwd_step_pm_batch(bq, count, t, t == K - 1, params->lambda, params->tau, ws + to, stream);
    }
    if (!lm) {
        size_t cost_off = 0;
        for (int i = 0; i < count && st == BP_OK; ++i) {
            st = launch_gcost_to_planar(plans[i], bq[i].gcost, grad_cost + cost_off, stream);
            cost_off += (size_t)probs[i].num_labels * probs[i].height * probs[i].width;
        }
    }
    delete[] ck;
    delete[] bp;
    delete[] bq;
    delete[] rsrc;
    if (st == BP_OK)
        st = launch_bwd_finish(partial, np, grad_lambda, grad_tau,
                               ws + to + bwd_tables_bytes(count), stream);
    delete[] plans;
    delete[] mo;
    delete[] go;
    return st;
}

bp_status bp_load_tune_table(const char *path)
{
    std::vector<TuneEntry> t;
    if (path && !read_tune_file(path, &t)) return BP_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.swap(t);
    g_tune_init = true;
    return BP_OK;
}

int32_t bp_variant_count(int32_t num_labels)
{
    if (!supported_labels(num_labels)) return 0;
    const int lm = iteration_variants(num_labels), pm = pm_variants(num_labels);
    return lm > pm ? lm : pm;
}

}  // extern "C"
