// C ABI of libbpstereo (include/bp.h): host-side validation, workspace
// planning and the launch sequence of the hierarchical BP path.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

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
    return true;
}

bool valid_problem(const bp_problem &q, const bp_params &p)
{
    if (q.width <= 0 || q.height <= 0 || !q.cost) return false;
    if (q.soft_disparity && !(p.temperature > 0.0f)) return false;
    // Every level keeps at least one pixel.
    return true;
}

bool supported_labels(int L) { return L >= 2 && L <= kMaxLabels; }

// Problem plans laid out back to back in the workspace.
bool plan_all(const bp_problem *probs, int32_t count, const bp_params *p, Plan *plans, size_t *total)
{
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        const bp_problem &q = probs[i];
        if (!make_plan(q.width, q.height, q.num_labels, p->levels, p->msg_dtype, off, &plans[i])) return false;
        off += plans[i].bytes;
    }
    *total = align_up(off);
    return true;
}

// Optional per-launch timing of the half-sweep kernels (bp_run_profiled).
struct Recorder {
    bp_launch_record *rec;
    hipEvent_t (*ev)[2];
    int cap, n;
};

// Runs the whole hierarchical BP of one problem.
bp_status run_one(const bp_problem &q, const Plan &pl, const bp_params &p, uint8_t *ws, hipStream_t s,
                  Recorder *prof = nullptr)
{
    bp_status st;
    const int n = pl.levels, K = p.iters_per_level;
    for (int l = 0; l < n; ++l)
        if ((st = launch_zero_border(pl, l, ws, s)) != BP_OK) return st;
    if ((st = launch_split_cost(q.cost, pl, ws, s)) != BP_OK) return st;
    for (int l = 1; l < n; ++l)
        if ((st = launch_pyramid_level(pl, l, ws, s)) != BP_OK) return st;
    // The finest level's last half-sweep also reads out its senders' labels.
    const bool fuse_ro = q.disparity && !q.soft_disparity && K >= 1;
    for (int l = n - 1; l >= 0; --l) {
        int first_src = 0;
        if (l == n - 1) {
            // The coarsest level starts from zero messages.
            if ((st = launch_zero_level(pl, l, ws, s)) != BP_OK) return st;
        } else {
            const bool same_fmt = pl.lv[l].fmt == pl.lv[l + 1].fmt;
            if (K >= 2 && same_fmt) first_src = 1;        // t = 0 reads the parent's slots
            else if ((st = launch_parent_copy(pl, l, ws, s)) != BP_OK) return st;
        }
        for (int t = 0; t < K; ++t) {
            int32_t *ro = (l == 0 && t == K - 1 && fuse_ro) ? q.disparity : nullptr;
            const bool rec = prof && prof->n < prof->cap;
            if (rec && hipEventRecord(prof->ev[prof->n][0], s) != hipSuccess) return BP_ERR_HIP;
            if ((st = launch_iteration(pl, l, t, t == 0 ? first_src : 0, p.lambda, p.tau, ro, p.variant, ws, s)) != BP_OK)
                return st;
            if (rec) {
                if (hipEventRecord(prof->ev[prof->n][1], s) != hipSuccess) return BP_ERR_HIP;
                bp_launch_record &r = prof->rec[prof->n++];
                r.level = l;
                r.half_sweep = t;
                r.readout_fused = ro != nullptr;
                r.msg_bytes = fmt_bytes(pl.lv[l].fmt);
                r.units = (double)pl.lv[l].w * pl.lv[l].h * pl.L;
                r.ms = 0.0f;
            }
        }
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
        if (probs[i].width <= 0 || probs[i].height <= 0 || !supported_labels(probs[i].num_labels)) return 0;
    Plan *plans = new Plan[count];
    size_t total = 0;
    bool ok = plan_all(probs, count, params, plans, &total);
    delete[] plans;
    return ok ? total : 0;
}

size_t bp_checkpoint_size(const bp_problem *probs, int32_t count, const bp_params *params)
{
    if (!probs || count < 1 || !valid_params(params) || params->checkpoint_every <= 0) return 0;
    return 0;
}

bp_status bp_run(const bp_problem *probs, int32_t count, const bp_params *params, void *workspace, size_t ws_bytes,
                 void *checkpoints, size_t ckpt_bytes, hipStream_t stream)
{
    if (!probs || count < 1 || !valid_params(params)) return BP_ERR_INVALID_ARGUMENT;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return BP_ERR_INVALID_ARGUMENT;
    for (int i = 0; i < count; ++i) {
        if (!valid_problem(probs[i], *params)) return BP_ERR_INVALID_ARGUMENT;
        if (!supported_labels(probs[i].num_labels)) return BP_ERR_UNSUPPORTED;
    }
    if (params->checkpoint_every > 0) return BP_ERR_UNSUPPORTED;
    (void)checkpoints;
    (void)ckpt_bytes;
    Plan *plans = new Plan[count];
    size_t total = 0;
    if (!plan_all(probs, count, params, plans, &total)) {
        delete[] plans;
        return BP_ERR_UNSUPPORTED;
    }
    if (ws_bytes < total) {
        delete[] plans;
        return BP_ERR_WORKSPACE_TOO_SMALL;
    }
    (void)hipGetLastError();
    bp_status st = BP_OK;
    for (int i = 0; i < count && st == BP_OK; ++i) st = run_one(probs[i], plans[i], *params, (uint8_t *)workspace, stream);
    delete[] plans;
    return st;
}

bp_status bp_run_profiled(const bp_problem *probs, int32_t count, const bp_params *params, void *workspace,
                          size_t ws_bytes, hipStream_t stream, bp_launch_record *records, int32_t capacity,
                          int32_t *n_records)
{
    if (!records || capacity < 0 || !n_records) return BP_ERR_INVALID_ARGUMENT;
    if (!probs || count != 1 || !valid_params(params)) return BP_ERR_INVALID_ARGUMENT;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return BP_ERR_INVALID_ARGUMENT;
    if (!valid_problem(probs[0], *params)) return BP_ERR_INVALID_ARGUMENT;
    if (!supported_labels(probs[0].num_labels)) return BP_ERR_UNSUPPORTED;
    if (params->checkpoint_every > 0) return BP_ERR_UNSUPPORTED;
    Plan plan;
    size_t total = 0;
    if (!plan_all(probs, 1, params, &plan, &total)) return BP_ERR_UNSUPPORTED;
    if (ws_bytes < total) return BP_ERR_WORKSPACE_TOO_SMALL;
    (void)hipGetLastError();
    Recorder prof{records, new hipEvent_t[capacity > 0 ? capacity : 1][2], capacity, 0};
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

bp_status bp_upsample(const int32_t *disp_lo, int32_t w_lo, int32_t h_lo, const uint8_t *guide_hi, int32_t w_hi,
                      int32_t h_hi, int32_t channels, int64_t guide_row_stride, float sigma_s, float sigma_r,
                      int32_t radius_lo, float *disp_hi, hipStream_t stream)
{
    if (!disp_lo || !guide_hi || !disp_hi || w_lo <= 0 || h_lo <= 0 || w_hi <= 0 || h_hi <= 0)
        return BP_ERR_INVALID_ARGUMENT;
    if ((channels != 1 && channels != 3) || guide_row_stride < (int64_t)w_hi * channels) return BP_ERR_INVALID_ARGUMENT;
    if (w_hi % w_lo || h_hi % h_lo || w_hi / w_lo != h_hi / h_lo) return BP_ERR_INVALID_ARGUMENT;
    if (!(sigma_s > 0.0f) || !(sigma_r > 0.0f) || !std::isfinite(sigma_s) || !std::isfinite(sigma_r))
        return BP_ERR_INVALID_ARGUMENT;
    const int s = w_hi / w_lo;
    int R = radius_lo < 0 ? (int)std::ceil(2.0 * sigma_s / s) : radius_lo;
    if (R > 8) return BP_ERR_UNSUPPORTED;
    (void)hipGetLastError();
    return launch_upsample(disp_lo, w_lo, h_lo, guide_hi, w_hi, h_hi, channels, guide_row_stride, sigma_s, sigma_r,
                           R, disp_hi, stream);
}

bp_status bp_backward(const bp_problem *probs, int32_t count, const bp_params *params, const void *checkpoints,
                      size_t ckpt_bytes, const float *grad_soft, float *grad_cost, float *grad_lambda,
                      float *grad_tau, void *workspace, size_t ws_bytes, hipStream_t stream)
{
    (void)probs; (void)count; (void)params; (void)checkpoints; (void)ckpt_bytes; (void)grad_soft;
    (void)grad_cost; (void)grad_lambda; (void)grad_tau; (void)workspace; (void)ws_bytes; (void)stream;
    return BP_ERR_UNSUPPORTED;
}

size_t bp_backward_workspace_size(const bp_problem *probs, int32_t count, const bp_params *params)
{
    (void)probs; (void)count; (void)params;
    return 0;
}

int32_t bp_variant_count(int32_t num_labels)
{
    if (!supported_labels(num_labels)) return 0;
    return iteration_variants(num_labels);
}

}  // extern "C"
