/*
 * bp.h -- C ABI of libbpstereo: dense two-view stereo by hierarchical min-sum
 * loopy belief propagation with joint bilateral upsampling, for AMD Instinct
 * MI355X (gfx950).
 *
 * Method: "Towards Real-time 3D Reconstruction using Consumer UAVs", Sec. 2.2.
 * A rectified pair is downsampled, matched by minimising the per-pixel energy
 * of Eq. 1 (data term plus the messages of the four neighbours) with belief
 * propagation, read out as the minimising label, and upsampled to the full
 * resolution with the joint bilateral filter of Eq. 2.
 *
 * Conventions shared by every entry point:
 *  - Pointers to images, volumes, disparities, workspaces and checkpoints are
 *    DEVICE pointers owned by the caller.  Descriptor structs (bp_problem,
 *    bp_params) live in HOST memory and are only read during the call.
 *  - The library never allocates or frees device memory: scratch space comes
 *    from a caller-provided workspace whose size is returned by a query.
 *  - All work is enqueued on the given stream; no entry point except the
 *    measurement call bp_run_profiled synchronises the host, so every other
 *    call can be captured into a HIP graph.
 *  - Arguments are validated on the host before anything is enqueued.  On an
 *    error nothing is enqueued and a negative bp_status is returned.  A launch
 *    failure reported by the HIP runtime returns BP_ERR_HIP.  Text for any
 *    status: bp_status_string().
 *  - Calls are thread-safe: the only process-wide state is a read-only
 *    launch-shape table loaded at first use.
 *  - Image layout: row-major [H][row_stride] bytes, pixels of `channels`
 *    interleaved uint8 samples (1 = grey, 3 = RGB).  Volume layout: planar
 *    [L][H][W] float32, label-major.  Disparities: [H][W].
 *  - Left is the reference view: left pixel (x, y) at disparity d matches
 *    right pixel (x - d, y).
 */
#ifndef BPSTEREO_BP_H
#define BPSTEREO_BP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BP_OK = 0,
    BP_ERR_INVALID_ARGUMENT = -1,   /* a size, pointer or parameter is out of range */
    BP_ERR_UNSUPPORTED = -2,        /* valid but not supported (e.g. label count) */
    BP_ERR_WORKSPACE_TOO_SMALL = -3,/* workspace or checkpoint buffer smaller than queried */
    BP_ERR_HIP = -4                 /* the HIP runtime reported an error at launch */
} bp_status;

/* Storage format of BP messages.  Arithmetic is FP32 in every format; the
 * coarsest pyramid level always stores FP32. */
typedef enum { BP_MSG_F32 = 0, BP_MSG_F16 = 1, BP_MSG_BF16 = 2 } bp_msg_dtype;

/* A rectified pair from which bp_run computes the finest level's data term
 * itself, straight into its internal layout (the planar volume is never
 * stored).  The values are those bp_cost_volume writes for the same
 * arguments; the pair's size is (width * downsample) x (height * downsample)
 * with the bp_problem's width and height. */
typedef struct {
    const uint8_t *left, *right;   /* device images [height*downsample][row_stride_bytes] */
    int32_t channels;              /* 1 = grey, 3 = RGB */
    int32_t downsample;            /* s >= 1 */
    int64_t row_stride_bytes;      /* >= width * downsample * channels */
    float data_trunc;              /* >= 0 */
    int32_t rgb_mode;              /* 0 rounded channel mean, 1 exact (bp_cost_volume) */
} bp_pair;

/* One rectified pair's BP problem at the matching (low) resolution. */
typedef struct {
    int32_t width, height;     /* finest BP grid, >= 1 each */
    int32_t num_labels;        /* L in [2, 256] */
    const float *cost;         /* [L][height][width] data term E_D of Eq. 1, finest level */
    int32_t *disparity;        /* [height][width] argmin label output, or NULL */
    float *soft_disparity;     /* [height][width] soft-argmin output (label units), or NULL */
    float *messages_out;       /* [4][L][height][width] final finest-level messages, or NULL.
                                  Slot k = message received from the neighbour on side k
                                  (0 left, 1 right, 2 up, 3 down); 0 where there is none. */
    const bp_pair *pair;       /* host pointer, read when cost == NULL (bp_run, bp_run_profiled,
                                  bp_workspace_size); NULL otherwise */
} bp_problem;

/* Parameters of the method, shared by every problem of a call. */
typedef struct {
    int32_t levels;            /* pyramid levels n >= 1 (1 = single-level BP) */
    int32_t iters_per_level;   /* half-sweeps per level K >= 0 */
    float lambda;              /* smoothness weight >= 0: V(f,g) = lambda * min(|f-g|, tau) */
    float tau;                 /* truncation in labels > 0 */
    int32_t msg_dtype;         /* bp_msg_dtype */
    float temperature;         /* soft-argmin temperature T > 0 (used when soft_disparity != NULL) */
    int32_t checkpoint_every;  /* 0 = none; k > 0 saves, every k half-sweeps of the finest
                                  level, the part of the message state the adjoint reads
                                  (and the whole final state) into the checkpoint buffer,
                                  whose contents only bp_backward interprets */
    int32_t variant;           /* 0 = library choice: pixel-major levels with K >= 2 run two
                                  half-sweeps per launch (tiles whose colour-1 messages stay
                                  on chip between the two; a second buffer of half a level's
                                  messages in the workspace), also when checkpoints are saved
                                  every even number of half-sweeps; with count > 1 when K is
                                  even and every level of every problem does so (one launch
                                  per level, pair and lane split over the problems of a group
                                  whose working sets fit the on-package cache), otherwise one
                                  half-sweep per launch.  Else a half-sweep kernel variant in
                                  1..bp_variant_count() (testing and tuning).  Label-major
                                  levels: lanes per pixel 1/2/4 by label count.  Pixel-major
                                  levels: 1 default lane split, 2 half the lanes with twice
                                  the labels per lane, 3 and 4 the same with each direction's
                                  lanes reading only their own incoming message and sharing
                                  sums by lane shuffles, 5 (17..128 labels) a quarter of the
                                  lanes with shuffled sums.  A number beyond what one layout has
                                  selects that layout's variant 1.  Results do not depend on it. */
    int32_t pm_from;           /* first pyramid level stored pixel-major (labels of a pixel
                                  contiguous, half-sweep by lane-split scans); levels before it
                                  are label-major.  -1 = library choice, `levels` = none.
                                  Results do not depend on it. */
} bp_params;

/*
 * a1 + a2. Data term of Eq. 1 (the paper leaves its form open; this library
 * uses the truncated absolute difference).
 *   cost(d, x, y) = min(a(x, y, d), data_trunc)  if x - d >= 0, else data_trunc
 * where a is |I_L - I_R| for grey input and the channel mean of the absolute
 * differences for RGB: rounded to nearest, floor((sum + 1) / 3), when
 * rgb_mode == 0 (every value stays an integer), the exact mean when 1.
 * If downsample = s > 1 both images are first reduced by the s x s block mean
 * rounded half up (Sec. 2.2 matches on downsampled frames); width and height
 * must then be multiples of s and the output grid is (width/s) x (height/s).
 *   left, right   device images [height][row_stride_bytes], channels 1 or 3
 *   cost          device float32 [num_labels][height/s][width/s], written fully
 * Errors: BP_ERR_INVALID_ARGUMENT for NULL pointers, non-positive sizes,
 * channels not 1/3, stride < width*channels, s not dividing the sizes,
 * num_labels outside [1, 256], data_trunc < 0.
 */
bp_status bp_cost_volume(const uint8_t *left, const uint8_t *right, int32_t width, int32_t height,
                         int32_t channels, int64_t row_stride_bytes, int32_t downsample,
                         int32_t num_labels, float data_trunc, int32_t rgb_mode, float *cost,
                         hipStream_t stream);

/* Intrinsics of the distorted frame: pinhole focal lengths and principal point
 * in pixels, radial distortion coefficients (no tangential terms, Sec. 2.1). */
typedef struct {
    float fx, fy;     /* > 0 */
    float cx, cy;
    float k1, k2, k3;
} bp_intrinsics;

/*
 * Undistortion before matching (Sec. 2.1: radial-only model, every frame
 * undistorted and remapped).  Output pixel (u, v) = (column, row) samples
 * the input at
 *   xn = (u - cx) / fx, yn = (v - cy) / fy, r2 = xn^2 + yn^2,
 *   g = 1 + k1 r2 + k2 r2^2 + k3 r2^3,  (us, vs) = (cx + (u - cx) g, cy + (v - cy) g)
 * by bilinear interpolation of each channel, rounded half up; 0 where
 * (us, vs) lies outside [0, width-1] x [0, height-1].  Evaluated in FP32
 * with every operation rounded separately (1/fx and 1/fy once, as the
 * reciprocals in float), Horner form for g.  Zero coefficients reproduce the
 * input exactly.
 *   in, out   device images [height][stride] bytes, `channels` (1 or 3)
 *             interleaved u8 samples per pixel; must not overlap
 * Errors: BP_ERR_INVALID_ARGUMENT for NULL pointers, non-positive sizes,
 * channels not 1/3, strides < width * channels, non-finite intrinsics or
 * fx, fy not positive.
 */
bp_status bp_undistort(const uint8_t *in, int32_t width, int32_t height, int32_t channels, int64_t in_stride,
                       const bp_intrinsics *intrinsics, uint8_t *out, int64_t out_stride, hipStream_t stream);

/* A selected Harris corner: pixel and its response 25 R (Eq. 5 with
 * k = 1/25, an exact integer); x = y = -1 for a cell without a corner. */
typedef struct {
    int32_t x, y;
    int64_t response;
} bp_corner;

/* A ZSSD match: pixel of the second frame and its cost n * ZSSD (n patch
 * pixels, an exact integer); x = y = -1 when there is none. */
typedef struct {
    int32_t x, y;
    int64_t cost;
} bp_match;

/*
 * Harris corners of a grey frame (Sec. 2.3, Eq. 4-5, and the experiments' g x g
 * grid of cells with a hard threshold), in exact integers:
 *   A = I(x+1,y) - I(x-1,y), B = I(x,y+1) - I(x,y-1); M = sum w [A^2 AB; AB B^2]
 *   over the 5 x 5 binomial window w = (1 4 6 4 1)^T (1 4 6 4 1);
 *   response = 25 R = 25 det M - tr(M)^2 (k = 1/25), 0 within 3 pixels of
 *   the border.
 * Cell (i, j) covers columns [floor(j W/g), floor((j+1) W/g)) and rows
 * likewise; its corner is the pixel of largest response above `threshold`
 * among the 3 x 3 local maxima (no neighbour larger), first in row-major
 * order on ties.
 *   img        device u8 [height][stride]
 *   response   device int64 [height][width], written fully (the response map)
 *   corners    device bp_corner [grid * grid], cell (i, j) at i * grid + j
 * Errors: BP_ERR_INVALID_ARGUMENT for NULL pointers, non-positive sizes,
 * stride < width, grid outside [1, 1024].
 */
bp_status bp_harris(const uint8_t *img, int32_t width, int32_t height, int64_t stride, int32_t grid,
                    int64_t threshold, int64_t *response, bp_corner *corners, hipStream_t stream);

/*
 * ZSSD patch matching of corners of frame a in frame b (Sec. 2.3: a patch
 * around every corner, compared within a search range by zero-mean SSD):
 * cost = n sum (a - b)^2 - (sum a - sum b)^2 over (2 patch_radius + 1)^2 = n
 * pixels, i.e. n * ZSSD.  The match is the shift in [-search_radius,
 * search_radius]^2 whose patch lies inside frame b with the smallest cost,
 * the first in row-major (dy, dx) order on ties; none (-1) for a corner with
 * x < 0 or whose own patch leaves frame a.
 *   a, b       device u8 [height][stride], the two frames
 *   corners    device bp_corner [n] (e.g. from bp_harris)
 *   matches    device bp_match [n]
 * Errors: BP_ERR_INVALID_ARGUMENT for NULL pointers, non-positive sizes,
 * stride < width, n < 0, patch_radius outside [0, 15], search_radius
 * outside [0, 32].
 */
bp_status bp_zssd_match(const uint8_t *a, const uint8_t *b, int32_t width, int32_t height, int64_t stride,
                        const bp_corner *corners, int32_t n, int32_t patch_radius, int32_t search_radius,
                        bp_match *matches, hipStream_t stream);

/* Workspace bytes of bp_icp for n source and m target points (0 on invalid sizes). */
size_t bp_icp_workspace_size(int32_t n, int32_t m);

/*
 * Point-to-point ICP fine registration of a source cloud onto a target
 * cloud (Sec. 2.3: the clouds of Eq. 3 registered by ICP from the estimated
 * poses).  Per iteration:
 *  - every source point p is moved to p' = R p + T in FP32 (each operation
 *    rounded on its own: ((R_r0 p_0 + R_r1 p_1) + R_r2 p_2) + T_r) and paired
 *    with its nearest target within dmax (squared distance (dx^2 + dy^2) +
 *    dz^2 in FP32, ties to the lowest target index), or with none;
 *  - the least-squares rigid motion taking the paired p' onto their targets
 *    (FP64 centroids and cross-covariance, rotation by Horn's quaternion
 *    method) is composed onto the pose in FP64: R <- Ri R, T <- Ri T + Ti;
 *    an iteration with fewer than 3 pairs leaves the pose unchanged;
 *  - the next correspondences use the pose rounded to FP32.
 * Exact nearest neighbours as long as coordinates stay within about
 * 8e4 * dmax of the origin (a spatial hash of cells of edge dmax / 0.99).
 * Points with a non-finite coordinate never pair.
 *   src [n][3], dst [m][3]   device float32 points (n, m >= 0)
 *   pose_in, pose_out        device float64 [12]: R row-major, then T
 *   rms, pairs               device [iters] per-iteration RMS distance of the
 *                            pairs (float64) and pair count (int32), or NULL
 *   corr                     device int32 [n]: the last iteration's pairing
 *                            (target index or -1), or NULL
 *   workspace                bp_icp_workspace_size(n, m) bytes, 256-byte aligned
 * Errors: BP_ERR_INVALID_ARGUMENT for NULL points with n or m > 0, NULL
 * poses, negative sizes or iterations, dmax not positive and finite;
 * BP_ERR_WORKSPACE_TOO_SMALL; BP_ERR_HIP.
 */
bp_status bp_icp(const float *src, int32_t n, const float *dst, int32_t m, const double *pose_in, int32_t iters,
                 float dmax, double *pose_out, double *rms, int32_t *pairs, int32_t *corr, void *workspace,
                 size_t ws_bytes, hipStream_t stream);

/*
 * a1 alone: s x s block mean rounded half up, out [height/s][width/s][channels]
 * packed.  Same argument rules as bp_cost_volume.
 */
bp_status bp_downsample(const uint8_t *in, int32_t width, int32_t height, int32_t channels,
                        int64_t row_stride_bytes, int32_t downsample, uint8_t *out, hipStream_t stream);

/* Workspace bytes bp_run needs for `count` problems with `params` (a problem
 * without a cost volume must carry its valid pair); 0 on invalid input. */
size_t bp_workspace_size(const bp_problem *probs, int32_t count, const bp_params *params);

/* Checkpoint bytes bp_run writes when params->checkpoint_every > 0 (else 0). */
size_t bp_checkpoint_size(const bp_problem *probs, int32_t count, const bp_params *params);

/*
 * a3-a6 (and the batched form when count > 1). Minimises Eq. 1 by
 * coarse-to-fine min-sum BP and reads out the minimising label:
 *  - pyramid: level l cost = sum of its (up to four) level l-1 children;
 *    W_l = ceil(W_{l-1} / 2), likewise H;
 *  - the coarsest level starts from zero messages, each finer level from a
 *    copy of its parent's final messages (pixel (x,y) takes (x/2, y/2));
 *  - half-sweep t of a level (t = 0..K-1) updates every pixel with
 *    (x + y + t) mod 2 == 0: to each 4-neighbour q it sends the distance
 *    transform of h(f) = cost(f) + sum of its incoming messages except q's,
 *    m(f) = min_g h(g) + lambda * min(|f - g|, tau), minus min_f m(f);
 *  - readout: b(f) = cost(f) + sum of the four incoming messages; disparity =
 *    lowest f minimising b (Eq. 1's readout); soft = sum_f f w(f) / sum_f w(f)
 *    with w(f) = exp(-(b(f) - min b) / T).
 * probs     host array of `count` problems (count >= 1); each may differ in
 *           size and label count
 * workspace device scratch of at least bp_workspace_size() bytes, 256-byte aligned
 * checkpoints device buffer of bp_checkpoint_size() bytes, or NULL when
 *           checkpoint_every == 0 (used by bp_backward)
 * Errors: BP_ERR_INVALID_ARGUMENT (bad sizes, neither cost nor a valid pair, lambda < 0,
 * tau <= 0, soft output with T <= 0, misaligned workspace),
 * BP_ERR_UNSUPPORTED (label count outside [2, 256], 16-bit messages with
 * checkpointing), BP_ERR_WORKSPACE_TOO_SMALL, BP_ERR_HIP.
 */
bp_status bp_run(const bp_problem *probs, int32_t count, const bp_params *params, void *workspace,
                 size_t ws_bytes, void *checkpoints, size_t ckpt_bytes, hipStream_t stream);

/* Size of the fixed device array bp_run_noalloc works in: 640 MiB, which
 * holds bp_run's workspace for a 676 x 380 x 64-label five-level problem
 * computed from a pair (546 MiB); bp_workspace_size() tells whether a call
 * fits. */
#define BP_NOALLOC_SCRATCH_BYTES ((size_t)640 << 20)

/*
 * bp_run without a caller workspace, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  Same problems, parameters, checkpoints, launch
 * sequence, kernels and results as bp_run; the workspace is a fixed device
 * array of BP_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, which the
 * GPU holds from the first call on it until the process ends.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 *  - The array belongs to the current device; `stream` must be a stream of
 *    that device (or NULL).  The first call on each device resolves the
 *    array's device address (make it outside stream capture); later calls
 *    reuse it.
 *  - Every call on one GPU shares that GPU's array and leaves the last call's
 *    contents in it; each call initialises everything it reads, so results
 *    never depend on an earlier call.  Calls whose work overlaps on one GPU
 *    (other streams or threads, before the earlier call's work has finished)
 *    race on the array: serialise them, e.g. on one stream.
 * Errors: as bp_run, with BP_ERR_WORKSPACE_TOO_SMALL when the problems need
 * more than BP_NOALLOC_SCRATCH_BYTES (bp_workspace_size() > the array),
 * BP_ERR_INVALID_ARGUMENT for a stream of another device, BP_ERR_HIP when
 * the runtime cannot resolve the array's address.
 */
bp_status bp_run_noalloc(const bp_problem *probs, int32_t count, const bp_params *params, void *checkpoints,
                         size_t ckpt_bytes, hipStream_t stream);

/* One timed span of half-sweep launches (bp_run_profiled). */
typedef struct {
    int32_t level;          /* pyramid level of the launches (0 = finest) */
    int32_t half_sweep;     /* t of the first launch covered */
    int32_t launches;       /* launches covered: 1, or the level's K with per_level */
    int32_t readout_fused;  /* number of covered launches that also wrote the senders' labels */
    int32_t msg_bytes;      /* bytes per stored message value at this level (4 or 2) */
    double units;           /* pixel-label updates covered: half-sweeps * W_l * H_l * L */
    float ms;               /* time between HIP events recorded on `stream` around the span */
    double bytes;           /* algorithmic memory traffic of the covered launches, per pixel and
                               label of the level (mb = msg_bytes): a single half-sweep
                               (4 + 8 mb) / 2 (the active half reads its cost and four incoming
                               rows and writes four outgoing ones); a fused pair 4 + 4 mb (both
                               colours' costs, colour 0's rows read and written), plus 2 mb
                               for a pair that ends a level and stores colour 1's rows */
} bp_launch_record;

/*
 * Measurement form of bp_run for one problem (count must be 1): the same
 * launch sequence, with a HIP event pair recorded on `stream` around every
 * half-sweep launch (per_level = 0) or around the K back-to-back half-sweep
 * launches of every level (per_level = 1, which keeps the events' own cost
 * out of short launches), up to `capacity` records.  Unlike bp_run it
 * synchronises `stream` before returning.  Writes the number of records to
 * *n_records.  Errors as bp_run, plus BP_ERR_INVALID_ARGUMENT for NULL
 * records/n_records, negative capacity or per_level not 0/1.
 */
bp_status bp_run_profiled(const bp_problem *probs, int32_t count, const bp_params *params, void *workspace,
                          size_t ws_bytes, hipStream_t stream, int32_t per_level, bp_launch_record *records,
                          int32_t capacity, int32_t *n_records);

/*
 * a7. Joint bilateral upsampling, Eq. 2:
 *   D_p = (1/K_p) sum_{q in window} D'(q) s(|p_lo - q|) g(|I_p - I_q|)
 * with Gaussian s (sigma_s in full-resolution pixels) and g (sigma_r in
 * 0..255 units, Euclidean over channels); p_lo = (p + 0.5)/scale - 0.5;
 * window = low-resolution pixels within radius_lo of floor(p/scale) (clipped
 * to the grid); I_q is the guide at scale*q + floor(scale/2); scale =
 * w_hi / w_lo = h_hi / h_lo (an integer).  radius_lo < 0 selects
 * ceil(2 sigma_s / scale).  Output float32 [h_hi][w_hi] in low-resolution
 * label units (multiply by scale for full-resolution disparity).
 * Errors: BP_ERR_INVALID_ARGUMENT for NULL pointers, non-integer or unequal
 * scales, channels not 1/3, sigmas <= 0; BP_ERR_UNSUPPORTED for radius_lo > 8
 * or w_hi / h_hi of 2^20 or more.
 */
bp_status bp_upsample(const int32_t *disp_lo, int32_t w_lo, int32_t h_lo, const uint8_t *guide_hi,
                      int32_t w_hi, int32_t h_hi, int32_t channels, int64_t guide_row_stride,
                      float sigma_s, float sigma_r, int32_t radius_lo, float *disp_hi,
                      hipStream_t stream);

/* Pinhole camera of the full-resolution frame for bp_upsample_points. */
typedef struct {
    float baseline;   /* B: distance between the two views; points come out in its unit */
    float focal;      /* f > 0, in the unit of du and dv */
    float du, dv;     /* pixel pitch, horizontal and vertical, > 0 */
    float u0, v0;     /* principal point, full-resolution pixel coordinates (column, row) */
} bp_camera;

/*
 * a7 with its consumer fused (Eq. 3): joint bilateral upsampling as
 * bp_upsample, and in the same pass the camera-frame point of every
 * full-resolution pixel (u, v) = (column, row) with disparity
 * d = scale * D_p pixels:
 *   [x, y, z] = (B / d) [u - u0, (v - v0) dv / du, f / du]
 * which inverts Eq. 3's projection [u, v, d] = (1/z)[f x/du, f y/dv, f B/du]
 * + [u0, v0, 0] (the last entry of the printed inverse reads f B / du; the
 * projection fixes it as f / du).  Pixels with d <= 0 get NaN coordinates.
 *   disp_hi   float32 [h_hi][w_hi] as bp_upsample, or NULL to skip it
 *   points    float32 [h_hi][w_hi][3] (x, y, z), written fully
 * Errors: as bp_upsample, plus BP_ERR_INVALID_ARGUMENT for a NULL camera or
 * points, non-finite camera values, or focal, du or dv not positive.
 */
bp_status bp_upsample_points(const int32_t *disp_lo, int32_t w_lo, int32_t h_lo, const uint8_t *guide_hi,
                             int32_t w_hi, int32_t h_hi, int32_t channels, int64_t guide_row_stride,
                             float sigma_s, float sigma_r, int32_t radius_lo, const bp_camera *camera,
                             float *disp_hi, float *points, hipStream_t stream);

/*
 * a8. Adjoint of bp_run's single-level soft-argmin form: given the gradient
 * of a loss with respect to every problem's soft_disparity, returns its
 * gradient with respect to the cost volume, lambda and tau, by reverse-mode
 * differentiation through the K half-sweeps (each state rebuilt from the
 * checkpoints bp_run saved) and the soft-argmin.  The transform is piecewise
 * linear; the derivative follows the branch the forward pass took (forward
 * pass keeps h(f) on ties, backward pass keeps the current value, truncation
 * only when strictly smaller), and lambda/tau are shared scalars whose
 * gradients sum over the problems (reduced in a fixed order).  The forward
 * call stores its states pixel-major (the default) or label-major
 * (params->pm_from == levels); bp_backward uses the matching adjoint
 * kernels, so both calls must get the same params.  Results are
 * deterministic: repeated calls give identical bits.
 *   grad_soft   device float32, the problems' [H][W] arrays concatenated
 *   grad_cost   device float32, the problems' [L][H][W] arrays concatenated, overwritten
 *   grad_lambda, grad_tau  device float32[1] each, overwritten
 *   workspace   bp_backward_workspace_size() bytes, 256-byte aligned
 * Requires params->levels == 1, msg_dtype == BP_MSG_F32, checkpoint_every > 0,
 * temperature > 0 and the same problems, params and checkpoints as the
 * forward call.  Errors: BP_ERR_INVALID_ARGUMENT, BP_ERR_UNSUPPORTED (more
 * levels, 16-bit messages or more than 128 labels), BP_ERR_WORKSPACE_TOO_SMALL,
 * BP_ERR_HIP.
 */
bp_status bp_backward(const bp_problem *probs, int32_t count, const bp_params *params,
                      const void *checkpoints, size_t ckpt_bytes, const float *grad_soft,
                      float *grad_cost, float *grad_lambda, float *grad_tau, void *workspace,
                      size_t ws_bytes, hipStream_t stream);

/* Workspace bytes bp_backward needs; 0 on invalid input. */
size_t bp_backward_workspace_size(const bp_problem *probs, int32_t count, const bp_params *params);

/*
 * Launch-shape table written by the autotuner (paper_1902_09733_amd/tune.py):
 * text lines "width height labels fmt levels pm_from variant us".  When
 * bp_params.pm_from == -1 and variant == 0, a problem uses the entry with its
 * label count, format and level count whose pixel count is nearest (log
 * scale); results never depend on the choice.  In a batch (count > 1) that
 * can run fused pairs, the entries' layouts apply but not their half-sweep
 * variants (one problem on single half-sweeps would take the whole batch off
 * the pairs).  The table named by the
 * environment variable BP_TUNE_TABLE is read at the first planning call;
 * bp_load_tune_table replaces it (NULL clears it).  Errors:
 * BP_ERR_INVALID_ARGUMENT if the file cannot be opened.  Not to be called
 * concurrently with planning calls that should see a consistent table.
 */
bp_status bp_load_tune_table(const char *path);

/* Number of kernel variants bp_params.variant may select (1..count); 0 for an
 * unsupported label count. */
int32_t bp_variant_count(int32_t num_labels);

/*
 * Measurement aid, not part of the method: streams `read_bytes` from `src`
 * and writes `write_bytes` to `dst` in 16-byte accesses (chunk c of dst
 * receives a value derived from chunk c of src), so that the mix of a BP
 * launch's reads and writes can be timed alone and its sustained bandwidth
 * taken as the practical ceiling for that mix.  dst's first 16 bytes may
 * also be written when read_bytes > write_bytes.
 * Errors: BP_ERR_INVALID_ARGUMENT for NULL or misaligned pointers, sizes not
 * multiples of 16, or write_bytes < 16.
 */
bp_status bp_stream_probe(const void *src, size_t read_bytes, void *dst, size_t write_bytes, hipStream_t stream);

/* Static text for a status code. */
const char *bp_status_string(bp_status status);

#ifdef __cplusplus
}
#endif

#endif /* BPSTEREO_BP_H */
