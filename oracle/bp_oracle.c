/*
 * FP64 CPU oracle for the dense two-view stereo path of "Towards Real-time 3D
 * Reconstruction using Consumer UAVs" (Sec. 2.2, Eq. 1 and Eq. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library; it is written as plain loops in the
 * order the method states its steps, for a reader to check by eye.
 *
 * What it computes (readings of the paper are listed with each function):
 *   bpo_downsample   integer box downsampling of the 2.7K frames (Sec. 2.2)
 *   bpo_cost_volume  truncated absolute-difference data term E_D (Eq. 1)
 *   bpo_dt / bpo_dt_brute   one message update under a truncated-linear
 *                    smoothness term: the two-pass distance transform and
 *                    the O(L^2) min-plus definition it must equal
 *   bpo_run          hierarchical min-sum loopy BP on the 4-connected grid,
 *                    checkerboard schedule, then the label minimising
 *                    E_X(d) = E_D,X(d) + sum_Y M_{Y,X}(d) (Eq. 1), or the
 *                    soft-argmin of the same energy
 *   bpo_upsample     joint bilateral upsampling of the disparity (Eq. 2)
 *   bpo_triangulate  camera-frame point of every full-resolution pixel from
 *                    its disparity (Eq. 3)
 *
 * Message slot convention: m[k][d][y][x] is the message pixel (x,y) received
 * from its neighbour on side k, k = 0 left, 1 right, 2 up, 3 down.
 * Messages from outside the grid (or across an edge removed by the optional
 * test-only edge mask) are zero and are never sent.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BPO_OK 0
#define BPO_EINVAL (-1)
#define BPO_ENOMEM (-2)

/* ------------------------------------------------------------------ */
/* Storage rounding used to emulate 16-bit message storage.            */
/* ------------------------------------------------------------------ */

/* Round x to a binary float with `mant` explicit mantissa bits, minimum
 * normal exponent `emin` (unbiased) and maximum finite value `maxval`,
 * round-to-nearest-even, with gradual underflow.  IEEE binary16: mant 10,
 * emin -14, max 65504.  bfloat16: mant 7, emin -126, max 3.3895e38. */
static double round_to_format(double x, int mant, int emin, double maxval)
{
    if (x == 0.0 || !isfinite(x)) return x;
    double ax = fabs(x);
    int e;
    frexp(ax, &e);               /* ax = f * 2^e, f in [0.5, 1) */
    int exp_unbiased = e - 1;    /* ax in [2^(e-1), 2^e) */
    if (exp_unbiased < emin) exp_unbiased = emin;   /* subnormal spacing */
    double ulp = ldexp(1.0, exp_unbiased - mant);
    double r = nearbyint(ax / ulp) * ulp;           /* default mode: ties to even */
    if (r > maxval) r = INFINITY;
    return x < 0 ? -r : r;
}

double bpo_round_f16(double x) { return round_to_format(x, 10, -14, 65504.0); }
double bpo_round_bf16(double x) { return round_to_format(x, 7, -126, 3.3895313892515355e38); }
double bpo_round_f32(double x) { return (double)(float)x; }

/* ------------------------------------------------------------------ */
/* a1: box downsampling                                                */
/* ------------------------------------------------------------------ */

/* Each output channel value is the s x s block mean, rounded half up:
 * floor((sum + s*s/2) / (s*s)).  Width and height must be multiples of s.
 * Layout [H][W][C] with rows packed. */
int bpo_downsample(const uint8_t *in, int W, int H, int C, int s, uint8_t *out)
{
    if (!in || !out || W <= 0 || H <= 0 || C <= 0 || s <= 0 || W % s || H % s) return BPO_EINVAL;
    int w = W / s, h = H / s;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x)
            for (int c = 0; c < C; ++c) {
                long sum = 0;
                for (int j = 0; j < s; ++j)
                    for (int i = 0; i < s; ++i)
                        sum += in[((long)(s * y + j) * W + (s * x + i)) * C + c];
                out[((long)y * w + x) * C + c] = (uint8_t)((sum + (s * s) / 2) / (s * s));
            }
    return BPO_OK;
}

/* ------------------------------------------------------------------ */
/* a2: data term                                                       */
/* ------------------------------------------------------------------ */

/* C(d, x, y) = min(a, T) with a the absolute intensity difference between the
 * left pixel (x, y) and the right pixel (x - d, y); C = T when x - d < 0 (the
 * match leaves the right image).  Colour: a is the channel mean of the
 * absolute differences, rounded to nearest (floor((sum + 1) / 3)) when
 * rgb_mode = 0, or the unrounded mean when rgb_mode = 1.  Output [L][H][W]. */
int bpo_cost_volume(const uint8_t *left, const uint8_t *right, int W, int H, int C, int L,
                    double trunc, int rgb_mode, double *cost)
{
    if (!left || !right || !cost || W <= 0 || H <= 0 || (C != 1 && C != 3) || L <= 0) return BPO_EINVAL;
    for (int d = 0; d < L; ++d)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double v;
                if (x - d < 0) {
                    v = trunc;
                } else {
                    const uint8_t *pl = left + ((long)y * W + x) * C;
                    const uint8_t *pr = right + ((long)y * W + (x - d)) * C;
                    double a;
                    if (C == 1) {
                        a = fabs((double)pl[0] - (double)pr[0]);
                    } else {
                        int sum = 0;
                        for (int c = 0; c < 3; ++c) sum += abs((int)pl[c] - (int)pr[c]);
                        a = rgb_mode == 0 ? (double)((sum + 1) / 3) : (double)sum / 3.0;
                    }
                    v = a < trunc ? a : trunc;
                }
                cost[((long)d * H + y) * W + x] = v;
            }
    return BPO_OK;
}

/* ------------------------------------------------------------------ */
/* a5: one message update                                              */
/* ------------------------------------------------------------------ */

/* Message for smoothness V(f, g) = lambda * min(|f - g|, tau):
 *   m(f) = min_g h(g) + V(f, g), then m -= min_f m.
 * Two-pass distance transform: a forward pass a(f) = min(h(f), a(f-1) + lambda),
 * a backward pass a(f) = min(a(f), a(f+1) + lambda), then truncation at
 * min_g h(g) + lambda * tau, then subtraction of the minimum. */
void bpo_dt(const double *h, int L, double lambda, double tau, double *out)
{
    double hmin = h[0];
    for (int f = 1; f < L; ++f) if (h[f] < hmin) hmin = h[f];
    out[0] = h[0];
    for (int f = 1; f < L; ++f) {
        double v = out[f - 1] + lambda;
        out[f] = h[f] < v ? h[f] : v;
    }
    for (int f = L - 2; f >= 0; --f) {
        double v = out[f + 1] + lambda;
        if (v < out[f]) out[f] = v;
    }
    double cap = hmin + lambda * tau;
    for (int f = 0; f < L; ++f) if (cap < out[f]) out[f] = cap;
    double mmin = out[0];
    for (int f = 1; f < L; ++f) if (out[f] < mmin) mmin = out[f];
    for (int f = 0; f < L; ++f) out[f] -= mmin;
}

/* The same message by its definition, O(L^2). */
void bpo_dt_brute(const double *h, int L, double lambda, double tau, double *out)
{
    for (int f = 0; f < L; ++f) {
        double best = INFINITY;
        for (int g = 0; g < L; ++g) {
            double dist = fabs((double)(f - g));
            double v = h[g] + lambda * (dist < tau ? dist : tau);
            if (v < best) best = v;
        }
        out[f] = best;
    }
    double mmin = out[0];
    for (int f = 1; f < L; ++f) if (out[f] < mmin) mmin = out[f];
    for (int f = 0; f < L; ++f) out[f] -= mmin;
}

/* ------------------------------------------------------------------ */
/* a3-a6: hierarchical checkerboard BP and readout                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int W, H, L;
    const uint8_t *edges;  /* [H][W]: bit 0 = edge to (x+1,y), bit 1 = edge to (x,y+1); NULL = full grid */
} grid_t;

/* Does pixel (x, y) have a neighbour on side k (0 left, 1 right, 2 up, 3 down)? */
static int has_nb(const grid_t *g, int x, int y, int k)
{
    switch (k) {
    case 0: return x > 0 && (!g->edges || (g->edges[(long)y * g->W + x - 1] & 1));
    case 1: return x < g->W - 1 && (!g->edges || (g->edges[(long)y * g->W + x] & 1));
    case 2: return y > 0 && (!g->edges || (g->edges[(long)(y - 1) * g->W + x] & 2));
    default: return y < g->H - 1 && (!g->edges || (g->edges[(long)y * g->W + x] & 2));
    }
}

static const int DX[4] = {-1, 1, 0, 0};
static const int DY[4] = {0, 0, -1, 1};

#define MSG(m, g, k, d, y, x) ((m)[(((long)(k) * (g)->L + (d)) * (g)->H + (y)) * (g)->W + (x)])
#define CST(c, g, d, y, x) ((c)[((long)(d) * (g)->H + (y)) * (g)->W + (x)])

/* Storage rounding applied to every stored message (emulates 16-bit storage). */
static double store_round(double v, int store_mode)
{
    switch (store_mode) {
    case 1: return bpo_round_f16(v);
    case 2: return bpo_round_bf16(v);
    case 3: return bpo_round_f32(v);
    default: return v;
    }
}

/* One checkerboard half-sweep: every pixel with (x + y + t) mod 2 == 0 sends
 * to each of its neighbours q the distance transform of
 *   h(f) = C(f) + sum of its incoming messages except the one from q,
 * summed in the fixed order left, right, up, down; the result lands in q's
 * slot for messages from that side.  Senders only read their own slots and
 * only write the other colour's slots, so the order of pixels is free. */
static void half_sweep(const grid_t *g, const double *cost, double *m, int t, double lambda, double tau,
                       int store_mode, int dt_mode)
{
    const int L = g->L;
#pragma omp parallel
    {
        double *h = (double *)malloc(sizeof(double) * (size_t)L * 2);
        double *out = h + L;
#pragma omp for schedule(static)
        for (int y = 0; y < g->H; ++y) {
            for (int x = (y + t) & 1; x < g->W; x += 2) {
                for (int q = 0; q < 4; ++q) {
                    if (!has_nb(g, x, y, q)) continue;
                    for (int d = 0; d < L; ++d) {
                        double v = CST(cost, g, d, y, x);
                        for (int k = 0; k < 4; ++k)
                            if (k != q && has_nb(g, x, y, k)) v += MSG(m, g, k, d, y, x);
                        h[d] = v;
                    }
                    if (dt_mode == 0) bpo_dt(h, L, lambda, tau, out);
                    else bpo_dt_brute(h, L, lambda, tau, out);
                    int nx = x + DX[q], ny = y + DY[q];
                    int slot = q ^ 1;  /* q sees p on the opposite side */
                    for (int d = 0; d < L; ++d) MSG(m, g, slot, d, ny, nx) = store_round(out[d], store_mode);
                }
            }
        }
        free(h);
    }
}

/* Belief b(f) = C(f) + sum of incoming messages (Eq. 1), its lowest-index
 * minimiser and, if requested, the soft-argmin sum_f f w(f) / sum_f w(f)
 * with w(f) = exp(-(b(f) - min b) / T). */
static void readout(const grid_t *g, const double *cost, const double *m, int32_t *disp, double *soft,
                    double temperature)
{
    const int L = g->L;
#pragma omp parallel
    {
        double *b = (double *)malloc(sizeof(double) * (size_t)L);
#pragma omp for schedule(static)
        for (int y = 0; y < g->H; ++y)
            for (int x = 0; x < g->W; ++x) {
                int best = 0;
                for (int d = 0; d < L; ++d) {
                    double v = CST(cost, g, d, y, x);
                    for (int k = 0; k < 4; ++k)
                        if (has_nb(g, x, y, k)) v += MSG(m, g, k, d, y, x);
                    b[d] = v;
                    if (v < b[best]) best = d;
                }
                if (disp) disp[(long)y * g->W + x] = best;
                if (soft) {
                    double num = 0.0, den = 0.0;
                    for (int d = 0; d < L; ++d) {
                        double w = exp(-(b[d] - b[best]) / temperature);
                        num += d * w;
                        den += w;
                    }
                    soft[(long)y * g->W + x] = num / den;
                }
            }
        free(b);
    }
}

/* Grid size of level l: W_l = ceil(W_{l-1} / 2), the same for H. */
static int level_dim(int n, int l)
{
    for (int i = 0; i < l; ++i) n = (n + 1) / 2;
    return n;
}

/* Cost of level l: the sum of the (up to four) children at level l-1.  Label
 * count, smoothness weight and truncation are the same at every level. */
static void pyramid_level(const double *fine, int Wf, int Hf, int L, double *coarse, int Wc, int Hc)
{
    for (int d = 0; d < L; ++d)
        for (int y = 0; y < Hc; ++y)
            for (int x = 0; x < Wc; ++x) {
                double s = 0.0;
                for (int j = 0; j < 2; ++j)
                    for (int i = 0; i < 2; ++i) {
                        int fx = 2 * x + i, fy = 2 * y + j;
                        if (fx < Wf && fy < Hf) s += fine[((long)d * Hf + fy) * Wf + fx];
                    }
                coarse[((long)d * Hc + y) * Wc + x] = s;
            }
}

/* Hierarchical BP.
 *   cost         [L][H][W] data term at the finest level
 *   levels       number of pyramid levels (1 = plain single-level BP)
 *   iters        half-sweeps per level; iteration t of every level updates
 *                the pixels with (x + y + t) mod 2 == 0
 *   store_mode   0 FP64 messages; 1/2 round every stored message (sent or
 *                copied from the parent) to binary16 / bfloat16, except at the
 *                coarsest level; 3 round to binary32
 *   dt_mode      0 two-pass distance transform, 1 O(L^2) definition
 *   edges        optional test-only edge mask at the finest level (levels must be 1)
 *   msgs_init    optional [4][L][H][W] initial messages (levels must be 1)
 *   msgs_out     optional [4][L][H][W] final messages at the finest level
 *   disp, soft   optional [H][W] argmin / soft-argmin readouts
 * The coarsest level starts from zero messages; every finer level starts from
 * a copy of its parent's final messages, m_l(x, y) = m_{l+1}(x/2, y/2). */
int bpo_run(const double *cost, int W, int H, int L, int levels, int iters, double lambda, double tau,
            int store_mode, int dt_mode, const uint8_t *edges, const double *msgs_init, double *msgs_out,
            int32_t *disp, double *soft, double temperature, int nthreads)
{
    if (!cost || W <= 0 || H <= 0 || L <= 0 || levels < 1 || iters < 0 || lambda < 0 || !(tau > 0))
        return BPO_EINVAL;
    if ((edges || msgs_init) && levels != 1) return BPO_EINVAL;
    if (soft && !(temperature > 0)) return BPO_EINVAL;
    if (levels > 1 && (level_dim(W, levels - 1) < 1)) return BPO_EINVAL;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    double **costs = (double **)calloc((size_t)levels, sizeof(double *));
    if (!costs) return BPO_ENOMEM;
    costs[0] = (double *)cost;
    for (int l = 1; l < levels; ++l) {
        int Wf = level_dim(W, l - 1), Hf = level_dim(H, l - 1);
        int Wc = level_dim(W, l), Hc = level_dim(H, l);
        costs[l] = (double *)malloc(sizeof(double) * (size_t)L * Wc * Hc);
        if (!costs[l]) return BPO_ENOMEM;
        pyramid_level(costs[l - 1], Wf, Hf, L, costs[l], Wc, Hc);
    }
    double *parent = NULL;
    int Wp = 0, Hp = 0;
    for (int l = levels - 1; l >= 0; --l) {
        grid_t g = {level_dim(W, l), level_dim(H, l), L, l == 0 ? edges : NULL};
        size_t n = (size_t)4 * L * g.H * g.W;
        double *m = (double *)calloc(n, sizeof(double));
        if (!m) return BPO_ENOMEM;
        /* 16-bit storage never applies to the coarsest level. */
        int sm = (l == levels - 1 && (store_mode == 1 || store_mode == 2)) ? 0 : store_mode;
        if (parent) {
            /* The copy lands in this level's storage format. */
            for (int k = 0; k < 4; ++k)
                for (int d = 0; d < L; ++d)
                    for (int y = 0; y < g.H; ++y)
                        for (int x = 0; x < g.W; ++x)
                            MSG(m, &g, k, d, y, x) =
                                store_round(parent[(((long)k * L + d) * Hp + y / 2) * Wp + x / 2], sm);
            free(parent);
        } else if (msgs_init) {
            memcpy(m, msgs_init, n * sizeof(double));
        }
        for (int t = 0; t < iters; ++t) half_sweep(&g, costs[l], m, t, lambda, tau, sm, dt_mode);
        if (l == 0) {
            readout(&g, costs[0], m, disp, soft, temperature);
            if (msgs_out) {
                for (int k = 0; k < 4; ++k)
                    for (int d = 0; d < L; ++d)
                        for (int y = 0; y < g.H; ++y)
                            for (int x = 0; x < g.W; ++x)
                                MSG(msgs_out, &g, k, d, y, x) = has_nb(&g, x, y, k) ? MSG(m, &g, k, d, y, x) : 0.0;
            }
            free(m);
        } else {
            parent = m;
            Wp = g.W;
            Hp = g.H;
        }
    }
    for (int l = 1; l < levels; ++l) free(costs[l]);
    free(costs);
    return BPO_OK;
}

/* Cost of pyramid level `level` from the finest-level cost (exposed for tests). */
int bpo_pyramid(const double *cost, int W, int H, int L, int level, double *out)
{
    if (!cost || !out || level < 0) return BPO_EINVAL;
    int Wf = W, Hf = H;
    double *cur = (double *)malloc(sizeof(double) * (size_t)L * W * H);
    if (!cur) return BPO_ENOMEM;
    memcpy(cur, cost, sizeof(double) * (size_t)L * W * H);
    for (int l = 1; l <= level; ++l) {
        int Wc = (Wf + 1) / 2, Hc = (Hf + 1) / 2;
        double *nxt = (double *)malloc(sizeof(double) * (size_t)L * Wc * Hc);
        if (!nxt) { free(cur); return BPO_ENOMEM; }
        pyramid_level(cur, Wf, Hf, L, nxt, Wc, Hc);
        free(cur);
        cur = nxt;
        Wf = Wc;
        Hf = Hc;
    }
    memcpy(out, cur, sizeof(double) * (size_t)L * Wf * Hf);
    free(cur);
    return BPO_OK;
}

/* ------------------------------------------------------------------ */
/* a7: joint bilateral upsampling (Eq. 2)                              */
/* ------------------------------------------------------------------ */

/* For every full-resolution pixel p:
 *   D_p = (1/K_p) sum_{q_lo in W} D'(q_lo) s(|p_lo - q_lo|) g(|I_p - I_q|)
 * with Gaussian s (sigma_s in full-resolution pixels) and g (sigma_r in
 * 0..255 intensity units, Euclidean over the channels), K_p the sum of the
 * weights.  p_lo = (p + 0.5) / s - 0.5 per axis (pixel centres aligned); the
 * window W is the square of radius R low-resolution pixels around floor(p/s),
 * clipped to the grid; I_q is the guide at the full-resolution pixel
 * s * q_lo + floor(s/2).  The weights are evaluated as exp(-(e - e_min)) with
 * e the sum of both Gaussian exponents and e_min its minimum over the window:
 * the common factor cancels in the ratio, so this is Eq. 2 exactly, and no
 * weight underflows to an all-zero K_p.  Output is in low-resolution label
 * units.  R < 0 selects R = ceil(2 sigma_s / s). */
int bpo_upsample(const int32_t *disp_lo, int wl, int hl, const uint8_t *guide, int wh, int hh, int C,
                 double sigma_s, double sigma_r, int R, double *out, int nthreads)
{
    if (!disp_lo || !guide || !out || wl <= 0 || hl <= 0 || wh <= 0 || hh <= 0 || (C != 1 && C != 3))
        return BPO_EINVAL;
    if (wh % wl || hh % hl || wh / wl != hh / hl || !(sigma_s > 0) || !(sigma_r > 0)) return BPO_EINVAL;
    int s = wh / wl;
    if (R < 0) R = (int)ceil(2.0 * sigma_s / s);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int ntap = (2 * R + 1) * (2 * R + 1);
#pragma omp parallel
    {
        double *e = (double *)malloc(sizeof(double) * (size_t)ntap);
        int32_t *dv = (int32_t *)malloc(sizeof(int32_t) * (size_t)ntap);
#pragma omp for schedule(static)
        for (int py = 0; py < hh; ++py)
            for (int px = 0; px < wh; ++px) {
                double plx = (px + 0.5) / s - 0.5, ply = (py + 0.5) / s - 0.5;
                int cx = px / s, cy = py / s;
                const uint8_t *ip = guide + ((long)py * wh + px) * C;
                int n = 0;
                for (int qy = cy - R; qy <= cy + R; ++qy) {
                    if (qy < 0 || qy >= hl) continue;
                    for (int qx = cx - R; qx <= cx + R; ++qx) {
                        if (qx < 0 || qx >= wl) continue;
                        double dsx = s * (plx - qx), dsy = s * (ply - qy);
                        const uint8_t *iq = guide + ((long)(s * qy + s / 2) * wh + (s * qx + s / 2)) * C;
                        double r2 = 0.0;
                        for (int c = 0; c < C; ++c) {
                            double dc = (double)ip[c] - (double)iq[c];
                            r2 += dc * dc;
                        }
                        e[n] = (dsx * dsx + dsy * dsy) / (2.0 * sigma_s * sigma_s) + r2 / (2.0 * sigma_r * sigma_r);
                        dv[n] = disp_lo[(long)qy * wl + qx];
                        ++n;
                    }
                }
                double emin = e[0];
                for (int i = 1; i < n; ++i) if (e[i] < emin) emin = e[i];
                double num = 0.0, den = 0.0;
                for (int i = 0; i < n; ++i) {
                    double w = exp(-(e[i] - emin));
                    num += w * dv[i];
                    den += w;
                }
                out[(long)py * wh + px] = num / den;
            }
        free(e);
        free(dv);
    }
    return BPO_OK;
}

int bpo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Triangulation (Eq. 3).                                              */
/* ------------------------------------------------------------------ */

/* Eq. 3, first line: a camera-frame point (x, y, z) projects to
 *   u = f x / (du z) + u0,  v = f y / (dv z) + v0,  d = f B / (du z).
 * Solving for the point with the disparity d in pixels:
 *   z = f B / (du d),  x = (u - u0) du z / f = (B / d)(u - u0),
 *   y = (v - v0) dv z / f = (B / d)(v - v0) dv / du,
 * so [x, y, z] = (B / d) [u - u0, (v - v0) dv / du, f / du].  (The printed
 * second line has f B / du as its last entry, which would make z grow with
 * B^2; the first line fixes it as f / du.)
 * disp: full-resolution disparity [h][w] in units of 1/scale pixels (the
 * upsampled low-resolution labels), so d = scale * disp; (u, v) = (column,
 * row) of the pixel.  Pixels with d <= 0 (no finite depth) get NaN.
 * out: [h][w][3] (x, y, z). */
int bpo_triangulate(const double *disp, int w, int h, double scale, double B, double f, double du, double dv,
                    double u0, double v0, double *out)
{
    if (!disp || !out || w <= 0 || h <= 0 || !(scale > 0) || !(f > 0) || !(du > 0) || !(dv > 0)) return BPO_EINVAL;
    for (int v = 0; v < h; ++v)
        for (int u = 0; u < w; ++u) {
            const double d = scale * disp[(size_t)v * w + u];
            double *o = out + ((size_t)v * w + u) * 3;
            if (!(d > 0)) {
                o[0] = o[1] = o[2] = NAN;
                continue;
            }
            const double k = B / d;
            o[0] = k * (u - u0);
            o[1] = k * (v - v0) * dv / du;
            o[2] = k * f / du;
        }
    return BPO_OK;
}
