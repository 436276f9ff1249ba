/*
 * FP64 CPU oracle for the differentiation form of the stereo path: reverse-mode
 * derivative of single-level checkerboard min-sum BP with a soft-argmin
 * readout, with respect to the data term, the smoothness weight lambda and the
 * truncation tau.
 *
 * TEST INFRASTRUCTURE ONLY (see bp_oracle.c).  Pinned by central finite
 * differences of its own forward pass in the CPU tests.
 *
 * Forward model (the same as bpo_run with one level): K half-sweeps from zero
 * messages; half-sweep t updates the pixels with (x + y + t) mod 2 == 0; a
 * message is the truncated-linear distance transform of
 * h = cost + incoming messages except the receiver's, minus its minimum; the
 * readout is d(p) = sum_f f w_f / sum_f w_f, w_f = exp(-(b_p(f) - min b_p) / T),
 * b_p = cost_p + sum of incoming messages.  Loss = sum_p g(p) d(p).
 *
 * The transform is piecewise linear in h, lambda and tau.  On each piece:
 *  - untruncated label f: m(f) = h(gB) + lambda |f - gB| - h(gmin), where gB
 *    is the label the two passes carried to f and gmin the lowest minimiser
 *    of h;
 *  - truncated label f: m(f) = lambda * tau.
 * Tie rule (a subgradient choice): the forward pass keeps h(f) when it equals
 * the carried value, the backward pass keeps the current value, truncation
 * applies only when min h + lambda tau is strictly smaller.
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

/* Distance transform of h with the winning source label of every output
 * label, the lowest minimiser of h and the truncation flags. */
static void dt_winners(const double *h, int L, double lambda, double tau, double *out, int *gB, int *gmin_out,
                       unsigned char *trunc)
{
    int gmin = 0;
    for (int f = 1; f < L; ++f)
        if (h[f] < h[gmin]) gmin = f;
    double *b = out;
    b[0] = h[0];
    gB[0] = 0;
    for (int f = 1; f < L; ++f) {
        double v = b[f - 1] + lambda;
        if (h[f] <= v) {
            b[f] = h[f];
            gB[f] = f;
        } else {
            b[f] = v;
            gB[f] = gB[f - 1];
        }
    }
    for (int f = L - 2; f >= 0; --f) {
        double v = b[f + 1] + lambda;
        if (v < b[f]) {
            b[f] = v;
            gB[f] = gB[f + 1];
        }
    }
    double cap = h[gmin] + lambda * tau;
    for (int f = 0; f < L; ++f) {
        trunc[f] = cap < b[f];
        out[f] = (trunc[f] ? cap : b[f]) - h[gmin];
    }
    *gmin_out = gmin;
}

typedef struct { int W, H, L; } geo_t;

#define IDX(g, k, d, y, x) ((((long)(k) * (g)->L + (d)) * (g)->H + (y)) * (g)->W + (x))
#define CIDX(g, d, y, x) (((long)(d) * (g)->H + (y)) * (g)->W + (x))

static int nb(const geo_t *g, int x, int y, int k)
{
    switch (k) {
    case 0: return x > 0;
    case 1: return x < g->W - 1;
    case 2: return y > 0;
    default: return y < g->H - 1;
    }
}

static const int DXA[4] = {-1, 1, 0, 0};
static const int DYA[4] = {0, 0, -1, 1};

/* One forward half-sweep from state `m` (updated in place). */
static void sweep(const geo_t *g, const double *cost, double *m, int t, double lambda, double tau)
{
    const int L = g->L;
#pragma omp parallel
    {
        double *h = (double *)malloc(sizeof(double) * L * 2);
        int *gB = (int *)malloc(sizeof(int) * L);
        unsigned char *tr = (unsigned char *)malloc((size_t)L);
        double *out = h + L;
        int gmin;
#pragma omp for schedule(static)
        for (int y = 0; y < g->H; ++y)
            for (int x = (y + t) & 1; x < g->W; x += 2)
                for (int q = 0; q < 4; ++q) {
                    if (!nb(g, x, y, q)) continue;
                    for (int d = 0; d < L; ++d) {
                        double v = cost[CIDX(g, d, y, x)];
                        for (int k = 0; k < 4; ++k)
                            if (k != q && nb(g, x, y, k)) v += m[IDX(g, k, d, y, x)];
                        h[d] = v;
                    }
                    dt_winners(h, L, lambda, tau, out, gB, &gmin, tr);
                    for (int d = 0; d < L; ++d) m[IDX(g, q ^ 1, d, y + DYA[q], x + DXA[q])] = out[d];
                }
        free(h);
        free(gB);
        free(tr);
    }
}

/* Forward pass (states kept) and reverse pass.  Outputs: soft [H][W] (forward
 * readout, may be NULL), grad_cost [L][H][W], *grad_lambda, *grad_tau. */
int bpo_backward(const double *cost, int W, int H, int L, int K, double lambda, double tau, double T,
                 const double *grad_soft, double *soft, double *grad_cost, double *grad_lambda, double *grad_tau,
                 int nthreads)
{
    if (!cost || !grad_soft || !grad_cost || !grad_lambda || !grad_tau || W <= 0 || H <= 0 || L <= 0 || K < 0 ||
        lambda < 0 || !(tau > 0) || !(T > 0))
        return BPO_EINVAL;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    geo_t G = {W, H, L};
    const geo_t *g = &G;
    const size_t n = (size_t)4 * L * H * W;
    double *states = (double *)calloc(n * (size_t)(K + 1), sizeof(double));
    double *mbar = (double *)calloc(n, sizeof(double));
    if (!states || !mbar) {
        free(states);
        free(mbar);
        return BPO_ENOMEM;
    }
    for (int t = 0; t < K; ++t) {
        memcpy(states + n * (t + 1), states + n * t, n * sizeof(double));
        sweep(g, cost, states + n * (t + 1), t, lambda, tau);
    }
    const double *mK = states + n * K;
    double gl = 0.0, gt = 0.0;
    memset(grad_cost, 0, sizeof(double) * (size_t)L * H * W);

    /* Readout adjoint: d = sum f p_f, dd/db_f = -(1/T) p_f (f - d). */
    double *b = (double *)malloc(sizeof(double) * L);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double bmin = INFINITY;
            for (int d = 0; d < L; ++d) {
                double v = cost[CIDX(g, d, y, x)];
                for (int k = 0; k < 4; ++k)
                    if (nb(g, x, y, k)) v += mK[IDX(g, k, d, y, x)];
                b[d] = v;
                if (v < bmin) bmin = v;
            }
            double den = 0.0, num = 0.0;
            for (int d = 0; d < L; ++d) {
                double w = exp(-(b[d] - bmin) / T);
                den += w;
                num += d * w;
            }
            double dh = num / den;
            if (soft) soft[(long)y * W + x] = dh;
            double gp = grad_soft[(long)y * W + x];
            for (int d = 0; d < L; ++d) {
                double pf = exp(-(b[d] - bmin) / T) / den;
                double bb = -gp / T * pf * (d - dh);
                grad_cost[CIDX(g, d, y, x)] += bb;
                for (int k = 0; k < 4; ++k)
                    if (nb(g, x, y, k)) mbar[IDX(g, k, d, y, x)] = bb;
            }
        }
    free(b);

    /* Reverse half-sweeps.  Sender pixels of step t read only their own slots
     * and write (here: consume the adjoint of) the other colour's, so pixels
     * are independent within a step. */
    for (int t = K - 1; t >= 0; --t) {
        const double *m = states + n * t;
        double lsum = 0.0, tsum = 0.0;
#pragma omp parallel reduction(+ : lsum, tsum)
        {
            double *h = (double *)malloc(sizeof(double) * L * 3);
            double *out = h + L, *hb = h + 2 * L;
            int *gB = (int *)malloc(sizeof(int) * L);
            unsigned char *tr = (unsigned char *)malloc((size_t)L);
            int gmin;
#pragma omp for schedule(static)
            for (int y = 0; y < H; ++y)
                for (int x = (y + t) & 1; x < W; x += 2)
                    for (int q = 0; q < 4; ++q) {
                        if (!nb(g, x, y, q)) continue;
                        for (int d = 0; d < L; ++d) {
                            double v = cost[CIDX(g, d, y, x)];
                            for (int k = 0; k < 4; ++k)
                                if (k != q && nb(g, x, y, k)) v += m[IDX(g, k, d, y, x)];
                            h[d] = v;
                            hb[d] = 0.0;
                        }
                        dt_winners(h, L, lambda, tau, out, gB, &gmin, tr);
                        const int nx = x + DXA[q], ny = y + DYA[q], slot = q ^ 1;
                        for (int d = 0; d < L; ++d) {
                            double mb = mbar[IDX(g, slot, d, ny, nx)];
                            if (tr[d]) {
                                lsum += mb * tau;
                                tsum += mb * lambda;
                            } else {
                                hb[gB[d]] += mb;
                                hb[gmin] -= mb;
                                lsum += mb * fabs((double)(d - gB[d]));
                            }
                            mbar[IDX(g, slot, d, ny, nx)] = 0.0;   /* overwritten at step t */
                        }
                        for (int d = 0; d < L; ++d) {
                            grad_cost[CIDX(g, d, y, x)] += hb[d];
                            for (int k = 0; k < 4; ++k)
                                if (k != q && nb(g, x, y, k)) mbar[IDX(g, k, d, y, x)] += hb[d];
                        }
                    }
            free(h);
            free(gB);
            free(tr);
        }
        gl += lsum;
        gt += tsum;
    }
    *grad_lambda = gl;
    *grad_tau = gt;
    free(states);
    free(mbar);
    return BPO_OK;
}
