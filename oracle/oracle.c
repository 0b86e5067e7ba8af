/*
 * oracle.c -- plain, slow, FP64 CPU reference of the direct-form filter and
 * its closed-form backward.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code with the HIP path.
 *
 * Paper: Yu & Fazekas, "Accelerating Automatic Differentiation of Direct Form
 * Digital Filters" (arXiv 2511.14390).
 *
 * Notation (paper -> here):
 *   paper's signal length N  -> T,  filter order M -> N (feedback) / M (feed-forward)
 *   x(n), y(n)               -> x[n], y[n]
 *   dL/dy(n)                 -> gy[n]
 *   dL/dz(n) (Eq. 7, scalar) -> ybar[n]   (gradient w.r.t. the all-pole input)
 *
 * Forward (Eq. 1 read as a difference equation with per-sample coefficients,
 * sign convention a_0 = 1 of Eq. 1):
 *   y[n] = sum_{k=0..M} b_k[n] x[n-k] - sum_{k=1..N} a_k[n] y[n-k],  n = 0..T-1,
 *   with x[-j] = xi[j-1], y[-j] = yi[j-1] (zero where not given).
 *
 * Backward (Sec. 3.1, Eqs. 6-9 and Appendix A, written for the scalar
 * direct form with the all-pole state [y(n-1) .. y(n-N)] of Eq. 4/5):
 *   ybar[n] = gy[n] - sum_{k=1..N, n+k<T} a_k[n+k] ybar[n+k]     (Eq. 7, reverse time,
 *             the recursion starts from zero past the last sample, App. A.1)
 *   gx[n]   = sum_{k=0..M, n+k<T} b_k[n+k] ybar[n+k]              (Eq. 8)
 *   gb_k[n] = ybar[n] x[n-k],  ga_k[n] = -ybar[n] y[n-k]         (Eqs. 6, 9; summed over n
 *                                                                  when the coefficients are
 *                                                                  time-invariant)
 *   gxi[j-1] = sum_{k=j..M} b_k[k-j] ybar[k-j]                    (initial-condition
 *   gyi[j-1] = -sum_{k=j..N} a_k[k-j] ybar[k-j]                    gradients, Eq. 9 / App. A.3)
 *
 * Every function is a direct loop over these definitions, in the order the
 * equations are written; no blocking or reordering.
 *
 * Layouts: signals are [T][B] (layout 0, channel fastest) or [B][T] (layout 1,
 * time fastest).  Time-invariant coefficients are [B][K]; per-sample
 * coefficients follow the signal layout with the tap index innermost:
 * [T][B][K] or [B][T][K].  a holds a_1..a_N (K = N), b holds b_0..b_M (K = M+1).
 * Initial conditions are [B][M] (xi, most recent first) and [B][N] (yi).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef struct {
    int64_t B, T;
    int M, N, tv, layout;
} oprob;

static int64_t sig(const oprob *p, int64_t b, int64_t t)
{
    return p->layout == 0 ? t * p->B + b : b * p->T + t;
}

static int64_t coef(const oprob *p, int64_t b, int64_t t, int K)
{
    if (!p->tv)
        return b * K;
    return (p->layout == 0 ? t * p->B + b : b * p->T + t) * (int64_t)K;
}

/* b_k[n]; a missing b means b = [1] (M must then be 0). */
static double bcoef(const oprob *p, const double *bc, int64_t b, int64_t n, int k)
{
    if (!bc)
        return k == 0 ? 1.0 : 0.0;
    return bc[coef(p, b, n, p->M + 1) + k];
}

/* a_k[n], k = 1..N */
static double acoef(const oprob *p, const double *ac, int64_t b, int64_t n, int k)
{
    return ac[coef(p, b, n, p->N) + (k - 1)];
}

/* x[m] for any integer m < T: negative times come from the initial conditions. */
static double xval(const oprob *p, const double *x, const double *xi, int64_t b, int64_t m)
{
    if (m >= 0)
        return x[sig(p, b, m)];
    int64_t j = -m; /* x[-j] = xi[j-1] */
    if (!xi || j > p->M)
        return 0.0;
    return xi[b * p->M + (j - 1)];
}

static double yval(const oprob *p, const double *y, const double *yi, int64_t b, int64_t m)
{
    if (m >= 0)
        return y[sig(p, b, m)];
    int64_t j = -m;
    if (!yi || j > p->N)
        return 0.0;
    return yi[b * p->N + (j - 1)];
}

static void forward_channel(const oprob *p, int64_t b, const double *x, const double *bc,
                            const double *ac, const double *xi, const double *yi, double *y)
{
    for (int64_t n = 0; n < p->T; ++n) {
        double acc = 0.0;
        for (int k = 0; k <= p->M; ++k)
            acc += bcoef(p, bc, b, n, k) * xval(p, x, xi, b, n - k);
        for (int k = 1; k <= p->N; ++k)
            acc -= acoef(p, ac, b, n, k) * yval(p, y, yi, b, n - k);
        y[sig(p, b, n)] = acc;
    }
}

typedef struct {
    const oprob *p;
    int64_t b0, b1;
    const double *gy, *x, *y, *bc, *ac, *xi, *yi;
    double *out_y, *gx, *gb, *ga, *gxi, *gyi;
    int backward;
    int status;
} job;

static int backward_channel(const oprob *p, int64_t b, const double *gy, const double *x,
                            const double *y, const double *bc, const double *ac,
                            const double *xi, const double *yi, double *gx, double *gb,
                            double *ga, double *gxi, double *gyi)
{
    const int64_t T = p->T;
    double *ybar = (double *)malloc((size_t)(T > 0 ? T : 1) * sizeof(double));
    if (!ybar)
        return 1;
    /* Eq. 7: reverse-time adjoint; terms past the last sample are absent. */
    for (int64_t n = T - 1; n >= 0; --n) {
        double acc = gy[sig(p, b, n)];
        for (int k = 1; k <= p->N; ++k)
            if (n + k < T)
                acc -= acoef(p, ac, b, n + k, k) * ybar[n + k];
        ybar[n] = acc;
    }
    /* Eq. 8: gradient of the input. */
    if (gx) {
        for (int64_t n = 0; n < T; ++n) {
            double acc = 0.0;
            for (int k = 0; k <= p->M; ++k)
                if (n + k < T)
                    acc += bcoef(p, bc, b, n + k, k) * ybar[n + k];
            gx[sig(p, b, n)] = acc;
        }
    }
    /* Eqs. 6 and 9: coefficient gradients. */
    if (gb) {
        const int K = p->M + 1;
        if (p->tv) {
            for (int64_t n = 0; n < T; ++n)
                for (int k = 0; k <= p->M; ++k)
                    gb[coef(p, b, n, K) + k] = ybar[n] * xval(p, x, xi, b, n - k);
        } else {
            for (int k = 0; k <= p->M; ++k) {
                double acc = 0.0;
                for (int64_t n = 0; n < T; ++n)
                    acc += ybar[n] * xval(p, x, xi, b, n - k);
                gb[b * K + k] = acc;
            }
        }
    }
    if (ga) {
        const int K = p->N;
        if (p->tv) {
            for (int64_t n = 0; n < T; ++n)
                for (int k = 1; k <= p->N; ++k)
                    ga[coef(p, b, n, K) + (k - 1)] = -ybar[n] * yval(p, y, yi, b, n - k);
        } else {
            for (int k = 1; k <= p->N; ++k) {
                double acc = 0.0;
                for (int64_t n = 0; n < T; ++n)
                    acc -= ybar[n] * yval(p, y, yi, b, n - k);
                ga[b * K + (k - 1)] = acc;
            }
        }
    }
    /* Initial-condition gradients: x[-j] and y[-j] enter outputs n = k - j. */
    if (gxi) {
        for (int j = 1; j <= p->M; ++j) {
            double acc = 0.0;
            for (int k = j; k <= p->M; ++k)
                if (k - j < T)
                    acc += bcoef(p, bc, b, k - j, k) * ybar[k - j];
            gxi[b * p->M + (j - 1)] = acc;
        }
    }
    if (gyi) {
        for (int j = 1; j <= p->N; ++j) {
            double acc = 0.0;
            for (int k = j; k <= p->N; ++k)
                if (k - j < T)
                    acc -= acoef(p, ac, b, k - j, k) * ybar[k - j];
            gyi[b * p->N + (j - 1)] = acc;
        }
    }
    free(ybar);
    return 0;
}

static void *run_job(void *arg)
{
    job *J = (job *)arg;
    for (int64_t b = J->b0; b < J->b1; ++b) {
        if (J->backward) {
            if (backward_channel(J->p, b, J->gy, J->x, J->y, J->bc, J->ac, J->xi, J->yi,
                                 J->gx, J->gb, J->ga, J->gxi, J->gyi))
                J->status = 1;
        } else {
            forward_channel(J->p, b, J->x, J->bc, J->ac, J->xi, J->yi, J->out_y);
        }
    }
    return NULL;
}

static int check(const oprob *p, const double *bc)
{
    if (p->B < 0 || p->T < 0 || p->M < 0 || p->N < 0)
        return 1;
    if (!bc && p->M != 0)
        return 1;
    if (p->layout != 0 && p->layout != 1)
        return 1;
    return 0;
}

/* Runs the channels on `nthreads` threads (contiguous channel ranges). */
static int dispatch(job *proto, int nthreads)
{
    const int64_t B = proto->p->B;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > B)
        nthreads = (int)(B > 0 ? B : 1);
    job *jobs = (job *)calloc((size_t)nthreads, sizeof(job));
    pthread_t *tid = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return 1;
    }
    int status = 0;
    for (int i = 0; i < nthreads; ++i) {
        jobs[i] = *proto;
        jobs[i].b0 = B * i / nthreads;
        jobs[i].b1 = B * (i + 1) / nthreads;
        jobs[i].status = 0;
    }
    if (nthreads == 1) {
        run_job(&jobs[0]);
    } else {
        for (int i = 0; i < nthreads; ++i)
            if (pthread_create(&tid[i], NULL, run_job, &jobs[i]))
                status = 1;
        for (int i = 0; i < nthreads; ++i)
            pthread_join(tid[i], NULL);
    }
    for (int i = 0; i < nthreads; ++i)
        status |= jobs[i].status;
    free(jobs);
    free(tid);
    return status;
}

/* Forward filter.  Returns 0 on success, 1 on invalid arguments. */
int oracle_forward(int64_t B, int64_t T, int M, int N, int tv, int layout, const double *x,
                   const double *bc, const double *ac, const double *xi, const double *yi,
                   double *y, int nthreads)
{
    oprob p = {B, T, M, N, tv, layout};
    if (check(&p, bc) || (N > 0 && !ac))
        return 1;
    job J;
    memset(&J, 0, sizeof J);
    J.p = &p;
    J.x = x;
    J.bc = bc;
    J.ac = ac;
    J.xi = xi;
    J.yi = yi;
    J.out_y = y;
    return dispatch(&J, nthreads);
}

/* Backward.  Any of gx, gb, ga, gxi, gyi may be NULL (not computed). */
int oracle_backward(int64_t B, int64_t T, int M, int N, int tv, int layout, const double *gy,
                    const double *x, const double *y, const double *bc, const double *ac,
                    const double *xi, const double *yi, double *gx, double *gb, double *ga,
                    double *gxi, double *gyi, int nthreads)
{
    oprob p = {B, T, M, N, tv, layout};
    if (check(&p, bc) || (N > 0 && !ac))
        return 1;
    job J;
    memset(&J, 0, sizeof J);
    J.p = &p;
    J.gy = gy;
    J.x = x;
    J.y = y;
    J.bc = bc;
    J.ac = ac;
    J.xi = xi;
    J.yi = yi;
    J.gx = gx;
    J.gb = gb;
    J.ga = ga;
    J.gxi = gxi;
    J.gyi = gyi;
    J.backward = 1;
    return dispatch(&J, nthreads);
}
