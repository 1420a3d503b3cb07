/*
 * Stencil oracle: plain, slow, FP64 reference of the explicit stencil sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library.
 *
 * What it computes (paper, Introduction: every grid point is replaced by a
 * weighted sum of its neighbours in a fixed pattern, characterised by shape,
 * radius r and dimensionality d; box = all points of the hyper-rectangle of
 * radius r, star = points on the coordinate axes; Sec. "Original Stencil
 * Problem": K points, one multiply-add per point):
 *
 *     u'[x] = sum_{o in O} w[o] * ext(u)[x + o]
 *
 * O_box  = [-r, r]^d                    (K = (2r+1)^d)
 * O_star = {0} u {+-k e_i : 1 <= k <= r} (K = 2dr + 1)
 *
 * ext(u)[y] = u[y] inside the grid; outside it is the fixed halo value h
 * (Dirichlet) or u[y mod n] (periodic).  Steps are explicit and out of place:
 * step s reads only the result of step s-1.  N steps give step^N(u0).
 *
 * Canonical offset order (also the order of the weight vector and of the
 * summation):
 *   box : row-major over (o_0, ..., o_{d-1}), each in [-r, r], o_{d-1} fastest
 *   star: centre, then axis 0 offsets -r..-1, +1..+r, then axis 1, ...
 *
 * Arithmetic: float64, multiply then add as separate roundings (the build
 * uses -ffp-contract=off), summation in canonical order starting from 0.0.
 *
 * Window evaluation: oracle_run_window returns step^N(u0) on a sub-box
 * [lo, hi) of the grid.  It evaluates step s only on the points the window
 * depends on (the window grown by r*(N-s) per side, clipped to the grid for
 * Dirichlet, wrapped for periodic).  Each evaluated point uses exactly the
 * same arithmetic as the full-grid loop, so the values are bit-identical.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAXD 3

enum { ORACLE_STAR = 0, ORACLE_BOX = 1 };
enum { ORACLE_DIRICHLET = 0, ORACLE_PERIODIC = 1 };

/* Writes the K offsets (K*d ints, canonical order) and returns K, or -1. */
int oracle_offsets(int shape, int d, int r, int *offs)
{
    if (d < 1 || d > ORACLE_MAXD || r < 0) return -1;
    int K = 0;
    if (shape == ORACLE_BOX) {
        int side = 2 * r + 1;
        int total = 1;
        for (int i = 0; i < d; ++i) total *= side;
        for (int idx = 0; idx < total; ++idx) {
            int rem = idx;
            /* last axis fastest */
            for (int ax = d - 1; ax >= 0; --ax) {
                if (offs) offs[K * d + ax] = (rem % side) - r;
                rem /= side;
            }
            ++K;
        }
        return K;
    }
    if (shape == ORACLE_STAR) {
        if (offs) for (int ax = 0; ax < d; ++ax) offs[ax] = 0;
        K = 1;
        for (int ax = 0; ax < d; ++ax) {
            for (int k = -r; k <= r; ++k) {
                if (k == 0) continue;
                if (offs) {
                    for (int b = 0; b < d; ++b) offs[K * d + b] = 0;
                    offs[K * d + ax] = k;
                }
                ++K;
            }
        }
        return K;
    }
    return -1;
}

/* A rectangular set of points of one intermediate field.  Per axis it holds
 * len consecutive coordinates starting at start (wrapping modulo n for the
 * periodic boundary). */
typedef struct {
    int64_t start[ORACLE_MAXD];
    int64_t len[ORACLE_MAXD];
} region_t;

static int64_t region_size(const region_t *g, int d)
{
    int64_t s = 1;
    for (int i = 0; i < d; ++i) s *= g->len[i];
    return s;
}

/* Region the window [lo, hi) needs at a distance of `grow` points. */
static void grown_region(region_t *g, int d, const int64_t *dims, const int64_t *lo,
                         const int64_t *hi, int64_t grow, int boundary)
{
    for (int i = 0; i < d; ++i) {
        int64_t a = lo[i] - grow, b = hi[i] + grow;
        if (boundary == ORACLE_DIRICHLET) {
            if (a < 0) a = 0;
            if (b > dims[i]) b = dims[i];
            g->start[i] = a;
            g->len[i] = b - a;
        } else {
            if (b - a >= dims[i]) {
                g->start[i] = 0;
                g->len[i] = dims[i];
            } else {
                g->start[i] = ((a % dims[i]) + dims[i]) % dims[i];
                g->len[i] = b - a;
            }
        }
    }
}

/* ext(u)[y] for a field stored over region g.  y is a global coordinate that
 * may lie outside the grid. */
static double ext_value(const double *u, const region_t *g, int d, const int64_t *dims,
                        const int64_t *y, int boundary, double h)
{
    int64_t lin = 0;
    for (int i = 0; i < d; ++i) {
        int64_t yi = y[i];
        int64_t idx;
        if (boundary == ORACLE_DIRICHLET) {
            if (yi < 0 || yi >= dims[i]) return h;
            idx = yi - g->start[i];
        } else {
            idx = (((yi - g->start[i]) % dims[i]) + dims[i]) % dims[i];
        }
        lin = lin * g->len[i] + idx;
    }
    return u[lin];
}

static void one_step(int d, const int64_t *dims, int K, const int *offs, const double *w,
                     int boundary, double h, const double *src, const region_t *gs,
                     double *dst, const region_t *gd)
{
    int64_t n0 = gd->len[0];
    int64_t inner = 1;
    for (int i = 1; i < d; ++i) inner *= gd->len[i];
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n0; ++a) {
        int64_t x[ORACLE_MAXD], y[ORACLE_MAXD];
        for (int64_t q = 0; q < inner; ++q) {
            /* coordinates of this output point */
            int64_t rem = q;
            for (int i = d - 1; i >= 1; --i) {
                int64_t c = rem % gd->len[i];
                rem /= gd->len[i];
                x[i] = gd->start[i] + c;
            }
            x[0] = gd->start[0] + a;
            double acc = 0.0;
            for (int k = 0; k < K; ++k) {
                for (int i = 0; i < d; ++i) y[i] = x[i] + offs[k * d + i];
                double v = ext_value(src, gs, d, dims, y, boundary, h);
                double p = w[k] * v;
                acc = acc + p;
            }
            dst[a * inner + q] = acc;
        }
    }
}

/*
 * step^steps(u0) on the window [lo, hi).  Returns 0 on success, a negative
 * value on invalid arguments or allocation failure.  `out` holds
 * prod(hi - lo) values in row-major order.  nthreads <= 0 keeps the OpenMP
 * default.
 */
int oracle_run_window(int shape, int d, int r, const double *w, const int64_t *dims,
                      int boundary, double h, int64_t steps, const double *u0,
                      const int64_t *lo, const int64_t *hi, double *out, int nthreads)
{
    if (d < 1 || d > ORACLE_MAXD || r < 0 || steps < 0) return -1;
    for (int i = 0; i < d; ++i)
        if (dims[i] < 1 || lo[i] < 0 || hi[i] > dims[i] || lo[i] >= hi[i]) return -2;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int K = oracle_offsets(shape, d, r, NULL);
    if (K < 1) return -3;
    int *offs = (int *)malloc((size_t)K * d * sizeof(int));
    if (!offs) return -4;
    oracle_offsets(shape, d, r, offs);

    region_t full;
    memset(&full, 0, sizeof full);
    for (int i = 0; i < d; ++i) { full.start[i] = 0; full.len[i] = dims[i]; }

    region_t gcur = full;
    const double *cur = u0;
    double *buf[2] = {NULL, NULL};
    int which = 0;
    for (int64_t s = 1; s <= steps; ++s) {
        region_t gnext;
        grown_region(&gnext, d, dims, lo, hi, (int64_t)r * (steps - s), boundary);
        int64_t sz = region_size(&gnext, d);
        free(buf[which]);
        buf[which] = (double *)malloc((size_t)sz * sizeof(double));
        if (!buf[which]) { free(buf[0]); free(buf[1]); free(offs); return -4; }
        one_step(d, dims, K, offs, w, boundary, h, cur, &gcur, buf[which], &gnext);
        cur = buf[which];
        gcur = gnext;
        which ^= 1;
    }
    /* copy the window out of the last field */
    region_t gw;
    memset(&gw, 0, sizeof gw);
    for (int i = 0; i < d; ++i) { gw.start[i] = lo[i]; gw.len[i] = hi[i] - lo[i]; }
    int64_t nw = region_size(&gw, d);
    for (int64_t q = 0; q < nw; ++q) {
        int64_t y[ORACLE_MAXD];
        int64_t rem = q;
        for (int i = d - 1; i >= 0; --i) {
            y[i] = gw.start[i] + rem % gw.len[i];
            rem /= gw.len[i];
        }
        out[q] = ext_value(cur, &gcur, d, dims, y, boundary, h);
    }
    free(buf[0]);
    free(buf[1]);
    free(offs);
    return 0;
}

/* step^steps(u0) on the whole grid. */
int oracle_run(int shape, int d, int r, const double *w, const int64_t *dims, int boundary,
               double h, int64_t steps, const double *u0, double *out, int nthreads)
{
    int64_t lo[ORACLE_MAXD] = {0, 0, 0};
    return oracle_run_window(shape, d, r, w, dims, boundary, h, steps, u0, lo, dims, out,
                             nthreads);
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
