/*
 * ccoracle.c -- serial FP64 CPU reference for the regularised correlation-
 * clustering LP (test infrastructure only).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code with the GPU library: it is a
 * plain, slow, serial statement of the method, used to check the GPU path.
 *
 * What it computes (paper, Sec. II-B and Sec. III):
 *   problem (mn1):  min sum_p w_p f_p
 *                   s.t. x_ij <= x_ik + x_jk       for every triplet, all
 *                                                  three orientations,
 *                        x_p - d_p <= f_p,  d_p - x_p <= f_p   per pair;
 *   regularised (qp): min c'v + (eps/2) v'Wv  s.t. Av <= b, with v = (x, f),
 *                   c = (0, w), W = diag(w) on both x and f, gamma = 1/eps;
 *   Algorithm 1 (Dykstra = Hildreth): the constraints are visited
 *                   cyclically, and a visit makes the exact best move of
 *                   that constraint's dual in the dual of (qp) (visit_row);
 *   visiting order: the tiled block-diagonal schedule of Sec. III-B/C.
 * Other visiting orders (Sec. IV-E: the order changes the iteration count,
 * not the limit): plain lexicographic order, and the sum-mod-n colouring
 * (the colouring view of the related-work section: triplets that share a
 * pair conflict; colour t = every triplet with i + j + k = t (mod n), in
 * which a pair fixes the third index, so no two triplets of a colour share
 * a pair), colours t = 0..n-1 in turn.
 * Also the l2 metric nearness problem (Sec. II-A, p = 2) on the same metric
 * rows and schedule, at the end of this file, and the l1 metric nearness
 * problem, which is (mn1) itself with real dissimilarities d in place of
 * the 0/1 ones of correlation clustering (orc_l1_*).
 *
 * Schedule (Sec. III-B/C; the reading of its unspecified parts is stated in
 * the design notes):  indices 0..n-1 are cut into aligned blocks of size b,
 * nb = ceil(n/b).  Tile (P,Q), P <= Q, holds every triplet i<j<k with i in
 * block P and k in block Q (a b x b group of the sets S_{i,k}).  Rounds are
 * the block anti-diagonals s = P+Q, taken in the order s = nb-1, nb-2, ..., 0
 * and then s = nb, ..., 2nb-2 (the two double loops of Fig. 2); tiles of a
 * round go by ascending P.  Inside a tile the middle block J runs from Q down
 * to P in the rounds of the first loop (s < nb) and from P up to Q in those
 * of the second loop (s >= nb); inside
 * a (tile, J) cube the sub-steps t = 0..b-1 each take, for every local pair
 * (il, kl) in row-major order, the middle index with local offset
 * jl = (t - il - kl) mod b, so that il + jl + kl = t (mod b).  A triplet is
 * visited if i < j < k < n.  Per triplet the orientations are visited in the
 * order o = 0: x_ij <= x_ik + x_jk, o = 1: x_ik <= x_ij + x_jk,
 * o = 2: x_jk <= x_ij + x_ik.  Per sweep: every metric round, then every pair
 * in packed order with its constraint x - f <= d before -x - f <= -d.
 *
 * Layouts:  pairs in packed column-major order p(i,j) = j(j-1)/2 + i (i<j);
 * metric duals in colex triplet order y[3 t + o], t = C(k,3) + C(j,2) + i;
 * pair duals y_pair[2 p + c], c = 0 for x - f <= d, c = 1 for -x - f <= -d.
 *
 * Parity pins for every function here are in the test suite; none of them
 * is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t pidx(int64_t i, int64_t j) { return j * (j - 1) / 2 + i; }
static int64_t tidx(int64_t i, int64_t j, int64_t k)
{
    return k * (k - 1) * (k - 2) / 6 + j * (j - 1) / 2 + i;
}

int64_t orc_num_pairs(int64_t n) { return n * (n - 1) / 2; }
int64_t orc_num_triplets(int64_t n) { return n * (n - 1) * (n - 2) / 6; }

/* ------------------------------------------------------------------------ */
/* The schedule as a visitor: calls fn(ctx, i, j, k, round, tile_P, J, t)    */
/* for every triplet in visiting order; stops after max_rounds rounds        */
/* (max_rounds < 0: all).                                                    */
/* ------------------------------------------------------------------------ */
typedef void (*visit_fn)(void *ctx, int64_t i, int64_t j, int64_t k,
                         int64_t round, int64_t P, int64_t J, int64_t t);

static void visit_schedule(int64_t n, int64_t b, int64_t max_rounds,
                           visit_fn fn, void *ctx)
{
    int64_t nb = (n + b - 1) / b;
    int64_t nrounds = 2 * nb - 1;
    if (max_rounds < 0 || max_rounds > nrounds) max_rounds = nrounds;
    for (int64_t r = 0; r < max_rounds; r++) {
        /* first nb rounds: anti-diagonals nb-1 down to 0; then nb .. 2nb-2 */
        int64_t s = (r < nb) ? (nb - 1 - r) : r;
        for (int64_t P = 0; 2 * P <= s; P++) {
            int64_t Q = s - P;
            if (Q >= nb) continue;
            /* middle blocks: descending in the first loop's rounds,
             * ascending in the second loop's */
            for (int64_t m = 0; m <= Q - P; m++) {
                int64_t J = (s < nb) ? Q - m : P + m;
                for (int64_t t = 0; t < b; t++)
                    for (int64_t il = 0; il < b; il++)
                        for (int64_t kl = 0; kl < b; kl++) {
                            int64_t jl = ((t - il - kl) % b + b) % b;
                            int64_t i = P * b + il, j = J * b + jl, k = Q * b + kl;
                            if (i < j && j < k && k < n)
                                fn(ctx, i, j, k, r, P, J, t);
                        }
            }
        }
    }
}

/* Plain lexicographic order (i, then j, then k ascending): a second fixed
 * order, used only to check that the limit does not depend on the order. */
static void visit_lex(int64_t n, visit_fn fn, void *ctx)
{
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i + 1; j < n; j++)
            for (int64_t k = j + 1; k < n; k++)
                fn(ctx, i, j, k, 0, 0, 0, 0);
}

/* Sum-mod-n colouring: colours t = 0, 1, ..., n-1 in turn; inside a colour
 * the triplets go by (i, j) lexicographically, the third index being
 * k = (t - i - j) mod n, taken when k > j (so each triplet is visited once,
 * from its two smallest indices).  The triplets of a colour share no pair,
 * so their order inside the colour cannot change the result. */
static void visit_colour(int64_t n, visit_fn fn, void *ctx)
{
    for (int64_t t = 0; t < n; t++)
        for (int64_t i = 0; i < n; i++)
            for (int64_t j = i + 1; j < n; j++) {
                int64_t k = ((t - i - j) % n + n) % n;
                if (k > j) fn(ctx, i, j, k, t, 0, 0, 0);
            }
}

/* Enumerate the schedule into arrays (small n only, for schedule tests).
 * Each output row: i, j, k, round, P, J, t.  Returns the number of rows. */
int64_t orc_schedule(int64_t n, int64_t b, int64_t *out, int64_t cap);

struct enum_ctx { int64_t *out; int64_t cap, cnt; };
static void enum_visit(void *c, int64_t i, int64_t j, int64_t k,
                       int64_t r, int64_t P, int64_t J, int64_t t)
{
    struct enum_ctx *e = (struct enum_ctx *)c;
    if (e->cnt < e->cap) {
        int64_t *o = e->out + 7 * e->cnt;
        o[0] = i; o[1] = j; o[2] = k; o[3] = r; o[4] = P; o[5] = J; o[6] = t;
    }
    e->cnt++;
}

int64_t orc_schedule(int64_t n, int64_t b, int64_t *out, int64_t cap)
{
    struct enum_ctx e = { out, cap, 0 };
    visit_schedule(n, b, -1, enum_visit, &e);
    return e.cnt;
}

/* The colour order into arrays, rows (i, j, k, colour, 0, 0, 0). */
int64_t orc_colour_order(int64_t n, int64_t *out, int64_t cap)
{
    struct enum_ctx e = { out, cap, 0 };
    visit_colour(n, enum_visit, &e);
    return e.cnt;
}

/* ------------------------------------------------------------------------ */
/* One visit of one row (Sec. II-B, Algorithm 1).                            */
/*                                                                           */
/* A row is a'v <= beta with a sparse a (entries coef[] at the variables     */
/* *v[]) and its dual y >= 0; rinv[] holds the matching diagonal entries of  */
/* W^{-1}, and gamma = 1/eps.  The iterate always satisfies the stationarity */
/* condition v = -gamma W^{-1} (c + A'y).  Along this row's dual alone the   */
/* dual objective of (qp) is then a concave parabola: its slope at the       */
/* current y is a'v - beta (the row's violation) and its curvature is        */
/* -gamma a'W^{-1}a.  A visit moves y to the top of that parabola, kept at   */
/* or above zero, and moves v with it (v changes by -gamma W^{-1}a per unit  */
/* of y).  This is the point Algorithm 1 reaches through its two steps: the  */
/* correction adds y gamma W^{-1}a back to v, the projection onto the        */
/* halfspace takes theta gamma W^{-1}a off again, and theta is the new dual. */
/* ------------------------------------------------------------------------ */
static void visit_row(double *v[], const double coef[], const double rinv[],
                      int m, double beta, double *y, double gamma)
{
    double slope = 0.0, awa = 0.0;
    for (int e = 0; e < m; e++) {
        slope += coef[e] * (*v[e]);
        awa += coef[e] * coef[e] * rinv[e];
    }
    slope -= beta;
    /* top of the parabola, clipped to the feasible dual set y >= 0 */
    double ynew = *y + slope / (gamma * awa);
    if (!(ynew > 0.0)) ynew = 0.0;
    /* v follows: dv = -gamma W^{-1} a (ynew - y) */
    double dy = ynew - *y;
    for (int e = 0; e < m; e++)
        *v[e] -= gamma * dy * (rinv[e] * coef[e]);
    *y = ynew;
}

typedef struct {
    int64_t n;
    double gamma;
    const double *r;      /* W^{-1} diagonal per pair: 1 / w_p */
    double *x;
    double *y;            /* colex metric duals, or NULL in prefix mode */
    /* prefix mode: visit-order list of nonzero duals */
    int64_t *lst_t;
    int8_t *lst_o;
    double *lst_y;
    int64_t lst_cap, lst_cnt;
} sweep_ctx;

/* The three metric rows of triplet (i,j,k).  o selects the long side. */
static void metric_triplet(sweep_ctx *c, int64_t i, int64_t j, int64_t k)
{
    int64_t pij = pidx(i, j), pik = pidx(i, k), pjk = pidx(j, k);
    int64_t t = tidx(i, j, k);
    /* long side first, then the two short sides */
    const int64_t sides[3][3] = { { pij, pik, pjk }, { pik, pij, pjk }, { pjk, pij, pik } };
    const double coef[3] = { 1.0, -1.0, -1.0 };
    for (int o = 0; o < 3; o++) {
        double *v[3];
        double rinv[3];
        for (int e = 0; e < 3; e++) {
            v[e] = &c->x[sides[o][e]];
            rinv[e] = c->r[sides[o][e]];
        }
        if (c->y) {
            visit_row(v, coef, rinv, 3, 0.0, &c->y[3 * t + o], c->gamma);
        } else {
            /* prefix mode: every dual is 0 before its first visit */
            double yv = 0.0;
            visit_row(v, coef, rinv, 3, 0.0, &yv, c->gamma);
            if (yv != 0.0 && c->lst_cnt < c->lst_cap) {
                c->lst_t[c->lst_cnt] = t;
                c->lst_o[c->lst_cnt] = (int8_t)o;
                c->lst_y[c->lst_cnt] = yv;
            }
            if (yv != 0.0) c->lst_cnt++;
        }
    }
}

static void metric_visit(void *cv, int64_t i, int64_t j, int64_t k,
                         int64_t r, int64_t P, int64_t J, int64_t t)
{
    (void)r; (void)P; (void)J; (void)t;
    metric_triplet((sweep_ctx *)cv, i, j, k);
}

/* Pair constraints of (mn1): x_p - f_p <= d_p and -x_p - f_p <= -d_p. */
static void pair_pass(int64_t np, double gamma, const double *r, const uint8_t *d,
                      double *x, double *f, double *y_pair)
{
    for (int64_t p = 0; p < np; p++) {
        double *v[2] = { &x[p], &f[p] };
        double rinv[2] = { r[p], r[p] };
        const double c1[2] = { 1.0, -1.0 };
        const double c2[2] = { -1.0, -1.0 };
        visit_row(v, c1, rinv, 2, (double)d[p], &y_pair[2 * p], gamma);
        visit_row(v, c2, rinv, 2, -(double)d[p], &y_pair[2 * p + 1], gamma);
    }
}

/* The same pair rows for real d (l1 metric nearness). */
static void pair_pass_real(int64_t np, double gamma, const double *r, const double *dd,
                           double *x, double *f, double *y_pair)
{
    for (int64_t p = 0; p < np; p++) {
        double *v[2] = { &x[p], &f[p] };
        double rinv[2] = { r[p], r[p] };
        const double c1[2] = { 1.0, -1.0 };
        const double c2[2] = { -1.0, -1.0 };
        visit_row(v, c1, rinv, 2, dd[p], &y_pair[2 * p], gamma);
        visit_row(v, c2, rinv, 2, -dd[p], &y_pair[2 * p + 1], gamma);
    }
}

static double *inverse_weights(int64_t np, const double *w)
{
    double *r = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    if (!r) return NULL;
    for (int64_t p = 0; p < np; p++) r[p] = 1.0 / w[p];
    return r;
}

/* Starting point of Algorithm 1: y = 0 and v = -(1/eps) W^{-1} c with
 * c = (0 on x, w on f), i.e. x = 0 and f = -gamma. */
void orc_init_cold(int64_t n, double gamma, const double *w, double *x, double *f,
                   double *y, double *y_pair)
{
    int64_t np = orc_num_pairs(n);
    for (int64_t p = 0; p < np; p++) {
        x[p] = 0.0;                       /* c is 0 on the x block */
        f[p] = -gamma * (w[p] / w[p]);    /* c_f = w on the f block */
        y_pair[2 * p] = 0.0;
        y_pair[2 * p + 1] = 0.0;
    }
    if (y) memset(y, 0, (size_t)(3 * orc_num_triplets(n)) * sizeof(double));
}

/* nsweeps full sweeps.  order 0: the tiled schedule with tile size b;
 * order 1: plain lexicographic order; order 2: the sum-mod-n colouring.
 * Returns 0, or -1 on bad input. */
int orc_sweeps(int64_t n, int64_t b, double gamma, const double *w, const uint8_t *d,
               double *x, double *f, double *y, double *y_pair, int32_t nsweeps,
               int32_t order)
{
    if (n < 2 || b < 1 || !(gamma > 0.0)) return -1;
    int64_t np = orc_num_pairs(n);
    double *r = inverse_weights(np, w);
    if (!r) return -1;
    sweep_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n; c.gamma = gamma; c.r = r; c.x = x; c.y = y;
    for (int32_t s = 0; s < nsweeps; s++) {
        if (n >= 3) {
            if (order == 0) visit_schedule(n, b, -1, metric_visit, &c);
            else if (order == 1) visit_lex(n, metric_visit, &c);
            else visit_colour(n, metric_visit, &c);
        }
        pair_pass(np, gamma, r, d, x, f, y_pair);
    }
    free(r);
    return 0;
}

/* nsweeps sweeps that visit the given triplets (count rows i, j, k with
 * i < j < k < n) in the given order, then the pair pass.  For checks that
 * the result depends only on the order of conflicting triplets. */
int orc_sweeps_list(int64_t n, double gamma, const double *w, const uint8_t *d, double *x,
                    double *f, double *y, double *y_pair, int32_t nsweeps,
                    const int64_t *trip, int64_t count)
{
    if (n < 2 || !(gamma > 0.0)) return -1;
    for (int64_t e = 0; e < count; e++)
        if (!(0 <= trip[3 * e] && trip[3 * e] < trip[3 * e + 1] &&
              trip[3 * e + 1] < trip[3 * e + 2] && trip[3 * e + 2] < n))
            return -1;
    int64_t np = orc_num_pairs(n);
    double *r = inverse_weights(np, w);
    if (!r) return -1;
    sweep_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n; c.gamma = gamma; c.r = r; c.x = x; c.y = y;
    for (int32_t s = 0; s < nsweeps; s++) {
        for (int64_t e = 0; e < count; e++)
            metric_visit(&c, trip[3 * e], trip[3 * e + 1], trip[3 * e + 2], 0, 0, 0, 0);
        pair_pass(np, gamma, r, d, x, f, y_pair);
    }
    free(r);
    return 0;
}

/* The pair constraints alone, once (the tail of a sweep). */
int orc_pair_pass(int64_t n, double gamma, const double *w, const uint8_t *d,
                  double *x, double *f, double *y_pair)
{
    int64_t np = orc_num_pairs(n);
    double *r = inverse_weights(np, w);
    if (!r) return -1;
    pair_pass(np, gamma, r, d, x, f, y_pair);
    free(r);
    return 0;
}

/* The first max_rounds metric rounds of a sweep that starts with every
 * metric dual at zero (true for the second sweep after a cold start: at
 * x = 0 every metric row holds with equality, so the first sweep leaves all
 * metric duals at zero).  No dense dual storage: nonzero duals are appended
 * in visiting order to (lst_t, lst_o, lst_y) -- the serial sparse dual list
 * of Sec. III-D.  x is updated in place.  Returns the number of nonzero
 * duals (which may exceed cap; only cap are written), or -1. */
int64_t orc_round_prefix(int64_t n, int64_t b, double gamma, const double *w,
                         double *x, int64_t max_rounds, int64_t *lst_t, int8_t *lst_o,
                         double *lst_y, int64_t cap)
{
    int64_t np = orc_num_pairs(n);
    double *r = inverse_weights(np, w);
    if (!r) return -1;
    sweep_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n; c.gamma = gamma; c.r = r; c.x = x; c.y = NULL;
    c.lst_t = lst_t; c.lst_o = lst_o; c.lst_y = lst_y; c.lst_cap = cap;
    visit_schedule(n, b, max_rounds, metric_visit, &c);
    free(r);
    return c.lst_cnt;
}

/* ------------------------------------------------------------------------ */
/* A'y, the point v(y) = -gamma W^{-1} (c + A'y) it defines (the stationarity */
/* condition c + eps W v + A'y = 0), and convergence measures.               */
/* ------------------------------------------------------------------------ */

/* aty_x[p], aty_f[p] = the x_p and f_p components of A'y. */
static void accumulate_aty(int64_t n, const double *y, const double *y_pair,
                           double *aty_x, double *aty_f)
{
    int64_t np = orc_num_pairs(n);
    for (int64_t p = 0; p < np; p++) {
        aty_x[p] = y_pair[2 * p] - y_pair[2 * p + 1];
        aty_f[p] = -y_pair[2 * p] - y_pair[2 * p + 1];
    }
    if (!y) return;
    for (int64_t k = 2; k < n; k++)
        for (int64_t j = 1; j < k; j++)
            for (int64_t i = 0; i < j; i++) {
                int64_t t = tidx(i, j, k);
                int64_t pij = pidx(i, j), pik = pidx(i, k), pjk = pidx(j, k);
                double y0 = y[3 * t], y1 = y[3 * t + 1], y2 = y[3 * t + 2];
                aty_x[pij] += y0 - y1 - y2;
                aty_x[pik] += y1 - y0 - y2;
                aty_x[pjk] += y2 - y0 - y1;
            }
}

/* x = -gamma W^{-1} (c + A'y) on both blocks of v. */
int orc_x_from_y(int64_t n, double gamma, const double *w, const double *y,
                 const double *y_pair, double *x, double *f)
{
    int64_t np = orc_num_pairs(n);
    double *ax = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    double *af = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    if (!ax || !af) { free(ax); free(af); return -1; }
    accumulate_aty(n, y, y_pair, ax, af);
    for (int64_t p = 0; p < np; p++) {
        x[p] = -gamma * (0.0 + ax[p]) / w[p];
        f[p] = -gamma * (w[p] + af[p]) / w[p];
    }
    free(ax); free(af);
    return 0;
}

typedef struct {
    double max_viol_metric;  /* max over metric rows of (a'x - b)^+          */
    double max_viol_pair;    /* max over pair rows of (a'v - b)^+            */
    double primal_qp;        /* c'v + (eps/2) v'Wv                           */
    double dual_qp;          /* -b'y - (1/(2 eps)) (c+A'y)' W^{-1} (c+A'y)   */
    double gap;              /* primal_qp - dual_qp                          */
    double lp_cost;          /* sum_p w_p |x_p - d_p|: LP objective at x     */
    double cs_max;           /* max over rows of |y (b - a'v)|               */
    double stat_resid;       /* max |v - v(y)|                               */
} orc_resid;

static double dmax(double a, double b) { return a > b ? a : b; }

static int residuals_real(int64_t n, double gamma, const double *w, const double *dd,
                          const double *x, const double *f, const double *y,
                          const double *y_pair, orc_resid *out)
{
    int64_t np = orc_num_pairs(n);
    memset(out, 0, sizeof(*out));
    double *ax = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    double *af = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    if (!ax || !af) { free(ax); free(af); return -1; }
    accumulate_aty(n, y, y_pair, ax, af);

    double primal = 0.0, lp = 0.0, quad_dual = 0.0, by = 0.0;
    double vpair = 0.0, cs = 0.0, stat = 0.0;
    for (int64_t p = 0; p < np; p++) {
        double dp = dd[p];
        primal += w[p] * f[p] + (w[p] * (x[p] * x[p] + f[p] * f[p])) / (2.0 * gamma);
        lp += w[p] * fabs(x[p] - dp);
        double s1 = dp - (x[p] - f[p]);      /* slack of  x - f <= d  */
        double s2 = -dp - (-x[p] - f[p]);    /* slack of -x - f <= -d */
        vpair = dmax(vpair, dmax(-s1, -s2));
        cs = dmax(cs, dmax(fabs(y_pair[2 * p] * s1), fabs(y_pair[2 * p + 1] * s2)));
        by += dp * y_pair[2 * p] - dp * y_pair[2 * p + 1];
        double gx = 0.0 + ax[p], gf = w[p] + af[p];
        quad_dual += (gx * gx + gf * gf) / w[p];
        stat = dmax(stat, fabs(x[p] - (-gamma * gx / w[p])));
        stat = dmax(stat, fabs(f[p] - (-gamma * gf / w[p])));
    }
    double vmet = 0.0;
    for (int64_t k = 2; k < n; k++)
        for (int64_t j = 1; j < k; j++)
            for (int64_t i = 0; i < j; i++) {
                double xij = x[pidx(i, j)], xik = x[pidx(i, k)], xjk = x[pidx(j, k)];
                double s[3] = { xik + xjk - xij, xij + xjk - xik, xij + xik - xjk };
                for (int o = 0; o < 3; o++) {
                    vmet = dmax(vmet, -s[o]);
                    if (y) cs = dmax(cs, fabs(y[3 * tidx(i, j, k) + o] * s[o]));
                }
            }
    out->max_viol_metric = vmet;
    out->max_viol_pair = vpair;
    out->primal_qp = primal;
    out->dual_qp = -by - 0.5 * gamma * quad_dual;
    out->gap = out->primal_qp - out->dual_qp;
    out->lp_cost = lp;
    out->cs_max = cs;
    out->stat_resid = stat;
    free(ax); free(af);
    return 0;
}

/* Residuals of (mn1)/(qp) for 0/1 d (correlation clustering): d as doubles
 * (exact), then the same evaluation. */
int orc_residuals(int64_t n, double gamma, const double *w, const uint8_t *d,
                  const double *x, const double *f, const double *y,
                  const double *y_pair, orc_resid *out)
{
    int64_t np = orc_num_pairs(n);
    double *dd = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    if (!dd) return -1;
    for (int64_t p = 0; p < np; p++) dd[p] = (double)d[p];
    int rc = residuals_real(n, gamma, w, dd, x, f, y, y_pair, out);
    free(dd);
    return rc;
}

/* l1 metric nearness: nsweeps sweeps of (qp) with real d (orders as in
 * orc_sweeps), and its residuals; the starting point is orc_init_cold's,
 * and x(y) is orc_x_from_y's (neither depends on d). */
int orc_l1_sweeps(int64_t n, int64_t b, double gamma, const double *w, const double *dd,
                  double *x, double *f, double *y, double *y_pair, int32_t nsweeps,
                  int32_t order)
{
    if (n < 2 || b < 1 || !(gamma > 0.0)) return -1;
    int64_t np = orc_num_pairs(n);
    double *r = inverse_weights(np, w);
    if (!r) return -1;
    sweep_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n; c.gamma = gamma; c.r = r; c.x = x; c.y = y;
    for (int32_t s = 0; s < nsweeps; s++) {
        if (n >= 3) {
            if (order == 0) visit_schedule(n, b, -1, metric_visit, &c);
            else if (order == 1) visit_lex(n, metric_visit, &c);
            else visit_colour(n, metric_visit, &c);
        }
        pair_pass_real(np, gamma, r, dd, x, f, y_pair);
    }
    free(r);
    return 0;
}

int orc_l1_residuals(int64_t n, double gamma, const double *w, const double *dd,
                     const double *x, const double *f, const double *y,
                     const double *y_pair, orc_resid *out)
{
    return residuals_real(n, gamma, w, dd, x, f, y, y_pair, out);
}

/* Dual objective D(y) alone (used for the monotonicity check). */
double orc_dual_objective(int64_t n, double gamma, const double *w, const uint8_t *d,
                          const double *y, const double *y_pair)
{
    int64_t np = orc_num_pairs(n);
    double *ax = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    double *af = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    if (!ax || !af) { free(ax); free(af); return NAN; }
    accumulate_aty(n, y, y_pair, ax, af);
    double by = 0.0, q = 0.0;
    for (int64_t p = 0; p < np; p++) {
        double dp = (double)d[p];
        by += dp * y_pair[2 * p] - dp * y_pair[2 * p + 1];
        double gx = ax[p], gf = w[p] + af[p];
        q += (gx * gx + gf * gf) / w[p];
    }
    free(ax); free(af);
    return -by - 0.5 * gamma * q;
}

/* ------------------------------------------------------------------------ */
/* l2 metric nearness (Sec. II-A, the metric nearness problem with p = 2):  */
/*   min (1/2) sum_p w_p (x_p - d_p)^2   s.t.  x_ij <= x_ik + x_jk          */
/* for real dissimilarities d_p.  It is (qp) with v = x alone, W = diag(w), */
/* eps = 1 and c = -W d (so c'x + (1/2) x'Wx differs from the objective by  */
/* the constant (1/2) d'Wd), and A the metric rows only, b = 0.             */
/* Algorithm 1 then starts from x = -(1/eps) W^{-1} c = d with y = 0, and a */
/* sweep is the metric rounds of the schedule alone: no pair rows.          */
/* Dual:  D(y) = d'A'y - (1/2) (A'y)' W^{-1} (A'y), stationarity            */
/* x = d - W^{-1} A'y; both differ from (qp)'s by the same constant.        */
/* ------------------------------------------------------------------------ */
void orc_nearness_init(int64_t n, const double *dv, double *x, double *y)
{
    int64_t np = orc_num_pairs(n);
    for (int64_t p = 0; p < np; p++) x[p] = dv[p];
    if (y) memset(y, 0, (size_t)(3 * orc_num_triplets(n)) * sizeof(double));
}

/* nsweeps sweeps (order 0: tiled schedule with tile size b; 1: plain
 * lexicographic order; 2: the sum-mod-n colouring).  Returns 0, or -1 on
 * bad input. */
int orc_nearness_sweeps(int64_t n, int64_t b, const double *w, double *x, double *y,
                        int32_t nsweeps, int32_t order)
{
    if (n < 2 || b < 1 || !y) return -1;
    int64_t np = orc_num_pairs(n);
    double *r = inverse_weights(np, w);
    if (!r) return -1;
    sweep_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n; c.gamma = 1.0; c.r = r; c.x = x; c.y = y;
    for (int32_t s = 0; s < nsweeps && n >= 3; s++) {
        if (order == 0) visit_schedule(n, b, -1, metric_visit, &c);
        else if (order == 1) visit_lex(n, metric_visit, &c);
        else visit_colour(n, metric_visit, &c);
    }
    free(r);
    return 0;
}

typedef struct {
    double max_viol;    /* max over metric rows of (a'x)^+                  */
    double primal;      /* (1/2) sum_p w_p (x_p - d_p)^2                    */
    double dual;        /* d'A'y - (1/2) (A'y)' W^{-1} (A'y)                */
    double gap;         /* primal - dual                                    */
    double cs_max;      /* max over rows of |y (0 - a'x)|                   */
    double stat_resid;  /* max |x - (d - W^{-1} A'y)|                       */
} orc_nres;

int orc_nearness_residuals(int64_t n, const double *w, const double *dv, const double *x,
                           const double *y, orc_nres *out)
{
    int64_t np = orc_num_pairs(n);
    memset(out, 0, sizeof(*out));
    double *ax = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    double *af = (double *)malloc((size_t)(np > 0 ? np : 1) * sizeof(double));
    double *yp0 = (double *)calloc((size_t)(np > 0 ? 2 * np : 1), sizeof(double));
    if (!ax || !af || !yp0) { free(ax); free(af); free(yp0); return -1; }
    accumulate_aty(n, y, yp0, ax, af);   /* no pair rows: their duals are 0 */
    double primal = 0.0, dual_lin = 0.0, dual_quad = 0.0, stat = 0.0;
    for (int64_t p = 0; p < np; p++) {
        double e = x[p] - dv[p];
        primal += 0.5 * w[p] * e * e;
        dual_lin += dv[p] * ax[p];
        dual_quad += ax[p] * ax[p] / w[p];
        stat = dmax(stat, fabs(x[p] - (dv[p] - ax[p] / w[p])));
    }
    double vmet = 0.0, cs = 0.0;
    for (int64_t k = 2; k < n; k++)
        for (int64_t j = 1; j < k; j++)
            for (int64_t i = 0; i < j; i++) {
                double xij = x[pidx(i, j)], xik = x[pidx(i, k)], xjk = x[pidx(j, k)];
                double s[3] = { xik + xjk - xij, xij + xjk - xik, xij + xik - xjk };
                for (int o = 0; o < 3; o++) {
                    vmet = dmax(vmet, -s[o]);
                    if (y) cs = dmax(cs, fabs(y[3 * tidx(i, j, k) + o] * s[o]));
                }
            }
    out->max_viol = vmet;
    out->primal = primal;
    out->dual = dual_lin - 0.5 * dual_quad;
    out->gap = out->primal - out->dual;
    out->cs_max = cs;
    out->stat_resid = stat;
    free(ax); free(af); free(yp0);
    return 0;
}
