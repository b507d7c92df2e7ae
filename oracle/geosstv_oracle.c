/*
 * FP64 oracle for the GeoSSTV P-PDS solver (Takemoto and Ono, "Geometric
 * Spatio-Spectral Total Variation for Hyperspectral Image Denoising and
 * Destriping").
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The GPU product path
 * shares no code with it and never calls it.
 *
 * Plain, slow and obviously correct on purpose: one loop per operator, the
 * generic P-PDS update (eq. (7)) applied to problem (20) block by block (the
 * same iteration that Alg. 1 spells out), double precision throughout, no
 * fusion and no blocking. OpenMP only splits the outer loop of each sweep.
 *
 * Cube layout: band-sequential, element (i, j, k) of the N1 x N2 x N3 cube
 * (vertical i, horizontal j, band k) at index (k*N1 + i)*N2 + j.
 * Multi-plane fields are stored plane after plane, each plane one cube:
 *   D x, y1, y2        : [vertical, horizontal]                    (2 planes)
 *   L y, w1, w2        : [ud_v, ud_h, lr_v, lr_h, c_v, c_h]         (6 planes)
 *                        ud = the (i+1/2, j) grid, lr = the (i, j+1/2) grid,
 *                        c = the pixel grid (i, j).
 *
 * Readings where the paper is silent (every one is listed with its reason in
 * the design notes of the repository):
 *  - D_v differences along i (vertical), D_h along j, D_s along k; the
 *    Neumann boundary of Sec. II-A gives a zero forward difference at the last
 *    index of each axis.
 *  - Condat's interpolation operators (Sec. II-D, eq. (10)-(12), defined in
 *    the cited work, not in the paper): 2- and 4-point averages of the dual
 *    edge fields onto the three grids; dual edge fields exist on interior
 *    edges only, so their entries on the last row (vertical field) and last
 *    column (horizontal field) are masked to zero on input, and the ud and lr
 *    grids likewise hold only interior edges.
 *  - Initial point: u = v, every other variable zero.
 *  - Dual step of eq. (7) taken with "+ Sigma K x'", as Alg. 1 has it.
 *  - l1-ball projection (cited fast algorithm): any exact Euclidean
 *    projection; here Michelot's active-set iteration.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int64_t ix;

#define AT(a, k, i, j) (a)[(((ix)(k) * n1 + (i)) * n2) + (j)]

/* masks m_v(i) = [i <= N1-2], m_h(j) = [j <= N2-2], m_s(k) = [k <= N3-2] */
static inline double mv(int i, int n1) { return (i >= 0 && i <= n1 - 2) ? 1.0 : 0.0; }
static inline double mh(int j, int n2) { return (j >= 0 && j <= n2 - 2) ? 1.0 : 0.0; }
static inline double ms(int k, int n3) { return (k >= 0 && k <= n3 - 2) ? 1.0 : 0.0; }

/* ---------------- forward differences, Sec. II-A (Neumann) ---------------- */

void ora_dv(int n1, int n2, int n3, const double *x, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j)
                AT(out, k, i, j) = (i <= n1 - 2) ? AT(x, k, i + 1, j) - AT(x, k, i, j) : 0.0;
}

void ora_dv_t(int n1, int n2, int n3, const double *p, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                double a = (i >= 1) ? mv(i - 1, n1) * AT(p, k, i - 1, j) : 0.0;
                double b = mv(i, n1) * AT(p, k, i, j);
                AT(out, k, i, j) = a - b;
            }
}

void ora_dh(int n1, int n2, int n3, const double *x, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j)
                AT(out, k, i, j) = (j <= n2 - 2) ? AT(x, k, i, j + 1) - AT(x, k, i, j) : 0.0;
}

void ora_dh_t(int n1, int n2, int n3, const double *p, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                double a = (j >= 1) ? mh(j - 1, n2) * AT(p, k, i, j - 1) : 0.0;
                double b = mh(j, n2) * AT(p, k, i, j);
                AT(out, k, i, j) = a - b;
            }
}

void ora_ds(int n1, int n2, int n3, const double *x, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j)
                AT(out, k, i, j) = (k <= n3 - 2) ? AT(x, k + 1, i, j) - AT(x, k, i, j) : 0.0;
}

void ora_ds_t(int n1, int n2, int n3, const double *p, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                double a = (k >= 1) ? ms(k - 1, n3) * AT(p, k - 1, i, j) : 0.0;
                double b = ms(k, n3) * AT(p, k, i, j);
                AT(out, k, i, j) = a - b;
            }
}

/* D = (D_v; D_h): R^N -> R^2N, and its adjoint. */
void ora_d(int n1, int n2, int n3, const double *x, double *out)
{
    ix N = (ix)n1 * n2 * n3;
    ora_dv(n1, n2, n3, x, out);
    ora_dh(n1, n2, n3, x, out + N);
}

static void d_t_ws(int n1, int n2, int n3, const double *p, double *out, double *tmp)
{
    ix N = (ix)n1 * n2 * n3;
    ora_dv_t(n1, n2, n3, p, out);
    ora_dh_t(n1, n2, n3, p + N, tmp);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) out[q] += tmp[q];
}

void ora_d_t(int n1, int n2, int n3, const double *p, double *out)
{
    double *tmp = (double *)malloc(sizeof(double) * (ix)n1 * n2 * n3);
    d_t_ws(n1, n2, n3, p, out, tmp);
    free(tmp);
}

/* ---------- Condat's interpolation operators, Sec. II-D and III-A ---------- */

/* masked dual edge fields: vertical field lives on rows 0..N1-2, horizontal
 * field on columns 0..N2-2; anything outside the index box reads as zero. */
static inline double yv_m(const double *yv, int n1, int n2, int k, int i, int j)
{
    if (i < 0 || i > n1 - 2 || j < 0 || j >= n2) return 0.0;
    return AT(yv, k, i, j);
}
static inline double yh_m(const double *yh, int n1, int n2, int k, int i, int j)
{
    if (j < 0 || j > n2 - 2 || i < 0 || i >= n1) return 0.0;
    return AT(yh, k, i, j);
}

/* L_ud: onto the (i+1/2, j) grid; vertical part copied, horizontal part the
 * mean of the four horizontal edges around the vertical edge. */
void ora_l_ud(int n1, int n2, int n3, const double *y, double *w)
{
    ix N = (ix)n1 * n2 * n3;
    const double *yv = y, *yh = y + N;
    double *wv = w, *wh = w + N;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                double m = mv(i, n1);
                AT(wv, k, i, j) = m * yv_m(yv, n1, n2, k, i, j);
                AT(wh, k, i, j) = m * 0.25 * (yh_m(yh, n1, n2, k, i, j) + yh_m(yh, n1, n2, k, i, j - 1)
                                            + yh_m(yh, n1, n2, k, i + 1, j) + yh_m(yh, n1, n2, k, i + 1, j - 1));
            }
}

/* L_lr: onto the (i, j+1/2) grid. */
void ora_l_lr(int n1, int n2, int n3, const double *y, double *w)
{
    ix N = (ix)n1 * n2 * n3;
    const double *yv = y, *yh = y + N;
    double *wv = w, *wh = w + N;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                double m = mh(j, n2);
                AT(wv, k, i, j) = m * 0.25 * (yv_m(yv, n1, n2, k, i, j) + yv_m(yv, n1, n2, k, i - 1, j)
                                            + yv_m(yv, n1, n2, k, i, j + 1) + yv_m(yv, n1, n2, k, i - 1, j + 1));
                AT(wh, k, i, j) = m * yh_m(yh, n1, n2, k, i, j);
            }
}

/* L_c: onto the pixel grid (i, j); mean of the two edges on either side. */
void ora_l_c(int n1, int n2, int n3, const double *y, double *w)
{
    ix N = (ix)n1 * n2 * n3;
    const double *yv = y, *yh = y + N;
    double *wv = w, *wh = w + N;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                AT(wv, k, i, j) = 0.5 * (yv_m(yv, n1, n2, k, i, j) + yv_m(yv, n1, n2, k, i - 1, j));
                AT(wh, k, i, j) = 0.5 * (yh_m(yh, n1, n2, k, i, j) + yh_m(yh, n1, n2, k, i, j - 1));
            }
}

/* Adjoints, obtained by transposing the sums above term by term. The ud and
 * lr grids keep interior edges only, so their entries outside the masks read
 * as zero. */
static inline double wud(const double *w, int n1, int n2, int k, int i, int j)
{
    if (i < 0 || i > n1 - 2 || j < 0 || j >= n2) return 0.0;
    return AT(w, k, i, j);
}
static inline double wlr(const double *w, int n1, int n2, int k, int i, int j)
{
    if (j < 0 || j > n2 - 2 || i < 0 || i >= n1) return 0.0;
    return AT(w, k, i, j);
}
static inline double wc(const double *w, int n1, int n2, int k, int i, int j)
{
    if (i < 0 || i >= n1 || j < 0 || j >= n2) return 0.0;
    return AT(w, k, i, j);
}

void ora_l_ud_t(int n1, int n2, int n3, const double *w, double *y)
{
    ix N = (ix)n1 * n2 * n3;
    const double *wv = w, *wh = w + N;
    double *yv = y, *yh = y + N;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                AT(yv, k, i, j) = mv(i, n1) * wud(wv, n1, n2, k, i, j);
                AT(yh, k, i, j) = mh(j, n2) * 0.25 * (wud(wh, n1, n2, k, i, j) + wud(wh, n1, n2, k, i, j + 1)
                                                     + wud(wh, n1, n2, k, i - 1, j) + wud(wh, n1, n2, k, i - 1, j + 1));
            }
}

void ora_l_lr_t(int n1, int n2, int n3, const double *w, double *y)
{
    ix N = (ix)n1 * n2 * n3;
    const double *wv = w, *wh = w + N;
    double *yv = y, *yh = y + N;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                AT(yv, k, i, j) = mv(i, n1) * 0.25 * (wlr(wv, n1, n2, k, i, j) + wlr(wv, n1, n2, k, i + 1, j)
                                                     + wlr(wv, n1, n2, k, i, j - 1) + wlr(wv, n1, n2, k, i + 1, j - 1));
                AT(yh, k, i, j) = mh(j, n2) * wlr(wh, n1, n2, k, i, j);
            }
}

void ora_l_c_t(int n1, int n2, int n3, const double *w, double *y)
{
    ix N = (ix)n1 * n2 * n3;
    const double *wv = w, *wh = w + N;
    double *yv = y, *yh = y + N;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n3; ++k)
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j) {
                AT(yv, k, i, j) = mv(i, n1) * 0.5 * (wc(wv, n1, n2, k, i, j) + wc(wv, n1, n2, k, i + 1, j));
                AT(yh, k, i, j) = mh(j, n2) * 0.5 * (wc(wh, n1, n2, k, i, j) + wc(wh, n1, n2, k, i, j + 1));
            }
}

/* L = (L_ud; L_lr; L_c): R^2N -> R^6N, block-diagonal over the bands
 * (Sec. III-A), and L^T = L_ud^T + L_lr^T + L_c^T. */
void ora_l(int n1, int n2, int n3, const double *y, double *w)
{
    ix N = (ix)n1 * n2 * n3;
    ora_l_ud(n1, n2, n3, y, w);
    ora_l_lr(n1, n2, n3, y, w + 2 * N);
    ora_l_c(n1, n2, n3, y, w + 4 * N);
}

static void l_t_ws(int n1, int n2, int n3, const double *w, double *y, double *a, double *b)
{
    ix N = (ix)n1 * n2 * n3;
    ora_l_ud_t(n1, n2, n3, w, y);
    ora_l_lr_t(n1, n2, n3, w + 2 * N, a);
    ora_l_c_t(n1, n2, n3, w + 4 * N, b);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < 2 * N; ++q) y[q] += a[q] + b[q];
}

void ora_l_t(int n1, int n2, int n3, const double *w, double *y)
{
    ix N = (ix)n1 * n2 * n3;
    double *a = (double *)malloc(sizeof(double) * 2 * N);
    double *b = (double *)malloc(sizeof(double) * 2 * N);
    l_t_ws(n1, n2, n3, w, y, a, b);
    free(a);
    free(b);
}

/* ------------------------------ projections ------------------------------ */

/* Box projection, eq. (21). */
void ora_proj_box(const double *x, ix n, double lo, double hi, double *out)
{
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < n; ++q) out[q] = x[q] < lo ? lo : (x[q] > hi ? hi : x[q]);
}

/* Projection onto the ball of radius eps centred at c, eq. (23). Returns the
 * distance ||x - c||_2. */
double ora_proj_l2(const double *x, const double *c, ix n, double eps, double *out)
{
    double ss = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : ss)
    for (ix q = 0; q < n; ++q) ss += (x[q] - c[q]) * (x[q] - c[q]);
    double r = sqrt(ss);
    if (r <= eps) {
        if (out != x) memcpy(out, x, sizeof(double) * n);
    } else {
        double f = eps / r;
#pragma omp parallel for schedule(static)
        for (ix q = 0; q < n; ++q) out[q] = c[q] + f * (x[q] - c[q]);
    }
    return r;
}

/* Projection onto {z : ||z||_1 <= radius} (constraint sets (16), (17); the
 * paper cites a fast exact algorithm). The result is the soft threshold
 * sign(x) max(|x| - tau, 0) with tau the root of sum max(|x| - tau, 0) =
 * radius. tau comes from Michelot's active-set iteration: start from all
 * nonzero entries, set tau to (sum of active |x| - radius) / (active count),
 * drop the entries with |x| <= tau and repeat until nothing is dropped.
 * Returns tau: 0 when x is already inside the ball, +inf for radius 0. */
double ora_proj_l1(const double *x, ix n, double radius, double *out)
{
    double tot = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : tot)
    for (ix q = 0; q < n; ++q) tot += fabs(x[q]);
    if (radius <= 0.0) {
        memset(out, 0, sizeof(double) * n);
        return INFINITY;
    }
    if (tot <= radius) {
        if (out != x) memcpy(out, x, sizeof(double) * n);
        return 0.0;
    }
    unsigned char *act = (unsigned char *)malloc(n ? n : 1);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < n; ++q) act[q] = fabs(x[q]) > 0.0;
    double tau = 0.0;
    for (;;) {
        double s = 0.0;
        ix c = 0;
#pragma omp parallel for schedule(static) reduction(+ : s, c)
        for (ix q = 0; q < n; ++q)
            if (act[q]) { s += fabs(x[q]); ++c; }
        tau = (s - radius) / (double)c;
        int dropped = 0;
#pragma omp parallel for schedule(static) reduction(| : dropped)
        for (ix q = 0; q < n; ++q)
            if (act[q] && fabs(x[q]) <= tau) { act[q] = 0; dropped = 1; }
        if (!dropped) break;
    }
    free(act);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < n; ++q) {
        double a = fabs(x[q]) - tau;
        out[q] = a > 0.0 ? copysign(a, x[q]) : 0.0;
    }
    return tau;
}

/* Prox of gamma * ||.||_{1,2}, eq. (24): each group of two entries (one
 * from plane a, one from plane b at the same index) is scaled by
 * max(1 - gamma / ||x_g||_2, 0); a group with norm <= gamma becomes zero. */
void ora_prox_l12(const double *xa, const double *xb, ix n, double gamma, double *oa, double *ob)
{
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < n; ++q) {
        double nr = sqrt(xa[q] * xa[q] + xb[q] * xb[q]);
        double f = (nr > gamma) ? 1.0 - gamma / nr : 0.0;
        oa[q] = f * xa[q];
        ob[q] = f * xb[q];
    }
}

/* --------------- P-PDS (eq. (7)) applied to problem (20) --------------- */

typedef struct {
    double eps, alpha, beta; /* radii of (18), (16), (17)              */
    double mu_lo, mu_hi;     /* box (19)                                 */
    double omega;            /* balance of GeoSSTV, eq. (13)             */
} ora_params;

/* Step sizes printed after eq. (24): the primal ones form the diagonal
 * preconditioner T = diag(G_U, G_S, G_T, G_W1, G_W2), the dual one Sigma =
 * G_Y I for all four dual blocks. */
static const double G_U = 1.0 / 13.0, G_W1 = 0.25, G_W2 = 0.25, G_S = 1.0,
                    G_T = 1.0 / 3.0, G_Y = 0.2;

/* Thread count of the OpenMP loops (tiny cubes run faster on one thread). */
void ora_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int ora_get_threads(void) { return omp_get_max_threads(); }

/* The step sizes in the order u, w1, w2, s, t, y (for the tests). */
void ora_step_sizes(double *out)
{
    out[0] = G_U; out[1] = G_W1; out[2] = G_W2; out[3] = G_S; out[4] = G_T; out[5] = G_Y;
}

/* Initial point: u = v, everything else zero. */
void ora_init(int n1, int n2, int n3, const double *v, double *u, double *s, double *t,
              double *w1, double *w2, double *y1, double *y2, double *y3, double *y4)
{
    ix N = (ix)n1 * n2 * n3;
    memcpy(u, v, sizeof(double) * N);
    memset(s, 0, sizeof(double) * N);
    memset(t, 0, sizeof(double) * N);
    memset(w1, 0, sizeof(double) * 6 * N);
    memset(w2, 0, sizeof(double) * 6 * N);
    memset(y1, 0, sizeof(double) * 2 * N);
    memset(y2, 0, sizeof(double) * 2 * N);
    memset(y3, 0, sizeof(double) * N);
    memset(y4, 0, sizeof(double) * N);
}

/* Problem (20) in the form of problem (6): five primal blocks
 * x = (u, s, t, w1, w2) with
 *   f(x) = iota_R(u) + iota_{B1,alpha}(s) + iota_{B1,beta}(t)
 *          + omega ||w1||_{1,2} + ||w2||_{1,2},
 * four dual blocks z = K x with
 *   K x = ( D u - L^T w1,  D D_s u - L^T w2,  D_v t,  u + s + t ),
 * and g(z) = iota_{0}(z1) + iota_{0}(z2) + iota_{0}(z3) + iota_{B2,eps}^v(z4). */
typedef struct { double *u, *s, *t, *w1, *w2; } primal; /* 1+1+1+6+6 planes */
typedef struct { double *y1, *y2, *y3, *y4; } dual;     /* 2+2+1+1 planes   */

/* out = K x. tmp holds 6N doubles. */
static void apply_k(int n1, int n2, int n3, const primal *x, const dual *out, double *tmp)
{
    ix N = (ix)n1 * n2 * n3;
    double *a = tmp, *b = tmp + 2 * N, *c = tmp + 4 * N;
    /* first row: D u - L^T w1 */
    ora_d(n1, n2, n3, x->u, out->y1);
    l_t_ws(n1, n2, n3, x->w1, a, b, c);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < 2 * N; ++q) out->y1[q] -= a[q];
    /* second row: D (D_s u) - L^T w2 */
    ora_ds(n1, n2, n3, x->u, c);
    ora_d(n1, n2, n3, c, out->y2);
    l_t_ws(n1, n2, n3, x->w2, a, b, c);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < 2 * N; ++q) out->y2[q] -= a[q];
    /* third row: D_v t */
    ora_dv(n1, n2, n3, x->t, out->y3);
    /* fourth row: u + s + t */
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) out->y4[q] = x->u[q] + x->s[q] + x->t[q];
}

/* out = K^T y, column by column of K. tmp holds 6N doubles. */
static void apply_kt(int n1, int n2, int n3, const dual *y, const primal *out, double *tmp)
{
    ix N = (ix)n1 * n2 * n3;
    double *a = tmp, *b = tmp + 2 * N, *c = tmp + 4 * N;
    /* u column: D^T y1 + D_s^T (D^T y2) + y4 */
    d_t_ws(n1, n2, n3, y->y1, out->u, a);
    d_t_ws(n1, n2, n3, y->y2, b, a);
    ora_ds_t(n1, n2, n3, b, c);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) out->u[q] = out->u[q] + c[q] + y->y4[q];
    /* s column: y4 */
    memcpy(out->s, y->y4, sizeof(double) * N);
    /* t column: D_v^T y3 + y4 */
    ora_dv_t(n1, n2, n3, y->y3, out->t);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) out->t[q] += y->y4[q];
    /* w1 and w2 columns: -L y1 and -L y2 */
    ora_l(n1, n2, n3, y->y1, out->w1);
    ora_l(n1, n2, n3, y->y2, out->w2);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < 6 * N; ++q) {
        out->w1[q] = -out->w1[q];
        out->w2[q] = -out->w2[q];
    }
}

/* x <- prox_{T f}(x), block by block: the box (21), the two l1 balls
 * (16), (17) and the group shrinks (24) with thresholds G_W1 omega and G_W2.
 * The l1 thresholds go to tau[0] (s) and tau[1] (t). */
static void prox_tf(int n1, int n2, int n3, const ora_params *p, const primal *x, double *tau)
{
    ix N = (ix)n1 * n2 * n3;
    ora_proj_box(x->u, N, p->mu_lo, p->mu_hi, x->u);
    tau[0] = ora_proj_l1(x->s, N, p->alpha, x->s);
    tau[1] = ora_proj_l1(x->t, N, p->beta, x->t);
    for (int g = 0; g < 3; ++g) {
        ora_prox_l12(x->w1 + 2 * g * N, x->w1 + (2 * g + 1) * N, N, G_W1 * p->omega,
                     x->w1 + 2 * g * N, x->w1 + (2 * g + 1) * N);
        ora_prox_l12(x->w2 + 2 * g * N, x->w2 + (2 * g + 1) * N, N, G_W2,
                     x->w2 + 2 * g * N, x->w2 + (2 * g + 1) * N);
    }
}

/* y <- prox_{Sigma g*}(y). The conjugate's prox comes from the Moreau
 * decomposition (3): prox_{G g*}(z) = z - G prox_{g/G}(z / G). For the three
 * iota_{0} blocks prox_{g/G} is 0 (eq. (22)), so those blocks pass through;
 * for the fourth it is the projection (23) onto B_{2,eps}^v. tmp holds 2N
 * doubles. Returns the distance ||y4/G - v||_2 that the projection tests. */
static double prox_sgstar(int n1, int n2, int n3, const ora_params *p, const double *v,
                          const dual *y, double *tmp)
{
    ix N = (ix)n1 * n2 * n3;
    double *a = tmp, *b = tmp + N;
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) a[q] = y->y4[q] / G_Y;
    double r = ora_proj_l2(a, v, N, p->eps, b);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) y->y4[q] = y->y4[q] - G_Y * b[q];
    return r;
}

/* number of doubles of scratch that one iteration needs, in units of N */
#define STEP_WS 42

/* One P-PDS iteration, eq. (7), with T and Sigma above and the dual update
 * written with "+ Sigma K x'" as Alg. 1 has it:
 *   x+ = prox_{T f}(x - T K^T y),   x' = 2 x+ - x,
 *   y+ = prox_{Sigma g*}(y + Sigma K x'). */
static void step_ws(int n1, int n2, int n3, const ora_params *p, const double *v,
                    const primal *x, const dual *y, double *trace, double *ws)
{
    ix N = (ix)n1 * n2 * n3;
    /* scratch: g (15N) holds K^T y, then x'; xn (15N) holds x+; z (6N)
     * holds K x'; tmp (6N) is operator scratch */
    double *g0 = ws, *xn0 = ws + 15 * N, *z0 = ws + 30 * N, *tmp = ws + 36 * N;
    primal g = {g0, g0 + N, g0 + 2 * N, g0 + 3 * N, g0 + 9 * N};
    primal xn = {xn0, xn0 + N, xn0 + 2 * N, xn0 + 3 * N, xn0 + 9 * N};
    dual z = {z0, z0 + 2 * N, z0 + 4 * N, z0 + 5 * N};
    const double step[5] = {G_U, G_S, G_T, G_W1, G_W2};
    const ix len[5] = {N, N, N, 6 * N, 6 * N};
    double *xb[5] = {x->u, x->s, x->t, x->w1, x->w2};
    double *gb[5] = {g.u, g.s, g.t, g.w1, g.w2};
    double *nb[5] = {xn.u, xn.s, xn.t, xn.w1, xn.w2};

    /* primal half: forward step on each block, then the block proxes */
    apply_kt(n1, n2, n3, y, &g, tmp);
    for (int b = 0; b < 5; ++b) {
        const double *xo = xb[b], *gg = gb[b];
        double *xnew = nb[b], gam = step[b];
#pragma omp parallel for schedule(static)
        for (ix q = 0; q < len[b]; ++q) xnew[q] = xo[q] - gam * gg[q];
    }
    double tau[2];
    prox_tf(n1, n2, n3, p, &xn, tau);

    /* extrapolated point x' = 2 x+ - x, kept in g */
    for (int b = 0; b < 5; ++b) {
        const double *xo = xb[b], *xnew = nb[b];
        double *xe = gb[b];
#pragma omp parallel for schedule(static)
        for (ix q = 0; q < len[b]; ++q) xe[q] = 2.0 * xnew[q] - xo[q];
    }

    /* dual half: forward step with K x', then the conjugate proxes */
    apply_k(n1, n2, n3, &g, &z, tmp);
    double *yb[4] = {y->y1, y->y2, y->y3, y->y4};
    const double *zb[4] = {z.y1, z.y2, z.y3, z.y4};
    const ix ylen[4] = {2 * N, 2 * N, N, N};
    for (int b = 0; b < 4; ++b) {
        double *yy = yb[b];
        const double *zz = zb[b];
#pragma omp parallel for schedule(static)
        for (ix q = 0; q < ylen[b]; ++q) yy[q] += G_Y * zz[q];
    }
    double r = prox_sgstar(n1, n2, n3, p, v, y, tmp);

    /* stopping quantity of eq. (28) */
    double dn = 0.0, un2 = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : dn, un2)
    for (ix q = 0; q < N; ++q) {
        dn += (xn.u[q] - x->u[q]) * (xn.u[q] - x->u[q]);
        un2 += x->u[q] * x->u[q];
    }
    double rel = un2 > 0.0 ? sqrt(dn) / sqrt(un2) : INFINITY;

    for (int b = 0; b < 5; ++b) memcpy(xb[b], nb[b], sizeof(double) * len[b]);
    if (trace) {
        trace[0] = rel;
        trace[1] = r;
        trace[2] = tau[0];
        trace[3] = tau[1];
    }
}

/* One P-PDS iteration for problem (20), updating the state in place. trace
 * (may be NULL) receives
 *   [0] ||u+ - u||_2 / ||u||_2    (stopping quantity of eq. (28); +inf when
 *                                  ||u|| = 0)
 *   [1] ||y4'/gamma - v||_2       (the distance tested in the l2 projection)
 *   [2] tau_s, [3] tau_t          (soft-threshold levels of the l1 balls)
 */
void ora_step(int n1, int n2, int n3, const ora_params *p, const double *v,
              double *u, double *s, double *t, double *w1, double *w2,
              double *y1, double *y2, double *y3, double *y4, double *trace)
{
    primal x = {u, s, t, w1, w2};
    dual y = {y1, y2, y3, y4};
    double *ws = (double *)malloc(sizeof(double) * STEP_WS * (ix)n1 * n2 * n3);
    step_ws(n1, n2, n3, p, v, &x, &y, trace, ws);
    free(ws);
}

/* Iterate: at most max_iter iterations, stopping after the first one whose
 * stopping quantity (eq. (28)) is below tol (tol <= 0: run all of them).
 * done_before: iterations made since the initial point by earlier calls.
 * The rule is not applied to the first iteration after the initial point:
 * from u = v with zero duals that iteration changes u only by the box
 * projection, so a cube already inside the box would stop there unchanged.
 * trace_all (may be NULL) gets 4 numbers per iteration. Returns the
 * iteration count. */
int ora_run(int n1, int n2, int n3, const ora_params *p, const double *v,
            double *u, double *s, double *t, double *w1, double *w2,
            double *y1, double *y2, double *y3, double *y4,
            int max_iter, double tol, int done_before, double *trace_all)
{
    primal x = {u, s, t, w1, w2};
    dual y = {y1, y2, y3, y4};
    double tr[4];
    int it = 0;
    double *ws = (double *)malloc(sizeof(double) * STEP_WS * (ix)n1 * n2 * n3);
    while (it < max_iter) {
        step_ws(n1, n2, n3, p, v, &x, &y, tr, ws);
        if (trace_all) memcpy(trace_all + 4 * it, tr, sizeof tr);
        ++it;
        if (tol > 0.0 && done_before + it >= 2 && tr[0] < tol) break;
    }
    free(ws);
    return it;
}

/* ------- the comparison regularizers through the same P-PDS (Sec. IV-A) -------
 *
 * The paper solves problem (15) with the GeoSSTV term replaced by the
 * regularizers of its comparison methods. Their definitions come from the
 * cited works:
 *   SSTV (Aggarwal and Majumdar):  ||D D_s u||_1;
 *   HSSTV (Takeyama et al.):       ||A_w u||_{1,p} with A_w u = (D D_s u, omega D u)
 *                                  in R^{4N}; HSSTV1: p = 1, the l1 norm of all
 *                                  4N entries; HSSTV2: p = 2, per voxel the l2
 *                                  norm of its four entries, summed.
 * Problem (15) with such a term is P-PDS-ready as it stands: primal blocks
 * x = (u, s, t) with f = iota_R(u) + iota_{B1,alpha}(s) + iota_{B1,beta}(t),
 * dual blocks z = K x = (A u, D_v t, u + s + t) with g = R_A(z1) +
 * iota_{0}(z2) + iota_{B2,eps}^v(z3), R_A the variant's norm.
 * Step sizes: eq. (8) with the operator-norm bounds ||D_v||^2 <= 4,
 * ||D||^2 <= 8, ||D D_s||^2 <= 32, ||omega D||^2 <= 8 omega^2:
 *   g_u = 1 / (||A||^2 + 1), g_s = 1, g_t = 1 / (4 + 1), g_y = 1/3 (three
 * primal blocks). */

enum { VAR_SSTV = 1, VAR_HSSTV1 = 2, VAR_HSSTV2 = 3 };

/* entries of A u per voxel: 2 (SSTV) or 4 (HSSTV) */
int ora_var_planes(int variant) { return variant == VAR_SSTV ? 2 : 4; }

static double var_norm_a2(int variant, double omega)
{
    return variant == VAR_SSTV ? 32.0 : 32.0 + 8.0 * omega * omega;
}

/* The step sizes (u, s, t, y) of a variant, for the tests. */
void ora_var_step_sizes(int variant, double omega, double *out)
{
    out[0] = 1.0 / (var_norm_a2(variant, omega) + 1.0);
    out[1] = 1.0;
    out[2] = 1.0 / 5.0;
    out[3] = 1.0 / 3.0;
}

/* out = A u: planes [D_v D_s u, D_h D_s u] and, for HSSTV, [omega D_v u,
 * omega D_h u]. tmp: N doubles. */
static void var_apply_a(int n1, int n2, int n3, int variant, double omega, const double *u,
                        double *out, double *tmp)
{
    ix N = (ix)n1 * n2 * n3;
    ora_ds(n1, n2, n3, u, tmp);
    ora_d(n1, n2, n3, tmp, out);
    if (variant != VAR_SSTV) {
        ora_d(n1, n2, n3, u, out + 2 * N);
#pragma omp parallel for schedule(static)
        for (ix q = 2 * N; q < 4 * N; ++q) out[q] *= omega;
    }
}

/* out = A^T y. tmp: 3N doubles. */
static void var_apply_at(int n1, int n2, int n3, int variant, double omega, const double *y,
                         double *out, double *tmp)
{
    ix N = (ix)n1 * n2 * n3;
    double *a = tmp, *b = tmp + N, *c = tmp + 2 * N;
    d_t_ws(n1, n2, n3, y, a, b);
    ora_ds_t(n1, n2, n3, a, out);
    if (variant != VAR_SSTV) {
        d_t_ws(n1, n2, n3, y + 2 * N, c, b);
#pragma omp parallel for schedule(static)
        for (ix q = 0; q < N; ++q) out[q] += omega * c[q];
    }
}

/* The stacked operator K of a variant and its adjoint, for the tests:
 * x = (u, s, t) (3N) -> z = (A u, D_v t, u + s + t) ((P + 2) N, P planes of
 * A u); adjoint = 1 maps z back. */
void ora_var_apply_k(int n1, int n2, int n3, int variant, double omega, int adjoint,
                     const double *in, double *out)
{
    ix N = (ix)n1 * n2 * n3;
    const int P = ora_var_planes(variant);
    double *tmp = (double *)malloc(sizeof(double) * 3 * N);
    if (!adjoint) {
        const double *u = in, *s = in + N, *t = in + 2 * N;
        var_apply_a(n1, n2, n3, variant, omega, u, out, tmp);
        ora_dv(n1, n2, n3, t, out + P * N);
        double *z3 = out + (P + 1) * N;
#pragma omp parallel for schedule(static)
        for (ix q = 0; q < N; ++q) z3[q] = u[q] + s[q] + t[q];
    } else {
        const double *y1 = in, *y3 = in + P * N, *y4 = in + (P + 1) * N;
        double *gu = out, *gs = out + N, *gt = out + 2 * N;
        var_apply_at(n1, n2, n3, variant, omega, y1, gu, tmp);
        ora_dv_t(n1, n2, n3, y3, gt);
#pragma omp parallel for schedule(static)
        for (ix q = 0; q < N; ++q) {
            gu[q] += y4[q];
            gs[q] = y4[q];
            gt[q] += y4[q];
        }
    }
    free(tmp);
}

/* prox of g_y R_A^* on the first dual block, by the Moreau decomposition (3):
 * prox_{G R*}(z) = z - G prox_{R/G}(z/G). For the l1 norm prox_{R/G} is the
 * soft threshold at 1/G, which leaves the clip of z to [-1, 1]; for the
 * l1,2 norm over 4-entry groups it is the group shrink at 1/G, which leaves
 * each group scaled into the unit l2 ball. */
static void var_prox_dual(int variant, ix N, double *y)
{
    if (variant != VAR_HSSTV2) {
#pragma omp parallel for schedule(static)
        for (ix q = 0; q < ora_var_planes(variant) * N; ++q) y[q] = y[q] < -1.0 ? -1.0 : (y[q] > 1.0 ? 1.0 : y[q]);
        return;
    }
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) {
        double nr = 0.0;
        for (int g = 0; g < 4; ++g) nr += y[g * N + q] * y[g * N + q];
        nr = sqrt(nr);
        if (nr > 1.0)
            for (int g = 0; g < 4; ++g) y[g * N + q] /= nr;
    }
}

/* Initial point: u = v, s = t = 0, every dual zero. y1: P planes. */
void ora_var_init(int n1, int n2, int n3, int variant, const double *v, double *u, double *s,
                  double *t, double *y1, double *y3, double *y4)
{
    ix N = (ix)n1 * n2 * n3;
    memcpy(u, v, sizeof(double) * N);
    memset(s, 0, sizeof(double) * N);
    memset(t, 0, sizeof(double) * N);
    memset(y1, 0, sizeof(double) * ora_var_planes(variant) * N);
    memset(y3, 0, sizeof(double) * N);
    memset(y4, 0, sizeof(double) * N);
}

/* One P-PDS iteration, eq. (7), for a variant:
 *   x+ = prox_{T f}(x - T K^T y),  x' = 2 x+ - x,  y+ = prox_{Sigma g*}(y + Sigma K x').
 * trace as for ora_step. ws: (P + 12) N doubles. */
static void var_step_ws(int n1, int n2, int n3, const ora_params *p, int variant, const double *v,
                        double *u, double *s, double *t, double *y1, double *y3, double *y4,
                        double *trace, double *ws)
{
    ix N = (ix)n1 * n2 * n3;
    const int P = ora_var_planes(variant);
    double st[4];
    ora_var_step_sizes(variant, p->omega, st);
    const double gu = st[0], gs = st[1], gt = st[2], gy = st[3];
    double *un = ws, *sn = ws + N, *tn = ws + 2 * N, *ga = ws + 3 * N, *gb = ws + 4 * N;
    double *z1 = ws + 5 * N, *tmp = ws + (5 + P) * N; /* tmp: 7N */

    /* primal half: forward step with K^T y, then the block proxes */
    var_apply_at(n1, n2, n3, variant, p->omega, y1, ga, tmp);
    ora_dv_t(n1, n2, n3, y3, gb);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) {
        un[q] = u[q] - gu * (ga[q] + y4[q]);
        sn[q] = s[q] - gs * y4[q];
        tn[q] = t[q] - gt * (gb[q] + y4[q]);
    }
    ora_proj_box(un, N, p->mu_lo, p->mu_hi, un);
    const double tau_s = ora_proj_l1(sn, N, p->alpha, sn);
    const double tau_t = ora_proj_l1(tn, N, p->beta, tn);

    /* extrapolated point x' = 2 x+ - x (into ga, gb, tmp) */
    double *up = ga, *sp = gb, *tp = tmp + 3 * N;
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) {
        up[q] = 2.0 * un[q] - u[q];
        sp[q] = 2.0 * sn[q] - s[q];
        tp[q] = 2.0 * tn[q] - t[q];
    }

    /* dual half: forward step with K x', then the conjugate proxes */
    var_apply_a(n1, n2, n3, variant, p->omega, up, z1, tmp);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < P * N; ++q) y1[q] += gy * z1[q];
    var_prox_dual(variant, N, y1);
    ora_dv(n1, n2, n3, tp, tmp);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) {
        y3[q] += gy * tmp[q];
        y4[q] += gy * (up[q] + sp[q] + tp[q]);
    }
    /* the l2-ball block, as for GeoSSTV: y4 - g_y P_B(y4 / g_y) */
    double *a = tmp, *b = tmp + N;
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) a[q] = y4[q] / gy;
    const double r = ora_proj_l2(a, v, N, p->eps, b);
#pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) y4[q] = y4[q] - gy * b[q];

    double dn = 0.0, un2 = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : dn, un2)
    for (ix q = 0; q < N; ++q) {
        dn += (un[q] - u[q]) * (un[q] - u[q]);
        un2 += u[q] * u[q];
    }
    memcpy(u, un, sizeof(double) * N);
    memcpy(s, sn, sizeof(double) * N);
    memcpy(t, tn, sizeof(double) * N);
    if (trace) {
        trace[0] = un2 > 0.0 ? sqrt(dn) / sqrt(un2) : INFINITY;
        trace[1] = r;
        trace[2] = tau_s;
        trace[3] = tau_t;
    }
}

/* As ora_run, for a variant (same stopping rule and trace). */
int ora_var_run(int n1, int n2, int n3, const ora_params *p, int variant, const double *v,
                double *u, double *s, double *t, double *y1, double *y3, double *y4,
                int max_iter, double tol, int done_before, double *trace_all)
{
    double tr[4];
    int it = 0;
    const int P = ora_var_planes(variant);
    double *ws = (double *)malloc(sizeof(double) * (ix)(P + 12) * n1 * n2 * n3);
    while (it < max_iter) {
        var_step_ws(n1, n2, n3, p, variant, v, u, s, t, y1, y3, y4, tr, ws);
        if (trace_all) memcpy(trace_all + 4 * it, tr, sizeof tr);
        ++it;
        if (tol > 0.0 && done_before + it >= 2 && tr[0] < tol) break;
    }
    free(ws);
    return it;
}
