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
 * steps of Alg. 1 in the paper's order, double precision throughout, no
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
 *  - Initial point of Alg. 1: u = v, every other variable zero.
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

/* ----------------------------- Algorithm 1 ------------------------------ */

typedef struct {
    double eps, alpha, beta; /* radii of (18), (16), (17)              */
    double mu_lo, mu_hi;     /* box (19)                                 */
    double omega;            /* balance of GeoSSTV, eq. (13)             */
} ora_params;

/* Step sizes printed after eq. (24). */
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

/* number of doubles of scratch that one step needs, in units of N */
#define STEP_WS 46

static void step_ws(int n1, int n2, int n3, const ora_params *p, const double *v,
                    double *u, double *s, double *t, double *w1, double *w2,
                    double *y1, double *y2, double *y3, double *y4, double *trace, double *ws)
{
    ix N = (ix)n1 * n2 * n3;
    double *a = ws, *b = a + N, *c2 = b + N, *c6 = c2 + 2 * N, *un = c6 + 6 * N;
    double *sn = un + N, *tn = sn + N, *w1n = tn + N, *w2n = w1n + 6 * N, *up = w2n + 6 * N;
    double *sp = up + N, *tp = sp + N, *w1p = tp + N, *w2p = w1p + 6 * N;
    double *t1 = w2p + 6 * N, *t2 = t1 + 2 * N; /* operator temporaries, 2N each */

    /* step 1: u+ = P_R(u - g_u (D^T y1 + D_s^T D^T y2 + y4)) */
    d_t_ws(n1, n2, n3, y1, a, t1);
    d_t_ws(n1, n2, n3, y2, b, t1);
    ora_ds_t(n1, n2, n3, b, up); /* up used as scratch here */
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) a[q] = u[q] - G_U * (a[q] + up[q] + y4[q]);
    ora_proj_box(a, N, p->mu_lo, p->mu_hi, un);

    /* step 2: s+ = P_{B1,alpha}(s - g_s y4) */
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) a[q] = s[q] - G_S * y4[q];
    double tau_s = ora_proj_l1(a, N, p->alpha, sn);

    /* step 3: t+ = P_{B1,beta}(t - g_t (D_v^T y3 + y4)) */
    ora_dv_t(n1, n2, n3, y3, a);
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) a[q] = t[q] - G_T * (a[q] + y4[q]);
    double tau_t = ora_proj_l1(a, N, p->beta, tn);

    /* step 4: w1+ = prox_{g_w1 omega ||.||_{1,2}}(w1 + g_w1 L y1) */
    ora_l(n1, n2, n3, y1, c6);
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < 6 * N; ++q) c6[q] = w1[q] + G_W1 * c6[q];
    for (int g = 0; g < 3; ++g)
        ora_prox_l12(c6 + 2 * g * N, c6 + (2 * g + 1) * N, N, G_W1 * p->omega,
                     w1n + 2 * g * N, w1n + (2 * g + 1) * N);

    /* step 5: w2+ = prox_{g_w2 ||.||_{1,2}}(w2 + g_w2 L y2) */
    ora_l(n1, n2, n3, y2, c6);
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < 6 * N; ++q) c6[q] = w2[q] + G_W2 * c6[q];
    for (int g = 0; g < 3; ++g)
        ora_prox_l12(c6 + 2 * g * N, c6 + (2 * g + 1) * N, N, G_W2,
                     w2n + 2 * g * N, w2n + (2 * g + 1) * N);

    /* steps 6-10: extrapolation x' = 2 x+ - x */
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) {
        up[q] = 2.0 * un[q] - u[q];
        sp[q] = 2.0 * sn[q] - s[q];
        tp[q] = 2.0 * tn[q] - t[q];
    }
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < 6 * N; ++q) {
        w1p[q] = 2.0 * w1n[q] - w1[q];
        w2p[q] = 2.0 * w2n[q] - w2[q];
    }

    /* step 11: y1 += g_y (D u' - L^T w1') */
    ora_d(n1, n2, n3, up, c2);
    l_t_ws(n1, n2, n3, w1p, c6, t1, t2); /* first 2N entries of c6 as scratch */
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < 2 * N; ++q) y1[q] += G_Y * (c2[q] - c6[q]);

    /* step 12: y2 += g_y (D D_s u' - L^T w2') */
    ora_ds(n1, n2, n3, up, a);
    ora_d(n1, n2, n3, a, c2);
    l_t_ws(n1, n2, n3, w2p, c6, t1, t2);
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < 2 * N; ++q) y2[q] += G_Y * (c2[q] - c6[q]);

    /* step 13: y3 += g_y D_v t' */
    ora_dv(n1, n2, n3, tp, a);
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) y3[q] += G_Y * a[q];

    /* step 14: y4' = y4 + g_y (u' + s' + t') */
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) y4[q] += G_Y * (up[q] + sp[q] + tp[q]);

    /* step 15: y4+ = y4' - g_y P_{B2,eps}^v(y4' / g_y)  (eq. (3), (23)) */
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) a[q] = y4[q] / G_Y;
    double r = ora_proj_l2(a, v, N, p->eps, b);
    #pragma omp parallel for schedule(static)
    for (ix q = 0; q < N; ++q) y4[q] = y4[q] - G_Y * b[q];

    /* stopping quantity of eq. (28) */
    double dn = 0.0, un2 = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : dn, un2)
    for (ix q = 0; q < N; ++q) {
        dn += (un[q] - u[q]) * (un[q] - u[q]);
        un2 += u[q] * u[q];
    }
    double rel = un2 > 0.0 ? sqrt(dn) / sqrt(un2) : INFINITY;

    memcpy(u, un, sizeof(double) * N);
    memcpy(s, sn, sizeof(double) * N);
    memcpy(t, tn, sizeof(double) * N);
    memcpy(w1, w1n, sizeof(double) * 6 * N);
    memcpy(w2, w2n, sizeof(double) * 6 * N);
    if (trace) {
        trace[0] = rel;
        trace[1] = r;
        trace[2] = tau_s;
        trace[3] = tau_t;
    }
}

/* One pass of the loop body of Alg. 1 for problem (20), updating the state
 * in place. trace (may be NULL) receives
 *   [0] ||u+ - u||_2 / ||u||_2    (stopping quantity of eq. (28); +inf when
 *                                  ||u|| = 0)
 *   [1] ||y4'/gamma - v||_2       (the distance tested in the l2 projection)
 *   [2] tau_s, [3] tau_t          (soft-threshold levels of the l1 balls)
 */
void ora_step(int n1, int n2, int n3, const ora_params *p, const double *v,
              double *u, double *s, double *t, double *w1, double *w2,
              double *y1, double *y2, double *y3, double *y4, double *trace)
{
    double *ws = (double *)malloc(sizeof(double) * STEP_WS * (ix)n1 * n2 * n3);
    step_ws(n1, n2, n3, p, v, u, s, t, w1, w2, y1, y2, y3, y4, trace, ws);
    free(ws);
}

/* Run the loop of Alg. 1: at most max_iter passes, stopping after the first
 * pass whose stopping quantity (eq. (28)) is below tol (tol <= 0: run all
 * passes). done_before: passes made since the initial point by earlier
 * calls. The rule is not applied to the first pass after the initial point:
 * from u = v with zero duals that pass changes u only by the box projection,
 * so a cube already inside the box would stop there unchanged.
 * trace_all (may be NULL) gets 4 numbers per pass. Returns the pass count. */
int ora_run(int n1, int n2, int n3, const ora_params *p, const double *v,
            double *u, double *s, double *t, double *w1, double *w2,
            double *y1, double *y2, double *y3, double *y4,
            int max_iter, double tol, int done_before, double *trace_all)
{
    double tr[4];
    int it = 0;
    double *ws = (double *)malloc(sizeof(double) * STEP_WS * (ix)n1 * n2 * n3);
    while (it < max_iter) {
        step_ws(n1, n2, n3, p, v, u, s, t, w1, w2, y1, y2, y3, y4, tr, ws);
        if (trace_all) memcpy(trace_all + 4 * it, tr, sizeof tr);
        ++it;
        if (tol > 0.0 && done_before + it >= 2 && tr[0] < tol) break;
    }
    free(ws);
    return it;
}
