/*
 * FP64 CPU oracle for parallel-beam FBP, the matched projector pair and the
 * TV solvers of PyHST2 (Mirone et al., NIM B).  TEST INFRASTRUCTURE ONLY: it is
 * loaded by the tests, by the smoke check and by the bench's CPU-baseline leg,
 * never by the reconstruction library.  It is written from the definitions
 * (plain loops, double precision, no blocking, no FFT) and shares no code with
 * the GPU path.
 *
 * Conventions (section 2.1, parallel geometry):
 *   pixel (ix, iy) centre: x = ix - (n_x-1)/2, y = iy - (n_y-1)/2, pixel units
 *   detector coordinate of that centre at projection k:
 *       t = s*(x cos th_k + y sin th_k) + c + sigma_k     (bin j centred at j)
 *   hat(d) = max(0, 1 - |d|)
 *   backprojection  B: img[px]   = sum_k sum_j q[k][j] hat(t_k(px) - j)
 *   projection      A: sino[k][j] = s^2 sum_px img[px] hat(t_k(px) - j)
 * so A = s^2 B^T exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Dark / flat normalisation and -log (section 2.3; Beer-Lambert for
 * absorption data).  Flats are interpolated linearly in the projection index
 * between their acquisition positions and held constant outside them.
 *   p = -ln(max((I - D)/(F_k - D), eps));  p = 0 where F_k - D <= 0.
 * raw: [K][R][nb] (radiographs, as acquired), out: [R][K][nb] (sinograms).
 * ------------------------------------------------------------------------- */
void or_normalize(int K, int R, int nb, const double *raw, int n_flats, const double *flats,
                  const double *flat_pos, const double *dark, double eps, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < K; ++k) {
        int i0 = 0, i1 = 0;
        double a = 0.0;
        if (n_flats > 1) {
            if (k <= flat_pos[0]) {
                i0 = i1 = 0;
            } else if (k >= flat_pos[n_flats - 1]) {
                i0 = i1 = n_flats - 1;
            } else {
                int i = 0;
                while (i + 1 < n_flats && !(k < flat_pos[i + 1])) ++i;
                i0 = i;
                i1 = i + 1;
                a = (k - flat_pos[i0]) / (flat_pos[i1] - flat_pos[i0]);
            }
        }
        for (int r = 0; r < R; ++r) {
            for (int j = 0; j < nb; ++j) {
                double d = dark[(size_t)r * nb + j];
                double f = (1.0 - a) * flats[((size_t)i0 * R + r) * nb + j] + a * flats[((size_t)i1 * R + r) * nb + j];
                double den = f - d;
                double v = 0.0;
                if (den > 0.0) {
                    double ratio = (raw[((size_t)k * R + r) * nb + j] - d) / den;
                    if (!(ratio >= eps)) ratio = eps;
                    v = -log(ratio);
                }
                out[((size_t)r * K + k) * nb + j] = v;
            }
        }
    }
}

/* ---------------------------------------------------------------------------
 * Hot-spot removal (section 2.3, processing pipe): after the flat-field
 * correction t = (I - D)/(F_k - D), a pixel whose neighbours' median is below
 * t by more than thr is replaced by that median.  Neighbours: the up to 8
 * pixels of the 3x3 window of the same radiograph (rows r +- 1 of the rows
 * given, bins j +- 1), taken before any replacement; the median of an even
 * count is the mean of the two middle values.  Dead pixels (F_k - D <= 0)
 * count as t = 1 and stay p = 0.  Then p = -ln(max(t, eps)) as above.
 * raw: [K][R][nb], out: [R][K][nb].
 * ------------------------------------------------------------------------- */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

void or_normalize_hotspot(int K, int R, int nb, const double *raw, int n_flats, const double *flats,
                          const double *flat_pos, const double *dark, double eps, double thr, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < K; ++k) {
        int i0 = 0, i1 = 0;
        double a = 0.0;
        if (n_flats > 1) {
            if (k <= flat_pos[0]) {
                i0 = i1 = 0;
            } else if (k >= flat_pos[n_flats - 1]) {
                i0 = i1 = n_flats - 1;
            } else {
                int i = 0;
                while (i + 1 < n_flats && !(k < flat_pos[i + 1])) ++i;
                i0 = i;
                i1 = i + 1;
                a = (k - flat_pos[i0]) / (flat_pos[i1] - flat_pos[i0]);
            }
        }
        double *t = (double *)malloc(sizeof(double) * (size_t)R * nb);
        char *dead = (char *)malloc((size_t)R * nb);
        for (int r = 0; r < R; ++r)
            for (int j = 0; j < nb; ++j) {
                size_t o = (size_t)r * nb + j;
                double d = dark[o];
                double f = (1.0 - a) * flats[(size_t)i0 * R * nb + o] + a * flats[(size_t)i1 * R * nb + o];
                dead[o] = !(f - d > 0.0);
                t[o] = dead[o] ? 1.0 : (raw[(size_t)k * R * nb + o] - d) / (f - d);
            }
        for (int r = 0; r < R; ++r)
            for (int j = 0; j < nb; ++j) {
                size_t o = (size_t)r * nb + j;
                double v = 0.0;
                if (!dead[o]) {
                    double nbv[8];
                    int n = 0;
                    for (int dr = -1; dr <= 1; ++dr)
                        for (int dj = -1; dj <= 1; ++dj) {
                            if (dr == 0 && dj == 0) continue;
                            int rr = r + dr, jj = j + dj;
                            if (rr < 0 || rr >= R || jj < 0 || jj >= nb) continue;
                            nbv[n++] = t[(size_t)rr * nb + jj];
                        }
                    double tv = t[o];
                    if (n > 0) {
                        qsort(nbv, (size_t)n, sizeof(double), cmp_double);
                        double med = (n & 1) ? nbv[n / 2] : 0.5 * (nbv[n / 2 - 1] + nbv[n / 2]);
                        if (tv - med > thr) tv = med;
                    }
                    if (!(tv >= eps)) tv = eps;
                    v = -log(tv);
                }
                out[((size_t)r * K + k) * nb + j] = v;
            }
        free(t);
        free(dead);
    }
}

/* ---------------------------------------------------------------------------
 * Ring-artifact filter (section 2.3): the sinogram is reduced to a 1-D signal
 * by averaging over the projection angles, m[j] = (1/K) sum_k (p[k][j] - obj[k][j]),
 * its high frequencies hp = m - (moving average of m over the 2w+1 bins
 * j-w..j+w that exist) are extracted, and hp is subtracted from every row.
 * obj (or NULL) is a sinogram of the object's strongly absorbing part (the
 * projection of a thresholded first reconstruction), removed from the data
 * before the average so that sharp object borders do not leak into hp.
 * p: [K][L], modified in place.
 * ------------------------------------------------------------------------- */
void or_ring_filter(int K, int L, double *p, const double *obj, int w)
{
    double *m = (double *)calloc((size_t)L, sizeof(double));
    double *hp = (double *)malloc(sizeof(double) * (size_t)L);
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < L; ++j) m[j] += p[(size_t)k * L + j] - (obj ? obj[(size_t)k * L + j] : 0.0);
    for (int j = 0; j < L; ++j) m[j] /= K;
    for (int j = 0; j < L; ++j) {
        double s = 0.0;
        int n = 0;
        for (int i = j - w; i <= j + w; ++i)
            if (i >= 0 && i < L) {
                s += m[i];
                ++n;
            }
        hp[j] = m[j] - s / n;
    }
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < L; ++j) p[(size_t)k * L + j] -= hp[j];
    free(m);
    free(hp);
}

/* ---------------------------------------------------------------------------
 * Ram-Lak ramp filter at unit bin spacing (Kak & Slaney ch. 3):
 *   h[0] = 1/4, h[n odd] = -1/(pi^2 n^2), h[n even != 0] = 0.
 * Linear convolution restricted to [0, L), zero outside the row, each row
 * scaled by its weight:  q[n] = w_r * sum_{m=0}^{L-1} h[n - m] p[m].
 * ------------------------------------------------------------------------- */
static double ramlak(long n)
{
    if (n == 0) return 0.25;
    if ((n & 1) == 0) return 0.0;
    return -1.0 / (OR_PI * OR_PI * (double)n * (double)n);
}

void or_ramp_filter(int rows, int L, const double *in, const double *w, double *out)
{
#pragma omp parallel for schedule(static)
    for (int r = 0; r < rows; ++r) {
        const double *p = in + (size_t)r * L;
        double *q = out + (size_t)r * L;
        for (int n = 0; n < L; ++n) {
            double acc = 0.0;
            for (int m = 0; m < L; ++m) acc += ramlak((long)n - m) * p[m];
            q[n] = w[r] * acc;
        }
    }
}

/* Angle weights: mid-point rule with circular wrap over the scan period
 * theta_span (pi or 2 pi), scaled by 'factor'.  Angles are visited in
 * ascending order; a negative gap is clamped to zero. */
void or_angle_weights(int K, const double *ang, double span, double factor, double *w)
{
    int *ord = (int *)malloc(sizeof(int) * (size_t)K);
    for (int i = 0; i < K; ++i) ord[i] = i;
    /* insertion sort: plain and stable */
    for (int i = 1; i < K; ++i) {
        int v = ord[i], j = i - 1;
        while (j >= 0 && ang[ord[j]] > ang[v]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = v;
    }
    for (int i = 0; i < K; ++i) {
        double prev = (i == 0) ? ang[ord[K - 1]] - span : ang[ord[i - 1]];
        double next = (i == K - 1) ? ang[ord[0]] + span : ang[ord[i + 1]];
        double g0 = ang[ord[i]] - prev, g1 = next - ang[ord[i]];
        if (g0 < 0) g0 = 0;
        if (g1 < 0) g1 = 0;
        if (K == 1) { g0 = span / 2; g1 = span / 2; }
        w[ord[i]] = factor * 0.5 * (g0 + g1);
    }
    free(ord);
}

/* ---------------------------------------------------------------------------
 * Backprojection (pixel driven, linear detector interpolation as hat weights).
 * sino: [K][L], img: [n_y][n_x].  img = sum_k sum_{j in [0,L)} q hat(t - j).
 * ------------------------------------------------------------------------- */
void or_backproject(int n_x, int n_y, int K, int L, const double *ang, double axis, const double *shift,
                    double s, const double *sino, double *img)
{
    double cx = 0.5 * (n_x - 1), cy = 0.5 * (n_y - 1);
    double *ct = (double *)malloc(sizeof(double) * (size_t)K), *st = (double *)malloc(sizeof(double) * (size_t)K);
    for (int k = 0; k < K; ++k) { ct[k] = cos(ang[k]); st[k] = sin(ang[k]); }
#pragma omp parallel for schedule(static)
    for (int iy = 0; iy < n_y; ++iy) {
        for (int ix = 0; ix < n_x; ++ix) {
            double x = ix - cx, y = iy - cy, acc = 0.0;
            for (int k = 0; k < K; ++k) {
                double t = s * (x * ct[k] + y * st[k]) + axis + (shift ? shift[k] : 0.0);
                long j0 = (long)floor(t);
                for (long j = j0; j <= j0 + 1; ++j) {
                    if (j < 0 || j >= L) continue;
                    double h = 1.0 - fabs(t - (double)j);
                    if (h > 0.0) acc += sino[(size_t)k * L + j] * h;
                }
            }
            img[(size_t)iy * n_x + ix] = acc;
        }
    }
    free(ct);
    free(st);
}

/* Forward projection, written as a scatter over pixels (the transpose of the
 * backprojection above, times s^2).  sino: [K][L] (overwritten). */
void or_forward_project(int n_x, int n_y, int K, int L, const double *ang, double axis, const double *shift,
                        double s, const double *img, double *sino)
{
    double cx = 0.5 * (n_x - 1), cy = 0.5 * (n_y - 1);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < K; ++k) {
        double *row = sino + (size_t)k * L;
        double c = cos(ang[k]), sn = sin(ang[k]);
        for (int j = 0; j < L; ++j) row[j] = 0.0;
        for (int iy = 0; iy < n_y; ++iy) {
            for (int ix = 0; ix < n_x; ++ix) {
                double v = img[(size_t)iy * n_x + ix];
                if (v == 0.0) continue;
                double t = s * ((ix - cx) * c + (iy - cy) * sn) + axis + (shift ? shift[k] : 0.0);
                long j0 = (long)floor(t);
                for (long j = j0; j <= j0 + 1; ++j) {
                    if (j < 0 || j >= L) continue;
                    double h = 1.0 - fabs(t - (double)j);
                    if (h > 0.0) row[j] += s * s * v * h;
                }
            }
        }
    }
}

/* ---------------------------------------------------------------------------
 * Discrete isotropic TV (eq. 2) with the discretisation of Chambolle (2004):
 * forward differences, zero at the last column / row; div = -grad^T.
 * Arrays are [n_y][n_x]; g1 is the x (column) component, g2 the y (row) one.
 * ------------------------------------------------------------------------- */
void or_grad(int n_y, int n_x, const double *x, double *g1, double *g2)
{
    for (int i = 0; i < n_y; ++i)
        for (int j = 0; j < n_x; ++j) {
            size_t o = (size_t)i * n_x + j;
            g1[o] = (j + 1 < n_x) ? x[o + 1] - x[o] : 0.0;
            g2[o] = (i + 1 < n_y) ? x[o + n_x] - x[o] : 0.0;
        }
}

void or_div(int n_y, int n_x, const double *q1, const double *q2, double *d)
{
    for (int i = 0; i < n_y; ++i)
        for (int j = 0; j < n_x; ++j) {
            size_t o = (size_t)i * n_x + j;
            double a, b;
            if (j == 0) a = q1[o];
            else if (j == n_x - 1) a = -q1[o - 1];
            else a = q1[o] - q1[o - 1];
            if (i == 0) b = q2[o];
            else if (i == n_y - 1) b = -q2[o - n_x];
            else b = q2[o] - q2[o - n_x];
            if (n_x == 1) a = 0.0;
            if (n_y == 1) b = 0.0;
            d[o] = a + b;
        }
}

double or_tv(int n_y, int n_x, const double *x)
{
    size_t n = (size_t)n_y * n_x;
    double *g1 = (double *)malloc(n * sizeof(double)), *g2 = (double *)malloc(n * sizeof(double));
    or_grad(n_y, n_x, x, g1, g2);
    double s = 0.0;
    for (size_t o = 0; o < n; ++o) s += sqrt(g1[o] * g1[o] + g2[o] * g2[o]);
    free(g1);
    free(g2);
    return s;
}

/* ROF proximal map  u = argmin 1/2|u - g|^2 + lambda TV(u)  by the dual
 * projection algorithm of Chambolle (2004), step tau = 1/8, p^0 = 0:
 *   p <- (p + tau grad(div p - g/lambda)) / (1 + tau |grad(div p - g/lambda)|)
 *   u = g - lambda div p                                                   */
void or_tv_prox(int n_y, int n_x, const double *g, double lambda, int n_inner, double *u)
{
    size_t n = (size_t)n_y * n_x;
    if (lambda <= 0.0 || n_inner <= 0) {
        memcpy(u, g, n * sizeof(double));
        return;
    }
    double *p1 = (double *)calloc(n, sizeof(double)), *p2 = (double *)calloc(n, sizeof(double));
    double *v = (double *)malloc(n * sizeof(double));
    double *a1 = (double *)malloc(n * sizeof(double)), *a2 = (double *)malloc(n * sizeof(double));
    const double tau = 0.125;
    for (int it = 0; it < n_inner; ++it) {
        or_div(n_y, n_x, p1, p2, v);
        for (size_t o = 0; o < n; ++o) v[o] -= g[o] / lambda;
        or_grad(n_y, n_x, v, a1, a2);
        for (size_t o = 0; o < n; ++o) {
            double m = sqrt(a1[o] * a1[o] + a2[o] * a2[o]);
            p1[o] = (p1[o] + tau * a1[o]) / (1.0 + tau * m);
            p2[o] = (p2[o] + tau * a2[o]) / (1.0 + tau * m);
        }
    }
    or_div(n_y, n_x, p1, p2, v);
    for (size_t o = 0; o < n; ++o) u[o] = g[o] - lambda * v[o];
    free(p1); free(p2); free(v); free(a1); free(a2);
}

/* ---------------------------------------------------------------------------
 * Chambolle-Pock primal-dual iteration for eq. (3):
 *     min_x 1/2 |A x - y|^2 + lambda TV(x),   K = [A; mu grad],  tau = sigma = 1/Lk
 * (lambda TV(x) = (lambda/mu) sum_i |(mu grad x)_i|, so the dual field of the
 * second block lives in the ball of radius lambda/mu; mu = 1 is the plain
 * operator) with theta = 1 and x = xbar = p = q = 0 initially.  One iteration:
 *     p  <- (p + sigma (A xbar - y)) / (1 + sigma)
 *     q  <- q + sigma mu grad xbar, then q <- q / max(1, |q| / (lambda/mu)) pointwise
 *     x+ <- x - tau (A^T p - mu div q)
 *     xbar <- 2 x+ - x,  x <- x+
 * 'identity' != 0 replaces A by the identity (then y has the image shape).
 * energy[i] (if non-NULL) = 1/2|A x - y|^2 + lambda TV(x) after iteration i.
 * ------------------------------------------------------------------------- */
static void apply_A(int identity, int n_x, int n_y, int K, int L, const double *ang, double axis,
                    const double *shift, double s, const double *x, double *out)
{
    if (identity) memcpy(out, x, sizeof(double) * (size_t)n_x * n_y);
    else or_forward_project(n_x, n_y, K, L, ang, axis, shift, s, x, out);
}

static void apply_AT(int identity, int n_x, int n_y, int K, int L, const double *ang, double axis,
                     const double *shift, double s, const double *y, double *out)
{
    size_t n = (size_t)n_x * n_y;
    if (identity) { memcpy(out, y, sizeof(double) * n); return; }
    or_backproject(n_x, n_y, K, L, ang, axis, shift, s, y, out);
    for (size_t o = 0; o < n; ++o) out[o] *= s * s;
}

void or_cp_tv(int identity, int n_x, int n_y, int K, int L, const double *ang, double axis, const double *shift,
              double s, const double *y, double lambda, int n_iter, double Lk, double mu, double *x_out,
              double *energy)
{
    size_t n = (size_t)n_x * n_y, m = identity ? n : (size_t)K * L;
    double *x = (double *)calloc(n, sizeof(double)), *xb = (double *)calloc(n, sizeof(double));
    double *p = (double *)calloc(m, sizeof(double)), *ax = (double *)malloc(m * sizeof(double));
    double *q1 = (double *)calloc(n, sizeof(double)), *q2 = (double *)calloc(n, sizeof(double));
    double *g1 = (double *)malloc(n * sizeof(double)), *g2 = (double *)malloc(n * sizeof(double));
    double *atp = (double *)malloc(n * sizeof(double)), *dv = (double *)malloc(n * sizeof(double));
    double tau = 1.0 / Lk, sigma = 1.0 / Lk;
    for (int it = 0; it < n_iter; ++it) {
        apply_A(identity, n_x, n_y, K, L, ang, axis, shift, s, xb, ax);
        for (size_t o = 0; o < m; ++o) p[o] = (p[o] + sigma * (ax[o] - y[o])) / (1.0 + sigma);
        or_grad(n_y, n_x, xb, g1, g2);
        for (size_t o = 0; o < n; ++o) {
            double a = q1[o] + sigma * mu * g1[o], b = q2[o] + sigma * mu * g2[o];
            double nrm = sqrt(a * a + b * b) / (lambda / mu);
            double d = nrm > 1.0 ? nrm : 1.0;
            if (lambda <= 0.0) { a = 0.0; b = 0.0; d = 1.0; }
            q1[o] = a / d;
            q2[o] = b / d;
        }
        apply_AT(identity, n_x, n_y, K, L, ang, axis, shift, s, p, atp);
        or_div(n_y, n_x, q1, q2, dv);
        for (size_t o = 0; o < n; ++o) {
            double xn = x[o] - tau * (atp[o] - mu * dv[o]);
            xb[o] = 2.0 * xn - x[o];
            x[o] = xn;
        }
        if (energy) {
            apply_A(identity, n_x, n_y, K, L, ang, axis, shift, s, x, ax);
            double r = 0.0;
            for (size_t o = 0; o < m; ++o) r += (ax[o] - y[o]) * (ax[o] - y[o]);
            energy[it] = 0.5 * r + lambda * or_tv(n_y, n_x, x);
        }
    }
    memcpy(x_out, x, n * sizeof(double));
    free(x); free(xb); free(p); free(ax); free(q1); free(q2); free(g1); free(g2); free(atp); free(dv);
}

/* ---------------------------------------------------------------------------
 * ISTA and FISTA for eq. (3), the solvers the paper names for the TV mode
 * (section 3.1; Daubechies et al. 2004, Beck & Teboulle 2009).  With
 * f(x) = 1/2|A x - y|^2, whose gradient A^T (A x - y) is La-Lipschitz for
 * La >= |A|^2, every iteration takes a gradient step of length 1/La from z and
 * then the proximal map of (lambda/La) TV:
 *     x_k = prox_{(lambda/La) TV}( z - (1/La) A^T (A z - y) )
 * The proximal map is or_tv_prox with n_inner dual iterations from zero.
 *     ISTA : z <- x_k
 *     FISTA: t' = (1 + sqrt(1 + 4 t^2)) / 2,  z <- x_k + ((t - 1) / t') (x_k - x_{k-1}),  t <- t'
 * starting from x_0 = z = 0, t = 1.  'identity' replaces A by the identity.
 * energy[i] (if non-NULL) = 1/2|A x_i - y|^2 + lambda TV(x_i) after iteration i.
 * ------------------------------------------------------------------------- */
void or_fista_tv(int fast, int identity, int n_x, int n_y, int K, int L, const double *ang, double axis,
                 const double *shift, double s, const double *y, double lambda, int n_iter, double La,
                 int n_inner, double *x_out, double *energy)
{
    size_t n = (size_t)n_x * n_y, m = identity ? n : (size_t)K * L;
    double *x = (double *)calloc(n, sizeof(double)), *xprev = (double *)calloc(n, sizeof(double));
    double *z = (double *)calloc(n, sizeof(double)), *v = (double *)malloc(n * sizeof(double));
    double *r = (double *)malloc(m * sizeof(double)), *atr = (double *)malloc(n * sizeof(double));
    double t = 1.0;
    for (int it = 0; it < n_iter; ++it) {
        /* gradient step from z */
        apply_A(identity, n_x, n_y, K, L, ang, axis, shift, s, z, r);
        for (size_t o = 0; o < m; ++o) r[o] -= y[o];
        apply_AT(identity, n_x, n_y, K, L, ang, axis, shift, s, r, atr);
        for (size_t o = 0; o < n; ++o) v[o] = z[o] - atr[o] / La;
        /* proximal step */
        memcpy(xprev, x, n * sizeof(double));
        or_tv_prox(n_y, n_x, v, lambda / La, n_inner, x);
        /* next extrapolation point */
        if (fast) {
            double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
            double mom = (t - 1.0) / tn;
            for (size_t o = 0; o < n; ++o) z[o] = x[o] + mom * (x[o] - xprev[o]);
            t = tn;
        } else {
            memcpy(z, x, n * sizeof(double));
        }
        if (energy) {
            apply_A(identity, n_x, n_y, K, L, ang, axis, shift, s, x, r);
            double e = 0.0;
            for (size_t o = 0; o < m; ++o) e += (r[o] - y[o]) * (r[o] - y[o]);
            energy[it] = 0.5 * e + lambda * or_tv(n_y, n_x, x);
        }
    }
    memcpy(x_out, x, n * sizeof(double));
    free(x); free(xprev); free(z); free(v); free(r); free(atr);
}

/* Operator norm |K|_2 of K = [A; mu grad] (with_grad != 0) or of A alone
 * (with_grad == 0) by power iteration on K^T K (or A^T A) from the caller's
 * start vector x0 (n_y*n_x).  Returns sqrt of the Rayleigh quotient. */
double or_opnorm(int n_x, int n_y, int K, int L, const double *ang, double axis, const double *shift, double s,
                 const double *x0, int n_iter, int with_grad, double mu)
{
    size_t n = (size_t)n_x * n_y, m = (size_t)K * L;
    double *x = (double *)malloc(n * sizeof(double)), *ax = (double *)malloc(m * sizeof(double));
    double *g1 = (double *)malloc(n * sizeof(double)), *g2 = (double *)malloc(n * sizeof(double));
    double *a = (double *)malloc(n * sizeof(double)), *b = (double *)malloc(n * sizeof(double));
    memcpy(x, x0, n * sizeof(double));
    double nrm = 0.0, lam = 0.0;
    for (size_t o = 0; o < n; ++o) nrm += x[o] * x[o];
    nrm = sqrt(nrm);
    for (size_t o = 0; o < n; ++o) x[o] /= nrm;
    for (int it = 0; it < n_iter; ++it) {
        or_forward_project(n_x, n_y, K, L, ang, axis, shift, s, x, ax);
        apply_AT(0, n_x, n_y, K, L, ang, axis, shift, s, ax, a);
        if (with_grad) {
            or_grad(n_y, n_x, x, g1, g2);
            or_div(n_y, n_x, g1, g2, b);
            for (size_t o = 0; o < n; ++o) a[o] -= mu * mu * b[o];   /* K^T K x = A^T A x - mu^2 div grad x */
        }
        double dot = 0.0, nn = 0.0;
        for (size_t o = 0; o < n; ++o) { dot += a[o] * x[o]; nn += a[o] * a[o]; }
        lam = dot;
        nn = sqrt(nn);
        for (size_t o = 0; o < n; ++o) x[o] = a[o] / nn;
    }
    free(x); free(ax); free(g1); free(g2); free(a); free(b);
    return sqrt(lam);
}

/* The backprojection above evaluated at selected pixels only (ix[i], iy[i]),
 * for checks of full-size images where computing every pixel is too slow. */
void or_backproject_points(int n_x, int n_y, int K, int L, const double *ang, double axis, const double *shift,
                           double s, const double *sino, int npts, const int *pix_x, const int *pix_y, double *out)
{
    double cx = 0.5 * (n_x - 1), cy = 0.5 * (n_y - 1);
    double *ct = (double *)malloc(sizeof(double) * (size_t)K), *st = (double *)malloc(sizeof(double) * (size_t)K);
    for (int k = 0; k < K; ++k) { ct[k] = cos(ang[k]); st[k] = sin(ang[k]); }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < npts; ++i) {
        double x = pix_x[i] - cx, y = pix_y[i] - cy, acc = 0.0;
        for (int k = 0; k < K; ++k) {
            double t = s * (x * ct[k] + y * st[k]) + axis + (shift ? shift[k] : 0.0);
            long j0 = (long)floor(t);
            for (long j = j0; j <= j0 + 1; ++j) {
                if (j < 0 || j >= L) continue;
                double h = 1.0 - fabs(t - (double)j);
                if (h > 0.0) acc += sino[(size_t)k * L + j] * h;
            }
        }
        out[i] = acc;
    }
    free(ct);
    free(st);
}
