/*
 * FP64 CPU oracle for the pixel-basis (box-spline) parallel-beam CT path of
 * Shu & Entezari, "Gram Filtering and Sinogram Interpolation for Pixel-basis
 * in Parallel-beam X-ray CT Reconstruction" (arXiv 2005.13471).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load or call it.  The product
 * library never links it.  It shares no code, header, table or constant
 * generator with the HIP path: every quantity below is computed from its
 * plain definition by geometry (chord lengths, polygon clipping) and exact
 * Gauss-Legendre quadrature, or by direct summation.  No box-spline closed
 * form is used anywhere in this file.
 *
 * Conventions (the paper leaves them open; the readings are listed in the
 * design notes of the repository):
 *   pixel k = (k1, k2), 0 <= k1, k2 < N, is the indicator of the rectangle of
 *   sides lx1 x lx2 centred at x_k = (lx1 (k1 - (N-1)/2), lx2 (k2 - (N-1)/2));
 *   images are row-major [k2][k1];
 *   u = (cos t, sin t) is the detector axis, a ray is the line {x : x.u = y};
 *   detector bin m sits at y_m = ly (m - (M-1)/2); sinograms are [angle][bin];
 *   the detector blur is the unit-integral box (1/zeta) box(./zeta) (Sec. 2),
 *   so the blurred footprint averages the projection over [y - zeta/2,
 *   y + zeta/2].
 *
 * Every floating-point value is double.  OpenMP parallelises only over
 * independent outputs, so results do not depend on the thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define OR_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre, 3 nodes: exact for polynomials of degree <= 5.           */
/* ------------------------------------------------------------------------ */
static const double GL_X[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
static const double GL_W[3] = {0.55555555555555555556, 0.88888888888888888889, 0.55555555555555555556};

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* sort + drop exact duplicates; returns the new count */
static int sort_unique(double *v, int n)
{
    qsort(v, (size_t)n, sizeof(double), cmp_double);
    int w = 0;
    for (int i = 0; i < n; ++i)
        if (w == 0 || v[i] != v[w - 1]) v[w++] = v[i];
    return w;
}

/* ------------------------------------------------------------------------ */
/* Footprints by geometry (Sec. 2 forward model, Sec. 4 eq. xray_of_f and    */
/* eq. blurxray_of_f).                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    double x0, x1, y0, y1; /* rectangle [x0,x1] x [y0,y1] */
} rect;

static rect pixel_rect(double cx, double cy, double lx1, double lx2)
{
    rect r = {cx - 0.5 * lx1, cx + 0.5 * lx1, cy - 0.5 * lx2, cy + 0.5 * lx2};
    return r;
}

/* Length of the line {x : x.u = y} inside the rectangle (the X-ray transform
 * of the pixel indicator).  The line is x = y u + tau v with v = (-s, c). */
static double chord_length(const rect *R, double c, double s, double y)
{
    double tlo = -HUGE_VAL, thi = HUGE_VAL;
    /* x-coordinate: y c - tau s must lie in [x0, x1] */
    double px = y * c;
    if (s == 0.0) {
        if (px < R->x0 || px > R->x1) return 0.0;
    } else {
        double a = (px - R->x1) / s, b = (px - R->x0) / s;
        if (a > b) { double t = a; a = b; b = t; }
        if (a > tlo) tlo = a;
        if (b < thi) thi = b;
    }
    /* y-coordinate: y s + tau c must lie in [y0, y1] */
    double py = y * s;
    if (c == 0.0) {
        if (py < R->y0 || py > R->y1) return 0.0;
    } else {
        double a = (R->y0 - py) / c, b = (R->y1 - py) / c;
        if (a > b) { double t = a; a = b; b = t; }
        if (a > tlo) tlo = a;
        if (b < thi) thi = b;
    }
    return thi > tlo ? thi - tlo : 0.0;
}

/* Clip a convex polygon against the half-plane  sgn * (x.u - lim) <= 0. */
static int clip_halfplane(const double *px, const double *py, int n, double c, double s,
                          double lim, double sgn, double *qx, double *qy)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        int j = (i + 1) % n;
        double di = sgn * (px[i] * c + py[i] * s - lim);
        double dj = sgn * (px[j] * c + py[j] * s - lim);
        if (di <= 0.0) { qx[m] = px[i]; qy[m] = py[i]; ++m; }
        if ((di < 0.0 && dj > 0.0) || (di > 0.0 && dj < 0.0)) {
            double t = di / (di - dj);
            qx[m] = px[i] + t * (px[j] - px[i]);
            qy[m] = py[i] + t * (py[j] - py[i]);
            ++m;
        }
    }
    return m;
}

/* Detector kernel (Sec. 2: the detector cell as boxes of different heights
 * and lengths): K(t) = sum_i h[i] 1{|t| <= w[i]/2}, nb boxes; nb = 0 is the
 * point sample of the X-ray transform (no blur).  The paper's single box
 * of width zeta and height 1/zeta is nb = 1.  Callers pass it as the array
 * det = {nb, w0, h0, w1, h1, ...}. */
#define OR_MAXB 4
typedef struct {
    int nb;
    double w[OR_MAXB], h[OR_MAXB];
} detector;

static detector det_from(const double *det)
{
    detector D;
    D.nb = (int)det[0];
    if (D.nb < 0) D.nb = 0;
    if (D.nb > OR_MAXB) D.nb = OR_MAXB;
    for (int i = 0; i < D.nb; ++i) {
        D.w[i] = det[1 + 2 * i];
        D.h[i] = det[2 + 2 * i];
    }
    return D;
}

/* widest box (0 without blur): the kernel's support is [-wmax/2, wmax/2] */
static double det_wmax(const detector *D)
{
    double m = 0.0;
    for (int i = 0; i < D->nb; ++i)
        if (D->w[i] > m) m = D->w[i];
    return m;
}

/* area(R intersect {x : |x.u - y| <= w/2}) by clipping the rectangle
 * against the two half-planes of the slab (Sutherland-Hodgman) and the
 * shoelace formula. */
static double slab_area(const rect *R, double c, double s, double zeta, double y)
{
    double ax[8] = {R->x0, R->x1, R->x1, R->x0}, ay[8] = {R->y0, R->y0, R->y1, R->y1};
    double bx[8], by[8], cx[8], cy[8];
    int n = clip_halfplane(ax, ay, 4, c, s, y + 0.5 * zeta, 1.0, bx, by);
    if (n < 3) return 0.0;
    n = clip_halfplane(bx, by, n, c, s, y - 0.5 * zeta, -1.0, cx, cy);
    if (n < 3) return 0.0;
    double area = 0.0; /* shoelace */
    for (int i = 0; i < n; ++i) {
        int j = (i + 1) % n;
        area += cx[i] * cy[j] - cx[j] * cy[i];
    }
    return 0.5 * fabs(area);
}

/* Footprint of the pixel rectangle through the detector kernel: the chord
 * length without blur, else sum_i h[i] area(R intersect slab of width w[i]
 * around y) (the projection integrated against each box; one box of width
 * zeta and height 1/zeta averages it over the cell). */
static double footprint_rect(const rect *R, double c, double s, const detector *D, double y)
{
    if (D->nb == 0) return chord_length(R, c, s, y);
    double acc = 0.0;
    for (int i = 0; i < D->nb; ++i) acc += D->h[i] * slab_area(R, c, s, D->w[i], y);
    return acc;
}

/* Breakpoints in y of the footprint: projections of the 4 corners, each
 * shifted by +-w[i]/2 for every box.  Writes 4 or 8 nb values (at most
 * OR_BRK), returns the count. */
#define OR_BRK (8 * OR_MAXB)
static int footprint_breaks(const rect *R, double c, double s, const detector *D, double *out)
{
    double p[4] = {R->x0 * c + R->y0 * s, R->x1 * c + R->y0 * s, R->x0 * c + R->y1 * s,
                   R->x1 * c + R->y1 * s};
    if (D->nb > 0) {
        int n = 0;
        for (int b = 0; b < D->nb; ++b)
            for (int i = 0; i < 4; ++i) {
                out[n++] = p[i] - 0.5 * D->w[b];
                out[n++] = p[i] + 0.5 * D->w[b];
            }
        return n;
    }
    for (int i = 0; i < 4; ++i) out[i] = p[i];
    return 4;
}

static void support(const double *br, int n, double *lo, double *hi)
{
    double a = br[0], b = br[0];
    for (int i = 1; i < n; ++i) {
        if (br[i] < a) a = br[i];
        if (br[i] > b) b = br[i];
    }
    *lo = a;
    *hi = b;
}

OR_API double or_footprint(double c, double s, double lx1, double lx2, const double *det, double cx,
                           double cy, double y)
{
    rect R = pixel_rect(cx, cy, lx1, lx2);
    detector D = det_from(det);
    return footprint_rect(&R, c, s, &D, y);
}

/* ------------------------------------------------------------------------ */
/* Continuous-y inner product of two footprints at one angle (Sec. 4: the    */
/* entries of H^T H with H's rows indexed by angle and continuous y).       */
/* Both footprints are piecewise polynomials of degree <= 2 between their    */
/* breakpoints, so the product has degree <= 4 and 3-point Gauss-Legendre    */
/* on every segment of the merged breakpoint list is exact.                  */
/* ------------------------------------------------------------------------ */
static double inner_product_angle(const rect *A, const rect *B, double c, double s, const detector *zeta)
{
    double br[2 * OR_BRK], lo1, hi1, lo2, hi2;
    int na = footprint_breaks(A, c, s, zeta, br);
    support(br, na, &lo1, &hi1);
    int nb = footprint_breaks(B, c, s, zeta, br + na);
    support(br + na, nb, &lo2, &hi2);
    double lo = lo1 > lo2 ? lo1 : lo2, hi = hi1 < hi2 ? hi1 : hi2;
    if (!(hi > lo)) return 0.0;
    int n = sort_unique(br, na + nb);
    double acc = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        double a = br[i], b = br[i + 1];
        if (b <= lo || a >= hi) continue;
        double h = 0.5 * (b - a), m = 0.5 * (a + b);
        for (int q = 0; q < 3; ++q) {
            double y = m + h * GL_X[q];
            acc += h * GL_W[q] * footprint_rect(A, c, s, zeta, y) * footprint_rect(B, c, s, zeta, y);
        }
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Gram filter by per-tap exact integrals (Sec. 4):                          */
/*   G[k] = sum_theta < F_0 , F_k >_theta ,  k in [-(N-1), N-1]^2,           */
/* with pixel 0 at the origin and pixel k centred at (k1 lx1, k2 lx2).       */
/* Output layout: G[(k2 + N-1) * (2N-1) + (k1 + N-1)].  Pairs of disjoint     */
/* footprints contribute exactly zero and are skipped.                       */
/* ------------------------------------------------------------------------ */
OR_API void or_gram(int N, double lx1, double lx2, int n, const double *theta, const double *det,
                    double *G)
{
    detector Dz = det_from(det);
    const detector *zeta = &Dz;
    const double wmax = det_wmax(zeta);
    const int W = 2 * N - 1;
    rect P0 = pixel_rect(0.0, 0.0, lx1, lx2);
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < W; ++r) {
        int k2 = r - (N - 1);
        for (int col = 0; col < W; ++col) {
            int k1 = col - (N - 1);
            rect Pk = pixel_rect(k1 * lx1, k2 * lx2, lx1, lx2);
            double acc = 0.0;
            for (int a = 0; a < n; ++a) {
                double c = cos(theta[a]), s = sin(theta[a]);
                double half = 0.5 * (lx1 * fabs(c) + lx2 * fabs(s) + wmax);
                double d = k1 * lx1 * c + k2 * lx2 * s;
                if (fabs(d) >= 2.0 * half) continue;
                acc += inner_product_angle(&P0, &Pk, c, s, zeta);
            }
            G[(size_t)r * W + col] = acc;
        }
    }
}

/* Selected taps only: taps[2i], taps[2i+1] = (k1, k2). */
OR_API void or_gram_at(int N, double lx1, double lx2, int n, const double *theta, const double *det,
                       int cnt, const int *taps, double *out)
{
    detector Dz = det_from(det);
    const detector *zeta = &Dz;
    const double wmax = det_wmax(zeta);
    (void)N;
    rect P0 = pixel_rect(0.0, 0.0, lx1, lx2);
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < cnt; ++i) {
        int k1 = taps[2 * i], k2 = taps[2 * i + 1];
        rect Pk = pixel_rect(k1 * lx1, k2 * lx2, lx1, lx2);
        double acc = 0.0;
        for (int a = 0; a < n; ++a) {
            double c = cos(theta[a]), s = sin(theta[a]);
            double half = 0.5 * (lx1 * fabs(c) + lx2 * fabs(s) + wmax);
            double d = k1 * lx1 * c + k2 * lx2 * s;
            if (fabs(d) >= 2.0 * half) continue;
            acc += inner_product_angle(&P0, &Pk, c, s, zeta);
        }
        out[i] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Explicit forward matrix H for tiny N (Sec. 4, the matrix H with one block */
/* of rows per angle).  Rows are (angle, segment, Gauss node) over the       */
/* merged breakpoints of all pixels at that angle; entry = sqrt(w) F_k(y_q), */
/* so (H^T H)_{ij} equals the continuous-y inner product exactly.            */
/* Call with H == NULL to get the row count.  H is row-major [rows][N*N].    */
/* ------------------------------------------------------------------------ */
OR_API int or_explicit_H(int N, double lx1, double lx2, int n, const double *theta, const double *det,
                         double *H)
{
    const int NN = N * N;
    detector Dz = det_from(det);
    const detector *zeta = &Dz;
    double *br = (double *)malloc(sizeof(double) * OR_BRK * (size_t)NN);
    int row = 0;
    for (int a = 0; a < n; ++a) {
        double c = cos(theta[a]), s = sin(theta[a]);
        int nb = 0;
        for (int k = 0; k < NN; ++k) {
            int k1 = k % N, k2 = k / N;
            rect R = pixel_rect(lx1 * (k1 - 0.5 * (N - 1)), lx2 * (k2 - 0.5 * (N - 1)), lx1, lx2);
            nb += footprint_breaks(&R, c, s, zeta, br + nb);
        }
        nb = sort_unique(br, nb);
        for (int i = 0; i + 1 < nb; ++i) {
            double h = 0.5 * (br[i + 1] - br[i]), m = 0.5 * (br[i] + br[i + 1]);
            for (int q = 0; q < 3; ++q) {
                if (H) {
                    double y = m + h * GL_X[q], sw = sqrt(h * GL_W[q]);
                    for (int k = 0; k < NN; ++k) {
                        int k1 = k % N, k2 = k / N;
                        rect R = pixel_rect(lx1 * (k1 - 0.5 * (N - 1)), lx2 * (k2 - 0.5 * (N - 1)),
                                            lx1, lx2);
                        H[(size_t)row * NN + k] = sw * footprint_rect(&R, c, s, zeta, y);
                    }
                }
                ++row;
            }
        }
    }
    free(br);
    return row;
}

/* ------------------------------------------------------------------------ */
/* Normal operator by direct spatial summation (Sec. 4, closing remark:     */
/* the Toeplitz-block-Toeplitz Gram matrix acts as a (2N-1)^2 filter):       */
/*   y[i] = sum_{j in [0,N)^2} G[i - j] c[j].                                */
/* ------------------------------------------------------------------------ */
static double apply_one(int N, const double *G, const double *c, int i1, int i2)
{
    const int W = 2 * N - 1;
    double acc = 0.0;
    for (int j2 = 0; j2 < N; ++j2) {
        const double *grow = G + (size_t)(i2 - j2 + N - 1) * W + (i1 + N - 1);
        const double *crow = c + (size_t)j2 * N;
        for (int j1 = 0; j1 < N; ++j1) acc += grow[-j1] * crow[j1];
    }
    return acc;
}

OR_API void or_apply(int N, const double *G, const double *c, double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N * N; ++i) y[i] = apply_one(N, G, c, i % N, i / N);
}

/* Selected outputs: idx[i] = k2 * N + k1. */
OR_API void or_apply_at(int N, const double *G, const double *c, int cnt, const int *idx,
                        double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < cnt; ++i) y[i] = apply_one(N, G, c, idx[i] % N, idx[i] / N);
}

/* ------------------------------------------------------------------------ */
/* Sinogram interpolation (Sec. 5).                                          */
/* ------------------------------------------------------------------------ */

/* Centred cardinal B-splines of degree 0..3 (textbook piecewise forms). */
OR_API double or_bspline(int d, double x)
{
    double a = fabs(x);
    switch (d) {
    case 0: return a < 0.5 ? 1.0 : (a == 0.5 ? 0.5 : 0.0);
    case 1: return a < 1.0 ? 1.0 - a : 0.0;
    case 2:
        if (a <= 0.5) return 0.75 - a * a;
        if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
        return 0.0;
    case 3:
        if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        if (a < 2.0) return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
        return 0.0;
    default: return 0.0;
    }
}

/* B-spline degree per angle (Sec. 5): the projected signal is C^0 (C^-1 for
 * an axis-aligned angle) without blur and C^1 (C^0 axis-aligned) with blur;
 * the interpolating B-spline has degree one above that continuity order. */
OR_API int or_degree(double theta, double zeta)  /* zeta > 0: any detector blur */
{
    double c = fabs(cos(theta)), s = fabs(sin(theta));
    int axis = (c < 1e-12 || s < 1e-12);
    if (zeta > 0.0) return axis ? 1 : 2;
    return axis ? 0 : 1;
}

/* Digital correction filter (Sec. 5, eq. correction filter): q is the
 * inverse of b[m] = beta_d(m) under convolution, Q(z) = 1 / B(z).  Computed
 * from that definition by solving the finite Toeplitz section
 * sum_j b[i - j] x[j] = delta[i] on |i|, |j| <= L with L = K + 80; the
 * central taps then match the bi-infinite inverse to far below rounding.
 * Returns q[-K..K] in q[0..2K]. */
OR_API void or_prefilter_taps(int d, int K, double *q)
{
    int L = K + 80, n = 2 * L + 1;
    int bw = (d + 1) / 2; /* half-bandwidth of b */
    double *A = (double *)calloc((size_t)n * n, sizeof(double));
    double *x = (double *)calloc((size_t)n, sizeof(double));
    for (int i = 0; i < n; ++i)
        for (int j = i - bw; j <= i + bw; ++j)
            if (j >= 0 && j < n) A[(size_t)i * n + j] = or_bspline(d, (double)(i - j));
    x[L] = 1.0;
    /* Gaussian elimination (the matrix is diagonally dominant for d <= 3) */
    for (int k = 0; k < n; ++k) {
        double piv = A[(size_t)k * n + k];
        int hi = k + bw < n ? k + bw : n - 1;
        for (int i = k + 1; i <= hi; ++i) {
            double f = A[(size_t)i * n + k] / piv;
            if (f == 0.0) continue;
            for (int j = k; j <= hi; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
            x[i] -= f * x[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double acc = x[k];
        int hi = k + bw < n ? k + bw : n - 1;
        for (int j = k + 1; j <= hi; ++j) acc -= A[(size_t)k * n + j] * x[j];
        x[k] = acc / A[(size_t)k * n + k];
    }
    for (int m = -K; m <= K; ++m) q[m + K] = x[L + m];
    free(A);
    free(x);
}

/* p = q_d * g for one detector row, g zero outside [0, M).  p has length
 * M + 2K and p[m + K] holds bin m, m in [-K, M-1+K]. */
static void prefilter_row(const double *g, int M, int K, const double *q, double *p)
{
    for (int m = -K; m < M + K; ++m) {
        double acc = 0.0;
        for (int j = -K; j <= K; ++j) {
            int src = m - j;
            if (src >= 0 && src < M) acc += q[j + K] * g[src];
        }
        p[m + K] = acc;
    }
}

OR_API void or_prefilter(int n, const double *theta, const double *det, int M, int K, const double *g,
                         double *p)
{
    const double zeta = det[0] > 0.0 ? 1.0 : 0.0; /* blurred or not: the degree rule */
    double *qs[3];
    for (int d = 0; d < 3; ++d) {
        qs[d] = (double *)malloc(sizeof(double) * (2 * K + 1));
        or_prefilter_taps(d, K, qs[d]);
    }
#pragma omp parallel for schedule(static)
    for (int a = 0; a < n; ++a) {
        int d = or_degree(theta[a], zeta);
        prefilter_row(g + (size_t)a * M, M, K, qs[d], p + (size_t)a * (M + 2 * K));
    }
    for (int d = 0; d < 3; ++d) free(qs[d]);
}

/* ghat(y) = sum_m p[m] beta_d((y - y_m) / ly),  m in [-K, M-1+K]. */
static double ghat_eval(const double *prow, int M, int K, double ly, int d, double y)
{
    double z = y / ly + 0.5 * (M - 1); /* fractional bin index */
    double r = 0.5 * (d + 1);
    int lo = (int)ceil(z - r), hi = (int)floor(z + r);
    if (lo < -K) lo = -K;
    if (hi > M - 1 + K) hi = M - 1 + K;
    double acc = 0.0;
    for (int m = lo; m <= hi; ++m) acc += prow[m + K] * or_bspline(d, z - m);
    return acc;
}

/* Evaluate ghat for every angle at arbitrary points (tests of Sec. 5). */
OR_API void or_ghat(int n, const double *theta, const double *det, double ly, int M, int K,
                    const double *g, int cnt, const double *y, double *out /* n x cnt */)
{
    const double zeta = det[0] > 0.0 ? 1.0 : 0.0;
    double *p = (double *)malloc(sizeof(double) * (size_t)n * (M + 2 * K));
    or_prefilter(n, theta, det, M, K, g, p);
    for (int a = 0; a < n; ++a) {
        int d = or_degree(theta[a], zeta);
        for (int i = 0; i < cnt; ++i)
            out[(size_t)a * cnt + i] = ghat_eval(p + (size_t)a * (M + 2 * K), M, K, ly, d, y[i]);
    }
    free(p);
}

/* ------------------------------------------------------------------------ */
/* Back projection with the exact adjoint (Sec. 5):                          */
/*   b[k] = sum_theta  integral F_{k,theta}(y) ghat_theta(y) dy.             */
/* Segments are cut at the footprint breakpoints and at the knots of ghat;   */
/* the integrand has degree <= 2 + 2 there, so Gauss-Legendre is exact.      */
/* ------------------------------------------------------------------------ */
static double bp_pixel(int N, double lx1, double lx2, int n, const double *theta, const detector *zeta,
                       double ly, int M, int K, const double *p, int k1, int k2)
{
    rect R = pixel_rect(lx1 * (k1 - 0.5 * (N - 1)), lx2 * (k2 - 0.5 * (N - 1)), lx1, lx2);
    double acc = 0.0;
    double br[OR_BRK + 1024];
    const double blur = zeta->nb > 0 ? 1.0 : 0.0;
    for (int a = 0; a < n; ++a) {
        double c = cos(theta[a]), s = sin(theta[a]);
        int d = or_degree(theta[a], blur);
        const double *prow = p + (size_t)a * (M + 2 * K);
        int nb = footprint_breaks(&R, c, s, zeta, br);
        double lo, hi;
        support(br, nb, &lo, &hi);
        /* knots of ghat: y_m (d odd) or y_m +- ly/2 (d even) */
        double off = (d % 2 == 0) ? 0.5 : 0.0;
        double z0 = lo / ly + 0.5 * (M - 1) - off, z1 = hi / ly + 0.5 * (M - 1) - off;
        for (int m = (int)ceil(z0); m <= (int)floor(z1) && nb < OR_BRK + 1024; ++m)
            br[nb++] = ly * (m + off - 0.5 * (M - 1));
        nb = sort_unique(br, nb);
        for (int i = 0; i + 1 < nb; ++i) {
            double h = 0.5 * (br[i + 1] - br[i]), mid = 0.5 * (br[i] + br[i + 1]);
            if (mid < lo || mid > hi) continue;
            for (int q = 0; q < 3; ++q) {
                double y = mid + h * GL_X[q];
                acc += h * GL_W[q] * footprint_rect(&R, c, s, zeta, y) *
                       ghat_eval(prow, M, K, ly, d, y);
            }
        }
    }
    return acc;
}

OR_API void or_backproject(int N, double lx1, double lx2, int n, const double *theta, const double *det,
                           double ly, int M, int K, const double *g, double *b)
{
    detector Dz = det_from(det);
    double *p = (double *)malloc(sizeof(double) * (size_t)n * (M + 2 * K));
    or_prefilter(n, theta, det, M, K, g, p);
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < N * N; ++i)
        b[i] = bp_pixel(N, lx1, lx2, n, theta, &Dz, ly, M, K, p, i % N, i / N);
    free(p);
}

OR_API void or_backproject_at(int N, double lx1, double lx2, int n, const double *theta,
                              const double *det, double ly, int M, int K, const double *g, int cnt,
                              const int *idx, double *b)
{
    detector Dz = det_from(det);
    double *p = (double *)malloc(sizeof(double) * (size_t)n * (M + 2 * K));
    or_prefilter(n, theta, det, M, K, g, p);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < cnt; ++i)
        b[i] = bp_pixel(N, lx1, lx2, n, theta, &Dz, ly, M, K, p, idx[i] % N, idx[i] / N);
    free(p);
}

/* ------------------------------------------------------------------------ */
/* Forward model (Sec. 2 and Sec. 4): g_s[theta, m] = (H c)(y_m)             */
/*   = sum_k c_k F_{k,theta}(y_m), point samples of the (blurred) projection. */
/* ------------------------------------------------------------------------ */
static double fp_bin(int N, double lx1, double lx2, double c, double s, const detector *zeta,
                     const double *img, double y)
{
    double half = 0.5 * (lx1 * fabs(c) + lx2 * fabs(s) + det_wmax(zeta));
    double acc = 0.0;
    for (int k2 = 0; k2 < N; ++k2) {
        double cy = lx2 * (k2 - 0.5 * (N - 1));
        for (int k1 = 0; k1 < N; ++k1) {
            double cx = lx1 * (k1 - 0.5 * (N - 1));
            if (fabs(cx * c + cy * s - y) >= half) continue;
            rect R = pixel_rect(cx, cy, lx1, lx2);
            acc += img[(size_t)k2 * N + k1] * footprint_rect(&R, c, s, zeta, y);
        }
    }
    return acc;
}

OR_API void or_forward(int N, double lx1, double lx2, int n, const double *theta, const double *det,
                       double ly, int M, const double *img, double *g)
{
    detector Dz = det_from(det);
    const detector *zeta = &Dz;
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int a = 0; a < n; ++a)
        for (int m = 0; m < M; ++m)
            g[(size_t)a * M + m] = fp_bin(N, lx1, lx2, cos(theta[a]), sin(theta[a]), zeta, img,
                                          ly * (m - 0.5 * (M - 1)));
}

/* Selected bins: idx[i] = angle * M + m. */
OR_API void or_forward_at(int N, double lx1, double lx2, int n, const double *theta, const double *det,
                          double ly, int M, const double *img, int cnt, const int *idx, double *g)
{
    detector Dz = det_from(det);
    const detector *zeta = &Dz;
    (void)n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < cnt; ++i) {
        int a = idx[i] / M, m = idx[i] % M;
        g[i] = fp_bin(N, lx1, lx2, cos(theta[a]), sin(theta[a]), zeta, img,
                      ly * (m - 0.5 * (M - 1)));
    }
}

/* <H c, ghat>_{L2} = sum_theta integral (sum_k c_k F_k(y)) ghat_theta(y) dy,
 * integrated over the whole detector line with the breakpoints of every
 * pixel and every knot of ghat (tiny N only).  This takes the inner product
 * on the sinogram side, independently of the pixel-by-pixel back projection,
 * for the adjoint test. */
OR_API double or_l2_inner(int N, double lx1, double lx2, int n, const double *theta, const double *det,
                          double ly, int M, int K, const double *img, const double *g)
{
    detector Dz = det_from(det);
    const detector *zeta = &Dz;
    const double blur = Dz.nb > 0 ? 1.0 : 0.0;
    double *p = (double *)malloc(sizeof(double) * (size_t)n * (M + 2 * K));
    or_prefilter(n, theta, det, M, K, g, p);
    int cap = OR_BRK * N * N + 2 * (M + 2 * K) + 8;
    double *br = (double *)malloc(sizeof(double) * (size_t)cap);
    double total = 0.0;
    for (int a = 0; a < n; ++a) {
        double c = cos(theta[a]), s = sin(theta[a]);
        int d = or_degree(theta[a], blur);
        int nb = 0;
        for (int k = 0; k < N * N; ++k) {
            rect R = pixel_rect(lx1 * (k % N - 0.5 * (N - 1)), lx2 * (k / N - 0.5 * (N - 1)), lx1,
                                lx2);
            nb += footprint_breaks(&R, c, s, zeta, br + nb);
        }
        double off = (d % 2 == 0) ? 0.5 : 0.0;
        for (int m = -K - 2; m <= M + K + 1; ++m) br[nb++] = ly * (m + off - 0.5 * (M - 1));
        nb = sort_unique(br, nb);
        for (int i = 0; i + 1 < nb; ++i) {
            double h = 0.5 * (br[i + 1] - br[i]), mid = 0.5 * (br[i] + br[i + 1]);
            for (int q = 0; q < 3; ++q) {
                double y = mid + h * GL_X[q];
                double proj = 0.0;
                for (int k = 0; k < N * N; ++k) {
                    rect R = pixel_rect(lx1 * (k % N - 0.5 * (N - 1)),
                                        lx2 * (k / N - 0.5 * (N - 1)), lx1, lx2);
                    proj += img[k] * footprint_rect(&R, c, s, zeta, y);
                }
                total += h * GL_W[q] * proj * ghat_eval(p + (size_t)a * (M + 2 * K), M, K, ly, d, y);
            }
        }
    }
    free(br);
    free(p);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradients on the normal equations (H^T H) x = b, textbook       */
/* Hestenes-Stiefel in FP64 with the direct-sum operator.  The paper itself  */
/* iterates with steepest descent (Sec. 6.2); both solve the same system.    */
/* hist[k] = ||r_k|| / ||b|| (recursive residual), k = 0..iters.  x holds    */
/* the start vector on entry (zeros for the plain form) and the iterate on   */
/* exit.  Returns the iteration count; stops at ||r|| <= rtol ||b||.         */
/* ------------------------------------------------------------------------ */
OR_API int or_cg(int N, const double *G, const double *b, double *x, int maxit, double rtol,
                 double *hist)
{
    size_t NN = (size_t)N * N;
    double *r = (double *)malloc(sizeof(double) * NN), *p = (double *)malloc(sizeof(double) * NN);
    double *Ap = (double *)malloc(sizeof(double) * NN);
    or_apply(N, G, x, Ap);
    double bb = 0.0, rr = 0.0;
    for (size_t i = 0; i < NN; ++i) {
        r[i] = b[i] - Ap[i];
        p[i] = r[i];
        bb += b[i] * b[i];
        rr += r[i] * r[i];
    }
    double bn = sqrt(bb);
    hist[0] = sqrt(rr) / bn;
    int k = 0;
    while (k < maxit && sqrt(rr) > rtol * bn) {
        or_apply(N, G, p, Ap);
        double pAp = 0.0;
        for (size_t i = 0; i < NN; ++i) pAp += p[i] * Ap[i];
        double alpha = rr / pAp, rr1 = 0.0;
        for (size_t i = 0; i < NN; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * Ap[i];
            rr1 += r[i] * r[i];
        }
        double beta = rr1 / rr;
        rr = rr1;
        for (size_t i = 0; i < NN; ++i) p[i] = r[i] + beta * p[i];
        ++k;
        hist[k] = sqrt(rr) / bn;
    }
    free(r);
    free(p);
    free(Ap);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Steepest descent on the same normal equations, the paper's own solver     */
/* (Sec. 6.2): r = b - A x, alpha = (r.r)/(r.A r), x += alpha r, r -= alpha  */
/* A r, in FP64 with the direct-sum operator.  hist, x and the return value  */
/* as for or_cg.                                                             */
/* ------------------------------------------------------------------------ */
OR_API int or_sd(int N, const double *G, const double *b, double *x, int maxit, double rtol,
                 double *hist)
{
    size_t NN = (size_t)N * N;
    double *r = (double *)malloc(sizeof(double) * NN), *Ar = (double *)malloc(sizeof(double) * NN);
    or_apply(N, G, x, Ar);
    double bb = 0.0, rr = 0.0;
    for (size_t i = 0; i < NN; ++i) {
        r[i] = b[i] - Ar[i];
        bb += b[i] * b[i];
        rr += r[i] * r[i];
    }
    double bn = sqrt(bb);
    hist[0] = sqrt(rr) / bn;
    int k = 0;
    while (k < maxit && sqrt(rr) > rtol * bn) {
        or_apply(N, G, r, Ar);
        double rAr = 0.0;
        for (size_t i = 0; i < NN; ++i) rAr += r[i] * Ar[i];
        double alpha = rr / rAr, rr1 = 0.0;
        for (size_t i = 0; i < NN; ++i) {
            x[i] += alpha * r[i];
            r[i] -= alpha * Ar[i];
            rr1 += r[i] * r[i];
        }
        rr = rr1;
        ++k;
        hist[k] = sqrt(rr) / bn;
    }
    free(r);
    free(Ar);
    return k;
}

/* Thread count of the parallel loops (for timing the oracle on a stated
 * number of host cores). */
int or_max_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
