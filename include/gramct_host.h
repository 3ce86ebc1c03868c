/*
 * gramct host-only helpers: the exact piecewise-polynomial box-spline code
 * that builds the back-projection tables, exposed for inspection and for
 * CPU-side tests.  None of these touch a GPU; all arrays are HOST arrays.
 */
#ifndef GRAMCT_HOST_H
#define GRAMCT_HOST_H

#include "gramct.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Centred univariate box spline (Sec. 3, eq. boxconv: the convolution of the
 * elementary boxes M_w, each of unit integral on [-w/2, w/2]) with the
 * ndirs directions dirs[] (absolute values are used; zero directions are the
 * identity), times `scale`, evaluated at x[0..npts-1] into out[].  Built as
 * an exact piecewise polynomial in FP64.  1 <= ndirs <= 8, at least one
 * direction non-zero.  Returns GCT_OK or GCT_EINVAL. */
int gct_host_boxspline_eval(const double *dirs, int ndirs, double scale, const double *x,
                            int npts, double *out);

/* Back-projection weights of one angle (Sec. 5): for a pixel whose centre
 * projects to fractional bin index z = m0 + t, t in [0, 1), the weights
 * w[j] multiply the prefiltered sinogram entries p[m0 + jlo + j],
 * j < nw.  w must hold 64 doubles.  These are the same sub-interval
 * polynomials the device kernel evaluates. */
int gct_host_bp_weights(const gct_geometry *geom, int angle, double t, double *w, int *jlo,
                        int *nw);

/* B-spline degree used for angle theta (Sec. 5 continuity rule): 1 in
 * general and 0 axis-aligned without blur; 2 in general and 1 axis-aligned
 * with blur (zeta_blur > 0). */
int gct_host_degree(double theta, double zeta_blur);

#ifdef __cplusplus
}
#endif
#endif /* GRAMCT_HOST_H */
