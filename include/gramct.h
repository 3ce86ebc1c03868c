/*
 * gramct -- pixel-basis (box-spline) Gram filtering, box-spline back
 * projection and CG on the normal equations for parallel-beam X-ray CT,
 * hand-written HIP for AMD Instinct MI355X (gfx950).
 *
 * Method: Shu & Entezari, "Gram Filtering and Sinogram Interpolation for
 * Pixel-basis in Parallel-beam X-ray CT Reconstruction" (arXiv 2005.13471).
 *
 * C ABI.  Plain pointers and sizes only.  Conventions shared by every call:
 *
 *   - Pixel k = (k1, k2), 0 <= k1, k2 < N, is the indicator of the rectangle
 *     of sides lambda_x[0] x lambda_x[1] centred at
 *     x_k = (lambda_x[0] (k1 - (N-1)/2), lambda_x[1] (k2 - (N-1)/2))
 *     (Sec. 2: f = sum_k c_k psi(x - Lambda_x k) with psi the pixel, i.e. the
 *     two-direction bivariate box spline of Sec. 3).  Images are row-major
 *     [k2][k1], N*N elements.
 *   - Angle theta_i has detector axis u = (cos theta_i, sin theta_i); a ray is
 *     the line {x : x.u = y}.  Detector bin m in [0, M) sits at
 *     y_m = lambda_y (m - (M-1)/2).  Sinograms are row-major [angle][bin].
 *   - The detector blur is the unit-integral box of width zeta_blur (Sec. 2);
 *     zeta_blur = 0 means no blur.
 *   - Gram filter G: (2N-1) x (2N-1), row-major, tap (k1, k2) at
 *     [(k2 + N-1) * (2N-1) + (k1 + N-1)]; G[k] = G[-k].
 *   - All array pointers are DEVICE pointers owned by the caller, unless a
 *     comment says "host".  Data arrays are float (GCT_F32) or double
 *     (GCT_F64) as selected by the dtype argument.  `stream` is a
 *     hipStream_t (NULL = the default stream).  Calls are stream-ordered and
 *     do not block the host, except where stated.
 *   - Return value: GCT_OK (0) or a negative error code; gct_last_error()
 *     returns a thread-local message for the last failure.  No C++
 *     exception crosses this interface.
 *
 * Device memory: every data array and every scratch workspace is passed in
 * by the caller; gct_workspace_size reports the bytes each operation needs.
 * The one exception is the geometry a plan (or batch) is made of: the plan's
 * per-angle tables (box-spline parameters, back-projection polynomials, FFT
 * twiddles, correction-filter taps: O(n_angles) bytes, a few hundred per
 * angle) and a batch's block maps and slice descriptors (O(total transform
 * blocks)) are built on the host in FP64 at creation, uploaded once and
 * freed at destruction.  They are read-only, their layout is internal (it
 * changes with the kernels), and they live exactly as long as the handle,
 * so the handle owns them rather than the caller; gct_plan_device_bytes and
 * gct_batch_device_bytes report their size.  A plan also keeps the solvers'
 * captured iteration graphs and one pinned host copy of the solver state, so
 * solves on one plan (and one batch) must not run from two host threads at
 * once; the stream-ordered calls may share a plan freely.
 */
#ifndef GRAMCT_H
#define GRAMCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCT_OK 0
#define GCT_EINVAL (-1)      /* bad argument: null pointer, size, geometry, aliasing */
#define GCT_EHIP (-2)        /* a HIP runtime call or kernel launch failed */
#define GCT_ENOTCONV (-3)    /* cg_solve: max_iter reached; x holds the last iterate */
#define GCT_EBREAKDOWN (-4)  /* cg_solve: p.Ap <= 0 or a non-finite value */

typedef enum { GCT_F32 = 0, GCT_F64 = 1 } gct_dtype;

/* Problem statement of Sec. 2: N^2 pixel coefficients, Lambda_x =
 * diag(lambda_x), the angle set, the detector sampling step lambda_y and bin
 * count M, the blur width zeta_blur, and the truncation K of the quadratic
 * B-spline correction filter of Sec. 5 (q[m] kept for |m| <= K; the paper
 * truncates at 40).  `theta` is a HOST array of n_angles radians, read only
 * during gct_plan_create.  Limits: 1 <= N <= 2048, n_angles >= 1, M >= 1,
 * lambda_x, lambda_y > 0, zeta_blur >= 0, 0 <= prefilter_K <= 256. */
typedef struct {
    int32_t N;
    double lambda_x[2];
    int32_t n_angles;
    const double *theta;
    double lambda_y;
    int32_t M;
    double zeta_blur;
    int32_t prefilter_K;
} gct_geometry;

typedef struct gct_plan gct_plan;

#define GCT_MAX_BOXES 4

/* Sizes (in elements) of the arrays a plan works on. */
typedef struct {
    int32_t N, n_angles, M, prefilter_K;
    int32_t fft_size;        /* P >= 2N-1 of the circulant embedding: the smallest power of two,
                                or three times a power of two (1536, 3072) where that is smaller */
    int64_t gram_elems;      /* (2N-1)^2 */
    int64_t spectrum_elems;  /* (P/2+1) * P, real */
    int64_t image_elems;     /* N^2 */
    int64_t sino_elems;      /* n_angles * M */
    int64_t prefiltered_elems; /* n_angles * (M + 2K) */
    int32_t gram_symmetry;   /* 8: G has the square's eight symmetries (square pixels, an angle
                                set closed under theta -> theta + pi/2 and theta -> -theta mod pi,
                                e.g. theta_i = i pi / n with n even), so gct_gram_build
                                evaluates one octant of taps; 2: G[k] = G[-k] only, half the
                                taps evaluated */
} gct_plan_info;

/* Validate the geometry and build the per-angle tables: box-spline
 * parameters of the Gram filter (Sec. 4), exact piecewise-polynomial
 * back-projection kernels (Sec. 5), B-spline degrees from the continuity
 * rule of Sec. 5, correction-filter taps and FFT twiddles, in FP64 on the
 * host, then copied to the current device (blocking).  *plan is owned by the
 * caller and released with gct_plan_destroy. */
int gct_plan_create(const gct_geometry *geom, gct_plan **plan);
/* As gct_plan_create with a detector kernel made of several boxes of
 * different heights and lengths (Sec. 2, the detector cell model before the
 * paper's simplification to one box): K(t) = sum_i box_height[i] for
 * |t| <= box_width[i]/2, 1 <= n_boxes <= GCT_MAX_BOXES (HOST arrays, read
 * during the call; widths > 0, heights non-zero).  The measurement of bin m
 * is then the projection integrated against K(y_m - y); one box of width
 * zeta and height 1/zeta is gct_plan_create with zeta_blur = zeta.
 * geom->zeta_blur must be 0.  Every operation of the plan uses this kernel:
 * the footprint is sum_i h_i w_i l1 l2 M_[l1|c|, l2|s|, w_i] (Sec. 4 eq.
 * blurxray_of_f per box), the Gram filter the angle sum of the
 * autocorrelation of that footprint (each pair of boxes as a difference of
 * two six-direction closed forms), back projection the exact adjoint with the
 * blurred degree rule of Sec. 5.  The Gram filter's FP32 accuracy needs box
 * widths and half-differences of widths that are not tiny against the pixel
 * (>= 0.1 l); FP64 has no such limit. */
int gct_plan_create_detector(const gct_geometry *geom, int32_t n_boxes, const double *box_width,
                             const double *box_height, gct_plan **plan);
int gct_plan_destroy(gct_plan *plan);
int gct_plan_get_info(const gct_plan *plan, gct_plan_info *info);

/* Bytes of device memory the plan's tables hold (HOST int64 out). */
int gct_plan_device_bytes(const gct_plan *plan, int64_t *bytes);

/* Operation ids for gct_workspace_size. */
enum {
    GCT_OP_GRAM_BUILD = 0,
    GCT_OP_GRAM_SPECTRUM = 1,
    GCT_OP_GRAM_APPLY = 2,
    GCT_OP_PREFILTER = 3,
    GCT_OP_BACKPROJECT = 4,
    GCT_OP_FORWARD = 5,
    GCT_OP_CG = 6
};

/* Bytes of device workspace operation `op` needs in `dtype` (0 if none).
 * Workspace must be 256-byte aligned; its contents on entry are ignored. */
size_t gct_workspace_size(const gct_plan *plan, int op, gct_dtype dtype);

/* Gram filter (Sec. 4): G[k] = sum over angles of the autocorrelation of
 * the projected pixel, a univariate box spline with directions
 * {l1|c|, l1|c|, l2|s|, l2|s|} (plus {zeta, zeta} with blur), evaluated at
 * the projected tap offset l1 k1 c + l2 k2 s, times (l1 l2)^2.  Exact up to
 * floating-point rounding.  Output G: gram_elems. */
int gct_gram_build(const gct_plan *plan, gct_dtype dtype, void *G, void *stream);

/* Real, even spectrum of the P x P circulant embedding of G (taps with
 * |k1| or |k2| = P/2 .. are zero), pre-scaled by 1/P^2 so that gram_apply
 * needs no further normalisation.  Layout [w1][w2], w1 in [0, P/2],
 * w2 in [0, P): spectrum_elems reals.  Needs workspace. */
int gct_gram_spectrum(const gct_plan *plan, gct_dtype dtype, const void *G, void *Ghat,
                      void *ws, void *stream);

/* Normal operator as Gram filtering (Sec. 4, Toeplitz-block-Toeplitz
 * remark): y[i] = sum_{j in [0,N)^2} G[i - j] c[j], a zero-padded linear
 * convolution of the N x N coefficients with the (2N-1)^2 filter, computed
 * exactly (up to rounding) through the P x P circulant embedding.
 * c, y: image_elems; y must not alias c.  Needs workspace. */
int gct_gram_apply(const gct_plan *plan, gct_dtype dtype, const void *Ghat, const void *c,
                   void *y, void *ws, void *stream);

/* gct_gram_apply without the workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The scratch of the three passes is a
 * static device array of 24 MiB per GPU, held until the process ends:
 * enough for N <= 1024 in FP32 and N <= 767 in FP64 (the call needs
 * gct_workspace_size(plan, GCT_OP_GRAM_APPLY, dtype) bytes; larger plans
 * return GCT_EINVAL).  The current device must be the plan's.  Allocates
 * nothing and calls no allocating routine.  Every call on one GPU shares the
 * array: calls that may overlap in time (other streams, other host threads)
 * race and must be serialised by the caller.  Same kernels and results as
 * gct_gram_apply. */
int gct_gram_apply_static(const gct_plan *plan, gct_dtype dtype, const void *Ghat, const void *c,
                          void *y, void *stream);

/* Digital correction filter of Sec. 5 (eq. correction filter) per angle
 * row: p = q_d * g_s with g_s zero outside [0, M); q_d = delta for
 * B-spline degree d <= 1 and q[m] = sqrt(2) (2 sqrt(2) - 3)^|m|, |m| <= K,
 * for d = 2.  p: [angle][M + 2K], element m + K holds bin m. */
int gct_prefilter(const gct_plan *plan, gct_dtype dtype, const void *g_s, void *p, void *stream);

/* Back projection with the exact adjoint and box-spline sinogram
 * interpolation (Sec. 5): b[k] = sum_theta integral F_k(y) ghat_theta(y) dy,
 * ghat_theta(y) = sum_m p[m] beta_d((y - y_m)/lambda_y).  Each (pixel, angle,
 * bin) weight is a univariate box spline with directions {l1|c|, l2|s|,
 * zeta, lambda_y x (d+1)}, evaluated exactly from per-angle piecewise
 * polynomials.  g_s: sino_elems; b: image_elems.  Workspace
 * (gct_workspace_size(plan, GCT_OP_BACKPROJECT, dtype) bytes) holds the
 * prefiltered sinogram, the per-angle polynomial tables of the weighted
 * sinogram sums (one row per angle, detector bin reached by the image and
 * sub-interval) and the partial images of the angle groups. */
int gct_backproject_boxspline(const gct_plan *plan, gct_dtype dtype, const void *g_s, void *b,
                              void *ws, void *stream);

/* Forward model (Sec. 2, Sec. 4 eq. xray_of_f and eq. blurxray_of_f):
 * g_s[theta, m] = sum_k c_k l1 l2 M_{l1|c|, l2|s|, zeta}(y_m - x_k.u).
 * Supporting operation (sinogram synthesis, adjoint tests). */
int gct_forward_project(const gct_plan *plan, gct_dtype dtype, const void *c, void *g_s,
                        void *stream);

/* Autotuner of the Gram-filtering passes (the FFT realisation of Sec. 4's
 * Toeplitz-block-Toeplitz product): times one apply for each candidate
 * number of elements per thread of the transforms (16, 8 or 4 where the
 * transform size allows; fewer elements mean more threads per transform),
 * chosen independently for the two row passes and for the column pass, and
 * keeps the fastest pair in the plan for `dtype`; separately for the fused
 * CG passes of gct_cg_solve, timed on a trial solve.  Results of later applies
 * and solves agree with the untuned ones to rounding.  ws must be a CG
 * workspace of the plan (gct_workspace_size(plan, GCT_OP_CG, dtype)); its
 * contents are overwritten.  reps: timed repetitions per candidate (<= 0:
 * 3).  chosen: optional HOST int receiving the choice for the row passes of
 * the apply (gct_plan_get_pass_elems reports all four).  Changes the plan:
 * do not call while other streams use it.  Blocks the host. */
int gct_plan_autotune(gct_plan *plan, gct_dtype dtype, const void *Ghat, void *ws, int32_t reps,
                      int32_t *chosen, void *stream);

/* Set the elements per thread of the Gram-filtering transforms for `dtype`
 * directly (a candidate the autotuner would consider: 16, 8 or 4 as the
 * transform size allows; otherwise GCT_EINVAL); elems_per_thread = 0
 * restores the default.  Changes the plan like gct_plan_autotune. */
int gct_plan_set_fft_elems(gct_plan *plan, gct_dtype dtype, int32_t elems_per_thread);

/* As gct_plan_set_fft_elems with separate values for the two row passes
 * (rows_elems) and the column pass (cols_elems), for the apply and the fused
 * CG passes alike; 0 selects the default for that pass. */
int gct_plan_set_pass_elems(gct_plan *plan, gct_dtype dtype, int32_t rows_elems, int32_t cols_elems);

/* The plan's current elements per thread for `dtype`: out (HOST, 4 ints) =
 * {apply row passes, apply column pass, CG row passes, CG column pass}. */
int gct_plan_get_pass_elems(const gct_plan *plan, gct_dtype dtype, int32_t *out);

/* Launch shape the plan chose for gct_backproject_boxspline in `dtype`
 * (Sec. 5 back projection; the arithmetic is the same on every path): out
 * (HOST, 4 ints) = {angles per chunk of the pixel-tiled kernel, whose
 * per-(tile, angle) tables must fit in 64 KB of LDS (0: they do not, and the
 * per-angle kernel runs instead), angle groups of the tiled kernel (1 when
 * it does not run), tile side of the per-angle kernel (32, 16 or 8; 0
 * when the tiled kernel runs; also 0 when neither fits, and back projection
 * then returns GCT_EHIP), sub-interval breakpoints the tiled kernel holds in
 * registers per angle (5, 9 or, FP32 only, 16: at least the most
 * sub-intervals of any angle; 0 when they are searched in LDS or the tiled
 * kernel does not run)}.  Fine detector sampling (small lambda_y relative to
 * the pixel) and FP64 widen the tables; detectors of several boxes add
 * sub-intervals. */
int gct_plan_get_bp_shape(const gct_plan *plan, gct_dtype dtype, int32_t *out);

/* Result of gct_cg_solve (host struct). */
typedef struct {
    int32_t iters;        /* iterations performed */
    int32_t status;       /* GCT_OK, GCT_ENOTCONV or GCT_EBREAKDOWN */
    double rel_res;       /* recursive ||r_k|| / ||b|| at exit */
    double rel_res_true;  /* ||b - A x_k|| / ||b|| recomputed at exit */
    double rel_res0;      /* ||b - A x_0|| / ||b|| of the start actually used */
    int32_t fell_back;    /* 1 if the given start vector was no better than zero
                             (||b - A x_0|| >= ||b|| or non-finite) and CG restarted
                             from x_0 = 0 */
} gct_cg_result;

/* Conjugate gradients on (H^T H) x = b with the Gram-filter operator
 * (Sec. 2: a single back projection, then the filter in every iteration;
 * the paper iterates with steepest descent, Sec. 6.2).  Vectors in dtype;
 * inner products and residual norms in FP64 on the device.  Iterations use
 * the Chronopoulos-Gear arrangement of CG (one Gram-filter product w = A r
 * and one reduction point per iteration, A p carried by recurrence), fused
 * into the three Gram-filtering passes: in exact arithmetic the textbook CG
 * iterates; the stopping test uses ||r_k||^2 reduced from r_k.  Stops when
 * ||r_k|| <= rtol ||b|| or after max_iter iterations.  x: on entry the start
 * vector if use_x0 != 0 (else ignored and zero is used); on exit the last
 * iterate.  A start vector with ||b - A x_0|| >= ||b|| is replaced by zero
 * (result->fell_back = 1).  Success (GCT_OK) means the recomputed residual
 * ||b - A x||/||b|| of the returned iterate is <= rtol: when the recursive
 * residual meets the rule but the recomputed one does not (rounding drift),
 * CG restarts from the current iterate with r = b - A x (at most 4 times,
 * within max_iter iterations in total), else GCT_ENOTCONV.  hist: optional
 * HOST array of max_iter + 1 doubles receiving ||r_k||/||b|| (at a restart
 * the recomputed residual).  check_every: iterations between host convergence checks
 * (<= 0 selects 8); iterations after convergence are skipped on the device.
 * BLOCKS the host until the solve is complete. */
int gct_cg_solve(const gct_plan *plan, gct_dtype dtype, const void *Ghat, const void *b, void *x,
                 int use_x0, double rtol, int32_t max_iter, int32_t check_every, double *hist,
                 gct_cg_result *result, void *ws, void *stream);

/* Steepest descent on the same system, the paper's own solver (Sec. 6.2):
 * r = b - A x, alpha = (r.r)/(r.A r), x += alpha r, r -= alpha A r, one
 * Gram-filter product per iteration, fused into the three Gram-filtering
 * passes like gct_cg_solve (same FP64 inner products, stopping rule,
 * start-vector fallback, arguments, workspace and errors; GCT_EBREAKDOWN for
 * r.A r <= 0 or a non-finite value).  BLOCKS the host. */
int gct_sd_solve(const gct_plan *plan, gct_dtype dtype, const void *Ghat, const void *b, void *x,
                 int use_x0, double rtol, int32_t max_iter, int32_t check_every, double *hist,
                 gct_cg_result *result, void *ws, void *stream);

/* ------------------------------------------------------------------------
 * Batches of independent slices (uneven N, angle sets and blur widths).
 *
 * A batch groups existing plans (not owned: they must outlive the batch).
 * Its data arrays are PACKED: slice i occupies [offset_i, offset_i + size_i)
 * of each array, with the per-slice layouts of the single-slice calls
 * (images N_i^2, Gram filters (2N_i - 1)^2, spectra (P_i/2 + 1) P_i);
 * gct_batch_get_info reports the offsets.  Each phase is one launch over all
 * slices (one per FFT size for the transform passes), so a batch keeps the
 * GPU busy where one small slice cannot.  The method per slice is exactly
 * that of the single-slice calls (Sec. 4: Gram filter and Gram filtering;
 * CG on the normal equations).
 * ------------------------------------------------------------------------ */
typedef struct gct_batch gct_batch;

typedef struct {
    int32_t slices;
    int32_t groups;          /* distinct FFT sizes */
    int64_t image_elems;     /* sum of N_i^2 */
    int64_t gram_elems;      /* sum of (2N_i - 1)^2 */
    int64_t spectrum_elems;  /* sum of (P_i/2 + 1) P_i */
} gct_batch_info;

/* plans: host array of `count` plan pointers, all created on the current
 * device.  Uploads the block maps and slice descriptors (blocking). */
int gct_batch_create(const gct_plan *const *plans, int32_t count, gct_batch **batch);
int gct_batch_destroy(gct_batch *batch);

/* Bytes of device memory the batch's maps and descriptors hold (HOST out;
 * the plans' own tables not included). */
int gct_batch_device_bytes(const gct_batch *batch, int64_t *bytes);

/* Sizes; the three offset arrays (host, `slices` entries each) may be NULL. */
int gct_batch_get_info(const gct_batch *batch, gct_batch_info *info, int64_t *image_offsets,
                       int64_t *gram_offsets, int64_t *spectrum_offsets);

/* Workspace bytes for GCT_OP_GRAM_SPECTRUM, GCT_OP_GRAM_APPLY or GCT_OP_CG. */
size_t gct_batch_workspace_size(const gct_batch *batch, int op, gct_dtype dtype);

/* Packed Gram filters of every slice (as gct_gram_build per slice). */
int gct_batch_gram_build(const gct_batch *batch, gct_dtype dtype, void *G, void *stream);

/* Packed spectra of every slice (as gct_gram_spectrum per slice). */
int gct_batch_gram_spectrum(const gct_batch *batch, gct_dtype dtype, const void *G, void *Ghat,
                            void *ws, void *stream);

/* y_i = H_i^T H_i c_i for every slice (as gct_gram_apply per slice). */
int gct_batch_gram_apply(const gct_batch *batch, gct_dtype dtype, const void *Ghat, const void *c,
                         void *y, void *ws, void *stream);

/* CG from x_i = 0 on every slice to ||r_i|| <= rtol ||b_i|| (per slice) or
 * max_iter iterations; converged slices stop while the others continue.
 * Textbook arrangement (products A p, then the x, r update and ||r||^2,
 * then beta), FP64 inner products as in gct_cg_solve.  As there, success
 * means the recomputed residual of the returned iterate meets rtol: slices
 * whose recursive residual alone met it restart from their iterate with
 * r = b - A x (at most 4 times, within max_iter iterations per slice), else
 * they report GCT_ENOTCONV.
 * results: HOST array of `slices` entries.  Returns GCT_OK if all slices
 * converged, else GCT_ENOTCONV / GCT_EBREAKDOWN (see results[i].status).
 * Chunks of check_every iterations (<= 0 selects 8) are replayed as a
 * captured HIP graph.  BLOCKS the host until the solve is complete. */
int gct_batch_cg_solve(const gct_batch *batch, gct_dtype dtype, const void *Ghat, const void *b,
                       void *x, double rtol, int32_t max_iter, int32_t check_every,
                       gct_cg_result *results, void *ws, void *stream);

/* As gct_batch_cg_solve, starting from the iterates in x (the learned warm
 * start of a stack of slices, Sec. 6.2's iteration from a given image): per
 * slice r = b - A x_0; a slice whose ||b - A x_0|| >= ||b|| (or not finite)
 * starts from zero instead (results[i].fell_back = 1), and
 * results[i].rel_res0 reports the start actually used. */
int gct_batch_cg_solve_x0(const gct_batch *batch, gct_dtype dtype, const void *Ghat, const void *b,
                          void *x, double rtol, int32_t max_iter, int32_t check_every,
                          gct_cg_result *results, void *ws, void *stream);

/* Autotuner: for each FFT size of the batch, times the batched apply with
 * each candidate number of elements per thread of the transforms (the work
 * tile of one thread), for the row passes and for the column pass in turn,
 * and keeps the fastest for `dtype`.  ws must be a CG workspace of the
 * batch; reps timed repetitions per candidate (<= 0: 3).  chosen: optional
 * HOST array of `groups` entries receiving the choice for the row passes.
 * Blocks the host. */
int gct_batch_autotune(gct_batch *batch, gct_dtype dtype, const void *Ghat, void *ws,
                       int32_t reps, int32_t *chosen, void *stream);

/* The batch's current elements per thread for `dtype`: out (HOST, 2 x groups
 * ints) = {row passes, column pass} for each FFT size in increasing order. */
int gct_batch_get_pass_elems(const gct_batch *batch, gct_dtype dtype, int32_t *out);

/* Thread-local description of the last error (never NULL). */
const char *gct_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GRAMCT_H */
