/*
 * gramct_unet -- learned warm start for the CG solve of gramct.h: a small
 * U-Net maps the back projection b = H^T g of a slice to an initial iterate
 * x0 for cg_solve, trained on the GPU by the kernels behind this interface.
 * CG from x0 = 0 stays the fallback (gct_cg_solve drops a warm start whose
 * residual is not below ||b||) and the measure of the net's error: the solve
 * always runs to the same stopping rule ||b - A x_k|| <= rtol ||b||.
 *
 * The paper (Sec. 6) reconstructs with plain iterations from zero; the warm
 * start is an addition of this library and has no equation in the paper.
 *
 * Network (levels L, base channels C0, C_l = C0 2^l):
 *   encoder level l = 0..L-1 at (H/2^l) x (W/2^l): two 3x3 convolutions
 *   (zero padding 1) with bias and ReLU; between levels 2x2 max pooling;
 *   decoder level l = L-2..0: 2x2 stride-2 transposed convolution with bias
 *   (no activation), concatenated with the encoder's level-l output as
 *   [up | skip], two 3x3 convolutions with bias and ReLU; a final 1x1
 *   convolution with bias to one channel.  The input image is multiplied by
 *   in_scale, the output by out_scale.
 * Arithmetic: activations and weights BF16 (round to nearest even),
 * products accumulated in FP32 on the matrix cores, FP32 master weights and
 * Adam moments.  Loss: mean squared error over all pixels of the batch.
 *
 * Parameters are one flat FP32 vector, layer after layer in this order:
 * encoder (conv1, conv2) for l = 0..L-1, then per decoder level
 * l = L-2..0 (transposed conv, conv1, conv2), then the final 1x1.  Each
 * layer stores its weight then its bias, each starting at a multiple of 64
 * elements (gaps are zero).  Weight layouts (Cin contiguous):
 *   3x3 conv:        w[t][co][ci], t = 3 dy + dx, output(i, j) takes input
 *                    (i + dy - 1, j + dx - 1); the first layer has Cin = 16
 *                    of which only channel 0 is fed (the others see zeros);
 *   transposed conv: w[2a + b][co][ci]: input pixel (i, j) feeds output
 *                    pixel (2i + a, 2j + b);
 *   final 1x1:       w[0][0][ci].
 * gct_unet_layer_info reports each layer's offsets and sizes.
 *
 * Images are FP32 [batch][H][W] device arrays.  Every pointer is a DEVICE
 * pointer unless a comment says "host"; `stream` is a hipStream_t (NULL =
 * default stream); calls are stream-ordered.  Return values and
 * gct_last_error() as in gramct.h.
 *
 * Memory: gct_unet_create allocates the parameters, gradients, moments,
 * their BF16 copies and the activations of every layer for max_batch images
 * (about 2 x 176 C0/32 bytes per pixel per image at level 0, summed over
 * levels); the other calls allocate nothing.  One gct_unet serves one stream
 * at a time: calls on different streams that overlap race.
 */
#ifndef GRAMCT_UNET_H
#define GRAMCT_UNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gct_unet gct_unet;

typedef struct gct_unet_config {
    int32_t levels;         /* L in [1, 6] */
    int32_t base_channels;  /* C0: a multiple of 16, C0 2^(L-1) <= 1024 */
    int32_t height, width;  /* H, W: positive multiples of 2^(L-1) */
    int32_t max_batch;      /* >= 1, max_batch H W <= 2^28 */
} gct_unet_config;

enum { GCT_UNET_CONV3 = 0, GCT_UNET_UPCONV = 1, GCT_UNET_FINAL = 2 };

typedef struct gct_unet_layer {
    int32_t kind;           /* GCT_UNET_CONV3 / UPCONV / FINAL */
    int32_t taps;           /* 9, 4 or 1 */
    int32_t in_channels;    /* Cin of the weight layout */
    int32_t out_channels;   /* co */
    int64_t weight_offset;  /* elements into the flat parameter vector */
    int64_t bias_offset;
} gct_unet_layer;

/* Create a network with all parameters zero (set them with
 * gct_unet_set_params).  Synchronises the device once.  Errors: GCT_EINVAL
 * for a config outside the ranges above, GCT_EHIP if allocation fails. */
int gct_unet_create(const gct_unet_config *cfg, gct_unet **out);
int gct_unet_destroy(gct_unet *u);

/* Length of the flat parameter vector (host output). */
int gct_unet_param_count(const gct_unet *u, int64_t *n);
int gct_unet_layer_count(const gct_unet *u, int32_t *n);
/* Layer i in the order above (host output). */
int gct_unet_layer_info(const gct_unet *u, int32_t i, gct_unet_layer *info);

/* Copy the flat FP32 parameters in (and refresh the BF16 copies) or out. */
int gct_unet_set_params(gct_unet *u, const float *params, void *stream);
int gct_unet_get_params(const gct_unet *u, float *params, void *stream);
/* Gradients of the last gct_unet_backward, same layout. */
int gct_unet_get_grads(const gct_unet *u, float *grads, void *stream);
/* Adam moments, same layout; set with m = v = NULL zeroes them. */
int gct_unet_get_moments(const gct_unet *u, float *m, float *v, void *stream);
int gct_unet_set_moments(gct_unet *u, const float *m, const float *v, void *stream);

/* y = out_scale * net(in_scale * x) for `batch` images (1 <= batch <=
 * max_batch); keeps the activations for gct_unet_backward.  x, y: FP32
 * [batch][H][W]; y must not alias x.  The launch sequence is captured as a
 * HIP graph on the first call with a given (batch, x, y, in_scale,
 * out_scale) and replayed by later calls with the same arguments (the
 * newest 8 are kept; a capture costs about a millisecond of host time), so
 * callers in a loop should reuse their x and y buffers.  A replay reads the
 * current contents of x and the current weights.  Not to be called while
 * the calling thread captures a graph of its own. */
int gct_unet_forward(gct_unet *u, int32_t batch, const float *x, float in_scale, float out_scale, float *y,
                     void *stream);

/* Loss mean((y - target)^2) over batch H W pixels into *loss (a device
 * float; NULL = internal) and the gradient of the loss with respect to every
 * parameter, kept for gct_unet_get_grads / gct_unet_adam_step.  y must be
 * the output of the preceding gct_unet_forward with the same batch, and
 * that forward's x must still hold the same values (the backward rebuilds
 * the prepared input from it). */
int gct_unet_backward(gct_unet *u, int32_t batch, const float *y, const float *target, float *loss,
                      void *stream);

/* One Adam step (bias-corrected; `step` counts from 1) on the master
 * weights with the last gradients, then refresh of the BF16 copies. */
int gct_unet_adam_step(gct_unet *u, float lr, float beta1, float beta2, float eps, int32_t step,
                       void *stream);

#ifdef __cplusplus
}
#endif

#endif
