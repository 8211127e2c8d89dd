/*
 * fdtd_nn.h -- C ABI of the surrogate network's kernels.
 *
 * A small U-Net maps a design density to the objective and its sensitivity
 * map (eq. (27)'s dF/drho); it is trained on (rho, F, dF/drho) triples that
 * the FDTD optimization produces and proposes design steps that full
 * forward + adjoint FDTD solves accept or reject.  These are its layers:
 *
 *   fdtd_nn_conv3x3        3x3 convolution, stride 1, zero padding 1, as an
 *                          implicit GEMM on BF16 matrix cores with FP32
 *                          accumulation: z = w * x + b
 *   fdtd_nn_conv3x3_dgrad  dL/dx of the same convolution (the forward GEMM with
 *                          the weights turned by 180 degrees and transposed);
 *                          _dgrad_relu fuses the ReLU backward of the layer below;
 *                          fdtd_nn_rot_weights turns many layers' weights at once
 *   fdtd_nn_conv3x3_wgrad  dL/dw and dL/db (GEMM over all pixels of the batch)
 *   fdtd_nn_relu_bf16      a = bf16(max(z, 0)) and its backward
 *   fdtd_nn_pool2 / up2    2x2 average pooling and 2x nearest upsampling (and
 *                          their transposes)
 *   fdtd_nn_gap_linear     scalar head: global average pooling and a linear
 *                          layer, and its backward
 *   fdtd_nn_mse            squared-error sum and its gradient
 *   fdtd_nn_adam           one Adam step on FP32 master weights, refreshing
 *                          the BF16 copy; fdtd_nn_axpy for gradient sums
 *
 * Layout: activations channel-major [C][N][H][W] (a channel concatenation is
 * two writes into one buffer; for one image this is NCHW); weights
 * [cout][3][3][cin] (eight input channels of one tap are one 16-byte load).
 * BF16 data
 * are passed as uint16_t (bits of the IEEE binary32 high half, rounded to
 * nearest even).  All pointers are device pointers; work runs in order on
 * `stream` (NULL: the default stream).  Functions return an fdtd_status and
 * never abort; EINVAL for non-positive sizes or missing pointers.  Sums over
 * the batch (weight and bias gradients, the head, the loss) are taken in a
 * fixed order, so results do not depend on scheduling.
 *
 * Device memory: the convolutions (forward and data gradient) on their
 * matrix-core path stage the input through a channel-last copy held by the
 * library, one buffer per (device, stream), allocated on first use and grown
 * (after a device synchronisation) when a larger input arrives; it is kept
 * until the process ends.  Calls on one stream are ordered, so they share
 * it safely; calls on different streams use different buffers.  Only
 * fdtd_nn_conv3x3_wgrad_noalloc allocates nothing.
 */
#ifndef FDTD_NN_H
#define FDTD_NN_H

#include <stdint.h>

#include "fdtd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* z[co][n][y][x] = b[co] + sum_{ci,ky,kx} w[co][ky][kx][ci] x[ci][n][y+ky-1][x+kx-1]
 * (x outside the image = 0; bias may be NULL).  Writes z (FP32) if z is not
 * NULL and a = bf16(max(z, 0)) if a is not NULL (at least one of them).
 * n <= 65535. */
fdtd_status fdtd_nn_conv3x3(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w, const uint16_t *x,
                            const uint16_t *wt, const float *bias, float *z, uint16_t *a, void *stream);

/* dx[ci][n][y][x] = sum_{co,ky,kx} w[co][ky][kx][ci] dz[co][n][y-ky+1][x-kx+1];
 * wrot: caller workspace of cout*cin*9 BF16 values, into which the weights
 * wt are turned first -- or, with wt = NULL, the turned weights themselves,
 * as fdtd_nn_rot_weights writes them (then nothing is written to wrot). */
fdtd_status fdtd_nn_conv3x3_dgrad(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w, const uint16_t *dz,
                                  const uint16_t *wt, uint16_t *wrot, float *dx, void *stream);

/* The data gradient fused with the backward of the ReLU whose BF16 output a
 * ([cin][n][h][w], the convolution's input) fed this layer:
 * dza = bf16(dx * (a > 0)) with dx as fdtd_nn_conv3x3_dgrad computes it --
 * the same BF16 values as fdtd_nn_conv3x3_dgrad followed by
 * fdtd_nn_relu_bf16_backward(a, dx), without the FP32 dx in memory (wt and
 * wrot as there, wt = NULL included).  dza must not overlap dz or a. */
fdtd_status fdtd_nn_conv3x3_dgrad_relu(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w, const uint16_t *dz,
                                       const uint16_t *wt, uint16_t *wrot, const uint16_t *a, uint16_t *dza,
                                       void *stream);

/* The turned weights of several layers in one launch, for data gradients
 * called with wt = NULL (e.g. once per optimizer step instead of once per
 * data gradient).  Layer l (0 <= l < nlayers <= 32; cin, cout, off are host
 * arrays of nlayers entries) has its weights at w + off[l], layout
 * [cout[l]][3][3][cin[l]]; its turned weights go to wrot + off[l], layout
 * [cin[l]][3][3][cout[l]] with the taps turned by 180 degrees: wrot[off +
 * (ci*9 + 8 - tap)*cout + co] = w[off + (co*9 + tap)*cin + ci].  The layers'
 * ranges must not overlap, and wrot must not overlap w.  EINVAL on a bad
 * count, size or offset. */
fdtd_status fdtd_nn_rot_weights(int32_t nlayers, const int32_t *cin, const int32_t *cout, const int64_t *off,
                                const uint16_t *w, uint16_t *wrot, void *stream);

/* dw[co][ky][kx][ci] = sum_{n,y,x} dz[co][n][y][x] x[ci][n][y+ky-1][x+kx-1];
 * db[co] = sum_{n,y,x} dz; work: caller workspace of fdtd_nn_wgrad_work(...)
 * floats. */
int64_t fdtd_nn_wgrad_work(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w);
fdtd_status fdtd_nn_conv3x3_wgrad(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w, const uint16_t *x,
                                  const uint16_t *dz, float *dw, float *db, float *work, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * dw and db as fdtd_nn_conv3x3_wgrad, bit for bit (same kernels and split
 * plan), with the partial sums in a scratch array the library holds on each
 * device (64 MiB = 16 Mi floats, kept until the process ends) instead of a
 * caller workspace.  Allocates nothing and calls no allocating routine; the
 * device is the current one.  EINVAL when fdtd_nn_wgrad_work(...) exceeds
 * 16 Mi floats (every layer of the surrogate fits: the plan's largest
 * workspace is about 14.2 Mi floats).  Calls on one device share the array:
 * calls that overlap on one GPU (different streams or threads) race and
 * must be serialized by the caller. */
fdtd_status fdtd_nn_conv3x3_wgrad_noalloc(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w,
                                          const uint16_t *x, const uint16_t *dz, float *dw, float *db, void *stream);

/* Elementwise: a = bf16(relu(z)); backward dz = bf16(da * (a > 0)) with the
 * layer's BF16 output a as the mask and an FP32 incoming gradient da. */
fdtd_status fdtd_nn_relu_bf16(int64_t count, const float *z, uint16_t *a, void *stream);
fdtd_status fdtd_nn_relu_bf16_backward(int64_t count, const uint16_t *a, const float *da, uint16_t *dz,
                                       void *stream);

/* Round FP32 to BF16 (nearest even) and back. */
fdtd_status fdtd_nn_to_bf16(int64_t count, const float *x, uint16_t *y, void *stream);
fdtd_status fdtd_nn_from_bf16(int64_t count, const uint16_t *x, float *y, void *stream);

/* 2x2 average pooling of `planes` planes h x w (h, w even) and its transpose
 * (FP32 gradients); 2x nearest upsampling of planes h x w and its transpose. */
fdtd_status fdtd_nn_pool2(int64_t planes, int32_t h, int32_t w, const uint16_t *x, uint16_t *y, void *stream);
fdtd_status fdtd_nn_pool2_backward(int64_t planes, int32_t h, int32_t w, const float *dy, float *dx, void *stream);
fdtd_status fdtd_nn_up2(int64_t planes, int32_t h, int32_t w, const uint16_t *x, uint16_t *y, void *stream);
fdtd_status fdtd_nn_up2_backward(int64_t planes, int32_t h, int32_t w, const float *dy, float *dx, void *stream);

/* One Adam step (bias-corrected, step t >= 1) on FP32 master weights p with
 * moments m, v and gradient g; writes the BF16 copy pb (may be NULL). */
fdtd_status fdtd_nn_adam(int64_t count, float *p, float *m, float *v, const float *g, uint16_t *pb, float lr,
                         float beta1, float beta2, float eps, int32_t t, void *stream);

/* y += a x (FP32). */
fdtd_status fdtd_nn_axpy(int64_t count, float a, const float *x, float *y, void *stream);

/* out[i] = bl[0] + sum_c wl[c] mean_p a[c][i][p] for i < n (a: c x n x hw BF16).
 * Backward: da[c][i][p] = dout[i] wl[c] / hw (FP32), dwl[c] = sum_i dout[i]
 * mean_p a[c][i][p], dbl[0] = sum_i dout[i]. */
fdtd_status fdtd_nn_gap_linear(int32_t n, int32_t c, int32_t hw, const uint16_t *a, const float *wl, const float *bl,
                               float *out, void *stream);
fdtd_status fdtd_nn_gap_linear_backward(int32_t n, int32_t c, int32_t hw, const uint16_t *a, const float *wl,
                                        const float *dout, float *da, float *dwl, float *dbl, void *stream);

/* sum_sq[0] = sum_i (pred[i] - target[i])^2 in FP64 (device scalar);
 * grad[i] = 2 scale (pred[i] - target[i]) unless grad is NULL.  work: caller
 * workspace of fdtd_nn_mse_work(count) doubles. */
int64_t fdtd_nn_mse_work(int64_t count);
fdtd_status fdtd_nn_mse(int64_t count, const float *pred, const float *target, float scale, float *grad,
                        double *work, double *sum_sq, void *stream);

/* Message of the last failing call of this header's functions on the calling
 * thread. */
const char *fdtd_nn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_NN_H */
