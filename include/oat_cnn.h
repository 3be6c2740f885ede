/*
 * oat_cnn.h -- C ABI of the small 3-D convolution network used as a learned
 * preconditioner for the penalised least-squares reconstruction (training
 * and inference on gfx950).  The network and its use are not part of the
 * paper: they extend the PLS iteration of Sec. IV.A-B, whose gradient they
 * map to a search direction.
 *
 * Volumes are C-contiguous [C][D][H][W] (W fastest), one sample per call;
 * zero padding of one voxel on every face ("same" 3x3x3 convolution).
 * Activations may be stored in FP32 or BF16 (oat_dtype of oat.h); all
 * arithmetic accumulates in FP32.  Weights, biases, gradients and optimiser
 * state are FP32.  Weight layout: [C_out][C_in][3][3][3].
 *
 * Every pointer is a DEVICE pointer owned by the caller; calls are
 * asynchronous on `stream` (hipStream_t, NULL = default stream).  Channel
 * counts must be 1 or 16.  Returns an oat_status (oat.h); sizes and
 * pointers are checked on the host before any launch.
 */
#ifndef OAT_CNN_H
#define OAT_CNN_H

#include <stddef.h>
#include <stdint.h>

#include "oat.h"

#ifdef __cplusplus
extern "C" {
#endif

/* y[co] = b[co] + sum_ci sum_taps w[co][ci][tap] x[ci][v + tap - 1], then
 * y = max(y, 0) if relu != 0, then y = 0 wherever mask (same shape as y,
 * dtype ydt) is <= 0 if mask != NULL.  bias may be NULL (zero).  x and y
 * must not overlap. */
int oat_conv3d_forward(const void *x, oat_dtype xdt, int c_in, int d, int h, int w,
                       const float *weight, const float *bias, int c_out, void *y, oat_dtype ydt,
                       int relu, const void *mask, void *stream);

/* Bytes of device workspace oat_conv3d_backward_weight needs for this shape. */
size_t oat_conv3d_backward_weight_workspace(int c_in, int c_out, int d, int h, int w);

/* dweight[co][ci][tap] = sum_v dy[co][v] x[ci][v + tap - 1] (zero padding),
 * dbias[co] = sum_v dy[co][v]; both overwritten (dbias may be NULL).  The
 * sum is taken per tile of voxels into `workspace` and the tiles are added
 * in a fixed order, so the result is deterministic. */
int oat_conv3d_backward_weight(const void *x, oat_dtype xdt, const void *dy, oat_dtype dydt,
                               int c_in, int c_out, int d, int h, int w, float *dweight,
                               float *dbias, void *workspace, size_t workspace_bytes,
                               void *stream);

/* One Adam step on n parameters (FP32, in place):
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), t = step >= 1. */
int oat_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, float lr,
                  float beta1, float beta2, float eps, int step, void *stream);

/* Mean squared error over n values: loss[0] = sum (y - t)^2 / n (FP64
 * accumulation, FP32 result); dy = 2 (y - t) / n in ydt.  `loss` is a device
 * float; `workspace` holds at least oat_mse_workspace() bytes. */
size_t oat_mse_workspace(void);
int oat_mse(const void *y, oat_dtype ydt, const void *target, oat_dtype tdt, int64_t n,
            float *loss, void *dy, void *workspace, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* OAT_CNN_H */
