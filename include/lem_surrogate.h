/* lem_surrogate.h -- C ABI of the learned warm start for runs to steady state.
 *
 * The landscape-evolution method of Barnes, "Accelerating a Landscape
 * Evolution Model with Parallelism" (arXiv:1803.02977) is run to a steady
 * state by repeating its Steps 2-7 until heights stop changing (section
 * "Rinse, Repeat").  At a steady state uplift balances erosion, so every
 * cell's slope is (U/K) A^-m (the n = 1 stream power law of section "The
 * Equation").  This library adds a small convolutional network that predicts
 * that steady state from the erodibility field K, the uplift field U and the
 * initial surface h0; the solver then starts from the prediction (a warm
 * start) and alone decides the result: a prediction only changes
 * where the run starts, never the steady-state test.  The network is not
 * part of the paper.
 *
 * Network: features (ln K - ln 1e-5)/0.5, U/1e-3 and h0 (padded with zero
 * channels to 32); a four-level encoder (32, 64, 128, 256 channels; two 3x3
 * convolutions with bias and ReLU per level; 2x2 average pooling between
 * levels) and a decoder (nearest 2x upsampling, concatenation
 * [upsampled, encoder output of the level], two 3x3 convolutions with ReLU);
 * a 1x1 head to one channel y.  Predicted heights are y * (U/1e-3) * 100 m
 * inside the grid and 0 on the perimeter (the base level).  Weights are
 * kept as float32 master copies and used as bfloat16; activations are
 * bfloat16, accumulation float32 (MFMA).  Training minimises the mean of
 * (y - t)^2 over interior cells, t = h_target / ((U/1e-3) * 100), with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).
 *
 * Parameters form one float32 vector: per 3x3 convolution (lem_sur_layer
 * 0..13) weights [Cout][3][3][Cin] then bias [Cout]; then the head weights
 * [32] and bias [1] (layer 14).
 *
 * Memory: all arrays are device memory owned by the caller; fields are FP64
 * [batch][ny][nx] row-major, one grid after another.  The library allocates
 * no device memory; the workspace (lem_sur_workspace_bytes) holds the
 * parameters, Adam moments, gradients and activations.  Calls enqueue on the
 * context's stream and return before the device finishes unless they say
 * otherwise.  Status codes are those of lem.h.
 */
#ifndef LEM_SURROGATE_H
#define LEM_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "lem.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lem_sur_ctx lem_sur_ctx;

/* Number of float32 parameters. */
int64_t lem_sur_param_count(void);

/* Shape and offset of parameter block i: 0..13 the 3x3 convolutions in the
 * order enc0a, enc0b, enc1a, enc1b, enc2a, enc2b, enc3a, enc3b, dec2a,
 * dec2b, dec1a, dec1b, dec0a, dec0b; 14 the head (cin 32, cout 1).
 * LEM_E_ARG for other i or NULL outputs. */
lem_status lem_sur_layer(int32_t i, int32_t* cin, int32_t* cout, int64_t* offset);

/* Workspace bytes for up to `batch` grids of ny x nx (ny and nx >= 8 and
 * divisible by 8, batch >= 1), or 0 if the shape is invalid. */
size_t lem_sur_workspace_bytes(int32_t batch, int32_t ny, int32_t nx);

/* Creates a context on d_ws (>= lem_sur_workspace_bytes, 256-byte aligned,
 * owned by the caller) that enqueues on hip_stream (NULL: default stream).
 * Parameters start at zero: call lem_sur_set_params before use. */
lem_status lem_sur_create(int32_t batch, int32_t ny, int32_t nx, void* d_ws, size_t bytes,
                          void* hip_stream, lem_sur_ctx** out);

/* Copies the parameter vector (device, lem_sur_param_count floats) into the
 * context and resets Adam (zero moments, step 0). */
lem_status lem_sur_set_params(lem_sur_ctx* ctx, const float* d_params);

/* Copies the context's float32 parameters to d_params (device). */
lem_status lem_sur_get_params(lem_sur_ctx* ctx, float* d_params);

/* Prediction for `batch` grids (1 <= batch <= the context's): writes the
 * predicted heights to d_h (FP64, may be NULL) and the raw network output y
 * to d_y (float32 [batch][ny][nx], may be NULL). */
lem_status lem_sur_predict(lem_sur_ctx* ctx, int32_t batch, const double* d_K, const double* d_U,
                           const double* d_h0, double* d_h, float* d_y);

/* Loss and gradient for `batch` grids with steady-state heights d_target;
 * writes the gradient (float32, lem_sur_param_count) to d_grad when it is
 * not NULL and, when h_loss is not NULL, waits for the stream and stores the
 * loss.  Parameters are not changed. */
lem_status lem_sur_loss_grad(lem_sur_ctx* ctx, int32_t batch, const double* d_K,
                             const double* d_U, const double* d_h0, const double* d_target,
                             float* d_grad, double* h_loss);

/* One training step: loss and gradient as lem_sur_loss_grad, then one Adam
 * update with learning rate lr (> 0).  h_loss as in lem_sur_loss_grad. */
lem_status lem_sur_train_step(lem_sur_ctx* ctx, int32_t batch, const double* d_K,
                              const double* d_U, const double* d_h0, const double* d_target,
                              float lr, double* h_loss);

/* Copies activation map `index` of the most recent forward pass (grids
 * 0..batch-1) to d_dst (device): 0 the features; for level l = 0..3
 * 1 + 2l the first and 2 + 2l the second convolution's output of encoder
 * level l; 9, 10, 11 the pooled maps of levels 0, 1, 2; for decoder level
 * l = 2, 1, 0: 12 + 3(2-l) the concatenated input, 13 + 3(2-l) the first
 * and 14 + 3(2-l) the second convolution's output.  All are bfloat16 NHWC
 * (raw 16-bit patterns); *channels and *height, *width (may be NULL)
 * receive the map's shape.  d_dst may be NULL to query the shape only.
 * LEM_E_ARG for an unknown index or batch out of range. */
lem_status lem_sur_activation(lem_sur_ctx* ctx, int32_t index, int32_t batch, uint16_t* d_dst,
                              int32_t* channels, int32_t* height, int32_t* width);

/* Waits for the context's stream; reports a failed launch. */
lem_status lem_sur_sync(lem_sur_ctx* ctx);

/* Destroys the context (host state only).  NULL is a no-op. */
lem_status lem_sur_destroy(lem_sur_ctx* ctx);

/* Message of the last failure on ctx ("" if none). */
const char* lem_sur_last_error(const lem_sur_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif
