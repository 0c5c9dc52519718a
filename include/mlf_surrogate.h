/*
 * mlf_surrogate.h -- C ABI of the learned surrogate in libmlfilm: a
 * convolutional neural operator that advances the layer heights of a
 * periodic multilayer film by a fixed window of K lattice Boltzmann steps
 * (the solver of mlfilm.h generates its training data and judges it).
 *
 * The paper has no learned model; the quantities it maps are the paper's
 * layer heights h_i (Sec. II).  Network, for one sample of N layers on an
 * ny x nx grid (all convolutions periodic):
 *   x_i = (h_i - mean h_i) / s
 *   r_0 = E patches_4x4(x) + b_E            latent grid ny/4 x nx/4, C channels
 *   r_{l+1} = r_l + W2_l * gelu(W1_l * r_l + b1_l) + b2_l,   l = 0..L-1, 3x3
 *   D = pixel_shuffle(W_D r_L + b_D),  Delta_i = D_i - mean D_i
 *   h_i(t + K) ~ h_i(t) + s Delta_i          (each layer's mass is kept)
 * The 3x3 convolutions run on BF16 matrix cores with FP32 accumulation,
 * the rest in FP32.  Training minimises mean((Delta - (h(t+K) - h(t))/s)^2)
 * with Adam (beta = 0.9, 0.999, eps = 1e-8).
 *
 * Parameters are one FP32 vector, in this order: E [16N][C] (patch index
 * (i*4+u)*4+v major), b_E [C]; per block l: W1 [9][C][C] (offset
 * o = 3(dy+1)+(dx+1), then output, then input channel), b1 [C], W2, b2;
 * W_D [16N][C], b_D [16N].
 *
 * Conventions as in mlfilm.h: MLF_OK or a negative mlf_status, caller-owned
 * device memory (one workspace buffer, 256-byte aligned), work issued on the
 * stream given at creation; calls returning host data synchronise.  Height
 * tensors are device FP32 [batch][N][ny][nx].
 */
#ifndef MLF_SURROGATE_H
#define MLF_SURROGATE_H

#include "mlfilm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlf_nop_params {
  int32_t n_layers;  /* N, 1..4                                             */
  int32_t nx, ny;    /* grid: nx a multiple of 256, ny a multiple of 16;
                        (ny/4)(nx/4)*width < 2^31 (one latent image)      */
  int32_t width;     /* C, 64 or 128 (EUNSUPPORTED otherwise)                */
  int32_t blocks;    /* L residual blocks, 0..32                              */
  int32_t batch;     /* largest batch passed to the calls below, 1..4096      */
  double scale;      /* s > 0: height perturbations are divided by it         */
} mlf_nop_params;

typedef struct mlf_nop mlf_nop;

/* Number of FP32 parameters and workspace bytes.  EINVAL on bad sizes. */
mlf_status mlf_nop_query_sizes(const mlf_nop_params* p, size_t* param_count, size_t* workspace_bytes);

/* Create a handle on the current device.  workspace: workspace_bytes of
 * device memory (256-byte aligned), owned by the caller and kept alive
 * until mlf_nop_destroy; stream: hipStream_t for all work (NULL = default).
 * EINVAL / EUNSUPPORTED on p as mlf_nop_query_sizes, EINVAL for a null or
 * misaligned workspace or a null out; EDEVICE if the convolution kernels'
 * LDS limits cannot be set on this device.  Parameters are undefined until
 * mlf_nop_set_params. */
mlf_status mlf_nop_create(const mlf_nop_params* p, void* workspace, void* stream, mlf_nop** out);

/* Set (host FP32 vector of param_count) / read the parameters.  Setting
 * also clears the Adam moments and step count.  Synchronise. */
mlf_status mlf_nop_set_params(mlf_nop* m, const float* host);
mlf_status mlf_nop_get_params(mlf_nop* m, float* host);

/* out = h + s Delta(h): predicted heights one window later (device, may
 * not alias h).  Asynchronous. */
mlf_status mlf_nop_predict(mlf_nop* m, int32_t batch, const float* h, float* out);

/* Training loss for pairs (h0, h1 = heights K steps later); synchronises. */
mlf_status mlf_nop_loss(mlf_nop* m, int32_t batch, const float* h0, const float* h1, double* loss);

/* Loss and its gradient w.r.t. every parameter (host FP32 vector of
 * param_count, may be NULL); synchronises. */
mlf_status mlf_nop_gradient(mlf_nop* m, int32_t batch, const float* h0, const float* h1, float* host_grad,
                            double* loss);

/* One Adam step with learning rate lr > 0 on the pairs (h0, h1); returns
 * the loss before the step; synchronises. */
mlf_status mlf_nop_train_step(mlf_nop* m, int32_t batch, const float* h0, const float* h1, float lr, double* loss);

/* Event-timed average duration (ms) of one 3x3 convolution of the first
 * block on `batch` samples, `reps` launches each, on the activations as
 * they stand (run mlf_nop_predict first): ms[0] forward with the plain
 * epilogue (also the input-gradient kernel), ms[1] forward with the GELU
 * epilogue, ms[2] forward with the residual epilogue, ms[3] weight
 * gradient.  ms: host float[4].  Overwrites the first block's activations
 * and scratch only.  Synchronises.  EINVAL for NULL pointers or reps < 1. */
mlf_status mlf_nop_time_conv(mlf_nop* m, int32_t batch, int32_t reps, float* ms);

/* Judge arithmetic.  Errors of n samples of a against the reference b
 * (device FP32 [n][N][ny][nx] each), reduced in FP64 in a fixed order:
 * out[2s] = |a_s - b_s| / |b_s| (relative L2 over all layers and nodes)
 * and out[2s+1] = |a_s - b_s| / |b_s - mean b_s| (relative to the
 * reference's perturbation, the per-layer means removed).  out: device
 * FP64 [2n], caller-owned.  Asynchronous.  EINVAL for NULL pointers or
 * n < 1. */
mlf_status mlf_nop_errors(mlf_nop* m, int32_t n, const float* a, const float* b, double* out);

/* Height conversion between the solver (FP64) and the network (FP32):
 * n elements; to_f32 != 0: src FP64 -> dst FP32 (round to nearest), else
 * src FP32 -> dst FP64 (exact).  Device arrays, caller-owned, not
 * aliased; stream: hipStream_t (NULL: default).  Asynchronous.  EINVAL
 * for NULL pointers or n < 1, EDEVICE if the launch fails. */
mlf_status mlf_convert_heights(const void* src, int32_t to_f32, void* dst, int64_t n, void* stream);

/* Adam steps taken since the parameters were last set (-1 for NULL). */
int32_t mlf_nop_steps_done(const mlf_nop* m);
/* Text of the last failure on this handle ("" if none); valid until the
 * next call on it. */
const char* mlf_nop_last_error(const mlf_nop* m);
/* Free the host handle (not the workspace); EINVAL for NULL. */
mlf_status mlf_nop_destroy(mlf_nop* m);

#ifdef __cplusplus
}
#endif
#endif
