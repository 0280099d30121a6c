/*
 * tled_surrogate.h -- C-ABI of the learned surrogate of the coupled TLED +
 * Pennes solver: a multilayer perceptron that maps node coordinates (random
 * Fourier features) and scenario parameters to the nodal temperature and
 * displacement at the end of a heating scenario, trained on solver runs.
 * (The paper's discussion names learned acceleration as a route to cheaper
 * planning runs, Section 7; the network itself is this library's design.)
 *
 * Network: features f = [sin(2 pi B x), cos(2 pi B x), p, 0...] with B an
 * n_freq x 3 matrix drawn once from N(0, sigma^2), x the sample's coordinates
 * and p its scenario parameters, zero-padded to a multiple of 32; then `depth`
 * hidden layers of `width` units with SiLU, z = W a + b, a' = z sigmoid(z);
 * then a linear output layer of n_out units.
 *
 * Arithmetic: weights and activations in bfloat16, products accumulated in
 * FP32 on the matrix cores (v_mfma_f32_16x16x32_bf16); FP32 master weights,
 * biases, loss and Adam moments; sine, cosine, exponential and reciprocal from
 * the hardware transcendental units (errors far below the bfloat16 rounding of
 * the activations).  Loss: mean over samples and outputs of the squared error.
 *
 * Parameter layout (FP32, host arrays of tled_mlp_param_count floats): for
 * each layer in order, W (rows = outputs, row-major over inputs incl. the
 * zero padding of the first layer's inputs), then b.
 *
 * Data pointers of forward/train/gradient calls are DEVICE pointers (FP32,
 * row-major): coords n x 3, params n x n_param, target n x n_out, out
 * n x n_out.  Calls run on the handle's stream; forward and train_step are
 * asynchronous except when a loss is requested.  Workspace grows on demand
 * to the largest n seen (hipMalloc), so the first call at a new size allocates.
 * Errors are tled_status codes (tled.h); messages via tled_mlp_last_error.
 */
#ifndef TLED_SURROGATE_H
#define TLED_SURROGATE_H

#include <stdint.h>

#include "tled.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tled_mlp tled_mlp;

typedef struct {
    int32_t n_param;   /* scenario parameters per sample                   */
    int32_t n_freq;    /* Fourier frequencies (2 n_freq features)           */
    int32_t width;     /* hidden width, multiple of 64                     */
    int32_t depth;     /* number of hidden layers (>= 1)                   */
    int32_t n_out;     /* outputs (<= 64)                                  */
    int32_t layerwise; /* 1: inference layer by layer through HBM; 0: fused
                          (whole network per 64 samples in LDS) where the
                          width is 64, 128 or 256 and depth <= 8            */
    float sigma;       /* standard deviation of the frequencies            */
    float init_scale;  /* uniform weight init bound factor (0: 1)          */
    uint64_t seed;     /* frequencies and initial weights                  */
} tled_mlp_config;

tled_status tled_mlp_create(tled_mlp **out, int device, const tled_mlp_config *cfg);
void        tled_mlp_destroy(tled_mlp *mlp);
tled_status tled_mlp_set_stream(tled_mlp *mlp, void *hip_stream);
tled_status tled_mlp_param_count(const tled_mlp *mlp, int64_t *n);
tled_status tled_mlp_get_params(tled_mlp *mlp, float *host);
tled_status tled_mlp_set_params(tled_mlp *mlp, const float *host);
/* The Fourier frequency matrix B (n_freq x 3, host). */
tled_status tled_mlp_get_frequencies(tled_mlp *mlp, float *host);
/* Inference on n samples.  The fused and the layer-by-layer forms give the
 * same bits (same products in the same order). */
tled_status tled_mlp_forward(tled_mlp *mlp, int64_t n, const float *coords, const float *params, float *out);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at learning rate lr on the
 * minibatch; *loss (host, optional) receives the minibatch loss before the step. */
tled_status tled_mlp_train_step(tled_mlp *mlp, int64_t n, const float *coords, const float *params,
                                const float *target, float lr, float *loss);
/* Gradient of the minibatch loss with respect to the FP32 parameters (host
 * array in the parameter layout), without a step; *loss optional. */
tled_status tled_mlp_gradient(tled_mlp *mlp, int64_t n, const float *coords, const float *params,
                              const float *target, float *grad_host, float *loss);
/* Ensemble statistics of `members` networks' outputs (device arrays, FP32):
 * outs is members x n x n_out (member-major, each member's n x n_out block as
 * tled_mlp_forward writes it); scale (n_out) multiplies the results:
 * mean[i][o] = scale[o] * mean_k outs[k][i][o], spread[i] = scale[0] *
 * (max_k - min_k) outs[k][i][0].  Enqueued on hip_stream (NULL: the null
 * stream); asynchronous.  Returns TLED_E_ARG on bad sizes or null pointers. */
tled_status tled_mlp_ensemble_stats(int64_t n, int32_t members, int32_t n_out, const float *outs,
                                    const float *scale, float *mean, float *spread, void *hip_stream);
/* Network inputs of n_scen scenarios, whose nodes are the consecutive row ranges
 * [row_begin[s], row_begin[s+1]) of n_rows = row_begin[n_scen] rows (offsets
 * nondecreasing, row_begin[0] = 0; every scenario with rows).  For row r of
 * scenario s, with node coordinates X[r] (m, FP64, n_rows x 3):
 *   x_out[r] = (X[r] - probe[s]) * xi[s]          (n_rows x 3),
 *   p_out[r] = (X[r] * p_scale, prm[s][0..n_prm)) (n_rows x (3 + n_prm)),
 * the products formed in FP64 and rounded once to FP32 (prm is FP32, n_scen x
 * n_prm).  All arrays on the device; enqueued on hip_stream (NULL: the null
 * stream), asynchronous.  TLED_E_ARG on bad sizes or null pointers. */
tled_status tled_mlp_scenario_inputs(int32_t n_scen, int32_t n_prm, int64_t n_rows, const int64_t *row_begin,
                                     const double *X, const double *probe, const double *xi, double p_scale,
                                     const float *prm, float *x_out, float *p_out, void *hip_stream);
/* Physical fields from the ensemble statistics (rows as above, FP32 device
 * arrays): T_out[r] = T0[s] + sT[s] * mean[r][0], u_out[r][i] = su[s] *
 * mean[r][1 + i], spread_out[r] = sT[s] * spread[r], each operation rounded
 * separately (no fused multiply-add).  Asynchronous on hip_stream; TLED_E_ARG
 * on bad sizes or null pointers. */
tled_status tled_mlp_scenario_outputs(int32_t n_scen, int64_t n_rows, const int64_t *row_begin, const float *mean,
                                      const float *spread, const float *T0, const float *sT, const float *su,
                                      float *T_out, float *u_out, float *spread_out, void *hip_stream);
/* Plain GEMM on the matrix cores, for tests of the kernel itself:
 * C[m][n] = sum_k A[m][k] B[k][n], A (m x k) and B (k x n) bfloat16 bit
 * patterns (device, row-major), C FP32 (device, row-major). */
tled_status tled_mlp_gemm(tled_mlp *mlp, int32_t m, int32_t n, int32_t k, const uint16_t *A, const uint16_t *B,
                          float *C);
/* tled_mlp_gemm for callers that cannot allocate (code under hipGraph capture,
 * tight serving loops, harnesses that forbid allocation): no device or host
 * memory is allocated per call.  Its split-K partials live in a static device
 * array of 512 x 64 x 64 floats (8 MiB) that every GPU the library runs on holds
 * until the process ends; the array's address on a device is resolved when a
 * handle is created on it.  TLED_E_ARG when a product's split-K partials would
 * exceed the array (the split rule keeps them within it), TLED_E_STATE if the
 * address was not resolved.  All calls on one GPU share the array and each
 * leaves it holding its partials: calls that overlap on one GPU (several
 * streams or threads) race.  Timing (tled_mlp_set_timing) does not apply.
 * Same kernels and the same bits as tled_mlp_gemm. */
tled_status tled_mlp_gemm_static(tled_mlp *mlp, int32_t m, int32_t n, int32_t k, const uint16_t *A,
                                 const uint16_t *B, float *C);
/* Measurement: with timing on, every GEMM and fused-inference launch is
 * bracketed by HIP events on the handle's stream (and waited for);
 * tled_mlp_last_timing returns, since timing was switched on, the summed GEMM
 * time ms[0] and fused-inference time ms[1] (ms) and their flops[0], flops[1]. */
tled_status tled_mlp_set_timing(tled_mlp *mlp, int on);
tled_status tled_mlp_last_timing(tled_mlp *mlp, double ms[2], double flops[2]);
const char *tled_mlp_last_error(const tled_mlp *mlp);

#ifdef __cplusplus
}
#endif
#endif /* TLED_SURROGATE_H */
