/*
 * gpop_mlp.h -- C ABI of the learned scatter-mode selector.
 *
 * The analytical model of the performance-modelling section (Eq. 1) picks,
 * per partition and per iteration, source-centric (SC) or partition-centric
 * (PC) scatter from a byte count and a fixed bandwidth ratio. The learned
 * selector replaces that rule with a small multilayer perceptron over
 * GPOP_MLP_IN per-partition features, trained on per-partition scatter times
 * the engine measures itself (gpop_probe_scatter in gpop.h). The mode never
 * changes any result (inactive PC sources send the combine identity), so the
 * selector affects time only. The analytical model stays the fallback: a
 * partition whose standardised features leave [-6, 6] or whose logit is not
 * finite is decided by Eq. 1.
 *
 * Network: x (12 features, f32) -> standardise ((x - mean) * inv_std)
 *   -> h1 = relu(W1 x + b1) (64) -> h2 = relu(W2 h1 + b2) (64)
 *   -> z = w3 . h2 + b3; PC iff z >= 0.
 * Weights are bf16 (round to nearest even from f32 masters). Training and
 * gpop_mlp_forward compute in f32; the per-iteration mode selection evaluates
 * the two hidden layers on the matrix cores, with the input of each (the
 * standardised features, then the first hidden layer after its ReLU) rounded
 * to bf16 (nearest even) and f32 accumulation. Parameters are stored in this
 * order (row-major, output-major):
 *   W1[64][12], b1[64], W2[64][64], b2[64], w3[64], b3   (5057 values).
 *
 * Features of partition p (vertices q_p, out-edges E^p, all-active messages
 * M^p, active vertices V_a, active out-edges E_a, iteration t):
 *   0 log1p(V_a)        1 log1p(E_a)        2 log1p(E^p)       3 log1p(M^p)
 *   4 r^p = M^p / E^p   5 V_a / q_p         6 E_a / E^p        7 non-empty bins of row p / k
 *   8 log(max out-degree in p / mean out-degree in p)          9 log1p(t)
 *  10 sum over partitions of E_a / |E|
 *  11 log(cost_PC / cost_SC), the two byte counts of Eq. 1 with the
 *     selector's s_i and s_v (Eq. 1 picks PC iff this is <= log(ratio))
 * Ratios with a zero denominator are 0.
 *
 * Training: binary cross-entropy on the logit with label [t_PC < t_SC] and
 * per-sample weight |t_SC - t_PC| (a sample costs what a wrong choice would
 * cost), averaged with those weights over the batch; gradients are taken
 * with respect to the bf16 weights and applied to the f32 masters by Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).
 *
 * Conventions are those of gpop.h: gpop_status returns, caller-owned device
 * memory, `stream` is a hipStream_t, work is enqueued without synchronising.
 */
#ifndef GPOP_MLP_H
#define GPOP_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPOP_MLP_IN 12
#define GPOP_MLP_HIDDEN 64
#define GPOP_MLP_PARAMS 5057
#define GPOP_MLP_MAGIC 0x504C4D47u /* "GMLP" */

/* Offsets of the parameter blocks inside gpop_mlp_model.w and the masters. */
#define GPOP_MLP_W1 0
#define GPOP_MLP_B1 768
#define GPOP_MLP_W2 832
#define GPOP_MLP_B2 4928
#define GPOP_MLP_W3 4992
#define GPOP_MLP_B3 5056

/* A model as the selector reads it (device memory, 10240 bytes, 4-byte
 * aligned). */
typedef struct gpop_mlp_model {
    uint32_t magic;                /* GPOP_MLP_MAGIC                          */
    uint32_t n_params;             /* GPOP_MLP_PARAMS                         */
    float mean[GPOP_MLP_IN];       /* feature standardisation                 */
    float inv_std[GPOP_MLP_IN];
    uint16_t w[GPOP_MLP_PARAMS];   /* bf16 bit patterns                       */
    uint16_t pad0;
    float margin;                  /* confidence gate: a partition whose |logit|
                                      is below it keeps Eq. 1's mode (0: the
                                      network decides alone, +inf: Eq. 1 alone) */
    uint16_t pad[8];
} gpop_mlp_model;

/* Starts a model: writes the header, sets mean / inv_std from the n x 12
 * training features d_x (inv_std = 1 / max(std, 1e-6), population std,
 * n >= 1), copies the n_params initial f32 weights d_init into the masters,
 * rounds them into d_model->w, and zeroes the Adam moments d_m, d_v (each
 * GPOP_MLP_PARAMS floats). Errors: GPOP_EINVAL on NULL or n = 0. */
int gpop_mlp_init(gpop_mlp_model* d_model, float* d_master, float* d_m, float* d_v,
                  const float* d_init, const float* d_x, uint32_t n, void* stream);

/* Logits of n samples: d_x is n x 12 raw features (row-major), d_logits n
 * floats. */
int gpop_mlp_forward(const gpop_mlp_model* d_model, const float* d_x, uint32_t n,
                     float* d_logits, void* stream);

/* Workspace bytes gpop_mlp_grad needs for n samples. */
size_t gpop_mlp_grad_workspace(uint32_t n);

/* Gradient of the weighted loss over n samples with respect to the bf16
 * weights: d_t_sc / d_t_pc are the measured per-sample times of the two
 * modes (any unit, >= 0). Writes GPOP_MLP_PARAMS floats to d_grad and, if
 * d_loss is not NULL, the loss to d_loss[0] and the weight sum to d_loss[1].
 * A batch whose weights are all zero gives a zero gradient. Errors:
 * GPOP_EINVAL on NULL arguments or n = 0, GPOP_ENOMEM if ws_bytes is too
 * small. */
int gpop_mlp_grad(const gpop_mlp_model* d_model, const float* d_x, const float* d_t_sc,
                  const float* d_t_pc, uint32_t n, float* d_grad, float* d_loss, void* d_ws,
                  size_t ws_bytes, void* stream);

/* Allocation-free gpop_mlp_grad, for callers that cannot allocate device
 * memory or pass a workspace (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc). The per-chunk partial sums live in a
 * fixed array inside the library, one copy per GPU (5.2 MB, held until the
 * process ends); the call allocates nothing. Results are bit-identical to
 * gpop_mlp_grad on the same inputs (same kernels, same summation order).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (concurrent streams or threads) race and must be serialised by the
 * caller. Errors: GPOP_EINVAL on NULL arguments, n = 0 or
 * n > GPOP_MLP_NOALLOC_MAX_SAMPLES; GPOP_EDEVICE if the array's device
 * address cannot be obtained. */
#define GPOP_MLP_NOALLOC_MAX_SAMPLES 16384u
int gpop_mlp_grad_noalloc(const gpop_mlp_model* d_model, const float* d_x, const float* d_t_sc,
                          const float* d_t_pc, uint32_t n, float* d_grad, float* d_loss, void* stream);

/* One Adam step (step counts from 1) of the masters with gradient d_grad,
 * learning rate lr; rewrites d_model->w from the new masters. */
int gpop_mlp_adam(gpop_mlp_model* d_model, float* d_master, float* d_m, float* d_v,
                  const float* d_grad, uint32_t step, float lr, void* stream);

/* gpop_mlp_grad followed by gpop_mlp_adam; d_grad receives the gradient. */
int gpop_mlp_train_step(gpop_mlp_model* d_model, float* d_master, float* d_m, float* d_v,
                        const float* d_x, const float* d_t_sc, const float* d_t_pc, uint32_t n,
                        uint32_t step, float lr, float* d_grad, float* d_loss, void* d_ws,
                        size_t ws_bytes, void* stream);

/* Adds delta to the output bias b3 (the f32 master d_master[GPOP_MLP_B3] and
 * its bf16 copy in d_model->w), which moves every logit by about delta: a
 * positive delta makes partition-centric choices more frequent. For
 * calibrating the decision threshold against whole-run timings after
 * training. Errors: GPOP_EINVAL on NULL arguments or a non-finite delta. */
int gpop_mlp_shift_logit(gpop_mlp_model* d_model, float* d_master, float delta, void* stream);

/* Sets the model's confidence margin: the learned selector takes the
 * network's mode for a partition only where |logit| >= margin, and Eq. 1's
 * mode (at the graph's bandwidth ratio) elsewhere, counted as a fallback in
 * the iteration records. gpop_mlp_init sets 0. For calibrating, after
 * training, how far the network is trusted against whole-run timings.
 * Errors: GPOP_EINVAL on NULL, a negative or NaN margin (+inf is allowed). */
int gpop_mlp_set_margin(gpop_mlp_model* d_model, float margin, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GPOP_MLP_H */
