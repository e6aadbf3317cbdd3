/* spmd_mlp.h -- the learned schedule cost model: a small multilayer
 * perceptron run and trained by hand-written kernels.
 *
 * The model maps a launch's features and one candidate schedule to the
 * predicted natural log of its running time in microseconds:
 *   x  = (launch features[9], schedule inputs[3])           12 inputs
 *   xn = (x - mu) * inv_sd                                  norm = mu[12], inv_sd[12]
 *   h1 = relu(xn W1 + b1), h2 = relu(h1 W2 + b2)            64 units each
 *   y  = h2 . w3 + b3
 * Parameters are one fp32 vector of SPMD_MLP_NPARAM values in the order
 * W1 (12 x 64, row-major), b1, W2 (64 x 64), b2, w3, b3.  Training
 * minimises mean((y - t)^2) with Adam.  All sums run in a fixed order, so
 * results do not depend on scheduling (no floating-point atomics).
 *
 * This component is not described by the paper, which picks the blocks per
 * fetch by hand-tuned heuristics (Section IV-A); it replaces those
 * heuristics with a model trained on measured timings.
 */
#ifndef SPMD_MLP_H
#define SPMD_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPMD_MLP_DIN 12
#define SPMD_MLP_NFEAT 9
#define SPMD_MLP_NSCHED 3
#define SPMD_MLP_H 64
#define SPMD_MLP_NPARAM (12 * 64 + 64 + 64 * 64 + 64 + 64 + 1)
#define SPMD_MLP_MAX_MODELS 4
#define SPMD_MLP_MAX_CANDS 256

/* Predictions y[n] for rows x[n x 12] (device pointers).  When h1t and h2t
 * are not NULL the hidden activations are also stored feature-major
 * (h1t[j * n + i]) for spmd_mlp_backward. */
int spmd_mlp_forward(const float* params, const float* norm, const float* x, uint32_t n, float* y, float* h1t,
                     float* h2t, void* stream);

/* Workspace bytes for spmd_mlp_backward over n rows. */
size_t spmd_mlp_workspace_size(uint32_t n);

/* Gradient of mean((y - t)^2) over the n rows into grad[SPMD_MLP_NPARAM],
 * and the loss into loss[0]; y, h1t and h2t come from spmd_mlp_forward with
 * the same parameters. */
int spmd_mlp_backward(const float* params, const float* norm, const float* x, const float* t, uint32_t n,
                      const float* y, const float* h1t, const float* h2t, float* grad, float* loss, void* workspace,
                      size_t ws_bytes, void* stream);

/* One Adam step (step counts from 1) over the SPMD_MLP_NPARAM parameters. */
int spmd_mlp_adam(float* params, const float* grad, float* m, float* v, uint32_t step, float lr, float beta1,
                  float beta2, float eps, void* stream);

/* Schedule choice for m launches: launch features feats[m x 9], candidate
 * schedule inputs cands[c x 3] (c <= SPMD_MLP_MAX_CANDS), valid[m x c]
 * (non-zero where candidate j is allowed for launch i).  Each of k_models
 * models (params: k_models consecutive parameter vectors, one norm for
 * all) predicts every (launch, candidate); the chosen candidate minimises
 * the mean prediction over the models (ties to the lowest index).  Out:
 * best[m], best_pred[m] (that mean) and best_sd[m] (the models' standard
 * deviation there: the confidence measure).  A launch with no valid
 * candidate gets best = 0xFFFFFFFF. */
int spmd_mlp_choose(const float* params, uint32_t k_models, const float* norm, const float* feats, uint32_t m,
                    const float* cands, uint32_t c, const uint8_t* valid, uint32_t* best, float* best_pred,
                    float* best_sd, void* stream);

/* Batch-aware choice.  In a batch every launch's chunks are fetched from
 * its queue's cursors by one atomic each, so the number of chunks
 * is a cost of the batch that a launch timed alone does not show (fetching
 * is atomic and costs, Section IV-A).  chunks[m x c] holds the chunk count
 * of launch i under candidate j (spmd_sched_chunks).  Among the candidates
 * whose mean prediction is within ln(1 + slack) of the least, the chosen
 * one has the fewest chunks (then the smaller mean, then the lower index);
 * slack 0 keeps only the candidates that tie with the least.  Outputs as
 * spmd_mlp_choose (best_pred and best_sd at the chosen candidate).
 * SPMD_ERR_ARGS for a null chunks or a negative or non-finite slack. */
int spmd_mlp_choose_batch(const float* params, uint32_t k_models, const float* norm, const float* feats,
                          uint32_t m, const float* cands, uint32_t c, const uint8_t* valid, const uint32_t* chunks,
                          float slack, uint32_t* best, float* best_pred, float* best_sd, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SPMD_MLP_H */
