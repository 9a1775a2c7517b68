/*
 * Policy in the loop for libnavsim (C ABI, version 1): the paper's actor
 * (section 2.1: a four-layer perceptron with 100 hidden units per layer and
 * leaky-ReLU activations, input = the state of eq. 1 with each pooled range
 * l passed through the reciprocal transform 1 / (l - beta) of eq. 2) run on
 * the GPU in front of every step, so that a rollout collects experience
 * under the current policy without leaving the device.
 *
 * Readings (the paper leaves these open): the actor's output layer is tanh,
 * giving the normalised action in [-1, 1]^2 that navsim_step maps to
 * (v, omega); beta is one scalar shared by all ranges; exploration adds
 * Gaussian noise of a given standard deviation and clips to [-1, 1].
 * Weights, inputs and hidden activations are bfloat16 on the matrix cores
 * with float accumulation; the transform, biases and output are float.
 */
#ifndef NAVSIM_POLICY_H
#define NAVSIM_POLICY_H

#include <stdint.h>

#include "navsim.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct navsim_policy_s *navsim_policy_t;

/* Actor for handle h: dims = [m + 4, hidden x hidden_layers, 2] (paper: 100
 * and 3).  Parameters start at zero (set them with navsim_policy_set_params).
 * Errors: INVALID_ARG (hidden not in 1..1024, hidden_layers not in 1..4,
 * slope <= 0), BAD_HANDLE, OOM, HIP. */
navsim_status navsim_policy_create(navsim_t h, int32_t hidden, int32_t hidden_layers,
                                   float leaky_slope, navsim_policy_t *out);

/* Layout of the flat float parameter vector: for layer l the weight
 * [dims[l+1]][dims[l]] at offsets[2 l] and the bias at offsets[2 l + 1];
 * beta at offsets[2 L]; *count floats in all.  NULL arrays are skipped. */
navsim_status navsim_policy_layout(navsim_policy_t pol, int32_t *num_layers, int32_t *dims,
                                   int64_t *offsets, int64_t *count);

/* Copy parameters from host memory (count floats, layout above). */
navsim_status navsim_policy_set_params(navsim_policy_t pol, const float *host, int64_t count);

/* Actions for N observations: obs device float [N][m+4] -> act device float
 * [N][2].  noise_std > 0 makes a = clip(a + noise_std n, -1, 1) with n
 * standard normal by Box-Muller from Philox4x32-10 (key = the handle's seed,
 * counter (e, step mod 2^32, step div 2^32, 11), words 0 and 1). */
navsim_status navsim_policy_act(navsim_policy_t pol, const float *obs, float *act,
                                float noise_std, uint64_t step, void *hip_stream);

/* `steps` steps with the actor in the loop: step i's action comes from the
 * actor on obs row i - 1 (obs0 for i = 0; device float [N][m+4]) with noise
 * step index first_step + i, then the step itself (navsim_step or
 * navsim_step_plain by `kernel`).  Output rows as navsim_rollout (act
 * [steps][N][2] required here, final_obs may be NULL).  flags:
 * NAVSIM_ROLLOUT_GRAPH captures the steps' launches once into a HIP graph
 * kept in the policy (replayed while buffers, steps, noise, kernel and launch
 * shape stay the same).  Errors as navsim_rollout. */
navsim_status navsim_policy_rollout(navsim_t h, navsim_policy_t pol, int32_t steps,
                                    uint64_t first_step, const float *obs0, float noise_std,
                                    float *act, float *obs, float *reward, uint8_t *terminated,
                                    uint8_t *truncated, float *final_obs, int32_t kernel,
                                    int32_t flags, void *hip_stream);

navsim_status navsim_policy_destroy(navsim_policy_t pol);

#ifdef __cplusplus
}
#endif
#endif
