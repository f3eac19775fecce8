/* ttnn.h -- learned propagator of the electronic reduced density matrix,
 * C ABI (HIP, gfx950).
 *
 * A multilayer perceptron advances the electronic reduced density matrix
 * (RDM) of the root of a TTNS run by one time step from the last `window`
 * RDMs and a vector of model parameters ("conditioning").  It is trained on
 * RDM trajectories that the TTNS-TDVP library itself produces (the RDM is
 * the root's C_(sigma) C_(sigma)^dagger of the tree state, sections "Tree
 * tensor network states" and "Results": populations and coherences of the
 * electronic states), and every rollout is judged against the full TTNS
 * trajectory by the trace distance; a rejected rollout falls back to the
 * TTNS trajectory.  The paper itself has no such propagator (its only
 * learning step is the k-means clustering of the couplings, section
 * "Interface to TTNS"); this is an addition built on the method's output.
 *
 * Encoding of an n x n Hermitian RDM as n^2 reals ("enc"): the n diagonal
 * entries, then Re rho_jk for j < k (row-major upper triangle), then
 * Im rho_jk in the same order.
 *
 * Network (FP32 storage, FP32 matrix-core products with FP32 accumulation):
 *   x   = [enc(rho_{t-window+1}), ..., enc(rho_t), cond]      (window n^2 + n_cond)
 *   h_1 = tanh(W_1 x + b_1), ..., h_L = tanh(W_L h_{L-1} + b_L)  (L = layers, width hidden)
 *   enc(rho_{t+1}) = enc(U rho_t U^dagger) + W_{L+1} h_L + b_{L+1} (residual output)
 * with U = exp(-i H_S dt) the free propagator of the electronic system
 * Hamiltonian of Eq. (2) (or the identity when none is given): the network
 * learns what the environment adds to the known system dynamics, as a
 * transfer-tensor scheme learns a memory kernel on top of free evolution.
 * With skip = 1 the input also carries cond_c * enc(rho_t)_e for every
 * (c, e) (row-major), and the output adds W_s x (no bias): a linear,
 * parameter-dependent transfer term with the MLP on top.
 * Loss: mean squared error over the batch and the n^2 outputs.  Optimiser:
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 * Rollout: propagate, predict, divide by the trace, append, shift the window.
 *
 * Parameter layout ("flat"): for each layer in order, W (out x in,
 * row-major) then b (out); with the skip, W_s (n^2 x input, row-major) last.
 *
 * Conventions shared with ttns.h: calls return TTNS_OK or a negative
 * TTNS_E* code and never abort; ttns_last_error(NULL) gives the calling thread's
 * message.  Device pointers are HIP device addresses on the device that is
 * current when ttnn_build is called; all work is enqueued on the stream
 * given to ttnn_build.  Calls that return host data synchronise that stream.
 * The workspace belongs to the caller (allocated once, e.g. by PyTorch) and
 * must outlive the network; the library allocates no device memory.
 */
#ifndef TTNN_H
#define TTNN_H

#include <stddef.h>
#include <stdint.h>

#include "ttns.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ttnn_net ttnn_net; /* opaque, library-owned host state */

typedef struct {
  int32_t n_levels;  /* n: the RDM is n x n (1..8), n^2 encoded reals     */
  int32_t window;    /* memory length in RDMs (>= 1)                      */
  int32_t n_cond;    /* conditioning reals per parameter set (>= 0)       */
  int32_t hidden;    /* width of every hidden layer (>= 1)                */
  int32_t layers;    /* number of hidden layers (1..8)                    */
  int32_t max_batch; /* largest training or rollout batch (>= 1)          */
  int32_t skip;      /* 1: linear skip path (see above), 0: plain MLP     */
} ttnn_config;

/* Number of parameters (floats) in the flat layout. */
int ttnn_param_count(const ttnn_config* cfg, int64_t* count);

/* Device workspace bytes the network needs (parameters, gradients, Adam
 * moments, activations and gradients of one max_batch batch). */
int ttnn_workspace_size(const ttnn_config* cfg, size_t* bytes);

/* Lay the network out in dev_ws (>= ttnn_workspace_size bytes, 256-byte
 * aligned), copy the caller's initial parameters (host, flat layout,
 * ttnn_param_count floats) and zero the Adam state.  The library draws no
 * random numbers.  Synchronous. */
int ttnn_build(const ttnn_config* cfg, const float* host_params, void* dev_ws, size_t ws_bytes,
               void* hip_stream, ttnn_net** out);

/* Conditioning vector of a star model (host, FP64 -> FP32): Re diag H_S,
 * Re of the upper triangle of H_S (row-major), alpha of every chain, Re of
 * the diagonal of every chain's coupling A_i.  n_out must be at least
 * n + n(n-1)/2 + n_chains (1 + n); the count written is returned in
 * *written. */
int ttnn_conditioning(const ttns_star_model* model, float* host_out, int32_t n_out, int32_t* written);

/* Free propagator U = exp(-i H_S dt) of a star model's electronic system
 * Hamiltonian (host, FP64 scaling and squaring of a Taylor series, rounded
 * to FP32): 2 n^2 floats, (re, im) row-major; n_out >= 2 n^2.  dt is in the
 * Hamiltonian's inverse energy unit (as ttns_tdvp_step's dt). */
int ttnn_propagator(const ttns_star_model* model, double dt, float* host_out, int32_t n_out);

/* Encode `count` RDMs (device, count x n x n complex, (re, im) doubles,
 * row-major) into dev_out (device, count x n^2 floats). */
int ttnn_encode(ttnn_net* net, const double* dev_rdm, int64_t count, float* dev_out);

/* Training data: n_sets encoded trajectories of n_times RDMs each (device,
 * n_sets x n_times x n^2 floats), their conditioning (device,
 * n_sets x n_cond floats) and their free propagators (device,
 * n_sets x 2 n^2 floats from ttnn_propagator, or NULL for the identity).
 * The arrays stay the caller's and must outlive the training calls that use
 * them. */
int ttnn_set_data(ttnn_net* net, const float* dev_traj, const float* dev_cond, const float* dev_prop,
                  int32_t n_sets, int32_t n_times);

/* Loss and gradient of one batch without an update.  host_samples holds
 * `batch` pairs (set, t) with window-1 <= t < n_times-1 (the pair predicts
 * RDM t+1 from RDMs t-window+1..t of that set).  Writes the loss to
 * *host_loss and, if host_grad is not NULL, the gradient (flat layout).
 * Synchronous. */
int ttnn_gradients(ttnn_net* net, const int32_t* host_samples, int32_t batch, float* host_loss,
                   float* host_grad);

/* One Adam step on one batch (same samples as ttnn_gradients) with
 * learning rate lr.  dev_noise (device, batch x window n^2 floats, or NULL)
 * is added to the input RDM window of each sample (not to the target): the
 * caller draws it, e.g. Gaussian, to train a map that pulls perturbed
 * histories back towards the data, which keeps long rollouts stable.
 * Asynchronous; ttnn_last_loss reads its loss. */
int ttnn_train_step(ttnn_net* net, const int32_t* host_samples, int32_t batch, float lr, const float* dev_noise);

/* Loss of the last ttnn_train_step or ttnn_gradients call.  Synchronous. */
int ttnn_last_loss(ttnn_net* net, float* host_loss);

/* Copy the parameters out (host, flat layout) or in (also zeroes the Adam
 * moments and step count).  Synchronous. */
int ttnn_get_params(ttnn_net* net, float* host_out);
int ttnn_set_params(ttnn_net* net, const float* host_in);

/* Autoregressive rollout of `batch` sets for n_steps steps.  dev_init:
 * batch x window x n^2 floats (the last `window` encoded RDMs, oldest
 * first), dev_cond: batch x n_cond, dev_prop: batch x 2 n^2 (or NULL, as
 * in training), dev_out: batch x n_steps x n^2 (the predicted,
 * trace-normalised RDMs).  Asynchronous. */
int ttnn_rollout(ttnn_net* net, const float* dev_init, const float* dev_cond, const float* dev_prop,
                 int32_t batch, int32_t n_steps, float* dev_out);

/* Judge rollouts against reference (TTNS) trajectories, both encoded
 * (device, batch x n_steps x n^2): dev_dist[b][t] = trace distance
 * 1/2 ||rho - sigma||_1 (device, batch x n_steps floats); dev_worst[b] =
 * max_t dist; dev_accept[b] = worst <= tol.  Asynchronous. */
int ttnn_judge(ttnn_net* net, const float* dev_pred, const float* dev_ref, int32_t batch, int32_t n_steps,
               float tol, float* dev_dist, float* dev_worst, int32_t* dev_accept);

/* Fallback: dev_out[b] = accept[b] ? pred[b] : ref[b] (whole trajectories,
 * batch x n_steps x n^2 floats; out may alias pred).  Asynchronous. */
int ttnn_select(ttnn_net* net, const float* dev_pred, const float* dev_ref, const int32_t* dev_accept,
                int32_t batch, int32_t n_steps, float* dev_out);

/* Release the host state (the workspace stays the caller's). */
int ttnn_destroy(ttnn_net* net);

#ifdef __cplusplus
}
#endif

#endif /* TTNN_H */
