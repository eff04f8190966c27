/*
 * vk_mlp.h -- C ABI of the learned Newton initial guess (a project extension to
 * the solver of vk.h; the paper's Newton iteration, Sec. 3, starts every slab
 * from a guess, which these calls supply).
 *
 * A small multilayer perceptron maps the values of two earlier slab solutions
 * on a cell patch (the n_K DoFs of a cell, Sec. 3's dof(K, .)) to a correction
 * of the extrapolated guess on the same patch; corrections of the cells sharing
 * a DoF are averaged, as the Vanka update averages its local results (Eq. 3.5).
 *
 * Network: n_in -> width (tanh) -> ... (n_hidden hidden layers, tanh) -> n_out
 * (linear).  Parameters form one packed FP32 vector, layer by layer: W_l
 * (out x in, row-major) followed by b_l.
 *
 * Precision: products run on BF16 matrix cores with FP32 accumulation.  Inputs,
 * the weights used in products, hidden activations and back-propagated
 * pre-activation gradients are stored in BF16 (round to nearest even); biases,
 * outputs, the loss, weight gradients, the master weights and the Adam moments
 * are FP32.
 *
 * Conventions are those of vk.h: device pointers unless marked (host), the
 * caller owns every array, work is enqueued on the context's stream, and the
 * calls return a vk_status with vk_mlp_last_error giving the message.  The
 * library allocates no device memory; the caller provides the workspace.
 */
#ifndef VK_MLP_H
#define VK_MLP_H

#include "vk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vk_mlp vk_mlp;

/* Create a network context.  1 <= n_hidden <= 8, 1 <= n_in, width, n_out <= 1024,
 * 1 <= max_batch <= 1 << 20 (the largest batch of any later call).
 * hip_stream may be NULL (the null stream). */
vk_status vk_mlp_create(vk_mlp** out, int32_t n_in, int32_t width, int32_t n_hidden, int32_t n_out,
                        int32_t max_batch, void* hip_stream);
void vk_mlp_destroy(vk_mlp* mlp);
const char* vk_mlp_last_error(const vk_mlp* mlp);   /* NULL mlp: the last vk_mlp_create failure */

/* Number of packed parameters. */
int64_t vk_mlp_param_count(const vk_mlp* mlp);

/* Workspace: master weights, their BF16 copy, gradient, Adam moments,
 * activations of max_batch samples and reduction scratch. */
size_t vk_mlp_workspace_bytes(const vk_mlp* mlp);
vk_status vk_mlp_set_workspace(vk_mlp* mlp, void* dev, size_t bytes);

/* Load the packed FP32 parameters (device), refresh the BF16 copy and reset
 * the Adam moments and step counter.  vk_mlp_get_params copies them out. */
vk_status vk_mlp_set_params(vk_mlp* mlp, const float* params);
vk_status vk_mlp_get_params(vk_mlp* mlp, float* params);

/* y[m, :] = net(x[rows[m], :]) for m < batch.  x: BF16 (uint16 bit patterns),
 * row-major with n_in columns; rows: int32 sample indices into x (NULL: m);
 * y: FP32 batch x n_out. */
vk_status vk_mlp_forward(vk_mlp* mlp, int32_t batch, const uint16_t* x, const int32_t* rows, float* y);

/* Mean squared error of the batch against target[rows[m], :] (FP32, n_out
 * columns) and its gradient with respect to the parameters, kept in the
 * workspace for vk_mlp_adam.  loss (FP32 scalar) and grad (FP32, packed like the
 * parameters) are optional copies (NULL: skipped).
 *   L = 1 / (batch n_out) sum_{m, j} (y_mj - t_mj)^2 */
vk_status vk_mlp_gradient(vk_mlp* mlp, int32_t batch, const uint16_t* x, const int32_t* rows,
                          const float* target, float* loss, float* grad);

/* One Adam step (Kingma & Ba) with the last gradient: increments the step
 * counter t and updates the master weights and their BF16 copy. */
vk_status vk_mlp_adam(vk_mlp* mlp, float lr, float beta1, float beta2, float eps);

/* ---- patch data --------------------------------------------------------------
 * cell_dofs: int32 n_cells x n_K global DoF ids (the patch maps of vk.h). */

/* Features of the cells from the two previous slab solutions X1 = X_{n-2}, X2 = X_{n-1} and
 * B = the extrapolation of X_{n-2} to slab n-1's nodes: for j < n_K, with d = dof(c, j),
 *   out[c, j]       = bf16((float)((X2[d] - X1[d]) - mean[j]) * inv_std[j])
 *   out[c, n_K + j] = bf16((float)((X2[d] - B[d]) - mean[n_K + j]) * inv_std[n_K + j])
 * (the change between the slabs and the previous slab's extrapolation error, formed in FP64:
 * BF16 keeps about 3 significant digits, too few for the slab values themselves to carry their
 * slab-to-slab change).  mean, inv_std: FP32, 2 n_K entries; out: n_cells x 2 n_K BF16. */
vk_status vk_mlp_patch_features(vk_mlp* mlp, int32_t n_cells, int32_t n_K, const int32_t* cell_dofs,
                                const double* X1, const double* X2, const double* B, const float* mean,
                                const float* inv_std, uint16_t* out);

/* Training targets: out[c, j] = ((X - base)[dof(c, j)] - mean[j]) * inv_std[j] (FP32, n_K columns). */
vk_status vk_mlp_patch_targets(vk_mlp* mlp, int32_t n_cells, int32_t n_K, const int32_t* cell_dofs,
                               const double* X, const double* base, const float* mean, const float* inv_std,
                               float* out);

/* Averaged guess: out[mu] = base[mu] + (1 / #entries(mu)) sum over the entries e of mu of
 * (pred[e] * std[e mod n_K] + mean[e mod n_K]), where dof_ptr (n + 1) and dof_list give, for
 * every DoF mu < n, its entries e = cell * n_K + local in pred (FP32, n_cells x n_K).  DoFs in
 * no patch keep base.  std, mean: FP32, n_K entries. */
vk_status vk_mlp_patch_average(vk_mlp* mlp, int64_t n, const int64_t* dof_ptr, const int64_t* dof_list,
                               int32_t n_K, const float* pred, const float* mean, const float* std,
                               const double* base, double* out);

/* Extrapolation of a slab vector (time-node major: n_time blocks of n_space):
 * out[a, i] = sum_b E[a, b] X[b, i], E (host, n_time x n_time row-major, n_time <= 8);
 * with E[a, b] = chi_b(1 + s_a) this evaluates the previous slab's time polynomial at
 * the next slab's Radau nodes (the fallback guess).  out must not alias X. */
vk_status vk_mlp_slab_extrapolate(vk_mlp* mlp, int64_t n_space, int32_t n_time, const double* E,
                                  const double* X, double* out);

#ifdef __cplusplus
}
#endif

#endif /* VK_MLP_H */
