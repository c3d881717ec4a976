/*
 * Warm-start network of the MI355X PIC-MCC library: a fully connected network
 * trained and evaluated with BF16 matrix-core products and FP32 accumulation,
 * FP32 master weights and Adam.
 *
 * The network is not part of the paper's method.  The paper restarts a case
 * from its converged state after a parameter change (Section 2); here a new
 * discharge instead starts from density and mean-energy profiles that this
 * network predicts from the discharge parameters, and the plain method then
 * runs to its own periodic steady state.  The network only sets the initial
 * particles; nothing else of the step depends on it.
 *
 * Network: widths w[0] .. w[L]; layer l maps w[l] inputs to w[l+1] outputs,
 * z = W_l a + b_l, followed by the exact GELU z Phi(z) on every layer but the
 * last.  Loss: mean squared error over all outputs of all samples of a batch.
 * Optimiser: Adam with bias correction (Kingma and Ba, 2015).
 *
 * Parameter layout (flat float array, host side): one block per layer, in
 * order, each the row-major matrix [w[l+1]][w[l] + 1] whose last column is
 * the bias.  Count: sum over l of w[l+1] (w[l] + 1).
 *
 * Conventions: the caller owns every pointer.  x_dev, t_dev, y_dev and
 * loss_dev are device pointers on the context's device, row-major
 * [batch][width], FP32; host pointers are read or written during the call
 * only.  Device work is queued on the stream given at creation; calls that
 * return host data synchronise it.  Errors in the arguments return
 * PIC_EINVAL with no state change; a failed HIP call returns PIC_EHIP.
 */
#ifndef PIC_MLP_H
#define PIC_MLP_H

#include <stdint.h>

#include "pic.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MLP_MAX_LAYERS 15     /* at most 16 widths */
#define PIC_MLP_MAX_WIDTH 4096

typedef struct pic_mlp pic_mlp;

/* pic_mlp_create: a network of n_widths widths (2 .. 16, each 1 .. 4096) with
 * room for batches of up to max_batch samples.  Parameters start at zero
 * (set them with pic_mlp_set_params); device memory comes from `alloc`
 * (hipMalloc when NULL) and work goes to `hip_stream` (NULL: the null stream). */
pic_status pic_mlp_create(const int32_t* widths, int32_t n_widths, int32_t max_batch,
                          const pic_allocator* alloc, void* hip_stream, pic_mlp** out);

/* number of parameters (floats) of the network */
int64_t pic_mlp_n_params(const pic_mlp* net);

/* pic_mlp_set_params: copy n = pic_mlp_n_params floats from host `params` into
 * the FP32 master weights and their BF16 copy, and clear the Adam state
 * (moments and update count).  Synchronous. */
pic_status pic_mlp_set_params(pic_mlp* net, const float* params, int64_t n);

/* pic_mlp_get_params: copy the FP32 master weights to host `params`.  Synchronous. */
pic_status pic_mlp_get_params(pic_mlp* net, float* params, int64_t n);

/* pic_mlp_forward: y_dev[batch][w[L]] = network(x_dev[batch][w[0]]), with the
 * BF16 weights.  Asynchronous. */
pic_status pic_mlp_forward(pic_mlp* net, int32_t batch, const float* x_dev, float* y_dev);

/* pic_mlp_train_step: one Adam update on the batch (x_dev, t_dev[batch][w[L]]):
 * forward, loss, backward, then w <- w - lr m_hat / (sqrt(v_hat) + eps) with
 * moments of rates beta1, beta2.  The loss of the batch before the update goes
 * to loss_dev[0] when it is not NULL.  Asynchronous. */
pic_status pic_mlp_train_step(pic_mlp* net, int32_t batch, const float* x_dev, const float* t_dev, float lr,
                              float beta1, float beta2, float eps, float* loss_dev);

/* pic_mlp_grad: the loss of the batch and its gradient with respect to the
 * parameters (layout above) into host grad[n_params] and loss[0], without an
 * update.  Synchronous. */
pic_status pic_mlp_grad(pic_mlp* net, int32_t batch, const float* x_dev, const float* t_dev, float* grad,
                        float* loss);

/* wait for the network's queued work */
pic_status pic_mlp_sync(pic_mlp* net);

/* release everything; NULL is a no-op */
void pic_mlp_free(pic_mlp* net);

#ifdef __cplusplus
}
#endif

#endif
