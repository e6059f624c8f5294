/*
 * adr_cnn.h -- learned initial guess for the solver of adr.h.
 *
 * A small convolutional network maps per-node input fields of an instance on
 * the (nx+2) x (ny+2) node grid (interior unknowns plus the boundary ring) to
 * a guess of u; the guess only seeds BiCGSTAB (Section 5.2), which still runs
 * in FP64 to the same stopping test, so the answer is that of the plain
 * solver.  A guess that is not finite or whose residual is not below that of
 * the zero guess (||b - A x0||_2 >= ||b||_2) is replaced by zero.
 *
 * Network (fixed architecture): six 3x3 convolutions with zero padding,
 * channels 10 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, exact GELU
 * (x * Phi(x)) after the first five.  Weights and the activations between
 * layers are stored in bfloat16 (round to nearest even); products are
 * accumulated in FP32.  The pre-activations of the hidden layers are kept in
 * FP32 for the backward pass.  Training minimises the mean squared error
 * over the interior nodes with Adam; gradients entering each convolution are
 * rounded to bfloat16, accumulations are FP32 (weight and bias gradients are
 * summed over the batch in FP64 from FP32 per-workgroup partials, in a fixed
 * order, so a step is deterministic).
 *
 * Tensors are channels-last ("NHWC"): element (b, row, col, c) of a
 * [B][H][W][C] tensor is at ((b*H + row)*W + col)*C + c; row is the y index
 * and col the x index of the node, both counted from the boundary ring.
 * Network inputs always have 32 channels in memory, of which the first ten
 * are the fields below and the rest are zero.
 *
 * Input fields of node (I, J), x = I*dx, y = J*dy, I, J in [0, n+1]:
 *   0: a(x)/5 = (1 + x^2)/5
 *   1: b(y)/2 = X exp(-y)/2
 *   2: interior node: f/10; ring node with Dirichlet data: the exact u;
 *      ring node on a Neumann side: the exact normal derivative
 *      (x = X: du/dx, y = Y: du/dy; 0 at the corner (X, Y))
 *   3: log10(eps)/3
 *   4: 0 for interior nodes, +1 for Dirichlet ring nodes, -1 for Neumann
 *   5, 6: x/X, y/Y;  7, 8: X/2, Y/2 (the node's place in its domain: six
 *      layers of 3x3 convolutions see 13 x 13 nodes, far too few to locate a
 *      node of a large grid from the other fields)
 *   9: the scheme of the convection term: 0 upwind, 1 centered (Section 4)
 *
 * Parameters are exchanged as one packed FP32 vector: for each layer in
 * order, its weights W[ky][kx][ci][co] (cross-correlation: output at node
 * (row, col) reads input (row + ky - 1, col + kx - 1)) followed by its biases
 * b[co].  adr_cnn_param_count() gives the length (40193).
 *
 * All device pointers are plain HIP device memory owned by the caller; all
 * calls are synchronous on the network's stream on return.  Errors: as in
 * adr.h (ADR_ERR_ARG before any device work, ADR_ERR_NOMEM, ADR_ERR_DEVICE;
 * text from adr_last_error()).
 */
#ifndef ADR_CNN_H
#define ADR_CNN_H

#include <stdint.h>

#include "adr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adr_cnn adr_cnn;

/* Number of packed FP32 parameters. */
int64_t adr_cnn_param_count(void);

/* Network for node grids of height x width (= ny+2, nx+2) and batches of at
 * most max_batch instances; parameters start at zero (set them with
 * adr_cnn_set_params).  stream: hipStream_t or NULL.  Device memory is about
 * max_batch * height * width * 1 KB. */
adr_status adr_cnn_create(int32_t height, int32_t width, int32_t max_batch, void *stream,
                          adr_cnn **out);
void adr_cnn_destroy(adr_cnn *net);

/* Copy the packed parameters in (host, param_count floats) and reset the
 * Adam moments and step count; or copy them out. */
adr_status adr_cnn_set_params(adr_cnn *net, const float *params_host);
adr_status adr_cnn_get_params(const adr_cnn *net, float *params_host);

/* Inference: in_dev [batch][H][W][32] bfloat16 bits, u_dev [batch][H][W]
 * FP32 (output of the last layer). */
adr_status adr_cnn_forward(adr_cnn *net, const uint16_t *in_dev, int32_t batch, float *u_dev);

/* Forward and backward pass of the loss
 *   L = sum over the batch and interior nodes of (u - target)^2 / (batch (H-2) (W-2))
 * target_dev: [batch][H-2][W-2] FP32 (interior nodes, x fastest).  The
 * gradient is kept on the device for adr_cnn_adam; grad_host (param_count
 * floats) and loss_host receive copies when not NULL; u_dev, when not NULL,
 * receives the network output [batch][H][W]. */
adr_status adr_cnn_gradient(adr_cnn *net, const uint16_t *in_dev, const float *target_dev,
                            int32_t batch, float *u_dev, float *grad_host, double *loss_host);

/* One Adam step (Kingma & Ba, ICLR 2015, with bias correction) on the last
 * gradient: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
adr_status adr_cnn_adam(adr_cnn *net, float lr, float beta1, float beta2, float eps);

/* adr_cnn_gradient followed by adr_cnn_adam(lr, 0.9, 0.999, 1e-8). */
adr_status adr_cnn_train_step(adr_cnn *net, const uint16_t *in_dev, const float *target_dev,
                              int32_t batch, float lr, double *loss_host);

/* Input fields (see above) of instances [first, first + count) of a problem
 * from adr_assemble / adr_batch_assemble, written to out_dev
 * [count][ny+2][nx+2][32] bfloat16 bits.  The instances must share nx and
 * ny.  Synchronous on the problem's stream. */
adr_status adr_cnn_features(const adr_problem *p, int32_t first, int32_t count, uint16_t *out_dev);

/* Initial guess for every instance of p (all of nx = width-2, ny = height-2
 * of the network): features, inference in chunks of max_batch, interior
 * values widened to FP64 into x_dev (the batched layout of adr_batch_layout),
 * then the fallback test against the zero guess.  used_guess (host, count
 * entries, may be NULL): 1 where the network's guess was kept, 0 where x_dev
 * was set to zero.  Pass x_dev as x0 to adr_batch_solve. */
adr_status adr_batch_warm_start(adr_problem *p, adr_cnn *net, double *x_dev, int32_t *used_guess);

#ifdef __cplusplus
}
#endif

#endif /* ADR_CNN_H */
