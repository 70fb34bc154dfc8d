/*
 * sur.h -- C ABI of the surrogate of the hybrid lattice Boltzmann step on
 * MI355X (gfx950): a convolutional network that maps the state of a
 * periodic D2Q9 simulation (phi, rho u_x, rho u_y) to the state 50
 * timesteps later (the method of arXiv:0902.3921, Sec. 2, advanced 50 times).
 * The network is trained on trajectories of that method computed by the
 * library's own solver, and the solver remains the reference for its error.
 *
 * Network.  A U-Net of periodic 3x3 convolutions, each followed by a bias
 * and ReLU, with channel widths c0, c1, c2 at full, half and quarter
 * resolution (2x2 mean pooling down, nearest-neighbour upsampling up, skip
 * connections by concatenation), a 1x1 head to 3 channels, and a residual
 * output y = x + head:
 *     e0a 3->c0, e0b c0->c0 | pool | e1a c0->c1, e1b c1->c1 | pool |
 *     b2a c1->c2, b2b c2->c2 | up, concat e1b | d1a c2+c1->c1, d1b c1->c1 |
 *     up, concat e0b | d0a c1+c0->c0, d0b c0->c0 | head c0->3.
 * Convolutions run on the matrix cores with bfloat16 inputs and weights
 * and FP32 accumulation; activations are stored in FP32.
 *
 * Conventions
 *   - States are NHWC FP32 device arrays [batch][height][width][3] with the
 *     channels (phi, rho u_x, rho u_y) in physical units; the network works
 *     on the channels divided by scale[c].
 *   - height and width are multiples of 4; the lattice is periodic.
 *   - Parameters are one FP32 vector: for each convolution in the order
 *     above, W[tap][cin][cout] (tap = 3 (dy + 1) + (dx + 1) for the 3x3
 *     offsets, a single tap for the head), then b[cout].
 *   - Device memory: the caller owns one workspace of sur_workspace_size()
 *     bytes (256-byte aligned); the library allocates nothing.  All work is
 *     enqueued on the caller's stream; calls that return host data
 *     synchronise it.
 *   - Errors: every call returns an hlb_status (include/hlb.h);
 *     sur_last_error() describes the last failure.  Not thread-safe.
 */
#ifndef SUR_H
#define SUR_H

#include <stddef.h>

#include "hlb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sur_net sur_net;

typedef struct {
  int batch;         /* largest batch of any call */
  int height, width; /* lattice, multiples of 4 */
  int c0, c1, c2;    /* channel widths (32, 64, 128 by default) */
  double scale[3];   /* normalisation of (phi, rho u_x, rho u_y) */
} sur_config;

/* Default configuration: batch 1, 256 x 256, widths 32, 64, 128, scales
 * (1, 0.05, 0.05) (rho u of the spinodal workload has an rms of about 0.02
 * at t >= 1000, phi of about 0.9). */
hlb_status sur_config_default(sur_config *cfg);

/* Number of FP32 parameters.  HLB_EINVAL for a NULL argument, a batch or
 * width < 1, or a height or width that is not a positive multiple of 4. */
hlb_status sur_param_count(const sur_config *cfg, size_t *n);

/* Bytes of device workspace (activations and their gradients for the
 * largest batch, parameters, Adam moments, packed bf16 weights, reduction
 * partials). */
hlb_status sur_workspace_size(const sur_config *cfg, size_t *bytes);

/* Creates a network in the caller's workspace (HLB_ESHAPE if it is missing
 * or too small, HLB_EINVAL if not 256-byte aligned).  Parameters start at
 * zero: set them with sur_set_params. */
hlb_status sur_create(sur_net **out, const sur_config *cfg, void *workspace, size_t bytes, void *stream);

/* Copies sur_param_count() FP32 parameters from the host, repacks the bf16
 * weights and resets the Adam moments and step counter.  Synchronises. */
hlb_status sur_set_params(sur_net *net, const float *host);

/* Copies the FP32 parameters to the host.  Synchronises. */
hlb_status sur_get_params(sur_net *net, float *host);

/* y = network(x) for `batch` states (1 <= batch <= cfg.batch); x and y are
 * device arrays as above and may be the same array.  Asynchronous. */
hlb_status sur_forward(sur_net *net, const float *x, float *y, int batch);

/* Loss and gradient: the mean squared error between network(x) and target
 * in normalised units, over every element, and its gradient with respect to
 * the parameters (kept for sur_adam_step; also copied to host_grads if not
 * NULL).  *loss may be NULL.  Synchronises when loss or host_grads is
 * given. */
hlb_status sur_loss_grad(sur_net *net, const float *x, const float *target, int batch, double *loss,
                         float *host_grads);

/* One Adam update (Kingma and Ba) of the parameters with the gradient of
 * the last sur_loss_grad, then a repack of the bf16 weights.  HLB_ESTATE if
 * no gradient has been computed.  Asynchronous. */
hlb_status sur_adam_step(sur_net *net, double lr, double beta1, double beta2, double eps);

/* Runs sur_forward `reps` times with HIP events: ms[0] receives the mean
 * milliseconds of the convolution kernels of one forward, ms[1] of the
 * whole forward; *flops the algorithmic FLOPs of the convolutions of one
 * forward (2 x multiply-adds, unpadded channel counts).  Synchronises. */
hlb_status sur_forward_timed(sur_net *net, const float *x, float *y, int batch, int reps, double ms[2],
                             double *flops);

/* Message of the last failure; net may be NULL for sur_create. */
const char *sur_last_error(const sur_net *net);

/* Destroys the network; does not free the workspace. */
hlb_status sur_destroy(sur_net *net);

#ifdef __cplusplus
}
#endif

#endif /* SUR_H */
