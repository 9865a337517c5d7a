/*
 * libnfa -- learned preconditioner for flexible CG (a small 3-D U-Net).
 *
 * Not a method of the paper: the paper's projection uses a preconditioned
 * conjugate-gradient solver with an unnamed preconditioner (Introduction);
 * this network is an optional preconditioner of the flexible-CG variant of
 * that solve (NFA_PC_UNET), held to the same FP64 true residual and backed
 * by Jacobi-PCG.
 *
 * Network (channels-last BF16 activations, FP32 accumulation, 3x3x3
 * cross-correlations with zero padding, 2x2x2 average pooling, nearest x2
 * upsampling, additive skips):
 *   x0 = [r/s, (log(1/rho) - L0)/L1]     s = RMS of r over the unknowns
 *   a0 = relu(conv0(x0))            2 -> 16   full resolution
 *   a1 = relu(conv1(pool(a0)))     16 -> 32   1/2
 *   a2 = relu(conv2(pool(a1)))     32 -> 64   1/4
 *   b2 = relu(conv3(a2))           64 -> 32   1/4
 *   d1 = relu(conv4(up(b2) + a1))  32 -> 16   1/2
 *   d0 = relu(conv5(up(d1) + a0))  16 -> 16   full resolution
 *   z  = D^-1 (r/s + head(d0))               16 -> 1, full resolution
 * with D^-1 the Jacobi inverse diagonal of the assembled operator, so the
 * network with a zero head is the Jacobi step.  conv0..conv5 are 3x3x3; the
 * head is 1x1x1.  Grid sizes must be multiples of 4 in every direction.
 *
 * Parameters: weights [taps][cin][cout] (tap t = 9(dz+1) + 3(dy+1) + (dx+1);
 * one tap for the head) then bias [cout] per convolution; FP32 master copies,
 * BF16 used in the convolutions.
 *
 * Training loss for a (residual r, scalar e.A'e with e = A'^-1 r) pair: the
 * share of the A-norm error left by one optimal step along z,
 *   L = 1 - (z.r)^2 / ((z.A'z)(e.A'e)).
 */
#ifndef NFA_UNET_H
#define NFA_UNET_H

#include "nfa.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nfa_unet_s* nfa_unet;

/* Bytes of device workspace a network with `levels` levels on an
 * nx x ny x nz grid needs: its parameters, their gradients and the two Adam
 * moments (FP32, nfa_unet_param_count each), the packed weight fragments,
 * every activation and activation gradient (BF16, channels-last), the head
 * terms and the weight-gradient partials.  0 for invalid sizes. */
size_t nfa_unet_workspace_bytes(int nx, int ny, int nz, int levels);

/* Network with `levels` resolution levels (3 = the network above; each
 * further level adds a 64-channel level with the same encoder / decoder
 * pattern; 3..6) for an nx x ny x nz grid (multiples of 2^(levels-1), at
 * most 2^28 cells: the kernels use 32-bit element offsets);
 * weights He-initialised from `seed`, biases and head zero, Adam moments zero.
 *   workspace : DEVICE, 256-byte aligned, ws_bytes >=
 *               nfa_unet_workspace_bytes(...), owned by the caller and kept
 *               alive while the network exists: every device buffer of the
 *               network is a slice of it, so forward, gradient and training
 *               steps never allocate.  NULL: the library allocates the same
 *               buffers itself, here.
 * Errors: NFA_ERR_NOMEM (workspace too short; nothing created),
 * NFA_ERR_INVALID, NFA_ERR_HIP. */
nfa_status nfa_unet_create(int nx, int ny, int nz, int levels, int seed, void* workspace, size_t ws_bytes,
                           nfa_unet* out);

/* nfa_unet_bind -- keep the parameters (FP32 master copies; the BF16 ones
 * the convolutions read are packed from them), their gradients and the Adam
 * moments in four caller-owned DEVICE arrays of nfa_unet_param_count floats
 * each (distinct, 4-byte aligned, kept alive while the network uses them).
 *   copy = 1 : the network's current values are copied into them first (the
 *              caller takes over the state, e.g. right after creation);
 *   copy = 0 : their contents are the state (resuming saved training); the
 *              packed weights are rebuilt from `params`.
 * Later training steps update them in place.  Synchronous.  Errors:
 * NFA_ERR_INVALID, NFA_ERR_HIP. */
nfa_status nfa_unet_bind(nfa_unet u, float* params, float* grads, float* adam_m, float* adam_v, int copy);
/* Number of FP32 parameters of a network with `levels` levels (-1 if out of
 * range).  Parameter order: encoder e_0..e_{L-1}, bottleneck, decoder
 * d_{L-2}..d_0, head; each weights [taps][cin][cout] then bias [cout], with
 * 27 taps but 1 for the head. */
long long nfa_unet_param_count(int levels);
int nfa_unet_levels(nfa_unet u);
/* HOST buffers of nfa_unet_param_count() floats.  Synchronous. */
nfa_status nfa_unet_get_params(nfa_unet u, float* host);
nfa_status nfa_unet_set_params(nfa_unet u, const float* host);
/* Gradients of the last nfa_unet_grad / nfa_unet_train_step.  Synchronous. */
nfa_status nfa_unet_get_grads(nfa_unet u, float* host);

/* z = network(r) on the operator's grid (same shape as the network).
 *   op   : assembled operator (supplies rho and the Jacobi inverse diagonal).
 *   r    : DEVICE float cells (a residual: zero on slaves and inactive cells).
 *   z    : DEVICE float cells, 16-byte aligned (output; zero on slaves and
 *          inactive cells).
 *   keep : 1 stores every activation (for nfa_unet_export); 0 stores only what
 *          later layers read (the preconditioner's form: the full-resolution
 *          activations stay on chip).
 * ASYNC. */
nfa_status nfa_unet_forward(nfa_unet u, nfa_poisson op, const float* r, float* z, int keep, nfa_stream s);

/* Forward, loss and backward for one pair; gradients replace the previous
 * ones.  eAe = e.A'e > 0.  loss: HOST out.  Synchronous. */
nfa_status nfa_unet_grad(nfa_unet u, nfa_poisson op, const float* r, double eAe, double* loss,
                         nfa_stream s);

/* nfa_unet_grad followed by one Adam step (beta1 0.9, beta2 0.999, eps 1e-8)
 * with learning rate lr at step count t >= 1.  Synchronous. */
nfa_status nfa_unet_train_step(nfa_unet u, nfa_poisson op, const float* r, double eAe, float lr,
                               int t, double* loss, nfa_stream s);

/* Gradients of every parameter for a loss of the caller's: dz (DEVICE, FP32,
 * one value per cell in the grid's layout) is dL/dz at the output z of the
 * last nfa_unet_forward, which must have run with keep = 1 on this operator
 * (its D^-1 scales the output) with the current parameters; otherwise
 * NFA_ERR_INVALID.  The gradients replace the previous ones (read them with
 * nfa_unet_get_grads or from the array bound by nfa_unet_bind).  The same
 * chain rule as nfa_unet_grad, which is forward + the step loss's dL/dz +
 * this call.  ASYNC. */
nfa_status nfa_unet_backward(nfa_unet u, nfa_poisson op, const float* dz, nfa_stream s);

/* One Adam step on the current gradients g:  m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2,  w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t))
 * + eps), elementwise in FP32, then the packed BF16 weights are rebuilt.
 * t >= 1 counts steps from 1; 0 <= b1, b2 < 1; eps > 0.  nfa_unet_train_step
 * uses b1 = 0.9, b2 = 0.999, eps = 1e-8.  ASYNC. */
nfa_status nfa_unet_adam_step(nfa_unet u, float lr, float b1, float b2, float eps, int t, nfa_stream s);

/* Activations of the last forward with keep = 1 or training step (DEVICE
 * destination): BF16 raw uint16,
 * channels-last; level l has n_l = cells / 8^l positions and c_l = 16, 32,
 * 64, 64, ... channels. */
#define NFA_UNET_X0 0  /* n_0 x 2 */
#define NFA_UNET_A 16  /* + l: encoder a_l, n_l x c_l */
#define NFA_UNET_P 32  /* + l: pool(a_l), n_{l+1} x c_l */
#define NFA_UNET_D 48  /* + l: decoder d_l (d_{L-1}: bottleneck), n_l x c_{l-1} (d_0: n_0 x 16) */
/* Gradients of the last nfa_unet_grad, nfa_unet_train_step or
 * nfa_unet_backward (the chain rule through the layers above, in the same
 * order): */
#define NFA_UNET_DZ 64     /* dL/dz of the step loss, FP32, n_0 (nfa_unet_grad / nfa_unet_train_step only) */
#define NFA_UNET_DD 80     /* + l: at decoder l's pre-activation (l = L-1: the bottleneck), shaped as d_l */
#define NFA_UNET_SKIP 96   /* + l, l <= L-2: at decoder l's input up(d_{l+1}) + a_l, n_l x c_l */
#define NFA_UNET_DA 112    /* + l: at encoder l's pre-activation, n_l x c_l */
#define NFA_UNET_DP 128    /* + l, l <= L-2: at the pooled p_l, n_{l+1} x c_l */
nfa_status nfa_unet_export(nfa_unet u, int what, void* dst, nfa_stream s); /* ASYNC */
void nfa_unet_destroy(nfa_unet u);

#ifdef __cplusplus
}
#endif
#endif /* NFA_UNET_H */
