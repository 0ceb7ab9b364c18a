/*
 * ep_net.h - learned warm start of the 3D increment solver (libep.so).
 *
 * An addition to the paper's method, not part of it: the paper starts the
 * PT iteration of every increment from the previous increment's velocities.
 * Here a small convolutional network predicts the velocity change of the
 * next increment from the current state, and ep_load_step starts from the
 * predicted velocities when their physical residual is lower than that of
 * the previous velocities (otherwise from the previous velocities, as the
 * paper does).  The stopping rule and its normaliser are those of the plain
 * start, so a warm-started increment is converged to the same tolerance.
 *
 * Network: 3-level encoder-decoder of 3x3x3 'same' convolutions (zero
 * padding) with ReLU; widths 16 -> C -> 2C -> 4C -> 2C -> C -> 16; 2x2x2 mean
 * pooling down, nearest-neighbour upsampling and additive skips up.  Weights
 * and activations are bfloat16, products accumulate in FP32 on the matrix
 * cores; master weights, gradients and Adam moments are FP32.
 *   input channels at cell (i,j,k): tau_xx, tau_yy, tau_zz, and tau_xy,
 *     tau_xz, tau_yz averaged from the 4 surrounding edges (/ scale[0]);
 *     p (/ scale[0]); accumulated plastic strain (/ scale[1]); the previous
 *     increment's velocity change at the cell's lower x, y, z faces
 *     (/ scale[2]); channels 11..15 zero.
 *   output channels 0..2 at cell (i,j,k): the velocity change of the next
 *     increment at the cell's lower x, y, z faces, times scale[3].  Wall
 *     faces keep their prescribed velocities.
 *   the network volume is the grid rounded up to multiples of 4; cells
 *     beyond the grid have zero features and are not trained.
 * Training: mean squared error over the interior faces, Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).
 *
 * Parameters (ep_net_params): FP32, per layer l = 0..10 the weights
 * [Cout][27][Cin] (taps (dz,dy,dx) in {-1,0,1}^3, dz slowest) then the
 * biases [Cout].
 *
 * Conventions as in ep.h: return codes EP_*; one caller-owned device
 * workspace; all work on the stream given to ep_net_init; a network serves
 * solver handles of exactly its grid (3D) on the same device.
 */
#ifndef EP_NET_H
#define EP_NET_H

#include "ep.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ep_net_config {
    int   nx, ny, nz;        /* solver grid (cells), each >= 4 */
    int   base;              /* level-0 channels C: 16 or 32 */
    int   max_samples;       /* training samples held on the device (>= 0); 0: an inference-only
                                network (no sample slots, no activation gradients: about half
                                the workspace); ep_net_train and ep_net_gradient then fail.
                                A training network (> 0) also holds a 32 MiB buffer of partial
                                gradient sums, added in a fixed order: its gradients and training
                                runs repeat bit for bit */
    float scale[4];          /* stress, plastic strain, input velocity change, output velocity change (> 0) */
    int   seed;              /* weight initialisation: He-normal, zero head */
} ep_net_config;

typedef struct ep_net ep_net;

/* Workspace bytes; EP_EINVAL for an invalid configuration. */
int ep_net_workspace_size(const ep_net_config* c, size_t* bytes);

/* Create a network in a caller-owned workspace (256-byte aligned). */
int ep_net_init(const ep_net_config* c, void* d_workspace, size_t ws_bytes, void* stream, ep_net** out);

/* Number of FP32 parameters. */
long ep_net_param_count(const ep_net* n);

/* Copy the FP32 master parameters to (EP_GET) or from (EP_SET) the host
 * (count = ep_net_param_count).  EP_SET resets the Adam moments. */
int ep_net_params(ep_net* n, int dir, float* host, size_t count);

/* Sample slot I/O (for checks): x = D*H*W*16 FP32 values (network volume,
 * x fastest, channel last; rounded to bfloat16 on EP_SET), t = D*H*W*4
 * FP32 targets (channels 0..2 used).  Either pointer may be NULL. */
int ep_net_sample(ep_net* n, int slot, int dir, float* x, float* t);

/* Features of the solver's current state into sample slot `slot` (slot -1:
 * the inference input). */
int ep_net_record(ep_net* n, ep_handle* h, int slot);

/* After an increment of h: the velocity change since the previous call is
 * the tracked "previous change" of the features and, for slot >= 0, the
 * target of that slot.  The first call only starts the tracking (change 0). */
int ep_net_observe(ep_net* n, ep_handle* h, int slot);

/* Forget the tracked velocities: the next ep_net_observe starts a new
 * trajectory (change 0). */
int ep_net_reset(ep_net* n);

/* Forward pass on a slot (-1: the inference input); y (may be NULL):
 * D*H*W*16 FP32 outputs. */
int ep_net_forward(ep_net* n, int slot, float* y);

/* Loss and FP32 parameter gradient of one slot, without updating. */
int ep_net_gradient(ep_net* n, int slot, double* loss, float* grad);

/* nsteps Adam steps, step s on slot slots[s % nslots]; losses (may be NULL)
 * gets the loss of each step (before its update). */
int ep_net_train(ep_net* n, const int* slots, int nslots, int nsteps, float lr, float* losses);

/* Predict the next increment's velocities of h from its current state (the
 * tracked previous change included) and hand them to h as the starting
 * guess of its next ep_load_step. */
int ep_net_predict(ep_net* n, ep_handle* h);

void ep_net_destroy(ep_net* n);
const char* ep_net_last_error(const ep_net* n);

#ifdef __cplusplus
}
#endif
#endif /* EP_NET_H */
