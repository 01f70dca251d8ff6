/*
 * gs_cnn.h -- C ABI of the learned-correction form in libgs_fluid.so:
 * a small 3D convolutional network, run and trained by hand-written BF16
 * MFMA kernels for AMD gfx950, that corrects a 2x coarser FP32 solve of the
 * Euler step (include/gs_fluid.h) toward the fine FP64 solve restricted to
 * the coarse mesh.  Not part of the paper, whose fluid example is the plain
 * step (Section 3); this is a form built on top of that step.
 *
 * Network.  Three 3 x 3 x 3 convolutions, 5 -> 32 -> 32 -> 5 channels, ReLU
 * after the first two.  Ghost cells of every convolution follow the mesh's
 * boundary kind (periodic wrap, or outflow: repeat the edge cell).  Inputs
 * x_f = (U_f - mu_f) / sigma_f for the conserved fields f of the coarse
 * state after a plain step; the correction is delta_f = tau_f (y_f -
 * mean(y_f)), so that it moves no conserved total.  Weights and activations
 * are BF16 (rounded to nearest even from FP32 master copies), products
 * accumulate in FP32 on the matrix cores, biases and outputs are FP32.
 *
 * Parameters (host arrays of gs_cnn_param_count() floats, in this order):
 * W1[32][5][3][3][3], b1[32], W2[32][32][3][3][3], b2[32], W3[5][32][3][3][3],
 * b3[5]; a weight W[o][i][kz][ky][kx] multiplies input channel i at offset
 * (kz-1, ky-1, kx-1) (z, y, x) from the output cell.
 *
 * States.  U is a state of the FP32 form of gs_fluid.h: 2 x 5 x nz x ny x nx
 * floats, head then compensation.  The network reads the head.  Fine states
 * are FP64 [5][2nz][2ny][2nx]; a coarse cell is the mean of the 2 x 2 x 2
 * fine cells it covers.  All pointers are device pointers unless named
 * host_*, aligned to 16 bytes; the caller owns them.
 *
 * Training (gs_cnn_gradients, gs_cnn_train_step) needs periodic boundaries
 * and nx a multiple of 32: the input gradient of a convolution is then
 * again a convolution, with the taps mirrored.
 *
 * Streams and errors follow gs_fluid.h: calls queue work on the handle's
 * stream; those that return host values wait for it.  Status codes are the
 * GS_* codes of gs_fluid.h.
 */
#ifndef GS_CNN_H
#define GS_CNN_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_cnn gs_cnn;

/* Number of floats in a parameter array (36357). */
int gs_cnn_param_count(void);

/*
 * A network for an nx*ny*nz coarse mesh with boundary kind bc (GS_BC_*),
 * ratio of specific heats gamma (for the positivity check of a corrected
 * state), on the current device and the given stream.  Allocates the
 * activations, gradients and optimizer state for that mesh (about 1 KB per
 * cell, plus 57 MB of weight-gradient partial sums); parameters start at
 * zero until gs_cnn_set_params.
 */
int gs_cnn_create(int nx, int ny, int nz, int bc, double gamma, void* stream, gs_cnn** out);

/* Copy parameters in / out (host_params: gs_cnn_param_count() floats).
 * Setting them also resets the optimizer state.  get waits. */
int gs_cnn_set_params(gs_cnn* h, const float* host_params);
int gs_cnn_get_params(gs_cnn* h, float* host_params);

/* Normalisation: mu, sigma (> 0) of the inputs and tau (> 0) of the
 * corrections, 5 host doubles each, one per conserved field. */
int gs_cnn_set_norm(gs_cnn* h, const double* mu, const double* sigma, const double* tau);

/*
 * Input features and correction scales.  mode 0 (default): the inputs are
 * the conserved fields and delta_f = tau_f (y_f - mean(y_f)), as above.
 * mode 1 (scale-aware): the inputs are (log rho, v_x, v_y, v_z, log p) of
 * the cell (FP64 primitive recovery, then normalised by mu and sigma), and
 * delta_f = tau_f (S_f y_f - mean(S_f y_f)) with the cell's local scales
 * S = (rho, rho c, rho c, rho c, E), c the sound speed; training targets are
 * divided by tau_f S_f accordingly.  Under rho, p -> lambda rho, lambda p the
 * inputs only shift and the corrections scale with the state, so one network
 * serves density and pressure ratios far from its training data.
 * clip > 0 clamps each normalised output y_f to [-clip, clip] before it is
 * applied (a per-cell trust region against outputs far outside the
 * training distribution); 0 applies y as it is.  Training is unaffected.
 */
int gs_cnn_set_features(gs_cnn* h, int mode, double clip);

/* Network output y (device [5][nz][ny][nx] floats) for the head of U. */
int gs_cnn_forward(gs_cnn* h, const void* U, float* y);

/*
 * Restriction: U = R(fine) as an FP32 pair (head = R rounded to FP32,
 * compensation = head - R rounded to FP32).
 */
int gs_cnn_restrict(gs_cnn* h, const double* fine, void* U);

/*
 * Training target for the plain-step state U: target_f = (R(fine)_f -
 * (head - compensation)_f) / tau_f (mode 1: / (tau_f S_f)), device
 * [5][nz][ny][nx] floats, computed in FP64.
 */
int gs_cnn_make_target(gs_cnn* h, const double* fine, const void* U, float* target);

/*
 * Loss L = mean over cells and fields of (y - target)^2 for the head of U,
 * and the gradient of L with respect to every parameter (host_grads, the
 * parameter layout).  Waits; *loss receives L.  No update.
 */
int gs_cnn_gradients(gs_cnn* h, const void* U, const float* target, float* host_grads,
                     double* loss);

/*
 * One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on L
 * for one sample.  If loss is not NULL the call waits and *loss receives L
 * before the update; otherwise it does not wait.
 */
int gs_cnn_train_step(gs_cnn* h, const void* U, const float* target, float lr, double* loss);

/*
 * Apply the correction to the state U in place (head and compensation,
 * Kahan-summed).  Falls back to leaving U unchanged when the corrected state
 * would hold a cell with density or pressure <= 0 or not finite, or when,
 * for some conserved field, the summed change of the represented state
 * (head - compensation) exceeds 1e-5 of the summed magnitudes of the
 * per-cell changes (or either sum is not finite).  Since the mean is removed
 * in FP64 before the per-cell deltas are rounded to FP32, a finite
 * correction moves each total by rounding only and passes this second
 * check; it guards against rounding blow-up and non-finite sums.  The
 * decision is taken on the device, no host wait.
 */
int gs_cnn_correct(gs_cnn* h, void* U);

/* Corrections applied and fallbacks taken since creation (waits). */
int gs_cnn_counts(gs_cnn* h, int* applied, int* fallbacks);

int gs_cnn_set_stream(gs_cnn* h, void* stream);
void gs_cnn_destroy(gs_cnn* h);
const char* gs_cnn_last_error(const gs_cnn* h);

#ifdef __cplusplus
}
#endif

#endif /* GS_CNN_H */
