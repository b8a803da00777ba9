/*
 * beamlearning.h -- C-ABI of the BeamLearning forward pass in libism.so
 * (AMD Instinct MI355X, gfx950).
 *
 * The operation (paper section II.B): a raw multichannel frame x[c][n],
 * c < c_in, n < n_t, goes through
 *   1. three cascaded filterbank modules of six layers each (II.B.1 and the
 *      filterbank figure).  Layer l (D = 1, 2, 4, 8, 16, 32 in each module):
 *        z[n][c*4 + j] = sum_{k<3} dw[c][j][k] * h[n + (k-1) D][c]   (depthwise,
 *                        channel multiplier 4, zero outside [0, n_t))
 *        a[n][o]       = b[o] + sum_i z[n][i] * pw[i][o]           (pointwise, 128 out)
 *        y             = tanh(LN(a)): the layer norm takes mean and variance
 *                        over all n_t x 128 values of the frame, then applies
 *                        g[o] (a - mean) / sqrt(var + eps) + be[o]
 *        h_next        = y for the first layer, h + y for the other 17
 *      h of the first layer is the frame itself; the last h is S[n][o].
 *   2. pseudo-energy (II.B.2): e[o] = mean over n in [189, n_t - 189) of S[n][o]^2
 *      (the samples that every atrous layer computed from inside the frame),
 *      then f = SELU(LN(e)) with the head's own layer norm (gain g_e, offset be_e).
 *   3. output (II.B.3): out[j] = fc_b[j] + sum_o f[o] fc_w[o][j]; with
 *      BL_CLASSIFICATION the outputs are then a softmax over j.
 *
 * Parameters: one FP32 array of bl_param_count(c_in, n_out) floats in this
 * order (C = c_in for layer 0, 128 after it):
 *   per layer l = 0..17: dw[C][4][3], pw[4C][128], b[128], g[128], be[128];
 *   then g_e[128], be_e[128], fc_w[128][n_out], fc_b[n_out].
 *
 * Arithmetic: layer 0 in FP32 on the vector units; each later layer is one
 * dilated convolution on the matrix cores: the depthwise taps are folded into
 * the pointwise weights (W[k][c][o] = sum_j dw[c][j][k] pw[c*4+j][o], exact in
 * real arithmetic), and the products run as FP16 pairs (hi*hi + hi*lo + lo*hi,
 * FP32 sums), close to FP32 accuracy.  Layer-norm statistics, the
 * pseudo-energies and the head use FP64 sums.
 *
 * Conventions: as for ism.h.  Device pointers stay valid until the queued work
 * has finished; work is queued on `stream`; errors are return codes
 * (ism_status) with text in ism_last_error(h); arguments are validated before
 * any work is queued.  Outputs are bitwise reproducible for the same inputs,
 * batch size and frame length.
 */
#ifndef BEAMLEARNING_H
#define BEAMLEARNING_H

#include <stddef.h>
#include <stdint.h>

#include "ism.h"

#ifdef __cplusplus
extern "C" {
#endif

enum bl_mode {
    BL_REGRESSION = 0,     /* outputs are the fully connected layer's values */
    BL_CLASSIFICATION = 1  /* outputs are a softmax of them (class probabilities) */
};

#define BL_NF 128          /* filter channels per layer */
#define BL_MAX_CIN 32      /* largest number of input channels */
#define BL_MAX_NOUT 1024   /* largest number of outputs */
#define BL_MARGIN 189      /* samples dropped at each end by the valid crop */

typedef struct bl_model bl_model;

/* Number of floats in the parameter array (layout above); 0 for sizes out of range. */
size_t bl_param_count(int c_in, int n_out);

/*
 * Prepares a model from its parameters: allocates the model's device memory
 * once, and queues on `stream` the kernel that folds each layer's depthwise
 * taps into its pointwise weights, splits them into FP16 pairs and lays them
 * out for the matrix cores.
 *   c_in: 1..BL_MAX_CIN input channels; n_out: 1..BL_MAX_NOUT outputs;
 *   mode: BL_REGRESSION or BL_CLASSIFICATION; ln_eps: the layer norms' eps (> 0).
 *   params: device FP32 array, read by the queued kernel only (it may be freed
 *   once that work is done).  *model receives the model; bl_model_destroy frees it
 *   (after waiting for the device).  The model lives on the device that is current
 *   at creation and is ready once the work queued on `stream` has finished: a
 *   forward pass on another stream must be ordered after it (an event, or a
 *   stream or device synchronisation).
 * ISM_EINVAL for sizes out of range or non-finite eps, ISM_ENOMEM if the
 * allocation fails.
 */
int bl_model_create(ism_handle *h, int c_in, int n_out, int mode, float ln_eps, const float *params,
                    ism_stream stream, bl_model **model);
void bl_model_destroy(bl_model *model);

/* Device workspace bytes bl_forward needs for `batch` frames of n_t samples. */
size_t bl_workspace_bytes(int batch, int n_t);

/*
 * Forward pass over `batch` frames.
 *   x: device FP32; frame b, channel c, sample n at
 *      x[off_b + c * ch_stride + n], off_b = x_offsets[b] if x_offsets is not
 *      NULL (a device int64 array of batch entries), else b * ex_stride.  Frames
 *      may overlap (read only).  Every such element, for b < batch, c < c_in and
 *      n < n_t, must lie inside the caller's allocation: the library cannot check
 *      device offsets.
 *   n_t: frame length, 2*BL_MARGIN + 1 .. 1 << 20.
 *   workspace: device, at least bl_workspace_bytes(batch, n_t) bytes, owned by
 *      the caller; its contents on entry do not matter.  The call allocates nothing.
 *      Calls that share a workspace must not run concurrently.
 *   features: device FP32 batch x 128 (f above), or NULL.
 *   out: device FP32 batch x n_out.
 * A frame's features and outputs are bitwise the same whatever the batch it runs
 * in (the launch shape changes with the batch size, the arithmetic does not).
 * batch = 0 queues nothing.  ISM_EINVAL for a NULL pointer, n_t out of range,
 * a negative stride or a workspace that is too small.
 */
int bl_forward(ism_handle *h, const bl_model *model, int batch, int n_t, const float *x,
               const int64_t *x_offsets, int64_t ex_stride, int64_t ch_stride, void *workspace,
               size_t workspace_bytes, float *features, float *out, ism_stream stream);

/*
 * bl_forward without allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid it).
 * Arguments and results as for bl_forward, without the workspace: the workspace is a
 * fixed device array of bl_noalloc_scratch_bytes() bytes (64 MiB) per GPU inside the
 * library, held until the process ends, through which the batch passes as many frames
 * at a time as it holds (the results equal bl_forward's bitwise).  The call allocates
 * nothing.  Every call on one GPU shares that array: calls that overlap on a GPU (on
 * different streams, or from different threads) race and must be serialised by the
 * caller.  Call with the handle's device current.  ISM_EINVAL as for bl_forward, and
 * when one frame's workspace exceeds the array (n_t above about 32 600 samples).
 */
size_t bl_noalloc_scratch_bytes(void);
int bl_forward_noalloc(ism_handle *h, const bl_model *model, int batch, int n_t, const float *x,
                       const int64_t *x_offsets, int64_t ex_stride, int64_t ch_stride, float *features,
                       float *out, ism_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* BEAMLEARNING_H */
