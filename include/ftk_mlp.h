/*
 * ftk_mlp.h -- learned template proposal for the FTK library (gfx950).
 *
 * The paper aligns every image against every template.  This part adds a
 * small network that looks at rotation-invariant Fourier-Bessel features of
 * an image and proposes a short list of templates; the FTK then aligns the
 * image against that list only, and falls back to the full FTK search when
 * the network is not confident.  The FTK itself produces the training
 * labels (best template and shift radius of each synthetic image).
 *
 *   features  F[m * n_q + q] = |a(k_m; q)|^2, m < n_r, 0 <= q < n_q: a
 *             rotation multiplies a(k; q) by a phase (Section 3's rotation
 *             property of the coefficients), so F is rotation invariant;
 *             for a real image |a(k; -q)| = |a(k; q)|.
 *   network   x = (F - mu) * inv_sigma; h_{l+1} = relu(h_l W_l^T + b_l)
 *             for the hidden layers, the last layer linear; W_l is
 *             [dims[l+1]][dims[l]] row-major; the logits split into a
 *             template head [0, n_template) and a shift-radius head
 *             [n_template, n_template + n_shift).
 *   loss      mean over the batch of the softmax cross-entropy of each head.
 *   optimiser AdamW (decoupled weight decay on weights, not biases) on FP32
 *             master parameters.
 *   precision FTK_MLP_BF16: bf16 copies of weights and activations as MFMA
 *             operands, FP32 accumulation, FP32 master weights and
 *             gradients; FTK_MLP_FP32: FP32 operands on FP32 MFMA.
 *
 * Conventions are those of ftk.h (status codes, device pointers, streams as
 * void*, ftk_last_error_message).  An ftk_mlp is not thread safe.
 */
#ifndef FTK_MLP_H
#define FTK_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "ftk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ftk_mlp ftk_mlp;

enum { FTK_MLP_FP32 = 0, FTK_MLP_BF16 = 1 };
enum { FTK_MLP_MAX_LAYERS = 8 };

typedef struct ftk_mlp_info_t {
  int nlayers;
  int dims[FTK_MLP_MAX_LAYERS + 1];
  int n_template;
  int n_shift;
  int precision;
  int max_batch;
  int64_t step;            /* AdamW steps taken */
  size_t param_count;
  size_t device_bytes;
} ftk_mlp_info_t;

/* Create a network with nlayers linear layers of widths dims[0..nlayers]
 * (dims[nlayers] = n_template + n_shift, n_template >= 1, n_shift >= 0,
 * every width in [1, 65536], nlayers in [1, FTK_MLP_MAX_LAYERS]).  All
 * device memory for batches of up to max_batch rows (1..65536) is
 * allocated here.  Parameters start at zero, the input standardisation at
 * mu = 0, inv_sigma = 1.  Errors: FTK_EINVAL, FTK_ENOMEM, FTK_EDEVICE. */
int ftk_mlp_create(ftk_mlp** out, const int* dims, int nlayers, int n_template, int n_shift, int precision,
                   int max_batch);
void ftk_mlp_destroy(ftk_mlp* mlp);
int ftk_mlp_info(const ftk_mlp* mlp, ftk_mlp_info_t* out);

/* Host copies of one layer's FP32 master parameters (W [out][in], b [out]);
 * set also refreshes the bf16 copies and clears that layer's AdamW moments.
 * Synchronous.  Errors: FTK_EINVAL, FTK_EDEVICE. */
int ftk_mlp_set_layer(ftk_mlp* mlp, int layer, const float* W, const float* b);
int ftk_mlp_get_layer(const ftk_mlp* mlp, int layer, float* W, float* b);
/* Feature standardisation, host arrays [dims[0]].  Synchronous. */
int ftk_mlp_set_input_norm(ftk_mlp* mlp, const float* mu, const float* inv_sigma);

/* Rotation-invariant (and for FTK_FEATURES_INVARIANT shift-invariant)
 * features of nA images from their coefficients
 * (device [nA][Qa][M] complex64, the layout of ftk_transform) into device
 * float [nA][D], over the first n_r rings (n_r <= M) and modes
 * 0 <= q < n_q (n_q <= Qa/2):
 *   FTK_FEATURES_POWER: D = n_r n_q, F[m n_q + q] = |a(k_m; q)|^2;
 *   FTK_FEATURES_CROSS: D = n_q n_r^2; per mode q a block of the products
 *     c = a(k1; q) conj a(k2; q) of two rings (a rotation multiplies both
 *     factors by the same phase, which cancels; unlike the power features
 *     they keep the phase between rings): s(Re c) for k1 <= k2, then
 *     s(Im c) for k1 < k2, pairs in row-major (k1, k2) order, with
 *     s(x) = sign(x) sqrt|x|;
 *   FTK_FEATURES_INVARIANT: D = n_r n_q, F[m n_q + j] = sqrt|P(k_m; 2 j)|,
 *     P(k; s) = sum_q a(k; q) conj a(k; q - s) (indices mod Qa): the
 *     angular Fourier coefficients of the ring power |Ahat(k, psi)|^2, which
 *     a shift of the image leaves unchanged (eq. Fdk is a phase) and a
 *     rotation only turns (so their moduli are invariant to both); odd s
 *     vanish for real images.
 * Errors: FTK_EINVAL, FTK_EDEVICE. */
enum { FTK_FEATURES_POWER = 0, FTK_FEATURES_CROSS = 1, FTK_FEATURES_INVARIANT = 2 };
int ftk_features(const ftk_plan* plan, const void* coeffs, int nA, int kind, int n_r, int n_q, float* F,
                 void* stream);

/* Logits of nB <= max_batch rows: x device float [B][dims[0]] (raw
 * features; standardised inside), logits device float [B][dims[nlayers]].
 * Errors: FTK_EINVAL, FTK_EDEVICE. */
int ftk_mlp_forward(ftk_mlp* mlp, const float* x, int B, float* logits, void* stream);

/* Loss and gradients of one batch without updating: rows idx[0..B) of the
 * device dataset x_all [n_rows][dims[0]] with labels lab_t, lab_s
 * (device int32 [n_rows]; lab_t in [0, n_template), lab_s in [0, n_shift)
 * or ignored when n_shift = 0).  idx is a device int32 [B] array of row
 * numbers (no bounds check beyond the kernels' own: rows must be valid).
 * The mean loss is written to device float *loss.  Gradients stay in the
 * network (ftk_mlp_get_grad).  Errors: FTK_EINVAL, FTK_EDEVICE. */
int ftk_mlp_gradients(ftk_mlp* mlp, const float* x_all, const int32_t* lab_t, const int32_t* lab_s,
                      const int32_t* idx, int B, float* loss, void* stream);
/* Host copies of the last gradients of a layer (dW [out][in], db [out]).
 * Synchronous. */
int ftk_mlp_get_grad(const ftk_mlp* mlp, int layer, float* dW, float* db);

/* One training step: ftk_mlp_gradients, then AdamW on every layer with
 * the step counter incremented (t starts at 1).  Allocates nothing.
 * Errors: those of ftk_mlp_gradients; FTK_EINVAL for lr < 0, betas outside
 * [0, 1), eps < 0, wd < 0. */
int ftk_mlp_train_step(ftk_mlp* mlp, const float* x_all, const int32_t* lab_t, const int32_t* lab_s,
                       const int32_t* idx, int B, float lr, float beta1, float beta2, float eps, float wd,
                       float* loss, void* stream);

/* Proposal for nA rows of raw features x (device [nA][dims[0]]), in
 * slices of max_batch: the topk templates by logit (ties to the lower
 * index) into top [nA][topk] (device int32), the softmax probability mass
 * of those templates into mass [nA] (device float), and the most likely
 * shift-radius bin into shift_bin [nA] (device int32, 0 if n_shift = 0).
 * 1 <= topk <= min(n_template, 64).  Errors: FTK_EINVAL, FTK_EDEVICE. */
int ftk_propose(ftk_mlp* mlp, const float* x, int nA, int topk, int32_t* top, float* mass, int32_t* shift_bin,
                void* stream);

/* Alignment of each image against its own list of templates:
 *   img_coeffs  : device [nA][Qa][M] complex64
 *   tmpl_coeffs : device [nB][Qa][M] complex64
 *   lists       : device int32 [nA][K], template numbers in [0, nB)
 *   best        : device ftk_pose [nA][K]: the pose of image i against
 *                 template lists[i][j] (bitwise the value ftk_align_coeffs
 *                 gives for that pair)
 * 1 <= K <= 4096.  Requires ftk_set_shifts.  Errors: FTK_EINVAL,
 * FTK_ESTATE, FTK_ENOMEM, FTK_EDEVICE. */
int ftk_align_lists(ftk_plan* plan, const void* img_coeffs, int nA, const void* tmpl_coeffs, int nB,
                    const int32_t* lists, int K, ftk_pose* best, void* stream);

/* Best template per image from per-pair poses: for image i the pair j
 * with the largest value (ties: lower template number), written as
 * best_t[i] = lists[i][j] (or j when lists is NULL) and best_pose[i] =
 * poses[i][j].  poses device [nA][K], outputs device [nA].
 * Errors: FTK_EINVAL, FTK_EDEVICE. */
int ftk_best_template(const ftk_pose* poses, const int32_t* lists, int nA, int K, int32_t* best_t,
                      ftk_pose* best_pose, void* stream);

/* The proposal search: transform the images, features, ftk_propose,
 * ftk_align_lists over the proposed templates, then the full FTK
 * (ftk_align_coeffs against all nB templates) for every image whose mass
 * is below tau; per image the best template and its pose.
 *   images      : device float [nA][n][n]
 *   tmpl_coeffs : device [nB][Qa][M] complex64 (nB = n_template)
 *   best_t      : device int32 [nA]; best_pose: device ftk_pose [nA]
 *   fallback    : device int32 [nA] (1 where the full search ran) or NULL
 *   n_fallback  : host int, number of images searched in full, or NULL
 *   kind, n_r, n_q : the features (ftk_features); their count must equal
 *                 dims[0]
 * With shift windows on the plan (ftk_plan_set_shift_windows, one per shift
 * bin of the network), each image at or above tau is aligned against its
 * list over the shifts of the window of its predicted bin only (the
 * restricted search); images below tau get the full search over all shifts
 * and templates as without windows.  The poses index the plan's shift list.
 * Waits for the proposal before launching the fallback (one host sync; with
 * windows one more per window).
 * Workspace (coefficients, features, proposal, per-pair poses) is held by
 * the plan and the network and grown on demand.
 * Errors: FTK_EINVAL, FTK_ESTATE, FTK_ENOMEM, FTK_EDEVICE. */
int ftk_align_proposed(ftk_plan* plan, ftk_mlp* mlp, const float* images, int nA, const void* tmpl_coeffs, int nB,
                       int kind, int n_r, int n_q, int topk, float tau, int32_t* best_t, ftk_pose* best_pose,
                       int32_t* fallback, int* n_fallback, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FTK_MLP_H */
