/*
 * kl_surrogate.h -- C ABI of the learned occupancy surrogate of libkl.
 *
 * A small network maps the traces (ta, tb) of a once-punctured-torus group
 * to a 128 x 128 occupancy image of its depth-14 limit set over [-2, 2]^2
 * (the image the renderer of kl.h draws, thresholded at count > 0).  It is
 * trained on renders the renderer itself produces, and the plain renderer
 * remains both its fallback and the reference for its IoU.  None of this is in
 * the paper (whose Section 7 only notes that the method needs
 * acceleration); the shapes are:
 *   u  = [(Re ta - 2.4)/0.6, Im ta/0.3, (Re tb - 2.4)/0.6, Im tb/0.3]
 *   h1 = relu(u W1 + b1)            W1: 4 x 256      (row = input feature)
 *   h2 = relu(h1 W2 + b2)           W2: 256 x 256;   h2 read as 16 x 4 x 4 (c, y, x)
 *   c1 = relu(convT(h2, K1, s4 p0)) K1: 16 x 64 x 4 x 4  (in, out, ky, kx)
 *   c2 = relu(convT(c1, K2, s2 p1)) K2: 64 x 32 x 4 x 4
 *   c3 = relu(convT(c2, K3, s2 p1)) K3: 32 x 16 x 4 x 4
 *   z  =      convT(c3, K4, s2 p1)  K4: 16 x 1 x 4 x 4;  z: logits, 128 x 128
 * where convT(x, K, s, p)[o, s*i - p + ky, s*j - p + kx] += x[c, i, j] K[c, o, ky, kx],
 * plus a bias per output channel.  Loss: mean binary cross entropy of
 * sigmoid(z) against the occupancy.  Optimiser: Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8) on FP32 master weights.
 *
 * Arithmetic: the operands of every matrix product are rounded to bfloat16
 * (nearest even) and its products accumulated in FP32; everything else is
 * FP32.  kl_sur_forward runs the whole network of one set in one workgroup,
 * activations in LDS: the first linear layer (four inputs) on the vector
 * ALUs, every other product on the BF16 matrix cores.  Training runs every
 * product (the transposed convolutions in their column form, and all the
 * gradients) on the matrix cores.
 *
 * Parameters: one flat FP32 device vector of kl_sur_num_params() values in
 * the order W1 b1 W2 b2 K1 c1 K2 c2 K3 c3 K4 c4, each row-major as shaped
 * above.  Pointers are device pointers unless stated otherwise; `stream` is
 * a hipStream_t (NULL = null stream); all calls are asynchronous.  Error
 * codes as in kl.h; arguments are checked before anything is enqueued.
 */
#ifndef KL_SURROGATE_H
#define KL_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "kl.h"

#ifdef __cplusplus
extern "C" {
#endif

#define KL_SUR_IMG 128

size_t kl_sur_num_params(void);

/* Bytes of device workspace one forward / training call on `batch` sets needs
 * (1 <= batch <= 512 for the calls below). */
size_t kl_sur_workspace_bytes(int batch);

/* The training path's FP32 buffers in a workspace of `batch` sets, as
 * kl_sur_loss_grad (and kl_sur_train_step) leave them, for checking each
 * layer on its own inputs: offset in bytes from the workspace's start and
 * number of floats.  Layouts (b the set; NHWC = set, row, column, channel):
 *   U       b x 4 features       H1, H2   b x 256 (after bias and ReLU)
 *   X0      H2 as NHWC 4 x 4 x 16 (H2 feature c * 16 + q is pixel q, channel c)
 *   Y1      NHWC 16 x 16 x 64    Y2  NHWC 32 x 32 x 32    Y3  NHWC 64 x 64 x 16
 *   LOGITS  b x 128 x 128        DLOGITS  d loss / d logits, b x 128 x 128
 *   DY3, DY2, DY1  d loss / d Y3, Y2, Y1 (ReLU mask applied), as Y3, Y2, Y1
 *   DX0     d loss / d X0 (NHWC 4 x 4 x 16)
 *   DH2, DH1  d loss / d H2, H1 (ReLU mask applied), b x 256
 * Errors: KL_EINVAL (batch <= 0, NULL outputs, unknown tensor). */
enum {
    KL_SUR_T_U = 0, KL_SUR_T_H1, KL_SUR_T_H2, KL_SUR_T_X0, KL_SUR_T_Y1, KL_SUR_T_Y2, KL_SUR_T_Y3, KL_SUR_T_LOGITS,
    KL_SUR_T_DLOGITS, KL_SUR_T_DY3, KL_SUR_T_DY2, KL_SUR_T_DY1, KL_SUR_T_DX0, KL_SUR_T_DH2, KL_SUR_T_DH1
};
int kl_sur_workspace_tensor(int batch, int which, size_t *offset_bytes, size_t *n_floats);

/* logits_out: batch x 128 x 128 FP32 (row-major image per set). */
int kl_sur_forward(const float *params, const kl_c64 *ta, const kl_c64 *tb, int batch,
                   float *logits_out, void *workspace, size_t workspace_bytes, void *stream);

/* Mean loss (one FP32 in loss_out) and its gradient (grad_out, kl_sur_num_params
 * FP32) against targets (batch x 128 x 128 bytes, 0 or 1). */
int kl_sur_loss_grad(const float *params, const kl_c64 *ta, const kl_c64 *tb, const uint8_t *targets,
                     int batch, float *grad_out, float *loss_out, void *workspace,
                     size_t workspace_bytes, void *stream);

/* One Adam step (step counts from 1) on params with moments m, v. */
int kl_sur_adam(float *params, const float *grad, float *m, float *v, int step, float lr, void *stream);

/* kl_sur_loss_grad then kl_sur_adam; grad_scratch holds kl_sur_num_params FP32. */
int kl_sur_train_step(float *params, float *m, float *v, float *grad_scratch, int step, float lr,
                      const kl_c64 *ta, const kl_c64 *tb, const uint8_t *targets, int batch,
                      float *loss_out, void *workspace, size_t workspace_bytes, void *stream);

/* occ_out[i] = counts[i] > 0 (the occupancy of a rendered image). */
int kl_occupancy(const uint32_t *counts, uint64_t n, uint8_t *occ_out, void *stream);

/* occ_out[i] = logits[i] > 0 (the surrogate's predicted occupancy). */
int kl_sur_predict_occupancy(const float *logits, uint64_t n, uint8_t *occ_out, void *stream);

/* Per set: mean over pixels of the binary entropy (nats) of sigmoid(logit);
 * the gate accepts a prediction whose value is below a calibrated threshold. */
int kl_sur_uncertainty(const float *logits, int batch, float *out, void *stream);

/* Per set: |P and T| / |P or T| with P = logits > 0 (or pred_occ if logits
 * is NULL) and T = target occupancy; 1 when both are empty. */
int kl_iou(const float *logits, const uint8_t *pred_occ, const uint8_t *target_occ, int batch,
           float *iou_out, void *stream);

/* The matrix product the network is built from, exposed for testing:
 * C (M x N, FP32, row stride ldc) = [C +] A B [+ bias[n]], [relu], with
 * A(i, k) = A[i * lda_m + k * lda_k] and B(k, j) = B[k * ldb_k + j * ldb_n]
 * rounded to bfloat16, FP32 accumulation.  accumulate != 0 adds to C (no
 * bias or relu then). */
int kl_gemm_bf16(int M, int N, int K, const float *A, int64_t lda_m, int64_t lda_k, const float *B,
                 int64_t ldb_k, int64_t ldb_n, float *C, int64_t ldc, const float *bias, int relu,
                 int accumulate, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* KL_SURROGATE_H */
