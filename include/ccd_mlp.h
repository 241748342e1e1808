/*
 * ccd_mlp.h -- C ABI of the learned warm start of the CCD iteration
 * (companion of ccd.h; same library, same status codes).
 *
 * The iteration of eq. ccd3 starts from the MBPT2 amplitudes
 * t0 = <ab||ij> / eps_ij^ab (eq. ccdGuess).  At the fixed point,
 * t eps_ij^ab = <ab||ij> + (ladder, ring, one-body and quadratic terms): a
 * small network predicts that remainder per amplitude,
 *
 *     t_ij^ab = (v + y / s) / D,   D = eps_i + eps_j - eps_a - eps_b,
 *     v = <ab||ij>,   s = L^3 / (1000 MeV fm^3),
 *
 * so y = 0 is exactly the MBPT2 start.  Packed features of an amplitude
 * (8 floats):
 *     rho / 0.16,  |q|,  |q'|,  eps_i / 100,  eps_j / 100,  eps_a / 100,  eps_b / 100,  v s
 * with q = (k_a - k_b - k_i + k_j) / 2 the relative momentum transfer of
 * <ab|v|ij> (sec. "Two-body interaction"), q' = (k_b - k_a - k_i + k_j) / 2
 * that of the exchanged element, momenta in fm^-1, energies in MeV.
 *
 * Network: g(x) = W3 relu(W2 relu(W1 x + b1) + b2) + b3, 7 inputs, two hidden
 * layers of width 128, relu(z) = max(z, 0).  Prediction, antisymmetric
 * under a <-> b and under i <-> j like t_ij^ab itself:
 *     y = ( g(x) - g(x_ab) - g(x_ij) + g(x_abij) ) / 4,
 * where a swap exchanges the two energies of the pair, takes |q| to |q'| (one
 * swap) and flips the sign of v (one swap).
 *
 * Parameters: one float32 vector of CCD_MLP_NPARAM entries in device memory,
 * offsets below (row-major; W1 column 7 is unused and kept zero).
 * All device pointers are caller-owned.  Work is ordered on the given HIP
 * stream (NULL = default stream); only calls that return host values
 * synchronise it.
 */
#ifndef CCD_MLP_H
#define CCD_MLP_H

#include "ccd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CCD_MLP_WIDTH  128
#define CCD_MLP_NPACK  8
#define CCD_MLP_OFF_W1 0      /* [128][8]   first layer (column 7 unused) */
#define CCD_MLP_OFF_B1 1024   /* [128]                                  */
#define CCD_MLP_OFF_W2 1152   /* [128][128] row = output unit           */
#define CCD_MLP_OFF_B2 17536  /* [128]                                  */
#define CCD_MLP_OFF_W3 17664  /* [128]                                  */
#define CCD_MLP_OFF_B3 17792  /* [1]                                    */
#define CCD_MLP_NPARAM 17800

/* Packed features of every canonical amplitude of `problem` (layout of
 * ccd.h), written to dev_feat [n_amplitudes][8]; if dev_target is not NULL
 * also the training target y* = (t D - v) s of the context's current
 * amplitudes (e.g. after convergence), [n_amplitudes].  Needs a bound
 * workspace.  Errors: CCD_EINVAL, CCD_ESTATE, CCD_EHIP. */
ccd_status ccd_mlp_features(const ccd_ctx* ctx, int32_t problem, float* dev_feat, float* dev_target);

/* y for n amplitudes from packed features (16-byte aligned buffers), with the
 * 128 x 128 layer on FP32 (CCD_PREC_FP32) or BF16 (CCD_PREC_BF16, FP32
 * accumulation) MFMA; in the BF16 form the first layer runs on FP16 MFMA
 * (FP32 accumulation), in the FP32 form in FP32.  dev_y [n]. */
ccd_status ccd_mlp_forward(const float* dev_params, const float* dev_feat, int64_t n, int32_t precision,
                           float* dev_y, void* hip_stream);

/* Bytes of the work buffer (256-byte aligned) for a gradient over n
 * amplitudes, or for training with minibatch n. */
ccd_status ccd_mlp_work_size(int64_t n, size_t* bytes);

/* Loss L = (1/n) sum_e (y_e - y*_e)^2 / 2 over n amplitudes and its gradient
 * dL/dparams (FP32 arithmetic, CCD_MLP_NPARAM entries to dev_grad; b3 and the
 * padding get 0).  loss (host, nullable) synchronises the stream. */
ccd_status ccd_mlp_loss_grad(const float* dev_params, const float* dev_feat, const float* dev_target, int64_t n,
                             float* dev_grad, double* loss, void* dev_work, size_t work_bytes, void* hip_stream);

/* Adam (Kingma and Ba, 2015, Algorithm 1):
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   p -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps). */
typedef struct {
    float lr, beta1, beta2, eps;
    int32_t batch;   /* amplitudes per step */
} ccd_adam_opts;

/* floor(n_order / batch) Adam steps; step s uses the amplitudes
 * dev_order[s*batch .. (s+1)*batch), indices into the n_rows rows of dev_feat
 * ([n_rows][8]) and dev_target ([n_rows]), e.g. a seeded permutation.  An
 * index outside [0, n_rows) is skipped (its amplitude counts as absent) and
 * the call returns CCD_EINVAL after the steps.  dev_m, dev_v: Adam moments
 * (CCD_MLP_NPARAM each, zero before the first step).  *step (host) is Adam's t
 * before the call and is advanced by the number of steps.  mean_loss (host,
 * nullable): mean of the minibatch losses.  Synchronises the stream once at
 * the end.  The work buffer must hold ccd_mlp_work_size(batch) bytes. */
ccd_status ccd_mlp_train(float* dev_params, float* dev_m, float* dev_v, int64_t* step, const float* dev_feat,
                         const float* dev_target, int64_t n_rows, const int32_t* dev_order, int64_t n_order,
                         const ccd_adam_opts* opts, void* dev_work, size_t work_bytes, double* mean_loss,
                         void* hip_stream);

/* Warm start of every problem of the context: features computed on the fly,
 * prediction on MFMA (CCD_PREC_BF16 or CCD_PREC_FP32), amplitudes
 * t = (v + y / s) / D written as the current iterate and the energies
 * recomputed.  A problem falls back to its MBPT2 amplitudes when its warm
 * energy is not finite or when E_warm / E_MBPT2 lies outside [0.5, 2].
 * used_net (host, n_problems, nullable): 1 where the network's amplitudes
 * were kept, 0 where the MBPT2 start was restored.  dev_params NULL restores
 * the MBPT2 start everywhere.  Synchronises the stream. */
ccd_status ccd_warm_start(ccd_ctx* ctx, const float* dev_params, int32_t precision, int32_t* used_net);

#ifdef __cplusplus
}
#endif
#endif /* CCD_MLP_H */
