/* Learned surrogate for the fine-region substeps of LTS3, with a residual
 * gate that falls back to the plain solver step.
 *
 * The paper has no surrogate: this is an optional accelerator that replaces
 * Step 3 of Algorithm 2.2 (the M fine SSPRK3 substeps on F) by one evaluation
 * of a message-passing network, and keeps the solver as the authority: every
 * step whose trapezoid residual exceeds the caller's bound tau is recomputed
 * by the plain LTS3 step.
 *
 * Network (the nodes are the cells of F, I1 and I2; two nodes are neighbours
 * when they share an edge):
 *   X   [N x 16] normalised node features (see lts_sur_features)
 *   H0 = relu(X W0 + b0)                                 W0 [16 x 64]
 *   Hl = relu([H_{l-1} | mean over neighbours of H_{l-1}] Wl + bl),
 *                                               l = 1, 2, 3, Wl [128 x 64]
 *   out_h[i] = H3[i] . wh + bh                   fine cells i
 *   out_u[e] = (H3[c1(e)] - H3[c0(e)]) . wu      fine edges e, normal c0 -> c1
 * and the prediction of the state on F one coarse step dt ahead is a
 * forward-Euler step plus the network's correction,
 *   h + dt R_h(x_n) + rms_h * out_h,  u + dt R_u(x_n) + rms_u * out_u,
 * with R the right-hand side of eq:sweTimeStepping.
 * Weights and activations are BF16 with FP32 accumulation on the matrix
 * cores; biases, head weights and the Adam state are FP32.
 *
 * Parameter vector (FP32, n_params = 25985), row-major matrices in order:
 *   W0[16][64], b0[64], W1[128][64], b1[64], W2[128][64], b2[64],
 *   W3[128][64], b3[64], wh[64], wu[64], bh.
 * Normalisation vector (16 floats):
 *   [0:5] feature means, [5:10] inverse standard deviations (0 drops the
 *   column), [10] 1/rms_h, [11] 1/rms_u, [12] rms_h, [13] rms_u, [14:16] 0.
 *
 * Node order: device cell order restricted to F u I1 u I2; fine cells are
 * nodes 0 .. n_fine_cells-1.  lts_sur_node_map gives the caller's numbering.
 *
 * All functions return LTS_OK or an error code with a message in
 * lts_sur_last_error.  A surrogate is tied to the mesh its context had when it
 * was created; re-uploading a mesh invalidates it (LTS_EINVAL afterwards).
 */
#ifndef LTS_SURROGATE_H
#define LTS_SURROGATE_H

#include "lts.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lts_sur lts_sur;

/* Create a surrogate on ctx (mesh uploaded, state set) with n_layers = 3
   message-passing layers of width hidden = 64 (the only supported shape),
   parameters drawn from seed (uniform Glorot bounds, zero biases) and room
   for max_samples training samples.  LTS_EINVAL for other shapes or an empty
   fine region. */
lts_status lts_sur_create(lts_sur **out, lts_ctx *ctx, int n_layers, int hidden, uint64_t seed,
                          int max_samples);

/* Sizes: nodes, fine cells, fine edges, parameters, samples recorded. */
lts_status lts_sur_info(const lts_sur *s, int *n_nodes, int *n_fine_cells, int *n_fine_edges,
                        int *n_params, int *n_samples);

/* Caller numbering of every node (n_nodes) and every fine edge
   (n_fine_edges); either may be NULL. */
lts_status lts_sur_node_map(const lts_sur *s, int32_t *node_cell, int32_t *fine_edge);

/* Training data from the solver itself: n_steps times, store the raw
   features of the context state x_n, advance it one plain LTS3 coarse step
   (Algorithm 2.2, dt, M) and store the correction targets
   x_{n+1} - x_n - dt R(x_n) of h on the fine cells and u on the fine edges.
   Advances the context by n_steps. */
lts_status lts_sur_record(lts_sur *s, double dt, int M, int n_steps);

/* Compute the normalisation vector from samples 0 .. n_samples-1 (feature
   mean and deviation, target RMS; FP64 sums), or set / read it. */
lts_status lts_sur_normalize(lts_sur *s, int n_samples);
lts_status lts_sur_set_norm(lts_sur *s, const float *norm16);
lts_status lts_sur_get_norm(const lts_sur *s, float *norm16);

/* Parameters (n_params floats).  set_params also resets the Adam state. */
lts_status lts_sur_get_params(const lts_sur *s, float *p);
lts_status lts_sur_set_params(lts_sur *s, const float *p);

/* Save the network to the file `path` (its shape, the normalisation vector
   when one is set, and the parameters; FP32, little-endian), or load a file
   written by lts_sur_save into a surrogate of the same shape, on any context
   and mesh (the parameters do not depend on the mesh).  Loading sets the
   normalisation vector when the file holds one and resets the Adam state;
   recorded training samples are not part of the file.  LTS_EINVAL for a file
   that cannot be opened or written, is not such a file, is truncated or
   longer, or has another shape. */
lts_status lts_sur_save(const lts_sur *s, const char *path);
lts_status lts_sur_load(lts_sur *s, const char *path);

/* n_iters Adam steps (lr, beta1 0.9, beta2 0.999, eps 1e-8), step i on the
   recorded sample idx[i].  Loss per step = mean over fine cells of
   (out_h - th/rms_h)^2 + mean over fine edges of (out_u - tu/rms_u)^2 with
   (th, tu) the sample's correction targets;
   losses[i] (may be NULL) receives it.  Synchronises. */
lts_status lts_sur_train(lts_sur *s, const int32_t *idx, int n_iters, float lr, float *losses);

/* Loss and its gradient (n_params) at recorded sample k, parameters
   unchanged. */
lts_status lts_sur_grad(lts_sur *s, int k, float *loss, float *grad);

/* Raw node features of the current context state, [n_nodes][16] FP32:
   0 h + b (in every precision), 1 b, 2 div u =
   (1/A_i) sum_e n_{e,i} l_e u_e, 3 cell vorticity = sum over the cell's
   vertices of (kite area / A_i) times the vertex vorticity, 4 kinetic
   energy K_i (the K of the momentum equation), 5..8 region one-hot
   (F interior, underlined F, I1, I2), 9..15 zero. */
lts_status lts_sur_features(lts_sur *s, float *raw);

/* Network outputs out_h (n_fine_cells) and out_u (n_fine_edges), in
   normalised units, for the current context state. */
lts_status lts_sur_predict(lts_sur *s, float *out_h, float *out_u);

/* n_steps gated coarse steps of size dt with fine ratio M: the network
   advances F; I1, I2 and C follow Algorithm 2.2 with the fine substeps
   replaced by the prediction: Steps 1 and 2 (the coarse stages on
   underlined F, I and C), the interface accumulation of Step 3 over all 3M
   fine stages (F read linearly in time between x_n and the prediction at
   the SSPRK3 stage times t_k, t_k + dt/M, t_k + dt/(2M); interface 1
   predicted from the coarse stages as in Steps 3.x.1; I2 and C at the coarse
   stage), Step 4 on C and Step 5 on I1 u I2.  F then takes the prediction,
   its thickness shifted uniformly by the step's total mass change divided
   by the area of F, so an accepted step conserves mass to rounding.  Then
     r = max over (h on fine cells, u on fine edges) of
         || (x_new - x_n)/dt - (R(x_n) + R(x_new))/2 ||
         / ((|| R(x_n) || + || R(x_new) ||) / 2)
   (the trapezoid-rule defect of the step on F; L2 norms over the fine cells
   or fine edges).  A step with r < tau is kept, any other (r NaN included) is
   recomputed from x_n by the plain LTS3 step (dt, M).  With max_backoff > 0
   a rejection also skips the surrogate for the next b steps (plain LTS3),
   b doubling with every further rejection up to max_backoff and resetting on
   an acceptance; the back-off state persists across calls.  max_backoff = 0
   tries the surrogate on every step.  n_accepted and residuals[n_steps]
   (-1 for a skipped step; either may be NULL) report the outcome.
   Synchronises once per attempted step.  The first call with a new (dt, M)
   allocates the 3M-layer stage buffers of the interface accumulation and
   captures the step's graph.  While the context is in timing mode
   (lts_set_timing), each attempted step is launched rather than replayed and
   its right-hand-side passes (vertex, cell and edge kernels of R(x_n) and
   R(x_new) on F and of Steps 1, 2 and 4) are event-stamped into
   lts_kernel_stats, as are the fallback steps. */
lts_status lts_sur_step(lts_sur *s, double dt, int M, int n_steps, double tau, int max_backoff,
                        int *n_accepted, double *residuals);

const char *lts_sur_last_error(const lts_sur *s);
void lts_sur_destroy(lts_sur *s);

/* The matrix-core kernels of the network on host buffers, for verification:
   Y[N x 64] = A[N x K] W[K x 64] + bias (bias may be NULL; K = 16, 32, ...,
   128) and P[K x 64] = A^T D (D [N x 64]), BF16 inputs as uint16 bit
   patterns, FP32 outputs.  Uses HIP device `device`. */
lts_status lts_nn_gemm_bf16(int device, const uint16_t *A, int N, int K, const uint16_t *W,
                            const float *bias, float *Y);
lts_status lts_nn_gemm_tn_bf16(int device, const uint16_t *A, int N, int K, const uint16_t *D,
                               float *P);

/* The forward product on device buffers, enqueued on `stream` (a hipStream_t;
   NULL: the null stream) without synchronising, for callers that hold device
   memory and for timing the kernel alone: A [N x K] BF16 (K = 16, 32, ...,
   128), W [K x 64] BF16, bias [64] FP32 or NULL; Y_f32 [N x 64] receives
   A W + bias in FP32 and Y_bf16 [N x 64] relu(A W + bias) in BF16, as the
   network's layers store it; either output may be NULL, not both.  All
   pointers are device pointers owned by the caller; N = 0 reads and writes
   nothing (the pointers may then be NULL).  Alignment: A, W, bias and
   Y_f32 16 bytes, Y_bf16 8 bytes.  LTS_EINVAL for bad sizes, missing or
   misaligned operands, LTS_EDEVICE if the launch fails. */
lts_status lts_nn_gemm_bf16_device(const uint16_t *A, int N, int K, const uint16_t *W,
                                   const float *bias, float *Y_f32, uint16_t *Y_bf16,
                                   void *stream);

/* lts_nn_gemm_tn_bf16_device_noalloc: for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving or training
   loops, harnesses that forbid hipMalloc).  Computes the same product as
   lts_nn_gemm_tn_bf16, P [K x 64] FP32 = A^T D with A [N x K] and D [N x 64]
   BF16 bit patterns (K = 16, 32, ..., 128), on device buffers owned by the
   caller, enqueued on `stream` (a hipStream_t of the current device; NULL:
   the null stream) without synchronising.  It calls no hipMalloc, hipFree or
   other allocating routine: the per-block partial sums go to a fixed 16 MiB
   device array inside the library (one copy per GPU, held until the process
   ends), whose address is looked up once per device on the first call made
   with that device current.  N may be at most
   lts_nn_gemm_tn_noalloc_max_rows(K) = 512 * floor(2^24 / (256 K)) rows
   (262,144 at K = 128, 2,097,152 at K = 16); larger N, bad K or a missing
   operand give LTS_EINVAL and enqueue nothing; a failed launch LTS_EDEVICE.
   N = 0 writes zeros to P.  The result is bitwise that of
   lts_nn_gemm_tn_bf16 (same kernels, same row partition).  Every call on one
   GPU shares that GPU's array: calls that overlap in time on one GPU (other
   streams, other host threads) race and give undefined results; calls
   ordered on one stream do not.  lts_nn_gemm_tn_noalloc_max_rows returns 0
   for an unsupported K. */
lts_status lts_nn_gemm_tn_bf16_device_noalloc(const uint16_t *A, int N, int K, const uint16_t *D,
                                              float *P, void *stream);
long long lts_nn_gemm_tn_noalloc_max_rows(int K);

#ifdef __cplusplus
}
#endif

#endif /* LTS_SURROGATE_H */
