/*
 * randqlp.h -- C ABI of the MI355X (gfx950) randomized QLP library.
 *
 * Randomized QLP (Kaloorazi, Liu, Chen, de Lamare, arXiv 2110.01011,
 * Section 3, Algorithm 1) factors an m x n matrix A as A ~= Q L P^T with Q
 * (m x d) and P (n x d) orthonormal and L (d x d) lower-triangular whose
 * diagonal tracks the singular values of A.  This library computes the
 * generalised form with d = min(k + p, m, n) sketch columns and q power
 * iterations:
 *
 *   Omega (m x d) standard Gaussian                  (the randn step)
 *   Qbar = orth(A^T Omega)                            (first orth)
 *   repeat q times: Q = orth(A Qbar); Qbar = orth(A^T Q)
 *   Q = orth(A Qbar)                                  (range basis)
 *   P R = A^T Q = (Q^T A)^T,  L = R^T                 (final QR)
 *
 * orth() is the reduced, unpivoted QR with a non-negative R diagonal; q = 0
 * and d = n is Algorithm 1 itself.  Omega is Philox4x64-10 (key = (seed, 0),
 * counter = (l / 4, 0, 0, 0) for the column-major index l = i + j*m, lane
 * l % 4) mapped to normals by Box-Muller, so the leading columns of Omega,
 * Q, P and L do not depend on p.
 *
 * Conventions for every entry point:
 *  - All matrices are column-major with a leading dimension; all matrix
 *    pointers are DEVICE pointers on the current HIP device.
 *  - The caller owns A, Q, L, P.  A is read-only.  Q (m x d), L (d x d) and
 *    P (n x d) are completely overwritten, including the zeros above the
 *    diagonal of L.
 *  - Argument errors are reported before any work is enqueued.
 *  - randqlp_factor returns after the work has completed on opts->stream
 *    (it reads back a small status word), so the outputs are ready.
 *  - The last error message is kept per thread (randqlp_last_error).
 */
#ifndef RANDQLP_H
#define RANDQLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RQLP_OK = 0,
  RQLP_E_INVALID_ARG = 1,  /* bad size, pointer, leading dimension, option */
  RQLP_E_NONFINITE = 2,    /* A holds NaN or Inf; outputs are unspecified  */
  RQLP_E_NOMEM = 3,        /* device allocation failed                     */
  RQLP_E_WORKSPACE = 4,    /* caller workspace smaller than required       */
  RQLP_E_HIP = 5,          /* a HIP runtime call or kernel launch failed   */
  RQLP_E_UNSUPPORTED = 6   /* combination not implemented (see message)    */
} rqlp_status;

/* Element types:
 *  RQLP_F64         A, Q, L, P double.
 *  RQLP_F32         A, Q, P float; L double.
 *  RQLP_MIXED_BF16  A, Q, P float; L double.  A is copied once to bfloat16
 *  RQLP_MIXED_F16   (resp. half), both as A and as A^T, rounded to nearest
 *                   even; the sketch and power-iteration products run on the
 *                   16-bit copies with fp32 accumulation (panels rounded to
 *                   16 bits as they are read); the final projection A^T Q
 *                   uses the fp32 A.  Panels are fp32.
 *  RQLP_MIXED_BF16X3  as RQLP_MIXED_BF16, except that the final projection
 *                   A^T Q runs as a split bfloat16 product: with A = A1 + A2
 *                   and Q = Q1 + Q2 (A1, Q1 rounded to bfloat16, A2, Q2 their
 *                   rounded residuals) it sums A1^T Q1 + A1^T Q2 + A2^T Q1
 *                   with fp32 accumulation: relative error about 2^-16 per
 *                   product term (fp32 accumulation as in RQLP_F32), on the
 *                   bfloat16 matrix cores.  A's residual is a third 16-bit
 *                   copy in the workspace.
 * In every mode the Gram matrices, Cholesky factors and R are double. */
typedef enum {
  RQLP_F64 = 0,
  RQLP_F32 = 1,
  RQLP_MIXED_BF16 = 2,
  RQLP_MIXED_F16 = 3,
  RQLP_MIXED_BF16X3 = 4
} rqlp_precision;

/* Panel QR used for every orth():
 *  AUTO    Cholesky QR with a second pass; if any pass reports a non-positive
 *          or unsafe pivot, the whole factorisation is recomputed with ROBUST.
 *  CHOLQR2 Cholesky QR with a second pass only (no automatic retry).
 *  ROBUST  shifted Cholesky QR, completion of numerically dependent columns
 *          by fresh Gaussian directions, then two more Cholesky QR passes:
 *          an orthonormal Q for any panel, rank-deficient or zero. */
typedef enum { RQLP_PANEL_AUTO = 0, RQLP_PANEL_CHOLQR2 = 1, RQLP_PANEL_ROBUST = 2 } rqlp_panel;

typedef struct {
  int32_t d;            /* sketch width used                              */
  int32_t q_used;       /* power iterations performed                     */
  int32_t breakdowns;   /* Cholesky passes that flagged an unsafe pivot   */
  int32_t robust_rerun; /* 1 if the factorisation was redone with ROBUST  */
  int32_t completed;    /* dependent columns replaced by fresh directions */
  int32_t reserved;
} rqlp_info;

typedef struct {
  int32_t precision;       /* rqlp_precision                               */
  int32_t panel_qr;        /* rqlp_panel                                   */
  int64_t lda, ldq, ldl, ldp; /* leading dimensions; 0 means tight (rows)  */
  void* stream;            /* hipStream_t to run on; NULL = null stream    */
  void* workspace;         /* device scratch; NULL = library-managed cache */
  size_t workspace_bytes;  /* size of workspace when given                 */
  rqlp_info* info;         /* optional host struct filled on return        */
  /* randqlp_factor_auto with k <= 0 (the rank is predicted) only:          */
  double tol;              /* target relative Frobenius error of the rank-k
                              approximation Q L[:, :k] P[:, :k]^T, in (0, 1] */
  int32_t k_max;           /* largest rank: Q, L, P hold min(k_max + p, m, n)
                              columns                                       */
} rqlp_opts;

/* ---- Learned power-iteration and rank predictor ----
 * A small MLP (fp32) reads the spectrum of a cheap sketch and predicts how
 * many power rounds the method needs.  Input: 65 features, the singular
 * values of the 64-column sketch A^T Omega[:, :64] (the leading columns of
 * the method's own Gaussian sketch, same seed) as
 * clamp(log10(sigma_i / sigma_1), -6, 0) / 6 for i = 1..64, then k / 256.
 * Network: 65 -> 128 (ReLU) -> 128 (ReLU) -> 6 logits, class c = q for
 * c = 0..4 and c = 5 for "more than 4".  Parameters: one float vector
 * [W1 b1 W2 b2 W3 b3], each W (fan_in x fan_out) stored column by column.
 * Activations and feature rows are row-major (one sample contiguous).
 * The rank network has the same shape and layout: the same 64 spectrum
 * features, then clamp(-log10(tol), 0, 6) / 6 for the target error tol, and
 * class c means rank k = 8 * 2^c (8 ... 256); it is trained to pick the
 * smallest class whose optimal rank-k error (Eckart-Young, ||sigma_{>k}|| /
 * ||sigma||) is at most tol / 1.05, so that the rank-k QLP approximation
 * with enough power rounds (within 1.05x of that optimum) meets tol. */
#define RQLP_MLP_INPUTS 65
#define RQLP_MLP_HIDDEN 128
#define RQLP_MLP_CLASSES 6
#define RQLP_MLP_PARAMS 25734

typedef struct {
  int32_t q_predicted; /* predictor's class (0..4, 5 = more than 4)          */
  int32_t q_used;      /* power rounds in the returned factors                */
  int32_t judged;      /* 1 if the error judge ran (q_predicted < q_fallback) */
  int32_t resumed;     /* 1 if the judge rejected q_predicted and the power
                          rounds were resumed up to q_fallback                */
  double judge_ratio;  /* the judge's statistic Delta / e^2 (0 if not run)    */
  double est_rel_err;  /* sqrt(1 - ||L||_F^2 / ||A||_F^2) for the q_predicted
                          factors, when judged                                */
  int32_t k_predicted; /* k <= 0: the rank network's k_hat; else k            */
  int32_t k_used;      /* k <= 0: smallest k whose rank-k approximation of the
                          returned factors meets tol (d if none does); else k */
  int32_t d;           /* columns of the returned Q, P (and order of L)       */
  int32_t rank_fallback; /* k <= 0: 1 if no rank <= d met tol and the method
                          was rerun with k_max and q_fallback                 */
  double rank_err;     /* k <= 0: error of the rank-k_used approximation, from
                          sqrt(1 - ||L[:, :k]||_F^2 / ||A||_F^2) (resolves
                          errors down to about 1e-8)                          */
} rqlp_auto_info;

/* Fill *opts with defaults: F64, AUTO, tight leading dimensions, null
 * stream, library-managed workspace, no info. */
void rqlp_opts_default(rqlp_opts* opts);

/* d = min(k + p, m, n), or -1 for negative or zero sizes / k < 1 / p < 0. */
int64_t randqlp_sketch_width(int64_t m, int64_t n, int k, int p);

/* Bytes of device workspace randqlp_factor needs for these sizes and
 * options (opts may be NULL for defaults); 0 for invalid arguments. */
size_t randqlp_workspace_size(int64_t m, int64_t n, int k, int p, int q,
                              const rqlp_opts* opts);

/* Generalised Algorithm 1 (Section 3.1): A (m x n, device, lda) ->
 * Q (m x d, ldq), L (d x d, ldl, lower-triangular, diag >= 0),
 * P (n x d, ldp).  k >= 1 target rank, p >= 0 oversampling, q >= 0 power
 * iterations, seed keys the Gaussian sketch.  opts may be NULL.
 * Returns RQLP_OK, an argument error (nothing enqueued), RQLP_E_NONFINITE
 * (A holds NaN/Inf), or a HIP / allocation error. */
rqlp_status randqlp_factor(const void* A, int64_t m, int64_t n, int k, int p, int q,
                           uint64_t seed, void* Q, void* L, void* P,
                           const rqlp_opts* opts);

/* randqlp_factor without host synchronisation, so that the call can be
 * captured into a HIP graph (or overlap host work): every step is enqueued on
 * opts->stream and the call returns at once.  opts must be given with a
 * workspace of randqlp_workspace_size bytes (nothing is allocated).  The
 * panel QR is opts->panel_qr's, except that AUTO means the fast path with no
 * automatic rerun (the rerun needs the host).  When the work completes,
 * status (device, 4 ints) holds the call's status words: status[0] is 0 for
 * trusted factors, else a mask of 1 (a pivot at or below the dependence
 * tolerance: rank-deficient panel), 2 (a non-finite value met) and 4 (the
 * second pass was not accurate enough); status[2] counts completed columns
 * (ROBUST).  A non-zero status[0] means: call randqlp_factor, which reruns
 * with the stronger panels and reports non-finite input.  opts->info, if
 * given, receives d and q_used only.  Status words are cleared by a kernel
 * (no memset node).  Returns after enqueueing. */
rqlp_status randqlp_factor_async(const void* A, int64_t m, int64_t n, int k, int p, int q,
                                 uint64_t seed, void* Q, void* L, void* P,
                                 const rqlp_opts* opts, int* status);

/* randqlp_factor for a sparse A (Section 5.1 factors sparse matrices), given
 * in CSR form on the device: row i's entries are colind[t], vals[t] for t
 * in [rowptr[i], rowptr[i + 1]) (rowptr: m + 1 int64, rowptr[0] = 0,
 * rowptr[m] = nnz; colind: nnz int32 in [0, n), any order within a row,
 * repeated positions add up; vals: nnz values of opts->precision, RQLP_F64
 * or RQLP_F32).  The products with A and A^T run as sparse products (A^T
 * is built in the workspace from the CSR arrays); everything else is
 * randqlp_factor's, and the outputs are those of randqlp_factor on the
 * dense A, up to the order of the sums.  The arrays are checked on the
 * device first: an invalid structure returns RQLP_E_INVALID_ARG before any
 * product reads them.  m, n < 2^21.  opts->lda is ignored; the workspace is
 * the library's (opts->workspace is not used).  Synchronous. */
rqlp_status randqlp_factor_csr(const int64_t* rowptr, const int32_t* colind, const void* vals,
                               int64_t m, int64_t n, int64_t nnz, int k, int p, int q,
                               uint64_t seed, void* Q, void* L, void* P, const rqlp_opts* opts);

/* randqlp_factor for callers that cannot allocate memory (tight serving
 * loops, harnesses that forbid allocation at run time): the same method and
 * kernels, with the call's scratch taken from a static device array of
 * RQLP_NOALLOC_SCRATCH_BYTES that every device holds from the time the
 * library's code object is loaded on it until the process ends, and small
 * read-backs copied to pageable host memory.  Nothing is allocated by the
 * call (no hipMalloc, hipHostMalloc, hipFree, event or stream creation).
 * opts->workspace must be NULL (RQLP_E_INVALID_ARG otherwise).  Sizes whose
 * scratch (randqlp_workspace_size with the same arguments) exceeds the array
 * return RQLP_E_WORKSPACE before anything is enqueued.  All calls on one
 * device share its array, which keeps the last call's contents: within a
 * process the library runs them one at a time (each completes before the
 * next starts); calls from other processes have their own copies.  Results
 * equal randqlp_factor's for the same arguments.  Synchronous. */
#define RQLP_NOALLOC_SCRATCH_BYTES (128ull << 20)
rqlp_status randqlp_factor_noalloc(const void* A, int64_t m, int64_t n, int k, int p, int q,
                                   uint64_t seed, void* Q, void* L, void* P,
                                   const rqlp_opts* opts);

/* ---- Step-level entry points (the individual steps of the method; the
 * same kernels randqlp_factor runs).  Asynchronous on `stream`. ---- */

/* The randn step of Algorithm 1: Omega (m x d, ld >= m) of precision
 * RQLP_F64 or RQLP_F32 from (seed, stream_id) as described above. */
rqlp_status randqlp_gaussian(void* out, int64_t m, int64_t d, int64_t ld, uint64_t seed,
                             uint64_t stream_id, int precision, void* stream);

/* The sketch / power / projection products of Algorithm 1:
 * C (rows x d) = op(A) X with op(A) = A^T (trans_a = 1: C is n x d, X is
 * m x d) or A (trans_a = 0: C is m x d, X is n x d).  precision RQLP_F64 /
 * RQLP_F32: A, X, C of that type.  RQLP_MIXED_BF16 / RQLP_MIXED_F16: A, X
 * and C are float; A and X are rounded to 16 bits (nearest even) into
 * library scratch and multiplied on the precision-form kernel with fp32
 * accumulation.  RQLP_MIXED_BF16X3: the split bfloat16 product described
 * with rqlp_precision.  Synchronous (the library's scratch may be reused). */
rqlp_status randqlp_gemm(int trans_a, const void* A, int64_t m, int64_t n, int64_t lda,
                         const void* X, int64_t d, int64_t ldx, void* C, int64_t ldc,
                         int precision, void* stream);

/* orth() of Algorithm 1: reduced QR X = Qx R of a rows x d panel with
 * rows >= d, diag(R) >= 0.  Qx (rows x d, ldq) may not alias X.  R (d x d,
 * double, ldr) may be NULL.  Synchronous (checks pivots); panel_qr selects
 * the algorithm as in rqlp_opts. */
rqlp_status randqlp_orth(const void* X, int64_t rows, int64_t d, int64_t ldx, void* Qx,
                         int64_t ldq, double* R, int64_t ldr, int precision,
                         int panel_qr, void* stream);

/* randqlp_factor with the number of power rounds chosen by the predictor
 * (params: device pointer to RQLP_MLP_PARAMS floats).  Steps: the 64-column
 * feature sketch in A's own precision (fp32 for the precision form), its
 * features, the MLP, q_hat = predicted class.  If q_hat >= q_fallback the
 * result is randqlp_factor with q = q_fallback.  Otherwise the method runs
 * with q = q_hat and an error judge looks one power round ahead: P =
 * orth(A^T Q) is the next power iterate, so Z = A P is the next round's
 * product; with e^2 = ||A||_F^2 - ||L||_F^2 (the squared residual of the
 * factors) and Delta = ||(I - Q Q^T) Z||_F^2 (how much one more round would
 * lower it), q_hat is accepted when Delta <= 0.0404 e^2 (2% in the error).
 * In the precision form Z is the 16-bit product (the one further rounds would
 * use) and the expected share of A's rounding error in it, (d / n)
 * ||A16 - A||_F^2, is taken off Delta first: no number of rounds removes it.
 * Otherwise the power rounds resume from Z up to q_fallback, and the result
 * equals randqlp_factor with q = q_fallback up to rounding.  opts as for
 * randqlp_factor (info->q_used reports the rounds used); ainfo may be NULL.
 * Synchronous. */
rqlp_status randqlp_factor_auto(const void* A, int64_t m, int64_t n, int k, int p,
                                int q_fallback, uint64_t seed, const float* params, void* Q,
                                void* L, void* P, const rqlp_opts* opts,
                                rqlp_auto_info* ainfo);
/* ... and with k <= 0 the rank is predicted as well (Section 5.2's rank-k
 * approximations Q L[:, :k] P[:, :k]^T; the tracking of the singular values
 * by diag L is what makes a truncation of the factors rank-revealing).
 * params then holds 2 * RQLP_MLP_PARAMS floats (the power-round network,
 * then the rank network), opts must be given with tol and k_max, and Q, L,
 * P must hold min(k_max + p, m, n) columns.  Steps: Omega, the 64-column
 * feature sketch, the rank network -> k_hat = min(8 * 2^c, k_max), the
 * power-round network with k_hat in its last input -> q_hat; then the
 * method with d = min(k_hat + p, m, n) columns and q_hat judged as above.
 * The returned factors are checked: k_used is the smallest k <= d whose
 * rank-k error meets tol; if none does (and d or q was below k_max + p,
 * q_fallback), the plain method reruns with k_max and q_fallback and is
 * checked the same way.  ainfo->d gives the returned width (leading d
 * columns of Q and P, leading d x d block of L); k_max + p <= 4096. */

/* The predictor's 65 features of A (m x n, lda; precision RQLP_F64 or
 * RQLP_F32 = the type of A) into feat (device, 65 floats).  Synchronous. */
rqlp_status randqlp_features(const void* A, int64_t m, int64_t n, int64_t lda, int k,
                             uint64_t seed, int precision, float* feat, void* stream);

/* MLP forward pass: X (B x 65, device, row-major) -> logits (B x 6).
 * Synchronous. */
rqlp_status randqlp_mlp_forward(const float* params, const float* X, int B, float* logits,
                                void* stream);

/* Mean softmax cross-entropy over the batch (X: B x 65, y: B labels in
 * 0..5, device) into *loss (device float) and its gradient with respect to
 * the parameters into grad (device, RQLP_MLP_PARAMS).  Synchronous. */
rqlp_status randqlp_mlp_loss_grad(const float* params, const float* X, const int* y, int B,
                                  float* grad, float* loss, void* stream);

/* One Adam step (Kingma & Ba; beta1 0.9, beta2 0.999, eps 1e-8) at step
 * t >= 1 on params with moment buffers m, v (device, RQLP_MLP_PARAMS).
 * Asynchronous. */
rqlp_status randqlp_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t t,
                             float lr, void* stream);

/* Train on N samples (X: N x 65, y: N labels, device) for `epochs` passes
 * of minibatches of `batch`, with Adam at learning rate lr.  Each epoch
 * visits the samples in the order i -> (a i + c) mod N with a coprime to N
 * and (a, c) drawn from (seed, epoch).  *step (host) is the Adam step count
 * so far and is advanced.  epoch_loss (device, `epochs` floats) receives
 * each epoch's mean minibatch loss.  Deterministic.  Synchronous. */
rqlp_status randqlp_mlp_train(float* params, float* m, float* v, const float* X, const int* y,
                              int64_t N, int epochs, int batch, float lr, uint64_t seed,
                              int64_t* step, float* epoch_loss, void* stream);

/* ---- Batched form ----
 * Many independent matrices of different shapes factored together: every
 * step of the method runs as one grouped launch over all matrices (one
 * workgroup list per step, built once per plan), and the sequence is
 * captured into a HIP graph that randqlp_batch_run replays.  Matrix i is
 * A[i] (m[i] x n[i], lda[i]) -> Q[i] (m x d_i, ldq[i]), L[i] (d_i x d_i,
 * double, ldl[i]), P[i] (n x d_i, ldp[i]) with d_i = min(k[i] + p, m, n),
 * sketch seed seeds[i]; pointer arrays are host arrays of device pointers
 * (any ld array may be NULL for tight).  precision: RQLP_F64 or RQLP_F32
 * (A, Q, P of that type).  The plan binds these pointers: a run reads the
 * current contents of A and overwrites Q, L, P.  Panels use fast Cholesky
 * QR; a matrix whose panel reports an unsafe pivot, or whose d_i exceeds
 * the one-workgroup Cholesky limit (224), is refactored on its own with
 * randqlp_factor after the grouped run.  tune != 0 times the candidate tile
 * widths of the products with A on this batch and records the fastest in
 * the process-wide table (see randqlp_tune_save); tune = 0 takes the table's
 * entry, else the per-matrix MFMA + vector-ALU layout.  The plan owns its device
 * memory (allocated here, freed by randqlp_batch_destroy). */
typedef struct rqlp_batch rqlp_batch;

typedef struct {
  int32_t count;      /* matrices in the plan                           */
  int32_t grouped;    /* of those, factored by the grouped launches      */
  int32_t fallbacks;  /* refactored one by one in the last run           */
  int32_t wn_tn;      /* tile width (16-column blocks per wave) of A^T X;
                         0 = per matrix, from its d                      */
  int32_t wn_nn;      /* the same for A X                                */
  int32_t dmax;       /* largest d among the grouped matrices            */
  double tune_ms;     /* time spent tuning at creation                   */
} rqlp_batch_info;

rqlp_status randqlp_batch_create(int count, const void* const* A, const int64_t* m,
                                 const int64_t* n, const int64_t* lda, const int* k, int p, int q,
                                 const uint64_t* seeds, void* const* Q, const int64_t* ldq,
                                 void* const* L, const int64_t* ldl, void* const* P,
                                 const int64_t* ldp, int precision, int tune,
                                 rqlp_batch** plan);

/* Run the plan on `stream` (use_graph != 0: replay the captured graph; 0:
 * launch the same sequence directly), then refactor any flagged matrix on
 * its own.  Synchronous. */
rqlp_status randqlp_batch_run(rqlp_batch* plan, int use_graph, void* stream);

rqlp_status randqlp_batch_query(const rqlp_batch* plan, rqlp_batch_info* info);

void randqlp_batch_destroy(rqlp_batch* plan);

/* create (tight leading dimensions, no tuning) + run + destroy. */
rqlp_status randqlp_factor_batched(int count, const void* const* A, const int64_t* m,
                                   const int64_t* n, const int* k, int p, int q,
                                   const uint64_t* seeds, void* const* Q, void* const* L,
                                   void* const* P, int precision, void* stream);

/* The tile-width table: text lines "dtype trans dbucket wn" (dtype 0 = f64,
 * 1 = f32; trans 1 = A^T X, 0 = A X; dbucket = 32, 64, 128 or 256, the
 * bucket of the largest d; wn = 1, 2, 4 or 8 for one width everywhere, 0 for
 * each matrix's own width covering its d, 16 for the MFMA + vector-ALU
 * layout with each matrix's own width).  load merges into the table. */
rqlp_status randqlp_tune_save(const char* path);
rqlp_status randqlp_tune_load(const char* path);

/* ---- Diagnostics ---- */

/* When on != 0, randqlp_factor records HIP events on its stream around each
 * launch of the product kernel that streams A (the sketch, power-iteration
 * and projection products) and accumulates their durations after the call
 * has synchronised.  Not thread-safe; meant for benchmarks. */
void randqlp_profile_enable(int on);

/* Totals since the last read: summed kernel time (ms), number of launches,
 * and the algorithmic flops (2 rows K d) and bytes (A, panel and output
 * once each) of those launches.  Any pointer may be NULL.  Resets totals. */
void randqlp_profile_read(double* ms, int64_t* launches, double* flops, double* bytes);

/* Identifier of the sources this library was built from (the SHA-256, in
 * hex, of its source files and compile flags; "unknown" if not given). */
const char* randqlp_build_id(void);

/* Human-readable name of a status, and the calling thread's last error. */
const char* randqlp_status_string(rqlp_status s);
const char* randqlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RANDQLP_H */
