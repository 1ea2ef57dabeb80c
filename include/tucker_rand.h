/*
 * tucker_rand.h -- C ABI of the MI355X (gfx950) randomized Tucker library.
 *
 * The library computes low multilinear rank approximations in Tucker format
 * (Problem 1 of Che, Wei, Yan, "Efficient algorithms for Tucker decomposition
 * via approximate matrix multiplication"): N orthonormal factors Q_n (I_n x mu_n)
 * and a core G (mu_1 x ... x mu_N) with A ~ G x_1 Q_1 ... x_N Q_N.
 *
 *   tucker_rand_thosvd   randomized T-HOSVD: Alg. 1 (exact power products) or
 *                        Alg. 4 (column-sampled approximate products).
 *   tucker_rand_sthosvd  randomized ST-HOSVD: Alg. 2 (exact) or Alg. 5 (sampled).
 *
 * Each step of the per-mode range finder is also exported on its own so that
 * it can be checked in isolation (Gaussian test matrix, column norms, sampler,
 * gather, power products, factor extraction, mode-n product).
 *
 * Conventions for every entry point:
 *  - Tensors are dense and column-major: index i_1 is fastest, so mode-1 fibers
 *    are contiguous (the unfolding order of Section 2).  A tensor's mode n is
 *    addressed through its 3-D view L x I x R with L = I_1...I_{n-1},
 *    I = I_n, R = I_{n+1}...I_N; element (l, i, r) sits at l + L*(i + I*r) and
 *    column j of the mode-n unfolding A_(n) is j = l + L*r (0-based).
 *  - Matrices are column-major with leading dimension equal to their row count.
 *  - "device" pointers are HIP device memory owned by the caller; the library
 *    never allocates or frees device memory.  Its only global state is the
 *    fixed scratch array of tucker_rand_sthosvd_noalloc and the per-device
 *    address of that array.  "host" pointers are read during the call only.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = default stream).
 *    Argument errors are detected on the host before anything is launched and
 *    returned synchronously; nothing is written in that case.  Numeric trouble
 *    found on the device (non-finite data, an all-zero sampling distribution)
 *    is reported through the optional device status word (TR_DEV_* bits).
 *  - Calls that share a workspace must not overlap in time.
 */
#ifndef TUCKER_RAND_H
#define TUCKER_RAND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TR_MAX_ORDER 8

/* Return codes. */
typedef enum {
  TR_OK = 0,
  TR_EINVAL = 1,   /* invalid argument (shape, rank, null pointer, ...)      */
  TR_ENOMEM = 2,   /* workspace smaller than tucker_rand_workspace_size()    */
  TR_EDEVICE = 3,  /* a HIP launch or runtime call failed                    */
  TR_ENOTSUP = 4,  /* valid request outside what this library implements    */
  TR_ENUMERIC = 5  /* reserved for numeric failures detected on the host    */
} tr_status;

/* Storage type of the input tensor, the factors and the core. */
typedef enum { TR_F64 = 0, TR_F32 = 1 } tr_dtype;

/* Probabilities of the sampled product (Remark after Alg. 3). */
typedef enum {
  TR_PROB_NONE = 0,            /* exact products: Alg. 1 / Alg. 2             */
  TR_PROB_NEARLY_OPTIMAL = 1,  /* p_j ~ ||A_(n)(:,j)||^2: Alg. 4 / Alg. 5      */
  TR_PROB_UNIFORM = 2          /* p_j = 1/J_n:             Alg. 4 / Alg. 5      */
} tr_prob;

/* Arithmetic of the power-scheme products C_n = (M D M^T)^q G_n, M = A_(n)
 * (Alg. 1 / 2) or the sampled C'_n (Alg. 4 / 5).
 *   TR_PREC_NATIVE: every product, norm and factor in float64 (float32
 *     inputs are widened exactly).
 *   TR_PREC_BF16 / TR_PREC_FP8E4M3: one fused pass over M per power step on
 *     the matrix cores.  M is rounded to bfloat16, or to FP8 e4m3 (OCP
 *     "e4m3fn", max 448) with one scale for a tensor and one per column for
 *     C'_n; C is rounded per step (per-column scale for e4m3); M^T C is
 *     formed in that format with float32 accumulation and D M^T C enters the
 *     second product as a bfloat16 pair (about 16 bits).  Block partial sums
 *     are added in float64.  For q > 1 (or with TR_FLAG_STABILIZED_POWER)
 *     the power scheme runs in its R-accumulated form (see the flag below):
 *     the iterate that is rounded is always orthonormal, and Rbar keeps
 *     C_n = Z_q Rbar equal to (M D M^T)^q G_n in exact arithmetic.  Only the
 *     caller's tensor (and columns sampled from it) is rounded: the modes of
 *     ST-HOSVD after the first are computed from the library's own float64
 *     shrunk tensor, whose energy sits in few columns (rounding them would
 *     rotate its range by the format's roundoff), with float64 products.
 *     Column norms, sampling probabilities, the QR / SVD
 *     of the sketch and the shrink stay float64.  Supported for I_n <= 512,
 *     s_n <= 48 and, for unsampled modes, J_n < 2^32 (else TR_ENOTSUP).
 *     The rounding of M adds about the format's unit roundoff (2^-9 or 2^-4
 *     relative) to each entry of the data the range finder sees. */
typedef enum { TR_PREC_NATIVE = 0, TR_PREC_BF16 = 1, TR_PREC_FP8E4M3 = 2 } tr_prec;

/* Device status bits (OR-ed into tr_diag.status). */
#define TR_DEV_NONFINITE 0x1u  /* a column norm or sketch entry was NaN/Inf   */
#define TR_DEV_ZERO_DIST 0x2u  /* every column norm was zero: nothing to draw */
#define TR_DEV_BAD_INDEX 0x4u  /* sparse input: a row index outside [0, I_1)
                                  (the entry was skipped)                     */

typedef struct tr_params {
  int32_t order;            /* N, 1 <= N <= TR_MAX_ORDER                          */
  const int64_t *dims;      /* host [N]: I_1..I_N, each >= 1                       */
  const int64_t *ranks;     /* host [N]: mu_n, 1 <= mu_n <= min(I_n, J_n) where J_n
                               is the column count of the unfolding that mode n is
                               computed from (original tensor for T-HOSVD, shrunk
                               tensor mu_1..mu_{n-1} I_{n+1}..I_N for ST-HOSVD)    */
  int32_t oversample;       /* K >= 0; sketch width s_n = min(mu_n + K, I_n) <= 128
                               (<= 64 with TR_FLAG_STABILIZED_POWER, TR_FLAG_RELATED_FORM
                               or a low precision; else TR_ENOTSUP)                */
  int32_t power;            /* q >= 1 power steps                                  */
  int32_t prob;             /* tr_prob                                             */
  const int64_t *samples;   /* host [N]: T_n >= 1 sampled columns (prob != NONE);
                               T_n > J_n computes that mode exactly.  May be NULL
                               when prob == TR_PROB_NONE.                          */
  uint64_t seed;            /* Philox4x64-10 key word 0                            */
  int32_t precision;        /* tr_prec                                             */
  uint32_t flags;           /* TR_FLAG_* bits; any other bit is TR_EINVAL          */
} tr_params;

/*
 * tr_params.flags.
 *   TR_FLAG_STABILIZED_POWER: the power scheme with an orthonormalisation
 *     after every step and the triangular factors accumulated (the QR form of
 *     the power iteration; equal to the plain products C_n = (M D M^T)^q G_n
 *     in exact arithmetic): Z_0 R_0 = G_n, Z_i R_i = M D M^T Z_{i-1}
 *     (i = 1..q), Rbar = R_q ... R_0, and Q_n = Z_q U'(:, 1:mu_n) for
 *     Rbar = U' S V'^T; the singular values reported are those of Rbar (those
 *     of C_n = Z_q Rbar).  Z_i is the orthonormal factor the factor kernel
 *     computes and R_i = Z_i^T (M D M^T Z_{i-1}).  The low-precision modes
 *     (TR_PREC_BF16 / TR_PREC_FP8E4M3) use this form whenever q > 1.
 *   TR_FLAG_UNFUSED_POWER: every exact power step as its two products
 *     (W = D M^T Y written to the workspace, then M W), as the Remark after
 *     Alg. 1 writes Strategy A, instead of the one-sweep kernel that keeps W
 *     on chip (where that kernel applies); same result up to rounding order.
 */
#define TR_FLAG_STABILIZED_POWER 0x1u
#define TR_FLAG_UNFUSED_POWER 0x2u
/*
 *   TR_FLAG_RELATED_FORM: the related forms of the subsection "Related forms
 *     for Algorithms 1 and 2" -- Alg. 6 (tucker_rand_thosvd) and Alg. 7
 *     (tucker_rand_sthosvd), and with sampling the same change to Alg. 4 / 5
 *     (the Remark closing that subsection): Q_n = P_n U_n where P_n is an
 *     orthonormal basis of range(C_n) and U_n the mu_n leading left singular
 *     vectors of P_n^T A_(n) (A_(n) the full unfolding of the mode's tensor).
 *     P_n is the s_n left singular vectors of C_n (with
 *     TR_FLAG_STABILIZED_POWER, Z_q); any orthonormal basis of range(C_n)
 *     gives the same Q_n in exact arithmetic.  U_n comes from the
 *     eigenvectors of P_n^T A_(n) A_(n)^T P_n, which one more exact power step
 *     over the mode's tensor forms.  Singular values reported: those of C_n.
 */
#define TR_FLAG_RELATED_FORM 0x4u

typedef struct tr_timer tr_timer;

/* Optional per-mode diagnostics, all device memory (except timer); any pointer
 * may be NULL. */
typedef struct tr_diag {
  int64_t *const *indices;  /* [N] -> T_n sampled column indices xi_t (0-based)   */
  double *const *scales;    /* [N] -> T_n rescale factors 1/sqrt(T_n p_xi)        */
  double *const *sketch;    /* [N] -> C_n, I_n x s_n float64                      */
  double *const *sigma;     /* [N] -> s_n singular values of C_n, descending      */
  uint32_t *status;         /* one word; TR_DEV_* bits are OR-ed in (caller zeroes) */
  tr_timer *timer;          /* host handle from tucker_rand_timer_create, or NULL */
  double *norms;            /* [3]: ||A||_F^2, ||G||_F^2 and the relative error
                               RE = ||A - G x_1 Q_1 ... x_N Q_N||_F / ||A||_F of
                               Eq. (8), as sqrt((||A||^2 - ||G||^2) / ||A||^2)
                               (exact for orthonormal factors), all float64 from
                               the float64 core.  ||A||^2 is the sum of mode 1's
                               column norms when nearly-optimal sampling takes
                               them, else one extra sweep over A.             */
} tr_diag;

/* Text for a tr_status value (static storage). */
const char *tucker_rand_status_string(int status);

/*
 * Bytes of device workspace needed by tucker_rand_thosvd (sthosvd == 0) or
 * tucker_rand_sthosvd (sthosvd != 0) for these parameters and input dtype.
 * Validates the parameters exactly as the decomposition calls do.
 */
int tucker_rand_workspace_size(const tr_params *p, int dtype, int sthosvd,
                               size_t *bytes);

/*
 * Randomized T-HOSVD (Section 3): for every mode n independently of the others
 * draw G_n (I_n x s_n Gaussian), form C_n = (A_(n) A_(n)^T)^q G_n (Alg. 1) or
 * C'_n = A_(n) S_n, S_n ~ RANDSAMPLE(T_n, p_n), C_n = (C'_n C'_n^T)^q G_n (Alg. 4),
 * take Q_n = the mu_n leading left singular vectors of C_n (Remark after Alg. 5),
 * then core = A x_1 Q_1^T ... x_N Q_N^T.
 *   A        device, column-major I_1 x ... x I_N, dtype; read only.
 *   Q        host array [N] of device pointers; Q[n] receives I_n x mu_n (dtype).
 *            Each column's largest-magnitude entry is positive.
 *   core     device, mu_1 x ... x mu_N (dtype).
 *   workspace, workspace_bytes: device scratch of at least the size reported by
 *            tucker_rand_workspace_size(p, dtype, 0, ...).
 *   diag     optional (may be NULL).
 */
int tucker_rand_thosvd(const tr_params *p, int dtype, const void *A,
                       void *const *Q, void *core, void *workspace,
                       size_t workspace_bytes, const tr_diag *diag, void *stream);

/*
 * Randomized ST-HOSVD (Section 4): modes in the order 1..N; after Q_n is found
 * the current tensor is replaced by its shrink A x_n Q_n^T (Alg. 2 / Alg. 5),
 * and the last shrink is the core.  Sampling probabilities of mode n refer to
 * the shrunk tensor.  Arguments as tucker_rand_thosvd (sthosvd workspace size).
 */
int tucker_rand_sthosvd(const tr_params *p, int dtype, const void *A,
                        void *const *Q, void *core, void *workspace,
                        size_t workspace_bytes, const tr_diag *diag, void *stream);

/*
 * Fixed-precision problem (Problem 2 of Section 7): multilinear ranks mu_n
 * and orthonormal Q_n with ||A - A x_1 Q_1 Q_1^T ... x_N Q_N Q_N^T||_F <= eps.
 * The paper poses it without an algorithm; the rule implemented: each mode is
 * computed by the related form (TR_FLAG_RELATED_FORM is implied), whose
 * P_n^T X_(n) gives the residual of every rank mu <= s_n exactly,
 * ||X||_F^2 - sum_{k <= mu} sigma_k(P_n^T X_(n))^2, and mu_n is the smallest
 * rank whose residual fits the mode's budget -- eps^2 / N per mode for
 * T-HOSVD (sthosvd == 0; Eq. (5)), the budget the earlier modes left split
 * evenly over the remaining ones for ST-HOSVD (Eq. (23)) -- capped at
 * p->ranks[n], at J_n and at s_n.
 *   p          p->ranks[n] are the largest ranks allowed; the sketch widths are
 *              s_n = min(p->ranks[n] + K, I_n) whatever ranks are chosen.
 *   tol        eps (relative == 0) or eps / ||A||_F (relative == 1), > 0.
 *   Q, core    as tucker_rand_thosvd / _sthosvd, sized for the largest ranks;
 *              Q[n] receives I_n x mu_n (its first mu_n columns), core the
 *              mu_1 x ... x mu_N tensor (its first prod mu_n entries).
 *   workspace  >= tucker_rand_workspace_size(p with TR_FLAG_RELATED_FORM set,
 *              dtype, sthosvd).
 *   ranks_out  host [N]: the chosen mu_n.
 *   bound_out  host: sqrt of the sum of the chosen residuals, which bounds
 *              ||A - A^||_F by Eq. (5) / Eq. (23); above eps when even the
 *              largest ranks do not reach the tolerance.
 * Unlike the other calls this one waits for the device: ||A||_F^2 and each
 * mode's s_n eigenvalues are read back (once per mode for ST-HOSVD, once for
 * all modes for T-HOSVD), because the later shapes depend on the ranks.  The
 * residuals are float64 differences with an absolute error of ~u ||A||_F^2,
 * so tolerances below ~1e-7 ||A||_F cannot be certified.
 */
int tucker_rand_adaptive(const tr_params *p, int dtype, int sthosvd, double tol,
                         int relative, const void *A, void *const *Q, void *core,
                         void *workspace, size_t workspace_bytes,
                         int64_t *ranks_out, double *bound_out,
                         const tr_diag *diag, void *stream);

/*
 * Batched randomized ST-HOSVD with sampled products (Alg. 5) for the serving
 * path: nreq independent requests of the same order N but different sizes,
 * ranks, sample counts and seeds advance through the modes together, and
 * every stage of a mode (column norms, weights and prefix sums, draws, gather,
 * power products, factorization, shrink) is one grouped launch over all of
 * them, driven by per-request descriptors the call writes to the start of the
 * workspace -- about eight launches per mode for the whole batch.  Each
 * request's arithmetic does not depend on the rest of the batch, so its
 * result is bitwise the same alone or in any batch (it is not bitwise the
 * same as tucker_rand_sthosvd, whose kernels sum in other orders).  A mode
 * whose T_n exceeds J_n takes every column once with weight 1 (the exact
 * product), as tucker_rand_sthosvd does.
 *   p          [nreq] host pointers to each request's parameters: the same
 *              order N, prob TR_PROB_NEARLY_OPTIMAL or TR_PROB_UNIFORM,
 *              precision native, flags 0.  Supported for I_n <= 512,
 *              s_n <= 48, mu_n <= 32, min(T_n, J_n) <= 8192 and
 *              J_n <= 2^20 per mode (else TR_ENOTSUP).
 *   dtype      storage type of every A, Q and core.
 *   A, Q, core host arrays [nreq] of device pointers (Q[r] is a host array [N]
 *              of device pointers), laid out as for tucker_rand_sthosvd.
 *   workspace  >= tucker_rand_batch_workspace_size(nreq, p, dtype, ...) bytes.
 *   status     device [nreq] (may be NULL): TR_DEV_* bits OR-ed into word r for
 *              request r (the caller zeroes them).
 * The call copies the descriptor table to the workspace synchronously with
 * respect to the host (after the stream's earlier work), then enqueues the
 * launches; a caller that overlaps batches gives each its own stream.
 */
int tucker_rand_batch_workspace_size(int nreq, const tr_params *const *p, int dtype,
                                     size_t *bytes);
int tucker_rand_sthosvd_batch(int nreq, const tr_params *const *p, int dtype,
                              const void *const *A, void *const *const *Q,
                              void *const *core, void *workspace,
                              size_t workspace_bytes, uint32_t *status,
                              void *stream);

/*
 * Randomized ST-HOSVD with sampled products (Alg. 5) of a sparse tensor (the
 * sparse examples of Sections 6.1 and 6.5): the mode-1 unfolding A_(1)
 * (I_1 x J_1, J_1 = I_2 ... I_N, column j = i_2 + I_2 (i_3 + I_3 (...)) as
 * in the dense layout) in compressed sparse columns.  Only the first mode
 * reads the sparse tensor -- its column norms, the gather of its sampled
 * columns and the shrink Q_1^T A_(1); the shrunk tensor is dense and the
 * later modes run as in tucker_rand_sthosvd.  The norms sum each column's
 * nonzeros in row order, so they, the draws, the gathered columns and Q_1
 * are those of tucker_rand_sthosvd on the dense tensor.
 *   p        as for tucker_rand_sthosvd; prob TR_PROB_NEARLY_OPTIMAL or
 *            TR_PROB_UNIFORM with T_1 <= J_1 (the first mode sampled),
 *            native precision, no flags (else TR_ENOTSUP).
 *   colptr   device int64 [J_1 + 1]: colptr[0] = 0, nondecreasing,
 *            colptr[J_1] = nnz.
 *   rowidx   device int32 [nnz]: rows in [0, I_1), increasing within each
 *            column (an index outside [0, I_1) is skipped and sets
 *            TR_DEV_BAD_INDEX; an unsorted column changes the rounding).
 *   vals     device [nnz] in dtype.
 *   workspace  >= tucker_rand_workspace_size(p, dtype, 1, ...) bytes.
 * Outputs, diagnostics and stream as for tucker_rand_sthosvd.
 */
int tucker_rand_sthosvd_csc(const tr_params *p, int dtype, int64_t nnz,
                            const int64_t *colptr, const int32_t *rowidx,
                            const void *vals, void *const *Q, void *core,
                            void *workspace, size_t workspace_bytes,
                            const tr_diag *diag, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): randomized
 * ST-HOSVD exactly as tucker_rand_sthosvd (same kernels, same results), with
 * the workspace taken from a fixed device array of TR_NOALLOC_SCRATCH_BYTES
 * inside the library instead of a caller buffer.  Nothing is allocated or
 * freed during the call.
 *   - Each GPU that runs it holds its own copy of the array until the process
 *     ends; the first call on a device looks up its address (with that device
 *     current).  `stream` must belong to the current device (TR_EINVAL).
 *   - Problems whose workspace (tucker_rand_workspace_size(p, dtype, 1, ...))
 *     exceeds TR_NOALLOC_SCRATCH_BYTES return TR_ENOMEM before anything runs.
 *   - Every call on one GPU shares that GPU's array: calls that overlap in time
 *     on one GPU (different streams, threads) race and give wrong results.
 *     Nothing in the array needs to start at zero; its contents after a call
 *     are unspecified.
 * A, Q, core, diag: as tucker_rand_sthosvd (caller-allocated).
 */
#define TR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int tucker_rand_sthosvd_noalloc(const tr_params *p, int dtype, const void *A,
                                void *const *Q, void *core,
                                const tr_diag *diag, void *stream);

/* ---------------------------------------------------------------------------
 * Individual steps of the per-mode range finder.
 * ------------------------------------------------------------------------- */

/*
 * Standard Gaussian matrix G_n (Alg. 1 step 2; Alg. 4 step 5): G device float64
 * I x s column-major.  Element e = i + I*c takes the Philox4x64-10 block with
 * counter (e/4, mode, 0, 0) and key (seed, 0); output words (0,1) and (2,3) are
 * Box-Muller pairs.
 */
int tucker_rand_gaussian(int64_t I, int64_t s, int32_t mode, uint64_t seed,
                         double *G, void *stream);

/*
 * Squared column norms n_j = ||A_(n)(:,j)||^2 of the mode-n unfolding of the
 * L x I x R view of X (device, dtype), summed in float64 over rows in
 * increasing order (Remark after Alg. 3, nearly-optimal probabilities).
 * norms: device float64 [L*R].  max_bits (device uint64, may be NULL): receives
 * the atomic maximum of the IEEE bit patterns of the norms; the caller sets it
 * to 0 beforehand.
 */
int tucker_rand_colnorms(int dtype, const void *X, int64_t L, int64_t I,
                         int64_t R, double *norms, uint64_t *max_bits,
                         void *stream);

/* Device workspace bytes needed by tucker_rand_sample for J columns. */
size_t tucker_rand_sample_workspace_size(int64_t J);

/*
 * RANDSAMPLE(T, p) of Section 3.2 as index/scale pairs: S[idx[t], t] = scale[t].
 * prob = TR_PROB_NEARLY_OPTIMAL: norms (device float64 [J], finite, not all 0)
 *   are quantised to integer weights w_j = floor((n_j / max n) * 2^(60 -
 *   ceil(log2 J))), raised to 1 for every non-zero column;
 * prob = TR_PROB_UNIFORM: w_j = 1 and norms may be NULL.
 * Draw t uses the Philox4x64-10 block with counter (t/2, mode, 1, 0), key
 * (seed, 0), words (2(t%2), 2(t%2)+1) = (h, l): x = floor((h 2^64 + l) W / 2^128),
 * idx[t] = min{ j : w_0 + ... + w_j > x }, scale[t] = sqrt((W / w_idx) / T)
 * with W = sum w.  idx: device int64 [T]; scale: device float64 [T].
 * workspace: device, >= tucker_rand_sample_workspace_size(J) bytes.
 * status (device, may be NULL) receives TR_DEV_* bits.
 */
int tucker_rand_sample(const double *norms, int64_t J, int64_t T, int prob,
                       uint64_t seed, int32_t mode, int64_t *idx, double *scale,
                       void *workspace, size_t workspace_bytes,
                       uint32_t *status, void *stream);

/*
 * Gather of the sampled product C'_n = A_(n) S_n without its rescale
 * (Alg. 4 step 4): Cp[:, t] = A_(n)(:, idx[t]) for the L x I x R view of X.
 * Cp: device I x T, same dtype as X.  idx: device int64 [T], each < L*R.
 */
int tucker_rand_gather(int dtype, const void *X, int64_t L, int64_t I,
                       int64_t R, const int64_t *idx, int64_t T, void *Cp,
                       void *stream);

/* Device workspace bytes needed by tucker_rand_power for these sizes
 * (0 for invalid sizes). */
size_t tucker_rand_power_workspace_size(int dtype, int64_t L, int64_t I,
                                        int64_t R, int64_t s);

/*
 * Power-scheme products (Alg. 1 step 4 by Strategy A of the Remark after
 * Alg. 1; Alg. 4 step 6): C = (M D M^T)^q G where M is the mode-n unfolding of
 * the L x I x R view of X (device, dtype) and D = diag(colweight) (device
 * float64 [L*R], or NULL for the identity).  With X a gathered I x T matrix
 * (L = 1, R = T) and colweight = scale^2 this is (C'_n C'_n^T)^q G_n.
 * G, C: device float64 I x s (may alias), s <= 128.  Float64 accumulation.
 */
int tucker_rand_power(int dtype, const void *X, int64_t L, int64_t I,
                      int64_t R, const double *colweight, int32_t q,
                      const double *G, int64_t s, double *C, void *workspace,
                      size_t workspace_bytes, void *stream);

/* Device workspace bytes needed by tucker_rand_factor (0 when the working
 * matrices fit in the workgroup's LDS). */
size_t tucker_rand_factor_workspace_size(int64_t I, int64_t s, int64_t mu);

/*
 * Factor of a sketch (Remark after Alg. 5): Q = the mu leading left singular
 * vectors of C (device float64 I x s, 1 <= mu <= s <= I, s <= 128), each
 * column's largest-magnitude entry made positive (lowest row on ties).
 * Computed on one workgroup in float64: Householder QR C = Q1 R1, a QR of
 * R1^T = Q2 R2, one-sided Jacobi on the columns of R2^T (whose rotated,
 * normalised columns are the left singular vectors U of R1), and
 * Q = Q1 U(:, 1:mu).  For s > 64 the second QR is skipped (the Jacobi runs
 * on the columns of R1) and the workspace holds the s x s matrices too.  Q: device float64 I x mu; sigma: device float64 [s]
 * singular values in descending order (may be NULL).
 */
int tucker_rand_factor(const double *C, int64_t I, int64_t s, int64_t mu,
                       double *Q, double *sigma, void *workspace,
                       size_t workspace_bytes, void *stream);

/* Device workspace bytes needed by tucker_rand_ttm (0 for invalid sizes). */
size_t tucker_rand_ttm_workspace_size(int64_t L, int64_t I, int64_t R,
                                      int64_t mu);

/*
 * Mode-n product Y = X x_n Q^T (Section 2): for the L x I x R view of X
 * (device, in_dtype) and Q (device float64 I x mu, mu <= 128), Y is
 * L x mu x R (device, out_dtype) with Y(l, k, r) = sum_i Q(i, k) X(l, i, r),
 * float64 accumulation.  This is the ST-HOSVD shrink (Alg. 2 step 6) and each
 * link of the T-HOSVD core chain.  workspace: device scratch of
 * tucker_rand_ttm_workspace_size bytes (Q^T rows and a float64 result).
 */
int tucker_rand_ttm(int in_dtype, const void *X, int64_t L, int64_t I,
                    int64_t R, const double *Q, int64_t mu, int out_dtype,
                    void *Y, void *workspace, size_t workspace_bytes,
                    void *stream);

/* ---------------------------------------------------------------------------
 * Kernel timing (benchmarking aid).  A timer owns a pool of HIP events; when it
 * is passed in tr_diag.timer, the decomposition calls record an event pair on the launch
 * stream around every kernel of the selected classes.  Read it after
 * synchronising the stream.
 * ------------------------------------------------------------------------- */
typedef enum {
  TR_KC_COLNORMS = 0, TR_KC_SAMPLE = 1, TR_KC_GATHER = 2, TR_KC_POWER = 3,
  TR_KC_FACTOR = 4, TR_KC_TTM = 5, TR_KC_GAUSSIAN = 6, TR_KC_COUNT = 7
} tr_kernel_class;

/* capacity: maximum number of timed launches; class_mask: bit c times class c. */
int tucker_rand_timer_create(int capacity, uint32_t class_mask, tr_timer **out);
int tucker_rand_timer_destroy(tr_timer *t);
/* Clears recorded launches. */
int tucker_rand_timer_reset(tr_timer *t);
/* Sum of elapsed milliseconds and number of launches recorded for a class, and
 * for the first-mode launch of that class only (mode-1 sweeps of the full
 * tensor); synchronises on the recorded events. */
int tucker_rand_timer_read(tr_timer *t, int kernel_class, double *total_ms,
                           int64_t *launches, double *mode0_ms,
                           int64_t *mode0_launches);

#ifdef __cplusplus
}
#endif
#endif /* TUCKER_RAND_H */
