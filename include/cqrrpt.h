/*
 * cqrrpt.h -- C ABI of the MI355X (gfx950) CQRRPT library.
 *
 * CQRRPT is the randomized, pivoted CholeskyQR for tall matrices of
 * Melnichenko, Balabanov, Murray, Demmel, Mahoney and Luszczek,
 * arXiv:2311.08316 ("CholeskyQR with Randomization and Pivoting for Tall
 * Matrices"). Given an m x n matrix A (m >= n) it returns a column pivot
 * order J, an m x k matrix Q with orthonormal columns, a k x n upper
 * trapezoidal R and the numerical rank k such that A[:, J] = Q R
 * (Algorithm 1 with the core of Algorithm 2; Theorem "correctness", Sec. 2.1).
 *
 * Conventions shared by every entry point
 *   - Matrices are FP64, column-major: element (i, j) of X is X[i + j*ldx].
 *   - Every array argument is a DEVICE pointer (hipMalloc / PyTorch tensor
 *     storage) unless the comment says "host". The caller owns all inputs and
 *     outputs; the library never allocates or frees them and never writes to A.
 *   - Indices (J) are 0-based int64.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Entry points taking a stream are stream-ordered and return before the
 *     GPU work finishes; entry points without one are synchronous.
 *   - Return value: 0 on success; -i when argument i (1-based, in the order of
 *     the prototype) is invalid, LAPACK INFO style, and nothing is launched;
 *     a positive CQRRPT_E* code for runtime failures (see below).
 *   - Calls on different streams with disjoint buffers may run concurrently.
 *     Results are deterministic: identical inputs give bit-identical outputs
 *     on the same GPU (no floating-point atomics; fixed reduction orders).
 */
#ifndef CQRRPT_H
#define CQRRPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Positive status codes. */
#define CQRRPT_OK            0
#define CQRRPT_ENONFINITE    1  /* A holds a NaN/Inf (seen as a non-finite sketch); rank = 0 */
#define CQRRPT_EBUDGET       2  /* request exceeds the server's device-memory budget        */
#define CQRRPT_EHIP          3  /* a HIP runtime call failed                                 */
#define CQRRPT_EWORKSPACE    4  /* workspace smaller than cqrrpt_workspace_bytes()           */
#define CQRRPT_EBARRIER      5  /* a persistent kernel's grid barrier timed out              */
#define CQRRPT_ELIMIT        6  /* size beyond what the library supports (see limits below) */

/* Precision modes (Sec. 3, Theorem "simple stability": the preconditioning
 * solve may run at a larger unit roundoff than the other steps).
 *   CQRRPT_FP64         : every step in FP64.
 *   CQRRPT_MIXED        : the preconditioning solve M_pre = A[:,J] R_sk^{-1}
 *                         runs on FP32 matrix cores and stores M_pre in FP32;
 *                         the Gram, the Q solve, the sketch QRCP, Cholesky and
 *                         R = R_pre R_sk stay FP64; one CholeskyQR pass, as
 *                         the theorem analyses.
 *   CQRRPT_MIXED_CHECKED: CQRRPT_MIXED, then G2 = Q^T Q (FP64) and an estimate
 *                         of ||Q^T Q - I||_2 (power iteration on G2 - I); when
 *                         it exceeds 5e-13, half the 1e-12 orthogonality
 *                         target, and G2 has a full Cholesky factor, one more
 *                         CholeskyQR pass (Sec. 1.2, "CholeskyQR2": R2 =
 *                         chol(G2), Q <- Q R2^{-1}, R <- R2 R) runs; the
 *                         decision is taken on the device.
 * In both mixed modes the second-stage rank bound on the diagonal of R_pre
 * is 1e6 instead of 10: the Sec. 3.3 bound sqrt(eps_tol/u) with u = 2^-53
 * (the CholeskyQR lines run in FP64) and eps_tol = 1e-4, the first-pass
 * orthogonality loss that the CholeskyQR2 re-pass still repairs. The FP32
 * solve alone spreads diag(R_pre) to about u_fp32 cond(R_sk), which the
 * FP64 bound 10 would cut. Hence CQRRPT_MIXED guarantees only
 * ||Q^T Q - I||_2 <~ 1e-4 in the worst case; CQRRPT_MIXED_CHECKED guarantees
 * the FP64 orthogonality bar. */
typedef enum {
  CQRRPT_FP64 = 0,
  CQRRPT_MIXED = 1,
  CQRRPT_MIXED_CHECKED = 2,
  /* FP32 lines + CholeskyQR2: the preconditioning solve, the Gram and the Q
   * product on FP32 matrix cores with FP32 accumulation (M_pre stored in
   * FP32), then one FP64 CholeskyQR pass on Q (always run: G2 = Q^T Q,
   * R2 = chol(G2), Q <- Q R2^{-1}, R <- R2 R). The sketch, its QRCP, the
   * Cholesky factorizations and R = R_pre R_sk stay FP64. The first pass's
   * orthogonality is FP32-level, so its second-stage bound is
   * sqrt(0.5 / 2^-24) = 2896 (the loss the FP64 pass still repairs). */
  CQRRPT_MIXED_FP32_CHOLQR2 = 3
} cqrrpt_mode_t;

/* Per-call diagnostics, written to DEVICE memory by cqrrpt_factor_ex and
 * copied to the host by cqrrpt_factor. */
typedef struct {
    int64_t rank;            /* k: final numerical rank (Sec. 3.3, second stage)          */
    int64_t rank_stage1;     /* k_o: first-stage bound (Sec. 3.3, first stage)             */
    int64_t chol_fail_col;   /* 0-based column where Cholesky stopped, -1 if it did not
                                (Remark on Cholesky failure, Sec. 3.3)                      */
    int32_t status;          /* CQRRPT_OK, CQRRPT_ENONFINITE or CQRRPT_EBARRIER             */
    int32_t cholqr2_passes;  /* extra CholeskyQR passes run (checked mixed mode), 0 or 1    */
    double  smax;            /* max |R_sk|, the scale of the first-stage test               */
    double  orth_est;        /* checked mixed mode: estimate of ||Q^T Q - I||_2 for the Q
                                of the first pass (16 power-iteration steps on G2 - I,
                                G2 = Q^T Q in FP64); 0 when no estimate was formed         */
} cqrrpt_info_t;

/* Limits of the library: n <= 8192, d <= 16384, 1 <= nnz <= 32. */

/* ------------------------------------------------------------------------
 * Sketching operator (Sec. 2.3.1, SASO)
 * ------------------------------------------------------------------------
 * Writes the d x m sparse sign operator S with exactly nnz nonzeros per
 * column: for source row j (column j of S) and t < nnz,
 *   rows[j*nnz + t]  = the row of S holding the t-th nonzero (distinct per j),
 *   signs[j*nnz + t] = +1 or -1; the value is signs/sqrt(nnz).
 * Rows are drawn by Floyd's subset sampler from exact uniform integers
 * (Lemire's multiply-shift with rejection) fed by Philox4x32-10 keyed by
 * `seed`, one counter stream per j; the sign bits are the stream's first
 * word. The operator therefore depends only on (seed, d, nnz, j) and is
 * bit-identical to any implementation of the same definition.
 * rows: int32[m*nnz], signs: int8[m*nnz], both device, caller-owned.
 * Errors: -1 m < 1, -2 d < 1, -3 nnz outside [1, min(32, d)], -5/-6 NULL. */
int cqrrpt_saso_sample(int64_t m, int64_t d, int32_t nnz, uint64_t seed,
                       int32_t* rows, int8_t* signs, void* stream);

/* ------------------------------------------------------------------------
 * Sketch Ahat = S A (Algorithm 2, first step)
 * ------------------------------------------------------------------------
 * A: m x n (lda >= m). Ahat: d x n (ldah >= d). S as in cqrrpt_saso_sample.
 * ws: device workspace of at least cqrrpt_sketch_workspace_bytes(m,n,d,nnz)
 * bytes. Each entry of Ahat is 1/sqrt(nnz) times a signed sum of entries of
 * A, accumulated in a fixed order (deterministic).
 * Returns CQRRPT_ENONFINITE (after the work completes on `stream`, i.e. the
 * check is synchronous) is NOT reported here; use cqrrpt_factor_ex's info.
 * Errors: -1..-8 bad sizes/pointers, CQRRPT_EWORKSPACE. */
size_t cqrrpt_sketch_workspace_bytes(int64_t m, int64_t n, int64_t d, int32_t nnz);
int cqrrpt_sketch(const double* A, int64_t lda, int64_t m, int64_t n,
                  int64_t d, int32_t nnz, uint64_t seed,
                  double* Ahat, int64_t ldah,
                  void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * QR with column pivoting of a short-wide-ish d x n matrix (Algorithm 2,
 * second step; Householder QR with max-norm pivoting as in LAPACK GEQP3)
 * ------------------------------------------------------------------------
 * X: d x n (ldx >= d, d >= n), OVERWRITTEN (it is the working array).
 * J: int64[n], the 0-based pivot order, always full length.
 * R: n x n (ldr >= n), upper triangular with non-negative diagonal; entries
 *    below the diagonal are written as zero.
 * Column norms are recomputed exactly at every step; ties go to the smallest
 * original column index. Runs as one cooperative (grid-synchronised) launch.
 * ws: at least cqrrpt_qrcp_workspace_bytes(d, n) bytes.
 * Errors: bad sizes/pointers (negative), CQRRPT_EWORKSPACE, CQRRPT_EHIP. */
size_t cqrrpt_qrcp_workspace_bytes(int64_t d, int64_t n);
int cqrrpt_qrcp(double* X, int64_t ldx, int64_t d, int64_t n,
                int64_t* J, double* R, int64_t ldr,
                void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * The whole factorization (Algorithm 1 with Algorithm 2's core)
 * ------------------------------------------------------------------------
 * A:    m x n input (lda >= m), read only.
 * d:    sketch rows, n <= d <= m (Algorithm 2's input condition); the paper's
 *       default is d = ceil(1.25 n) (Algorithm 1).
 * nnz:  nonzeros per column of the SASO, 1 <= nnz <= min(32, d).
 * seed: selects the sketching operator (see cqrrpt_saso_sample).
 * tol:  first-stage rank tolerance (takes the place of the unit roundoff u
 *       in the first-stage bound of Sec. 3.3), finite and >= 0; 1e-14 is a
 *       good default in FP64. The second stage keeps the largest leading
 *       block whose diagonal condition estimate is <= sqrt(100) = 10.
 * Q:    m x n output (ldq >= m): Q[:, :rank] orthonormal, Q[:, rank:] = 0.
 *       In the FP64 mode Q also holds M_pre until the Q step overwrites it;
 *       an ldq whose 8 ldq bytes are a multiple of 4 KiB (for example a
 *       power of two) puts the rows the Gram reads together on colliding
 *       cache sets and channels and takes the slower LDS-staged Gram
 *       (365 against 299 ms at 4194304 x 2048): prefer ldq = m + 16 there.
 * R:    n x n output (ldr >= n): R[:rank, :] upper trapezoidal with a
 *       non-negative diagonal, R[rank:, :] = 0.
 * J:    int64[n] output, 0-based pivots, always the full permutation.
 * rank: HOST pointer receiving k.
 * Synchronous, on the null stream. Its workspace is kept by the library per
 * device between calls: the first call on a device, and a call that needs
 * more than any earlier one, allocates it (growing, never shrinking; held
 * until the process ends); other calls allocate nothing. Calls from several
 * threads on one device are serialised. A rank of 0 (A = 0) is a valid result. A Cholesky failure is not an error: it truncates the
 * rank. Returns CQRRPT_ENONFINITE when A holds a NaN or Inf. */
int cqrrpt_factor(const double* A, int64_t lda, int64_t m, int64_t n,
                  int64_t d, int32_t nnz, uint64_t seed, double tol,
                  double* Q, int64_t ldq, double* R, int64_t ldr,
                  int64_t* J, int64_t* rank);

/* Workspace for cqrrpt_factor_ex, in bytes (256-byte aligned base needed). */
size_t cqrrpt_workspace_bytes(int64_t m, int64_t n, int64_t d, int32_t nnz,
                              cqrrpt_mode_t mode);

/* Stream-ordered form of cqrrpt_factor: no host synchronisation, no
 * allocation. ws: caller-owned device workspace of at least
 * cqrrpt_workspace_bytes() bytes (contents on entry are ignored).
 * info: DEVICE pointer to one cqrrpt_info_t (required; holds the rank).
 * Argument order: A lda m n d nnz seed tol Q ldq R ldr J mode ws ws_bytes
 * stream info. */
int cqrrpt_factor_ex(const double* A, int64_t lda, int64_t m, int64_t n,
                     int64_t d, int32_t nnz, uint64_t seed, double tol,
                     double* Q, int64_t ldq, double* R, int64_t ldr,
                     int64_t* J, cqrrpt_mode_t mode,
                     void* ws, size_t ws_bytes, void* stream,
                     cqrrpt_info_t* info);

/* Implicit Q (Sec. 2.1, arithmetic complexity paragraph): Q is returned as
 * the composition of M_pre and R_pre^{-1}, which skips the Q solve (the
 * leading cost drops from 3mn^2 to 2mn^2; stability is unchanged).
 * Same pipeline and workspace as cqrrpt_factor_ex in CQRRPT_FP64 mode
 * (ws_bytes >= cqrrpt_workspace_bytes(m, n, d, nnz, CQRRPT_FP64)), with
 * k = info->rank:
 * M:    m x n output (ldm >= m): M[:, :k] = M_pre[:, :k] = A[:, J[:k]] R_sk[:k,:k]^{-1},
 *       M[:, k:] = 0.
 * Rpre: n x n output (ldrp >= n): Rpre[:k, :k] = R_pre[:k, :k], upper
 *       triangular with a positive diagonal; zero elsewhere. The explicit
 *       factor is Q[:, :k] = M[:, :k] Rpre[:k, :k]^{-1}.
 * R, J, info: as in cqrrpt_factor_ex (R = R_pre[:k,:k] R_sk[:k, :]).
 * All pointers are device pointers owned by the caller; stream-ordered, no
 * allocation, no host synchronisation.
 * Argument order: A lda m n d nnz seed tol M ldm Rpre ldrp R ldr J ws
 * ws_bytes stream info.
 * Errors (nothing is launched): -1..-8 as cqrrpt_factor_ex, -9 M NULL,
 * -10 ldm < m, -11 Rpre NULL, -12 ldrp < n, -13 R NULL, -14 ldr < n,
 * -15 J NULL, -16 ws NULL, -19 info NULL, CQRRPT_ELIMIT, CQRRPT_EWORKSPACE. */
int cqrrpt_factor_implicit_ex(const double* A, int64_t lda, int64_t m, int64_t n,
                              int64_t d, int32_t nnz, uint64_t seed, double tol,
                              double* M, int64_t ldm, double* Rpre, int64_t ldrp,
                              double* R, int64_t ldr, int64_t* J,
                              void* ws, size_t ws_bytes, void* stream,
                              cqrrpt_info_t* info);

/* The unpivoted precursor of CQRRPT (Sec. 1.3, "Randomized preconditioning
 * for CholeskyQR"): sketch Ahat = S A with the SASO above, unpivoted
 * Householder QR Ahat = Q_sk R_sk, M_pre = A R_sk^{-1}, R_pre = chol(M_pre^T
 * M_pre), Q = M_pre R_pre^{-1}, R = R_pre R_sk. FP64. Like plain
 * CholeskyQR it needs A of full rank: there is no pivoting and no rank
 * detection; a Cholesky failure (A numerically rank deficient) truncates the
 * result at the failing column, reported in info->chol_fail_col and
 * info->rank (Q and R zero past it); an exactly zero trailing block of R_sk
 * is dropped the same way.
 * Arguments as cqrrpt_factor_ex without tol, J and mode (workspace:
 * cqrrpt_workspace_bytes(m, n, d, nnz, CQRRPT_FP64)). Argument order:
 * A lda m n d nnz seed Q ldq R ldr ws ws_bytes stream info.
 * Errors (nothing is launched): -1..-6 as cqrrpt_factor_ex, -8 Q NULL,
 * -9 ldq < m, -10 R NULL, -11 ldr < n, -12 ws NULL, -15 info NULL,
 * CQRRPT_ELIMIT, CQRRPT_EWORKSPACE. */
int cqrrpt_sketched_cholqr_ex(const double* A, int64_t lda, int64_t m, int64_t n,
                              int64_t d, int32_t nnz, uint64_t seed,
                              double* Q, int64_t ldq, double* R, int64_t ldr,
                              void* ws, size_t ws_bytes, void* stream,
                              cqrrpt_info_t* info);

/* CQRRPT with a dense sketching operator instead of the SASO (Sec. 2.3.1):
 *   CQRRPT_SKETCH_GAUSSIAN: iid N(0, 1/d) entries; entries (2q, j) and
 *     (2q+1, j) from one Philox4x32-10 block at counter (lo32(j), hi32(j), q,
 *     "GAUS") by Box-Muller (u1 = (U(w0,w1) + 1) 2^-53, u2 = U(w2,w3) 2^-53,
 *     U = top 27 bits of the first word and top 26 of the second; cosine for
 *     the even row, sine for the odd).
 *   CQRRPT_SKETCH_SRHT: S = sqrt(m/d) Pi[:d,:] H D, H the orthonormal
 *     Sylvester-Hadamard matrix of order m' = 2^ceil(log2 m) (zero padding),
 *     D the signs of bit 0 of word 0 at counter (lo32(j), hi32(j), 0, "SRHD"),
 *     Pi[:d,:] the d rows Floyd's sampler draws from [0, m') with exact
 *     uniform integers from the word stream at counters (lo32(w/4),
 *     hi32(w/4), 0, "SRHR"), key (lo32(seed), hi32(seed)) throughout.
 * S is formed explicitly (S^T in ws, m x d FP64) and Ahat = S A is one product
 * on the FP64 matrix cores: 2 d m n flops, against the SASO's m n nnz adds.
 * The SRHT is applied in this dense form, not by a fast transform. The rows
 * of the SRHT are drawn on the host and copied in, so this call synchronises
 * the stream once. The rest is cqrrpt_factor_ex in CQRRPT_FP64 mode.
 * ws: cqrrpt_dense_workspace_bytes(m, n, d) bytes (0: sizes out of range).
 * Argument order: A lda m n d kind seed tol Q ldq R ldr J ws ws_bytes stream
 * info. Errors: -1..-5, -8 as cqrrpt_factor_ex, -6 unknown kind, -9 Q NULL,
 * -10 ldq < m, -11 R NULL, -12 ldr < n, -13 J NULL, -14 ws NULL,
 * -17 info NULL, CQRRPT_ELIMIT, CQRRPT_EWORKSPACE, CQRRPT_EHIP. */
#define CQRRPT_SKETCH_GAUSSIAN 1
#define CQRRPT_SKETCH_SRHT     2
size_t cqrrpt_dense_workspace_bytes(int64_t m, int64_t n, int64_t d);
int cqrrpt_factor_dense_ex(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d,
                           int32_t kind, uint64_t seed, double tol,
                           double* Q, int64_t ldq, double* R, int64_t ldr, int64_t* J,
                           void* ws, size_t ws_bytes, void* stream, cqrrpt_info_t* info);

/* HQRRP on the sketch (Sec. 5.2.2): Householder QR with randomized block
 * pivoting of a d x n matrix X, the substitute the paper tries for GEQP3 on
 * the sketch, following the randomized QRCP loop it outlines in Sec. 1.
 * A Gaussian Omega (p = block + oversample rows; entries (2q, j) and
 * (2q + 1, j) by Box-Muller from one Philox4x32-10 block at counter
 * (lo32(j), hi32(j), q, "HQRP") under key (lo32(seed), hi32(seed)), scaled
 * by 1/sqrt(p)) gives the sample Y = Omega X; then per block of
 * bb = min(block, n - i) columns at position i:
 *   1. the first bb pivots of max-norm QRCP of Y's remaining columns (exact
 *      norms, ties to the smallest original column index); the chosen
 *      columns take positions i.. in pivot order, the others keep their
 *      relative order;
 *   2. unpivoted Householder QR of the chosen columns (LAPACK sign
 *      convention), applied to the remaining columns (compact WY form);
 *   3. the sample update Y2 <- Y2 - Y1 Z with R11 Z = R12 (a zero diagonal
 *      entry of R11 gives a zero row of Z).
 * Outputs as cqrrpt_qrcp: J (device int64[n]) the 0-based pivot order, R
 * (n x n, ldr >= n) upper triangular with rows negated to a non-negative
 * diagonal, X[:, J] = Q R. X is overwritten (Householder vectors).
 * Limits: 1 <= block <= 16, oversample >= 0, block + oversample <= 24,
 * n <= 2048, n <= d <= 3072 (else CQRRPT_ELIMIT). ws: device workspace of
 * cqrrpt_hqrrp_workspace_bytes() bytes (0: out of range); info: DEVICE
 * pointer to one cqrrpt_info_t, reset here; a non-finite X raises its status
 * to CQRRPT_ENONFINITE and the rest is skipped. Stream-ordered.
 * Argument order: X ldx d n block oversample seed J R ldr ws ws_bytes
 * stream info. Errors: -1 X NULL, -2 ldx < d, -3 d < 1, -4 n < 1 or n > d,
 * -5 block < 1, -6 oversample < 0, -8 J NULL, -9 R NULL, -10 ldr < n,
 * -11 ws NULL, -14 info NULL, CQRRPT_ELIMIT, CQRRPT_EWORKSPACE,
 * CQRRPT_EHIP. */
size_t cqrrpt_hqrrp_workspace_bytes(int64_t d, int64_t n, int32_t block, int32_t oversample);
int cqrrpt_hqrrp(double* X, int64_t ldx, int64_t d, int64_t n, int32_t block,
                 int32_t oversample, uint64_t seed, int64_t* J, double* R, int64_t ldr,
                 void* ws, size_t ws_bytes, void* stream, cqrrpt_info_t* info);

/* CQRRPT whose QRCP of the sketch is cqrrpt_hqrrp (Sec. 5.2.2) with
 * (block, oversample, hseed); everything else as cqrrpt_factor_ex in
 * CQRRPT_FP64 mode (the same SASO from seed, both rank stages, Q and R).
 * ws: cqrrpt_factor_hqrrp_workspace_bytes() bytes (0: out of range).
 * Argument order: A lda m n d nnz seed tol block oversample hseed Q ldq R
 * ldr J ws ws_bytes stream info. Errors: -1..-8 as cqrrpt_factor_ex,
 * -9 block < 1, -10 oversample < 0, -12 Q NULL, -13 ldq < m, -14 R NULL,
 * -15 ldr < n, -16 J NULL, -17 ws NULL, -20 info NULL, CQRRPT_ELIMIT (also
 * beyond cqrrpt_hqrrp's limits), CQRRPT_EWORKSPACE, CQRRPT_EHIP. */
size_t cqrrpt_factor_hqrrp_workspace_bytes(int64_t m, int64_t n, int64_t d, int32_t nnz,
                                           int32_t block, int32_t oversample);
int cqrrpt_factor_hqrrp_ex(const double* A, int64_t lda, int64_t m, int64_t n, int64_t d,
                           int32_t nnz, uint64_t seed, double tol, int32_t block,
                           int32_t oversample, uint64_t hseed, double* Q, int64_t ldq,
                           double* R, int64_t ldr, int64_t* J, void* ws, size_t ws_bytes,
                           void* stream, cqrrpt_info_t* info);

/* Allocation-free form of cqrrpt_factor_ex, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc). Same arguments and results as cqrrpt_factor_ex
 * without ws/ws_bytes: the workspace is a static device array of
 * CQRRPT_NOALLOC_SCRATCH_BYTES bytes inside the library (one per device,
 * held until the process ends). The call allocates nothing and returns
 * CQRRPT_EWORKSPACE, launching nothing, when cqrrpt_workspace_bytes(m, n, d,
 * nnz, mode) exceeds that size (the workspace is dominated by the Gram's
 * split partial sums, about 8 n^2 bytes per split: 30000 x 384 in FP64
 * needs about 34 MiB, 131072 x 1024 about 334 MiB; the mixed modes add
 * 4 m n bytes for the FP32 M_pre). Every call on
 * one device shares that device's array: calls that overlap on one device
 * (different streams or threads without ordering between them) race and
 * must not be issued; calls ordered on one stream are safe. Results are
 * bit-identical to cqrrpt_factor_ex's for the same arguments.
 * Argument order: A lda m n d nnz seed tol Q ldq R ldr J mode stream info.
 * Errors (nothing is launched): -1..-14 as cqrrpt_factor_ex, -16 info NULL,
 * CQRRPT_ELIMIT, CQRRPT_EWORKSPACE, CQRRPT_EHIP (symbol lookup failed). */
#define CQRRPT_NOALLOC_SCRATCH_BYTES (64u << 20)
int cqrrpt_factor_noalloc(const double* A, int64_t lda, int64_t m, int64_t n,
                          int64_t d, int32_t nnz, uint64_t seed, double tol,
                          double* Q, int64_t ldq, double* R, int64_t ldr,
                          int64_t* J, cqrrpt_mode_t mode, void* stream,
                          cqrrpt_info_t* info);

/* ------------------------------------------------------------------------
 * Stage timing (diagnostics)
 * ------------------------------------------------------------------------
 * cqrrpt_stage_timing(slots): with slots > 0, every later cqrrpt_factor_ex
 * call records HIP events on its own stream at the boundaries of its nine
 * stages (sketch, qrcp, rank_stage1, precondition, gram, cholesky, q_solve,
 * r_product, cholqr2 -- the last is empty outside the checked mixed mode),
 * using event set (call index mod slots); slots = 0 turns timing off and
 * frees the events.
 * Process-wide setting, guarded by a mutex.
 * cqrrpt_stage_times(slot, ms): waits for that slot's last event and writes
 * the nine stage durations in milliseconds to the HOST array ms[9].
 * Errors: -1 bad slot count / slot, -2 NULL ms, CQRRPT_EHIP. */
int cqrrpt_stage_timing(int slots);
int cqrrpt_stage_times(int slot, double* ms);
const char* cqrrpt_stage_name(int i);

/* ------------------------------------------------------------------------
 * Serving (derived from the serving goal; not in the paper)
 * ------------------------------------------------------------------------
 * A server admits factorization requests of any shape as they arrive and
 * runs them concurrently on the current device. Requests admitted together
 * form a batch: each runs its sketch, its solve and Gram, and its Q and R
 * products on its own slot stream, while the batch's QRCPs (grouped by
 * kernel shape) and its Cholesky steps run as single cooperative launches,
 * one gang of workgroups per request, on a server stream ordered against the
 * slot streams by events:
 *   cqrrpt_server_create(budget, max_slots, mode): allocates one device
 *     arena of `budget` bytes (all request workspaces are carved from it)
 *     and max_slots streams; NULL on bad arguments or HIP failure.
 *   cqrrpt_server_submit(...): queues one request with cqrrpt_factor_ex's
 *     arguments (device pointers, caller-owned; A must already hold its
 *     values: the server's streams do not wait on the caller's streams;
 *     info is a DEVICE cqrrpt_info_t). Returns at once with *ticket.
 *     Requests are admitted in arrival order when a slot is free and the
 *     arena fits their workspace (cqrrpt_workspace_bytes). Errors:
 *     CQRRPT_EBUDGET if the workspace exceeds the budget, -5 if the shape is
 *     out of range, -2 NULL buffer, -17 NULL ticket, -1 NULL/closing server.
 *   cqrrpt_server_poll(ticket, *done): *done = 1 once the request's work is
 *     complete on the device (its Q, R, J, info may then be read); returns
 *     the request's status once done: cqrrpt_factor_ex's return code, or,
 *     if that was 0, the device-side info->status (CQRRPT_ENONFINITE,
 *     CQRRPT_EBARRIER); -2 unknown ticket.
 *   cqrrpt_server_ticket_times(ticket, ms[3]): host steady-clock times (ms)
 *     of submission, admission and observed completion.
 *   cqrrpt_server_release(ticket): forgets a finished ticket (-3 if not
 *     finished).
 *   cqrrpt_server_drain(): blocks until every submitted request is done;
 *     returns the first non-zero request status, if any.
 *   cqrrpt_server_destroy(): drains, then frees the arena and streams.
 * A request's results are the same bits whether it runs alone or among
 * others. Any thread may submit and poll. */
typedef struct cqrrpt_server cqrrpt_server_t;
cqrrpt_server_t* cqrrpt_server_create(size_t hbm_budget_bytes, int32_t max_slots,
                                      cqrrpt_mode_t mode);
int cqrrpt_server_submit(cqrrpt_server_t* server, const double* A, int64_t lda,
                         int64_t m, int64_t n, int64_t d, int32_t nnz,
                         uint64_t seed, double tol, double* Q, int64_t ldq,
                         double* R, int64_t ldr, int64_t* J,
                         cqrrpt_info_t* info, uint64_t* ticket);
int cqrrpt_server_poll(cqrrpt_server_t* server, uint64_t ticket, int32_t* done);
int cqrrpt_server_ticket_times(cqrrpt_server_t* server, uint64_t ticket, double* ms3);
int cqrrpt_server_release(cqrrpt_server_t* server, uint64_t ticket);
int cqrrpt_server_drain(cqrrpt_server_t* server);
void cqrrpt_server_destroy(cqrrpt_server_t* server);

/* ------------------------------------------------------------------------
 * Hardware ceilings (diagnostics for roofline figures; not part of the
 * factorization)
 * ------------------------------------------------------------------------
 * cqrrpt_probe_copy: dst[i] = src[i], i < n (n even, both device, 16-byte
 *   aligned), a streaming copy: 16 n bytes of HBM traffic. Stream-ordered.
 *   Errors: -1/-2 NULL, -3 n odd or < 2.
 * cqrrpt_probe_mfma: a loop of independent 16x16x4 matrix-core instructions
 *   (fp64 != 0: FP64, else FP32 inputs and accumulation) on 8 workgroups of
 *   4 waves per compute unit, iters rounds of 8 per wave; one value per wave
 *   goes to the device array out (out_len >= 32 x compute units); *flops
 *   (host) receives the launch's floating-point operation count.
 *   Stream-ordered. Errors: -2 iters < 1, -3 NULL out, -4 out too short,
 *   -5 NULL flops. */
int cqrrpt_probe_copy(const double* src, double* dst, int64_t n, void* stream);
int cqrrpt_probe_mfma(int fp64, int iters, double* out, int64_t out_len, int64_t* flops,
                      void* stream);

/* Human-readable name of a return code. */
const char* cqrrpt_status_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* CQRRPT_H */
