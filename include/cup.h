/*
 * libcup -- rank-profile revealing CUP decomposition over a prime field
 * GF(p) on AMD MI355X (gfx950).
 *
 * The operations follow C.-P. Jeannerod, C. Pernet and A. Storjohann,
 * "Rank-profile revealing Gaussian elimination and the CUP matrix
 * decomposition" (J. Symbolic Computation):
 *   - CUP decomposition A = C U P with its rank and row rank profile
 *     (Section 3.3, Algorithm 6; Proposition 3),
 *   - transformation to reduced column echelon form (Section 3.4,
 *     Algorithm 7 and Section 3.5, Algorithm 8; Proposition 5),
 *   - the in-place inverse (Section 4.3),
 *   - the PLE decomposition (Section 5, Algorithm 10),
 *   - the determinant, system solution and nullspace basis (Sections 3.4
 *     and 4.4), TRLUM (Algorithm 5) and InPlaceMM (Algorithm 9).
 *
 * Conventions shared by every entry point
 *   - Matrices are row-major with leading dimension lda >= max(1, n):
 *     entry (i, j) is A[i * lda + j].  A is a DEVICE pointer.
 *   - Entries are canonical residues in [0, p); every output is canonical.
 *     p must be prime with 2 <= p < 2^26.  Entries outside [0, p) are
 *     undefined behaviour unless the environment variable CUP_CHECK=1 is
 *     set, in which case the call returns -3 before touching A.
 *   - Permutations are LAPACK-style transposition lists (Section 4.1):
 *       P[t] = p_t >= t for t < r and P[t] = t for t >= r, so that
 *       A P^T = A T(0,p_0) T(1,p_1) ... T(r-1,p_{r-1}) (applied left to right);
 *       Q[t] = i_t, the row rank profile i_0 < ... < i_{r-1}, for t < r and
 *       Q[t] = t for t >= r; applying T(t,Q[t]) to the rows for t = 0,1,...
 *       brings the pivot rows to the top.
 *     P (length n) and Q (length m) are DEVICE int64 arrays; either may be
 *     NULL when not wanted.  *rank is a HOST pointer.
 *   - m = 0 or n = 0 is a valid no-op: rank 0, identity P and Q.
 *   - The caller owns every buffer.  The library keeps no caller memory; it
 *     caches small device and pinned-host scratch (and, for the INT8 forms,
 *     a GEMM packing workspace) until cup_finalize().
 *   - Work is issued on the stream set by cup_set_stream (default: the null
 *     stream).  Single-matrix calls return after their work has completed.
 *   - On any error after work has started the contents of A are
 *     unspecified; callers that need the input keep a copy.
 *
 * Return codes (LAPACK style)
 *      0  CUP_OK
 *      1  CUP_SINGULAR  (inverse only; *rank is set, A is unspecified)
 *     -i  the i-th argument is invalid
 *  -1000 - e   a HIP runtime error e
 *  -2000  a device or host allocation failed (a test can force this path by
 *         setting CUP_FAULT=alloc in the environment: every allocation of the
 *         library then fails without allocating)
 */
#ifndef LIBCUP_CUP_H
#define LIBCUP_CUP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CUP_OK 0
#define CUP_SINGULAR 1
#define CUP_ERR_HIP (-1000)
#define CUP_ERR_ALLOC (-2000)
/* An internal consistency check of a kernel failed (a pivot row that a
 * waiting wave never received); the matrix is then unspecified. */
#define CUP_ERR_INTERNAL (-3000)
/* A size beyond the fixed scratch of an allocation-free entry point. */
#define CUP_ERR_NOALLOC_LIMIT (-4000)
/* Largest batch of cup_factor_batched_noalloc. */
#define CUP_NOALLOC_BATCH_MAX 32768

/* Forms of the modular matrix product (ffgemm) used inside every call.
 *   FP64   : FP64 MFMA as an exact integer carrier, any p < 2^26.
 *   I8     : INT8 MFMA with INT32 accumulation, p < 2^7.
 *   I8LIMB : each operand split into two signed 8-bit limbs, four INT8 MFMA
 *            products recombined exactly, p <= 2^16.
 *   AUTO   : the fastest form valid for p and the storage type. */
#define CUP_FORM_AUTO 0
#define CUP_FORM_FP64 1
#define CUP_FORM_I8 2
#define CUP_FORM_I8LIMB 3

/* Stream for all later work (a hipStream_t; NULL = the null stream). */
int cup_set_stream(void *hip_stream);

/* Select the ffgemm form for later calls.  Returns -1 for an unknown form.
 * A forced form that p does not allow makes later calls return -5.  The
 * initial form is CUP_FORM from the environment when it names one (auto,
 * fp64, i8, i8limb, or 0..3), read once when the library is first used;
 * otherwise CUP_FORM_AUTO. */
int cup_set_form(int form);
int cup_get_form(void);

/*
 * Strassen-Winograd products (Section 4.4, Table 1's exponent log2 7, after
 * Winograd's seven-product scheme) for later calls: every modular product
 * whose M, N and K are all at least min_dim is split into quadrants and
 * formed with seven half-size products instead of eight, recursively up to
 * `levels` times (0, the default, keeps the classical products).  Sums of
 * quadrants and the seven partial products are canonical residue matrices
 * in a library workspace of about (4/3)(MK + KN + MN) elements for one level
 * (reported by cup_workspace_bytes), so results are identical to the
 * classical product's.  Returns -1 for levels outside 0..8, -2 for
 * min_dim < 128.
 */
int cup_set_winograd(int levels, int64_t min_dim);

/*
 * CUP decomposition (Section 3.3, Algorithm 6).
 *   m, n  : dimensions (>= 0)
 *   A     : device, m x n, int64 residues; overwritten in place with the
 *           packed [C\U] of Section 3.1: C (column echelon, pivots kept) in
 *           the lower part including the diagonal of its first r columns,
 *           the strict upper part of the first r rows of U above it, and
 *           zero in every entry (i >= r, j >= r).
 *   lda   : leading dimension (>= max(1, n))
 *   p     : prime, 2 <= p < 2^26
 *   rank  : host, receives r
 *   P, Q  : device int64 transposition lists (see above), or NULL.
 * The pivot rule is the paper's: the leftmost nonzero of each row's residual
 * in the current column order, rows taken top to bottom, so the output is
 * unique (Section 2.2, Proposition 1).
 * Errors: -1 m, -2 n, -3 A (or an entry out of range under CUP_CHECK=1),
 * -4 lda, -5 p, -6 rank.
 */
int cup_factor(int64_t m, int64_t n, int64_t *A, int64_t lda, int64_t p, int64_t *rank,
               int64_t *P, int64_t *Q);

/* The same on int8 storage (residues of a prime p < 2^7). */
int cup_factor_i8(int64_t m, int64_t n, int8_t *A, int64_t lda, int64_t p, int64_t *rank,
                  int64_t *P, int64_t *Q);

/*
 * Rank and row rank profile (Section 2, definition; Section 4.3: CUP
 * suffices).  Runs cup_factor, so A is overwritten with [C\U].
 * Q: device int64 array of length m as above (or NULL).
 */
int cup_rank_profile(int64_t m, int64_t n, int64_t *A, int64_t lda, int64_t p, int64_t *rank,
                     int64_t *Q);

/*
 * Transformation to reduced column echelon form, in place (Section 3.5,
 * Algorithm 8 over Algorithm 7 over Algorithm 6; Proposition 5).
 *   A <- [X1 X2; R2 0] (Section 3.1 storage): with X = [X1 X2; 0 I_{n-r}]
 *   and R = Q^T [I_r 0; R2 0], A P^T X = R is the (canonical) reduced column
 *   echelon form of A.  P, Q, rank as for cup_factor.
 */
int cup_rref_inplace(int64_t m, int64_t n, int64_t *A, int64_t lda, int64_t p, int64_t *rank,
                     int64_t *P, int64_t *Q);
int cup_rref_inplace_i8(int64_t m, int64_t n, int8_t *A, int64_t lda, int64_t p, int64_t *rank,
                        int64_t *P, int64_t *Q);

/*
 * In-place inverse of an n x n matrix (Section 4.3: the reduced echelon
 * transformation of a nonsingular matrix is its inverse up to P):
 * A <- A^{-1} = P^T X.  Returns CUP_SINGULAR (1) with *rank < n when A is
 * singular; A is then unspecified.
 */
int cup_inverse_inplace(int64_t n, int64_t *A, int64_t lda, int64_t p, int64_t *rank);
int cup_inverse_inplace_i8(int64_t n, int8_t *A, int64_t lda, int64_t p, int64_t *rank);

/*
 * Batched CUP of independent matrices, each with its own prime
 * (Algorithm 6 per matrix; a multi-modular workload).  One GPU workgroup
 * factors one matrix; one persistent kernel per width class (n <= 128,
 * n <= 256, n <= 512) keeps as many workgroups as fit on the GPU, each
 * taking the class's matrices largest first (batches of up to 32768 are
 * ordered by m n min(m, n)) from a work counter; each result is the one
 * cup_factor gives.  Matrices with n > 512 are factored afterwards, one by
 * one, by the recursive single-matrix path on the same stream.
 *   batch          : number of matrices (>= 0)
 *   m, n, lda, p   : device int64 arrays of length batch
 *   A              : device array of batch device pointers (int64 matrices)
 *   rank           : device int64 array of length batch
 *   P, Q           : device arrays of batch device pointers (each P[i] of
 *                    length n[i], Q[i] of length m[i]); P or Q may be NULL
 *   info           : device int32 array; info[i] receives matrix i's status
 *                    with the argument codes of cup_factor (-1 m, -2 n,
 *                    -3 A, -4 lda, -5 p); rank[i] is 0 on error
 * Returns 0 when the batch was queued (per-matrix status in info), or a
 * negative code for an invalid batch-level argument (-1 batch, -2 m, -3 n,
 * -4 A, -5 lda, -6 p, -7 rank, -10 info; -2000 workspace allocation).  The
 * column counts are copied to the host on the stream ahead of the kernels
 * (the call waits for that copy): without a matrix wider than 512 the call
 * is asynchronous on the stream (outputs on the device only); with one, it
 * returns after those matrices are factored.
 */
int cup_factor_batched(int64_t batch, const int64_t *m, const int64_t *n, int64_t *const *A,
                       const int64_t *lda, const int64_t *p, int64_t *rank, int64_t *const *P,
                       int64_t *const *Q, int32_t *info);

/*
 * PLE decomposition (Section 5, Algorithm 10), the row-echelon twin of CUP:
 * P^T A = L E, revealing the column rank profile.  Computed as the
 * transpose of the CUP of A^T, the relation Section 5 states between the
 * two decompositions (the CUP pivot rule on A^T is PLE's rule on A: the
 * topmost nonzero of each column's residual, columns left to right).
 *   A : device m x n (lda), overwritten with the packed [L\E]: E (r x n row
 *       echelon, pivots kept) in the upper part including the diagonal of
 *       its first r rows, the strict lower part of L's first r columns
 *       (L unit lower) below it, zero in every entry (i >= r, j >= r).
 *   P : device int64, length m: the row transposition list, P[t] = i_t >= t
 *       for t < r and P[t] = t otherwise; applying T(t, P[t]) to the rows
 *       of A for t = 0, 1, ... gives P^T A = L E.
 *   Q : device int64, length n: Q[t] = j_t, the column rank profile, for
 *       t < r, Q[t] = t otherwise.  Either may be NULL.
 * A square matrix is transposed in place; a rectangular one goes through a
 * library workspace of m n elements (reported by cup_workspace_bytes).
 * Errors as cup_factor (-1 m, -2 n, -3 A, -4 lda, -5 p, -6 rank).
 */
int cup_ple(int64_t m, int64_t n, int64_t *A, int64_t lda, int64_t p, int64_t *rank, int64_t *P,
            int64_t *Q);
int cup_ple_i8(int64_t m, int64_t n, int8_t *A, int64_t lda, int64_t p, int64_t *rank, int64_t *P,
               int64_t *Q);

/*
 * Determinant (Section 4.4, an invariant the CUP decomposition yields): with
 * A P^T = C U, det A = det(P) * prod_t C[t][t] for a nonsingular n x n A (C
 * is then lower triangular and U unit upper), det(P) = (-1)^(number of t
 * with P[t] != t), and det A = 0 when the rank is below n.
 *   A    : device n x n (lda), overwritten with the packed [C\U]
 *   det  : host, receives det A in [0, p) (1 for n = 0)
 *   rank : host, receives the rank
 * Errors: -1 n, -2 A (or an entry out of range under CUP_CHECK=1), -3 lda,
 * -4 p, -5 det, -6 rank.
 */
int cup_det(int64_t n, int64_t *A, int64_t lda, int64_t p, int64_t *det, int64_t *rank);

/*
 * Solution of A X = B for a nonsingular n x n A (Section 4.4): CUP of A,
 * then X = P^T U^{-1} C^{-1} B by the Left-Lower-NonUnit and
 * Left-Upper-Unit triangular solves (Algorithm 2's variants) and the row
 * transpositions t <-> P[t] for t = n-1 down to 0.
 *   A : device n x n (lda), overwritten with the packed [C\U]
 *   B : device n x nrhs (ldb >= max(1, nrhs)), overwritten with X
 * Returns CUP_SINGULAR (1) with *rank < n when A is singular (B is then
 * untouched).  Errors: -1 n, -2 nrhs, -3 A, -4 lda, -5 B, -6 ldb, -7 p,
 * -8 rank.
 */
int cup_solve(int64_t n, int64_t nrhs, int64_t *A, int64_t lda, int64_t *B, int64_t ldb, int64_t p,
              int64_t *rank);

/*
 * Basis of the right nullspace of an m x n A of rank r (Section 3.4: with
 * A P^T X = [C 0] and X = [U1^{-1}, -U1^{-1} U2; 0, I_{n-r}], the last n - r
 * columns of P^T X span the kernel):  N = P^T [-U1^{-1} U2; I_{n-r}], so
 * A N = 0, and row P-position r + s of N is the unit vector e_s.
 *   A   : device m x n (lda), overwritten with [C\U] whose block right of
 *         the first r columns holds -U1^{-1} U2 (Algorithm 7's first steps)
 *   P   : device int64 transposition list of length n (or NULL)
 *   N   : device, n rows with leading dimension ldn >= max(1, n): receives
 *         the n x (n - r) basis in its first n - r columns
 * Errors: -1 m, -2 n, -3 A, -4 lda, -5 p, -6 rank, -8 N, -9 ldn.
 */
int cup_nullspace(int64_t m, int64_t n, int64_t *A, int64_t lda, int64_t p, int64_t *rank, int64_t *P,
                  int64_t *N, int64_t ldn);

/*
 * TRLUM (Section 3.2, Algorithm 5) in the variant that InPlaceMM applies to
 * a packed CUP: A = [L\U] (n x n, L lower triangular with its diagonal
 * stored, U unit upper with its strict upper part stored) <- L U, in place.
 * Errors: -1 n, -2 A, -3 lda, -4 p.
 */
int cup_trlum(int64_t n, int64_t *A, int64_t lda, int64_t p);

/*
 * InPlaceMM (Section 4.3, Algorithm 9): B <- A B for an m x m A and an
 * m x n B with no temporary of B's size: CUP of A (A = C U P), B <- P B,
 * B <- U B, B <- C B (triangular products), then A <- C U (TRLUM) and
 * A <- A P, which restores A.
 *   A : device m x m (lda), unchanged on return
 *   B : device m x n (ldb >= max(1, n)), overwritten with A B
 * Errors: -1 m, -2 n, -3 A, -4 lda, -5 B, -6 ldb, -7 p.
 */
int cup_inplace_mm(int64_t m, int64_t n, int64_t *A, int64_t lda, int64_t *B, int64_t ldb, int64_t p);

/*
 * cup_factor_batched for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same arguments, launches and results as cup_factor_batched, but the
 * library's scratch (the processing order of the batch, 4 bytes per matrix)
 * lives in a static device array of CUP_NOALLOC_BATCH_MAX + 64 entries
 * (128 KiB and 256 bytes, held on each GPU the library runs on until the
 * process ends, with the kernels' work counters), so the call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * The caller passes every input and output.  A batch above
 * CUP_NOALLOC_BATCH_MAX returns CUP_ERR_NOALLOC_LIMIT before any work.
 * Nothing is read back and nothing synchronises, so the call can be
 * captured in a HIP graph; matrices with n > 512 are not routed to the
 * single-matrix path here (that needs the host): they get info -2.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (on different streams, or from different threads without ordering)
 * race on it.  Asynchronous on the stream, like cup_factor_batched.
 */
int cup_factor_batched_noalloc(int64_t batch, const int64_t *m, const int64_t *n, int64_t *const *A,
                               const int64_t *lda, const int64_t *p, int64_t *rank,
                               int64_t *const *P, int64_t *const *Q, int32_t *info);

/*
 * Modular matrix product, the black box of Section 3.2 (Algorithm 1) that
 * every routine above reduces to:  C <- C + alpha A B mod p, alpha = +1 or
 * -1 (CUP's Schur complement uses -1, Algorithm 6), in the form selected by
 * cup_set_form.  A is M x K (lda), B is K x N (ldb), C is M x N (ldc), all
 * device row-major residues; C must not overlap A or B (Algorithm 1 Data).
 * Errors: -1 M, -2 N, -3 K, -5 A/lda, -7 B/ldb, -9 C/ldc, -10 p,
 * -11 alpha.  Returns after the product has completed.
 */
int cup_ffgemm(int64_t M, int64_t N, int64_t K, const int64_t *A, int64_t lda, const int64_t *B,
               int64_t ldb, int64_t *C, int64_t ldc, int64_t p, int alpha);
int cup_ffgemm_i8(int64_t M, int64_t N, int64_t K, const int8_t *A, int64_t lda, const int8_t *B,
                  int64_t ldb, int8_t *C, int64_t ldc, int64_t p, int alpha);

/* Text for a return code. */
const char *cup_strerror(int status);

/*
 * Kernel timing for measurement.  cup_profile(1) resets and starts timing
 * every ffgemm launch and every leaf-window launch with a pair of HIP events
 * on the launch stream (no extra synchronisation); cup_profile(0) stops.
 * A value above 1 times only the classes whose bits it sets, bit k + 1 for
 * class k below (2: the FP64-carrier and direct products, 8: the INT8
 * product kernel): those product launches record their own events, so
 * timing them alone adds no work to the stream, while the window and
 * packing classes (4 and 16) add an event record before and after each
 * launch.  Returns -1 for a value outside 0 .. 31.
 * cup_profile_read fills stats[16] with four figures for each of four
 * kernel classes: {launches, kernel ms, algorithmic field operations
 * (2MNK per product), algorithmic bytes} for (0) the products below the
 * INT8 kernel's threshold (FP64 carrier, or the direct INT8-limb kernel in
 * the INT8 forms; bytes (MK + KN + 2MN) x element size), (1) the leaf window kernel
 * (operations 0, bytes one read and one write of its tile), (2) the INT8
 * ffgemm product kernel (bytes: packed operands read once plus C read and
 * written), (3) the INT8 operand packing (operations 0, bytes read and
 * written).  Returns -1 if stats is NULL.
 */
int cup_profile(int enable);
int cup_profile_read(double *stats);

/*
 * Bytes of device workspace currently cached by the library (it grows to the
 * largest call since the last cup_finalize).  After calls on matrices of at
 * most m x n, with k = min(m, n), it is at most
 *     16 KiB                                  result words
 *   + 32 KiB * (max(64, ceil(k/64)) + floor(k/64))
 *                                             dense inverses of the 64 x 64
 *                                             diagonal blocks of the triangle
 *                                             being solved, and the cache of
 *                                             those of U (Section 3.2 leaves)
 *   + 4 * max(k, 1024)                        row rank profile (reduced forms)
 *   + 2 * (m + n + 256) * (k + 64)            INT8 forms only: packed limb
 *                                             operands of one product
 *   + 4 * max(batch + 64, 4096)               batched work counters and order
 * The two block caches are the library's departure from Definition 1
 * (Section 3.1: O(1) extra field elements outside matrix multiplication):
 * O(k) blocks of 64 x 64, i.e. 64 k field elements against the m n of A.
 * The packed operands are matrix-multiplication memory, which Definition 1
 * allows.
 */
size_t cup_workspace_bytes(void);

/* Release cached workspace. */
int cup_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* LIBCUP_CUP_H */
