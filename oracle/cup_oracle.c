/*
 * cup_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU oracle for the rank-profile revealing
 * CUP decomposition over a prime field GF(p) (Jeannerod, Pernet, Storjohann,
 * "Rank-profile revealing Gaussian elimination and the CUP matrix
 * decomposition", Section 3.3, Algorithm 6), together with independent
 * oracles for the reduced column echelon form (Section 2.2, Proposition 1 and
 * Section 3.5, Proposition 5), the inverse (Section 4.3), the matrix product
 * (Section 3.2, Algorithm 1), the PLE decomposition (Section 5,
 * Algorithm 10), and the invariants of Section 4.4 (determinant, system
 * solution, nullspace basis).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file.  The GPU library shares no code with it and
 * never links or calls it.
 *
 * Arithmetic: canonical residues in [0,p) held in int64, 2 <= p < 2^26, so a
 * product of two residues is below 2^52 and one '%' per update suffices.
 *
 * Readings of the paper used here (each is listed in the design doc):
 *  - The base case picks the leftmost nonzero of the row in the CURRENT
 *    column order, i.e. after all earlier column transpositions (Section 3.3,
 *    base case of Algorithm 6).  Unrolling the row recursion gives the
 *    iterative row-by-row elimination below; the recursion visits rows
 *    top-down, so the decisions happen in row order.
 *  - The pivot stays in C; U has an implicit unit diagonal (Section 3.1,
 *    space-sharing storage).
 *  - P is a list of transpositions, A.P^T = A.T(0,P[0]).T(1,P[1])...,
 *    applied left to right; Q lists the row rank profile the same way.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t md(int64_t x, int64_t p)
{
    int64_t r = x % p;
    return r < 0 ? r + p : r;
}

/* Inverse of a nonzero residue by the extended Euclidean algorithm. */
int64_t oracle_inv_mod(int64_t a, int64_t p)
{
    int64_t r0 = p, r1 = md(a, p), s0 = 0, s1 = 1;
    while (r1 != 0) {
        int64_t q = r0 / r1, t;
        t = r0 - q * r1; r0 = r1; r1 = t;
        t = s0 - q * s1; s0 = s1; s1 = t;
    }
    /* r0 == gcd == 1 for p prime and a != 0 */
    return md(s0, p);
}

/*
 * CUP decomposition, Algorithm 6 unrolled to one row at a time.
 *
 * In : A  m x n row-major (leading dimension n), residues in [0,p).
 * Out: A  overwritten with the packed [C\U] (Section 3.1): C (m x r, column
 *         echelon, pivots kept) in the lower part including the diagonal,
 *         the strict upper part of U's first r rows above it, zero elsewhere.
 *      *rank = r, P[0..n) transposition list (P[t] = t for t >= r),
 *      Q[0..m) with Q[t] = i_t, the row rank profile, for t < r (Q[t] = t
 *      otherwise).
 * Returns 0, or -1 on allocation failure.
 */
int oracle_cup(int64_t m, int64_t n, int64_t p, int64_t *A,
               int64_t *rank, int64_t *P, int64_t *Q)
{
    int64_t rmax = m < n ? m : n;
    int64_t *W = NULL, *C = NULL, *U = NULL;
    int64_t t = 0;

    for (int64_t c = 0; c < n; ++c) P[c] = c;
    for (int64_t i = 0; i < m; ++i) Q[i] = i;
    if (m == 0 || n == 0) { *rank = 0; return 0; }

    W = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m * n));   /* residuals   */
    C = (int64_t *)calloc((size_t)(m * n), sizeof(int64_t));     /* C, m x n    */
    U = (int64_t *)calloc((size_t)(rmax * n), sizeof(int64_t));  /* U rows < r  */
    if (!W || !C || !U) { free(W); free(C); free(U); return -1; }
    memcpy(W, A, sizeof(int64_t) * (size_t)(m * n));

    for (int64_t i = 0; i < m && t < n; ++i) {
        int64_t *wi = W + i * n;
        int64_t j = -1;
        /* leftmost nonzero of the residual of row i, positions t..n-1 */
        for (int64_t c = t; c < n; ++c)
            if (wi[c] != 0) { j = c; break; }
        if (j < 0) continue;                      /* row i is dependent */

        Q[t] = i;
        P[t] = j;
        /* column transposition t <-> j: residual rows and U rows above.
         * Columns >= t of C are still zero, so C needs no swap. */
        if (j != t) {
            for (int64_t l = i; l < m; ++l) {
                int64_t tmp = W[l * n + t]; W[l * n + t] = W[l * n + j]; W[l * n + j] = tmp;
            }
            for (int64_t s = 0; s < t; ++s) {
                int64_t tmp = U[s * n + t]; U[s * n + t] = U[s * n + j]; U[s * n + j] = tmp;
            }
        }
        int64_t inv = oracle_inv_mod(wi[t], p);
        U[t * n + t] = 1;
        for (int64_t c = t + 1; c < n; ++c)
            U[t * n + c] = md(wi[c] * inv, p);
        for (int64_t l = i; l < m; ++l)
            C[l * n + t] = W[l * n + t];
        /* eliminate column t from the rows below: W <- W - C[:,t] U[t,:] */
        #pragma omp parallel for schedule(static) if ((m - i) * (n - t) > 32768)
        for (int64_t l = i + 1; l < m; ++l) {
            int64_t f = W[l * n + t];
            if (f == 0) continue;
            int64_t *wl = W + l * n;
            const int64_t *ut = U + t * n;
            for (int64_t c = t + 1; c < n; ++c)
                wl[c] = md(wl[c] - f * ut[c], p);
        }
        ++t;
    }
    *rank = t;

    /* pack [C\U] */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            int64_t v = 0;
            if (j <= i && j < t) v = C[i * n + j];
            else if (i < t && j > i) v = U[i * n + j];
            A[i * n + j] = v;
        }
    free(W); free(C); free(U);
    return 0;
}

/*
 * Reduced column echelon form R of A (m x n), computed independently of
 * oracle_cup: the classical Gauss-Jordan reduced ROW echelon form of A^T,
 * transposed back.  Any pivot choice gives the same canonical R.
 * Out: R (m x n row-major), *rank, prof[0..rank) = the pivot positions,
 * which are the row rank profile of A.
 */
int oracle_rcef(int64_t m, int64_t n, int64_t p, const int64_t *A,
                int64_t *R, int64_t *rank, int64_t *prof)
{
    /* T = A^T, n x m */
    int64_t *T = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m * n > 0 ? m * n : 1));
    int64_t r = 0;
    if (!T) return -1;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            T[j * m + i] = A[i * n + j];
    for (int64_t c = 0; c < m && r < n; ++c) {
        int64_t piv = -1;
        for (int64_t l = r; l < n; ++l)
            if (T[l * m + c] != 0) { piv = l; break; }
        if (piv < 0) continue;
        if (piv != r)
            for (int64_t k = 0; k < m; ++k) {
                int64_t tmp = T[r * m + k]; T[r * m + k] = T[piv * m + k]; T[piv * m + k] = tmp;
            }
        int64_t inv = oracle_inv_mod(T[r * m + c], p);
        for (int64_t k = 0; k < m; ++k) T[r * m + k] = md(T[r * m + k] * inv, p);
        #pragma omp parallel for schedule(static) if (n * m > 32768)
        for (int64_t l = 0; l < n; ++l) {
            if (l == r) continue;
            int64_t f = T[l * m + c];
            if (f == 0) continue;
            for (int64_t k = 0; k < m; ++k)
                T[l * m + k] = md(T[l * m + k] - f * T[r * m + k], p);
        }
        prof[r] = c;
        ++r;
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            R[i * n + j] = T[j * m + i];
    *rank = r;
    free(T);
    return 0;
}

/*
 * Inverse of an n x n matrix by classical Gauss-Jordan on [A | I].
 * Out: Ainv (n x n).  Returns 0 if nonsingular, 1 if singular, -1 on
 * allocation failure.
 */
int oracle_inverse(int64_t n, int64_t p, const int64_t *A, int64_t *Ainv)
{
    int64_t w = 2 * n;
    int64_t *G = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n * w > 0 ? n * w : 1));
    if (!G) return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < w; ++j)
            G[i * w + j] = j < n ? A[i * n + j] : (j - n == i ? 1 : 0);
    for (int64_t c = 0; c < n; ++c) {
        int64_t piv = -1;
        for (int64_t l = c; l < n; ++l)
            if (G[l * w + c] != 0) { piv = l; break; }
        if (piv < 0) { free(G); return 1; }
        if (piv != c)
            for (int64_t k = 0; k < w; ++k) {
                int64_t tmp = G[c * w + k]; G[c * w + k] = G[piv * w + k]; G[piv * w + k] = tmp;
            }
        int64_t inv = oracle_inv_mod(G[c * w + c], p);
        for (int64_t k = 0; k < w; ++k) G[c * w + k] = md(G[c * w + k] * inv, p);
        #pragma omp parallel for schedule(static) if (n * w > 32768)
        for (int64_t l = 0; l < n; ++l) {
            if (l == c) continue;
            int64_t f = G[l * w + c];
            if (f == 0) continue;
            for (int64_t k = 0; k < w; ++k)
                G[l * w + k] = md(G[l * w + k] - f * G[c * w + k], p);
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            Ainv[i * n + j] = G[i * w + n + j];
    free(G);
    return 0;
}

/*
 * Packed output of the transformation to reduced column echelon form
 * (Section 3.1, the [X1 X2; R2 0] storage; Section 3.5, Proposition 5).
 *
 * In : packed [C\U] with rank r, P, Q as returned by oracle_cup, and the
 *      canonical R from oracle_rcef.
 * Out: O (m x n): rows 0..r hold X = U^{-1} diag(L1^{-1}, I_{n-r}) (first r
 *      rows: [X1 X2]); rows r..m hold R2 in columns 0..r, where
 *      Q R = [I_r 0; R2 0] (rows permuted by the transpositions of Q applied
 *      in increasing order), and zero in columns r..n.
 *      L1 is the r x r lower triangular block formed by the pivot rows
 *      i_0..i_{r-1} of C.
 */
int oracle_rref_pack(int64_t m, int64_t n, int64_t p, const int64_t *CU,
                     int64_t r, const int64_t *Q, const int64_t *R, int64_t *O)
{
    int64_t *Uinv = (int64_t *)calloc((size_t)(r * n > 0 ? r * n : 1), sizeof(int64_t));
    int64_t *L1inv = (int64_t *)calloc((size_t)(r * r > 0 ? r * r : 1), sizeof(int64_t));
    int64_t *QR = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m * n > 0 ? m * n : 1));
    if (!Uinv || !L1inv || !QR) { free(Uinv); free(L1inv); free(QR); return -1; }

    /* Rows 0..r of Y = U^{-1}, where U = [U1 U2; 0 I] is n x n unit upper
     * with U1, U2 read from the strict upper part of the packed rows 0..r.
     * Back substitution on U Y = I, bottom row first:
     *   Y[i] = e_i - sum_{i<s<r} U[i][s] Y[s] - sum_{s>=r} U[i][s] e_s,
     * since rows s >= r of Y are those of the identity. */
    for (int64_t i = r - 1; i >= 0; --i) {
        int64_t *yi = Uinv + i * n;
        for (int64_t j = 0; j < n; ++j) yi[j] = (i == j) ? 1 : 0;
        for (int64_t j = r; j < n; ++j) yi[j] = md(-CU[i * n + j], p);
        for (int64_t s = i + 1; s < r; ++s) {
            int64_t u = CU[i * n + s];
            if (u == 0) continue;
            const int64_t *ys = Uinv + s * n;
            #pragma omp parallel for schedule(static) if (n > 4096)
            for (int64_t j = s; j < n; ++j)
                yi[j] = md(yi[j] - u * ys[j], p);
        }
    }
    /* L1[a][b] = C[i_a][b] for b <= a (pivot rows of C, first r columns);
     * L1^{-1} by forward substitution, one column at a time. */
    #pragma omp parallel for schedule(dynamic) if (r > 64)
    for (int64_t b = 0; b < r; ++b) {
        for (int64_t a = b; a < r; ++a) {
            int64_t acc = (a == b) ? 1 : 0;
            for (int64_t s = b; s < a; ++s)
                acc = md(acc - CU[Q[a] * n + s] * L1inv[s * r + b], p);
            L1inv[a * r + b] = md(acc * oracle_inv_mod(CU[Q[a] * n + a], p), p);
        }
    }
    /* Q R */
    memcpy(QR, R, sizeof(int64_t) * (size_t)(m * n));
    for (int64_t t = 0; t < r; ++t) {
        int64_t q = Q[t];
        if (q != t)
            for (int64_t j = 0; j < n; ++j) {
                int64_t tmp = QR[t * n + j]; QR[t * n + j] = QR[q * n + j]; QR[q * n + j] = tmp;
            }
    }
    #pragma omp parallel for schedule(dynamic) if (m * n > 32768)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            int64_t v = 0;
            if (i < r) {
                if (j < r) {            /* X1 = U1^{-1} L1^{-1} */
                    int64_t acc = 0;
                    for (int64_t s = 0; s < r; ++s)
                        acc = md(acc + Uinv[i * n + s] * L1inv[s * r + j], p);
                    v = acc;
                } else {                /* X2 = rows 0..r of U^{-1}, columns r..n */
                    v = Uinv[i * n + j];
                }
            } else if (j < r) {
                v = QR[i * n + j];
            }
            O[i * n + j] = v;
        }
    free(Uinv); free(L1inv); free(QR);
    return 0;
}

/*
 * Matrix product over GF(p), the black box of Section 3.2 (Algorithm 1):
 * C <- C + alpha A B mod p for alpha = +1 or -1, written out from the
 * definition of a matrix product: one reduction after every term.
 * A is M x K, B is K x N, C is M x N, all row-major with leading dimensions
 * K, N and N.  Returns 0.
 */
int oracle_mm(int64_t M, int64_t N, int64_t K, int64_t p, const int64_t *A,
              const int64_t *B, int64_t *C, int64_t alpha)
{
    #pragma omp parallel for schedule(static) if (M * N * K > 1000000)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            int64_t acc = 0;
            for (int64_t k = 0; k < K; ++k)
                acc = md(acc + A[i * K + k] * B[k * N + j], p);
            C[i * N + j] = md(C[i * N + j] + alpha * acc, p);
        }
    return 0;
}

/*
 * PLE decomposition (Section 5, Algorithm 10) unrolled to one column at a
 * time: columns are taken left to right; for column j, with t pivots found
 * so far, the pivot is the first nonzero of the column's residual at rows
 * t..m-1 in the CURRENT row order (the base case of Algorithm 10 picks the
 * row index of the first nonzero entry).  Rows t and i are exchanged across
 * the residual and the columns of L already formed; the pivot row stays in E
 * (pivot kept), the entries below it are divided by the pivot to form
 * column t of the unit lower L, and the residual below is eliminated.
 *
 * In : A  m x n row-major (leading dimension n), residues in [0,p).
 * Out: A  overwritten with the packed [L\E] (Section 5's storage, the
 *         transpose of the [C\U] layout): E (r x n row echelon, pivots
 *         kept) in the upper part including the diagonal of its first r
 *         rows, the strict lower part of L's first r columns below it, zero
 *         in every entry (i >= r, j >= r).
 *      *rank = r; P[0..m) row transposition list (P[t] = i_t >= t for t < r,
 *      P[t] = t for t >= r: applying T(t,P[t]) to the rows of A for
 *      t = 0,1,... gives P^T A = L E); Q[0..n) with Q[t] = j_t, the column
 *      rank profile, for t < r and Q[t] = t otherwise.
 * Returns 0, or -1 on allocation failure.
 */
int oracle_ple(int64_t m, int64_t n, int64_t p, int64_t *A,
               int64_t *rank, int64_t *P, int64_t *Q)
{
    int64_t rmax = m < n ? m : n;
    int64_t *W = NULL, *L = NULL, *E = NULL;
    int64_t t = 0;

    for (int64_t i = 0; i < m; ++i) P[i] = i;
    for (int64_t c = 0; c < n; ++c) Q[c] = c;
    if (m == 0 || n == 0) { *rank = 0; return 0; }

    W = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m * n));   /* residual rows    */
    L = (int64_t *)calloc((size_t)(m * rmax), sizeof(int64_t));  /* L columns < r    */
    E = (int64_t *)calloc((size_t)(rmax * n), sizeof(int64_t));  /* E rows < r       */
    if (!W || !L || !E) { free(W); free(L); free(E); return -1; }
    memcpy(W, A, sizeof(int64_t) * (size_t)(m * n));

    for (int64_t j = 0; j < n && t < m; ++j) {
        int64_t i = -1;
        /* topmost nonzero of the residual of column j, rows t..m-1 */
        for (int64_t l = t; l < m; ++l)
            if (W[l * n + j] != 0) { i = l; break; }
        if (i < 0) continue;                     /* column j is dependent */

        P[t] = i;
        Q[t] = j;
        /* row transposition t <-> i: residual rows and the L columns < t */
        if (i != t) {
            for (int64_t c = 0; c < n; ++c) {
                int64_t tmp = W[t * n + c]; W[t * n + c] = W[i * n + c]; W[i * n + c] = tmp;
            }
            for (int64_t s = 0; s < t; ++s) {
                int64_t tmp = L[t * rmax + s]; L[t * rmax + s] = L[i * rmax + s]; L[i * rmax + s] = tmp;
            }
        }
        /* E row t: the residual pivot row, pivot kept */
        for (int64_t c = j; c < n; ++c) E[t * n + c] = W[t * n + c];
        int64_t inv = oracle_inv_mod(W[t * n + j], p);
        L[t * rmax + t] = 1;
        for (int64_t l = t + 1; l < m; ++l) L[l * rmax + t] = md(W[l * n + j] * inv, p);
        /* eliminate column j from the rows below: W[l] <- W[l] - L[l][t] E[t] */
        #pragma omp parallel for schedule(static) if ((m - t) * (n - j) > 32768)
        for (int64_t l = t + 1; l < m; ++l) {
            int64_t f = L[l * rmax + t];
            W[l * n + j] = 0;
            if (f == 0) continue;
            for (int64_t c = j + 1; c < n; ++c)
                W[l * n + c] = md(W[l * n + c] - f * E[t * n + c], p);
        }
        ++t;
    }
    *rank = t;

    /* pack [L\E] */
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            int64_t v = 0;
            if (i < t && j >= i) v = E[i * n + j];
            else if (j < t && j < i) v = L[i * rmax + j];
            A[i * n + j] = v;
        }
    free(W); free(L); free(E);
    return 0;
}

/*
 * Determinant of an n x n matrix (Section 4.4 lists it among the invariants
 * the CUP decomposition yields), by classical Gaussian elimination: the
 * first nonzero entry of each column at or below the diagonal is the pivot,
 * every row exchange flips the sign, and the determinant is the signed
 * product of the pivots (0 when a column has no pivot).  Returns det in
 * [0,p), or -1 on allocation failure.
 */
int64_t oracle_det(int64_t n, int64_t p, const int64_t *A)
{
    int64_t *G = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n * n > 0 ? n * n : 1));
    int64_t det = 1;
    if (!G) return -1;
    memcpy(G, A, sizeof(int64_t) * (size_t)(n * n));
    for (int64_t c = 0; c < n; ++c) {
        int64_t piv = -1;
        for (int64_t l = c; l < n; ++l)
            if (G[l * n + c] != 0) { piv = l; break; }
        if (piv < 0) { free(G); return 0; }
        if (piv != c) {
            for (int64_t k = 0; k < n; ++k) {
                int64_t tmp = G[c * n + k]; G[c * n + k] = G[piv * n + k]; G[piv * n + k] = tmp;
            }
            det = md(-det, p);
        }
        det = md(det * G[c * n + c], p);
        int64_t inv = oracle_inv_mod(G[c * n + c], p);
        #pragma omp parallel for schedule(static) if (n * n > 32768)
        for (int64_t l = c + 1; l < n; ++l) {
            int64_t f = md(G[l * n + c] * inv, p);
            if (f == 0) continue;
            for (int64_t k = c; k < n; ++k)
                G[l * n + k] = md(G[l * n + k] - f * G[c * n + k], p);
        }
    }
    free(G);
    return det;
}

/*
 * Solution of the linear system A X = B for a nonsingular n x n matrix A and
 * an n x nrhs right-hand side B (Section 4.4: the CUP decomposition suffices
 * for it), by classical Gauss-Jordan elimination on [A | B].
 * Out: X (n x nrhs).  Returns 0, 1 if A is singular, -1 on allocation failure.
 */
int oracle_solve(int64_t n, int64_t nrhs, int64_t p, const int64_t *A,
                 const int64_t *B, int64_t *X)
{
    int64_t w = n + nrhs;
    int64_t *G = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n * w > 0 ? n * w : 1));
    if (!G) return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < w; ++j)
            G[i * w + j] = j < n ? A[i * n + j] : B[i * nrhs + (j - n)];
    for (int64_t c = 0; c < n; ++c) {
        int64_t piv = -1;
        for (int64_t l = c; l < n; ++l)
            if (G[l * w + c] != 0) { piv = l; break; }
        if (piv < 0) { free(G); return 1; }
        if (piv != c)
            for (int64_t k = 0; k < w; ++k) {
                int64_t tmp = G[c * w + k]; G[c * w + k] = G[piv * w + k]; G[piv * w + k] = tmp;
            }
        int64_t inv = oracle_inv_mod(G[c * w + c], p);
        for (int64_t k = 0; k < w; ++k) G[c * w + k] = md(G[c * w + k] * inv, p);
        #pragma omp parallel for schedule(static) if (n * w > 32768)
        for (int64_t l = 0; l < n; ++l) {
            if (l == c) continue;
            int64_t f = G[l * w + c];
            if (f == 0) continue;
            for (int64_t k = 0; k < w; ++k)
                G[l * w + k] = md(G[l * w + k] - f * G[c * w + k], p);
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < nrhs; ++j)
            X[i * nrhs + j] = G[i * w + n + j];
    free(G);
    return 0;
}

/*
 * Basis of the right nullspace of an m x n matrix A of rank r, in the form
 * the transformation to column echelon form gives (Section 3.4: with
 * A P^T X = [C 0], the last n - r columns of P^T X span the nullspace).
 *
 * The column order comes from the transposition list P of the CUP
 * decomposition (P[t] for t < r): order[] starts as 0..n-1 and T(t,P[t]) is
 * applied to it for t = 0,1,..., so that column c of A P^T is column
 * order[c] of A, and the first r of them are linearly independent.  The
 * basis is then fixed by the definition: vector s (s = 0..n-r-1) has a one
 * at the free column order[r+s], zeros at the other free columns, and the
 * unique values at the columns order[0..r) that make A x = 0.  They are
 * found here by a classical Gauss-Jordan reduction of A P^T (m x n), whose
 * pivots fall on its first r columns: with the reduced rows [I_r R; 0 0],
 * x'[0..r) = -R[:, s] and x[order[c]] = x'[c].
 * Out: N (n x (n - r), row-major, leading dimension n - r).
 * Returns 0, or -1 on allocation failure, -2 if the first r columns of
 * A P^T are not independent (P is not a CUP transposition list of A).
 */
int oracle_nullspace(int64_t m, int64_t n, int64_t p, const int64_t *A,
                     int64_t r, const int64_t *P, int64_t *N)
{
    int64_t f = n - r;
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *G = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m * n > 0 ? m * n : 1));
    if (!order || !G) { free(order); free(G); return -1; }
    for (int64_t c = 0; c < n; ++c) order[c] = c;
    for (int64_t t = 0; t < r; ++t) {
        int64_t tmp = order[t]; order[t] = order[P[t]]; order[P[t]] = tmp;
    }
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < n; ++c)
            G[i * n + c] = A[i * n + order[c]];
    /* Gauss-Jordan on the rows of A P^T; pivots must be columns 0..r-1 */
    for (int64_t c = 0; c < r; ++c) {
        int64_t piv = -1;
        for (int64_t l = c; l < m; ++l)
            if (G[l * n + c] != 0) { piv = l; break; }
        if (piv < 0) { free(order); free(G); return -2; }
        if (piv != c)
            for (int64_t k = 0; k < n; ++k) {
                int64_t tmp = G[c * n + k]; G[c * n + k] = G[piv * n + k]; G[piv * n + k] = tmp;
            }
        int64_t inv = oracle_inv_mod(G[c * n + c], p);
        for (int64_t k = 0; k < n; ++k) G[c * n + k] = md(G[c * n + k] * inv, p);
        #pragma omp parallel for schedule(static) if (m * n > 32768)
        for (int64_t l = 0; l < m; ++l) {
            if (l == c) continue;
            int64_t g = G[l * n + c];
            if (g == 0) continue;
            for (int64_t k = 0; k < n; ++k)
                G[l * n + k] = md(G[l * n + k] - g * G[c * n + k], p);
        }
    }
    for (int64_t s = 0; s < f; ++s) {
        for (int64_t c = 0; c < n; ++c) N[order[c] * f + s] = 0;
        N[order[r + s] * f + s] = 1;
        for (int64_t c = 0; c < r; ++c)
            N[order[c] * f + s] = md(-G[c * n + r + s], p);
    }
    free(order); free(G);
    return 0;
}
