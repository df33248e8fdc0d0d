// Leaves of the triangular routines of Section 3.2 (TRSM, TRMM, TRTRI,
// TRULM) on diagonal blocks of order <= 64.
//
// A triangular solve B T^{-1} (or T^{-1} B) on a 64-column (64-row) block is
// a product with the block's inverse, and a triangular multiply is a product
// with the block itself.  So the solve/multiply leaves are two steps:
//
//  * diag_prep: one workgroup per diagonal block of the whole triangle
//    builds the dense 64 x 64 matrix W = T_bb^{-1} (solve) or W = T_bb
//    (multiply), padded with the identity, into a workspace.  The inverse
//    is computed column-parallel (thread j solves T x = e_j) with the
//    column held in registers and the loops fully unrolled.
//  * tri_apply: B <- B W (right) or W B (left) for one leaf, every output
//    an independent 64-term dot product; rows (columns) of B are staged in
//    LDS so the product can overwrite them in place.
//
// Dot products of canonical residues are exact in FP64 while their sum stays
// below 2^53: 64 terms suffice for p < 2^23.5; for larger p (below 2^26) the
// partial sum is reduced after every term (the BIG instantiations), since a
// reduced sum plus one product stays below p + p^2 < 2^53.
#include "modarith.h"
#include "tri64.h"

namespace cup {

namespace {

constexpr int NB = kTriNB;

// Load the triangle of block b (order nb <= 64, at A + o*lda + o) into
// M[64][65] with zeros outside the triangle, the unit diagonal if `unit`,
// and identity padding beyond nb.
template <typename T>
__device__ void load_triangle(double (*M)[NB + 1], const T* A, int64_t lda, int o, int nb,
                              int uplo, int unit)
{
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
        int i = idx >> 6, s = idx & 63;
        double v;
        if (i >= nb || s >= nb) {
            v = (i == s) ? 1.0 : 0.0;
        } else {
            bool in = (uplo == 0) ? (s >= i) : (s <= i);
            v = in ? ld_res(A + (int64_t)(o + i) * lda + o + s) : 0.0;
            if (i == s && unit) v = 1.0;
        }
        M[i][s] = v;
    }
}

// Column j of the inverse of the triangle in M (solves M x = e_j) for
// p >= 2^23.5: rolled loops, the column in LDS (X[.][j]), the partial sum
// reduced after every product.
__device__ __forceinline__ void inverse_column_big(const double (*M)[NB + 1], const double* dinv, int uplo,
                                   int j, double (*X)[NB + 1], double P, double PI)
{
    for (int i = 0; i < NB; ++i) X[i][j] = 0.0;
    for (int t = 0; t < NB; ++t) {
        const int i = (uplo == 1) ? t : NB - 1 - t;
        const int s0 = (uplo == 1) ? 0 : i + 1, s1 = (uplo == 1) ? i : NB;
        double acc = 0.0;
        for (int s = s0; s < s1; ++s) acc = mod_red(fma(M[i][s], X[s][j], acc), P, PI);
        double r = ((i == j) ? 1.0 : 0.0) - acc;
        r = (r < 0.0) ? r + P : r;
        X[i][j] = mod_mul(r, dinv[i], P, PI);
    }
}


// mode 0: W[b] = T_bb^{-1}; mode 1: W[b] = T_bb; mode 2: T_bb <- T_bb^{-1} in
// place (the unit diagonal, if any, is left untouched).  One workgroup of
// 256 threads per diagonal block; a lower triangle is handled as the
// transpose of an upper one.
// An optional second job (A2: one full 64 x 64 block, its own triangle and
// diagonal kind, output W2) runs as the last workgroup of the same launch.
template <typename T, bool BIG>
__global__ __launch_bounds__(256) void diag_prep_kernel(T* __restrict__ A, int64_t lda, int n, int uplo,
                                                        int unit, int mode, double* __restrict__ W,
                                                        ModP mp, T* __restrict__ A2, int uplo2,
                                                        int unit2, double* __restrict__ W2,
                                                        const int* __restrict__ guard, int expect)
{
    if (guard && *guard != expect) return;  // launched ahead of a pivot count that differs
    __shared__ double M[NB][NB + 1];
    __shared__ double X[NB][NB + 1];
    __shared__ double dinv[NB];
    int b = blockIdx.x;
    if (A2 != nullptr && b == (int)gridDim.x - 1) {
        A = A2;
        n = NB;
        uplo = uplo2;
        unit = unit2;
        W = W2;
        b = 0;
    }
    const int o = b * NB, nb = min(NB, n - o), tid = threadIdx.x;
    const double P = mp.p, PI = mp.pinv;
    // M = T_bb (upper) or its transpose (lower), identity-padded.  Every
    // address is clamped into the block so the 16 loads of a thread issue
    // together; the selects pick identity and zeros afterwards.
    {
        double ld_v[NB * NB / 256];
#pragma unroll
        for (int it = 0; it < NB * NB / 256; ++it) {
            const int idx = tid + 256 * it, i = idx >> 6, s = idx & 63;
            const int r = (uplo == 0) ? i : s, c = (uplo == 0) ? s : i;  // element (r, c) of T
            const int rc = min(r, nb - 1), cc = min(c, nb - 1);
            ld_v[it] = ld_res(A + (int64_t)(o + rc) * lda + o + cc);
        }
#pragma unroll
        for (int it = 0; it < NB * NB / 256; ++it) {
            const int idx = tid + 256 * it, i = idx >> 6, s = idx & 63;
            double v = (s >= i) ? ld_v[it] : 0.0;
            if (i == s && unit) v = 1.0;
            if (i >= nb || s >= nb) v = (i == s) ? 1.0 : 0.0;
            M[i][s] = v;
        }
    }
    __syncthreads();
    if (mode == 1) {
        double* Wb = W + (size_t)b * NB * NB;
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int i = idx >> 6, s = idx & 63;
            Wb[idx] = (uplo == 0) ? M[i][s] : M[s][i];
        }
        return;
    }
    if (tid < NB) dinv[tid] = (unit || tid >= nb) ? 1.0 : canon(inv_fermat26(M[tid][tid], P, PI), P);
    __syncthreads();
    if constexpr (BIG) {
        if (tid < NB) inverse_column_big(M, dinv, 0, tid, X, P, PI);
        __syncthreads();
    } else {
        // T = D T' with T' unit (rows scaled by the diagonal's inverses), so
        // T^{-1} = T'^{-1} D^{-1}: the unit inverse, then its columns scaled
        if (!unit) {
            double mv[NB * NB / 256];
#pragma unroll
            for (int it = 0; it < NB * NB / 256; ++it) {
                const int idx = tid + 256 * it, i = idx >> 6, s2 = idx & 63;
                mv[it] = red_near(M[i][s2] * dinv[i], P, PI);
            }
#pragma unroll
            for (int it = 0; it < NB * NB / 256; ++it) {
                const int idx = tid + 256 * it, i = idx >> 6, s2 = idx & 63;
                if (s2 > i) M[i][s2] = mv[it];
            }
            __syncthreads();
        }
        unit_upper_inverse(M, X, P, PI);
        if (!unit) {
            double xv[NB * NB / 256];
#pragma unroll
            for (int it = 0; it < NB * NB / 256; ++it) {
                const int idx = tid + 256 * it, i = idx >> 6, s2 = idx & 63;
                xv[it] = red_near(X[i][s2] * dinv[s2], P, PI);
            }
            __syncthreads();
#pragma unroll
            for (int it = 0; it < NB * NB / 256; ++it) {
                const int idx = tid + 256 * it, i = idx >> 6, s2 = idx & 63;
                X[i][s2] = xv[it];
            }
            __syncthreads();
        }
    }
    // X holds the inverse of the upper form; the lower inverse is its transpose
    if (mode == 0) {
        double* Wb = W + (size_t)b * NB * NB;
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int i = idx >> 6, s = idx & 63;
            Wb[idx] = canon((uplo == 0) ? X[i][s] : X[s][i], P);
        }
    } else {
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int i = idx >> 6, s = idx & 63;  // element (i, s) of the inverse
            if (i >= nb || s >= nb) continue;
            const bool write = (uplo == 0) ? (unit ? s > i : s >= i) : (unit ? s < i : s <= i);
            if (write) st_res(A + (int64_t)(o + i) * lda + o + s, canon((uplo == 0) ? X[i][s] : X[s][i], P));
        }
    }
}

// B <- B W (side 1, B is rows x nb) or W B (side 0, B is nb x cols), W dense
// 64 x 64 (identity beyond nb).  Each workgroup owns 16 rows (right) or 16
// columns (left) of B; each thread computes 4 of their 16 x 64 outputs.
constexpr int AV = 16;  // vectors per workgroup

// The work of workgroup blk (also run by the combined launch with the slab solve).
template <typename T, bool BIG>
__device__ __forceinline__ void tri_apply_block(int blk, int side, int nb, const double* __restrict__ W,
                                                T* __restrict__ B, int64_t ldb, int other, ModP mp)
{
    __shared__ double Ws[NB][NB + 1];
    __shared__ double Bs[AV][NB + 1];
    const int tid = threadIdx.x;
    const double P = mp.p, PI = mp.pinv;
    const int v0 = blk * AV;
    const int nv = min(AV, other - v0);
    // all loads of a thread issued together (addresses clamped, selects after)
    {
        double wv[NB * NB / 256];
#pragma unroll
        for (int it = 0; it < NB * NB / 256; ++it) {
            const int idx = tid + 256 * it, i = idx >> 6, e = idx & 63;
            // right: Ws[s][e] = W[s][e]; left: Ws[e][s] = W[e][s] read as Ws[s][e] = W[e][s]
            wv[it] = (side == 1) ? W[idx] : W[e * NB + i];
        }
        double bv[AV * NB / 256];
#pragma unroll
        for (int it = 0; it < AV * NB / 256; ++it) {
            const int idx = tid + 256 * it;
            if (side == 1) {
                const int v = idx >> 6, c = idx & 63;
                bv[it] = ld_res(B + (int64_t)(v0 + min(v, nv - 1)) * ldb + min(c, nb - 1));
            } else {
                const int a = idx >> 4, v = idx & 15;
                bv[it] = ld_res(B + (int64_t)min(a, nb - 1) * ldb + v0 + min(v, nv - 1));
            }
        }
#pragma unroll
        for (int it = 0; it < NB * NB / 256; ++it) {
            const int idx = tid + 256 * it;
            Ws[idx >> 6][idx & 63] = wv[it];
        }
        // Bs[v][s]: element s of vector v (row of B on the right, column on the left)
#pragma unroll
        for (int it = 0; it < AV * NB / 256; ++it) {
            const int idx = tid + 256 * it;
            if (side == 1) {
                const int v = idx >> 6, c = idx & 63;
                Bs[v][c] = (v < nv && c < nb) ? bv[it] : 0.0;
            } else {
                const int a = idx >> 4, v = idx & 15;
                Bs[v][a] = (a < nb && v < nv) ? bv[it] : 0.0;
            }
        }
    }
    __syncthreads();
    // thread: vector v = tid >> 4, outputs e = (tid & 15) + 16 q
    const int v = tid >> 4, e0 = tid & 15;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int s = 0; s < NB; ++s) {
        const double bv = Bs[v][s];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = fma(bv, Ws[s][e0 + 16 * q], acc[q]);
        if (BIG) {
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = mod_red(acc[q], P, PI);
        }
    }
    if (v < nv) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = e0 + 16 * q;
            if (e < nb) {
                T* dst = (side == 1) ? B + (int64_t)(v0 + v) * ldb + e : B + (int64_t)e * ldb + v0 + v;
                st_res(dst, mod_red(acc[q], P, PI));
            }
        }
    }
}

template <typename T, bool BIG>
__global__ __launch_bounds__(256) void tri_apply_kernel(int side, int nb, const double* __restrict__ W,
                                                        T* __restrict__ B, int64_t ldb, int other,
                                                        ModP mp, const int* __restrict__ guard,
                                                        int expect)
{
    if (guard && *guard != expect) return;  // launched ahead of a pivot count that differs
    tri_apply_block<T, BIG>(blockIdx.x, side, nb, W, B, ldb, other, mp);
}

// Whole right solve X = B U^{-1} for an upper U of order n <= 512 (n a
// multiple of 64) whose 64 x 64 diagonal-block inverses W are known:
// one workgroup per RV rows of B (16 for n <= 512, 8 for n <= 1024, so that
// the rows fit in LDS), left-looking over the 64-column blocks,
//     X_l = (B_l - sum_{j<l} X_j U_jl) W_l,
// with the rows of B in LDS and each 64 x 64 tile of U (or W) staged
// through LDS.  It replaces the n/64 leaf products and n/64 - 1 recursion
// products of Algorithm 2 by one launch.  Each thread computes QN of the
// RV x 64 outputs of a block; a 64-term sum of canonical products is exact
// for p < 2^23.5 and is reduced after every tile (BIG: after every term).
constexpr int SLAB_LIMIT = 512;  // largest order sent to the slab kernels (capacity: 1024)

template <typename T, bool BIG, int RV>
__global__ __launch_bounds__(256) void tri_slab_kernel(int n, const T* __restrict__ U, int64_t ldu,
                                                       const double* __restrict__ W,
                                                       T* __restrict__ B, int64_t ldb, int rows,
                                                       ModP mp)
{
    constexpr int NMAX = 8192 / RV;          // 512 or 1024 columns
    constexpr int TPR = 256 / RV;            // threads per row
    constexpr int QN = NB / TPR;             // outputs per thread per block
    __shared__ double Bs[RV][NMAX + 1];
    __shared__ double Ts[NB][NB + 1];
    const int tid = threadIdx.x;
    const double P = mp.p, PI = mp.pinv;
    const int v0 = blockIdx.x * RV;
    const int nv = min(RV, rows - v0);
    const int v = tid / TPR, e0 = tid % TPR;  // row v, outputs e0 + TPR q
    // the rows of B (addresses clamped; rows past the end are zeros)
    for (int idx = tid; idx < RV * n; idx += 256) {
        const int r = idx / n, c = idx % n;
        const double x = ld_res(B + (int64_t)(v0 + min(r, nv - 1)) * ldb + c);
        Bs[r][c] = (r < nv) ? x : 0.0;
    }
    // Tiles in order: for each block l, U_0l .. U_(l-1)l, then W_l.  The
    // next tile's 16 values per thread are loaded into registers while the
    // current one is used.
    const int nbk = n / NB;
    constexpr int TV = NB * NB / 256;
    auto fetch = [&](int l, int j, double (&r)[TV]) {
        if (j < l) {
#pragma unroll
            for (int it = 0; it < TV; ++it) {
                const int idx = tid + 256 * it;
                r[it] = ld_res(U + (int64_t)(NB * j + (idx >> 6)) * ldu + NB * l + (idx & 63));
            }
        } else {
            const double* Wl = W + (size_t)l * NB * NB;
#pragma unroll
            for (int it = 0; it < TV; ++it) r[it] = Wl[tid + 256 * it];
        }
    };
    auto stage = [&](const double (&r)[TV]) {
        __syncthreads();  // every read of the previous tile is done
#pragma unroll
        for (int it = 0; it < TV; ++it) {
            const int idx = tid + 256 * it;
            Ts[idx >> 6][idx & 63] = r[it];
        }
    };
    double cur[TV];
    fetch(0, 0, cur);
    // the rows of B were loaded by other threads than the ones that update
    // them below (block 0 has no tile stage before its update)
    __syncthreads();
    for (int l = 0; l < nbk; ++l) {
        double acc[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) acc[q] = 0.0;
        for (int j = 0; j < l; ++j) {
            stage(cur);
            __syncthreads();
            fetch(l, j + 1, cur);
            double part[QN];
#pragma unroll
            for (int q = 0; q < QN; ++q) part[q] = 0.0;
#pragma unroll 8
            for (int s = 0; s < NB; ++s) {
                const double xv = Bs[v][NB * j + s];
#pragma unroll
                for (int q = 0; q < QN; ++q) {
                    part[q] = fma(xv, Ts[s][e0 + TPR * q], part[q]);
                    if (BIG) part[q] = mod_red(part[q], P, PI);
                }
            }
#pragma unroll
            for (int q = 0; q < QN; ++q) acc[q] = mod_red(acc[q] + mod_red(part[q], P, PI), P, PI);
        }
        // B_l - sum (own outputs), then the W_l product
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const double b = Bs[v][NB * l + e0 + TPR * q] - acc[q];
            Bs[v][NB * l + e0 + TPR * q] = (b < 0.0) ? b + P : b;
        }
        stage(cur);
        __syncthreads();
        if (l + 1 < nbk) fetch(l + 1, 0, cur);
        double x[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) x[q] = 0.0;
#pragma unroll 8
        for (int s = 0; s < NB; ++s) {
            const double bv = Bs[v][NB * l + s];
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                x[q] = fma(bv, Ts[s][e0 + TPR * q], x[q]);
                if (BIG) x[q] = mod_red(x[q], P, PI);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QN; ++q) Bs[v][NB * l + e0 + TPR * q] = mod_red(x[q], P, PI);
    }
    __syncthreads();
    for (int idx = tid; idx < RV * n; idx += 256) {
        const int r = idx / n, c = idx % n;
        if (r < nv) st_res(B + (int64_t)(v0 + r) * ldb + c, Bs[r][c]);
    }
}

// The same solve on the FP64 matrix cores, for p < 2^23.5 (a 64-term sum of
// canonical products is exact).  One workgroup per 16 rows of B; wave w owns
// columns 16w..16w+15 of every 64-column block and forms its 16 x 16 part of
// a tile product with 16 v_mfma_f64_16x16x4f64 (K = 4 each).  The U and W
// tiles go from global memory (every workgroup reads the same ones, so they
// stay in L2) straight into the B operand, one tile ahead of use.  Solved
// columns are kept in LDS in A-operand order, entry [s][lane] holding
// X[lane % 16][4s + lane / 16], so that an operand read is one contiguous
// 512-byte row; B_l - sum_j X_j U_jl is exchanged the same way before its
// product with W_l.  Two barriers per 64-column block instead of two per
// tile, and no LDS traffic for U.

template <typename T, int NMAXC>
__global__ __launch_bounds__(256) void tri_slab_mfma_kernel(int n, const T* __restrict__ U, int64_t ldu,
                                                            const double* __restrict__ W,
                                                            T* __restrict__ B, int64_t ldb, int rows,
                                                            ModP mp)
{
    __shared__ double Xa[NMAXC / 4][64];
    __shared__ double Ea[NB / 4][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int hi = lane >> 4, lo = lane & 15;
    const double P = mp.p, PI = mp.pinv;
    const int v0 = blockIdx.x * 16;
    const int nbk = n / NB;
    // Result layout: this lane holds rows v0 + hi + 4e (e = 0..3) of column
    // 16w + lo of a block (rows past the end are clamped and not stored).
    int64_t roff[4];
    bool rok[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = v0 + hi + 4 * e;
        rok[e] = r < rows;
        roff[e] = (int64_t)min(r, rows - 1) * ldb;
    }
    // ... and its place in A-operand order: slot 4w + lo/4, lane hi + 4e + 16 (lo % 4)
    const int es = 4 * w + (lo >> 2);
    const int el = hi + 16 * (lo & 3);
    // Tile stream: for each block l, U_0l .. U_(l-1)l, then W_l; this lane's
    // B-operand entries are rows 4ks + hi, column 16w + lo of the tile.
    auto fetch = [&](int l, int j, double (&r)[16]) {
        if (j < l) {
            const T* src = U + (int64_t)(NB * j + hi) * ldu + NB * l + 16 * w + lo;
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) r[ks] = ld_res(src + (int64_t)(4 * ks) * ldu);
        } else {
            const double* src = W + (size_t)l * NB * NB + hi * NB + 16 * w + lo;
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) r[ks] = src[4 * ks * NB];
        }
    };
    double cur[16], nxt[16];
    fetch(0, 0, cur);
    for (int l = 0; l < nbk; ++l) {
        const int col = NB * l + 16 * w + lo;
        double b[4], tot[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            b[e] = ld_res(B + roff[e] + col);
            tot[e] = 0.0;
        }
        for (int j = 0; j < l; ++j) {
            fetch(l, j + 1, nxt);
            v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < 16; ++ks)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Xa[16 * j + ks][lane], cur[ks], acc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) tot[e] += mod_red(acc[e], P, PI);
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) cur[ks] = nxt[ks];
        }
        if (l + 1 < nbk) fetch(l + 1, 0, nxt);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double t = b[e] - mod_red(tot[e], P, PI);
            Ea[es][el + 4 * e] = (t < 0.0) ? t + P : t;
        }
        __syncthreads();
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ea[ks][lane], cur[ks], acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double x = mod_red(acc[e], P, PI);
            if (rok[e]) st_res(B + roff[e] + col, x);
            Xa[16 * l + es][el + 4 * e] = x;
        }
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) cur[ks] = nxt[ks];
        __syncthreads();
    }
}

// The same solve for p <= 2^16 on the INT8 matrix cores.  A residue x is
// split into two signed bytes x = 256 h + l (x taken in [-(p - 32640), 32639]
// first), and a 64-term product X U becomes four v_mfma_i32_16x16x64_i8
// (h h, the two cross terms sharing one accumulator, l l) instead of sixteen
// FP64 MFMAs, so the chain of dependent products that bounds the solve is
// about sixteen times shorter.  The INT32 sums of all the tiles of a block
// stay exact (at most 8 tiles of 64 terms, each below 2^15 in magnitude) and
// are recombined and reduced once per block.  One workgroup per 16 rows of
// B; wave w owns columns 16w..16w+15 of every 64-column block.  The solved
// blocks live in LDS as limb bytes in A-operand order ([row][k]); the U and
// W tiles stream from global memory as B operands (16 consecutive k of one
// column per lane) through three register buffers with identical loads in
// every step, so no use waits for a later fetch.  int64 storage only.
__device__ __forceinline__ void slab_limbs(int x, int p, int& h, int& l)
{
    const int xc = (x <= 32639) ? x : x - p;
    h = (xc + 128) >> 8;
    l = xc - 256 * h;
}

__device__ __forceinline__ int slab_byte4(const int* b)
{
    return (int)((unsigned)(b[0] & 0xff) | ((unsigned)(b[1] & 0xff) << 8) |
                 ((unsigned)(b[2] & 0xff) << 16) | ((unsigned)(b[3] & 0xff) << 24));
}

constexpr int SXR = 80;  // LDS row stride of the limb blocks, bytes (conflict-free 16-byte reads)

template <int NMAXC>
__device__ __forceinline__ void tri_slab_i8_block(int blk, int n, const int64_t* __restrict__ U,
                                                  int64_t ldu, const double* __restrict__ W,
                                                  int64_t* __restrict__ B, int64_t ldb, int rows, ModP mp)
{
    typedef int v4i_t __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) int8_t Xq[2][NMAXC / NB][16 * SXR];
    __shared__ __attribute__((aligned(16))) int8_t Eq[2][16 * SXR];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int hi = lane >> 4, lo = lane & 15;
    const int ip = (int)mp.p;
    const double P = mp.p, PI = mp.pinv;
    const int v0 = blk * 16;
    const int nbk = n / NB;
    // Result layout (v_mfma_i32_16x16x64_i8): rows 4 hi + e (e < 4), column
    // 16 w + lo of a block; rows past the end are clamped and not stored.
    int64_t roff[4];
    bool rok[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = v0 + 4 * hi + e;
        rok[e] = r < rows;
        roff[e] = (int64_t)min(r, rows - 1) * ldb;
    }
    // Tile stream: for each block l, U_0l .. U_(l-1)l, then W_l.  This lane's
    // B-operand entries are rows 16 hi + t (t < 16) of the tile, column
    // 16 w + lo; the B entries of the tile's block come along.  Registers hold
    // raw 64-bit words (a U residue, or the bits of a W double).
    struct Tile {
        long long r[16];
        long long bv[4];
    };
    int fl = 0, fj = 0;  // next tile to fetch
    auto fetch_next = [&](Tile& tl) {
        const int l = min(fl, nbk - 1);
        const int j = (fl < nbk) ? fj : l;
        const bool isu = j < l;
        const long long* usrc = reinterpret_cast<const long long*>(U) + (int64_t)(NB * j + 16 * hi) * ldu +
                                NB * l + 16 * w + lo;
        const long long* wsrc = reinterpret_cast<const long long*>(W) + (size_t)l * NB * NB +
                                16 * hi * NB + 16 * w + lo;
        const long long* src = isu ? usrc : wsrc;
        const int64_t st = isu ? ldu : (int64_t)NB;
#pragma unroll
        for (int t = 0; t < 16; ++t) tl.r[t] = src[t * st];
#pragma unroll
        for (int e = 0; e < 4; ++e) tl.bv[e] = B[roff[e] + NB * l + 16 * w + lo];
        if (fl < nbk && ++fj > fl) {
            ++fl;
            fj = 0;
        }
    };
    // The two limb operands of a tile (W entries may be negative: made canonical).
    auto operand = [&](const Tile& c, bool isw, v4i_t& oh, v4i_t& ol) {
        int hb[16], lb[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            int x = isw ? (int)__longlong_as_double(c.r[t]) : (int)c.r[t];
            x = (x < 0) ? x + ip : x;
            slab_limbs(x, ip, hb[t], lb[t]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            oh[q] = slab_byte4(hb + 4 * q);
            ol[q] = slab_byte4(lb + 4 * q);
        }
    };
    auto recombine = [&](const v4i_t (&a)[3], int e) {
        return mod_red(65536.0 * (double)a[0][e] + 256.0 * (double)a[1][e] + (double)a[2][e], P, PI);
    };
    // this lane's bytes of the limb blocks: rows 4 hi + e, column 16 w + lo
    auto put = [&](int8_t* hbase, int8_t* lbase, int e, int x) {
        int h, l;
        slab_limbs(x, ip, h, l);
        hbase[(4 * hi + e) * SXR + 16 * w + lo] = (int8_t)h;
        lbase[(4 * hi + e) * SXR + 16 * w + lo] = (int8_t)l;
    };

    const int ntiles = nbk * (nbk + 1) / 2;
    Tile buf0, buf1, buf2;
    fetch_next(buf0);
    fetch_next(buf1);
    int l = 0, j = 0;  // tile being used: U_jl (j < l) or W_l (j == l)
    v4i_t acc[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) acc[s] = v4i_t{0, 0, 0, 0};
    // Every step fetches (also the padding steps that complete the last group
    // of three, which do nothing else), so all paths issue the same loads.
    auto step = [&](const Tile& cur, Tile& pf, bool live) {
        fetch_next(pf);
        if (!live) {
        } else if (j < l) {
            v4i_t uh, ul;
            operand(cur, false, uh, ul);
            const v4i_t xh = *reinterpret_cast<const v4i_t*>(&Xq[0][j][lo * SXR + 16 * hi]);
            const v4i_t xl = *reinterpret_cast<const v4i_t*>(&Xq[1][j][lo * SXR + 16 * hi]);
            acc[0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xh, uh, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xh, ul, acc[1], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xl, uh, acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xl, ul, acc[2], 0, 0, 0);
            ++j;
        } else {
            // E = B_l - sum_j X_j U_jl, exchanged through LDS as limb bytes
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double tt = (double)(int)cur.bv[e] - recombine(acc, e);
                put(Eq[0], Eq[1], e, (int)((tt < 0.0) ? tt + P : tt));
            }
            __syncthreads();
            const v4i_t eh = *reinterpret_cast<const v4i_t*>(&Eq[0][lo * SXR + 16 * hi]);
            const v4i_t el = *reinterpret_cast<const v4i_t*>(&Eq[1][lo * SXR + 16 * hi]);
            v4i_t wh, wl;
            operand(cur, true, wh, wl);
            v4i_t xa[3];
            xa[0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(eh, wh, v4i_t{0, 0, 0, 0}, 0, 0, 0);
            xa[1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(eh, wl, v4i_t{0, 0, 0, 0}, 0, 0, 0);
            xa[1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(el, wh, xa[1], 0, 0, 0);
            xa[2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(el, wl, v4i_t{0, 0, 0, 0}, 0, 0, 0);
            const int col = NB * l + 16 * w + lo;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double x = recombine(xa, e);
                if (rok[e]) B[roff[e] + col] = (int64_t)(int)x;
                put(Xq[0][l], Xq[1][l], e, (int)x);
            }
#pragma unroll
            for (int s = 0; s < 3; ++s) acc[s] = v4i_t{0, 0, 0, 0};
            __syncthreads();
            ++l;
            j = 0;
        }
    };
    for (int t = 0; t < ntiles; t += 3) {
        step(buf0, buf2, true);
        step(buf1, buf0, t + 1 < ntiles);
        step(buf2, buf1, t + 2 < ntiles);
    }
}

// The left apply B <- W B (W 64 x 64, B 64 x other, in place) for p <= 2^16
// on the INT8 matrix cores: workgroup blk owns 16 columns of B, wave w forms
// rows 16w..16w+15 of them with four v_mfma_i32_16x16x64_i8 on the limbs.
// Operands come straight from global memory (a W row and a B column of 16
// entries per lane), so no LDS is needed; a barrier keeps every wave's reads
// of the old B ahead of the stores.
__device__ __forceinline__ void tri_apply_i8_block(int blk, const double* __restrict__ W,
                                                   int64_t* __restrict__ B, int64_t ldb, int other,
                                                   ModP mp)
{
    typedef int v4i_t __attribute__((ext_vector_type(4)));
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int hi = lane >> 4, lo = lane & 15;
    const int ip = (int)mp.p;
    const double P = mp.p, PI = mp.pinv;
    const int col = blk * 16 + lo;
    const int ccol = min(col, other - 1);
    double wv[16];
    int bv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        wv[t] = W[(16 * w + lo) * NB + 16 * hi + t];
        bv[t] = (int)B[(int64_t)(16 * hi + t) * ldb + ccol];
    }
    int ah[16], al[16], bh[16], bl[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        int x = (int)wv[t];
        x = (x < 0) ? x + ip : x;
        slab_limbs(x, ip, ah[t], al[t]);
        slab_limbs(bv[t], ip, bh[t], bl[t]);
    }
    v4i_t oah, oal, obh, obl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        oah[q] = slab_byte4(ah + 4 * q);
        oal[q] = slab_byte4(al + 4 * q);
        obh[q] = slab_byte4(bh + 4 * q);
        obl[q] = slab_byte4(bl + 4 * q);
    }
    const v4i_t z = {0, 0, 0, 0};
    const v4i_t s0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(oah, obh, z, 0, 0, 0);
    v4i_t s1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(oah, obl, z, 0, 0, 0);
    s1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(oal, obh, s1, 0, 0, 0);
    const v4i_t s2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(oal, obl, z, 0, 0, 0);
    double x[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
        x[e] = mod_red(65536.0 * (double)s0[e] + 256.0 * (double)s1[e] + (double)s2[e], P, PI);
    __syncthreads();  // every wave has read the old B columns
    if (col < other) {
#pragma unroll
        for (int e = 0; e < 4; ++e) B[(int64_t)(16 * w + 4 * hi + e) * ldb + col] = (int64_t)(int)x[e];
    }
}

template <int NMAXC>
__global__ __launch_bounds__(256) void tri_slab_i8_kernel(int n, const int64_t* __restrict__ U,
                                                          int64_t ldu, const double* __restrict__ W,
                                                          int64_t* __restrict__ B, int64_t ldb, int rows,
                                                          ModP mp)
{
    tri_slab_i8_block<NMAXC>(blockIdx.x, n, U, ldu, W, B, ldb, rows, mp);
}

// The slab solve and an independent left apply B2 <- W2 B2 (a 64-row leaf's
// solve of its columns right of its pivots, which the solve's rows and
// columns do not touch) in one launch: the first workgroups solve, the
// others apply.  Saves the launch gap between them and lets them overlap.
template <int NMAXC>
__global__ __launch_bounds__(256) void slab_apply_kernel(int n, const int64_t* __restrict__ U, int64_t ldu,
                                                         const double* __restrict__ W,
                                                         int64_t* __restrict__ B, int64_t ldb, int rows,
                                                         ModP mp, int nslab, const double* __restrict__ W2,
                                                         int64_t* __restrict__ B2, int64_t ldb2, int other2)
{
    if ((int)blockIdx.x < nslab)
        tri_slab_i8_block<NMAXC>(blockIdx.x, n, U, ldu, W, B, ldb, rows, mp);
    else
        tri_apply_i8_block(blockIdx.x - nslab, W2, B2, ldb2, other2, mp);
}

// Two-leaf node whose first leaf (rows 0..63, the pivots in columns 0..63)
// was decided as a full block with no column exchange, and whose second leaf
// is the 64 rows below.  The leaf's solve of its other columns, Algorithm 6's
// G (already formed in place by the window) and the Schur update are all
// column-parallel then, so one launch does them:  per 32-column block c
// right of the pivots,  U12_c = L^{-1} T_c  (top rows) and
// H_c = B_c - G U12_c  (bottom rows), on the FP64 matrix cores.  Wave w
// forms rows 16w..16w+15 of both products; T_c and U12_c pass through LDS as
// B operands, L^{-1} and G rows are read from global memory (every
// workgroup reads the same ones) as A operands.  A 64-term sum of canonical
// products is exact for p <= kExact64.  Does nothing unless the window
// found 64 pivots and exchanged no column.
constexpr int PC = 32;  // columns per workgroup

template <typename T>
__global__ __launch_bounds__(256) void pair_update_kernel(T* __restrict__ A, int64_t lda, int N,
                                                          const double* __restrict__ WL,
                                                          const int* __restrict__ guard, ModP mp)
{
    __shared__ double Ts[NB][PC + 1];
    __shared__ double Us[NB][PC + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, hi = lane >> 4, lo = lane & 15;
    const double P = mp.p, PI = mp.pinv;
    const int c0 = NB + PC * blockIdx.x;
    T* Bm = A + (int64_t)NB * lda;
    // (the guard is loaded with the operands and checked before anything is
    // written)
    const int g0 = guard[0], g1 = guard[kSwapWord];
    // T_c (columns past N clamped; not stored), B_c rows of this wave in
    // result layout, and the A operands: rows 16w.. of L^{-1} and G
    double tv[NB * PC / 256];
#pragma unroll
    for (int it = 0; it < NB * PC / 256; ++it) {
        const int idx = tid + 256 * it, r = idx / PC, cc = idx % PC;
        tv[it] = ld_res(A + (int64_t)r * lda + min(c0 + cc, N - 1));
    }
    double bv[2][4], wl[16], gv[16];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            bv[ct][e] = ld_res(Bm + (int64_t)(16 * w + hi + 4 * e) * lda + min(c0 + 16 * ct + lo, N - 1));
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
        wl[ks] = WL[(16 * w + lo) * NB + 4 * ks + hi];
        gv[ks] = ld_res(Bm + (int64_t)(16 * w + lo) * lda + 4 * ks + hi);
    }
    if (g0 != kLeafRows || g1 != 0) return;
#pragma unroll
    for (int it = 0; it < NB * PC / 256; ++it) {
        const int idx = tid + 256 * it;
        Ts[idx / PC][idx % PC] = tv[it];
    }
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wl[ks], Ts[4 * ks + hi][16 * ct + lo], acc, 0, 0, 0);
        const int c = c0 + 16 * ct + lo;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double u = mod_red(acc[e], P, PI);
            Us[16 * w + hi + 4 * e][16 * ct + lo] = u;
            if (c < N) st_res(A + (int64_t)(16 * w + hi + 4 * e) * lda + c, u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(gv[ks], Us[4 * ks + hi][16 * ct + lo], acc, 0, 0, 0);
        const int c = c0 + 16 * ct + lo;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double h = bv[ct][e] - mod_red(acc[e], P, PI);
            if (c < N) st_res(Bm + (int64_t)(16 * w + hi + 4 * e) * lda + c, (h < 0.0) ? h + P : h);
        }
    }
}

// The same two-leaf update for p <= 2^16 on the INT8 matrix cores (int64
// storage): each 64-term product of a 16 x 16 tile is four
// v_mfma_i32_16x16x64_i8 on the limbs.  Wave w forms rows 16w..16w+15 of
// U12 and of H for the workgroup's 32 columns; L^{-1} and G rows and the T
// columns are read from global memory straight into operands, and U12 goes
// through LDS as limb bytes in B-operand order ([column][k]).
template <typename T>
__global__ __launch_bounds__(256) void pair_update_i8_kernel(T* __restrict__ A, int64_t lda, int N,
                                                             const double* __restrict__ WL,
                                                             const int* __restrict__ guard, ModP mp)
{
    typedef int v4i_t __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) int8_t Uq[2][PC * SXR];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, hi = lane >> 4, lo = lane & 15;
    const int ip = (int)mp.p;
    const double P = mp.p, PI = mp.pinv;
    const int c0 = NB + PC * blockIdx.x;
    T* Bm = A + (int64_t)NB * lda;
    // every load first (columns past N clamped; not stored), the guard
    // checked before anything is written
    const int g0 = guard[0], g1 = guard[kSwapWord];
    double wl[16];
    int gv[16], tv[2][16], bv[2][4];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        wl[t] = WL[(16 * w + lo) * NB + 16 * hi + t];
        gv[t] = (int)Bm[(int64_t)(16 * w + lo) * lda + 16 * hi + t];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
            tv[ct][t] = (int)A[(int64_t)(16 * hi + t) * lda + min(c0 + 16 * ct + lo, N - 1)];
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            bv[ct][e] = (int)Bm[(int64_t)(16 * w + 4 * hi + e) * lda + min(c0 + 16 * ct + lo, N - 1)];
    if (g0 != kLeafRows || g1 != 0) return;
    auto split = [&](const int* x, v4i_t& oh, v4i_t& ol) {
        int h[16], l[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) slab_limbs(x[t], ip, h[t], l[t]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            oh[q] = slab_byte4(h + 4 * q);
            ol[q] = slab_byte4(l + 4 * q);
        }
    };
    v4i_t lh, ll, gh, gl;
    {
        int x[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const int v = (int)wl[t];
            x[t] = (v < 0) ? v + ip : v;
        }
        split(x, lh, ll);
        split(gv, gh, gl);
    }
    const v4i_t z = {0, 0, 0, 0};
    // U12 = L^{-1} T
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        v4i_t th, tl;
        split(tv[ct], th, tl);
        const v4i_t s0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(lh, th, z, 0, 0, 0);
        v4i_t s1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(lh, tl, z, 0, 0, 0);
        s1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(ll, th, s1, 0, 0, 0);
        const v4i_t s2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(ll, tl, z, 0, 0, 0);
        const int c = c0 + 16 * ct + lo;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int u = (int)mod_red(65536.0 * (double)s0[e] + 256.0 * (double)s1[e] + (double)s2[e], P, PI);
            const int row = 16 * w + 4 * hi + e;
            int h, l;
            slab_limbs(u, ip, h, l);
            Uq[0][(16 * ct + lo) * SXR + row] = (int8_t)h;
            Uq[1][(16 * ct + lo) * SXR + row] = (int8_t)l;
            if (c < N) A[(int64_t)row * lda + c] = (T)u;
        }
    }
    __syncthreads();
    // H = B - G U12
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        const v4i_t uh = *reinterpret_cast<const v4i_t*>(&Uq[0][(16 * ct + lo) * SXR + 16 * hi]);
        const v4i_t ul = *reinterpret_cast<const v4i_t*>(&Uq[1][(16 * ct + lo) * SXR + 16 * hi]);
        const v4i_t s0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(gh, uh, z, 0, 0, 0);
        v4i_t s1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(gh, ul, z, 0, 0, 0);
        s1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(gl, uh, s1, 0, 0, 0);
        const v4i_t s2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(gl, ul, z, 0, 0, 0);
        const int c = c0 + 16 * ct + lo;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double g = mod_red(65536.0 * (double)s0[e] + 256.0 * (double)s1[e] + (double)s2[e], P, PI);
            const double h = (double)bv[ct][e] - g;
            if (c < N) Bm[(int64_t)(16 * w + 4 * hi + e) * lda + c] = (T)(int)((h < 0.0) ? h + P : h);
        }
    }
}

// [N\T] <- T N on an nb x nb block (nb <= 64): T unit upper (strict upper
// part stored), N lower with its diagonal (TRULM's leaf); with LU, the
// other product of the same storage, [L\U] <- L U with L lower with its
// diagonal and U unit upper (TRLUM's leaf).  Thread j holds column j of the
// right factor; used for p > kExact64 (every product reduced as it is
// added).
template <typename T, bool BIG, bool LU>
__global__ __launch_bounds__(NB) void trulm_leaf_kernel(int nb, T* __restrict__ A, int64_t lda, ModP mp)
{
    __shared__ double Tu[NB][NB + 1];
    const int j = threadIdx.x;
    const double P = mp.p, PI = mp.pinv;
    for (int idx = j; idx < NB * NB; idx += NB) {
        int i = idx >> 6, s = idx & 63;
        double v = 0.0;
        if (i < nb && s < nb) {
            if (LU) v = (s <= i) ? ld_res(A + (int64_t)i * lda + s) : 0.0;
            else v = (s > i) ? ld_res(A + (int64_t)i * lda + s) : (s == i ? 1.0 : 0.0);
        }
        Tu[i][s] = v;
    }
    double ncol[NB];
#pragma unroll
    for (int s = 0; s < NB; ++s) {
        if (LU)
            ncol[s] = (j < nb && s < nb && s < j) ? ld_res(A + (int64_t)s * lda + j) : (s == j ? 1.0 : 0.0);
        else
            ncol[s] = (j < nb && s < nb && s >= j) ? ld_res(A + (int64_t)s * lda + j) : 0.0;
    }
    __syncthreads();
    double x[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) x[q] = 0.0;
    for (int i = 0; i < NB; ++i) {
        double acc = 0.0;
        const int s0 = LU ? 0 : i, s1 = LU ? i + 1 : NB;
        for (int s = s0; s < s1; ++s) {
            double nv = 0.0;
#pragma unroll
            for (int q = 0; q < NB; ++q) nv = (q == s) ? ncol[q] : nv;
            acc = BIG ? mod_red(fma(Tu[i][s], nv, acc), P, PI) : fma(Tu[i][s], nv, acc);
        }
        acc = mod_red(acc, P, PI);
#pragma unroll
        for (int q = 0; q < NB; ++q) x[q] = (q == i) ? acc : x[q];
    }
    __syncthreads();  // every read of the block is done before it is overwritten
    if (j < nb) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
            if (i < nb) st_res(A + (int64_t)i * lda + j, x[i]);
    }
}

// The same products on the FP64 matrix cores for p <= kExact64: the left
// factor (T unit upper, identity-padded; with LU, L lower with its
// diagonal) and the right one (N lower with its diagonal; with LU, U unit
// upper) are staged in LDS as dense 64 x 64 triangles, and wave w forms
// rows 16w..16w+15 of the product with 64 v_mfma_f64_16x16x4f64 (a sum of
// at most 64 canonical products is exact).  Every read of the block
// precedes the barrier before the block is overwritten.
template <typename T, bool LU>
__global__ __launch_bounds__(256) void trulm_mfma_kernel(int nb, T* __restrict__ A, int64_t lda, ModP mp)
{
    __shared__ double Tu[NB][NB + 1];
    __shared__ double Nl[NB][NB + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, hi = lane >> 4, lo = lane & 15;
    const double P = mp.p, PI = mp.pinv;
    double ev[NB * NB / 256];
#pragma unroll
    for (int it = 0; it < NB * NB / 256; ++it) {
        const int idx = tid + 256 * it, i = idx >> 6, s = idx & 63;
        ev[it] = ld_res(A + (int64_t)min(i, nb - 1) * lda + min(s, nb - 1));
    }
#pragma unroll
    for (int it = 0; it < NB * NB / 256; ++it) {
        const int idx = tid + 256 * it, i = idx >> 6, s = idx & 63;
        const bool in = i < nb && s < nb;
        const double up = (i == s) ? 1.0 : ((in && s > i) ? ev[it] : 0.0);
        const double lo_ = (in && s <= i) ? ev[it] : 0.0;
        Tu[i][s] = LU ? lo_ : up;
        Nl[i][s] = LU ? up : lo_;
    }
    __syncthreads();
    v4d acc[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
        const double a = Tu[16 * w + lo][4 * ks + hi];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Nl[4 * ks + hi][16 * ct + lo], acc[ct], 0, 0, 0);
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 16 * w + hi + 4 * e, j = 16 * ct + lo;
            if (i < nb && j < nb) st_res(A + (int64_t)i * lda + j, mod_red(acc[ct][e], P, PI));
        }
}

template <typename T>
__global__ void negate_kernel(T* __restrict__ B, int64_t ldb, int rows, int cols, double P)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (c < cols) {
        T* e = B + (int64_t)r * ldb + c;
        double v = ld_res(e);
        st_res(e, v == 0.0 ? 0.0 : P - v);
    }
}

inline bool big_prime(const ModP& mp) { return mp.p > kExact64; }

}  // namespace

template <typename T>
void launch_diag_prep(hipStream_t s, T* A, int64_t lda, int n, int uplo, int unit, int mode,
                      double* W, ModP mp, const int* guard, int expect)
{
    if (n <= 0) return;
    const int nblk = (mode == 2) ? 1 : (n + NB - 1) / NB;
    if (big_prime(mp))
        hipLaunchKernelGGL((diag_prep_kernel<T, true>), dim3(nblk), dim3(256), 0, s, A, lda, n, uplo,
                           unit, mode, W, mp, (T*)nullptr, 0, 0, (double*)nullptr, guard, expect);
    else
        hipLaunchKernelGGL((diag_prep_kernel<T, false>), dim3(nblk), dim3(256), 0, s, A, lda, n, uplo,
                           unit, mode, W, mp, (T*)nullptr, 0, 0, (double*)nullptr, guard, expect);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_diag_prep2(hipStream_t s, T* A, int64_t lda, int n, int uplo, int unit, double* W,
                       T* A2, int uplo2, int unit2, double* W2, ModP mp, const int* guard, int expect)
{
    if (n <= 0) return launch_diag_prep<T>(s, A2, lda, NB, uplo2, unit2, 0, W2, mp, guard, expect);
    const int nblk = (n + NB - 1) / NB + 1;
    if (big_prime(mp))
        hipLaunchKernelGGL((diag_prep_kernel<T, true>), dim3(nblk), dim3(256), 0, s, A, lda, n, uplo,
                           unit, 0, W, mp, A2, uplo2, unit2, W2, guard, expect);
    else
        hipLaunchKernelGGL((diag_prep_kernel<T, false>), dim3(nblk), dim3(256), 0, s, A, lda, n, uplo,
                           unit, 0, W, mp, A2, uplo2, unit2, W2, guard, expect);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_tri_apply(hipStream_t s, int side, int nb, const double* W, T* B, int64_t ldb, int other,
                      ModP mp, const int* guard, int expect)
{
    if (nb <= 0 || other <= 0) return;
    dim3 grid((other + AV - 1) / AV);
    if (big_prime(mp))
        hipLaunchKernelGGL((tri_apply_kernel<T, true>), grid, dim3(256), 0, s, side, nb, W, B, ldb,
                           other, mp, guard, expect);
    else
        hipLaunchKernelGGL((tri_apply_kernel<T, false>), grid, dim3(256), 0, s, side, nb, W, B, ldb,
                           other, mp, guard, expect);
    CUP_HIP(hipGetLastError());
}

template <typename T>
bool launch_tri_slab(hipStream_t s, int n, const T* U, int64_t ldu, const double* W, T* B,
                     int64_t ldb, int rows, ModP mp, bool int8_mfma, const LeftApply* carry,
                     bool* carried)
{
    if (carried) *carried = false;
    if (n <= 0 || n > SLAB_LIMIT || n % NB != 0 || rows <= 0) return false;
    const bool big = big_prime(mp);
    if constexpr (sizeof(T) == sizeof(int64_t)) {
        if (int8_mfma && mp.p <= 65536.0) {
            const int nslab = (rows + 15) / 16;
            if (carry && carry->other > 0 && carried) {
                const int napply = (carry->other + 15) / 16;
                hipLaunchKernelGGL((slab_apply_kernel<SLAB_LIMIT>), dim3(nslab + napply), dim3(256), 0, s, n,
                                   U, ldu, W, B, ldb, rows, mp, nslab, carry->W,
                                   static_cast<int64_t*>(carry->B), carry->ldb, carry->other);
                *carried = true;
            } else {
                hipLaunchKernelGGL((tri_slab_i8_kernel<SLAB_LIMIT>), dim3(nslab), dim3(256), 0, s, n, U,
                                   ldu, W, B, ldb, rows, mp);
            }
            CUP_HIP(hipGetLastError());
            return true;
        }
    }
    if (!big) {
        dim3 grid((rows + 15) / 16);
        if (n <= 256)
            hipLaunchKernelGGL((tri_slab_mfma_kernel<T, 256>), grid, dim3(256), 0, s, n, U, ldu, W, B,
                               ldb, rows, mp);
        else if (n <= 512)
            hipLaunchKernelGGL((tri_slab_mfma_kernel<T, 512>), grid, dim3(256), 0, s, n, U, ldu, W, B,
                               ldb, rows, mp);
        else
            hipLaunchKernelGGL((tri_slab_mfma_kernel<T, 1024>), grid, dim3(256), 0, s, n, U, ldu, W, B,
                               ldb, rows, mp);
    } else if (n <= 512) {
        hipLaunchKernelGGL((tri_slab_kernel<T, true, 16>), dim3((rows + 15) / 16), dim3(256), 0, s, n, U,
                           ldu, W, B, ldb, rows, mp);
    } else {
        hipLaunchKernelGGL((tri_slab_kernel<T, true, 8>), dim3((rows + 7) / 8), dim3(256), 0, s, n, U,
                           ldu, W, B, ldb, rows, mp);
    }
    CUP_HIP(hipGetLastError());
    return true;
}

template <typename T>
void launch_pair_update(hipStream_t s, T* A, int64_t lda, int N, const double* WL, const int* guard,
                        ModP mp, bool int8_mfma)
{
    if (N <= NB) return;
    if constexpr (sizeof(T) == sizeof(int64_t)) {
        if (int8_mfma && mp.p <= 65536.0) {
            hipLaunchKernelGGL(pair_update_i8_kernel<T>, dim3((N - NB + PC - 1) / PC), dim3(256), 0, s, A, lda,
                               N, WL, guard, mp);
            CUP_HIP(hipGetLastError());
            return;
        }
    }
    hipLaunchKernelGGL(pair_update_kernel<T>, dim3((N - NB + PC - 1) / PC), dim3(256), 0, s, A, lda, N,
                       WL, guard, mp);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_trulm_leaf(hipStream_t s, int nb, T* A, int64_t lda, ModP mp, int64_t kred)
{
    (void)kred;
    if (nb <= 0) return;
    if (big_prime(mp))
        hipLaunchKernelGGL((trulm_leaf_kernel<T, true, false>), dim3(1), dim3(NB), 0, s, nb, A, lda, mp);
    else
        hipLaunchKernelGGL((trulm_mfma_kernel<T, false>), dim3(1), dim3(256), 0, s, nb, A, lda, mp);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_trlum_leaf(hipStream_t s, int nb, T* A, int64_t lda, ModP mp)
{
    if (nb <= 0) return;
    if (big_prime(mp))
        hipLaunchKernelGGL((trulm_leaf_kernel<T, true, true>), dim3(1), dim3(NB), 0, s, nb, A, lda, mp);
    else
        hipLaunchKernelGGL((trulm_mfma_kernel<T, true>), dim3(1), dim3(256), 0, s, nb, A, lda, mp);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_negate(hipStream_t s, T* B, int64_t ldb, int rows, int cols, ModP mp)
{
    if (rows <= 0 || cols <= 0) return;
    for (int r0 = 0; r0 < rows; r0 += 65535) {
        int rr = std::min(65535, rows - r0);
        hipLaunchKernelGGL(negate_kernel<T>, dim3((cols + 255) / 256, rr), dim3(256), 0, s,
                           B + (int64_t)r0 * ldb, ldb, rr, cols, mp.p);
        CUP_HIP(hipGetLastError());
    }
}

#define CUP_INST(T)                                                                             \
    template void launch_diag_prep<T>(hipStream_t, T*, int64_t, int, int, int, int, double*,    \
                                      ModP, const int*, int);                                   \
    template void launch_diag_prep2<T>(hipStream_t, T*, int64_t, int, int, int, double*, T*,    \
                                       int, int, double*, ModP, const int*, int);               \
    template void launch_tri_apply<T>(hipStream_t, int, int, const double*, T*, int64_t, int,   \
                                      ModP, const int*, int);                                   \
    template void launch_trulm_leaf<T>(hipStream_t, int, T*, int64_t, ModP, int64_t);           \
    template void launch_trlum_leaf<T>(hipStream_t, int, T*, int64_t, ModP);                    \
    template void launch_pair_update<T>(hipStream_t, T*, int64_t, int, const double*, const int*, \
                                        ModP, bool);                                              \
    template bool launch_tri_slab<T>(hipStream_t, int, const T*, int64_t, const double*, T*,    \
                                     int64_t, int, ModP, bool, const LeftApply*, bool*);                                       \
    template void launch_negate<T>(hipStream_t, T*, int64_t, int, int, ModP);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
