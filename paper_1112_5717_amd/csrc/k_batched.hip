// Batched CUP: many independent small matrices, each over its own prime
// (Algorithm 6 applied to every matrix of a multi-modular batch).
//
// One workgroup factors one matrix, start to finish, in a single launch.
// The recursion of Algorithm 6 visits rows top-down and, with the pivot rule
// of its base case (leftmost nonzero in the current column order), the
// decisions it takes are those of a row-by-row elimination.  The kernel
// groups rows into blocks of 4 BW (BW waves per workgroup) and, for each
// block:
//
//  1. loads the block into registers in the current column order (the
//     composition of every transposition so far, kept in LDS);
//  2. eliminates it against the t pivots found before it (left-looking): for
//     s = 0..t-1 the block's residual at position s is its entry of C, and
//     the block rows lose C(., s) times U row s; the U rows live in the
//     matrix (rows 0..t-1, positions after the diagonal) and pass through
//     LDS in double-buffered chunks of BW, the next chunk in flight while
//     the current one is used;
//  3. runs the row-by-row base case inside the block (rows whose residual is
//     already zero need no step: later pivots leave them zero): the owner
//     wave reduces the next row, finds its leftmost nonzero at positions >= t
//     with a ballot and publishes the row and its pivot in LDS; every wave
//     swaps the two positions in its rows and, fraction free, replaces each
//     later row by piv row - residual(i, t) pivot row at the positions after
//     t, so that no modular inverse is on the chain of steps.  A step touches
//     no global memory: the block's pivot rows, transpositions and profile
//     entries collect in LDS;
//  4. recovers the true values (after step t0 + d every row of the block
//     stands at Sigma_{d+1}, the product of the stored pivots so far, times
//     its true value: one scan and one Fermat inverse per lane for the whole
//     block), writes the block's C entries (and the echelon zeros) and its
//     normalised U rows, applies its transpositions to the U rows of earlier
//     blocks, and appends its entries of P and Q.
//
// Left-looking updates are not reduced one by one.  A multiplier is reduced
// lazily, to x - floor(x / p) p in [-p, 2p), and a residual absorbs
// floor((2^53 - p) / (2p (p - 1))) products of such a multiplier with a
// canonical U entry before the block is reduced again.  The base case's
// fraction-free updates round every value to (-p, p), so both of its
// products stay below p^2 and their difference below 2^53 for p < 2^26.  A
// position that has become an entry of C is never updated again, so the C
// entries are the residuals themselves (scaled by Sigma in the block's own
// columns), reduced once when the block is written back.
//
// Layout: BW waves; wave w owns block rows w + BW k (k < 4); lane l holds
// positions l + 64q (q < BQ) of those rows.  Three widths are compiled
// (BQ = 2, 4, 8: n <= 128, 256, 512) so that a narrow matrix pays for its
// own width only and leaves room for more workgroups per CU; each uses 4
// waves (blocks of 16 rows), so that two or more of its workgroups fit a
// CU's registers and LDS together.  Inner
// loops run over every register of the width without per-register or
// per-row branches: positions past n and rows past m hold zeros, which the
// updates leave zero.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "batched_tune.h"

#include "modarith.h"
#include "tri64.h"

namespace cup {

namespace {

// A workgroup of BW waves (a template parameter; 4 for every width class:
// the wider ones' registers allow two waves per SIMD at most, and with 4
// waves two or more workgroups share a CU, so that one's pivot chain
// overlaps the others' updates; 8 waves measured slower for the narrow
// classes too) factors blocks of BR = 4 BW rows and stages U rows in chunks
// of CH = BW.
constexpr int BK = 4;          // block rows per wave
constexpr int BQMAX = 8;       // position registers per lane at most (n <= 512)
constexpr int kClassWaves[3] = {4, 4, 4};  // BW of the width classes (n <= 128, <= 256, <= 512)

// x - floor(x / p) p, in [-p, 2p) for |x| < 2^53 (the quotient from the
// rounded reciprocal is off by at most one; the fma is exact).
__device__ __forceinline__ double red_lazy(double x, double p, double pinv)
{
    return fma(-floor(x * pinv), p, x);
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Inverse of a nonzero residue in (-p, p), p < 2^26: the unrolled Fermat
// chain of tri64.h.
__device__ __forceinline__ double inv_pivot(double a, double p, double pinv) { return inv_fermat26(a, p, pinv); }

// f(std::integral_constant<int, 0>), ..., f(..., Q - 1): the index reaches
// the body as a constant, so register arrays indexed by it stay in registers.
template <int Q>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void run(F&& f)
    {
        Unroll<Q - 1>::run(f);
        f(std::integral_constant<int, Q - 1>{});
    }
};
template <>
struct Unroll<0> {
    template <class F>
    __device__ __forceinline__ static void run(F&&) {}
};

struct BatchDesc {
    const int64_t* m;
    const int64_t* n;
    int64_t* const* A;
    const int64_t* lda;
    const int64_t* p;
    int64_t* rank;
    int64_t* const* P;
    int64_t* const* Q;
    int32_t* info;
    const int* order;  // processing order (largest first), or null
};

// The workgroup's shared state for one matrix (BQ position registers per
// lane: n <= 64 BQ).
template <int BQ, int BW>
struct BatchShared {
    static constexpr int NP = 64 * BQ;
    static constexpr int BR = BK * BW;  // rows per block
    static constexpr int CH = BW;       // U rows per LDS chunk of the left-looking phase
    int perm[NP];               // position -> original column
    double urow[2][NP];         // published U rows (zeros up to the pivot)
    int s_j[2];
    int s_rowt[BR];             // pivots found before each block row
    int s_rowpiv[BR];           // 1 if the block row holds a pivot
    int s_composite;
    int s_nz[BR];               // block row has a nonzero residual
    double ush[2][CH][NP];      // staged U rows (zeros up to the diagonal)
    int ublk[BR][NP];           // U rows found in the current block
    int s_tj[BR];               // their transpositions t <-> s_tj
    int s_ti[BR];               // and their rows (entries of Q)
    double s_pv[2];             // published pivot (as stored: scaled)
    double s_piv[BR];           // the block's stored pivots
    double s_isg[BR];           // 1 / Sigma_d (C entries of the block's columns)
    double s_ipv[BR];           // 1 / stored pivot (U rows)
};

// CUP of matrix idx by the whole workgroup (every thread calls it with the
// same idx; it returns on every thread together).
template <int BQ, int BW>
__device__ __forceinline__ void factor_one(const BatchDesc& g, int idx, BatchShared<BQ, BW>& sh)
{
    constexpr int NP = 64 * BQ;        // positions
    constexpr int BT = 64 * BW;        // threads
    constexpr int BR = BK * BW;        // rows per block
    constexpr int CH = BW;             // U rows per staged chunk
    constexpr int SPT = CH * NP / BT;  // staged values per thread
    static_assert((CH * NP) % BT == 0, "threads tile the staged chunk");
    auto& perm = sh.perm;
    auto& urow = sh.urow;
    auto& s_j = sh.s_j;
    auto& s_rowt = sh.s_rowt;
    auto& s_rowpiv = sh.s_rowpiv;
    auto& s_composite = sh.s_composite;
    auto& s_nz = sh.s_nz;
    auto& ush = sh.ush;
    auto& ublk = sh.ublk;
    auto& s_tj = sh.s_tj;
    auto& s_ti = sh.s_ti;
    auto& s_pv = sh.s_pv;
    auto& s_piv = sh.s_piv;
    auto& s_isg = sh.s_isg;
    auto& s_ipv = sh.s_ipv;

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);

    const int64_t N64 = g.n[idx];
    const int64_t M64 = g.m[idx], ld = g.lda[idx], p64 = g.p[idx];
    int64_t* const A = g.A[idx];
    int64_t* const Pv = g.P ? g.P[idx] : nullptr;
    int64_t* const Qv = g.Q ? g.Q[idx] : nullptr;

    // Argument checks, in the order of the single-matrix entry point.
    int code = 0;
    if (M64 < 0 || M64 > 0x3fffffff) code = -1;
    else if (N64 < 0 || N64 > BQ * 64) code = -2;
    else if (!A && M64 > 0 && N64 > 0) code = -3;
    else if (ld < (N64 > 1 ? N64 : 1)) code = -4;
    else if (p64 < 2 || p64 >= (1 << 26)) code = -5;
    if (code == 0 && p64 > 3) {
        // trial division by 2 and the odd numbers up to sqrt(p) < 2^13
        if (tid == 0) s_composite = (p64 % 2 == 0);
        __syncthreads();
        const unsigned pu = (unsigned)p64;
        for (unsigned d = 3 + 2 * (unsigned)tid; d * d <= pu; d += 2 * BT)
            if (pu % d == 0) s_composite = 1;
        __syncthreads();
        if (s_composite) code = -5;
    }
    if (code) {
        if (tid == 0) {
            g.info[idx] = code;
            g.rank[idx] = 0;
        }
        return;
    }
    const int M = (int)M64, N = (int)N64;
    if (Pv)
        for (int c = tid; c < N; c += BT) Pv[c] = c;
    if (Qv)
        for (int i = tid; i < M; i += BT) Qv[i] = i;
    if (M == 0 || N == 0) {
        if (tid == 0) {
            g.info[idx] = 0;
            g.rank[idx] = 0;
        }
        return;
    }

    const double P = (double)p64, PI = 1.0 / P;
    const double kr = floor((9007199254740992.0 - P) / (2.0 * P * (P - 1.0)));
    const int kred = kr > 1e9 ? 1000000000 : (int)kr;  // >= 1 for p < 2^26
    const int nq = (N + 63) >> 6;
    for (int c = tid; c < NP; c += BT) perm[c] = c;

    double x[BK][BQ];
    auto reduce_all = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < BK; ++k)
#pragma unroll
            for (int q = 0; q < BQ; ++q)
                if (q < nq) x[k][q] = mod_red(x[k][q], P, PI);
    };

    int t = 0;
    for (int i0 = 0; i0 < M; i0 += BR) {
        const int rows = min(BR, M - i0);
        const int t0 = t;  // pivots before the block
        // the previous block's global writes are visible to the workgroup
        __syncthreads();

        // 1. load the block in the current column order
#pragma unroll
        for (int k = 0; k < BK; ++k) {
            // every address valid (row and position clamped), so the loads
            // of the block issue together
            const int row = w + BW * k;
            const int64_t* src = A + (int64_t)(i0 + min(row, rows - 1)) * ld;
#pragma unroll
            for (int q = 0; q < BQ; ++q) {
                const int c = lane + 64 * q;
                const double v = ld_res(src + perm[min(c, N - 1)]);
                x[k][q] = (row < rows && c < N) ? v : 0.0;
            }
        }
        int cnt = 0;

        // 2. left-looking elimination against U rows 0..t-1.  Thread tid
        // stages entries tid + BT e (e < SPT) of a chunk, row-major (row
        // (tid + BT e) / NP, position (tid + BT e) % NP).  The loads read
        // clamped (always valid) addresses and the entries that are not U
        // entries are zeroed only when the chunk goes to LDS, so that no load
        // waits on the one before it.
        const int nch = (t + CH - 1) / CH;
        int stg[SPT];
        auto fetch = [&](int ch) __attribute__((always_inline)) {
#pragma unroll
            for (int e = 0; e < SPT; ++e) {
                const int v = tid + BT * e, spos = v % NP;
                const int sr = min(ch * CH + v / NP, t - 1);
                // a global-memory load (not a flat one, which would also
                // hold the LDS counter that the steps below wait on)
                stg[e] = *(const __attribute__((address_space(1))) int*)(A + (int64_t)sr * ld + min(spos, N - 1));
            }
        };
        if (nch > 0) fetch(0);
        int ch = 0;
        Unroll<BQ>::run([&](auto qsc) __attribute__((always_inline)) {
            constexpr int qs = decltype(qsc)::value;
            for (; ch < nch && ch * CH < 64 * (qs + 1); ++ch) {
                const int buf = ch & 1;
#pragma unroll
                for (int e = 0; e < SPT; ++e) {
                    const int v = tid + BT * e, spos = v % NP;
                    const int sr = ch * CH + v / NP;
                    ush[buf][v / NP][spos] = (sr < t && spos > sr && spos < N) ? (double)stg[e] : 0.0;
                }
                __syncthreads();
                if (ch + 1 < nch) fetch(ch + 1);
                const int s0 = ch * CH, s1 = min(t, s0 + CH);
                for (int s = s0; s < s1; ++s) {
                    if (cnt >= kred) {
                        reduce_all();
                        cnt = 0;
                    }
                    const int ls = s & 63;
                    double u[BQ];
#pragma unroll
                    for (int q = qs; q < BQ; ++q) u[q] = ush[buf][s - s0][lane + 64 * q];
#pragma unroll
                    for (int k = 0; k < BK; ++k) {
                        const double mk = red_lazy(readlane_d(x[k][qs], ls), P, PI);
#pragma unroll
                        for (int q = qs; q < BQ; ++q) x[k][q] = fma(-mk, u[q], x[k][q]);
                    }
                    ++cnt;
                }
            }
        });

        // rows whose residual at positions >= t is zero need no base-case step
        reduce_all();
        cnt = 0;
#pragma unroll
        for (int k = 0; k < BK; ++k) {
            bool nz = false;
#pragma unroll
            for (int q = 0; q < BQ; ++q) {
                const int c = lane + 64 * q;
                nz |= __ballot(q < nq && c >= t && c < N && x[k][q] != 0.0) != 0ull;
            }
            const int row = w + BW * k;
            if (lane == 0) s_nz[row] = nz && row < rows;
        }
        __syncthreads();

        // 3. row-by-row base case inside the block
        int a = 0;
        Unroll<BQ>::run([&](auto qtc) __attribute__((always_inline)) {
            constexpr int qt = decltype(qtc)::value;
            while (a < rows && t < N && (t >> 6) == qt) {
                if (!s_nz[a]) {
                    if (tid == 0) {
                        s_rowt[a] = t;
                        s_rowpiv[a] = 0;
                    }
                    ++a;
                    continue;
                }
                if (cnt >= kred) {
                    reduce_all();
                    cnt = 0;
                }
                const int par = a & 1;
                const int lt = t & 63;
                if (w == (a & (BW - 1))) {
                    // the owner wave: row a, positions >= 64 qt (the rest are < t)
                    // row a = sum_k [k == a / BW] x[k]: products with 0 and 1 are
                    // exact, and a select between register-array elements could
                    // turn into an indexed access that keeps x out of registers
                    const int ka = a / BW;
                    double ek[BK];
#pragma unroll
                    for (int k = 0; k < BK; ++k) ek[k] = (ka == k) ? 1.0 : 0.0;
                    // residues in (-p, p), zero exactly where the entry is
                    // (positions past n hold zeros)
                    double rv[BQ];
#pragma unroll
                    for (int q = qt; q < BQ; ++q) {
                        double v = x[0][q] * ek[0];
#pragma unroll
                        for (int k = 1; k < BK; ++k) v = fma(x[k][q], ek[k], v);
                        rv[q] = red_near(v, P, PI);
                    }
                    // the entry at position t, read beside the pivot search:
                    // it is the pivot unless that entry is zero
                    const double vt = readlane_d(rv[qt], lt);
                    int j = -1;
#pragma unroll
                    for (int q = BQ - 1; q >= qt; --q) {
                        const int c = lane + 64 * q;
                        const unsigned long long mk = __ballot(c >= t && c < N && rv[q] != 0.0);
                        if (mk) j = 64 * q + __ffsll((long long)mk) - 1;
                    }
                    if (j >= 0) {
                        double piv = vt;
                        if (j != t) {
                            const int qj = j >> 6, lj = j & 63;
                            double sel = rv[qt];
#pragma unroll
                            for (int q = qt + 1; q < BQ; ++q) sel = (q == qj) ? rv[q] : sel;
                            piv = readlane_d(sel, lj);
                        }
                        // the pivot row as it stands (scaled, in (-p, p)),
                        // after the exchange, positions after t; it is
                        // normalised when the block is written out
                        int* ub = ublk[t - t0];
#pragma unroll
                        for (int q = 0; q < BQ; ++q) {
                            const int c = lane + 64 * q;
                            if (q < qt) {
                                urow[par][c] = 0.0;
                            } else {
                                const double val = (c == j) ? vt : rv[q];
                                const double u = (c > t && c < N) ? val : 0.0;
                                urow[par][c] = u;
                                ub[c] = (int)u;
                            }
                        }
                        if (lane == 0) {
                            s_pv[par] = piv;
                            s_piv[t - t0] = piv;
                        }
                    }
                    if (lane == 0) s_j[par] = j;
                }
                __syncthreads();
                const int j = s_j[par];
                if (tid == 0) {
                    s_rowt[a] = t;
                    s_rowpiv[a] = (j >= 0);
                }
                if (j >= 0) {
                    if (j != t) {
                        // transposition t <-> j (j > t) in the block rows
                        const int qj = j >> 6, lj = j & 63;
#pragma unroll
                        for (int k = 0; k < BK; ++k) {
                            const double vt = readlane_d(x[k][qt], lt);
                            double vj = 0.0;
#pragma unroll
                            for (int q = qt; q < BQ; ++q) vj = (q == qj) ? readlane_d(x[k][q], lj) : vj;
                            x[k][qt] = (lane == lt) ? vj : x[k][qt];
#pragma unroll
                            for (int q = qt; q < BQ; ++q) x[k][q] = (q == qj && lane == lj) ? vt : x[k][q];
                        }
                    }
                    // fraction free: a later row becomes piv row - m (pivot
                    // row) at positions after t (m: its entry at t, kept
                    // there as its C entry); every value stays in (-p, p)
                    // and every product below p^2, so the fma is exact
                    const double piv = s_pv[par];
                    double u[BQ];
#pragma unroll
                    for (int q = qt; q < BQ; ++q) u[q] = urow[par][lane + 64 * q];
#pragma unroll
                    for (int k = 0; k < BK; ++k) {
                        const int row = w + BW * k;
                        const bool later = row > a && row < rows;
                        const double mk = readlane_d(x[k][qt], lt);
#pragma unroll
                        for (int q = qt; q < BQ; ++q) {
                            const double y = red_near(fma(piv, x[k][q], -(mk * u[q])), P, PI);
                            x[k][q] = (later && (q > qt || lane > lt)) ? y : x[k][q];
                        }
                    }
                    if (j != t) {
                        // the block's earlier U rows (LDS) and the column order
                        for (int d = tid; d < t - t0; d += BT) {
                            const int e = ublk[d][t];
                            ublk[d][t] = ublk[d][j];
                            ublk[d][j] = e;
                        }
                        if (tid == 0) {
                            const int e = perm[t];
                            perm[t] = perm[j];
                            perm[j] = e;
                        }
                    }
                    if (tid == 0) {
                        s_tj[t - t0] = j;
                        s_ti[t - t0] = i0 + a;
                    }
                    ++t;
                    ++cnt;
                }
                ++a;
            }
        });
        // rows left once every position holds a pivot are dependent
        for (int aa = a + tid; aa < rows; aa += BT) {
            s_rowt[aa] = t;
            s_rowpiv[aa] = 0;
        }
        __syncthreads();

        // The block's steps scaled its rows: after step t0 + d a row stands
        // at Sigma_{d+1} = prod_{d' <= d} (stored pivot d') times its true
        // value.  Wave 0 forms Sigma by a scan and the inverses in parallel
        // lanes: 1 / Sigma_d for the C entries of column t0 + d, and
        // 1 / (stored pivot d) for U row t0 + d.
        const int nd = t - t0;
        if (w == 0 && nd > 0) {
            double sg = (lane < nd) ? s_piv[min(lane, BR - 1)] : 1.0;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const double o = __shfl_up(sg, off, 64);
                if (lane >= off) sg = red_near(sg * o, P, PI);
            }
            // lane d: Sigma_{d+1}
            const double isg_next = inv_pivot(sg, P, PI);
            double isg = __shfl_up(isg_next, 1, 64);  // 1 / Sigma_d
            double sg_prev = __shfl_up(sg, 1, 64);    // Sigma_d
            if (lane == 0) {
                isg = 1.0;
                sg_prev = 1.0;
            }
            if (lane < nd) {
                s_isg[lane] = isg;
                s_ipv[lane] = red_near(sg_prev * isg_next, P, PI);
            }
        }
        __syncthreads();

        // 4. the block's transpositions on the U rows of earlier blocks (one
        // thread per row, in order), its U rows, and its entries of P and Q
        for (int sr = tid; sr < t0; sr += BT) {
            int64_t* ur = A + (int64_t)sr * ld;
            for (int d = 0; d < nd; ++d) {
                const int tt = t0 + d, jj = s_tj[d];
                if (jj != tt) {
                    const int64_t e = ur[tt];
                    ur[tt] = ur[jj];
                    ur[jj] = e;
                }
            }
        }
        for (int d = 0; d < nd; ++d) {
            const int tt = t0 + d;
            int64_t* ur = A + (int64_t)tt * ld;
            const double ip = s_ipv[d];
            for (int c = tt + 1 + tid; c < N; c += BT) ur[c] = (int64_t)(int)mod_red((double)ublk[d][c] * ip, P, PI);
        }
        if (tid < nd) {
            if (Pv) Pv[t0 + tid] = s_tj[tid];
            if (Qv) Qv[t0 + tid] = s_ti[tid];
        }
        // C entries and echelon zeros, positions <= row
        reduce_all();
#pragma unroll
        for (int k = 0; k < BK; ++k) {
            const int row = w + BW * k;
            if (row < rows) {
                const int i = i0 + row;
                const int tr = s_rowt[row], pv = s_rowpiv[row];
                int64_t* dst = A + (int64_t)i * ld;
#pragma unroll
                for (int q = 0; q < BQ; ++q) {
                    const int c = lane + 64 * q;
                    if (q < nq && c <= i && c < N) {
                        const bool cpart = (c < tr) || (pv && c == tr);
                        // columns of this block's steps: true value = stored / Sigma
                        const double y = (c >= t0 && c < t) ? mod_red(x[k][q] * s_isg[min(c - t0, BR - 1)], P, PI)
                                                            : x[k][q];
                        dst[c] = cpart ? (int64_t)(int)y : 0;
                    }
                }
            }
        }
    }
    __syncthreads();
    // rows r..M-1 carry no U row: zeros after the diagonal
    const int r = t;
    for (int i = r + w; i < M; i += BW) {
        int64_t* dst = A + (int64_t)i * ld;
        for (int c = i + 1 + lane; c < N; c += 64) dst[c] = 0;
    }
    if (tid == 0) {
        g.info[idx] = 0;
        g.rank[idx] = r;
    }
}

// Width class of a matrix with n columns: 0 (n <= 128), 1 (n <= 256), 2 (the
// rest, including n > 512 and invalid n, which its kernel reports).
__device__ __forceinline__ int width_class(int64_t n) { return n <= 128 ? 0 : (n <= 256 ? 1 : 2); }

__device__ __forceinline__ double batch_cost(const int64_t* m, const int64_t* n, int e)
{
    const double a = (double)m[e], c = (double)n[e];
    return (a > 0.0 && c > 0.0) ? a * c * (a < c ? a : c) : 0.0;
}

// order[k]: the matrices by width class, and within a class by decreasing
// cost m n min(m, n) (ties by index), by counting: the position of matrix i
// is the number of matrices that precede it.  Each matrix is counted by 16
// threads (those of a 16-lane group, each over every 16th matrix of the
// staged tiles), whose counts add up by shuffles.  Also zeroes the classes'
// work counters (the persistent kernels that read them run after this
// kernel).
constexpr int kOrderSplit = 16;  // threads per counted matrix
__global__ __launch_bounds__(256) void batched_order_kernel(const int64_t* m, const int64_t* n,
                                                            int batch, int* order, int* counters)
{
    __shared__ double cost[256];
    __shared__ int cls[256];
    const int sub = threadIdx.x % kOrderSplit;
    const int i = blockIdx.x * (256 / kOrderSplit) + threadIdx.x / kOrderSplit;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) counters[c] = 0;
    const double mine = (i < batch) ? batch_cost(m, n, i) : 0.0;
    const int mc = (i < batch) ? width_class(n[i]) : 0;
    int pos = 0;
    for (int j0 = 0; j0 < batch; j0 += 256) {
        __syncthreads();
        const int e = j0 + threadIdx.x;
        cost[threadIdx.x] = (e < batch) ? batch_cost(m, n, e) : -1.0;
        cls[threadIdx.x] = (e < batch) ? width_class(n[e]) : 3;
        __syncthreads();
        const int lim = min(256, batch - j0);
        for (int jj = sub; jj < lim; jj += kOrderSplit) {
            const double o = cost[jj];
            const int oc = cls[jj];
            pos += (oc < mc) || (oc == mc && ((o > mine) || (o == mine && j0 + jj < i)));
        }
    }
#pragma unroll
    for (int off = kOrderSplit / 2; off > 0; off >>= 1) pos += __shfl_xor(pos, off, kOrderSplit);
    if (i < batch && sub == 0) order[pos] = i;
}

__global__ void batched_reset_kernel(int* counters)
{
    if (threadIdx.x < 3) counters[threadIdx.x] = 0;
}

// One persistent kernel per width class: each workgroup finds its class's
// range of the order (or, without an order, walks every index), then takes
// matrices one at a time from the class's counter until the class is done.
template <int BQ, int BW>
__global__ __launch_bounds__(64 * BW) void batched_cup_kernel(BatchDesc g, int batch, int cls, int* counters)
{
    constexpr int BT = 64 * BW;
    __shared__ BatchShared<BQ, BW> sh;
    __shared__ int s_base, s_count, s_next;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_base = 0;
        s_count = 0;
    }
    __syncthreads();
    if (g.order) {
        int below = 0, mine = 0;
        for (int e = tid; e < batch; e += BT) {
            const int c = width_class(g.n[e]);
            below += c < cls;
            mine += c == cls;
        }
        atomicAdd(&s_base, below);
        atomicAdd(&s_count, mine);
    }
    for (;;) {
        __syncthreads();  // the previous matrix is done with the shared state
        if (tid == 0) s_next = atomicAdd(counters + cls, 1);
        __syncthreads();
        const int k = s_next;
        int idx;
        if (g.order) {
            if (k >= s_count) break;
            idx = g.order[s_base + k];
        } else {
            if (k >= batch) break;
            idx = k;
            if (width_class(g.n[idx]) != cls) continue;
        }
        factor_one<BQ, BW>(g, idx, sh);
    }
}

// Workgroups of each class's persistent kernel: CUs x workgroups per CU,
// the latter from the tuning table (tune_batched.py measures every choice
// up to the resident maximum on the multi-modular workload and writes
// batched_tune.h), capped by what the occupancy calculator allows.  The
// environment variable CUP_BATCHED_TUNE="w0,w1,w2,concurrent" overrides the
// table (the tuner's measurements use it).
struct BatchTune {
    int per_cu[3];
    int concurrent;
};

BatchTune batch_tune()
{
    BatchTune t{{kTuneWgPerCu[0], kTuneWgPerCu[1], kTuneWgPerCu[2]}, kTuneConcurrent};
    if (const char* v = std::getenv("CUP_BATCHED_TUNE")) {
        int a = 0, b = 0, c = 0, d = 0;
        if (std::sscanf(v, "%d,%d,%d,%d", &a, &b, &c, &d) == 4) t = BatchTune{{a, b, c}, d};
    }
    return t;
}

int persistent_grid(int cls, const BatchTune& t)
{
    static int cus = 0, maxper[3] = {0, 0, 0};
    if (!cus) {
        int dev = 0;
        CUP_HIP(hipGetDevice(&dev));
        CUP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        CUP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&maxper[0], batched_cup_kernel<2, kClassWaves[0]>,
                                                             64 * kClassWaves[0], 0));
        CUP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&maxper[1], batched_cup_kernel<4, kClassWaves[1]>,
                                                             64 * kClassWaves[1], 0));
        CUP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&maxper[2], batched_cup_kernel<BQMAX, kClassWaves[2]>,
                                                             64 * kClassWaves[2], 0));
        cus = std::max(1, cus);
    }
    const int per = std::max(1, std::min(t.per_cu[cls], std::max(1, maxper[cls])));
    return cus * per;
}

// Side streams and events of the concurrent class launches (default
// priority), created on first use and kept.
struct ClassStreams {
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
};

ClassStreams& class_streams()
{
    static ClassStreams cs;
    if (!cs.fork) {
        for (int k = 0; k < 2; ++k) {
            CUP_HIP(hipStreamCreateWithFlags(&cs.side[k], hipStreamNonBlocking));
            CUP_HIP(hipEventCreateWithFlags(&cs.join[k], hipEventDisableTiming));
        }
        CUP_HIP(hipEventCreateWithFlags(&cs.fork, hipEventDisableTiming));
    }
    return cs;
}

template <int BQ, int BW>
void launch_class(hipStream_t s, const BatchDesc& g, int batch, int cls, int* counters, const BatchTune& t)
{
    hipLaunchKernelGGL((batched_cup_kernel<BQ, BW>), dim3(persistent_grid(cls, t)), dim3(64 * BW), 0, s, g, batch,
                       cls, counters);
    CUP_HIP(hipGetLastError());
}

}  // namespace

int batched_max_n() { return BQMAX * 64; }

size_t batched_scratch_ints(int batch, bool ordered) { return kBatchCounters + (ordered ? (size_t)batch : 0); }

void launch_batched_cup(hipStream_t s, int batch, const int64_t* m, const int64_t* n,
                        int64_t* const* A, const int64_t* lda, const int64_t* p, int64_t* rank,
                        int64_t* const* P, int64_t* const* Q, int32_t* info, int* scratch, bool ordered)
{
    if (batch <= 0) return;
    int* counters = scratch;
    int* order = ordered ? scratch + kBatchCounters : nullptr;
    if (order)
        hipLaunchKernelGGL(batched_order_kernel, dim3((batch + 256 / kOrderSplit - 1) / (256 / kOrderSplit)),
                           dim3(256), 0, s, m, n, batch, order, counters);
    else
        hipLaunchKernelGGL(batched_reset_kernel, dim3(1), dim3(64), 0, s, counters);
    CUP_HIP(hipGetLastError());
    // widest class first, so that the largest matrices start first; with
    // concurrent launches the narrower classes run on two side streams that
    // join the stream again, and take the CUs the wide class leaves idle
    BatchDesc g{m, n, A, lda, p, rank, P, Q, info, order};
    const BatchTune t = batch_tune();
    if (!t.concurrent) {
        launch_class<BQMAX, kClassWaves[2]>(s, g, batch, 2, counters, t);
        launch_class<4, kClassWaves[1]>(s, g, batch, 1, counters, t);
        launch_class<2, kClassWaves[0]>(s, g, batch, 0, counters, t);
        return;
    }
    ClassStreams& cs = class_streams();
    CUP_HIP(hipEventRecord(cs.fork, s));
    CUP_HIP(hipStreamWaitEvent(cs.side[0], cs.fork, 0));
    CUP_HIP(hipStreamWaitEvent(cs.side[1], cs.fork, 0));
    launch_class<BQMAX, kClassWaves[2]>(s, g, batch, 2, counters, t);
    launch_class<4, kClassWaves[1]>(cs.side[0], g, batch, 1, counters, t);
    launch_class<2, kClassWaves[0]>(cs.side[1], g, batch, 0, counters, t);
    for (int k = 0; k < 2; ++k) {
        CUP_HIP(hipEventRecord(cs.join[k], cs.side[k]));
        CUP_HIP(hipStreamWaitEvent(s, cs.join[k], 0));
    }
}

}  // namespace cup
