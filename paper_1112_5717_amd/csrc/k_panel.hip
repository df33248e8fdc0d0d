// Base case of the CUP recursion: pivot decisions on a leaf of up to 64 rows.
//
// The paper's base case (Section 3.3, Algorithm 6 with m = 1) takes one row,
// finds the leftmost nonzero entry in the current column order, swaps that
// column to the front and scales the rest of the row by the pivot's inverse.
// Unrolled over a block of rows, this is row-by-row elimination in which
// every decision depends on all earlier ones, so it is the sequential chain
// of the method.  It is confined here to one workgroup and to a window of 64
// columns (compiled for 64 or 128; a full-rank leaf of 64 rows finds its 64
// pivots in the first 64 columns) held in registers:
//
//  * Each row's residual is tested for its leftmost nonzero with one
//    wave-wide ballot per 64 columns.
//  * Elimination inside the window is fraction free:
//        row_l <- piv * row_l - row_l[t] * row_pivot   (mod p)
//    which multiplies later rows by nonzero scalars and so preserves every
//    zero test, but keeps modular inverses off the sequential chain.  The
//    tile lives in registers; residues stay in (-p, p) between steps, so
//    each update is two products and one rounding reduction, and every
//    product stays below 2 p^2 < 2^53.
//  * Afterwards the true values are recovered in one parallel pass: with
//    Sigma_s the product of the first s stored pivots, a C entry frozen at
//    step s is divided by Sigma_s, the U part of pivot row s by its stored
//    pivot, and a residual left after d pivots by Sigma_d.  The d + 1
//    inverses are computed in parallel lanes.
//
// The phase stops at the first row whose residual vanishes on the window
// (the host then decides that row with a full-width scan) or when the
// window or the rows are exhausted.  Pivot rows never move here; the host
// compacts the U rows at the end of the leaf.
#include "modarith.h"
#include "tri64.h"

namespace cup {

namespace {

constexpr int WT = 1024;            // threads of the window kernel (16 waves)
constexpr int NWV = WT / 64;        // waves
constexpr int KPW = kLeafRows / NWV; // tile rows per wave
static_assert(NWV >= 10, "the end phase inverts the two triangles on waves 0-3 and 6-9");

// Residue in (-p, p): x - round(x / p) p, exact for |x| < 2^53.  Zero iff
// x = 0 mod p.  The rounding adds and subtracts 1.5 * 2^52, which rounds any
// value of magnitude below 2^51 to the nearest integer with two full-rate
// additions.
__device__ __forceinline__ double red_c(double x, double p, double pinv)
{
    const double magic = 6755399441055744.0;  // 1.5 * 2^52
    const double q = fma(x, pinv, magic) - magic;
    return fma(-q, p, x);
}

// v[q][k] for a wave-uniform q (a select chain over the register halves)
template <int WQ>
__device__ __forceinline__ double pick(const double (&v)[WQ][KPW], int k, int q)
{
    double x = v[0][k];
#pragma unroll
    for (int e = 1; e < WQ; ++e) x = (q == e) ? v[e][k] : x;
    return x;
}

// Lanes l with lo <= l < hi, as a wave-uniform 64-bit mask.
__device__ __forceinline__ unsigned long long lane_span(int lo, int hi)
{
    const unsigned long long from = (lo <= 0) ? ~0ull : ((lo >= 64) ? 0ull : (~0ull << lo));
    const unsigned long long below = (hi >= 64) ? ~0ull : ((hi <= 0) ? 0ull : ((1ull << hi) - 1));
    return from & below;
}

// Leftmost position >= a (and < wc) of a nonzero entry of the row held one
// column per lane in u, or -1: one compare per 64 columns, the position
// limits applied to the ballot on the scalar unit.
template <int WQ>
__device__ __forceinline__ int leftmost(const double (&u)[WQ], int a, int wc)
{
#pragma unroll
    for (int q = 0; q < WQ; ++q) {
        const unsigned long long m = __builtin_amdgcn_ballot_w64(u[q] != 0.0) & lane_span(a - 64 * q, wc - 64 * q);
        if (m) return 64 * q + __builtin_ctzll(m);
    }
    return -1;
}

// u[q] for a wave-uniform q
template <int WQ>
__device__ __forceinline__ double pick1(const double (&u)[WQ], int q)
{
    double x = u[0];
#pragma unroll
    for (int e = 1; e < WQ; ++e) x = (q == e) ? u[e] : x;
    return x;
}

// One result word for the host: a single 64-bit store, tagged with the
// launch's sequence number, made at system scope so that it goes to host
// memory without waiting for the end of the kernel.
__device__ __forceinline__ void post_word(unsigned long long* w, unsigned seq, int v)
{
    __hip_atomic_store(w, ((unsigned long long)seq << 32) | (unsigned)v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ double readlane_d(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// Bound on the polls for a pivot row (about 0.1 s): a row that never comes is
// reported as a failure instead of waiting forever.
constexpr int kSpinMax = 1 << 22;

// Bit pattern of an LDS row slot not written yet (a NaN, which no residue is).
constexpr unsigned long long kEmpty = ~0ull;

// Register-resident tile: thread (wave w, lane l) holds the consecutive rows
// KPW w + k (k < KPW) of columns l + 64q (q < WQ).  So the pivot of step a + 1
// usually comes from the same wave as that of step a, and a wave takes its
// own KPW steps without waiting on anyone: leftmost nonzero by ballot, pivot
// and multipliers by readlane, update of its later rows in registers.  The
// multiplier of each row at each step (its frozen C entry) is copied aside
// in registers, so the update itself runs on every lane without a select
// (entries left of the pivot become don't-care values in (-p, p)).  Each
// pivot row goes, as it stands before its column exchange, to its own LDS
// slot, which holds a NaN pattern until then; every entry is written once,
// with one 64-bit store, so a reader polls the row itself until no entry is
// still empty and finds the pivot column from it as the owner did: one LDS
// round trip per pivot, no flag and no fence.  Pivot columns and pivots go
// to LDS once, after the wave's last step.
// The waves below follow the slots in order, applying every pivot to their
// rows as it arrives; a wave whose rows are all pivots stops following and
// applies the later column exchanges after the final barrier.  No barrier
// per step, and no slot is reused within a window.
template <typename T, int WQ>
__global__ __launch_bounds__(WT) void window_kernel(T* __restrict__ A, int64_t lda, int b, int N,
                                                    int i0, int t0, int wc, ModP mp,
                                                    int* __restrict__ out,
                                                    unsigned long long* __restrict__ mail,
                                                    unsigned seq, double* __restrict__ winv,
                                                    double* __restrict__ uinv, T* __restrict__ below)
{
    // The pivot-row slots during the elimination; afterwards the two unit
    // triangles and their inverses (padded rows).
    __shared__ double wbuf[4][kLeafRows][kTriNB + 1];
    double (*rowslot)[64 * WQ] = reinterpret_cast<double (*)[64 * WQ]>(&wbuf[0][0][0]);
    __shared__ int s_fail;
    __shared__ int s_d;  // pivots found (the step of a zero row, else min(rows, window))
    __shared__ int s_swap[kLeafRows];
    __shared__ double s_piv[kLeafRows];
    __shared__ double s_isig[kLeafRows + 1];
    __shared__ double s_ipiv[kLeafRows];
    __shared__ double s_dl[kLeafRows];  // inverses of the diagonal of C
    __shared__ int s_nswap;
    __shared__ int s_b[kLeafRows][kLeafRows + 1];  // the block under the leaf (two-leaf node)

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (uniform)
    const int R = b - i0;
    const int aend = max(0, min(R, wc));  // steps that can have a pivot
    const double P = mp.p, PI = mp.pinv;

    double v[WQ][KPW];
    double cm[WQ][KPW];  // multipliers: row k's value at column a, kept at lane a
#pragma unroll
    for (int q = 0; q < WQ; ++q)
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            const int r = KPW * w + k, c = lane + 64 * q;
            v[q][k] = (r < R && c < wc) ? ld_res(A + (int64_t)(i0 + r) * lda + t0 + c) : 0.0;
            cm[q][k] = 0.0;
        }
    for (int x = tid; x < kLeafRows * 64 * WQ; x += WT)
        rowslot[x / (64 * WQ)][x % (64 * WQ)] = __longlong_as_double((long long)kEmpty);
    if (tid == 0) {
        s_fail = 0;
        s_d = aend;
    }
    __syncthreads();
    // The block under the leaf, read for G = B U^{-1} at the end, is fetched
    // now by the last quarter of the waves (whose first own step is the
    // furthest away), so that its memory latency is off the end phase.
    if (WQ == 1 && below != nullptr && tid >= 3 * WT / 4)
        for (int x = tid - 3 * WT / 4; x < kLeafRows * kLeafRows; x += WT / 4)
            s_b[x >> 6][x & 63] = (int)ld_res(below + (int64_t)(x >> 6) * lda + (x & 63));

    const int own0 = KPW * w;
    // columns a and j (> a) exchange in every own row: the two entries are
    // read out to scalars and written back by lane selects, so the exchange
    // uses no LDS traffic (and no wait on it) on the chain
    auto swap_cols = [&](int a, int j) {
        const int qa = a >> 6, la = a & 63, qj = j >> 6, lj = j & 63;
        const bool at_a = lane == la, at_j = lane == lj;
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            const double xa = readlane_d(pick(v, k, qa), la);
            const double xj = readlane_d(pick(v, k, qj), lj);
#pragma unroll
            for (int q = 0; q < WQ; ++q) {
                v[q][k] = (at_a && q == qa) ? xj : v[q][k];
                v[q][k] = (at_j && q == qj) ? xa : v[q][k];
            }
        }
    };
    // fraction-free update of own row k by pivot row u of step a, with the
    // row's multiplier m (its entry at position a) read out beforehand; the
    // multiplier is also kept at lane a
    auto update = [&](int k, int a, double piv, double m, const double (&u)[WQ]) {
#pragma unroll
        for (int q = 0; q < WQ; ++q) {
            cm[q][k] = (lane + 64 * q == a) ? v[q][k] : cm[q][k];
            v[q][k] = red_c(fma(piv, v[q][k], -m * u[q]), P, PI);
        }
    };
    // The pivot entry and the multipliers are read out (lane to scalar) as
    // soon as the pivot row is there, on the guess that the pivot is at
    // position a, which holds unless the entry there is zero; the leftmost
    // test runs beside them and only a failed guess reads them again.  Each
    // read-out costs the latency of a vector-to-scalar transfer, so the
    // guess takes it off the pivot search's path.
    auto multipliers = [&](int a, int kfrom, double (&m)[KPW]) {
#pragma unroll
        for (int k = 0; k < KPW; ++k) m[k] = (k >= kfrom) ? readlane_d(pick(v, k, a >> 6), a & 63) : 0.0;
    };

    // Steps of the waves above: follow them in order (rows past the block
    // need no pivots; rows past the window need all of them).
    const int follow_end = (own0 < R) ? min(own0, aend) : 0;
    bool stopped = false;
    for (int a = 0; a < follow_end; ++a) {
        // the steps of the wave just above lead into this wave's own: they
        // are on the chain, so this wave is issued ahead of the others
        if (a == own0 - KPW) __builtin_amdgcn_s_setprio(2);
        // Row a as it stood before its column exchange, polled until no
        // entry holds the empty pattern; its pivot column is found here as
        // by its owner (leftmost nonzero at positions >= a; none: the
        // phase ends at a).
        double u[WQ];
        bool ready = false;
        for (int it = 0; it < kSpinMax; ++it) {
            bool empty = false;
#pragma unroll
            for (int q = 0; q < WQ; ++q) {
                const unsigned long long bits = __hip_atomic_load(
                    reinterpret_cast<unsigned long long*>(&rowslot[a][lane + 64 * q]), __ATOMIC_RELAXED,
                    __HIP_MEMORY_SCOPE_WORKGROUP);
                empty |= bits == kEmpty;
                u[q] = __longlong_as_double((long long)bits);
            }
            ready = __ballot(empty) == 0;
            if (ready) break;
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ready) {
            if (lane == 0) s_fail = 1;
            stopped = true;
            break;
        }
        double piv = readlane_d(pick1(u, a >> 6), a & 63);
        double m[KPW];
        multipliers(a, 0, m);
        const int j = leftmost(u, a, wc);
        if (j < 0) {
            stopped = true;
            break;
        }
        if (j != a) {
            // the exchange of positions a and j, in the pivot row and in
            // every own row
            const double ua = piv;
            piv = readlane_d(pick1(u, j >> 6), j & 63);
#pragma unroll
            for (int q = 0; q < WQ; ++q) {
                const int c = lane + 64 * q;
                u[q] = (c == a) ? piv : ((c == j) ? ua : u[q]);
            }
            swap_cols(a, j);
            multipliers(a, 0, m);
        }
#pragma unroll
        for (int k = 0; k < KPW; ++k) update(k, a, piv, m[k], u);
    }
    // Own steps, at the highest issue priority: they are the chain, and the
    // waves below share the SIMDs with updates that can wait.  Pivot
    // columns and pivots stay in registers until the end.
    __builtin_amdgcn_s_setprio(3);
    int own_j[KPW];
    double own_piv[KPW];
    int nown = 0;
    if (!stopped) {
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            const int a = own0 + k;
            if (a >= aend) break;
            double u[WQ];
#pragma unroll
            for (int q = 0; q < WQ; ++q) {
                u[q] = v[q][k];
                rowslot[a][lane + 64 * q] = u[q];  // published before the exchange
            }
            double piv = readlane_d(pick1(u, a >> 6), a & 63);
            double m[KPW];
            multipliers(a, k + 1, m);
            const int j = leftmost(u, a, wc);
            if (j < 0) {  // zero residual on the window: the phase ends at a
                if (lane == 0) s_d = a;
                break;
            }
            if (j != a) {
                swap_cols(a, j);
#pragma unroll
                for (int q = 0; q < WQ; ++q) u[q] = v[q][k];
                piv = readlane_d(pick1(u, a >> 6), a & 63);
                multipliers(a, k + 1, m);
            }
            own_j[k] = j;
            own_piv[k] = piv;
            nown = k + 1;
#pragma unroll
            for (int k2 = k + 1; k2 < KPW; ++k2) update(k2, a, piv, m[k2], u);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < KPW; ++k)
            if (k < nown) {
                s_swap[own0 + k] = own_j[k];
                s_piv[own0 + k] = own_piv[k];
            }
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    const int d = s_d;
    int stop = (d < aend) ? STOP_ZERO_ROW : ((R <= wc) ? STOP_ROWS : STOP_WINDOW);
    if (s_fail) stop = STOP_FAIL;
    // the result, for the host, as soon as it is known
    if (w == 0) {
        const bool sw = lane < d && s_swap[lane] != lane;
        const int nswap = __popcll(__ballot(sw));
        if (lane == 0) {
            s_nswap = nswap;
            out[kSwapWord] = nswap;
        }
    }
    if (tid == 0) {
        out[0] = d;
        out[1] = stop;
        if (mail) {
            post_word(mail + 1, seq, stop);
            post_word(mail, seq, d);
        }
    }
    for (int a = tid; a < d; a += WT) {
        out[2 + a] = t0 + s_swap[a];
        if (mail) post_word(mail + 2 + a, seq, t0 + s_swap[a]);
    }
    // column exchanges of the steps after this wave's rows (rows that
    // followed every step have them already)
    if (stop != STOP_FAIL && own0 < R && own0 + KPW <= aend) {
        const int a0 = own0 + KPW;
        for (int base = a0; base < d; base += 64) {
            const int a = base + lane;
            const bool sw = a < d && s_swap[min(a, kLeafRows - 1)] != a;
            unsigned long long mask = __ballot(sw);
            while (mask) {
                const int x = __ffsll((long long)mask) - 1;
                mask &= mask - 1;
                const int aa = base + x;
                swap_cols(aa, __builtin_amdgcn_readfirstlane(s_swap[aa]));
            }
        }
    }

    // Sigma_{s+1} = prod_{s' <= s} piv_{s'}: inclusive scan in wave 0, and the
    // inverses from it, every value kept in (-p, p) (short roundings on this
    // serial stretch; the stores below make the results canonical).
    if (w == 0) {
        double x = (lane < d) ? s_piv[lane] : 1.0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            double o = __shfl_up(x, off, 64);
            if (lane >= off) x = red_near(x * o, P, PI);
        }
        double sig_prev = __shfl_up(x, 1, 64);  // Sigma_lane
        if (lane == 0) sig_prev = 1.0;
        if (lane < d) {
            double isig_next = inv_fermat26(x, P, PI);  // 1 / Sigma_{lane+1}
            s_isig[lane + 1] = isig_next;
            const double ipiv = red_near(sig_prev * isig_next, P, PI);  // 1 / piv_lane
            s_ipiv[lane] = ipiv;
            s_dl[lane] = red_near(sig_prev * ipiv, P, PI);  // 1 / C[lane][lane]
        } else {
            s_dl[lane] = 1.0;  // identity padding of the inverse below
        }
        if (lane == 0) s_isig[0] = 1.0;
    }
    lds_barrier();

    // The pivot block's triangles are inverted here as well (padded with the
    // identity to 64 x 64): L^{-1} for any pivot count when `winv` is given,
    // U^{-1} (the cached one) and G only for a full 64 x 64 block.
    const bool full = d == kLeafRows && R == kLeafRows && wc == kLeafRows;
    const bool inv = WQ == 1 && d > 0 && P <= kExact64 &&
                     (winv != nullptr || (full && uinv != nullptr));
#pragma unroll
    for (int q = 0; q < WQ; ++q)
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            const int r = KPW * w + k, c = lane + 64 * q;
            if (r < R && c < wc) {
                // C below the diagonal from the kept multipliers (divided by
                // Sigma_c), the pivot itself (Sigma_c), the U part of a pivot
                // row (its pivot), or a residual entry (Sigma_d)
                const bool low = c < r && c < d;
                const double x = low ? cm[q][k] : v[q][k];
                const double f = (c <= r && c < d) ? s_isig[c] : ((r < d) ? s_ipiv[r] : s_isig[d]);
                const double y = canon(red_near(x * f, P, PI), P);
                st_res(A + (int64_t)(i0 + r) * lda + t0 + c, y);
            }
        }
    if (inv) {
        // the unit upper U, and L^T scaled to a unit triangle
        // (C[r][c] / C[c][c] = multiplier / stored pivot), zero outside the
        // d x d pivot block
        const int c = lane;
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            const int r = KPW * w + k;
            const bool in = r < d && c < d;
            wbuf[0][r][c] = (in && c > r) ? red_near(v[0][k] * s_ipiv[r], P, PI) : 0.0;
            wbuf[1][c][r] = (in && c < r) ? red_near(cm[0][k] * s_ipiv[c], P, PI) : 0.0;
        }
        // waves 0-3 invert U, waves 6-9 the scaled L^T (so that, with waves
        // placed on the four SIMDs in turn, the two groups' matrix-core
        // products of the later rounds fall on different SIMDs); then
        // U^{-1} as is, and L^{-1}[i][s] = (L^T scaled)^{-1}[s][i] / C[i][i]
        // (the barriers order LDS only: the stores of the block above are
        // left in flight)
        lds_barrier();
        const bool second = w >= 6 && w < 10;
        unit_upper_inverse<3>(wbuf[second ? 1 : 0], wbuf[second ? 3 : 2], P, PI, second ? 6 : 0);
        for (int idx = tid; idx < kLeafRows * kLeafRows; idx += WT) {
            const int i = idx >> 6, s = idx & 63;
            if (uinv && full) uinv[idx] = canon(wbuf[2][i][s], P);
            if (winv) winv[idx] = canon(red_near(wbuf[3][s][i] * s_dl[i], P, PI), P);
        }
        if (below != nullptr && full && s_nswap == 0) {
            // G = B U^{-1} for the block under the leaf (Algorithm 6's G
            // for a two-leaf node), 16 x 16 tiles spread over the waves, in
            // place (B comes from LDS, so no wave waits for another's reads)
            const int hi = lane >> 4, lo = lane & 15;
            for (int tile = w; tile < 16; tile += NWV) {
                const int tr = tile >> 2, tc = tile & 3;
                double bv[16];
#pragma unroll
                for (int ks = 0; ks < 16; ++ks) bv[ks] = (double)s_b[16 * tr + lo][4 * ks + hi];
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < 16; ++ks)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[ks], wbuf[2][4 * ks + hi][16 * tc + lo], acc, 0, 0, 0);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    st_res(below + (int64_t)(16 * tr + hi + 4 * e) * lda + 16 * tc + lo, mod_red(acc[e], P, PI));
            }
        }
    }
    // the same column swaps on the leaf rows above the window block
    for (int r = tid; r < i0; r += WT) {
        T* row = A + (int64_t)r * lda + t0;
        for (int a = 0; a < d; ++a) {
            int j = s_swap[a];
            if (j != a) {
                T x = row[a];
                row[a] = row[j];
                row[j] = x;
            }
        }
    }
}

// out[r - i0] = leftmost column >= t0 with a nonzero in row r, or N.
template <typename T>
__global__ __launch_bounds__(256) void row_scan_kernel(const T* __restrict__ A, int64_t lda,
                                                       int i0, int t0, int N, int* __restrict__ out,
                                                       unsigned long long* __restrict__ mail,
                                                       unsigned seq)
{
    __shared__ int best;
    const int r = i0 + blockIdx.x;
    if (threadIdx.x == 0) best = N;
    __syncthreads();
    const T* row = A + (int64_t)r * lda;
    for (int c = t0 + threadIdx.x; c < N; c += 256) {
        if (row[c] != 0) {
            atomicMin(&best, c);
            break;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[blockIdx.x] = best;
        if (mail) post_word(mail + kMailScan + blockIdx.x, seq, best);
    }
}

template <typename T>
__global__ void colswap_kernel(T* __restrict__ A, int64_t lda, int rows, int c0, int c1)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < rows) {
        T* row = A + (int64_t)r * lda;
        T x = row[c0];
        row[c0] = row[c1];
        row[c1] = x;
    }
}

}  // namespace

template <typename T>
void launch_window(hipStream_t s, T* A, int64_t lda, int b, int N, int i0, int t0, int wc,
                   ModP mp, int* out, unsigned long long* mail, unsigned seq, double* winv,
                   double* uinv, T* below)
{
    static_assert(kWin % 64 == 0 && kWin <= 128, "window of 64 or 128 columns");
    hipLaunchKernelGGL((window_kernel<T, kWin / 64>), dim3(1), dim3(WT), 0, s, A, lda, b, N, i0, t0,
                       wc, mp, out, mail, seq, winv, uinv, below);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_row_scan(hipStream_t s, const T* A, int64_t lda, int i0, int b, int t0, int N,
                     int* out, unsigned long long* mail, unsigned seq)
{
    if (b <= i0) return;
    hipLaunchKernelGGL(row_scan_kernel<T>, dim3(b - i0), dim3(256), 0, s, A, lda, i0, t0, N, out, mail,
                       seq);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_colswap(hipStream_t s, T* A, int64_t lda, int rows, int c0, int c1)
{
    if (rows <= 0 || c0 == c1) return;
    hipLaunchKernelGGL(colswap_kernel<T>, dim3((rows + 255) / 256), dim3(256), 0, s, A, lda, rows,
                       c0, c1);
    CUP_HIP(hipGetLastError());
}

#define CUP_INST(T)                                                                            \
    template void launch_window<T>(hipStream_t, T*, int64_t, int, int, int, int, int, ModP,    \
                                   int*, unsigned long long*, unsigned, double*, double*, T*); \
    template void launch_row_scan<T>(hipStream_t, const T*, int64_t, int, int, int, int, int*,  \
                                     unsigned long long*, unsigned);                            \
    template void launch_colswap<T>(hipStream_t, T*, int64_t, int, int, int);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
