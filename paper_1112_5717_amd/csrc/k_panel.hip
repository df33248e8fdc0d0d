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

namespace cup {

namespace {

constexpr int WT = 512;             // threads of the window kernel (8 waves)
constexpr int NWV = WT / 64;        // waves
constexpr int KPW = kLeafRows / NWV; // tile rows per wave

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

// Register-resident tile: thread (wave w, lane l) holds rows w + 8k
// (k = 0..7) of columns l + 64q (q < WQ).  The pivot row and the multiplier
// column of each step are exchanged through LDS buffers alternating with
// the step's parity, so one barrier per pivot suffices.
template <typename T, int WQ>
__global__ __launch_bounds__(WT) void window_kernel(T* __restrict__ A, int64_t lda, int b, int N,
                                                    int i0, int t0, int wc, ModP mp,
                                                    int* __restrict__ out)
{
    __shared__ double rowbuf[2][64 * WQ];
    __shared__ double colbuf[2][kLeafRows];
    __shared__ int s_j[2];
    __shared__ int s_swap[kLeafRows];
    __shared__ double s_piv[kLeafRows];
    __shared__ double s_isig[kLeafRows + 1];
    __shared__ double s_ipiv[kLeafRows];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (uniform)
    const int R = b - i0;
    const double P = mp.p, PI = mp.pinv;

    double v[WQ][KPW];
#pragma unroll
    for (int q = 0; q < WQ; ++q)
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            const int r = w + NWV * k, c = lane + 64 * q;
            v[q][k] = (r < R && c < wc) ? ld_res(A + (int64_t)(i0 + r) * lda + t0 + c) : 0.0;
        }

    // Publish row a (its owner wave: rowbuf and the leftmost nonzero at
    // positions >= a) and column a (its owner lane in every wave: colbuf)
    // into the buffers of parity a & 1.
    auto publish = [&](int a) {
        const int par = a & 1, qa = a >> 6, la = a & 63;
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            if (w + NWV * k == a) {
                int jj = -1;
#pragma unroll
                for (int q = WQ - 1; q >= 0; --q) {
                    const int c = lane + 64 * q;
                    const unsigned long long mq = __ballot(c >= a && c < wc && v[q][k] != 0.0);
                    rowbuf[par][c] = v[q][k];
                    if (mq) jj = 64 * q + __ffsll((long long)mq) - 1;
                }
                if (lane == 0) s_j[par] = jj;
            }
        }
        if (lane == la) {
#pragma unroll
            for (int k = 0; k < KPW; ++k) colbuf[par][w + NWV * k] = pick(v, k, qa);
        }
    };

    int d = 0, stop = STOP_ROWS;
    if (R > 0 && wc > 0) publish(0);
    __syncthreads();
    for (int a = 0;; ++a) {
        if (a >= R) { stop = STOP_ROWS; break; }
        if (a >= wc) { stop = STOP_WINDOW; break; }
        const int par = a & 1, qa = a >> 6, la = a & 63;
        // every LDS read of the step issued together (no swap assumed)
        const int j = s_j[par];
        double piv = rowbuf[par][a];
        double u[WQ];
#pragma unroll
        for (int q = 0; q < WQ; ++q) u[q] = rowbuf[par][lane + 64 * q];
        double mlt[KPW];
#pragma unroll
        for (int k = 0; k < KPW; ++k) mlt[k] = colbuf[par][w + NWV * k];
        if (j < 0) { stop = STOP_ZERO_ROW; break; }
        if (j != a) {
            // swap columns a and j: both live in the same lanes of every wave
            const int qj = j >> 6, lj = j & 63;
#pragma unroll
            for (int k = 0; k < KPW; ++k) {
                const double ca = pick(v, k, qa);
                const double cj = pick(v, k, qj);
                const double from_j = __shfl(cj, lj, 64);
                const double from_a = __shfl(ca, la, 64);
#pragma unroll
                for (int q = 0; q < WQ; ++q) {
                    if (lane == la && q == qa) v[q][k] = from_j;
                    if (lane == lj && q == qj) v[q][k] = from_a;
                }
            }
            __syncthreads();  // every wave has read the step's buffers
            if (lane == la) {
#pragma unroll
                for (int k = 0; k < KPW; ++k) colbuf[par][w + NWV * k] = pick(v, k, qa);
            }
            if (tid == 0) {
                double x = rowbuf[par][a];
                rowbuf[par][a] = rowbuf[par][j];
                rowbuf[par][j] = x;
            }
            __syncthreads();
            piv = rowbuf[par][a];
#pragma unroll
            for (int q = 0; q < WQ; ++q) u[q] = rowbuf[par][lane + 64 * q];
#pragma unroll
            for (int k = 0; k < KPW; ++k) mlt[k] = colbuf[par][w + NWV * k];
        }
        if (tid == 0) {
            s_swap[a] = j;
            s_piv[a] = mod_red(piv, P, PI);
        }
        // fraction-free update of rows > a, columns > a: rows skipped per
        // wave, columns masked per lane
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            if (w + NWV * k > a) {
#pragma unroll
                for (int q = 0; q < WQ; ++q) {
                    const double nq = red_c(fma(piv, v[q][k], -mlt[k] * u[q]), P, PI);
                    v[q][k] = (lane + 64 * q > a) ? nq : v[q][k];
                }
            }
        }
        d = a + 1;
        if (a + 1 < R && a + 1 < wc) publish(a + 1);
        __syncthreads();
    }
    __syncthreads();

    // Sigma_{s+1} = prod_{s' <= s} piv_{s'}: inclusive scan in wave 0.
    if (w == 0) {
        double x = (lane < d) ? s_piv[lane] : 1.0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            double o = __shfl_up(x, off, 64);
            if (lane >= off) x = mod_mul(x, o, P, PI);
        }
        double sig_prev = __shfl_up(x, 1, 64);  // Sigma_lane
        if (lane == 0) sig_prev = 1.0;
        if (lane < d) {
            double isig_next = mod_inv(x, P, PI);  // 1 / Sigma_{lane+1}
            s_isig[lane + 1] = isig_next;
            s_ipiv[lane] = mod_mul(sig_prev, isig_next, P, PI);  // 1 / piv_lane
        }
        if (lane == 0) s_isig[0] = 1.0;
    }
    __syncthreads();

#pragma unroll
    for (int q = 0; q < WQ; ++q)
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            const int r = w + NWV * k, c = lane + 64 * q;
            if (r < R && c < wc) {
                const int lim = (r + 1 < d) ? r + 1 : d;
                const double f = (c < lim) ? s_isig[c] : ((r < d) ? s_ipiv[r] : s_isig[d]);
                st_res(A + (int64_t)(i0 + r) * lda + t0 + c, mod_mul(v[q][k], f, P, PI));
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
    if (tid == 0) {
        out[0] = d;
        out[1] = stop;
    }
    for (int a = tid; a < d; a += WT) out[2 + a] = t0 + s_swap[a];
}

// out[r - i0] = leftmost column >= t0 with a nonzero in row r, or N.
template <typename T>
__global__ __launch_bounds__(256) void row_scan_kernel(const T* __restrict__ A, int64_t lda,
                                                       int i0, int t0, int N, int* __restrict__ out)
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
    if (threadIdx.x == 0) out[blockIdx.x] = best;
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
                   ModP mp, int* out)
{
    static_assert(kWin % 64 == 0 && kWin <= 128, "window of 64 or 128 columns");
    hipLaunchKernelGGL((window_kernel<T, kWin / 64>), dim3(1), dim3(WT), 0, s, A, lda, b, N, i0, t0,
                       wc, mp, out);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_row_scan(hipStream_t s, const T* A, int64_t lda, int i0, int b, int t0, int N,
                     int* out)
{
    if (b <= i0) return;
    hipLaunchKernelGGL(row_scan_kernel<T>, dim3(b - i0), dim3(256), 0, s, A, lda, i0, t0, N, out);
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
                                   int*);                                                      \
    template void launch_row_scan<T>(hipStream_t, const T*, int64_t, int, int, int, int, int*); \
    template void launch_colswap<T>(hipStream_t, T*, int64_t, int, int, int);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
