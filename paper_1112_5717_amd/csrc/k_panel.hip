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

constexpr int WT = 1024;            // threads of the window kernel (16 waves)
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

// Register-resident tile: thread (wave w, lane l) holds rows w + 16k
// (k = 0..3) of columns l + 64q (q < WQ).  Each step's pivot row goes to its
// own LDS slot with a ready flag (release/acquire at workgroup scope): the
// owner of row a + 1 updates that row first, publishes it, and only then
// updates its other rows, while every other wave starts step a + 1 as soon
// as the flag is up.  There is no barrier per step, and no slot is reused
// within a window.  Each wave keeps its own multipliers (column a of its
// rows) and applies every column exchange to its own registers.
template <typename T, int WQ>
__global__ __launch_bounds__(WT) void window_kernel(T* __restrict__ A, int64_t lda, int b, int N,
                                                    int i0, int t0, int wc, ModP mp,
                                                    int* __restrict__ out,
                                                    unsigned long long* __restrict__ mail,
                                                    unsigned seq)
{
    __shared__ double rowslot[kLeafRows][64 * WQ];
    __shared__ int s_jv[kLeafRows];
    __shared__ int s_flag[kLeafRows];
    __shared__ int s_fail;
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
    for (int x = tid; x < kLeafRows; x += WT) s_flag[x] = 0;
    if (tid == 0) s_fail = 0;
    __syncthreads();

    // The owner wave of row a publishes it: the row, its leftmost nonzero at
    // positions >= a (or -1), then the flag.
    auto publish = [&](int a) {
#pragma unroll
        for (int k = 0; k < KPW; ++k) {
            if (w + NWV * k == a) {
                int jj = -1;
#pragma unroll
                for (int q = WQ - 1; q >= 0; --q) {
                    const int c = lane + 64 * q;
                    const unsigned long long mq = __ballot(c >= a && c < wc && v[q][k] != 0.0);
                    rowslot[a][c] = v[q][k];
                    if (mq) jj = 64 * q + __ffsll((long long)mq) - 1;
                }
                if (lane == 0) {
                    s_jv[a] = jj;
                    __hip_atomic_store(&s_flag[a], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
    };
    // fraction-free update of own row k by pivot a (columns > a)
    auto update = [&](int k, int a, double piv, double m, const double (&u)[WQ]) {
#pragma unroll
        for (int q = 0; q < WQ; ++q) {
            const double nq = red_c(fma(piv, v[q][k], -m * u[q]), P, PI);
            v[q][k] = (lane + 64 * q > a) ? nq : v[q][k];
        }
    };

    int d = 0, stop = STOP_ROWS;
    if (R > 0 && wc > 0) publish(0);
    for (int a = 0;; ++a) {
        if (a >= R) { stop = STOP_ROWS; break; }
        if (a >= wc) { stop = STOP_WINDOW; break; }
        int f = 0;
        for (int it = 0; it < kSpinMax; ++it) {
            f = __hip_atomic_load(&s_flag[a], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (f) break;
            __builtin_amdgcn_s_sleep(1);
        }
        if (!f) {
            if (lane == 0) s_fail = 1;
            stop = STOP_FAIL;
            break;
        }
        const int qa = a >> 6, la = a & 63;
        const int j = s_jv[a];
        if (j < 0) { stop = STOP_ZERO_ROW; break; }
        double u[WQ];
#pragma unroll
        for (int q = 0; q < WQ; ++q) u[q] = rowslot[a][lane + 64 * q];
        const double piv = rowslot[a][j];
        if (j != a) {
            // positions a and j exchange, in the pivot row and in every own row
            const double ua = rowslot[a][a];
            const int qj = j >> 6, lj = j & 63;
#pragma unroll
            for (int q = 0; q < WQ; ++q) {
                const int c = lane + 64 * q;
                u[q] = (c == a) ? piv : ((c == j) ? ua : u[q]);
            }
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
        }
        if (tid == 0) {
            s_swap[a] = j;
            s_piv[a] = mod_red(piv, P, PI);
        }
        double mlt[KPW];
#pragma unroll
        for (int k = 0; k < KPW; ++k) mlt[k] = readlane_d(pick(v, k, qa), la);
        // row a + 1 first (then published), then the other own rows > a + 1
#pragma unroll
        for (int k = 0; k < KPW; ++k)
            if (w + NWV * k == a + 1) update(k, a, piv, mlt[k], u);
        if (a + 1 < R && a + 1 < wc) publish(a + 1);
#pragma unroll
        for (int k = 0; k < KPW; ++k)
            if (w + NWV * k > a + 1) update(k, a, piv, mlt[k], u);
        d = a + 1;
    }
    __syncthreads();
    if (s_fail) stop = STOP_FAIL;

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
        if (mail) {
            post_word(mail + 1, seq, stop);
            post_word(mail, seq, d);
        }
    }
    for (int a = tid; a < d; a += WT) {
        out[2 + a] = t0 + s_swap[a];
        if (mail) post_word(mail + 2 + a, seq, t0 + s_swap[a]);
    }
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
                   ModP mp, int* out, unsigned long long* mail, unsigned seq)
{
    static_assert(kWin % 64 == 0 && kWin <= 128, "window of 64 or 128 columns");
    hipLaunchKernelGGL((window_kernel<T, kWin / 64>), dim3(1), dim3(WT), 0, s, A, lda, b, N, i0, t0,
                       wc, mp, out, mail, seq);
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
                                   int*, unsigned long long*, unsigned);                       \
    template void launch_row_scan<T>(hipStream_t, const T*, int64_t, int, int, int, int, int*); \
    template void launch_colswap<T>(hipStream_t, T*, int64_t, int, int, int);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
