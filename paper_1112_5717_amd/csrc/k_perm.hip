// Data-movement kernels of the CUP driver: column transpositions (A P^T,
// Section 3.3), the row move that brings new U rows up next to the old ones
// (Algorithm 6, final loop), the row swaps of the reduced echelon form
// (Algorithm 8) and of the inverse (P^T X), transposition of a matrix (the
// PLE decomposition of Section 5 through the CUP of the transpose), a range
// check and a 2-D copy.
//
// Column-parallel kernels give each thread one column and walk the rows in
// the order the algorithm prescribes; accesses of one wave touch
// consecutive columns of a row, so they coalesce, and the sequential order
// on each column is the thread's own program order.
//
// A sequence of row or column transpositions is applied as composed
// gathers (GatherList): the host composes the sequence into one permutation
// of the positions it moves, and one launch moves each of them once.  Rows
// go through LDS in 64-column tiles (every access a 64-entry run of a row);
// columns are moved one row per wave, all of a row's loads before its
// stores.
#include <algorithm>

#include "modarith.h"

namespace cup {

namespace {

template <typename T>
__global__ void rowmove_list_kernel(T* __restrict__ A, int64_t lda, int ncols, MoveList ml)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    for (int k = 0; k < ml.n; ++k) {
        int d = ml.dst[k], s = ml.src[k];
        if (c > d && d != s) {
            A[(int64_t)d * lda + c] = A[(int64_t)s * lda + c];
            A[(int64_t)s * lda + c] = 0;
        }
    }
}

// Moves k = 0..count-1: row dst0+k <- row src0+k (src0 > dst0) on columns
// > dst0+k, then zero the source.  A source is never written by an earlier
// move, so each batch of loads may be issued before its stores.
template <typename T>
__global__ void rowmove_shift_kernel(T* __restrict__ A, int64_t lda, int ncols, int dst0, int src0,
                                     int count)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    constexpr int BATCH = 8;
    for (int k0 = 0; k0 < count; k0 += BATCH) {
        T v[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            int k = k0 + u;
            if (k < count && c > dst0 + k) v[u] = A[(int64_t)(src0 + k) * lda + c];
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            int k = k0 + u;
            if (k < count && c > dst0 + k) {
                A[(int64_t)(dst0 + k) * lda + c] = v[u];
                A[(int64_t)(src0 + k) * lda + c] = 0;
            }
        }
    }
}

// Composed column permutation: in every row, column g.dst[k] receives what
// column g.src[k] held (k < g.n <= kGatherMax).  One wave per row, lane l
// moving entries l, l + 64, ...  The values go through LDS: each is written
// there after its load has returned, and the barrier then orders every load
// of the workgroup before any store (a destination may be another lane's
// source).
template <typename T>
__global__ __launch_bounds__(256) void colgather_kernel(T* __restrict__ A, int64_t lda, int rows,
                                                        GatherList g)
{
    constexpr int PER = kGatherMax / 64;
    __shared__ T buf[4][kGatherMax];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t row = (int64_t)blockIdx.x * 4 + w;
    const bool live = row < rows;
    T* r = A + (live ? row : 0) * lda;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int k = lane + 64 * u;
        if (live && k < g.n) buf[w][k] = r[g.src[k]];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int k = lane + 64 * u;
        if (live && k < g.n) r[g.dst[k]] = buf[w][k];
    }
}

// Composed row permutation on columns [0, cols): row g.dst[k] receives what
// row g.src[k] held (k < g.n <= kGatherRows).  A workgroup moves one
// 64-column tile of every listed row through LDS.
template <typename T>
__global__ __launch_bounds__(256) void rowgather_kernel(T* __restrict__ A, int64_t lda, int cols,
                                                        GatherList g)
{
    __shared__ T buf[kGatherRows][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    const bool live = c < cols;
    for (int k = w; k < g.n; k += 4)
        if (live) buf[k][lane] = A[(int64_t)g.src[k] * lda + c];
    __syncthreads();
    for (int k = w; k < g.n; k += 4)
        if (live) A[(int64_t)g.dst[k] * lda + c] = buf[k][lane];
}

// Square transpose in place (n x n): the workgroup of tile pair (bi, bj),
// bi <= bj, stages both 64 x 64 tiles in LDS and writes each transposed
// into the other's place (a diagonal tile into its own).
template <typename T>
__global__ __launch_bounds__(256) void transpose_square_kernel(T* __restrict__ A, int64_t lda, int n)
{
    const int bi = blockIdx.y, bj = blockIdx.x;
    if (bi > bj) return;
    __shared__ T ta[64][65];
    __shared__ T tb[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int y = ty; y < 64; y += 4) {
        int r = bi * 64 + y, c = bj * 64 + tx;
        if (r < n && c < n) ta[y][tx] = A[(int64_t)r * lda + c];
        r = bj * 64 + y;
        c = bi * 64 + tx;
        if (r < n && c < n) tb[y][tx] = A[(int64_t)r * lda + c];
    }
    __syncthreads();
    for (int y = ty; y < 64; y += 4) {
        int r = bi * 64 + y, c = bj * 64 + tx;
        if (r < n && c < n) A[(int64_t)r * lda + c] = tb[tx][y];
        r = bj * 64 + y;
        c = bi * 64 + tx;
        if (bi != bj && r < n && c < n) A[(int64_t)r * lda + c] = ta[tx][y];
    }
}

// D (cols x rows) <- S^T (S rows x cols), 64 x 64 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ S, int64_t lds,
                                                        T* __restrict__ D, int64_t ldd, int rows, int cols)
{
    __shared__ T t[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    for (int y = ty; y < 64; y += 4) {
        const int r = r0 + y, c = c0 + tx;
        if (r < rows && c < cols) t[y][tx] = S[(int64_t)r * lds + c];
    }
    __syncthreads();
    for (int y = ty; y < 64; y += 4) {
        const int dr = c0 + y, dc = r0 + tx;  // D row = S column
        if (dr < cols && dc < rows) D[(int64_t)dr * ldd + dc] = t[tx][y];
    }
}

// Algorithm 8's row exchanges: for j ascending, rows j and q[j] (q[j] >= j,
// increasing) exchange their columns 0..j.  Column c takes the exchanges with
// j >= c, in order; columns are independent, so one wave owns a tile of 64
// columns and walks the exchanges in chunks of 64: the (at most 128) rows a
// chunk touches are loaded into LDS (rows j of the chunk at their offset,
// the other rows q[j] after them), each lane applies the chunk's exchanges
// that reach its column in LDS, and the rows are written back.  Chunks whose
// exchanges are all trivial are skipped.
template <typename T>
__global__ __launch_bounds__(64) void rowswap_lower_kernel(T* __restrict__ A, int64_t lda, int r,
                                                           const int* __restrict__ q)
{
    __shared__ T buf[2 * 64][64];
    __shared__ int slot_q[64];
    const int lane = threadIdx.x, c0 = blockIdx.x * 64, c = c0 + lane;
    for (int j0 = (c0 / 64) * 64; j0 < r; j0 += 64) {
        const int jn = min(64, r - j0);
        const int qj = (lane < jn) ? q[j0 + lane] : j0 + lane;
        if (__ballot(lane < jn && qj != j0 + lane) == 0ull) continue;
        // slot of row q[j]: its own offset when it is a row of the chunk
        slot_q[lane] = (qj - j0 < jn) ? qj - j0 : 64 + lane;
        __syncthreads();
        for (int k = 0; k < jn; ++k) {
            const int row = j0 + k, rq = __shfl(qj, k, 64);
            if (c < r) {
                buf[k][lane] = A[(int64_t)row * lda + c];
                if (rq - j0 >= jn) buf[64 + k][lane] = A[(int64_t)rq * lda + c];
            }
        }
        if (c < r) {
            for (int k = max(0, c - j0); k < jn; ++k) {
                const int sq = slot_q[k];
                if (sq != k) {
                    const T x = buf[k][lane];
                    buf[k][lane] = buf[sq][lane];
                    buf[sq][lane] = x;
                }
            }
            for (int k = 0; k < jn; ++k) {
                const int row = j0 + k, rq = __shfl(qj, k, 64);
                A[(int64_t)row * lda + c] = buf[k][lane];
                if (rq - j0 >= jn) A[(int64_t)rq * lda + c] = buf[64 + k][lane];
            }
        }
        __syncthreads();
    }
}


template <typename T>
__global__ void range_check_kernel(const T* __restrict__ A, int64_t lda, int rows, int cols, int64_t p,
                                   int* bad)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    for (int r = blockIdx.y; r < rows; r += gridDim.y) {
        const int64_t v = (int64_t)A[(int64_t)r * lda + c];
        if (v < 0 || v >= p) atomicAdd(bad, 1);
    }
}

template <typename T>
__global__ void copy2d_kernel(const T* __restrict__ S, int64_t lds, T* __restrict__ D, int64_t ldd,
                              int rows, int cols)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    for (int r = blockIdx.y; r < rows; r += gridDim.y) D[(int64_t)r * ldd + c] = S[(int64_t)r * lds + c];
}

}  // namespace

template <typename T>
void launch_rowmove_list(hipStream_t s, T* A, int64_t lda, int ncols, const MoveList& ml)
{
    if (ml.n <= 0 || ncols <= 0) return;
    hipLaunchKernelGGL(rowmove_list_kernel<T>, dim3((ncols + 255) / 256), dim3(256), 0, s, A, lda,
                       ncols, ml);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_rowmove_shift(hipStream_t s, T* A, int64_t lda, int ncols, int dst0, int src0,
                          int count)
{
    if (count <= 0 || ncols <= 0 || src0 == dst0) return;
    hipLaunchKernelGGL(rowmove_shift_kernel<T>, dim3((ncols + 255) / 256), dim3(256), 0, s, A, lda,
                       ncols, dst0, src0, count);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_colgather(hipStream_t s, T* A, int64_t lda, int rows, const GatherList& g)
{
    if (rows <= 0 || g.n <= 0) return;
    if (g.n > kGatherMax) throw CupError{-3000};
    hipLaunchKernelGGL(colgather_kernel<T>, dim3((rows + 3) / 4), dim3(256), 0, s, A, lda, rows, g);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_rowgather(hipStream_t s, T* A, int64_t lda, int cols, const GatherList& g)
{
    if (cols <= 0 || g.n <= 0) return;
    if (g.n > kGatherRows) throw CupError{-3000};
    hipLaunchKernelGGL(rowgather_kernel<T>, dim3((cols + 63) / 64), dim3(256), 0, s, A, lda, cols, g);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_transpose_square(hipStream_t s, T* A, int64_t lda, int n)
{
    if (n <= 1) return;
    const int nt = (n + 63) / 64;
    hipLaunchKernelGGL(transpose_square_kernel<T>, dim3(nt, nt), dim3(256), 0, s, A, lda, n);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_transpose(hipStream_t s, const T* S, int64_t lds, T* D, int64_t ldd, int rows, int cols)
{
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(transpose_kernel<T>, dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, s, S,
                       lds, D, ldd, rows, cols);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_rowswap_lower(hipStream_t s, T* A, int64_t lda, int r, const int* q)
{
    if (r <= 0) return;
    hipLaunchKernelGGL(rowswap_lower_kernel<T>, dim3((r + 63) / 64), dim3(64), 0, s, A, lda, r, q);
    CUP_HIP(hipGetLastError());
}


template <typename T>
void launch_range_check(hipStream_t s, const T* A, int64_t lda, int rows, int cols, int64_t p,
                        int* bad)
{
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(range_check_kernel<T>, dim3((cols + 255) / 256, std::min(rows, 65535)), dim3(256),
                       0, s, A, lda, rows, cols, p, bad);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_copy2d(hipStream_t s, const T* src, int64_t lds, T* dst, int64_t ldd, int rows, int cols)
{
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(copy2d_kernel<T>, dim3((cols + 255) / 256, std::min(rows, 65535)), dim3(256), 0, s,
                       src, lds, dst, ldd, rows, cols);
    CUP_HIP(hipGetLastError());
}

#define CUP_INST(T)                                                                          \
    template void launch_rowmove_list<T>(hipStream_t, T*, int64_t, int, const MoveList&);    \
    template void launch_rowmove_shift<T>(hipStream_t, T*, int64_t, int, int, int, int);     \
    template void launch_colgather<T>(hipStream_t, T*, int64_t, int, const GatherList&);     \
    template void launch_rowgather<T>(hipStream_t, T*, int64_t, int, const GatherList&);     \
    template void launch_transpose_square<T>(hipStream_t, T*, int64_t, int);                 \
    template void launch_transpose<T>(hipStream_t, const T*, int64_t, T*, int64_t, int, int);\
    template void launch_rowswap_lower<T>(hipStream_t, T*, int64_t, int, const int*);        \
    template void launch_range_check<T>(hipStream_t, const T*, int64_t, int, int, int64_t,   \
                                        int*);                                               \
    template void launch_copy2d<T>(hipStream_t, const T*, int64_t, T*, int64_t, int, int);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
