// Data-movement kernels of the CUP driver: column transpositions (A P^T,
// Section 3.3), the row move that brings new U rows up next to the old ones
// (Algorithm 6, final loop), the row swaps of the reduced echelon form
// (Algorithm 8) and of the inverse (P^T X), a range check and a 2-D copy.
//
// Column-parallel kernels give each thread one column and walk the rows in
// the order the algorithm prescribes; accesses of one wave touch
// consecutive columns of a row, so they coalesce, and the sequential order
// on each column is the thread's own program order.
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

// Column transpositions (a[k], b[k]) applied in order, one thread per row.
template <typename T>
__global__ void coltransp_kernel(T* __restrict__ A, int64_t lda, int rows, TranspList tl)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    T* row = A + (int64_t)r * lda;
    for (int k = 0; k < tl.n; ++k) {
        int x = tl.a[k], y = tl.b[k];
        T t = row[x];
        row[x] = row[y];
        row[y] = t;
    }
}

template <typename T>
__global__ void rowswap_lower_kernel(T* __restrict__ A, int64_t lda, int r, const int* __restrict__ q)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= r) return;
    for (int j = c; j < r; ++j) {
        int qj = q[j];
        if (qj != j) {
            T t = A[(int64_t)j * lda + c];
            A[(int64_t)j * lda + c] = A[(int64_t)qj * lda + c];
            A[(int64_t)qj * lda + c] = t;
        }
    }
}

template <typename T>
__global__ void rowswap_desc_kernel(T* __restrict__ A, int64_t lda, int r, int cols,
                                    const int* __restrict__ pv)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    for (int t = r - 1; t >= 0; --t) {
        int j = pv[t];
        if (j != t) {
            T x = A[(int64_t)t * lda + c];
            A[(int64_t)t * lda + c] = A[(int64_t)j * lda + c];
            A[(int64_t)j * lda + c] = x;
        }
    }
}

template <typename T>
__global__ void range_check_kernel(const T* __restrict__ A, int64_t lda, int rows, int cols, int64_t p,
                                   int* bad)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (c < cols && r < rows) {
        int64_t v = (int64_t)A[(int64_t)r * lda + c];
        if (v < 0 || v >= p) atomicAdd(bad, 1);
    }
}

template <typename T>
__global__ void copy2d_kernel(const T* __restrict__ S, int64_t lds, T* __restrict__ D, int64_t ldd,
                              int rows, int cols)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (c < cols && r < rows) D[(int64_t)r * ldd + c] = S[(int64_t)r * lds + c];
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
void launch_coltransp(hipStream_t s, T* A, int64_t lda, int rows, const TranspList& tl)
{
    if (rows <= 0 || tl.n <= 0) return;
    hipLaunchKernelGGL(coltransp_kernel<T>, dim3((rows + 127) / 128), dim3(128), 0, s, A, lda, rows,
                       tl);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_rowswap_lower(hipStream_t s, T* A, int64_t lda, int r, const int* q)
{
    if (r <= 0) return;
    hipLaunchKernelGGL(rowswap_lower_kernel<T>, dim3((r + 255) / 256), dim3(256), 0, s, A, lda, r, q);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_rowswap_desc(hipStream_t s, T* A, int64_t lda, int r, int cols, const int* pv)
{
    if (r <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(rowswap_desc_kernel<T>, dim3((cols + 255) / 256), dim3(256), 0, s, A, lda, r,
                       cols, pv);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_range_check(hipStream_t s, const T* A, int64_t lda, int rows, int cols, int64_t p,
                        int* bad)
{
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(range_check_kernel<T>, dim3((cols + 255) / 256, rows), dim3(256), 0, s, A, lda,
                       rows, cols, p, bad);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_copy2d(hipStream_t s, const T* src, int64_t lds, T* dst, int64_t ldd, int rows, int cols)
{
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(copy2d_kernel<T>, dim3((cols + 255) / 256, rows), dim3(256), 0, s, src, lds, dst,
                       ldd, rows, cols);
    CUP_HIP(hipGetLastError());
}

#define CUP_INST(T)                                                                          \
    template void launch_rowmove_list<T>(hipStream_t, T*, int64_t, int, const MoveList&);    \
    template void launch_rowmove_shift<T>(hipStream_t, T*, int64_t, int, int, int, int);     \
    template void launch_coltransp<T>(hipStream_t, T*, int64_t, int, const TranspList&);     \
    template void launch_rowswap_lower<T>(hipStream_t, T*, int64_t, int, const int*);        \
    template void launch_rowswap_desc<T>(hipStream_t, T*, int64_t, int, int, const int*);    \
    template void launch_range_check<T>(hipStream_t, const T*, int64_t, int, int, int64_t,   \
                                        int*);                                               \
    template void launch_copy2d<T>(hipStream_t, const T*, int64_t, T*, int64_t, int, int);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
