// Kernels of the invariants that the CUP decomposition yields (Section 4.4):
// the determinant as the signed product of the pivots, and the assembly of
// a nullspace basis from the column echelon transformation (Section 3.4).
#include "modarith.h"

namespace cup {

namespace {

// Product of the n diagonal entries mod p, negated if `negate`: each thread
// multiplies a strided share (products of two residues stay below 2^52,
// exact in int64), then a tree of modular products in LDS.
template <typename T>
__global__ __launch_bounds__(1024) void diag_prod_kernel(const T* __restrict__ A, int64_t lda, int n,
                                                         int64_t p, int negate, int64_t* out)
{
    __shared__ int64_t s[1024];
    const int tid = threadIdx.x;
    int64_t acc = 1 % p;
    for (int i = tid; i < n; i += 1024) acc = (acc * (int64_t)A[(int64_t)i * lda + i]) % p;
    s[tid] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) s[tid] = (s[tid] * s[tid + w]) % p;
        __syncthreads();
    }
    if (tid == 0) out[0] = negate ? (p - s[0]) % p : s[0];
}

// Row x of N (one grid row per x, strided over the grid): row pos[x] of M if
// it is one of the r pivot positions, else the unit vector e_{pos[x] - r}.
// Reads and writes are runs of one row each, so they coalesce.
template <typename T>
__global__ void nullspace_kernel(const T* __restrict__ M, int64_t ldm, int r, int f,
                                 const int* __restrict__ pos, T* __restrict__ N, int64_t ldn, int n)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= f) return;
    for (int x = blockIdx.y; x < n; x += gridDim.y) {
        const int c = pos[x];
        const T v = (c < r) ? M[(int64_t)c * ldm + s] : (T)((c - r == s) ? 1 : 0);
        N[(int64_t)x * ldn + s] = v;
    }
}

}  // namespace

template <typename T>
void launch_diag_prod(hipStream_t s, const T* A, int64_t lda, int n, int64_t p, int negate, int64_t* out)
{
    hipLaunchKernelGGL(diag_prod_kernel<T>, dim3(1), dim3(1024), 0, s, A, lda, n, p, negate, out);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_nullspace_assemble(hipStream_t s, const T* M, int64_t ldm, int r, int f, const int* pos,
                               T* N, int64_t ldn, int n)
{
    if (f <= 0 || n <= 0) return;
    hipLaunchKernelGGL(nullspace_kernel<T>, dim3((f + 255) / 256, n < 65535 ? n : 65535), dim3(256), 0, s,
                       M, ldm, r, f, pos, N, ldn, n);
    CUP_HIP(hipGetLastError());
}

#define CUP_INST(T)                                                                                 \
    template void launch_diag_prod<T>(hipStream_t, const T*, int64_t, int, int64_t, int, int64_t*); \
    template void launch_nullspace_assemble<T>(hipStream_t, const T*, int64_t, int, int, const int*, \
                                               T*, int64_t, int);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
