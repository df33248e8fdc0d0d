// Elementwise steps of one level of the Strassen-Winograd product (the
// exponent log2 7 column of Table 1, Section 4.4), whose seven half-size
// products are ordinary ffgemm calls.  Operands and results are canonical
// residues, so every temporary is reduced to [0, p) where it is formed and
// each of the seven products is an exact product of residue matrices: the
// delayed-reduction bounds of the product kernels apply unchanged.
//
// With X split into quadrants X11, X12, X21, X22:
//   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2
//   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21
//   P1 = A11 B11, P2 = A12 B21, P3 = S4 B22, P4 = A22 T4,
//   P5 = S1 T1,   P6 = S2 T2,   P7 = S3 T3
//   AB = [P1 + P2, P1 + P6 + P5 + P3; P1 + P6 + P7 - P4, P1 + P6 + P7 + P5]
// Each kernel is one pass over its quadrants: runs of one row per wave, so
// every access coalesces; the work is HBM-bound.
#include "modarith.h"

namespace cup {

namespace {

__device__ __forceinline__ int64_t addm(int64_t a, int64_t b, int64_t p)
{
    const int64_t s = a + b;
    return s >= p ? s - p : s;
}
__device__ __forceinline__ int64_t subm(int64_t a, int64_t b, int64_t p)
{
    const int64_t s = a - b;
    return s < 0 ? s + p : s;
}

// The four sums of A's quadrants (side 0: S1..S4) or of B's (side 1:
// T1..T4) for an h_r x h_c quadrant size; out[k] is h_r x h_c, leading
// dimension h_c.
template <typename T>
__global__ __launch_bounds__(256) void wino_pre_kernel(const T* __restrict__ X, int64_t ldx, int hr, int hc,
                                                       int side, int64_t p, T* __restrict__ o1,
                                                       T* __restrict__ o2, T* __restrict__ o3,
                                                       T* __restrict__ o4)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= hc) return;
    for (int i = blockIdx.y; i < hr; i += gridDim.y) {
        const int64_t x11 = X[(int64_t)i * ldx + j], x12 = X[(int64_t)i * ldx + hc + j];
        const int64_t x21 = X[(int64_t)(i + hr) * ldx + j], x22 = X[(int64_t)(i + hr) * ldx + hc + j];
        int64_t a, b, c, d;
        if (side == 0) {
            a = addm(x21, x22, p);  // S1
            b = subm(a, x11, p);       // S2
            c = subm(x11, x21, p);     // S3
            d = subm(x12, b, p);       // S4
        } else {
            a = subm(x12, x11, p);     // T1
            b = subm(x22, a, p);       // T2
            c = subm(x22, x12, p);     // T3
            d = subm(b, x21, p);       // T4
        }
        const int64_t o = (int64_t)i * hc + j;
        o1[o] = (T)a;
        o2[o] = (T)b;
        o3[o] = (T)c;
        o4[o] = (T)d;
    }
}

// Zero `count` consecutive elements (the product temporaries, which the
// products accumulate into).
template <typename T>
__global__ __launch_bounds__(256) void wino_zero_kernel(T* __restrict__ X, int64_t count)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
        X[e] = (T)0;
}

// C's quadrants += alpha (combinations of W = P1, X = P6, Y = P5, Z = P7);
// P2, P3 and P4 were accumulated into C11, C12 and C21 by their products:
//   C11 += a W, C12 += a (W + X + Y), C21 += a (W + X + Z),
//   C22 += a (W + X + Z + Y).
template <typename T>
__global__ __launch_bounds__(256) void wino_post_kernel(T* __restrict__ C, int64_t ldc, int hm, int hn,
                                                        const T* __restrict__ W, const T* __restrict__ Xp,
                                                        const T* __restrict__ Y, const T* __restrict__ Z,
                                                        int alpha, int64_t p)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= hn) return;
    for (int i = blockIdx.y; i < hm; i += gridDim.y) {
        const int64_t o = (int64_t)i * hn + j;
        const int64_t w = W[o], x = Xp[o], y = Y[o], z = Z[o];
        const int64_t u2 = addm(w, x, p);   // P1 + P6
        const int64_t u3 = addm(u2, z, p);  // + P7
        int64_t d[4] = {w, addm(u2, y, p), u3, addm(u3, y, p)};
        T* c[4] = {C + (int64_t)i * ldc + j, C + (int64_t)i * ldc + hn + j, C + (int64_t)(i + hm) * ldc + j,
                   C + (int64_t)(i + hm) * ldc + hn + j};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t v = *c[q];
            *c[q] = (T)(alpha > 0 ? addm(v, d[q], p) : subm(v, d[q], p));
        }
    }
}

}  // namespace

template <typename T>
void launch_wino_pre(hipStream_t s, const T* X, int64_t ldx, int hr, int hc, int side, int64_t p, T* o1,
                     T* o2, T* o3, T* o4)
{
    if (hr <= 0 || hc <= 0) return;
    hipLaunchKernelGGL(wino_pre_kernel<T>, dim3((hc + 255) / 256, hr < 65535 ? hr : 65535), dim3(256), 0, s,
                       X, ldx, hr, hc, side, p, o1, o2, o3, o4);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_wino_zero(hipStream_t s, T* X, int64_t count)
{
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(wino_zero_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, X, count);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_wino_post(hipStream_t s, T* C, int64_t ldc, int hm, int hn, const T* W, const T* X, const T* Y,
                      const T* Z, int alpha, int64_t p)
{
    if (hm <= 0 || hn <= 0) return;
    hipLaunchKernelGGL(wino_post_kernel<T>, dim3((hn + 255) / 256, hm < 65535 ? hm : 65535), dim3(256), 0, s,
                       C, ldc, hm, hn, W, X, Y, Z, alpha, p);
    CUP_HIP(hipGetLastError());
}

#define CUP_INST(T)                                                                                     \
    template void launch_wino_pre<T>(hipStream_t, const T*, int64_t, int, int, int, int64_t, T*, T*, T*, \
                                     T*);                                                               \
    template void launch_wino_zero<T>(hipStream_t, T*, int64_t);                                        \
    template void launch_wino_post<T>(hipStream_t, T*, int64_t, int, int, const T*, const T*, const T*, \
                                      const T*, int, int64_t);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
