// Leaves of the triangular routines of Section 3.2 (TRSM, TRMM, TRTRI,
// TRULM) on blocks of order <= 64, staged in LDS.
//
// A triangular solve or multiply treats each row (right side, B T^{-1} or
// B T) or each column (left side, T^{-1} B or T B) of B independently, so
// one thread owns one vector.  With Mt(i,s) = T[s][i] on the right and
// T[i][s] on the left, both sides become y = Mt x with Mt effectively lower
// or upper triangular; solves run in the dependency order, multiplies in
// the order that lets y overwrite x.  Dot products accumulate exact integer
// products in FP64 and are reduced mod p every `kred` terms (a bound the
// host derives from p).
#include "modarith.h"

namespace cup {

namespace {

constexpr int NB = kTriNB;
constexpr int VT = 128;  // vectors (threads) per workgroup

// Sum_{s in [s0,s1)} Mt[i][s] x[s] mod p with delayed reduction.
__device__ __forceinline__ double dot_red(const double* mt_row, const double* x, int xstride,
                                          int s0, int s1, double P, double PI, int64_t kred)
{
    double acc = 0.0;
    int64_t cnt = 0;
    for (int s = s0; s < s1; ++s) {
        acc = fma(mt_row[s], x[s * xstride], acc);
        if (++cnt == kred) {
            acc = mod_red(acc, P, PI);
            cnt = 0;
        }
    }
    return mod_red(acc, P, PI);
}

// side: 0 Left, 1 Right.  uplo: 0 Upper, 1 Lower.  op: 0 solve, 1 multiply.
template <typename T>
__global__ __launch_bounds__(VT) void tri_leaf_kernel(int side, int uplo, int unit, int op, int nb,
                                                      const T* __restrict__ Tm, int64_t ldt,
                                                      T* __restrict__ B, int64_t ldb, int other,
                                                      ModP mp, int64_t kred)
{
    __shared__ double Mt[NB][NB + 1];
    __shared__ double dinv[NB];
    __shared__ double X[NB][VT + 1];  // X[i][v]: element i of vector v

    const int tid = threadIdx.x;
    const double P = mp.p, PI = mp.pinv;
    const int v0 = blockIdx.x * VT;
    const int nv = min(VT, other - v0);

    // Mt(i,s) = T[i][s] (Left) or T[s][i] (Right), restricted to the triangle
    const bool upper_eff = (side == 0) ? (uplo == 0) : (uplo == 1);
    for (int idx = tid; idx < nb * nb; idx += VT) {
        int i = idx / nb, s = idx - i * nb;
        int tr = (side == 0) ? i : s, tc = (side == 0) ? s : i;
        bool in = upper_eff ? (s >= i) : (s <= i);
        double v = in ? ld_res(Tm + (int64_t)tr * ldt + tc) : 0.0;
        if (s == i && unit) v = 1.0;
        Mt[i][s] = v;
    }
    // vectors: rows of B (Right) or columns of B (Left)
    if (side == 1) {
        for (int idx = tid; idx < nv * nb; idx += VT) {
            int v = idx / nb, i = idx - v * nb;
            X[i][v] = ld_res(B + (int64_t)(v0 + v) * ldb + i);
        }
    } else {
        for (int idx = tid; idx < nv * nb; idx += VT) {
            int i = idx / nv, v = idx - i * nv;
            X[i][v] = ld_res(B + (int64_t)i * ldb + v0 + v);
        }
    }
    __syncthreads();
    if (op == 0 && !unit)
        for (int i = tid; i < nb; i += VT) dinv[i] = mod_inv(Mt[i][i], P, PI);
    __syncthreads();

    if (tid < nv) {
        double* x = &X[0][tid];
        const int xs = VT + 1;
        if (op == 0) {
            if (!upper_eff) {
                for (int i = 0; i < nb; ++i) {
                    double s = dot_red(Mt[i], x, xs, 0, i, P, PI, kred);
                    double r = x[i * xs] - s;
                    r = (r < 0.0) ? r + P : r;
                    x[i * xs] = unit ? r : mod_mul(r, dinv[i], P, PI);
                }
            } else {
                for (int i = nb - 1; i >= 0; --i) {
                    double s = dot_red(Mt[i], x, xs, i + 1, nb, P, PI, kred);
                    double r = x[i * xs] - s;
                    r = (r < 0.0) ? r + P : r;
                    x[i * xs] = unit ? r : mod_mul(r, dinv[i], P, PI);
                }
            }
        } else {
            if (!upper_eff) {
                for (int i = nb - 1; i >= 0; --i) x[i * xs] = dot_red(Mt[i], x, xs, 0, i + 1, P, PI, kred);
            } else {
                for (int i = 0; i < nb; ++i) x[i * xs] = dot_red(Mt[i], x, xs, i, nb, P, PI, kred);
            }
        }
    }
    __syncthreads();
    if (side == 1) {
        for (int idx = tid; idx < nv * nb; idx += VT) {
            int v = idx / nb, i = idx - v * nb;
            st_res(B + (int64_t)(v0 + v) * ldb + i, X[i][v]);
        }
    } else {
        for (int idx = tid; idx < nv * nb; idx += VT) {
            int i = idx / nv, v = idx - i * nv;
            st_res(B + (int64_t)i * ldb + v0 + v, X[i][v]);
        }
    }
}

// In-place inverse of a triangular block: column j of T^{-1} solves T x = e_j.
template <typename T>
__global__ __launch_bounds__(NB) void trtri_leaf_kernel(int uplo, int unit, int nb, T* __restrict__ A,
                                                        int64_t lda, ModP mp, int64_t kred)
{
    __shared__ double M[NB][NB + 1];
    __shared__ double X[NB][NB + 1];
    __shared__ double dinv[NB];
    const int tid = threadIdx.x;
    const double P = mp.p, PI = mp.pinv;
    for (int idx = tid; idx < nb * nb; idx += NB) {
        int i = idx / nb, s = idx - i * nb;
        bool in = (uplo == 0) ? (s >= i) : (s <= i);
        double v = in ? ld_res(A + (int64_t)i * lda + s) : 0.0;
        if (s == i && unit) v = 1.0;
        M[i][s] = v;
    }
    __syncthreads();
    if (tid < nb) dinv[tid] = unit ? 1.0 : mod_inv(M[tid][tid], P, PI);
    __syncthreads();
    if (tid < nb) {
        const int j = tid;
        double* x = &X[0][j];
        const int xs = NB + 1;
        for (int i = 0; i < nb; ++i) x[i * xs] = (i == j) ? 1.0 : 0.0;
        if (uplo == 1) {
            for (int i = j; i < nb; ++i) {
                double s = dot_red(M[i], x, xs, j, i, P, PI, kred);
                double r = x[i * xs] - s;
                r = (r < 0.0) ? r + P : r;
                x[i * xs] = mod_mul(r, dinv[i], P, PI);
            }
        } else {
            for (int i = j; i >= 0; --i) {
                double s = dot_red(M[i], x, xs, i + 1, j + 1, P, PI, kred);
                double r = x[i * xs] - s;
                r = (r < 0.0) ? r + P : r;
                x[i * xs] = mod_mul(r, dinv[i], P, PI);
            }
        }
    }
    __syncthreads();
    for (int idx = tid; idx < nb * nb; idx += NB) {
        int i = idx / nb, s = idx - i * nb;
        bool write = (uplo == 0) ? (unit ? s > i : s >= i) : (unit ? s < i : s <= i);
        if (write) st_res(A + (int64_t)i * lda + s, X[i][s]);
    }
}

// [N\T] <- T N with T unit upper (strict upper part stored) and N lower
// (diagonal stored): X[i][j] = sum_{s >= max(i,j)} T[i][s] N[s][j].
template <typename T>
__global__ __launch_bounds__(NB) void trulm_leaf_kernel(int nb, T* __restrict__ A, int64_t lda,
                                                        ModP mp, int64_t kred)
{
    __shared__ double Tu[NB][NB + 1];
    __shared__ double Nl[NB][NB + 1];
    __shared__ double X[NB][NB + 1];
    const int tid = threadIdx.x;
    const double P = mp.p, PI = mp.pinv;
    for (int idx = tid; idx < nb * nb; idx += NB) {
        int i = idx / nb, s = idx - i * nb;
        double v = ld_res(A + (int64_t)i * lda + s);
        Tu[i][s] = (s > i) ? v : (s == i ? 1.0 : 0.0);
        Nl[i][s] = (s <= i) ? v : 0.0;
    }
    __syncthreads();
    if (tid < nb) {
        const int j = tid;
        for (int i = 0; i < nb; ++i) {
            int s0 = i > j ? i : j;
            double acc = 0.0;
            int64_t cnt = 0;
            for (int s = s0; s < nb; ++s) {
                acc = fma(Tu[i][s], Nl[s][j], acc);
                if (++cnt == kred) { acc = mod_red(acc, P, PI); cnt = 0; }
            }
            X[i][j] = mod_red(acc, P, PI);
        }
    }
    __syncthreads();
    for (int idx = tid; idx < nb * nb; idx += NB) {
        int i = idx / nb, s = idx - i * nb;
        st_res(A + (int64_t)i * lda + s, X[i][s]);
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

}  // namespace

template <typename T>
void launch_tri_leaf(hipStream_t s, int side, int uplo, int unit, int op, int nb, const T* Tm,
                     int64_t ldt, T* B, int64_t ldb, int other, ModP mp, int64_t kred)
{
    if (nb <= 0 || other <= 0) return;
    hipLaunchKernelGGL(tri_leaf_kernel<T>, dim3((other + VT - 1) / VT), dim3(VT), 0, s, side, uplo,
                       unit, op, nb, Tm, ldt, B, ldb, other, mp, kred);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_trtri_leaf(hipStream_t s, int uplo, int unit, int nb, T* A, int64_t lda, ModP mp,
                       int64_t kred)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL(trtri_leaf_kernel<T>, dim3(1), dim3(NB), 0, s, uplo, unit, nb, A, lda, mp,
                       kred);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_trulm_leaf(hipStream_t s, int nb, T* A, int64_t lda, ModP mp, int64_t kred)
{
    if (nb <= 0) return;
    hipLaunchKernelGGL(trulm_leaf_kernel<T>, dim3(1), dim3(NB), 0, s, nb, A, lda, mp, kred);
    CUP_HIP(hipGetLastError());
}

template <typename T>
void launch_negate(hipStream_t s, T* B, int64_t ldb, int rows, int cols, ModP mp)
{
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(negate_kernel<T>, dim3((cols + 255) / 256, rows), dim3(256), 0, s, B, ldb,
                       rows, cols, mp.p);
    CUP_HIP(hipGetLastError());
}

#define CUP_INST(T)                                                                           \
    template void launch_tri_leaf<T>(hipStream_t, int, int, int, int, int, const T*, int64_t, \
                                     T*, int64_t, int, ModP, int64_t);                        \
    template void launch_trtri_leaf<T>(hipStream_t, int, int, int, T*, int64_t, ModP, int64_t); \
    template void launch_trulm_leaf<T>(hipStream_t, int, T*, int64_t, ModP, int64_t);         \
    template void launch_negate<T>(hipStream_t, T*, int64_t, int, int, ModP);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
