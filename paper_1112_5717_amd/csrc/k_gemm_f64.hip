// ffgemm, FP64-carrier form: C <- C + alpha A B mod p on FP64 MFMA.
//
// The matrix product (Algorithm 1 of the paper, used with alpha = -1,
// beta = 1 for the Schur complement update of Algorithm 6 and inside the
// triangular routines) is an exact integer contraction.  Operands are
// loaded in centred form (|x| <= p/2) and accumulated in FP64 MFMA
// registers; every partial sum is an integer of magnitude below 2^53, so the
// FP64 datapath is an exact integer carrier.  The accumulators are reduced
// mod p every `kred_steps` MFMA k-steps (4 products per lane-element each),
// a bound the host derives from p: p + 4 kred_steps (p/2)^2 < 2^53.
//
// Tiling: 128 x 128 output tile per 256-thread workgroup (4 wave64s, 64 x 64
// each as 4 x 4 blocks of v_mfma_f64_16x16x4f64), K tiles of 16 staged
// through LDS (double-buffered, register prefetch of the next tile).
#include "modarith.h"

namespace cup {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int PADM = 16;  // row stride 144 doubles: k-rows land 32 banks apart

template <typename T>
__device__ __forceinline__ double ld_centred(const T* a, double half, double p)
{
    double v = ld_res(a);
    return v > half ? v - p : v;
}

template <typename T>
__global__ __launch_bounds__(256) void ffgemm_f64_kernel(int M, int N, int K,
                                                         const T* __restrict__ A, int64_t lda,
                                                         const T* __restrict__ B, int64_t ldb,
                                                         T* __restrict__ C, int64_t ldc, ModP mp,
                                                         int alpha, int kred_steps)
{
    __shared__ double As[2][BK][BM + PADM];
    __shared__ double Bs[2][BK][BN + PADM];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave >> 1) * 64;
    const int wn = (wave & 1) * 64;
    const int m0 = blockIdx.y * BM;
    const int n0 = blockIdx.x * BN;
    const double P = mp.p, PI = mp.pinv, half = floor(mp.p * 0.5);

    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    double ra[8], rb[8];
    const int ac = tid & 15, ar = tid >> 4;    // A tile: 16 k-columns x 128 rows
    const int bc = tid & 127, br = tid >> 7;   // B tile: 16 k-rows x 128 columns

    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int gm = m0 + ar + 16 * i, gk = k0 + ac;
            ra[i] = (gm < M && gk < K) ? ld_centred(A + (int64_t)gm * lda + gk, half, P) : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int gk = k0 + br + 2 * i, gn = n0 + bc;
            rb[i] = (gk < K && gn < N) ? ld_centred(B + (int64_t)gk * ldb + gn, half, P) : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 8; ++i) As[buf][ac][ar + 16 * i] = ra[i];
#pragma unroll
        for (int i = 0; i < 8; ++i) Bs[buf][br + 2 * i][bc] = rb[i];
    };

    const int ntiles = (K + BK - 1) / BK;
    int since = 0;
    if (ntiles > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int kt = 0; kt < ntiles; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < ntiles) load((kt + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            double a[4], b[4];
            const int kk = ks * 4 + (lane >> 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[buf][kk][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[buf][kk][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            if (++since == kred_steps) {
                since = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[i][j][e] = mod_red(acc[i][j][e], P, PI);
            }
        }
        if (kt + 1 < ntiles) store(buf ^ 1);
        __syncthreads();
    }

    // Epilogue: in each 16x16 block, lane l holds column l%16 of rows
    // l/16 + 4e, e = 0..3 (the v_mfma_f64_16x16x4f64 result layout).
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int gm = m0 + wm + i * 16 + (lane >> 4) + 4 * e;
                int gn = n0 + wn + j * 16 + (lane & 15);
                if (gm < M && gn < N) {
                    T* cp = C + (int64_t)gm * ldc + gn;
                    double s = mod_red(acc[i][j][e], P, PI);
                    double c = ld_res(cp);
                    double r = (alpha < 0) ? c - s : c + s;
                    r = (r < 0.0) ? r + P : r;
                    r = (r >= P) ? r - P : r;
                    st_res(cp, r);
                }
            }
}

}  // namespace

template <typename T>
void launch_ffgemm_f64(hipStream_t s, int M, int N, int K, const T* A, int64_t lda, const T* B,
                       int64_t ldb, T* C, int64_t ldc, ModP mp, int alpha, int kred_steps)
{
    if (M <= 0 || N <= 0 || K <= 0) return;
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
    hipLaunchKernelGGL(ffgemm_f64_kernel<T>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C,
                       ldc, mp, alpha, kred_steps);
    CUP_HIP(hipGetLastError());
}

template void launch_ffgemm_f64<int64_t>(hipStream_t, int, int, int, const int64_t*, int64_t,
                                         const int64_t*, int64_t, int64_t*, int64_t, ModP, int,
                                         int);
template void launch_ffgemm_f64<int8_t>(hipStream_t, int, int, int, const int8_t*, int64_t,
                                        const int8_t*, int64_t, int8_t*, int64_t, ModP, int, int);

}  // namespace cup
