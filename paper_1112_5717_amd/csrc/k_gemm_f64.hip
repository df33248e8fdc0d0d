// ffgemm, FP64-carrier form: C <- C + alpha A B mod p on FP64 MFMA.
//
// The matrix product (Algorithm 1 of the paper, used with alpha = -1,
// beta = 1 for the Schur complement update of Algorithm 6 and inside the
// triangular routines) is an exact integer contraction.  Operands are
// loaded in centred form (|x| <= p/2) and accumulated in FP64 MFMA
// registers; every partial sum is an integer of magnitude below 2^53, so the
// FP64 datapath is an exact integer carrier.  The kernel reduces mod p only
// in its epilogue: the host splits K into chunks of at most kmax terms with
// kmax (p/2)^2 < 2^53 - p (over two million terms for p = 65521, 512 for
// p < 2^23), one launch per chunk.
//
// Tiling: 128 x 128 output tile per 256-thread workgroup (4 wave64s, 64 x 64
// each as 4 x 4 blocks of v_mfma_f64_16x16x4f64), K tiles of 16 staged
// through LDS (double-buffered, register prefetch of the next tile); products
// too small to give two such workgroups per CU take 64 x 64 tiles with K in
// steps of 128 (or all of K <= 64 at once), each step's loads in flight
// together.
#include <hip/hip_ext.h>

#include "modarith.h"

namespace cup {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int BK = 16;
constexpr int PADM = 16;  // LDS row stride BM+16 doubles: adjacent k-rows 16 double-banks apart

// The residue as a 32-bit integer (int64 storage: its low word).
__device__ __forceinline__ int ld_raw(const int64_t* a) { return *reinterpret_cast<const int*>(a); }
__device__ __forceinline__ int ld_raw(const int8_t* a) { return (int)*a; }

__device__ __forceinline__ double centre(double v, double half, double p)
{
    return v > half ? v - p : v;
}

// The epilogue of the lane's outputs in TM x TN 16 x 16 blocks (rows
// gm0 + 16 i + 4 e, columns gn0 + 16 j): epi_load reads every C entry from a
// clamped, always valid address, so that all the loads are in flight
// together (a load under the bounds test would wait on each one in turn);
// epi_store reduces the sums to canonical residues and stores
// C + alpha S mod p, predicated on the bounds.
template <typename T, int TM, int TN>
__device__ __forceinline__ void epi_load(int (&cv)[TM][TN][4], int gm0, int gn0, int M, int N,
                                         const T* C, int64_t ldc)
{
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gm = min(gm0 + i * 16 + 4 * e, M - 1), gn = min(gn0 + j * 16, N - 1);
                cv[i][j][e] = ld_raw(C + (int64_t)gm * ldc + gn);
            }
}

template <typename T, int TM, int TN>
__device__ __forceinline__ void epi_store(const v4d (&acc)[TM][TN], const int (&cv)[TM][TN][4],
                                          int gm0, int gn0, int M, int N, T* C, int64_t ldc,
                                          ModP mp, int alpha)
{
    const int ip = (int)mp.p;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gm = gm0 + i * 16 + 4 * e, gn = gn0 + j * 16;
                const int sv = (int)mod_red(acc[i][j][e], mp.p, mp.pinv);
                if (gm < M && gn < N) {
                    int r = (alpha < 0) ? cv[i][j][e] - sv : cv[i][j][e] + sv;
                    r = (r < 0) ? r + ip : r;
                    r = (r >= ip) ? r - ip : r;
                    C[(int64_t)gm * ldc + gn] = (T)r;
                }
            }
}

// Workgroup tile BM x BN computed by 4 waves arranged 2 x 2, each a
// (BM/2) x (BN/2) block of 16x16 MFMA tiles.
template <typename T, int BM, int BN>
__global__ __launch_bounds__(256, 2) void ffgemm_f64_kernel(int M, int N, int K,
                                                         const T* __restrict__ A, int64_t lda,
                                                         const T* __restrict__ B, int64_t ldb,
                                                         T* __restrict__ C, int64_t ldc, ModP mp,
                                                         int alpha)
{
    constexpr int TM = BM / 32, TN = BN / 32;      // 16x16 tiles per wave
    __shared__ double As[2][BK][BM + PADM];
    __shared__ double Bs[2][BK][BN + PADM];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave >> 1) * (BM / 2);
    const int wn = (wave & 1) * (BN / 2);
    const int m0 = blockIdx.y * BM;
    const int n0 = blockIdx.x * BN;
    const double P = mp.p, half = floor(mp.p * 0.5);

    v4d acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    // Rows beyond M and columns beyond N read a clamped (valid) address: they
    // only feed outputs that are never stored.  K is zero-padded.
    constexpr int NA = BM / 16;                // A loads per thread: 16 rows per pass
    constexpr int BSTEP = 256 / BN;            // B rows per pass
    constexpr int NB_ = BK / BSTEP;            // B loads per thread
    const int ac = tid & 15, ar = tid >> 4;    // A tile: 16 k-columns x BM rows
    const int bc = tid % BN, br = tid / BN;    // B tile: 16 k-rows x BN columns
    const T* pa[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) pa[i] = A + (int64_t)min(m0 + ar + 16 * i, M - 1) * lda + ac;
    const T* pb = B + (int64_t)br * ldb + min(n0 + bc, N - 1);
    const int64_t ldbs = BSTEP * ldb;
    // raw residues of the next tile; converted to centred doubles only when
    // they are written to LDS, after the MFMAs of the current tile
    int ra[NA], rb[NB_];

    auto load_full = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) ra[i] = ld_raw(pa[i] + k0);
#pragma unroll
        for (int i = 0; i < NB_; ++i) rb[i] = ld_raw(pb + (int64_t)k0 * ldb + i * ldbs);
    };
    auto load_tail = [&](int k0) {
        // out-of-range k reads a valid address and is zeroed
        const bool ka = k0 + ac < K;
        const int ka_off = ka ? k0 : K - 1 - ac;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            int x = ld_raw(pa[i] + ka_off);
            ra[i] = ka ? x : 0;
        }
#pragma unroll
        for (int i = 0; i < NB_; ++i) {
            const bool kb = k0 + br + BSTEP * i < K;
            const int64_t off = kb ? (int64_t)k0 * ldb + i * ldbs : (int64_t)(K - 1 - br) * ldb;
            int x = ld_raw(pb + off);
            rb[i] = kb ? x : 0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < NA; ++i) As[buf][ac][ar + 16 * i] = centre((double)ra[i], half, P);
#pragma unroll
        for (int i = 0; i < NB_; ++i) Bs[buf][br + BSTEP * i][bc] = centre((double)rb[i], half, P);
    };

    const int ntiles = (K + BK - 1) / BK;
    const int nfull = K / BK;
    if (nfull > 0) load_full(0);
    else load_tail(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < ntiles; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nfull) load_full((kt + 1) * BK);
        else if (kt + 1 < ntiles) load_tail((kt + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            double a[TM], b[TN];
            const int kk = ks * 4 + (lane >> 4);
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[buf][kk][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[buf][kk][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < ntiles) store(buf ^ 1);
        __syncthreads();
    }

    // Epilogue: in each 16x16 block, lane l holds column l%16 of rows
    // l/16 + 4e, e = 0..3 (the v_mfma_f64_16x16x4f64 result layout).
    const int gn0 = n0 + wn + (lane & 15);
    const int gm0 = m0 + wm + (lane >> 4);
    int cv[TM][TN][4];
    epi_load<T, TM, TN>(cv, gm0, gn0, M, N, C, ldc);
    epi_store<T, TM, TN>(acc, cv, gm0, gn0, M, N, C, ldc, mp, alpha);
}

// Products with K <= 64 (the thin updates of the triangular recursion and of
// the lowest CUP levels): one 64 x 64 tile per workgroup with the whole
// K-extent staged at once.  Every global load of the tile (A, B and the C
// entries the epilogue updates) is issued before the first wait, so the
// launch pays one memory latency instead of one per 16-deep K tile.
constexpr int SK = 64;  // largest K of this variant

template <typename T>
__global__ __launch_bounds__(256) void ffgemm_f64_k64_kernel(int M, int N, int K,
                                                           const T* __restrict__ A, int64_t lda,
                                                           const T* __restrict__ B, int64_t ldb,
                                                           T* __restrict__ C, int64_t ldc, ModP mp,
                                                           int alpha)
{
    constexpr int BM = 64, BN = 64, TM = 2, TN = 2;
    __shared__ double As[SK][BM + PADM];
    __shared__ double Bs[SK][BN + PADM];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const double P = mp.p, half = floor(mp.p * 0.5);

    // C entries of this thread's outputs (the MFMA result layout: lane l
    // holds column l % 16 of rows l / 16 + 4e of each 16 x 16 block)
    const int gn0 = n0 + wn + (lane & 15), gm0 = m0 + wm + (lane >> 4);
    int rc[TM][TN][4];
    epi_load<T, TM, TN>(rc, gm0, gn0, M, N, C, ldc);
    // A: 64 rows x 64 k, thread (row ar + 16 i, k = ac + 16 u); B: 64 k x 64 cols
    const int ac = tid & 15, ar = tid >> 4;
    int ra[4][4], rb[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const T* pa = A + (int64_t)min(m0 + ar + 16 * i, M - 1) * lda;
#pragma unroll
        for (int u = 0; u < 4; ++u) ra[i][u] = ld_raw(pa + min(ac + 16 * u, K - 1));
    }
    const int bc = tid & 63, br = tid >> 6;
#pragma unroll
    for (int u = 0; u < 16; ++u)
        rb[u] = ld_raw(B + (int64_t)min(br + 4 * u, K - 1) * ldb + min(n0 + bc, N - 1));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = ac + 16 * u;
            As[k][ar + 16 * i] = (k < K) ? centre((double)ra[i][u], half, P) : 0.0;
        }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int k = br + 4 * u;
        Bs[k][bc] = (k < K) ? centre((double)rb[u], half, P) : 0.0;
    }
    __syncthreads();

    v4d acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int nks = (K + 3) >> 2;
    for (int ks = 0; ks < nks; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        double a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[kk][wm + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[kk][wn + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }

    epi_store<T, TM, TN>(acc, rc, gm0, gn0, M, N, C, ldc, mp, alpha);
}

// Products too small for two 128 x 128 workgroups per CU, with K > 64 (the
// Schur complement updates of the low CUP levels, K = 128 to 512): 64 x 64
// tiles, K in steps of 128.  All the loads of the next step are in flight
// while the current step's 128 MFMAs per wave run, so a step pays its memory
// latency once; the residues are staged in LDS as centred 32-bit integers
// (80 KB for both operands) and converted to doubles as they are read.
constexpr int DK = 128;
constexpr int DPAD = 16;  // LDS row stride 64 + 16 ints: adjacent k-rows 16 banks apart

template <typename T>
__global__ __launch_bounds__(256, 2) void ffgemm_f64_deep_kernel(int M, int N, int K,
                                                               const T* __restrict__ A, int64_t lda,
                                                               const T* __restrict__ B, int64_t ldb,
                                                               T* __restrict__ C, int64_t ldc, ModP mp,
                                                               int alpha)
{
    constexpr int BM = 64, BN = 64, TM = 2, TN = 2;
    __shared__ int As[DK][BM + DPAD];
    __shared__ int Bs[DK][BN + DPAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int ip = (int)mp.p, ihalf = ip / 2;

    // A: thread (row ar + 16 i, k = ac + 16 u); B: (k = br + 4 u, column bc).
    // Rows beyond M and columns beyond N read a clamped (valid) address and
    // feed only outputs that are never stored; k beyond K is zeroed.
    const int ac = tid & 15, ar = tid >> 4, bc = tid & 63, br = tid >> 6;
    const T* pa[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) pa[i] = A + (int64_t)min(m0 + ar + 16 * i, M - 1) * lda;
    const T* pb = B + min(n0 + bc, N - 1);
    int ra[4][8], rb[32];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int u = 0; u < 8; ++u) ra[i][u] = ld_raw(pa[i] + min(k0 + ac + 16 * u, K - 1));
#pragma unroll
        for (int u = 0; u < 32; ++u) rb[u] = ld_raw(pb + (int64_t)min(k0 + br + 4 * u, K - 1) * ldb);
    };
    auto centre_i = [&](int x, bool in) { return in ? ((x > ihalf) ? x - ip : x) : 0; };
    auto store = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = ac + 16 * u;
                As[k][ar + 16 * i] = centre_i(ra[i][u], k0 + k < K);
            }
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int k = br + 4 * u;
            Bs[k][bc] = centre_i(rb[u], k0 + k < K);
        }
    };

    v4d acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    const int nk = (K + DK - 1) / DK;
    load(0);
    store(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load((kt + 1) * DK);
#pragma unroll 8
        for (int ks = 0; ks < DK / 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            double a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = (double)As[kk][wm + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = (double)Bs[kk][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) {
            __syncthreads();
            store((kt + 1) * DK);
            __syncthreads();
        }
    }

    const int gn0 = n0 + wn + (lane & 15), gm0 = m0 + wm + (lane >> 4);
    int cv[TM][TN][4];
    epi_load<T, TM, TN>(cv, gm0, gn0, M, N, C, ldc);
    epi_store<T, TM, TN>(acc, cv, gm0, gn0, M, N, C, ldc, mp, alpha);
}

}  // namespace

template <typename T>
void launch_ffgemm_f64(hipStream_t s, int M, int N, int K, const T* A, int64_t lda, const T* B,
                       int64_t ldb, T* C, int64_t ldc, ModP mp, int alpha, int kred_steps,
                       hipEvent_t ev0, hipEvent_t ev1)
{
    if (M <= 0 || N <= 0 || K <= 0) return;
    // products per lane-element before the sum could reach 2^53 (>= 4)
    const int64_t kmax = std::max<int64_t>(4, std::min<int64_t>(4 * (int64_t)kred_steps, K));
    if (K <= SK && K <= kmax) {
        dim3 grid((N + 63) / 64, (M + 63) / 64);
        hipExtLaunchKernelGGL((ffgemm_f64_k64_kernel<T>), grid, dim3(256), 0, s, ev0, ev1, 0, M, N, K,
                              A, lda, B, ldb, C, ldc, mp, alpha);
        CUP_HIP(hipGetLastError());
        return;
    }
    // 128 x 128 tiles when they give at least two workgroups per CU, else 64 x 64
    const bool big = (int64_t)((M + 127) / 128) * ((N + 127) / 128) >= 512;
    for (int64_t k0 = 0; k0 < K; k0 += kmax) {
        const int kc = (int)std::min<int64_t>(kmax, K - k0);
        // timing events (optional) open with the first chunk's dispatch and
        // close with the last one's
        hipEvent_t a = (k0 == 0) ? ev0 : nullptr;
        hipEvent_t b = (k0 + kmax >= K) ? ev1 : nullptr;
        if (big) {
            dim3 grid((N + 127) / 128, (M + 127) / 128);
            hipExtLaunchKernelGGL((ffgemm_f64_kernel<T, 128, 128>), grid, dim3(256), 0, s, a, b, 0, M,
                                  N, kc, A + k0, lda, B + k0 * ldb, ldb, C, ldc, mp, alpha);
        } else {
            dim3 grid((N + 63) / 64, (M + 63) / 64);
            hipExtLaunchKernelGGL((ffgemm_f64_deep_kernel<T>), grid, dim3(256), 0, s, a, b, 0, M, N,
                                  kc, A + k0, lda, B + k0 * ldb, ldb, C, ldc, mp, alpha);
        }
        CUP_HIP(hipGetLastError());
    }
}

template void launch_ffgemm_f64<int64_t>(hipStream_t, int, int, int, const int64_t*, int64_t,
                                         const int64_t*, int64_t, int64_t*, int64_t, ModP, int,
                                         int, hipEvent_t, hipEvent_t);
template void launch_ffgemm_f64<int8_t>(hipStream_t, int, int, int, const int8_t*, int64_t,
                                        const int8_t*, int64_t, int8_t*, int64_t, ModP, int, int,
                                        hipEvent_t, hipEvent_t);

}  // namespace cup
