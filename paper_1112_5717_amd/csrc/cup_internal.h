// Internal declarations of libcup: the context, error handling and the
// kernel launchers shared by the host driver.  Not part of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace cup {

// A prime p < 2^26 and its reciprocal; residues travel through kernels as
// doubles, which represent every integer below 2^53 exactly.
struct ModP {
    double p;
    double pinv;
};

enum Form { FORM_AUTO = 0, FORM_FP64 = 1, FORM_I8 = 2, FORM_I8LIMB = 3 };

// Largest p for which a sum of 64 products of canonical residues stays
// below 2^53, i.e. is exact in FP64: 64 (p - 1)^2 < 2^53.
constexpr double kExact64 = 11863283.0;

// Internal failure: unwinds to the C-ABI boundary, which returns `code`.
struct CupError {
    int code;
};

// Every device and pinned-host allocation of the library goes through these
// two calls.  With CUP_FAULT=alloc in the environment they report failure
// without allocating, so that the CUP_ERR_ALLOC path of every entry point can
// be exercised by a test; the variable is read on each allocation.
bool fault_alloc();
inline hipError_t dev_malloc(void** ptr, size_t bytes)
{
    if (fault_alloc()) {
        *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(ptr, bytes);
}
inline hipError_t host_malloc(void** ptr, size_t bytes, unsigned flags)
{
    if (fault_alloc()) {
        *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipHostMalloc(ptr, bytes, flags);
}

#define CUP_HIP(call)                                                   \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) throw ::cup::CupError{-1000 - (int)e_};   \
    } while (0)

// Leaf sizes of the recursions.
constexpr int kLeafRows = 64;   // rows of a CUP leaf (one window-elimination block)
constexpr int kWin = 64;        // window width of the leaf elimination
constexpr int kTriNB = 64;      // order of a triangular leaf block

// Stop reasons of the window elimination.
enum WindowStop { STOP_ROWS = 0, STOP_WINDOW = 1, STOP_ZERO_ROW = 2, STOP_FAIL = 3 };

// Rows of the largest block the rank-deficient (sparse) path takes at once:
// a node of two leaves.  (Nodes of four leaves were measured slower: each
// pivot's update then sweeps up to 255 rows below it, where two-leaf nodes
// leave most of that work to the batched Schur products of their parents.)
constexpr int kSparseNodeRows = 128;

// Rows passed by value to the row-move kernel.
struct MoveList {
    int n;
    int dst[kSparseNodeRows];
    int src[kSparseNodeRows];
};

// A composed permutation of at most kGatherMax positions (columns) or
// kGatherRows positions (rows), passed by value: position dst[k] receives
// what position src[k] held before the launch.
constexpr int kGatherMax = 256;
constexpr int kGatherRows = 128;
struct GatherList {
    int n;
    int dst[kGatherMax];
    int src[kGatherMax];
};

// ---------------------------------------------------------------- launchers
// All operate on row-major views (pointer, leading dimension) on `s`.

// C(MxN) <- C + alpha A(MxK) B(KxN) mod p, alpha = +1 or -1, FP64 MFMA carrier.
template <typename T>
void launch_ffgemm_f64(hipStream_t s, int M, int N, int K, const T* A, int64_t lda,
                       const T* B, int64_t ldb, T* C, int64_t ldc, ModP mp, int alpha,
                       int kred_steps, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// C(MxN) <- C + alpha A(MxK) B(KxN) mod p on INT8 MFMA: limb = 0 for p < 2^7
// (one signed byte per residue), 1 for p <= 2^16 (two signed limbs).  Per K
// chunk of at most ffgemm_i8_kmax(limb) terms: launch_pack_i8 packs A and B
// into `ws` (ffgemm_i8_workspace bytes) and returns the padded depth Kp,
// then launch_mma_i8 multiplies and adds alpha A B to C.
int ffgemm_i8_kmax(int limb);
size_t ffgemm_i8_workspace(int M, int N, int K, int limb);
template <typename T>
int launch_pack_i8(hipStream_t s, int M, int N, int kc, const T* A, int64_t lda, const T* B,
                   int64_t ldb, ModP mp, int limb, int8_t* ws);
template <typename T>
void launch_mma_i8(hipStream_t s, int M, int N, int Kp, const int8_t* ws, T* C, int64_t ldc,
                   ModP mp, int alpha, int limb, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// C(MxN) <- C + alpha A(MxK) B(KxN) mod p in I8LIMB arithmetic (p <= 2^16)
// straight from the residue matrices, without packing launches: for the
// products below the packed kernel's work threshold.
template <typename T>
void launch_mma_i8_direct(hipStream_t s, int M, int N, int K, const T* A, int64_t lda, const T* B,
                          int64_t ldb, T* C, int64_t ldc, ModP mp, int alpha, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr);

// One level of the Strassen-Winograd product (see k_wino.hip), on residue
// matrices: the four sums of the quadrants of X (2 hr x 2 hc; side 0 forms
// S1..S4 from A, side 1 T1..T4 from B) into o1..o4 (hr x hc, dense); zeroing
// of `count` elements; and C's quadrants (2 hm x 2 hn) += alpha times the
// combinations of P1 = W, P6 = X, P5 = Y, P7 = Z (hm x hn, dense).
template <typename T>
void launch_wino_pre(hipStream_t s, const T* X, int64_t ldx, int hr, int hc, int side, int64_t p, T* o1,
                     T* o2, T* o3, T* o4);
template <typename T>
void launch_wino_zero(hipStream_t s, T* X, int64_t count);
template <typename T>
void launch_wino_post(hipStream_t s, T* C, int64_t ldc, int hm, int hn, const T* W, const T* X, const T* Y,
                      const T* Z, int alpha, int64_t p);

// Window elimination of a leaf (see k_panel.hip).  Writes d, stop and the
// chosen columns to `out` (device ints: out[0]=d, out[1]=stop, out[2+a]=col)
// and, when `mail` is given (mapped host memory), the same values to
// mail[0], mail[1], mail[2+a] as 64-bit words (seq << 32) | value, so that
// the host can read them while later launches run.  When a full 64 x 64
// block is decided (64 pivots, 64 rows, 64 columns; p <= kExact64), it also
// writes the dense inverse of its lower pivot block to `winv` and that of
// its unit upper block to `uinv` (each 64 x 64 row-major, either may be null),
// and, when `below` is given and no column was exchanged, G = B U^{-1} for
// the 64 x 64 block B at `below` (the rows under the leaf), in place.  It
// also writes the number of column exchanges to out[kSwapWord].
template <typename T>
void launch_window(hipStream_t s, T* A, int64_t lda, int b, int N, int i0, int t0, int wc,
                   ModP mp, int* out, unsigned long long* mail = nullptr, unsigned seq = 0,
                   double* winv = nullptr, double* uinv = nullptr, T* below = nullptr);

// Index in the window's `out` of the number of column exchanges it made.
constexpr int kSwapWord = 2 + kLeafRows;

// Two-leaf node (see k_tri.hip): after the first leaf's window decided a full
// block with no exchange, U12 = L^{-1} T and H = B - G U12 for every column
// right of the block, in one launch; nothing unless guard[0] == 64 and
// guard[kSwapWord] == 0.
// With int8_mfma (the INT8 forms), p <= 2^16 and int64 storage, on the INT8
// matrix cores.
template <typename T>
void launch_pair_update(hipStream_t s, T* A, int64_t lda, int N, const double* WL, const int* guard,
                        ModP mp, bool int8_mfma = false);

// For each row r in [i0,b): leftmost nonzero column >= t0 (or N), into out[r-i0]
// and, when `mail` is given, into mail[kMailScan + r - i0] as a word tagged
// with `seq` (as the window's result).
template <typename T>
void launch_row_scan(hipStream_t s, const T* A, int64_t lda, int i0, int b, int t0, int N,
                     int* out, unsigned long long* mail = nullptr, unsigned seq = 0);

// Words of the host mailbox: a result count and status, then one word per
// pivot (the window's columns, at most kLeafRows; the sparse path's
// positions, at most kSparseNodeRows), then one word per row (the row scan's
// results, the sparse path's pivot rows).
constexpr int kMailScan = 2 + kSparseNodeRows;
constexpr int kMailWords = kMailScan + kSparseNodeRows;

// The rest of a rank-deficient leaf or node of b <= kSparseNodeRows rows (see
// k_sparse.hip): rows [i0, b) from position t0, one cooperative launch; ws holds sparse_ws_ints() device ints
// and receives the pivot count at ws[kSparseCount], the pivot rows at
// ws[kSparseRows + k] and positions at ws[kSparseCols + k], and posts them
// to the host mailbox, tagged with seq: the count in mail[0], 0 in mail[1],
// the positions in mail[2 + k] and the rows in mail[kMailScan + k] (nothing
// is posted when a grid barrier has waited longer than spin_max polls; ws[2]
// is then set).  The column exchanges t0 + k <-> position k are left to the
// caller (applied in that order to the leaf's rows [0, b)).  The grid
// barrier's words in ws carry over from launch to launch: `reset` zeroes
// them (first use, or after a failure).
constexpr int kSparseCount = 4, kSparseRows = 16, kSparseCols = 16 + kSparseNodeRows;
int sparse_ws_ints();
template <typename T>
int launch_sparse_leaf(hipStream_t s, T* A, int64_t lda, int b, int N, int i0, int t0, ModP mp, int* ws,
                       int spin_max, bool reset, unsigned long long* mail, unsigned seq);

// Swap columns c0 and c1 of rows [0,rows).
template <typename T>
void launch_colswap(hipStream_t s, T* A, int64_t lda, int rows, int c0, int c1);

// Row move: for k ascending, rows dst[k] <- src[k] on columns (dst[k], ncols),
// then zero those columns of src[k].
template <typename T>
void launch_rowmove_list(hipStream_t s, T* A, int64_t lda, int ncols, const MoveList& ml);
template <typename T>
void launch_rowmove_shift(hipStream_t s, T* A, int64_t lda, int ncols, int dst0, int src0,
                          int count);

// Composed column permutation g on rows [0,rows) (g.n <= kGatherMax).
template <typename T>
void launch_colgather(hipStream_t s, T* A, int64_t lda, int rows, const GatherList& g);

// Composed row permutation g on columns [0,cols) (g.n <= kGatherRows).
template <typename T>
void launch_rowgather(hipStream_t s, T* A, int64_t lda, int cols, const GatherList& g);

// In-place transpose of the n x n view at A.
template <typename T>
void launch_transpose_square(hipStream_t s, T* A, int64_t lda, int n);

// D (cols x rows, leading dimension ldd) <- S^T for S rows x cols.
template <typename T>
void launch_transpose(hipStream_t s, const T* S, int64_t lds, T* D, int64_t ldd, int rows, int cols);

// Diagonal blocks of a triangle of order n (uplo 0=Upper 1=Lower, unit 0/1):
// mode 0 writes W[b] = T_bb^{-1}, mode 1 writes W[b] = T_bb (each a dense
// 64 x 64 block of doubles, identity-padded), mode 2 inverts the single
// block of order n <= 64 in place.
template <typename T>
void launch_diag_prep(hipStream_t s, T* A, int64_t lda, int n, int uplo, int unit, int mode,
                      double* W, ModP mp, const int* guard = nullptr, int expect = 0);

// B <- B W (side 1: B is other x nb) or W B (side 0: B is nb x other).
// Two inversions in one launch (mode 0): the diagonal blocks of the n x n
// triangle at A into W, and the single 64 x 64 triangle at A2 (same lda)
// into W2.
template <typename T>
void launch_diag_prep2(hipStream_t s, T* A, int64_t lda, int n, int uplo, int unit, double* W,
                       T* A2, int uplo2, int unit2, double* W2, ModP mp, const int* guard = nullptr,
                       int expect = 0);

// A left apply B <- W B (W 64 x 64, B 64 x other): a 64-row leaf's solve of
// its columns right of its pivots, which a slab launch may carry along.
struct LeftApply {
    const double* W = nullptr;
    void* B = nullptr;
    int64_t ldb = 0;
    int other = 0;
};

// X = B U^{-1} in place for an upper U of order n (n <= 512, a multiple of
// 64) with its 64 x 64 diagonal-block inverses in W; B is rows x n.  With
// int8_mfma (the INT8 forms) and p <= 2^16, int64 storage runs on the INT8
// matrix cores, and then `carry` (if given) is done by the same launch, and
// *carried set; its B must not overlap U, W or this B.  Returns false
// (nothing launched) outside those limits.
template <typename T>
bool launch_tri_slab(hipStream_t s, int n, const T* U, int64_t ldu, const double* W, T* B,
                     int64_t ldb, int rows, ModP mp, bool int8_mfma, const LeftApply* carry = nullptr,
                     bool* carried = nullptr);

template <typename T>
void launch_tri_apply(hipStream_t s, int side, int nb, const double* W, T* B, int64_t ldb,
                      int other, ModP mp, const int* guard = nullptr, int expect = 0);

// [N\T] (N lower with diagonal, T unit upper) <- T.N for an nb x nb block.
template <typename T>
void launch_trulm_leaf(hipStream_t s, int nb, T* A, int64_t lda, ModP mp, int64_t kred);

// B <- -B mod p on a rows x cols view.
template <typename T>
void launch_negate(hipStream_t s, T* B, int64_t ldb, int rows, int cols, ModP mp);

// For j ascending in [0,r): swap A[j][0..j] with A[q[j]][0..j] (inclusive).
template <typename T>
void launch_rowswap_lower(hipStream_t s, T* A, int64_t lda, int r, const int* q);

// *out = (-1)^negate * prod_{i<n} A[i][i] mod p (one workgroup).
template <typename T>
void launch_diag_prod(hipStream_t s, const T* A, int64_t lda, int n, int64_t p, int negate, int64_t* out);

// Nullspace basis from ColEchTrans's block M (r x f at M, f = n - r, the
// negated U1^{-1} U2): row x of N (n x f) is row pos[x] of M when
// pos[x] < r, else the unit vector e_{pos[x] - r}.
template <typename T>
void launch_nullspace_assemble(hipStream_t s, const T* M, int64_t ldm, int r, int f, const int* pos,
                               T* N, int64_t ldn, int n);

// [L\U] (L lower with its diagonal, U unit upper) <- L U on an nb x nb block
// (nb <= 64): the leaf of TRLUM (Algorithm 5, in the variant of Algorithm 9).
template <typename T>
void launch_trlum_leaf(hipStream_t s, int nb, T* A, int64_t lda, ModP mp);

// Count entries outside [0,p) of a rows x cols view (atomic add into *bad).
template <typename T>
void launch_range_check(hipStream_t s, const T* A, int64_t lda, int rows, int cols, int64_t p,
                        int* bad);

// Device copy of a rows x cols view into a dense buffer and back.
template <typename T>
void launch_copy2d(hipStream_t s, const T* src, int64_t lds, T* dst, int64_t ldd, int rows,
                   int cols);

// Batched CUP (one workgroup per matrix, n <= batched_max_n()), all
// descriptors on the device.  `scratch` holds batched_scratch_ints(batch,
// ordered) ints: the classes' work counters, then (when `ordered`) the
// processing order (largest first within each width class).  The launches
// read and write nothing else of the library's, allocate nothing and never
// synchronise, so the sequence can be captured in a graph.
constexpr int kBatchCounters = 64;
int batched_max_n();
size_t batched_scratch_ints(int batch, bool ordered);
void launch_batched_cup(hipStream_t s, int batch, const int64_t* m, const int64_t* n,
                        int64_t* const* A, const int64_t* lda, const int64_t* p, int64_t* rank,
                        int64_t* const* P, int64_t* const* Q, int32_t* info, int* scratch, bool ordered);

}  // namespace cup
