// Host side of libcup: the in-place recursive drivers of Sections 3.2-3.5.
//
// Every routine works on row-major views (pointer, leading dimension) of
// the caller's matrix and allocates nothing of the matrix's size.  Memory
// besides the matrix (all of it reported by cup_workspace_bytes):
//   - O(m + n) bookkeeping (transposition lists, small result buffers);
//   - the ffgemm workspace of the INT8 forms (packed operands), which
//     Definition 1 (Section 3.1) allows inside matrix multiplication;
//   - two buffers outside matrix multiplication, a deliberate departure from
//     Definition 1's O(1) extra field elements: the dense inverses of the
//     64 x 64 diagonal blocks of the triangle being solved (ceil(n/64) blocks
//     of 32 KiB, at least 64 blocks, so n/2 KiB for large n) and the cache
//     of the inverses of U's 64 x 64 diagonal blocks (floor(min(m,n)/64)
//     blocks of 32 KiB, 4 MiB at r = 8192).  Both are O(n) blocks, i.e.
//     O(n * 64) field elements against the mn of the matrix.
// The recursions split on multiples of the leaf sizes; outputs do not depend
// on the split point because the pivot rule fixes P, and P fixes C and U
// (Section 2.2, Proposition 1).
#pragma once

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "cup_internal.h"

namespace cup {

enum { LEFT = 0, RIGHT = 1 };
enum { UPPER = 0, LOWER = 1 };
enum { SOLVE = 0, MULT = 1 };

// Kernel timing with HIP events (enabled by cup_profile): every ffgemm and
// leaf-window launch is bracketed by two events on the launch stream; the
// elapsed times are summed after the call has synchronised.
constexpr int kProfKinds = 4;  // 0 ffgemm FP64, 1 window, 2 ffgemm INT8 MFMA, 3 INT8 packing

struct ProfRec {
    int kind;            // 0 ffgemm FP64, 1 window, 2 ffgemm INT8
    double flops;        // algorithmic operations of the launch
    double bytes;        // algorithmic bytes of the launch
    hipEvent_t a, b;
};

struct Profiler {
    bool on = false;
    unsigned mask = 0;  // kernel classes timed (bit k: class k)
    bool want(int kind) const { return on && ((mask >> kind) & 1u); }
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<ProfRec> recs;
    double launches[kProfKinds] = {}, ms[kProfKinds] = {}, flops[kProfKinds] = {},
           bytes[kProfKinds] = {};

    void reset()
    {
        for (int k = 0; k < kProfKinds; ++k) launches[k] = ms[k] = flops[k] = bytes[k] = 0;
    }
    hipEvent_t next()
    {
        if (used == pool.size()) {
            hipEvent_t e;
            CUP_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin(hipStream_t s, int kind, double f, double by)
    {
        ProfRec r{kind, f, by, next(), next()};
        CUP_HIP(hipEventRecord(r.a, s));
        recs.push_back(r);
    }
    void end(hipStream_t s) { CUP_HIP(hipEventRecord(recs.back().b, s)); }
    // An event pair for a launch that records it itself (hipExtLaunchKernel):
    // the interval is then the kernel's own execution, as a profiler sees it.
    ProfRec& open(int kind, double f, double by)
    {
        recs.push_back(ProfRec{kind, f, by, next(), next()});
        return recs.back();
    }
    // After the stream has synchronised.  The pending records are taken out
    // first, so that a failure leaves nothing behind for the next call; a
    // pair whose events were not both recorded (a launch that failed) is
    // skipped.
    void collect()
    {
        std::vector<ProfRec> done;
        done.swap(recs);
        used = 0;
        for (auto& r : done) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) continue;
            launches[r.kind] += 1;
            ms[r.kind] += t;
            flops[r.kind] += r.flops;
            bytes[r.kind] += r.bytes;
        }
    }
    // Forget the records of a call that failed before collect().
    void drop()
    {
        recs.clear();
        used = 0;
    }
};

// Device scratch owned by the library (grown on demand, freed by
// cup_finalize): the dense 64 x 64 diagonal blocks of the triangular leaves.
struct Workspace {
    double* tri = nullptr;
    size_t tri_cap = 0;  // doubles
    double* uc = nullptr;  // inverses of the 64 x 64 unit-upper diagonal blocks of U
    size_t uc_cap = 0;     // blocks
    int8_t* pk = nullptr;  // packed ffgemm operands of the INT8 forms
    size_t pk_cap = 0;     // bytes
    void* tp = nullptr;    // the transpose of a rectangular matrix (PLE)
    size_t tp_cap = 0;     // bytes
    void* wg = nullptr;    // Strassen-Winograd temporaries
    size_t wg_cap = 0;     // bytes
    size_t bytes = 0;
};

struct Ctx {
    hipStream_t s = nullptr;
    Profiler* prof = nullptr;
    Workspace* ws = nullptr;
    int64_t p = 2;
    ModP mp{2.0, 0.5};
    int form = FORM_FP64;   // resolved ffgemm form
    int kred_steps = 1;     // FP64 MFMA k-steps between accumulator reductions
    int64_t kred = 1;       // canonical products per dot-product reduction
    int* d_small = nullptr; // device results of the leaf kernels
    int* h_small = nullptr; // pinned host mirror
    // Mapped host words the window kernel posts its result to, their device
    // address, and the sequence number of the last window launched.
    unsigned long long* mail_h = nullptr;
    unsigned long long* mail_d = nullptr;
    unsigned* mail_seq = nullptr;
    // Two-leaf node: the 64 rows under the leaf about to be factored (set by
    // the node, taken by the leaf), and whether the leaf has already done
    // the node's G and Schur update.
    void* pair_below = nullptr;
    bool pair_done = false;
    // A leaf with few pivots sends the next one straight to the sparse path;
    // whether the sparse kernel's barrier words are in a known state.
    bool sparse_next = false;
    bool* sparse_ready = nullptr;
    // A full leaf's solve of its columns right of its pivots, held back so
    // that the parent's slab launch can carry it (it touches neither the
    // parent's U block nor the rows below); launched by itself before
    // anything that does touch it.
    LeftApply defer;
    bool defer_on = false;
    int log = 0;
    double i8_min_work = 1.0e9;  // M N K below which products skip the packed INT8 kernel
    // Strassen-Winograd: recursion levels (0: classical products only) and
    // the smallest M, N, K that is split
    int wino_levels = 0;
    int wino_min = 2048;
    // The matrix being factored (its top-left and leading dimension) and
    // which 64 x 64 diagonal blocks of its U have their inverse in ws->uc.
    const void* base = nullptr;
    int64_t base_lda = 0;
    std::vector<char> uc_ok;
};

// Global diagonal index of the element at p (p on the diagonal of the matrix
// being factored), or -1.
template <typename T>
inline int64_t diag_index(const Ctx& c, const T* p)
{
    if (!c.base) return -1;
    const int64_t off = (int64_t)(p - static_cast<const T*>(c.base));
    if (off < 0 || off % (c.base_lda + 1) != 0) return -1;
    return off / (c.base_lda + 1);
}

// Slot for the inverse of the unit-upper diagonal block of U at global
// diagonal index g (a multiple of 64), or null when there is none.
inline double* ucache_slot(Ctx& c, int64_t g)
{
    if (g < 0 || g % kTriNB != 0) return nullptr;
    const size_t blk = (size_t)(g / kTriNB);
    return blk < c.uc_ok.size() ? c.ws->uc + blk * kTriNB * kTriNB : nullptr;
}

// Reserve the U-block cache of a factorization with at most `rmax` pivots.
inline void ucache_begin(Ctx& c, const void* base, int64_t lda, int rmax)
{
    const size_t blocks = (size_t)(rmax / kTriNB);
    Workspace& w = *c.ws;
    if (blocks > w.uc_cap) {
        if (w.uc) {
            CUP_HIP(hipStreamSynchronize(c.s));
            CUP_HIP(hipFree(w.uc));
            w.bytes -= w.uc_cap * kTriNB * kTriNB * sizeof(double);
            w.uc = nullptr;
            w.uc_cap = 0;
        }
        if (dev_malloc((void**)&w.uc, blocks * kTriNB * kTriNB * sizeof(double)) != hipSuccess) {
            w.uc = nullptr;
            throw CupError{-2000};
        }
        w.uc_cap = blocks;
        w.bytes += blocks * kTriNB * kTriNB * sizeof(double);
    }
    c.base = base;
    c.base_lda = lda;
    c.uc_ok.assign(blocks, 0);
}

constexpr int kSmallInts = 4096;

inline void ctx_set_prime(Ctx& c, int64_t p)
{
    c.p = p;
    c.mp.p = (double)p;
    c.mp.pinv = 1.0 / (double)p;
    const double two53 = 9007199254740992.0;
    double h = (double)(p / 2);
    double steps = std::floor((two53 - 1.0 - (double)p) / (4.0 * h * h));
    c.kred_steps = (int)std::min(steps, (double)(1 << 28));
    double pm1 = (double)(p - 1);
    double terms = std::floor((two53 - 1.0) / (pm1 * pm1));
    c.kred = (int64_t)std::min(terms, 1.0e12);
    if (c.kred_steps < 1) c.kred_steps = 1;
    if (c.kred < 1) c.kred = 1;
}

// The sparse leaf kernel's words in the small result buffer (sparse_ws_ints()
// = 1296 ints from here, within kSmallInts), the window pivot count below
// which a leaf stopped by a zero row finishes there, and the bound on its
// grid barriers' polls.
constexpr int kSparseWs = 1024;
constexpr int kSparseAfter = 16;
constexpr int kSparseSpin = 1 << 22;

// Device -> host copy of `count` small results from word `at`, then wait.
inline const int* fetch_small_at(Ctx& c, int at, int count)
{
    CUP_HIP(hipMemcpyAsync(c.h_small + at, c.d_small + at, sizeof(int) * (size_t)count,
                           hipMemcpyDeviceToHost, c.s));
    CUP_HIP(hipStreamSynchronize(c.s));
    return c.h_small + at;
}

// Device -> host copy of the first `count` small results, then wait.
inline const int* fetch_small(Ctx& c, int count)
{
    CUP_HIP(hipMemcpyAsync(c.h_small, c.d_small, sizeof(int) * (size_t)count,
                           hipMemcpyDeviceToHost, c.s));
    CUP_HIP(hipStreamSynchronize(c.s));
    return c.h_small;
}

// Wait for word k of the host mailbox to carry the tag `seq` of the launch
// that posts it, without synchronising the stream, so that launches queued
// behind it keep the GPU busy meanwhile.  The stream is queried now and then:
// an error ends the wait with that error, and a drained stream without the
// word is an internal error.
inline int await_word(Ctx& c, unsigned seq, int k)
{
    unsigned long long v = 0;
    for (unsigned spin = 1;; ++spin) {
        v = __atomic_load_n(c.mail_h + k, __ATOMIC_ACQUIRE);
        if ((unsigned)(v >> 32) == seq) break;
        if ((spin & 1023u) == 0) {
            const hipError_t e = hipStreamQuery(c.s);
            if (e == hipSuccess) {
                v = __atomic_load_n(c.mail_h + k, __ATOMIC_ACQUIRE);
                if ((unsigned)(v >> 32) == seq) break;
                throw CupError{-3000};
            }
            if (e != hipErrorNotReady) CUP_HIP(e);
        }
        __builtin_ia32_pause();
    }
    return (int)(unsigned)(v & 0xffffffffull);
}

// A window's result: d, stop, then d pivot columns.
inline void await_window(Ctx& c, unsigned seq, int* h)
{
    h[0] = await_word(c, seq, 0);
    h[1] = await_word(c, seq, 1);
    for (int a = 0; a < h[0] && a < kLeafRows; ++a) h[2 + a] = await_word(c, seq, 2 + a);
}

inline unsigned next_seq(Ctx& c)
{
    unsigned s = ++*c.mail_seq;
    if (s == 0) s = ++*c.mail_seq;  // 0 is the tag of words never written
    return s;
}

// Launch the held-back leaf solve, if any (only int64 storage holds one back).
inline void flush_defer(Ctx& c)
{
    if (!c.defer_on) return;
    c.defer_on = false;
    launch_tri_apply<int64_t>(c.s, LEFT, kLeafRows, c.defer.W, static_cast<int64_t*>(c.defer.B),
                              c.defer.ldb, c.defer.other, c.mp);
}

// The triangular workspace; a held-back leaf solve reads its inverse from it,
// so that solve is launched first (stream order) before the buffer is
// handed out again or reallocated.
inline double* tri_workspace(Ctx& c, int n)
{
    flush_defer(c);
    const size_t need = (size_t)((n + kTriNB - 1) / kTriNB) * kTriNB * kTriNB;
    Workspace& w = *c.ws;
    if (need > w.tri_cap) {
        if (w.tri) {
            CUP_HIP(hipStreamSynchronize(c.s));
            CUP_HIP(hipFree(w.tri));
            w.bytes -= w.tri_cap * sizeof(double);
            w.tri = nullptr;
            w.tri_cap = 0;
        }
        size_t cap = std::max(need, (size_t)64 * kTriNB * kTriNB);
        if (dev_malloc((void**)&w.tri, cap * sizeof(double)) != hipSuccess) {
            w.tri = nullptr;
            throw CupError{-2000};
        }
        w.tri_cap = cap;
        w.bytes += cap * sizeof(double);
    }
    return w.tri;
}

inline int8_t* pack_workspace(Ctx& c, size_t need)
{
    Workspace& w = *c.ws;
    if (need > w.pk_cap) {
        if (w.pk) {
            CUP_HIP(hipStreamSynchronize(c.s));
            CUP_HIP(hipFree(w.pk));
            w.bytes -= w.pk_cap;
            w.pk = nullptr;
            w.pk_cap = 0;
        }
        if (dev_malloc((void**)&w.pk, need) != hipSuccess) {
            w.pk = nullptr;
            throw CupError{-2000};
        }
        w.pk_cap = need;
        w.bytes += need;
    }
    return w.pk;
}

inline int split_at(int n, int unit)
{
    int k = ((n / 2 + unit / 2) / unit) * unit;
    if (k < unit) k = unit;
    if (k >= n) k = n - 1;
    return k;
}

// ------------------------------------------------------------------ ffgemm
template <typename T>
void gemm_classic(Ctx& c, int M, int N, int K, const T* A, int64_t lda, const T* B, int64_t ldb, T* C,
                  int64_t ldc, int alpha)
{
    if (M <= 0 || N <= 0 || K <= 0) return;
    // The packed INT8 kernel pays two packing launches per product, so only
    // large products take it; the others take the direct INT8-limb kernel or
    // the FP64 carrier below (the results are identical either way).
    const bool i8 = (c.form == FORM_I8 || c.form == FORM_I8LIMB) && M >= 128 && N >= 128 &&
                    K >= 64 && (double)M * N * K >= c.i8_min_work;
    const bool prof_pack = c.prof && c.prof->want(3);
    const bool prof_i8 = c.prof && c.prof->want(2);
    const bool prof_small = c.prof && c.prof->want(0);
    if (i8) {
        const int limb = (c.form == FORM_I8LIMB) ? 1 : 0;
        const int nl = limb ? 2 : 1;
        int8_t* ws = pack_workspace(c, ffgemm_i8_workspace(M, N, K, limb));
        const int kmax = ffgemm_i8_kmax(limb);
        for (int k0 = 0; k0 < K; k0 += kmax) {
            const int kc = std::min(kmax, K - k0);
            if (prof_pack)
                c.prof->begin(c.s, 3, 0.0,
                              ((double)M * kc + (double)kc * N) * (sizeof(T) + nl));
            const int Kp = launch_pack_i8<T>(c.s, M, N, kc, A + k0, lda, B + (int64_t)k0 * ldb, ldb,
                                             c.mp, limb, ws);
            if (prof_pack) c.prof->end(c.s);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (prof_i8) {
                ProfRec& r = c.prof->open(2, 2.0 * M * N * kc,
                                          ((double)M * kc + (double)kc * N) * nl + 2.0 * M * N * sizeof(T));
                e0 = r.a;
                e1 = r.b;
            }
            launch_mma_i8<T>(c.s, M, N, Kp, ws, C, ldc, c.mp, alpha, limb, e0, e1);
        }
    } else {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (prof_small) {
            ProfRec& r = c.prof->open(0, 2.0 * M * N * K,
                                      ((double)M * K + (double)K * N + 2.0 * M * N) * sizeof(T));
            e0 = r.a;
            e1 = r.b;
        }
        // In the INT8 forms (p <= 2^16) the smaller products with K > 64 take
        // the INT8-limb kernel that reads the residues directly (no packing
        // launches); K <= 64 stays on the FP64 carrier, whose single-step
        // kernel pays one memory latency.
        if ((c.form == FORM_I8 || c.form == FORM_I8LIMB) && K > 64)
            launch_mma_i8_direct<T>(c.s, M, N, K, A, lda, B, ldb, C, ldc, c.mp, alpha, e0, e1);
        else
            launch_ffgemm_f64<T>(c.s, M, N, K, A, lda, B, ldb, C, ldc, c.mp, alpha, c.kred_steps, e0,
                                 e1);
    }
}

// Strassen-Winograd (Table 1's exponent log2 7, Section 4.4): with the
// leading Me x Ke, Ke x Ne parts (multiples of 128) split into quadrants,
// C += alpha A B takes seven half-size products (each again split while
// `level` allows and the halves reach c.wino_min) instead of eight; P2, P3
// and P4 accumulate straight into their quadrant of C, P1, P5, P6 and P7
// into temporaries that one pass folds into C.  The rows, columns and depth
// beyond the even parts are classical products.  Every temporary is a
// canonical residue matrix, so results equal the classical product's.
inline size_t wino_elems(const Ctx& c, int M, int N, int K, int level)
{
    const int g = 2 * kTriNB;
    const int Me = M / g * g, Ne = N / g * g, Ke = K / g * g;
    if (level <= 0 || Me < c.wino_min || Ne < c.wino_min || Ke < c.wino_min) return 0;
    const size_t hm = (size_t)Me / 2, hn = (size_t)Ne / 2, hk = (size_t)Ke / 2;
    return 4 * (hm * hk + hk * hn + hm * hn) + wino_elems(c, (int)hm, (int)hn, (int)hk, level - 1);
}

template <typename T>
void gemm_wino(Ctx& c, int M, int N, int K, const T* A, int64_t lda, const T* B, int64_t ldb, T* C,
               int64_t ldc, int alpha, int level, T* ws)
{
    const int g = 2 * kTriNB;
    const int Me = M / g * g, Ne = N / g * g, Ke = K / g * g;
    if (level <= 0 || Me < c.wino_min || Ne < c.wino_min || Ke < c.wino_min) {
        gemm_classic(c, M, N, K, A, lda, B, ldb, C, ldc, alpha);
        return;
    }
    const int hm = Me / 2, hn = Ne / 2, hk = Ke / 2;
    const int64_t sa = (int64_t)hm * hk, sb = (int64_t)hk * hn, sc = (int64_t)hm * hn;
    T* S1 = ws;
    T* S2 = S1 + sa;
    T* S3 = S2 + sa;
    T* S4 = S3 + sa;
    T* T1 = S4 + sa;
    T* T2 = T1 + sb;
    T* T3 = T2 + sb;
    T* T4 = T3 + sb;
    T* Pw = T4 + sb;  // P1
    T* Px = Pw + sc;  // P6
    T* Py = Px + sc;  // P5
    T* Pz = Py + sc;  // P7
    T* next = Pz + sc;
    const T* A11 = A;
    const T* A12 = A + hk;
    const T* A21 = A + (int64_t)hm * lda;
    const T* A22 = A21 + hk;
    const T* B11 = B;
    const T* B21 = B + (int64_t)hk * ldb;
    const T* B22 = B21 + hn;
    T* C11 = C;
    T* C12 = C + hn;
    T* C21 = C + (int64_t)hm * ldc;
    launch_wino_pre<T>(c.s, A, lda, hm, hk, 0, c.p, S1, S2, S3, S4);
    launch_wino_pre<T>(c.s, B, ldb, hk, hn, 1, c.p, T1, T2, T3, T4);
    launch_wino_zero<T>(c.s, Pw, 4 * sc);
    gemm_wino(c, hm, hn, hk, A12, lda, B21, ldb, C11, ldc, alpha, level - 1, next);   // P2
    gemm_wino(c, hm, hn, hk, (const T*)S4, hk, B22, ldb, C12, ldc, alpha, level - 1, next);  // P3
    gemm_wino(c, hm, hn, hk, A22, lda, (const T*)T4, hn, C21, ldc, -alpha, level - 1, next); // P4
    gemm_wino(c, hm, hn, hk, A11, lda, B11, ldb, Pw, hn, +1, level - 1, next);         // P1
    gemm_wino(c, hm, hn, hk, (const T*)S1, hk, (const T*)T1, hn, Py, hn, +1, level - 1, next);  // P5
    gemm_wino(c, hm, hn, hk, (const T*)S2, hk, (const T*)T2, hn, Px, hn, +1, level - 1, next);  // P6
    gemm_wino(c, hm, hn, hk, (const T*)S3, hk, (const T*)T3, hn, Pz, hn, +1, level - 1, next);  // P7
    launch_wino_post<T>(c.s, C, ldc, hm, hn, Pw, Px, Py, Pz, alpha, c.p);
    if (Ke < K) gemm_classic(c, Me, Ne, K - Ke, A + Ke, lda, B + (int64_t)Ke * ldb, ldb, C, ldc, alpha);
    if (Ne < N) gemm_classic(c, Me, N - Ne, K, A, lda, B + Ne, ldb, C + Ne, ldc, alpha);
    if (Me < M) gemm_classic(c, M - Me, N, K, A + (int64_t)Me * lda, lda, B, ldb, C + (int64_t)Me * ldc, ldc,
                             alpha);
}

inline void* wino_workspace(Ctx& c, size_t bytes)
{
    Workspace& w = *c.ws;
    if (bytes > w.wg_cap) {
        if (w.wg) {
            CUP_HIP(hipStreamSynchronize(c.s));
            CUP_HIP(hipFree(w.wg));
            w.bytes -= w.wg_cap;
            w.wg = nullptr;
            w.wg_cap = 0;
        }
        if (dev_malloc(&w.wg, bytes) != hipSuccess) {
            w.wg = nullptr;
            throw CupError{-2000};
        }
        w.wg_cap = bytes;
        w.bytes += bytes;
    }
    return w.wg;
}

// C <- C + alpha A B mod p (Algorithm 1): Strassen-Winograd when it is
// enabled and the product is large enough, else the classical kernels.
template <typename T>
void gemm(Ctx& c, int M, int N, int K, const T* A, int64_t lda, const T* B, int64_t ldb, T* C,
          int64_t ldc, int alpha)
{
    if (M <= 0 || N <= 0 || K <= 0) return;
    const size_t need = wino_elems(c, M, N, K, c.wino_levels);
    if (need == 0) {
        gemm_classic(c, M, N, K, A, lda, B, ldb, C, ldc, alpha);
        return;
    }
    T* ws = static_cast<T*>(wino_workspace(c, need * sizeof(T)));
    gemm_wino(c, M, N, K, A, lda, B, ldb, C, ldc, alpha, c.wino_levels, ws);
}

// ------------------------------------------------------------ TRSM / TRMM
// Section 3.2, Algorithm 2 (and its eight variants), plus the TRMM twin:
// halve the triangle, recurse on the diagonal blocks and fold the
// off-diagonal block in with one ffgemm.  B is n x other (Left) or other x n
// (Right).  The leaves multiply by the precomputed inverse (solve) or copy
// (multiply) of their 64 x 64 diagonal block, W[offset / 64].
template <typename T>
void tri_rec(Ctx& c, int op, int side, int uplo, int n, const T* Tm, int64_t ldt, T* B,
             int64_t ldb, int other, const double* W)
{
    // right solves with an upper triangle of order <= 512: one fused launch
    if (op == SOLVE && side == RIGHT && uplo == UPPER && n > kTriNB) {
        bool carried = false;
        if (launch_tri_slab<T>(c.s, n, Tm, ldt, W, B, ldb, other, c.mp,
                               c.form == FORM_I8 || c.form == FORM_I8LIMB,
                               c.defer_on ? &c.defer : nullptr, &carried)) {
            if (carried) c.defer_on = false;
            return;
        }
    }
    if (n <= kTriNB) {
        launch_tri_apply<T>(c.s, side, n, W, B, ldb, other, c.mp);
        return;
    }
    const int k = split_at(n, kTriNB);
    const T* T12 = Tm + k;
    const T* T21 = Tm + (int64_t)k * ldt;
    const T* T22 = Tm + (int64_t)k * ldt + k;
    const double* W2 = W + (size_t)(k / kTriNB) * kTriNB * kTriNB;
    const int sg = (op == SOLVE) ? -1 : +1;
    if (side == RIGHT) {
        T* B1 = B;
        T* B2 = B + k;
        if ((uplo == UPPER) == (op == SOLVE)) {
            // solve upper: X1 = B1 U11^-1 ; X2 = (B2 - X1 U12) U22^-1
            // multiply lower: [B1 L11 + B2 L21, B2 L22]
            const T* Toff = (uplo == UPPER) ? T12 : T21;
            if (op == SOLVE) {
                tri_rec(c, op, side, uplo, k, Tm, ldt, B1, ldb, other, W);
                gemm(c, other, n - k, k, B1, ldb, Toff, ldt, B2, ldb, sg);
                tri_rec(c, op, side, uplo, n - k, T22, ldt, B2, ldb, other, W2);
            } else {
                tri_rec(c, op, side, uplo, k, Tm, ldt, B1, ldb, other, W);
                gemm(c, other, k, n - k, B2, ldb, Toff, ldt, B1, ldb, sg);
                tri_rec(c, op, side, uplo, n - k, T22, ldt, B2, ldb, other, W2);
            }
        } else {
            // solve lower: X2 = B2 L22^-1 ; X1 = (B1 - X2 L21) L11^-1
            // multiply upper: [B1 U11, B1 U12 + B2 U22]
            tri_rec(c, op, side, uplo, n - k, T22, ldt, B2, ldb, other, W2);
            if (op == SOLVE) gemm(c, other, k, n - k, B2, ldb, T21, ldt, B1, ldb, sg);
            else gemm(c, other, n - k, k, B1, ldb, T12, ldt, B2, ldb, sg);
            tri_rec(c, op, side, uplo, k, Tm, ldt, B1, ldb, other, W);
        }
    } else {
        T* B1 = B;
        T* B2 = B + (int64_t)k * ldb;
        if ((uplo == LOWER) == (op == SOLVE)) {
            // solve lower: X1 = L11^-1 B1 ; X2 = L22^-1 (B2 - L21 X1)
            // multiply upper: [U11 B1 + U12 B2; U22 B2]
            tri_rec(c, op, side, uplo, k, Tm, ldt, B1, ldb, other, W);
            if (op == SOLVE) gemm(c, n - k, other, k, T21, ldt, B1, ldb, B2, ldb, sg);
            else gemm(c, k, other, n - k, T12, ldt, B2, ldb, B1, ldb, sg);
            tri_rec(c, op, side, uplo, n - k, T22, ldt, B2, ldb, other, W2);
        } else {
            // solve upper: X2 = U22^-1 B2 ; X1 = U11^-1 (B1 - U12 X2)
            // multiply lower: [L11 B1; L21 B1 + L22 B2]
            tri_rec(c, op, side, uplo, n - k, T22, ldt, B2, ldb, other, W2);
            if (op == SOLVE) gemm(c, k, other, n - k, T12, ldt, B2, ldb, B1, ldb, sg);
            else gemm(c, n - k, other, k, T21, ldt, B1, ldb, B2, ldb, sg);
            tri_rec(c, op, side, uplo, k, Tm, ldt, B1, ldb, other, W);
        }
    }
}

template <typename T>
void trsm(Ctx& c, int side, int uplo, int unit, int n, const T* Tm, int64_t ldt, T* B,
          int64_t ldb, int other)
{
    if (n <= 0 || other <= 0) return;
    double* W = tri_workspace(c, n);
    launch_diag_prep<T>(c.s, const_cast<T*>(Tm), ldt, n, uplo, unit, 0, W, c.mp);
    tri_rec(c, SOLVE, side, uplo, n, Tm, ldt, B, ldb, other, W);
}

template <typename T>
void trmm(Ctx& c, int side, int uplo, int unit, int n, const T* Tm, int64_t ldt, T* B,
          int64_t ldb, int other)
{
    if (n <= 0 || other <= 0) return;
    double* W = tri_workspace(c, n);
    launch_diag_prep<T>(c.s, const_cast<T*>(Tm), ldt, n, uplo, unit, 1, W, c.mp);
    tri_rec(c, MULT, side, uplo, n, Tm, ldt, B, ldb, other, W);
}

// ----------------------------------------------------------------- TRTRI
// Section 3.2, Algorithm 3 and its lower twin: two half-size solves on the
// off-diagonal block, a negation, and two recursive inversions.
template <typename T>
void trtri(Ctx& c, int uplo, int unit, int n, T* A, int64_t lda)
{
    if (n <= 0) return;
    if (n <= kTriNB) {
        launch_diag_prep<T>(c.s, A, lda, n, uplo, unit, 2, nullptr, c.mp);
        return;
    }
    const int k = split_at(n, kTriNB);
    T* A11 = A;
    T* A22 = A + (int64_t)k * lda + k;
    if (uplo == UPPER) {
        T* V = A + k;  // k x (n-k)
        trsm(c, RIGHT, UPPER, unit, n - k, A22, lda, V, lda, k);
        trsm(c, LEFT, UPPER, unit, k, A11, lda, V, lda, n - k);
        launch_negate<T>(c.s, V, lda, k, n - k, c.mp);
    } else {
        T* W = A + (int64_t)k * lda;  // (n-k) x k
        trsm(c, RIGHT, LOWER, unit, k, A11, lda, W, lda, n - k);
        trsm(c, LEFT, LOWER, unit, n - k, A22, lda, W, lda, k);
        launch_negate<T>(c.s, W, lda, n - k, k, c.mp);
    }
    trtri(c, uplo, unit, k, A11, lda);
    trtri(c, uplo, unit, n - k, A22, lda);
}

// ----------------------------------------------------------------- TRULM
// Section 3.2, Algorithm 4, in the variant used by Algorithm 8: on
// [N\T] with T unit upper (strict upper part stored) and N lower (diagonal
// stored), A <- T N.
template <typename T>
void trulm(Ctx& c, int n, T* A, int64_t lda)
{
    if (n <= 0) return;
    if (n <= kTriNB) {
        launch_trulm_leaf<T>(c.s, n, A, lda, c.mp, c.kred);
        return;
    }
    const int k = split_at(n, kTriNB);
    T* A11 = A;
    T* A12 = A + k;
    T* A21 = A + (int64_t)k * lda;
    T* A22 = A + (int64_t)k * lda + k;
    trulm(c, k, A11, lda);                                   // X11 = T11 N11
    gemm(c, k, k, n - k, A12, lda, A21, lda, A11, lda, +1);  // X11 += T12 N21
    trmm(c, RIGHT, LOWER, 0, n - k, A22, lda, A12, lda, k);  // X12 = T12 N22
    trmm(c, LEFT, UPPER, 1, n - k, A22, lda, A21, lda, k);   // X21 = T22 N21
    trulm(c, n - k, A22, lda);                               // X22 = T22 N22
}

// ----------------------------------------------------------------- TRLUM
// Section 3.2, Algorithm 5, in the variant InPlaceMM (Algorithm 9) applies to
// the packed [C\U] of a CUP: on [L\U] with L lower (diagonal stored) and U
// unit upper (strict upper part stored), A <- L U.
template <typename T>
void trlum(Ctx& c, int n, T* A, int64_t lda)
{
    if (n <= 0) return;
    if (n <= kTriNB) {
        launch_trlum_leaf<T>(c.s, n, A, lda, c.mp);
        return;
    }
    const int k = split_at(n, kTriNB);
    T* A11 = A;
    T* A12 = A + k;
    T* A21 = A + (int64_t)k * lda;
    T* A22 = A + (int64_t)k * lda + k;
    trlum(c, n - k, A22, lda);                               // X4 = L3 U3
    gemm(c, n - k, n - k, k, A21, lda, A12, lda, A22, lda, +1); // X4 += L2 U2
    trmm(c, LEFT, LOWER, 0, k, A11, lda, A12, lda, n - k);   // X2 = L1 U2
    trmm(c, RIGHT, UPPER, 1, k, A11, lda, A21, lda, n - k);  // X3 = L2 U1
    trlum(c, k, A11, lda);                                   // X1 = L1 U1
}

// ------------------------------------------------------ permutations
// A sequence of transpositions T(t, piv[t]) (t = 0..count-1, or count-1
// down to 0 when `descending`), applied in that order to the rows or columns
// of a matrix, composed into gathers: each gather moves at most `lim`
// positions, position dst receiving what src held before it, and the
// gathers are launched in order.  Trivial transpositions cost nothing.
struct Gathers {
    std::vector<GatherList> lists;
};

inline void compose_transpositions(const int64_t* piv, int count, bool descending, int lim, Gathers& out)
{
    out.lists.clear();
    // moved[k] = (position x, the position whose entry (at the start of the
    // current gather) is now at x); slot[x] = k, or -1 for an untouched x
    std::vector<std::pair<int, int>> moved;
    std::vector<int> slot;
    auto at = [&](int x) -> int {
        if ((size_t)x >= slot.size()) slot.resize((size_t)x + 1 + slot.size() / 2, -1);
        return slot[(size_t)x];
    };
    auto flush = [&]() {
        GatherList g;
        g.n = 0;
        for (auto& pr : moved) {
            slot[(size_t)pr.first] = -1;
            if (pr.first != pr.second) {
                g.dst[g.n] = pr.first;
                g.src[g.n] = pr.second;
                ++g.n;
            }
        }
        if (g.n) out.lists.push_back(g);
        moved.clear();
    };
    for (int u = 0; u < count; ++u) {
        const int t = descending ? count - 1 - u : u;
        const int j = (int)piv[t];
        if (j == t) continue;
        const int fresh = (at(t) < 0 ? 1 : 0) + (at(j) < 0 ? 1 : 0);
        if ((int)moved.size() + fresh > lim) flush();
        int kt = at(t), kj = at(j);
        if (kt < 0) {
            kt = (int)moved.size();
            moved.push_back({t, t});
            slot[(size_t)t] = kt;
        }
        if (kj < 0) {
            kj = (int)moved.size();
            moved.push_back({j, j});
            slot[(size_t)j] = kj;
        }
        std::swap(moved[(size_t)kt].second, moved[(size_t)kj].second);
    }
    flush();
}

// A P^T on rows [0, rows): columns t <-> piv[t] for t = 0..count-1 in order.
template <typename T>
void apply_transpositions(Ctx& c, T* A, int64_t lda, int rows, const int64_t* piv, int count,
                          bool descending = false)
{
    if (rows <= 0 || count <= 0) return;
    Gathers gs;
    compose_transpositions(piv, count, descending, kGatherMax, gs);
    for (const GatherList& g : gs.lists) launch_colgather<T>(c.s, A, lda, rows, g);
}

// The same on rows: rows t <-> piv[t] over columns [0, cols).
template <typename T>
void apply_row_transpositions(Ctx& c, T* A, int64_t lda, int cols, const int64_t* piv, int count,
                              bool descending)
{
    if (cols <= 0 || count <= 0) return;
    Gathers gs;
    compose_transpositions(piv, count, descending, kGatherRows, gs);
    for (const GatherList& g : gs.lists) launch_rowgather<T>(c.s, A, lda, cols, g);
}

// ------------------------------------------------------------- CUP leaf
// Global diagonal index of a leaf's 64 x 64 pivot block when the leaf is
// decided by its first window (64 pivots in rows 0..63, which then never
// move): that block is a diagonal block of U whose inverse is kept for the
// Schur solves of the ancestors.  -1 otherwise.
template <typename T>
int64_t leaf_cache_index(Ctx& c, T* A, int64_t lda, int b, int i, int t, int d)
{
    if (!(i == 0 && t == 0 && d == kLeafRows && b == kLeafRows)) return -1;
    const int64_t g = diag_index(c, A + (int64_t)i * lda + t);
    return ucache_slot(c, g) ? g : -1;
}

// The launches after a window that chose d pivots in rows i.. and columns
// t..t+d-1: the pivot rows' U entries beyond the window (one lower solve with
// the d x d pivot block, whose inverse is formed first), the update of the
// rows below, and the inverse of the unit-upper block for the cache.  With
// `guard`, only for d = b = 64 at (0, 0), every kernel does nothing unless
// *guard (the count the window leaves on the device) equals d.  `w_ready`:
// the window has left the pivot block's inverse in the triangular workspace.
// Returns the cache index filled, or -1.
template <typename T>
int64_t leaf_followup(Ctx& c, T* A, int64_t lda, int b, int N, int i, int t, int wc, int d,
                      const int* guard, bool w_ready = false)
{
    const int tw = t + wc;
    T* blk = A + (int64_t)i * lda + t;
    const int64_t g = leaf_cache_index(c, A, lda, b, i, t, d);
    double* ucs = (g >= 0) ? ucache_slot(c, g) : nullptr;
    if (tw < N) {
        double* W = tri_workspace(c, d);
        if (w_ready) {
            // the window left the pivot block's inverse in W
            if (ucs) launch_diag_prep<T>(c.s, blk, lda, kTriNB, UPPER, 1, 0, ucs, c.mp, guard, d);
        } else if (ucs) {
            launch_diag_prep2<T>(c.s, blk, lda, d, LOWER, 0, W, blk, UPPER, 1, ucs, c.mp, guard, d);
        } else {
            launch_diag_prep<T>(c.s, blk, lda, d, LOWER, 0, 0, W, c.mp, guard, d);
        }
        // the solve with the d x d lower pivot block (d <= 64: one leaf of
        // the triangular recursion)
        launch_tri_apply<T>(c.s, LEFT, d, W, A + (int64_t)i * lda + tw, lda, N - tw, c.mp, guard, d);
        if (i + d < b)
            gemm(c, b - i - d, N - tw, d, A + (int64_t)(i + d) * lda + t, lda,
                 A + (int64_t)i * lda + tw, lda, A + (int64_t)(i + d) * lda + tw, lda, -1);
    } else if (ucs) {
        launch_diag_prep<T>(c.s, blk, lda, kTriNB, UPPER, 1, 0, ucs, c.mp, guard, d);
    }
    return g;
}

// Base case over a block of b <= 64 rows (Algorithm 6 with the row recursion
// unrolled): window eliminations decide the pivots; after each window the
// pivot rows' U entries beyond the window come from one lower-triangular
// solve and the remaining rows are updated by one ffgemm; a row whose
// residual vanishes on the window is decided by a full-width scan.  Pivot
// rows stay in place until the end, then the U rows are compacted upwards
// in increasing order (the row move of Algorithm 6).
// The rest of a rank-deficient leaf from row i and position t, every
// remaining row in order, in one launch that takes the pivots full width
// (no window, no host round trip per pivot); then the column exchanges it
// left virtual, as one composed gather over the leaf's rows.  Appends the
// pivots to P, Q and `rows`; returns their number.
template <typename T>
int sparse_rest(Ctx& c, T* A, int64_t lda, int b, int N, int i, int t, std::vector<int64_t>& P,
                std::vector<int64_t>& Q, std::vector<int>& rows)
{
    flush_defer(c);
    int* ws = c.d_small + kSparseWs;
    if (kSparseWs + sparse_ws_ints() > kSmallInts) throw CupError{-3000};
    const bool prof = c.prof && c.prof->want(1);
    if (prof) c.prof->begin(c.s, 1, 0.0, 2.0 * (b - i) * (N - t) * sizeof(T));
    const unsigned seq = next_seq(c);
    const bool reset = !*c.sparse_ready;
    *c.sparse_ready = false;  // (until this launch is known to have completed)
    launch_sparse_leaf<T>(c.s, A, lda, b, N, i, t, c.mp, ws, kSparseSpin, reset, c.mail_d, seq);
    if (prof) c.prof->end(c.s);
    const int cnt = await_word(c, seq, 0);
    if (await_word(c, seq, 1)) throw CupError{-3000};
    *c.sparse_ready = true;
    std::vector<int64_t> piv((size_t)(t + cnt));
    for (int x = 0; x < t; ++x) piv[(size_t)x] = x;
    for (int a = 0; a < cnt; ++a) {
        const int col = await_word(c, seq, 2 + a), row = await_word(c, seq, kMailScan + a);
        piv[(size_t)(t + a)] = col;
        P.push_back(col);
        Q.push_back(row);
        rows.push_back(row);
    }
    apply_transpositions(c, A, lda, b, piv.data(), t + cnt);
    return cnt;
}

// U rows up: for the pivots in order, the pivot row's part right of its
// position moves to the row of that index (Algorithm 6's row move).
template <typename T>
void compact_u_rows(Ctx& c, T* A, int64_t lda, int N, const std::vector<int>& piv_rows)
{
    MoveList ml;
    ml.n = 0;
    for (int s = 0; s < (int)piv_rows.size(); ++s)
        if (piv_rows[s] != s) {
            ml.dst[ml.n] = s;
            ml.src[ml.n] = piv_rows[s];
            ++ml.n;
        }
    launch_rowmove_list<T>(c.s, A, lda, N, ml);
}

// A node of up to kSparseNodeRows rows after a leaf with few pivots: every
// row in order on the sparse path (one launch, whatever the node's depth),
// then one row move.  The decisions, and so the results, are those of the
// node's recursion (Algorithm 6's pivots are those of a row-by-row
// elimination, and its row moves at every level together bring the U rows
// up in pivot order).  The next node stays on this path while the pivots
// are fewer than 16 per 64 rows.
template <typename T>
int sparse_node(Ctx& c, T* A, int64_t lda, int m, int n, std::vector<int64_t>& P,
                std::vector<int64_t>& Q)
{
    std::vector<int> rows;
    const int r = sparse_rest(c, A, lda, m, n, 0, 0, P, Q, rows);
    c.sparse_next = (int64_t)r * kLeafRows < (int64_t)kSparseAfter * m;
    compact_u_rows(c, A, lda, n, rows);
    return r;
}

template <typename T>
int cup_leaf(Ctx& c, T* A, int64_t lda, int b, int N, std::vector<int64_t>& P,
             std::vector<int64_t>& Q)
{
    int i = 0, t = 0;
    int pending = -1;  // column brought to position t by a full-width scan
    std::vector<int> piv_rows;
    T* below = static_cast<T*>(c.pair_below);
    c.pair_below = nullptr;
    if (c.sparse_next) {
        // the previous leaf had few pivots: this one starts on the sparse path
        t = sparse_rest(c, A, lda, b, N, 0, 0, P, Q, piv_rows);
        c.sparse_next = t < kSparseAfter;
        i = b;
    }
    while (i < b && t < N) {
        const int wc = std::min(kWin, N - t);
        flush_defer(c);  // (outside the window's timing)
        const bool prof = c.prof && c.prof->want(1);
        if (prof) c.prof->begin(c.s, 1, 0.0, 2.0 * (b - i) * wc * sizeof(T));
        const unsigned seq = next_seq(c);
        // The usual outcome of a leaf's first window, 64 pivots, has its
        // follow-up launched before the count is known, each kernel doing
        // nothing unless the count the window left in device memory is 64.
        // Where the products are exact in FP64, the window itself also
        // inverts the two triangles of the decided block (the solve's
        // inverse and the cached one), so only the solve follows it.
        const bool ahead = (i == 0 && t == 0 && b == kLeafRows && wc == kLeafRows);
        const bool fused = ahead && c.mp.p <= kExact64;
        double* winv = nullptr;
        double* uinv = nullptr;
        // every window inverts its pivot block when the products are exact
        if (c.mp.p <= kExact64 && t + wc < N) winv = tri_workspace(c, kLeafRows);
        if (fused) {
            const int64_t g = leaf_cache_index(c, A, lda, b, 0, 0, kLeafRows);
            if (g >= 0) uinv = ucache_slot(c, g);
        }
        // A leaf with 64 rows below it in a two-leaf node also forms the
        // node's G (in the window) and, with its own solve, the Schur update
        // of those rows (one launch), when the window exchanges no column.
        const bool pair = fused && below != nullptr && winv != nullptr;
        launch_window<T>(c.s, A, lda, b, N, i, t, wc, c.mp, c.d_small, c.mail_d, seq, winv, uinv,
                         pair ? below : nullptr);
        if (prof) c.prof->end(c.s);
        if (pair) {
            launch_pair_update<T>(c.s, A, lda, N, winv, c.d_small, c.mp,
                                  c.form == FORM_I8 || c.form == FORM_I8LIMB);
        } else if (fused) {
            // held back (and dropped unless the window finds 64 pivots) when
            // the parent's slab solve runs on the INT8 matrix cores and can
            // carry it; otherwise launched now, doing nothing unless it does
            if (winv && sizeof(T) == sizeof(int64_t) && c.mp.p <= 65536.0 &&
                (c.form == FORM_I8 || c.form == FORM_I8LIMB)) {
                c.defer.W = winv;
                c.defer.B = A + wc;
                c.defer.ldb = lda;
                c.defer.other = N - wc;
                c.defer_on = true;
            } else if (winv) {
                launch_tri_apply<T>(c.s, LEFT, kLeafRows, winv, A + wc, lda, N - wc, c.mp, c.d_small,
                                    kLeafRows);
            }
        } else if (ahead) {
            leaf_followup(c, A, lda, b, N, 0, 0, wc, kLeafRows, c.d_small);
        }
        int h[2 + kLeafRows];
        await_window(c, seq, h);
        const int d = h[0], stop = h[1];
        if (stop == STOP_FAIL) throw CupError{-3000};  // CUP_ERR_INTERNAL
        if (d != kLeafRows) c.defer_on = false;  // the held-back solve would do nothing
        for (int a = 0; a < d; ++a) {
            int col = h[2 + a];
            if (a == 0 && pending >= 0) col = pending;
            P.push_back(col);
            Q.push_back(i + a);
            piv_rows.push_back(i + a);
        }
        pending = -1;
        if (d > 0) {
            int64_t g;
            if (ahead && d == kLeafRows) {
                g = leaf_cache_index(c, A, lda, b, 0, 0, d);
                if (pair) {
                    bool exchanged = false;
                    for (int a = 0; a < d; ++a) exchanged |= h[2 + a] != a;
                    if (exchanged)  // the pair launch did nothing: the leaf's own solve
                        launch_tri_apply<T>(c.s, LEFT, kLeafRows, winv, A + wc, lda, N - wc, c.mp);
                    else
                        c.pair_done = true;
                }
            } else {
                g = leaf_followup(c, A, lda, b, N, i, t, wc, d, (const int*)nullptr, winv != nullptr);
            }
            if (g >= 0) c.uc_ok[(size_t)(g / kTriNB)] = 1;
            i += d;
            t += d;
        }
        if (stop == STOP_ZERO_ROW && i < b && t < N && d < kSparseAfter) {
            t += sparse_rest(c, A, lda, b, N, i, t, P, Q, piv_rows);
            c.sparse_next = t < kSparseAfter;
            break;
        }
        if (stop == STOP_ZERO_ROW && i < b && t < N) {
            // the rows' results in order, as they arrive, up to the first
            // row with a nonzero
            const unsigned sseq = next_seq(c);
            launch_row_scan<T>(c.s, A, lda, i, b, t, N, c.d_small, c.mail_d, sseq);
            int found = -1, j = N;
            for (int r = 0; r < b - i; ++r) {
                const int hr = await_word(c, sseq, kMailScan + r);
                if (hr < N) {
                    found = i + r;
                    j = hr;
                    break;
                }
            }
            if (found < 0) break;  // every remaining row is zero
            i = found;
            if (j != t) {
                launch_colswap<T>(c.s, A, lda, b, t, j);
                pending = j;
            }
        }
    }
    compact_u_rows(c, A, lda, N, piv_rows);
    return t;
}

// ------------------------------------------------------------------- CUP
// Section 3.3, Algorithm 6: factor the top rows, permute the columns of the
// bottom rows, TRSM for G, Schur complement H = A22 - G V1 by ffgemm, factor
// H, permute the columns of V1, move the new U rows up.  Appends the
// transpositions (local column positions) to P and the profile (local rows)
// to Q; returns the rank.
template <typename T>
int cup_rec(Ctx& c, T* A, int64_t lda, int m, int n, std::vector<int64_t>& P,
            std::vector<int64_t>& Q)
{
    if (m <= 0 || n <= 0) return 0;
    if (m <= kLeafRows) return cup_leaf(c, A, lda, m, n, P, Q);
    if (c.sparse_next && m <= kSparseNodeRows) return sparse_node(c, A, lda, m, n, P, Q);
    const int k = split_at(m, kLeafRows);
    const size_t p0 = P.size(), q0 = Q.size();
    if (c.log) std::fprintf(stderr, "[cup] node m=%d n=%d k=%d\n", m, n, k);
    // a node of two full leaves: the first may do G and H (cup_leaf)
    if (k == kLeafRows && m - k == kLeafRows && n > kLeafRows) c.pair_below = A + (int64_t)k * lda;
    const int r1 = cup_rec(c, A, lda, k, n, P, Q);
    c.pair_below = nullptr;
    T* A2 = A + (int64_t)k * lda;
    if (c.pair_done) {
        // G and H are formed and the bottom rows' column order is unchanged
        c.pair_done = false;
    } else if (r1 > 0) {
        apply_transpositions(c, A2, lda, m - k, P.data() + p0, r1);          // A2 <- A2 P1^T
        // G = A21 U1^-1, with the cached diagonal-block inverses when every
        // block of U1 has one
        const int64_t g0 = diag_index(c, A);
        double* W1 = (r1 % kTriNB == 0) ? ucache_slot(c, g0) : nullptr;
        for (int bb = 0; W1 && bb < r1 / kTriNB; ++bb)
            if ((size_t)(g0 / kTriNB + bb) >= c.uc_ok.size() || !c.uc_ok[(size_t)(g0 / kTriNB + bb)])
                W1 = nullptr;
        // (a leaf solve held back by the top half's last leaf touches its own
        // rows right of column r1 only: the solve for G may carry it, the
        // Schur update needs it done)
        if (W1)
            tri_rec(c, SOLVE, RIGHT, UPPER, r1, A, lda, A2, lda, m - k, (const double*)W1);
        else
            trsm(c, RIGHT, UPPER, 1, r1, A, lda, A2, lda, m - k);
        flush_defer(c);
        if (r1 == n) return r1;
        gemm(c, m - k, n - r1, r1, A2, lda, A + r1, lda, A2 + r1, lda, -1); // H = A22 - G V1
    }
    const int r2 = cup_rec(c, A2 + r1, lda, m - k, n - r1, P, Q);
    if (r2 > 0) {
        if (r1 > 0) apply_transpositions(c, A + r1, lda, r1, P.data() + p0 + r1, r2);  // V1 P2^T
        if (k > r1) {
            flush_defer(c);  // the moved rows include the bottom half's last leaf
            launch_rowmove_shift<T>(c.s, A, lda, n, r1, k, r2);
        }
    }
    for (size_t x = p0 + r1; x < P.size(); ++x) P[x] += r1;
    for (size_t x = q0 + r1; x < Q.size(); ++x) Q[x] += k;
    return r1 + r2;
}

// ---------------------------------------------- reduced column echelon form
// Algorithm 7 (ColEchTrans) then Algorithm 8 (RedColEchTrans) on the packed
// [C\U] of rank r with row rank profile q (device int32 array, length r).
template <typename T>
void rref_tail(Ctx& c, T* A, int64_t lda, int m, int n, int r, const int* d_q)
{
    if (r <= 0) return;
    // Algorithm 7: M = U1^-1 U2 ; N = -M ; U1 <- U1^-1 (unit upper)
    trsm(c, LEFT, UPPER, 1, r, A, lda, A + r, lda, n - r);
    launch_negate<T>(c.s, A + r, lda, r, n - r, c.mp);
    trtri(c, UPPER, 1, r, A, lda);
    // Algorithm 8: [L1; L2] <- Q C on columns 0..j of row j (inclusive)
    launch_rowswap_lower<T>(c.s, A, lda, r, d_q);
    trsm(c, RIGHT, LOWER, 0, r, A, lda, A + (int64_t)r * lda, lda, m - r);  // R2 = L2 L1^-1
    trtri(c, LOWER, 0, r, A, lda);                                       // N = L1^-1
    trulm(c, r, A, lda);                                                 // X1 = T1 N
}

}  // namespace cup
