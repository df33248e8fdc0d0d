// The C-ABI of libcup (declared in include/cup.h): argument validation,
// form selection, scratch management and the calls into the drivers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/cup.h"
#include "driver.h"

namespace cup {
namespace {

struct Global {
    std::mutex mu;
    hipStream_t stream = nullptr;
    int form = FORM_AUTO;
    int wino_levels = 0;     // Strassen-Winograd recursion levels (0: off)
    int wino_min = 2048;     // smallest dimension split by it
    int* d_small = nullptr;
    int* h_small = nullptr;
    bool sparse_ready = false;  // the sparse leaf kernel's barrier words in d_small are valid
    // Result words of the window kernel in mapped, coherent host memory (kept
    // until the process ends: GPU writes to it may still be in flight when a
    // call fails), their device address, and the last sequence number used.
    unsigned long long* h_mail = nullptr;
    unsigned long long* d_mail = nullptr;
    unsigned mail_seq = 0;
    int* d_list = nullptr;
    size_t list_cap = 0;  // ints
    int* d_order = nullptr;  // work counters and processing order of the batched entry point
    size_t order_cap = 0;    // ints
    int64_t* h_bn = nullptr;  // pinned copy of a batch's column counts
    size_t bn_cap = 0;        // entries
    size_t bytes = 0;
    Profiler prof;
    Workspace ws;
};

constexpr int64_t kOrderMax = 32768;  // largest batch that is sorted by cost

// Scratch of the allocation-free batched entry point: the work counters of
// the batched kernels and the processing order of up to
// CUP_NOALLOC_BATCH_MAX matrices, one copy per GPU in the device image of
// this file (128 KiB and 256 bytes), held until the process ends.  Host code never
// passes the array's name to a kernel (in host code it is a host-side
// stand-in); it passes the device address that hipGetSymbolAddress returns
// for the current device, resolved once per device.
static_assert(CUP_NOALLOC_BATCH_MAX <= kOrderMax, "the batched order covers the no-alloc limit");
static __device__ __align__(256) int scratch[kBatchCounters + CUP_NOALLOC_BATCH_MAX];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (under the library
// lock).
void* noalloc_scratch()
{
    int dev = 0;
    CUP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw CupError{CUP_ERR_HIP - (int)hipErrorInvalidDevice};
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        CUP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw CupError{CUP_ERR_INTERNAL};
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

// The initial form: CUP_FORM from the environment when it names one (auto,
// fp64, i8, i8limb, or 0..3), else automatic.
int env_form()
{
    const char* v = std::getenv("CUP_FORM");
    if (!v) return FORM_AUTO;
    static const char* const names[] = {"auto", "fp64", "i8", "i8limb"};
    for (int f = 0; f < 4; ++f)
        if (std::strcmp(v, names[f]) == 0) return f;
    if (v[0] >= '0' && v[0] <= '3' && v[1] == 0) return v[0] - '0';
    return FORM_AUTO;
}

Global& G()
{
    static Global g;
    static const bool form_set = (g.form = env_form(), true);  // once, before any use
    (void)form_set;
    return g;
}

bool env_flag(const char* name)
{
    const char* v = std::getenv(name);
    return v && v[0] && std::strcmp(v, "0") != 0;
}

}  // namespace

bool fault_alloc()
{
    const char* v = std::getenv("CUP_FAULT");
    return v && std::strcmp(v, "alloc") == 0;
}

namespace {

bool is_prime_i64(int64_t p)
{
    if (p < 2) return false;
    if (p < 4) return true;
    if (p % 2 == 0) return false;
    for (int64_t d = 3; d * d <= p; d += 2)
        if (p % d == 0) return false;
    return true;
}

void ensure_small(Global& g)
{
    if (!g.d_small) {
        if (dev_malloc((void**)&g.d_small, sizeof(int) * kSmallInts) != hipSuccess) {
            g.d_small = nullptr;
            throw CupError{CUP_ERR_ALLOC};
        }
        g.sparse_ready = false;
        g.bytes += sizeof(int) * kSmallInts;
    }
    if (!g.h_small) {
        if (host_malloc((void**)&g.h_small, sizeof(int) * kSmallInts, hipHostMallocDefault) !=
            hipSuccess) {
            g.h_small = nullptr;
            throw CupError{CUP_ERR_ALLOC};
        }
    }
    if (!g.h_mail) {
        const size_t bytes = sizeof(unsigned long long) * kMailWords;
        unsigned long long* h = nullptr;
        if (host_malloc((void**)&h, bytes,
                          hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable) !=
            hipSuccess)
            throw CupError{CUP_ERR_ALLOC};
        std::memset(h, 0, bytes);
        unsigned long long* d = nullptr;
        if (hipHostGetDevicePointer((void**)&d, h, 0) != hipSuccess || !d) throw CupError{CUP_ERR_ALLOC};
        g.h_mail = h;
        g.d_mail = d;
    }
}

int* ensure_list(Global& g, size_t ints)
{
    if (ints > g.list_cap) {
        if (g.d_list) {
            CUP_HIP(hipStreamSynchronize(g.stream));
            (void)hipFree(g.d_list);
            g.bytes -= sizeof(int) * g.list_cap;
            g.d_list = nullptr;
            g.list_cap = 0;
        }
        size_t cap = std::max<size_t>(ints, 1024);
        if (dev_malloc((void**)&g.d_list, sizeof(int) * cap) != hipSuccess) throw CupError{CUP_ERR_ALLOC};
        g.list_cap = cap;
        g.bytes += sizeof(int) * cap;
    }
    return g.d_list;
}

// Resolve the ffgemm form for prime p and storage element size; -5 if the
// forced form cannot carry p.
int resolve_form(int forced, int64_t p, bool int8_storage)
{
    (void)int8_storage;
    switch (forced) {
    case FORM_FP64:
        return FORM_FP64;
    case FORM_I8:
        return p < 128 ? FORM_I8 : -5;
    case FORM_I8LIMB:
        return p <= 65536 ? FORM_I8LIMB : -5;
    default:
        return p < 128 ? FORM_I8 : (p <= 65536 ? FORM_I8LIMB : FORM_FP64);
    }
}

template <typename T>
int validate(int64_t m, int64_t n, const T* A, int64_t lda, int64_t p, const int64_t* rank)
{
    if (m < 0 || m > INT32_MAX / 2) return -1;
    if (n < 0 || n > INT32_MAX / 2) return -2;
    if (!A && m > 0 && n > 0) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (!is_prime_i64(p) || p >= ((int64_t)1 << 26)) return -5;
    if (sizeof(T) == 1 && p >= 128) return -5;
    if (!rank) return -6;
    return 0;
}

template <typename T>
int check_range(Ctx& c, const T* A, int64_t lda, int m, int n, int64_t p)
{
    if (!env_flag("CUP_CHECK") || m == 0 || n == 0) return 0;
    CUP_HIP(hipMemsetAsync(c.d_small, 0, sizeof(int), c.s));
    launch_range_check<T>(c.s, A, lda, m, n, p, c.d_small);
    const int* h = fetch_small(c, 1);
    return h[0] ? -3 : 0;
}

void write_perm(Ctx& c, int64_t* dst, const std::vector<int64_t>& head, int64_t len)
{
    if (!dst || len <= 0) return;
    std::vector<int64_t> full((size_t)len);
    for (int64_t t = 0; t < len; ++t) full[(size_t)t] = t;
    for (size_t t = 0; t < head.size(); ++t) full[t] = head[t];
    CUP_HIP(hipMemcpyAsync(dst, full.data(), sizeof(int64_t) * (size_t)len, hipMemcpyHostToDevice,
                           c.s));
    CUP_HIP(hipStreamSynchronize(c.s));
}

Ctx make_ctx(Global& g, int64_t p, int form)
{
    ensure_small(g);
    Ctx c;
    c.s = g.stream;
    c.form = form;
    c.d_small = g.d_small;
    c.h_small = g.h_small;
    c.mail_h = g.h_mail;
    c.mail_d = g.d_mail;
    c.mail_seq = &g.mail_seq;
    c.sparse_ready = &g.sparse_ready;
    c.log = env_flag("CUP_LOG") ? 1 : 0;
    if (const char* v = std::getenv("CUP_I8_MIN_WORK")) c.i8_min_work = std::atof(v);
    c.prof = &g.prof;
    c.ws = &g.ws;
    c.wino_levels = g.wino_levels;
    c.wino_min = g.wino_min;
    ctx_set_prime(c, p);
    return c;
}

// CUP of the m x n view at A (Algorithm 6); returns the rank, with the
// transposition list and the row rank profile on the host.
template <typename T>
int run_cup(Ctx& c, T* A, int64_t lda, int m, int n, std::vector<int64_t>& Pl, std::vector<int64_t>& Ql)
{
    if (m <= 0 || n <= 0) return 0;
    Pl.reserve((size_t)std::min(m, n));
    Ql.reserve((size_t)std::min(m, n));
    ucache_begin(c, A, lda, std::min(m, n));
    const int r = cup_rec<T>(c, A, lda, m, n, Pl, Ql);
    flush_defer(c);
    c.base = nullptr;
    return r;
}

// Run `body` (which returns a status) under the library lock, turning the
// internal failures into status codes.
template <typename F>
int guarded(Global& g, F&& body)
{
    try {
        return body();
    } catch (const CupError& e) {
        g.prof.drop();
        return e.code;
    } catch (const std::bad_alloc&) {
        g.prof.drop();
        return CUP_ERR_ALLOC;
    }
}

template <typename T>
int factor_impl(int64_t m, int64_t n, T* A, int64_t lda, int64_t p, int64_t* rank, int64_t* P,
                int64_t* Q, int tail)
{
    int v = validate(m, n, A, lda, p, rank);
    if (v) return v;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    int form = resolve_form(g.form, p, sizeof(T) == 1);
    if (form < 0) return form;
    try {
        Ctx c = make_ctx(g, p, form);
        int chk = check_range(c, A, lda, (int)m, (int)n, p);
        if (chk) return chk;
        std::vector<int64_t> Pl, Ql;
        const int r = run_cup<T>(c, A, lda, (int)m, (int)n, Pl, Ql);
        if (tail >= 1 && r > 0) {
            int* dq = ensure_list(g, (size_t)r);
            std::vector<int> q32(Ql.begin(), Ql.end());
            CUP_HIP(hipMemcpyAsync(dq, q32.data(), sizeof(int) * (size_t)r, hipMemcpyHostToDevice,
                                   c.s));
            CUP_HIP(hipStreamSynchronize(c.s));
            rref_tail<T>(c, A, lda, (int)m, (int)n, r, dq);
            if (tail == 2 && r == (int)n) {
                // A^{-1} = P^T X: rows t <-> p_t for t = n-1 down to 0
                apply_row_transpositions<T>(c, A, lda, (int)n, Pl.data(), r, true);
            }
        }
        CUP_HIP(hipStreamSynchronize(c.s));
        if (g.prof.on) g.prof.collect();
        write_perm(c, P, Pl, n);
        write_perm(c, Q, Ql, m);
        *rank = r;
        if (tail == 2 && r < n) return CUP_SINGULAR;
        return CUP_OK;
    } catch (const CupError& e) {
        g.prof.drop();
        return e.code;
    } catch (const std::bad_alloc&) {
        g.prof.drop();
        return CUP_ERR_ALLOC;
    }
}

template <typename T>
int ffgemm_impl(int64_t M, int64_t N, int64_t K, const T* A, int64_t lda, const T* B,
                       int64_t ldb, T* C, int64_t ldc, int64_t p, int alpha)
{
    if (M < 0 || M > INT32_MAX / 2) return -1;
    if (N < 0 || N > INT32_MAX / 2) return -2;
    if (K < 0 || K > INT32_MAX / 2) return -3;
    if (M == 0 || N == 0) return CUP_OK;
    if (K > 0 && (!A || lda < std::max<int64_t>(1, K))) return -5;
    if (K > 0 && (!B || ldb < std::max<int64_t>(1, N))) return -7;
    if (!C || ldc < std::max<int64_t>(1, N)) return -9;
    if (!is_prime_i64(p) || p >= ((int64_t)1 << 26) || (sizeof(T) == 1 && p >= 128)) return -10;
    if (alpha != 1 && alpha != -1) return -11;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    int form = resolve_form(g.form, p, sizeof(T) == 1);
    if (form < 0) return -10;
    try {
        Ctx c = make_ctx(g, p, form);
        gemm<T>(c, (int)M, (int)N, (int)K, A, lda, B, ldb, C, ldc, alpha);
        CUP_HIP(hipStreamSynchronize(c.s));
        if (g.prof.on) g.prof.collect();
        return CUP_OK;
    } catch (const CupError& e) {
        g.prof.drop();
        return e.code;
    }
}

// The transposition workspace of a rectangular PLE (n x m elements).
void* transpose_workspace(Global& g, Ctx& c, size_t bytes)
{
    Workspace& w = g.ws;
    if (bytes > w.tp_cap) {
        if (w.tp) {
            CUP_HIP(hipStreamSynchronize(c.s));
            CUP_HIP(hipFree(w.tp));
            w.bytes -= w.tp_cap;
            w.tp = nullptr;
            w.tp_cap = 0;
        }
        if (dev_malloc(&w.tp, bytes) != hipSuccess) {
            w.tp = nullptr;
            throw CupError{CUP_ERR_ALLOC};
        }
        w.tp_cap = bytes;
        w.bytes += bytes;
    }
    return w.tp;
}

// PLE (Section 5, Algorithm 10) as the transpose of the CUP of A^T: the
// matrix is transposed (in place when square, else through the workspace),
// factored by Algorithm 6 and transposed back; the CUP's column
// transpositions are PLE's row transpositions and its row rank profile is
// A's column rank profile.
template <typename T>
int ple_impl(int64_t m, int64_t n, T* A, int64_t lda, int64_t p, int64_t* rank, int64_t* P, int64_t* Q)
{
    int v = validate(m, n, A, lda, p, rank);
    if (v) return v;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    int form = resolve_form(g.form, p, sizeof(T) == 1);
    if (form < 0) return form;
    return guarded(g, [&]() -> int {
        Ctx c = make_ctx(g, p, form);
        int chk = check_range(c, A, lda, (int)m, (int)n, p);
        if (chk) return chk;
        std::vector<int64_t> Pl, Ql;
        int r = 0;
        if (m > 0 && n > 0) {
            if (m == n) {
                launch_transpose_square<T>(c.s, A, lda, (int)n);
                r = run_cup<T>(c, A, lda, (int)n, (int)m, Pl, Ql);
                launch_transpose_square<T>(c.s, A, lda, (int)n);
            } else {
                T* Tb = static_cast<T*>(transpose_workspace(g, c, sizeof(T) * (size_t)m * (size_t)n));
                launch_transpose<T>(c.s, A, lda, Tb, m, (int)m, (int)n);
                r = run_cup<T>(c, Tb, m, (int)n, (int)m, Pl, Ql);
                launch_transpose<T>(c.s, Tb, m, A, lda, (int)n, (int)m);
            }
        }
        CUP_HIP(hipStreamSynchronize(c.s));
        if (g.prof.on) g.prof.collect();
        write_perm(c, P, Pl, m);
        write_perm(c, Q, Ql, n);
        *rank = r;
        return CUP_OK;
    });
}

// Determinant (Section 4.4): det A = det(P) prod C[t][t] for a nonsingular
// A, with A P^T = C U (C lower triangular, U unit upper) and det(P) = -1 to
// the number of nontrivial transpositions; 0 when the rank is below n.
int det_impl(int64_t n, int64_t* A, int64_t lda, int64_t p, int64_t* det, int64_t* rank)
{
    int64_t dummy = 0;
    int v = validate(n, n, A, lda, p, &dummy);
    if (v) return v == -1 || v == -2 ? -1 : v + 1;  // -3 A -> -2, -4 lda -> -3, -5 p -> -4
    if (!det) return -5;
    if (!rank) return -6;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    int form = resolve_form(g.form, p, false);
    if (form < 0) return -4;
    return guarded(g, [&]() -> int {
        Ctx c = make_ctx(g, p, form);
        int chk = check_range(c, A, lda, (int)n, (int)n, p);
        if (chk) return -2;
        std::vector<int64_t> Pl, Ql;
        const int r = run_cup<int64_t>(c, A, lda, (int)n, (int)n, Pl, Ql);
        int64_t d = (n == 0) ? 1 % p : 0;
        if (n > 0 && r == (int)n) {
            int odd = 0;
            for (int t = 0; t < r; ++t) odd ^= (Pl[(size_t)t] != t) ? 1 : 0;
            launch_diag_prod<int64_t>(c.s, A, lda, (int)n, p, odd, reinterpret_cast<int64_t*>(c.d_small));
            const int* h = fetch_small(c, 2);
            std::memcpy(&d, h, sizeof(int64_t));
        }
        CUP_HIP(hipStreamSynchronize(c.s));
        if (g.prof.on) g.prof.collect();
        *det = d;
        *rank = r;
        return CUP_OK;
    });
}

// A X = B (Section 4.4): with A P^T = C U, X = P^T U^{-1} C^{-1} B by two
// triangular solves (Algorithm 2's Left-Lower-NonUnit and Left-Upper-Unit
// variants) and the row transpositions t <-> p_t for t = n-1 down to 0.
int solve_impl(int64_t n, int64_t nrhs, int64_t* A, int64_t lda, int64_t* B, int64_t ldb, int64_t p,
               int64_t* rank)
{
    if (n < 0 || n > INT32_MAX / 2) return -1;
    if (nrhs < 0 || nrhs > INT32_MAX / 2) return -2;
    if (!A && n > 0) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (!B && n > 0 && nrhs > 0) return -5;
    if (ldb < std::max<int64_t>(1, nrhs)) return -6;
    if (!is_prime_i64(p) || p >= ((int64_t)1 << 26)) return -7;
    if (!rank) return -8;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    int form = resolve_form(g.form, p, false);
    if (form < 0) return -7;
    return guarded(g, [&]() -> int {
        Ctx c = make_ctx(g, p, form);
        if (check_range(c, A, lda, (int)n, (int)n, p)) return -3;
        if (check_range(c, B, ldb, (int)n, (int)nrhs, p)) return -5;
        std::vector<int64_t> Pl, Ql;
        const int r = run_cup<int64_t>(c, A, lda, (int)n, (int)n, Pl, Ql);
        *rank = r;
        if (r < (int)n) {
            CUP_HIP(hipStreamSynchronize(c.s));
            if (g.prof.on) g.prof.collect();
            return CUP_SINGULAR;
        }
        if (n > 0 && nrhs > 0) {
            trsm<int64_t>(c, LEFT, LOWER, 0, (int)n, A, lda, B, ldb, (int)nrhs);  // C^{-1} B
            trsm<int64_t>(c, LEFT, UPPER, 1, (int)n, A, lda, B, ldb, (int)nrhs);  // U^{-1} (.)
            apply_row_transpositions<int64_t>(c, B, ldb, (int)nrhs, Pl.data(), r, true);
        }
        CUP_HIP(hipStreamSynchronize(c.s));
        if (g.prof.on) g.prof.collect();
        return CUP_OK;
    });
}

// Right nullspace basis (Section 3.4): A P^T X = [C 0] with
// X = [U1^{-1}, -U1^{-1} U2; 0, I], so the last n - r columns of P^T X,
// N = P^T [-U1^{-1} U2; I_{n-r}], span ker A.  The block -U1^{-1} U2 is
// ColEchTrans's first two steps (Algorithm 7) on the packed [C\U].
int nullspace_impl(int64_t m, int64_t n, int64_t* A, int64_t lda, int64_t p, int64_t* rank, int64_t* P,
                   int64_t* N, int64_t ldn)
{
    int v = validate(m, n, A, lda, p, rank);
    if (v) return v;
    if (!N && n > 0) return -8;
    if (ldn < std::max<int64_t>(1, n)) return -9;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    int form = resolve_form(g.form, p, false);
    if (form < 0) return form;
    return guarded(g, [&]() -> int {
        Ctx c = make_ctx(g, p, form);
        if (check_range(c, A, lda, (int)m, (int)n, p)) return -3;
        std::vector<int64_t> Pl, Ql;
        const int r = run_cup<int64_t>(c, A, lda, (int)m, (int)n, Pl, Ql);
        const int f = (int)n - r;
        if (f > 0) {
            if (r > 0) {
                trsm<int64_t>(c, LEFT, UPPER, 1, r, A, lda, A + r, lda, f);  // U1^{-1} U2
                launch_negate<int64_t>(c.s, A + r, lda, r, f, c.mp);
            }
            // pos[x]: where column x of A stands in the CUP column order
            std::vector<int> order((size_t)n), pos((size_t)n);
            for (int x = 0; x < (int)n; ++x) order[(size_t)x] = x;
            for (int t = 0; t < r; ++t) std::swap(order[(size_t)t], order[(size_t)Pl[(size_t)t]]);
            for (int x = 0; x < (int)n; ++x) pos[(size_t)order[(size_t)x]] = x;
            int* dpos = ensure_list(g, (size_t)n);
            CUP_HIP(hipMemcpyAsync(dpos, pos.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, c.s));
            launch_nullspace_assemble<int64_t>(c.s, A + r, lda, r, f, dpos, N, ldn, (int)n);
            CUP_HIP(hipStreamSynchronize(c.s));  // `pos` is read by the copy
        }
        CUP_HIP(hipStreamSynchronize(c.s));
        if (g.prof.on) g.prof.collect();
        write_perm(c, P, Pl, n);
        *rank = r;
        return CUP_OK;
    });
}

int trlum_impl(int64_t n, int64_t* A, int64_t lda, int64_t p)
{
    if (n < 0 || n > INT32_MAX / 2) return -1;
    if (!A && n > 0) return -2;
    if (lda < std::max<int64_t>(1, n)) return -3;
    if (!is_prime_i64(p) || p >= ((int64_t)1 << 26)) return -4;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    int form = resolve_form(g.form, p, false);
    if (form < 0) return -4;
    return guarded(g, [&]() -> int {
        Ctx c = make_ctx(g, p, form);
        if (check_range(c, A, lda, (int)n, (int)n, p)) return -2;
        trlum<int64_t>(c, (int)n, A, lda);
        CUP_HIP(hipStreamSynchronize(c.s));
        if (g.prof.on) g.prof.collect();
        return CUP_OK;
    });
}

// InPlaceMM (Section 4.3, Algorithm 9): B <- A B for an m x m A, with no
// temporary of B's size.  CUP of A (A = C U P), B <- P B (row
// transpositions t <-> p_t for t ascending), B <- U B, B <- C B (TRMM), then
// A <- C U (TRLUM) and A <- A P (column transpositions, t descending),
// which gives back A.
int inplace_mm_impl(int64_t m, int64_t n, int64_t* A, int64_t lda, int64_t* B, int64_t ldb, int64_t p)
{
    if (m < 0 || m > INT32_MAX / 2) return -1;
    if (n < 0 || n > INT32_MAX / 2) return -2;
    if (!A && m > 0) return -3;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (!B && m > 0 && n > 0) return -5;
    if (ldb < std::max<int64_t>(1, n)) return -6;
    if (!is_prime_i64(p) || p >= ((int64_t)1 << 26)) return -7;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    int form = resolve_form(g.form, p, false);
    if (form < 0) return -7;
    return guarded(g, [&]() -> int {
        Ctx c = make_ctx(g, p, form);
        if (check_range(c, A, lda, (int)m, (int)m, p)) return -3;
        if (check_range(c, B, ldb, (int)m, (int)n, p)) return -5;
        if (m == 0) return CUP_OK;
        std::vector<int64_t> Pl, Ql;
        const int r = run_cup<int64_t>(c, A, lda, (int)m, (int)m, Pl, Ql);
        if (n > 0) {
            apply_row_transpositions<int64_t>(c, B, ldb, (int)n, Pl.data(), r, false);  // P B
            trmm<int64_t>(c, LEFT, UPPER, 1, (int)m, A, lda, B, ldb, (int)n);            // U B
            trmm<int64_t>(c, LEFT, LOWER, 0, (int)m, A, lda, B, ldb, (int)n);            // C B
        }
        trlum<int64_t>(c, (int)m, A, lda);                                              // C U
        apply_transpositions<int64_t>(c, A, lda, (int)m, Pl.data(), r, true);           // (C U) P
        CUP_HIP(hipStreamSynchronize(c.s));
        if (g.prof.on) g.prof.collect();
        return CUP_OK;
    });
}

// Batched entry point, wide matrices: the column counts are copied to pinned
// host memory on the stream ahead of the batched kernels (the host waits for
// that copy only, not for the kernels); matrices wider than the kernels take
// (n > batched_max_n(), reported by them with info -2 and left untouched)
// are then factored one by one by the recursive single-matrix path
// (Algorithm 6) on the same stream, after the kernels, and their rank, P, Q
// and info are written.  Without such matrices the call stays asynchronous.
struct WideCheck {
    hipEvent_t ev = nullptr;
    const int64_t* hn = nullptr;
};

WideCheck queue_wide_check(Global& g, int64_t batch, const int64_t* n)
{
    if ((size_t)batch > g.bn_cap) {
        if (g.h_bn) {
            CUP_HIP(hipStreamSynchronize(g.stream));
            (void)hipHostFree(g.h_bn);
            g.h_bn = nullptr;
            g.bn_cap = 0;
        }
        if (host_malloc((void**)&g.h_bn, sizeof(int64_t) * (size_t)batch, hipHostMallocDefault) != hipSuccess) {
            g.h_bn = nullptr;
            throw CupError{CUP_ERR_ALLOC};
        }
        g.bn_cap = (size_t)batch;
    }
    static hipEvent_t ev = nullptr;
    if (!ev) CUP_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    CUP_HIP(hipMemcpyAsync(g.h_bn, n, sizeof(int64_t) * (size_t)batch, hipMemcpyDeviceToHost, g.stream));
    CUP_HIP(hipEventRecord(ev, g.stream));
    return WideCheck{ev, g.h_bn};
}

template <typename V>
std::vector<V> fetch_vec(Global& g, const V* d, int64_t count)
{
    std::vector<V> h((size_t)count);
    CUP_HIP(hipMemcpyAsync(h.data(), d, sizeof(V) * (size_t)count, hipMemcpyDeviceToHost, g.stream));
    CUP_HIP(hipStreamSynchronize(g.stream));
    return h;
}

void route_wide(Global& g, const WideCheck& wc, int64_t batch, const int64_t* m, const int64_t* n,
                int64_t* const* A, const int64_t* lda, const int64_t* p, int64_t* rank, int64_t* const* P,
                int64_t* const* Q, int32_t* info)
{
    CUP_HIP(hipEventSynchronize(wc.ev));
    std::vector<int64_t> wide;
    for (int64_t i = 0; i < batch; ++i)
        if (wc.hn[i] > batched_max_n()) wide.push_back(i);
    if (wide.empty()) return;
    (void)n;
    const std::vector<int64_t> hm = fetch_vec(g, m, batch), hl = fetch_vec(g, lda, batch),
                               hp = fetch_vec(g, p, batch);
    const std::vector<int64_t*> hA = fetch_vec(g, A, batch);
    const std::vector<int64_t*> hP = P ? fetch_vec(g, P, batch) : std::vector<int64_t*>((size_t)batch, nullptr);
    const std::vector<int64_t*> hQ = Q ? fetch_vec(g, Q, batch) : std::vector<int64_t*>((size_t)batch, nullptr);
    for (int64_t i : wide) {
        const int64_t mi = hm[(size_t)i], ni = wc.hn[i];
        int64_t r = 0;
        int32_t code = validate<int64_t>(mi, ni, hA[(size_t)i], hl[(size_t)i], hp[(size_t)i], &r);
        if (code == -6) code = 0;  // (no rank pointer in the single-matrix sense)
        int form = code ? 0 : resolve_form(g.form, hp[(size_t)i], false);
        if (!code && form < 0) code = -5;
        if (!code) {
            Ctx c = make_ctx(g, hp[(size_t)i], form);
            std::vector<int64_t> Pl, Ql;
            r = run_cup<int64_t>(c, hA[(size_t)i], hl[(size_t)i], (int)mi, (int)ni, Pl, Ql);
            write_perm(c, hP[(size_t)i], Pl, ni);
            write_perm(c, hQ[(size_t)i], Ql, mi);
        }
        CUP_HIP(hipMemcpyAsync(rank + i, &r, sizeof(int64_t), hipMemcpyHostToDevice, g.stream));
        CUP_HIP(hipMemcpyAsync(info + i, &code, sizeof(int32_t), hipMemcpyHostToDevice, g.stream));
        CUP_HIP(hipStreamSynchronize(g.stream));
    }
}

}  // namespace
}  // namespace cup

using namespace cup;

extern "C" {

int cup_set_stream(void* hip_stream)
{
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    g.stream = (hipStream_t)hip_stream;
    return CUP_OK;
}

int cup_set_form(int form)
{
    if (form < CUP_FORM_AUTO || form > CUP_FORM_I8LIMB) return -1;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    g.form = form;
    return CUP_OK;
}

int cup_set_winograd(int levels, int64_t min_dim)
{
    if (levels < 0 || levels > 8) return -1;
    if (min_dim < 2 * kTriNB || min_dim > INT32_MAX / 2) return -2;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    g.wino_levels = levels;
    g.wino_min = (int)min_dim;
    return CUP_OK;
}

int cup_get_form(void)
{
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    return g.form;
}

int cup_factor(int64_t m, int64_t n, int64_t* A, int64_t lda, int64_t p, int64_t* rank, int64_t* P,
               int64_t* Q)
{
    return factor_impl<int64_t>(m, n, A, lda, p, rank, P, Q, 0);
}

int cup_factor_i8(int64_t m, int64_t n, int8_t* A, int64_t lda, int64_t p, int64_t* rank,
                  int64_t* P, int64_t* Q)
{
    return factor_impl<int8_t>(m, n, A, lda, p, rank, P, Q, 0);
}

int cup_rank_profile(int64_t m, int64_t n, int64_t* A, int64_t lda, int64_t p, int64_t* rank,
                     int64_t* Q)
{
    return factor_impl<int64_t>(m, n, A, lda, p, rank, nullptr, Q, 0);
}

int cup_rref_inplace(int64_t m, int64_t n, int64_t* A, int64_t lda, int64_t p, int64_t* rank,
                     int64_t* P, int64_t* Q)
{
    return factor_impl<int64_t>(m, n, A, lda, p, rank, P, Q, 1);
}

int cup_rref_inplace_i8(int64_t m, int64_t n, int8_t* A, int64_t lda, int64_t p, int64_t* rank,
                        int64_t* P, int64_t* Q)
{
    return factor_impl<int8_t>(m, n, A, lda, p, rank, P, Q, 1);
}

int cup_inverse_inplace(int64_t n, int64_t* A, int64_t lda, int64_t p, int64_t* rank)
{
    if (n < 0) return -1;
    int rc = factor_impl<int64_t>(n, n, A, lda, p, rank, nullptr, nullptr, 2);
    if (rc == -1 || rc == -2) return -1;
    if (rc == -3) return -2;
    if (rc == -4) return -3;
    if (rc == -5) return -4;
    if (rc == -6) return -5;
    return rc;
}

int cup_inverse_inplace_i8(int64_t n, int8_t* A, int64_t lda, int64_t p, int64_t* rank)
{
    if (n < 0) return -1;
    int rc = factor_impl<int8_t>(n, n, A, lda, p, rank, nullptr, nullptr, 2);
    if (rc == -1 || rc == -2) return -1;
    if (rc == -3) return -2;
    if (rc == -4) return -3;
    if (rc == -5) return -4;
    if (rc == -6) return -5;
    return rc;
}

int cup_factor_batched(int64_t batch, const int64_t* m, const int64_t* n, int64_t* const* A,
                       const int64_t* lda, const int64_t* p, int64_t* rank, int64_t* const* P,
                       int64_t* const* Q, int32_t* info)
{
    if (batch < 0) return -1;
    if (batch == 0) return CUP_OK;
    if (!m) return -2;
    if (!n) return -3;
    if (!A) return -4;
    if (!lda) return -5;
    if (!p) return -6;
    if (!rank) return -7;
    if (!info) return -10;
    if (batch > INT32_MAX) return -1;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    try {
        // Largest matrices first within each width class (a counting sort on
        // the device, quadratic in the batch, so only up to kOrderMax
        // matrices); then one persistent kernel per width class.
        const bool ordered = batch <= kOrderMax;
        const size_t need = batched_scratch_ints((int)batch, ordered);
        if (need > g.order_cap) {
            if (g.d_order) {
                CUP_HIP(hipDeviceSynchronize());
                (void)hipFree(g.d_order);
                g.bytes -= sizeof(int) * g.order_cap;
                g.d_order = nullptr;
                g.order_cap = 0;
            }
            size_t cap = std::max<size_t>(need, 4096);
            if (dev_malloc((void**)&g.d_order, sizeof(int) * cap) != hipSuccess) throw CupError{CUP_ERR_ALLOC};
            g.order_cap = cap;
            g.bytes += sizeof(int) * cap;
        }
        const WideCheck wc = queue_wide_check(g, batch, n);
        launch_batched_cup(g.stream, (int)batch, m, n, A, lda, p, rank, P, Q, info, g.d_order, ordered);
        route_wide(g, wc, batch, m, n, A, lda, p, rank, P, Q, info);
        return CUP_OK;
    } catch (const CupError& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return CUP_ERR_ALLOC;
    }
}

int cup_ple(int64_t m, int64_t n, int64_t* A, int64_t lda, int64_t p, int64_t* rank, int64_t* P,
            int64_t* Q)
{
    return ple_impl<int64_t>(m, n, A, lda, p, rank, P, Q);
}

int cup_ple_i8(int64_t m, int64_t n, int8_t* A, int64_t lda, int64_t p, int64_t* rank, int64_t* P,
               int64_t* Q)
{
    return ple_impl<int8_t>(m, n, A, lda, p, rank, P, Q);
}

int cup_det(int64_t n, int64_t* A, int64_t lda, int64_t p, int64_t* det, int64_t* rank)
{
    return det_impl(n, A, lda, p, det, rank);
}

int cup_solve(int64_t n, int64_t nrhs, int64_t* A, int64_t lda, int64_t* B, int64_t ldb, int64_t p,
              int64_t* rank)
{
    return solve_impl(n, nrhs, A, lda, B, ldb, p, rank);
}

int cup_nullspace(int64_t m, int64_t n, int64_t* A, int64_t lda, int64_t p, int64_t* rank, int64_t* P,
                  int64_t* N, int64_t ldn)
{
    return nullspace_impl(m, n, A, lda, p, rank, P, N, ldn);
}

int cup_trlum(int64_t n, int64_t* A, int64_t lda, int64_t p)
{
    return trlum_impl(n, A, lda, p);
}

int cup_inplace_mm(int64_t m, int64_t n, int64_t* A, int64_t lda, int64_t* B, int64_t ldb, int64_t p)
{
    return inplace_mm_impl(m, n, A, lda, B, ldb, p);
}

int cup_factor_batched_noalloc(int64_t batch, const int64_t* m, const int64_t* n, int64_t* const* A,
                               const int64_t* lda, const int64_t* p, int64_t* rank, int64_t* const* P,
                               int64_t* const* Q, int32_t* info)
{
    if (batch < 0) return -1;
    if (batch > CUP_NOALLOC_BATCH_MAX) return CUP_ERR_NOALLOC_LIMIT;
    if (batch == 0) return CUP_OK;
    if (!m) return -2;
    if (!n) return -3;
    if (!A) return -4;
    if (!lda) return -5;
    if (!p) return -6;
    if (!rank) return -7;
    if (!info) return -10;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    try {
        // the same launches as cup_factor_batched, with the work counters and
        // the processing order in this device's static scratch array instead
        // of library memory (the order kernel clears the counters)
        int* sc = static_cast<int*>(noalloc_scratch());
        launch_batched_cup(g.stream, (int)batch, m, n, A, lda, p, rank, P, Q, info, sc, true);
        return CUP_OK;
    } catch (const CupError& e) {
        return e.code;
    }
}

int cup_ffgemm(int64_t M, int64_t N, int64_t K, const int64_t* A, int64_t lda, const int64_t* B,
               int64_t ldb, int64_t* C, int64_t ldc, int64_t p, int alpha)
{
    return ffgemm_impl<int64_t>(M, N, K, A, lda, B, ldb, C, ldc, p, alpha);
}

int cup_ffgemm_i8(int64_t M, int64_t N, int64_t K, const int8_t* A, int64_t lda, const int8_t* B,
                  int64_t ldb, int8_t* C, int64_t ldc, int64_t p, int alpha)
{
    return ffgemm_impl<int8_t>(M, N, K, A, lda, B, ldb, C, ldc, p, alpha);
}

const char* cup_strerror(int status)
{
    if (status == CUP_OK) return "success";
    if (status == CUP_SINGULAR) return "matrix is singular";
    if (status == CUP_ERR_ALLOC) return "allocation failure";
    if (status == CUP_ERR_INTERNAL) return "internal kernel check failed";
    if (status == CUP_ERR_NOALLOC_LIMIT)
        return "batch larger than the allocation-free entry point's static scratch (CUP_NOALLOC_BATCH_MAX)";
    if (status <= CUP_ERR_HIP && status > CUP_ERR_ALLOC) return "HIP runtime error";
    switch (status) {
    case -1: return "argument 1 is invalid";
    case -2: return "argument 2 is invalid";
    case -3: return "argument 3 is invalid (or an entry is outside [0,p))";
    case -4: return "argument 4 is invalid";
    case -5: return "argument 5 is invalid (p must be prime, 2 <= p < 2^26, within the form)";
    case -6: return "argument 6 is invalid";
    case -7: return "argument 7 is invalid";
    case -8: return "argument 8 is invalid";
    case -9: return "argument 9 is invalid";
    case -10: return "argument 10 is invalid";
    default: return "unknown status";
    }
}

int cup_profile(int enable)
{
    // 1: every class; above 1: bit k + 1 selects class k
    if (enable < 0 || enable > (2 << kProfKinds) - 1) return -1;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    if (enable) g.prof.reset();
    g.prof.on = enable != 0;
    g.prof.mask = (enable == 1) ? ((1u << kProfKinds) - 1) : ((unsigned)enable >> 1);
    return CUP_OK;
}

int cup_profile_read(double* stats)
{
    if (!stats) return -1;
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    for (int k = 0; k < kProfKinds; ++k) {
        stats[4 * k + 0] = g.prof.launches[k];
        stats[4 * k + 1] = g.prof.ms[k];
        stats[4 * k + 2] = g.prof.flops[k];
        stats[4 * k + 3] = g.prof.bytes[k];
    }
    return CUP_OK;
}

size_t cup_workspace_bytes(void)
{
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    return g.bytes + g.ws.bytes;
}

int cup_finalize(void)
{
    Global& g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    if (g.d_small) (void)hipFree(g.d_small);
    if (g.h_small) (void)hipHostFree(g.h_small);
    if (g.d_list) (void)hipFree(g.d_list);
    if (g.d_order) (void)hipFree(g.d_order);
    if (g.h_bn) (void)hipHostFree(g.h_bn);
    g.h_bn = nullptr;
    g.bn_cap = 0;
    if (g.ws.tri) (void)hipFree(g.ws.tri);
    if (g.ws.uc) (void)hipFree(g.ws.uc);
    if (g.ws.pk) (void)hipFree(g.ws.pk);
    if (g.ws.tp) (void)hipFree(g.ws.tp);
    if (g.ws.wg) (void)hipFree(g.ws.wg);
    g.ws = Workspace{};
    g.d_small = nullptr;
    g.h_small = nullptr;
    g.d_list = nullptr;
    g.list_cap = 0;
    g.d_order = nullptr;
    g.order_cap = 0;
    g.bytes = 0;
    return CUP_OK;
}

}  // extern "C"
