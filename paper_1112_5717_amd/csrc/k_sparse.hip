// The rest of a rank-deficient CUP leaf in one launch.
//
// Algorithm 6's base case takes the rows in order; for each, the pivot is
// the leftmost nonzero of its residual at positions >= t (the current
// column order), the columns t and j exchange, the row is scaled into U and
// the rows below are eliminated.  When most rows of a leaf have a zero
// residual (a rank-deficient matrix: a row that is a combination of earlier
// rows vanishes once those are eliminated), deciding each row by a 64-column
// window and a separate full-width scan costs several launches and host
// round trips per pivot.  This kernel instead runs the row loop on the
// device for all remaining rows of the leaf, full width, with a grid of
// co-resident workgroups (a cooperative launch) that own chunks of 64
// columns and meet at grid barriers:
//
//   scan   each row's leftmost nonzero at positions >= t in the workgroup's
//          columns -> the workgroup's minimum (row, position) key, which
//          its next barrier word carries to the others;
//   decide every workgroup takes the minimum key over the grid from the
//          barrier: the first row p with a nonzero (the rows before it are
//          zero rows: no pivot, nothing to do) and its pivot position j;
//   read   the pivot, the multipliers (the rows below p at the pivot's
//          column) and the rows, issued together;
//   update row p scaled by the pivot's inverse into U; rows below p lose
//          their multiplier times U (their multiplier stays, as their C
//          entry, at position t after the exchange of t and j); then the
//          next scan of the rows below p, from position t + 1.
//
// One grid barrier per pivot, none per zero row, and no other round trip
// between the workgroups.  Residues are carried as doubles: a product of two
// stays below 2^52 (p < 2^26), so every update is exact before its
// reduction.
#include <algorithm>
#include <type_traits>

#include "modarith.h"
#include "tri64.h"

namespace cup {

namespace {

constexpr int SPT = 256;  // threads per workgroup (one column each per pass)

// Residues travel as doubles (exact below 2^53; a product of two residues is
// below 2^52): reductions by the rounded reciprocal, inverses by Fermat.
__device__ __forceinline__ double sub_mul(double x, double m, double u, double P, double PI)
{
    return mod_red(fma(-m, u, x), P, PI);
}

// One result word for the host (a 64-bit store tagged with the launch's
// sequence number, at system scope).
__device__ __forceinline__ void post_word(unsigned long long* w, unsigned seq, int v)
{
    __hip_atomic_store(w, ((unsigned long long)seq << 32) | (unsigned)v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

// Grid barrier over `nblk` co-resident workgroups, with no central counter,
// that also takes the minimum of the workgroups' scan keys: each workgroup
// stores the generation it reaches and its key, as one 64-bit word, into its
// own slot of the generation's parity, and one wave reads every slot (one
// per lane) until all hold that generation, then folds their keys.  A
// workgroup that has passed on to the next barrier writes the other parity,
// and cannot reach the one after before this workgroup has left this one,
// so a slot of the awaited parity holds either the awaited generation or an
// older one.  One store and one round of loads per barrier, and no atomic
// that the workgroups contend for.  Generations grow across launches (the
// last is kept in bar[1]); the wait is bounded, and on timeout the flag
// bar[2] is raised and every later barrier returns at once, so that each
// workgroup leaves the kernel.
constexpr int kMaxGrid = 256;  // workgroups of one launch at most
__device__ bool grid_barrier(unsigned* bar, unsigned long long* slots, int nblk, unsigned& gen, int spin_max,
                             unsigned key, unsigned* s_min)
{
    __syncthreads();
    __shared__ int s_ok;
    const unsigned next = gen + 1;
    unsigned long long* slot = slots + (next & 1u) * kMaxGrid;
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_store(&slot[blockIdx.x], ((unsigned long long)next << 32) | key, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x < 64) {
        int ok = 1;
        unsigned mn = ~0u;
        for (int it = 0;; ++it) {
            bool arrived = true;
            mn = ~0u;
            for (int b = (int)threadIdx.x; b < nblk; b += 64) {
                const unsigned long long w = __hip_atomic_load(&slot[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                arrived &= (unsigned)(w >> 32) == next;
                mn = min(mn, (unsigned)w);
            }
            if (__ballot(!arrived) == 0) break;
            if (it > spin_max ||
                ((it & 15) == 15 && __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                if (threadIdx.x == 0) atomicExch(&bar[2], 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mn = min(mn, (unsigned)__shfl_xor((int)mn, off, 64));
        __threadfence();
        if (threadIdx.x == 0) {
            s_ok = ok && !__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *s_min = mn;
        }
    }
    gen = next;
    __syncthreads();
    return s_ok != 0;
}

// ws layout (ints): [0..3) barrier, [4] pivot count, [kSparseRows..) pivot
// rows, [kSparseCols..) pivot columns (positions), then the barrier slots
// (two parities of kMaxGrid 64-bit words).
constexpr int WS_BAR = 0, WS_CNT = kSparseCount, WS_PR = kSparseRows, WS_PC = kSparseCols;
static_assert(WS_PR + kSparseNodeRows <= WS_PC, "pivot rows before the pivot columns");
constexpr int WS_FLAGS = WS_PC + kSparseNodeRows;
static_assert(WS_FLAGS % 2 == 0, "barrier slots 8-byte aligned");

// A scan result: the first row (leaf-relative, < 128) with a nonzero
// residual at the positions scanned, and its leftmost such position
// (relative to the launch's first position, < 2^24), as one ordered 32-bit
// key (row above position), so that the minimum over the workgroups' keys is
// the next pivot.  No key: no nonzero left.
constexpr unsigned kNoKey = ~0u;
__device__ __forceinline__ unsigned scan_key(int r, int rel_pos)
{
    return ((unsigned)r << 24) | (unsigned)rel_pos;
}

// Minimum of the workgroup's keys (every thread gets it).
__device__ unsigned wg_min_key(unsigned key, unsigned* s_keys)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) key = min(key, (unsigned)__shfl_xor((int)key, off, 64));
    if ((threadIdx.x & 63) == 0) s_keys[threadIdx.x >> 6] = key;
    __syncthreads();
    unsigned k = s_keys[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) k = min(k, s_keys[w]);
    return k;
}
constexpr int kMaxChunks = 64;  // 64-column chunks per workgroup at most

// The column exchanges of the leaf are kept virtual until the end: a
// workgroup owns the same physical columns throughout and records the
// position of each (s_pos); position x is held by the physical column found
// by undoing the exchanges so far (phys).  So a pivot's column, which holds
// the rows' C entries from then on, is never written again in the leaf, and
// the only data one workgroup reads from another's columns in a round (the
// pivot and the multipliers, in that column) is final when the round
// starts: one grid barrier per pivot.  The exchanges are applied to the
// leaf's rows afterwards (by the host, as one composed gather).
template <typename T, int MAXR>
__global__ __launch_bounds__(SPT) void sparse_leaf_kernel(T* __restrict__ A, int64_t lda, int b, int N,
                                                          int i0, int t0, ModP mp, int* __restrict__ ws,
                                                          int spin_max, unsigned long long* __restrict__ mail,
                                                          unsigned seq)
{
    __shared__ unsigned s_keys[SPT / 64];
    __shared__ unsigned s_min;
    __shared__ int s_ht[MAXR], s_hj[MAXR];  // exchanges so far (positions)
    __shared__ int s_pos[kMaxChunks * 64];  // position of each own column
    const double P = mp.p, PI = mp.pinv;
    unsigned* bar = reinterpret_cast<unsigned*>(ws + WS_BAR);
    unsigned long long* slots = reinterpret_cast<unsigned long long*>(ws + WS_FLAGS);
    const int tid = threadIdx.x, nblk = gridDim.x;
    // the barrier's generation continues from the previous launch (kept in
    // bar[1]), so nothing is reset per launch
    const unsigned gen0 = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned gen = gen0;
    const int lane = tid & 63, rg = tid >> 6;
    const int cstride = nblk * 64;
    const int nchunk = (N - t0 + cstride - 1) / cstride;  // own chunks (<= kMaxChunks)
    auto col_of = [&](int ch) { return t0 + blockIdx.x * 64 + ch * cstride + lane; };

    for (int ch = rg; ch < nchunk; ch += 4) s_pos[ch * 64 + lane] = col_of(ch);
    // first scan: the first row from i0 with a nonzero at a position >= t0,
    // and its leftmost one, as this workgroup sees them (rows in groups of
    // up to 128, sixteen per thread and 64-row pass); its key reaches the
    // other workgroups with the first barrier (the matrix was written by
    // earlier launches on the stream, so no barrier precedes the scan)
    // The rows of the first own chunk (thread: rows 64 ps + rg + 4 k of its
    // column, every row of the node) stay in registers for the whole launch:
    // a round reads only the multipliers and writes the updated rows back
    // (other workgroups read them as multipliers and pivots).
    constexpr int GP = MAXR >= 128 ? 2 : 1;  // 64-row passes per group of rows
    double xr[GP][16];
    unsigned wgkey;
    {
        unsigned key = kNoKey;
        {
            const int c = col_of(0);
#pragma unroll
            for (int ps = 0; ps < GP; ++ps)
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int r = 64 * ps + rg + 4 * k;
                    xr[ps][k] = (c < N && r < b) ? ld_res(A + (int64_t)r * lda + c) : 0.0;
                }
#pragma unroll
            for (int ps = 0; ps < GP; ++ps)
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int r = 64 * ps + rg + 4 * k;
                    if (r >= i0 && xr[ps][k] != 0.0) key = min(key, scan_key(r, c - t0));
                }
        }
        for (int ch = 1; ch < nchunk; ++ch) {
            const int c = col_of(ch);
            for (int g0 = i0; g0 < b; g0 += 64 * GP) {
                T x[GP][16];
#pragma unroll
                for (int ps = 0; ps < GP; ++ps)
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int r = g0 + 64 * ps + rg + 4 * k;
                        x[ps][k] = (c < N && r < b) ? A[(int64_t)r * lda + c] : (T)0;
                    }
#pragma unroll
                for (int ps = 0; ps < GP; ++ps)
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        if (x[ps][k] != 0) key = min(key, scan_key(g0 + 64 * ps + rg + 4 * k, c - t0));
            }
        }
        wgkey = wg_min_key(key, s_keys);
    }

    int i = i0, t = t0, count = 0;
    while (i < b && t < N) {
        if (!grid_barrier(bar, slots, nblk, gen, spin_max, wgkey, &s_min)) return;
        // decide (every thread, from the minimum key): the first row from i
        // with a nonzero residual and its pivot position
        const unsigned key = s_min;
        if (key == kNoKey) break;  // every remaining row is zero
        const int pr = (int)(key >> 24);
        const int j = t0 + (int)(key & 0xffffffu);
        // the physical columns holding positions j and t before this round's
        // exchange (the exchanges so far undone, latest first)
        int pc = j, ptc = t;
        for (int k = count - 1; k >= 0; --k) {
            const int ht = s_ht[k], hj = s_hj[k];
            pc = (pc == ht) ? hj : ((pc == hj) ? ht : pc);
            ptc = (ptc == ht) ? hj : ((ptc == hj) ? ht : ptc);
        }
        if (tid == 0) {
            s_ht[count] = t;
            s_hj[count] = j;
            if (blockIdx.x == 0) {
                ws[WS_PR + count] = pr;
                ws[WS_PC + count] = j;
            }
        }
        // the pivot, read at once; its inverse (a chain of dependent
        // operations) is formed after the first column's loads are issued
        T* prow = A + (int64_t)pr * lda;
        const double pv = ld_res(prow + pc);
        double iv = 0.0;
        bool have_iv = false;

        // update the rows below p in every own column at a position > t (the
        // pivot's column keeps their C entries), and scan them
        unsigned key2 = kNoKey;
        // one own column: the exchange of positions t and j, then (at a
        // position after t) the update and scan of the rows below p, from
        // the registers (first chunk) or from memory (the others)
        auto column = [&](int ch, auto in_regs) __attribute__((always_inline)) {
            constexpr bool R = decltype(in_regs)::value;
            const int c = col_of(ch);
            if (c >= N) return;
            // positions t and j exchange among own columns (the same value
            // from each of the column's four threads)
            int pos = s_pos[ch * 64 + lane];
            if (pc != ptc) pos = (c == pc) ? t : ((c == ptc) ? j : pos);
            if (rg == 0) s_pos[ch * 64 + lane] = pos;
            if (pos <= t) return;
            const double pu = ld_res(prow + c);
            // rows in groups of up to 128 (sixteen per thread and 64-row
            // pass), from the group holding the first row below p; the
            // group's multipliers (their entries in the pivot's column,
            // final: it is never written again in the leaf) and, outside the
            // registers, its rows are loaded together
            for (int g0 = ((pr + 1) >> 6) / GP * GP * 64; g0 < b; g0 += 64 * GP) {
                double x[GP][16], m[GP][16];
#pragma unroll
                for (int ps = 0; ps < GP; ++ps)
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int r = g0 + 64 * ps + rg + 4 * k;
                        const bool below = r > pr && r < b;
                        if (R)
                            x[ps][k] = xr[ps][k];
                        else
                            x[ps][k] = below ? ld_res(A + (int64_t)r * lda + c) : 0.0;
                        m[ps][k] = below ? ld_res(A + (int64_t)r * lda + pc) : 0.0;
                    }
                if (!have_iv) {
                    iv = inv_fermat26(pv, P, PI);
                    have_iv = true;
                }
                const double u = mod_mul(pu, iv, P, PI);
#pragma unroll
                for (int ps = 0; ps < GP; ++ps)
#pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int r = g0 + 64 * ps + rg + 4 * k;
                        if (r > pr && r < b) {
                            const double y = sub_mul(x[ps][k], m[ps][k], u, P, PI);
                            st_res(A + (int64_t)r * lda + c, y);
                            if (R) xr[ps][k] = y;
                            if (y != 0.0) key2 = min(key2, scan_key(r, pos - t0));
                        }
                    }
            }
        };
        column(0, std::true_type{});
        for (int ch = 1; ch < nchunk; ++ch) column(ch, std::false_type{});
        // the workgroup's key (its barrier also orders every read of row p
        // before the row is rescaled)
        wgkey = wg_min_key(key2, s_keys);
        if (rg == 0) {
            for (int ch = 0; ch < nchunk; ++ch) {
                const int c = col_of(ch);
                if (c < N && s_pos[ch * 64 + lane] > t) {
                    if (!have_iv) {
                        iv = inv_fermat26(pv, P, PI);
                        have_iv = true;
                    }
                    st_res(prow + c, mod_mul(ld_res(prow + c), iv, P, PI));
                }
            }
        }
        i = pr + 1;
        ++t;
        ++count;
    }
    if (blockIdx.x == 0 && tid == 0) {
        // the generation reached, for the next launch (every workgroup has
        // read bar[1] at its start, before the first barrier)
        __hip_atomic_store(&bar[1], gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ws[WS_CNT] = count;
        // the result for the host, in mapped memory: the pivot count, no
        // failure, then each pivot's position and row
        for (int a = 0; a < count; ++a) {
            post_word(mail + 2 + a, seq, ws[WS_PC + a]);
            post_word(mail + kMailScan + a, seq, ws[WS_PR + a]);
        }
        post_word(mail + 1, seq, 0);
        post_word(mail, seq, count);
    }
}

}  // namespace

int sparse_ws_ints() { return WS_FLAGS + 4 * kMaxGrid; }

template <typename T, int MAXR>
int launch_sparse(hipStream_t s, T* A, int64_t lda, int b, int N, int i0, int t0, ModP mp, int* ws,
                  int spin_max, bool reset, unsigned long long* mail, unsigned seq)
{
    static int max_grid = 0;
    if (!max_grid) {
        int dev = 0, cus = 0, per = 0;
        CUP_HIP(hipGetDevice(&dev));
        CUP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        CUP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, sparse_leaf_kernel<T, MAXR>, SPT, 0));
        max_grid = std::max(1, cus * std::max(1, per));
    }
    const int cols = N - t0;
    const int grid = std::max(1, std::min(std::min(max_grid, kMaxGrid), (cols + 63) / 64));
    if ((cols + grid * 64 - 1) / (grid * 64) > kMaxChunks) throw CupError{-3000};  // (N > 1M columns)
    if (reset) CUP_HIP(hipMemsetAsync(ws, 0, sizeof(int) * (size_t)sparse_ws_ints(), s));
    void* args[] = {&A, &lda, &b, &N, &i0, &t0, &mp, &ws, &spin_max, &mail, &seq};
    CUP_HIP(hipLaunchCooperativeKernel((const void*)sparse_leaf_kernel<T, MAXR>, dim3(grid), dim3(SPT), args, 0, s));
    return grid;
}

template <typename T>
int launch_sparse_leaf(hipStream_t s, T* A, int64_t lda, int b, int N, int i0, int t0, ModP mp, int* ws,
                       int spin_max, bool reset, unsigned long long* mail, unsigned seq)
{
    if (b <= i0 || N <= t0) return 0;
    if (b > kSparseNodeRows) throw CupError{-3000};
    if (b <= kLeafRows)
        return launch_sparse<T, kLeafRows>(s, A, lda, b, N, i0, t0, mp, ws, spin_max, reset, mail, seq);
    return launch_sparse<T, kSparseNodeRows>(s, A, lda, b, N, i0, t0, mp, ws, spin_max, reset, mail, seq);
}

#define CUP_INST(T)                                                                                   \
    template int launch_sparse_leaf<T>(hipStream_t, T*, int64_t, int, int, int, int, ModP, int*, int, bool, \
                                       unsigned long long*, unsigned);
CUP_INST(int64_t)
CUP_INST(int8_t)
#undef CUP_INST

}  // namespace cup
