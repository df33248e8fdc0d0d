// 64 x 64 triangular inverses on the FP64 matrix cores, shared by the
// diagonal-block preparation of the triangular routines and by the leaf
// window (which inverts its own pivot blocks).
#pragma once
#include <hip/hip_runtime.h>

#include "modarith.h"

namespace cup {

// Residue in (-p, p): x - round(x / p) p, exact for |x| < 2^53 with
// |x / p| < 2^51 (the rounding adds and subtracts 1.5 * 2^52; the quotient
// from the rounded reciprocal is within one of x / p, so |x - q p| < p).
// Three dependent operations, against six for the canonical reduction, on
// the latency-bound chains below.
__device__ __forceinline__ double red_near(double x, double p, double pinv)
{
    const double magic = 6755399441055744.0;  // 1.5 * 2^52
    const double q = fma(x, pinv, magic) - magic;
    return fma(-q, p, x);
}

__device__ __forceinline__ double canon(double x, double p) { return (x < 0.0) ? x + p : x; }

// Inverse of a nonzero residue a in (-p, p), p < 2^26, in (-p, p): a^(p-2)
// by square and multiply over the 26 bits of p - 2, unrolled and without
// branches (a bit of the exponent selects the product), every value kept in
// (-p, p) by red_near, so every product is below p^2 < 2^52 and exact.
__device__ __forceinline__ double inv_fermat26(double a, double p, double pinv)
{
    const unsigned e = (unsigned)p - 2u;
    double r = 1.0, b = a;
#pragma unroll
    for (int i = 0; i < 26; ++i) {
        const double rb = red_near(r * b, p, pinv);
        r = ((e >> i) & 1u) ? rb : r;
        b = red_near(b * b, p, pinv);
    }
    return r;
}

// Workgroup barrier that orders LDS accesses only: global stores still in
// flight are not waited for (the usual barrier waits for every memory
// operation of every wave).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Inverse of a unit upper triangle U (64 x 64; its strict upper part in M),
// into X, by 16 x 16 blocks.  The four diagonal blocks are inverted
// column-parallel by the first wave of the group (lane 16a + j solves for
// column j of block a; each of the 16 steps is one rounding and one fused
// multiply-add on the chain, the block's entries loaded a few steps ahead).
// The off-diagonal blocks follow by increasing block distance on the FP64
// matrix cores, one block per wave:  X_ab = -X_aa (sum_{a<k<=b} U_ak X_kb),
// each 16 x 16 x 16 product four v_mfma_f64_16x16x4f64.  The partial sum's
// result layout (lane l holds rows l/16 + 4e of column l%16) is already the
// B operand of the second product, so nothing moves between the two.  Run by
// the four waves wbase..wbase+3 of the workgroup (every thread takes the
// barriers); entries stay in (-p, p), so a sum of at most 48 products is
// exact for p < 2^23.5.
typedef double v4d __attribute__((ext_vector_type(4)));

template <int AHEAD = 3>  // steps between the load of a column of U and its use
__device__ __forceinline__ void unit_upper_inverse(const double (*M)[kTriNB + 1], double (*X)[kTriNB + 1], double P,
                                   double PI, int wbase = 0)
{
    const int tid = threadIdx.x, lane = tid & 63, w = (tid >> 6) - wbase;
    const int hi = lane >> 4, lo = lane & 15;
    if (w == 0) {
        const int a = lane >> 4, j = lane & 15, o = 16 * a;
        // Column i of the block (rows above the diagonal) is loaded AHEAD
        // steps before it is used, so that the chain need not wait on LDS.
        double u[16][16];
        auto fetch = [&](int i) {
#pragma unroll
            for (int t = 0; t < 15; ++t)
                if (t < i) u[t][i] = M[o + t][o + i];
        };
#pragma unroll
        for (int i = 15; i > 15 - AHEAD; --i) fetch(i);
        double acc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = (i == j) ? 1.0 : 0.0;
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            if (i - AHEAD >= 1) fetch(i - AHEAD);
            const double x = red_near(acc[i], P, PI);
            X[o + i][o + j] = x;
#pragma unroll
            for (int t = 0; t < i; ++t) acc[t] = fma(u[t][i], -x, acc[t]);
        }
    }
    // blocks below the diagonal are zero
    if (w >= 0 && w < 4)
        for (int idx = tid - 64 * wbase; idx < kTriNB * kTriNB; idx += 256) {
            const int i = idx >> 6, s = idx & 63;
            if ((s >> 4) < (i >> 4)) X[i][s] = 0.0;
        }
    lds_barrier();
#pragma unroll
    for (int d = 1; d < 4; ++d) {
        if (w >= 0 && w + d < 4) {
            const int a = w, b = w + d;
            double ma[3][4], xb[3][4], xa[4];
#pragma unroll
            for (int k = 0; k < d; ++k)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    ma[k][ks] = M[16 * a + lo][16 * (a + 1 + k) + 4 * ks + hi];
                    xb[k][ks] = X[16 * (a + 1 + k) + 4 * ks + hi][16 * b + lo];
                }
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) xa[ks] = X[16 * a + lo][16 * a + 4 * ks + hi];
            __builtin_amdgcn_sched_barrier(0);  // operands loaded before the products
            v4d sacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < d; ++k)
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    sacc = __builtin_amdgcn_mfma_f64_16x16x4f64(ma[k][ks], xb[k][ks], sacc, 0, 0, 0);
            double sv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) sv[e] = red_near(sacc[e], P, PI);
            v4d xacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                xacc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ks], sv[ks], xacc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) X[16 * a + hi + 4 * e][16 * b + lo] = -red_near(xacc[e], P, PI);
        }
        lds_barrier();
    }
}

}  // namespace cup
