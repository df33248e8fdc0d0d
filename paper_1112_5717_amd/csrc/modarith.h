// Exact arithmetic in GF(p), p < 2^26, on the GPU.
//
// Residues are carried as doubles: every integer of magnitude below 2^53 is
// exact, a product of two residues is below 2^52, and a sum of k products
// stays exact while its magnitude stays below 2^53.  Reduction computes
// q = floor(x / p) from the rounded reciprocal (off by at most one), then
// x - q p with one fused multiply-add (exact because the true remainder is a
// small integer), then one correction each way.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cup_internal.h"

namespace cup {

__device__ __forceinline__ double mod_red(double x, double p, double pinv)
{
    double q = floor(x * pinv);
    double r = fma(-q, p, x);
    r = (r < 0.0) ? r + p : r;
    r = (r >= p) ? r - p : r;
    return r;
}

__device__ __forceinline__ double mod_mul(double a, double b, double p, double pinv)
{
    return mod_red(a * b, p, pinv);
}

// Residue loads and stores: int64 storage holds values below 2^26, so its low
// 32-bit word carries the value; int8 storage holds values below 2^7.
__device__ __forceinline__ double ld_res(const int64_t* a) { return (double)(int)(*a); }
__device__ __forceinline__ double ld_res(const int8_t* a) { return (double)(int)(*a); }
__device__ __forceinline__ void st_res(int64_t* a, double v) { *a = (int64_t)(int)v; }
__device__ __forceinline__ void st_res(int8_t* a, double v) { *a = (int8_t)(int)v; }

}  // namespace cup
