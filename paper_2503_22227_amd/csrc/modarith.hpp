// Exact 64-bit modular arithmetic for gfx950 wavefronts.
//
// CDNA4 has no 64x64-bit multiplier: every 64-bit product below is built by the
// compiler from 32-bit v_mul_lo/v_mul_hi/v_mad_u64_u32 operations, so the
// routines keep the number of 64-bit products minimal:
//   * Shoup multiplication by a constant w with companion w' = floor(w 2^64 / q):
//     one high product and two low products, result in [0, 2q);
//   * 64x64 -> 128-bit multiply-accumulate for sums of products, reduced once
//     per sum by Barrett reduction with mu = floor(2^128 / q) (exact quotient
//     estimate, one conditional subtraction);
//   * Harvey's lazy butterflies keep NTT values in [0, 4q), so every prime must
//     be below 2^62 (the library accepts primes below 2^61).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rf {

struct u128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// a >= q ? a - q : a
__device__ __forceinline__ uint64_t csub(uint64_t a, uint64_t q) { return a >= q ? a - q : a; }

// x * w mod q in [0, 2q) for any 64-bit x, w < q, wp = floor(w 2^64 / q).
__device__ __forceinline__ uint64_t shoup_lazy(uint64_t x, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t h = mulhi64(x, wp);
    return x * w - h * q;
}

__device__ __forceinline__ uint64_t shoup(uint64_t x, uint64_t w, uint64_t wp, uint64_t q) {
    return csub(shoup_lazy(x, w, wp, q), q);
}

__device__ __forceinline__ u128 mul_wide(uint64_t a, uint64_t b) {
    u128 r;
    r.lo = a * b;
    r.hi = mulhi64(a, b);
    return r;
}

__device__ __forceinline__ void mac(u128 &acc, uint64_t a, uint64_t b) {
    uint64_t lo = a * b;
    uint64_t hi = mulhi64(a, b);
    acc.lo += lo;
    acc.hi += hi + (acc.lo < lo ? 1u : 0u);
}

__device__ __forceinline__ void add_wide(u128 &acc, uint64_t v) {
    acc.lo += v;
    acc.hi += (acc.lo < v ? 1u : 0u);
}

// x mod q for any 128-bit x, with (mu1, mu0) = floor(2^128 / q), q < 2^63.
// The quotient estimate floor(x * mu / 2^128) is computed exactly (the dropped
// low word can never carry), so it is floor(x / q) or one less.
__device__ __forceinline__ uint64_t barrett128(u128 x, uint64_t mu1, uint64_t mu0, uint64_t q) {
    uint64_t c0 = mulhi64(x.lo, mu0);
    // x.lo * mu1 (128-bit) + c0
    uint64_t t_lo = x.lo * mu1;
    uint64_t t_hi = mulhi64(x.lo, mu1);
    uint64_t s = t_lo + c0;
    uint64_t carry = (s < t_lo) ? 1u : 0u;
    uint64_t hi_sum = t_hi + carry;
    // + x.hi * mu0 (128-bit)
    uint64_t u_lo = x.hi * mu0;
    uint64_t u_hi = mulhi64(x.hi, mu0);
    uint64_t s2 = s + u_lo;
    carry = (s2 < s) ? 1u : 0u;
    hi_sum += u_hi + carry;
    uint64_t quot = x.hi * mu1 + hi_sum;
    uint64_t r = x.lo - quot * q;
    return csub(r, q);
}

// 64-bit x mod q (x < 2^64) with the same constants.
__device__ __forceinline__ uint64_t barrett64(uint64_t x, uint64_t mu1, uint64_t mu0, uint64_t q) {
    uint64_t c0 = mulhi64(x, mu0);
    uint64_t t_lo = x * mu1;
    uint64_t t_hi = mulhi64(x, mu1);
    uint64_t s = t_lo + c0;
    uint64_t quot = t_hi + (s < t_lo ? 1u : 0u);
    uint64_t r = x - quot * q;
    return csub(r, q);
}

// a * b mod q for a, b < q.
__device__ __forceinline__ uint64_t mulmod(uint64_t a, uint64_t b, uint64_t mu1, uint64_t mu0,
                                           uint64_t q) {
    return barrett128(mul_wide(a, b), mu1, mu0, q);
}

__device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
    return csub(a + b, q);
}

__device__ __forceinline__ uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
    return a >= b ? a - b : a + q - b;
}

}  // namespace rf
