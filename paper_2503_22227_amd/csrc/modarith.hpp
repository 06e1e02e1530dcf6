// Exact 64-bit modular arithmetic for gfx950 wavefronts.
//
// CDNA4 has no 64x64-bit multiplier: every 64-bit product below is built by the
// compiler from 32-bit v_mul_lo/v_mul_hi/v_mad_u64_u32 operations, so the
// routines keep the number of 64-bit products minimal:
//   * Shoup multiplication by a constant w with companion w' = floor(w 2^64 / q):
//     one high product and two low products, result in [0, 2q);
//   * sums of products accumulated exactly as 128-bit values (MacAcc: four
//     sums of 30x30-bit partial products, one v_mad_u64_u32 each), reduced once
//     per sum by Barrett reduction with mu = floor(2^128 / q) (exact quotient
//     estimate, one conditional subtraction) or, where a forward NTT follows,
//     by two Shoup products into [0, 4q);
//   * Harvey's lazy butterflies keep NTT values in [0, 4q), so every prime must
//     be below 2^62; the library accepts primes below 2^60, which the split
//     multiply-accumulate below relies on.
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

// x * w mod q in [0, 2q) for x < 2^62 (the NTT's lazy residues, q < 2^60), w < q,
// wp = floor(w 2^62 / q) < 2^62, nq = 2^64 - q.  With the companion scaled by
// 2^62 instead of 2^64 the middle partial products x0 wp1 + x1 wp0 + hi(x0 wp0)
// stay below 2^64, so the quotient floor(x wp / 2^62) = 4 x1 wp1 + (mid >> 30)
// takes one high and three multiply-adds with no zero-extended addends, and the
// result x w + quotient (2^64 - q) mod 2^64 is one multiply-add chain: about 15
// VALU operations against 21 for shoup_lazy.
__device__ __forceinline__ uint64_t shoup62_lazy(uint64_t x, uint64_t w, uint64_t wp, uint64_t nq) {
    const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
    const uint32_t p0 = (uint32_t)wp, p1 = (uint32_t)(wp >> 32);
    const uint64_t b = (uint64_t)x1 * p0 + __umulhi(x0, p0);
    const uint64_t mid = (uint64_t)x0 * p1 + b;
    const uint64_t qh = (uint64_t)(x1 << 2) * p1 + (mid >> 30);
    const uint32_t w0 = (uint32_t)w, w1 = (uint32_t)(w >> 32);
    const uint32_t n0 = (uint32_t)nq, n1 = (uint32_t)(nq >> 32);
    const uint32_t h0 = (uint32_t)qh, h1 = (uint32_t)(qh >> 32);
    const uint64_t lo = (uint64_t)x0 * w0 + (uint64_t)h0 * n0;
    const uint32_t hi = (uint32_t)(lo >> 32) + x1 * w0 + x0 * w1 + h1 * n0 + h0 * n1;
    return ((uint64_t)hi << 32) | (uint32_t)lo;
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

__device__ __forceinline__ void add_wide(u128 &acc, u128 v) {
    acc.lo += v.lo;
    acc.hi += v.hi + (acc.lo < v.lo ? 1u : 0u);
}

// Exact sum of up to 8 products x y of operands below 2^60 (plus up to 8
// 64-bit addends), kept as four sums of 30x30-bit partial products: with
// x = xh 2^30 + xl and y = yh 2^30 + yl, every partial product is below 2^60,
// so each sum takes one v_mad_u64_u32 per product with the sum itself as the
// addend and never overflows.  4 VALU operations per product once the operands
// are split (a scalar constant splits on the scalar unit), against ~25 for a
// full 128-bit product added to a 128-bit accumulator.
struct MacAcc {
    uint64_t ll, lh, hl, hh;
    __device__ __forceinline__ MacAcc() : ll(0), lh(0), hl(0), hh(0) {}
    // x = xh 2^30 + xl split once by the caller when it is used many times
    __device__ __forceinline__ void mac_split(uint32_t xl, uint32_t xh, uint64_t y) {
        const uint32_t yl = (uint32_t)y & 0x3fffffffu, yh = (uint32_t)(y >> 30);
        ll += (uint64_t)xl * yl;
        lh += (uint64_t)xl * yh;
        hl += (uint64_t)xh * yl;
        hh += (uint64_t)xh * yh;
    }
    __device__ __forceinline__ void mac(uint64_t x, uint64_t y) {
        const uint32_t xl = (uint32_t)x & 0x3fffffffu, xh = (uint32_t)(x >> 30);
        const uint32_t yl = (uint32_t)y & 0x3fffffffu, yh = (uint32_t)(y >> 30);
        ll += (uint64_t)xl * yl;
        lh += (uint64_t)xl * yh;
        hl += (uint64_t)xh * yl;
        hh += (uint64_t)xh * yh;
    }
    // + v (any 64-bit value)
    __device__ __forceinline__ void add(uint64_t v) {
        ll += v & 0x3fffffffu;
        hl += v >> 30;
    }
    __device__ __forceinline__ u128 value() const {
        const uint64_t m = lh + hl;               // weight 2^30, < 2^64
        u128 r;
        r.lo = ll + (m << 30);
        uint64_t hi = (m >> 34) + (r.lo < ll ? 1u : 0u);
        const uint64_t t = r.lo;
        r.lo += hh << 60;                         // weight 2^60
        hi += (hh >> 4) + (r.lo < t ? 1u : 0u);
        r.hi = hi;
        return r;
    }
};

// Exact sum of x[i] * coef(i) for i < n <= NMAX (operands below 2^60), in
// groups of 8 products.
template <int NMAX, typename F>
__device__ __forceinline__ u128 dot_wide(const uint64_t *x, F coef, int n) {
    u128 total = {0, 0};
#pragma unroll
    for (int g = 0; g < (NMAX + 7) / 8; ++g) {
        MacAcc acc;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = g * 8 + k;
            if (i < NMAX && i < n) acc.mac(x[i], coef(i));
        }
        add_wide(total, acc.value());
    }
    return total;
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

// x mod q up to a multiple of q, in [0, 4q), for any 128-bit x: the high word
// times 2^64 mod q and the low word are each reduced by a Shoup product (by
// r64 = 2^64 mod q with companion r64_p, and by 1 with companion
// one_p = floor(2^64 / q)).  For results that feed a forward NTT, whose first
// butterflies accept inputs below 4q.
__device__ __forceinline__ uint64_t reduce128_lazy(u128 x, uint64_t q, uint64_t r64, uint64_t r64_p,
                                                   uint64_t one_p) {
    const uint64_t a = shoup_lazy(x.hi, r64, r64_p, q);
    const uint64_t b = x.lo - mulhi64(x.lo, one_p) * q;
    return a + b;
}

// x mod q in [0, q) for any 128-bit x by reduce128_lazy and two conditional
// subtractions (cheaper than barrett128: two Shoup products instead of three
// high products).
__device__ __forceinline__ uint64_t reduce128(u128 x, uint64_t q, uint64_t r64, uint64_t r64_p, uint64_t one_p) {
    return csub(csub(reduce128_lazy(x, q, r64, r64_p, one_p), 2 * q), q);
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
