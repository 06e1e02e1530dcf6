// Device code of the element-wise and base-conversion steps of key switching,
// rescale and automorphism, written per work unit (gx = block of 256
// coefficients, gy = limb, digit or polynomial) so that the single-operation
// kernels (keyswitch.hip) and the persistent batched kernels (batch.hip) run
// the same code.
#pragma once
#include <hip/hip_runtime.h>

#include "modarith.hpp"
#include "rf_internal.hpp"

namespace rf {

constexpr int kEw = 256;  // threads per block of the element-wise kernels

// d0 = a0 b0, d1 = a0 b1 + a1 b0 (into d01 = [2][nl][N]), d2 = a1 b1 (into d2 = [nl][N]).
__device__ __forceinline__ void tensor_unit(const uint64_t *__restrict__ a, const uint64_t *__restrict__ b,
                                                     uint64_t *__restrict__ d01, uint64_t *__restrict__ d2,
                                                     const PrimeConst *__restrict__ pcs, uint32_t log_n, uint32_t nl, const uint32_t *pmap, uint32_t gx, uint32_t gy) {
    const uint32_t i = gy;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const size_t poly = (size_t)nl << log_n;
    const size_t off = ((size_t)i << log_n) + n;
    const PrimeConst pc = pcs[pmap ? (uint32_t)pmap[i] : i];
    const uint64_t a0 = a[off], a1 = a[poly + off], b0 = b[off], b1 = b[poly + off];
    u128 acc = mul_wide(a0, b1);
    mac(acc, a1, b0);
    d01[off] = barrett128(mul_wide(a0, b0), pc.mu1, pc.mu0, pc.q);
    d01[poly + off] = barrett128(acc, pc.mu1, pc.mu0, pc.q);
    d2[off] = barrett128(mul_wide(a1, b1), pc.mu1, pc.mu0, pc.q);
}

// Targets of a base conversion handled by one work unit: splitting the
// targets over several units multiplies the parallelism of the conversion
// (its inputs are re-read, from L2, and where not pre-scaled re-scaled per
// chunk, which is cheap next to the chunk's multiply-accumulates) and lets the
// unrolled target loop prefetch its uniform constants.
constexpr int kConvChunk = 8;
// ModUp targets per thread (the conversion's limb grouping; rf_tuning picks
// 4, 8 or 16 per level).  Measured at N = 2^16, 24 + 4 primes, alpha = 8 (20
// targets per digit): 8 targets 18.4 us, 10 targets 19.1 us, 20 targets 24.8 us
// per launch (fewer, longer waves hide less latency).
constexpr int kModupChunk = 8;

__host__ __device__ inline uint32_t modup_chunks(uint32_t nl, uint32_t K, uint32_t chunk) {
    return (nl + K - 1 + chunk - 1) / chunk;
}
__host__ __device__ inline uint32_t moddown_chunks(uint32_t nl) { return (nl + kConvChunk - 1) / kConvChunk; }

// ModUp conversion of one chunk of targets for a digit of S primes (S a
// compile-time constant, so the S multiply-accumulates per target are fully
// unrolled and the target's S constants, stored contiguously, can be fetched
// with wide scalar loads ahead of use).  SCALED: x already holds
// y_i = [x_i (Q_j/q_i)^-1]_{q_i} (an INTT with that factor folded into its last
// stage), so the digit's input products are skipped.
template <int S, bool SCALED, int CH>
__device__ __forceinline__ void modup_conv_s(const uint64_t *__restrict__ x, uint64_t *__restrict__ dst,
                                             const PrimeConst *__restrict__ pcs, const uint64_t *__restrict__ blk,
                                             uint32_t alpha, uint32_t start, uint32_t ntarget, uint32_t t0,
                                             uint32_t nl, uint32_t L, uint32_t log_n, size_t n) {
    uint32_t yl[S], yh[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        const uint64_t xi = x[((size_t)(start + i) << log_n) + n];
        const uint64_t y = SCALED ? xi : shoup(xi, blk[2 * i], blk[2 * i + 1], pcs[start + i].q);
        yl[i] = (uint32_t)y & 0x3fffffffu;
        yh[i] = (uint32_t)(y >> 30);
    }
    const uint64_t *cross = blk + 2 * alpha;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const uint32_t tt = t0 + k;
        if (tt < ntarget) {
            const uint32_t g = tt < start ? tt : (tt < nl - S ? tt + S : L + (tt - (nl - S)));
            const PrimeConst pc = pcs[g];
            const uint64_t *cg = cross + (size_t)g * alpha;
            MacAcc acc;
#pragma unroll
            for (int i = 0; i < S; ++i) acc.mac_split(yl[i], yh[i], cg[i]);
            dst[(size_t)tt << log_n] = reduce128_lazy(acc.value(), pc.q, pc.r64, pc.r64_p, pc.one_p);
        }
    }
}

// ModUp base conversion at level nl: x = [nl][N] coefficient domain; ext =
// digits back to back, digit j holding nl - s_j + K limbs ordered as the basis
// Q_l u P without the digit's own primes, each residue in [0, 4q) (the forward
// NTT that follows accepts that range).  gy = digit * modup_chunks + chunk,
// CH targets per chunk.  SCALED: x holds the digits' input factors already (see
// modup_conv_s).
template <bool SCALED, int CH>
__device__ __forceinline__ void modup_bconv_unit(const uint64_t *__restrict__ x, uint64_t *__restrict__ ext,
                                                 const PrimeConst *__restrict__ pcs,
                                                 const uint64_t *__restrict__ tab, size_t tab_stride,
                                                 uint32_t log_n, uint32_t nl, uint32_t L, uint32_t K,
                                                 uint32_t alpha, uint32_t gx, uint32_t gy) {
    const uint32_t nch = modup_chunks(nl, K, CH);
    const uint32_t j = gy / nch, ch = gy - j * nch;
    const uint32_t start = j * alpha;
    const uint32_t s = min(alpha, nl - start);
    const uint32_t ntarget = nl - s + K;
    const uint32_t t0 = ch * CH;
    if (t0 >= ntarget) return;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const uint64_t *blk = tab + ((size_t)j * alpha + (s - 1)) * tab_stride;
    uint64_t *dst = ext + (((size_t)j * (nl + K - alpha)) << log_n) + n;
    switch (s) {
        case 1: modup_conv_s<1, SCALED, CH>(x, dst, pcs, blk, alpha, start, ntarget, t0, nl, L, log_n, n); break;
        case 2: modup_conv_s<2, SCALED, CH>(x, dst, pcs, blk, alpha, start, ntarget, t0, nl, L, log_n, n); break;
        case 3: modup_conv_s<3, SCALED, CH>(x, dst, pcs, blk, alpha, start, ntarget, t0, nl, L, log_n, n); break;
        case 4: modup_conv_s<4, SCALED, CH>(x, dst, pcs, blk, alpha, start, ntarget, t0, nl, L, log_n, n); break;
        case 5: modup_conv_s<5, SCALED, CH>(x, dst, pcs, blk, alpha, start, ntarget, t0, nl, L, log_n, n); break;
        case 6: modup_conv_s<6, SCALED, CH>(x, dst, pcs, blk, alpha, start, ntarget, t0, nl, L, log_n, n); break;
        case 7: modup_conv_s<7, SCALED, CH>(x, dst, pcs, blk, alpha, start, ntarget, t0, nl, L, log_n, n); break;
        default: modup_conv_s<8, SCALED, CH>(x, dst, pcs, blk, alpha, start, ntarget, t0, nl, L, log_n, n); break;
    }
}

// V consecutive residues of one limb, read or written with one access of
// 8 V bytes (V = 2: 16-byte accesses, which the HBM streams faster than 8-byte
// ones).
template <int V>
__device__ __forceinline__ void load_v(const uint64_t *p, uint64_t (&r)[V]) {
    if constexpr (V == 2) {
        typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
        const u64x2 t = *reinterpret_cast<const u64x2 *>(p);
        r[0] = t.x;
        r[1] = t.y;
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) r[v] = p[v];
    }
}

template <int V>
__device__ __forceinline__ void store_v(uint64_t *p, const uint64_t (&r)[V]) {
    if constexpr (V == 2) {
        typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
        u64x2 t;
        t.x = r[0];
        t.y = r[1];
        *reinterpret_cast<u64x2 *>(p) = t;
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) p[v] = r[v];
    }
}

// Coefficients per thread of the inner product.  Two (16-byte accesses) was
// measured slower at N = 2^16, 24 + 4 limbs, alpha = 8: 36.0 against 34.8 us
// per launch (half the threads keep fewer loads in flight).
constexpr int kIpVec = 1;

// Inner product with the key on every limb m of Q_l u P (grid.y = m):
// ip[c][m] = sum_j src_j(m) * evk[j][c][g(m)], src_j(m) = d[m] if m is in digit j,
// else the ModUp output of digit j.  A thread takes V consecutive coefficients
// (gx = block of kEw V coefficients).
template <int V>
__device__ __forceinline__ void inner_product_unit(const uint64_t *__restrict__ d,
                                                   const uint64_t *__restrict__ ext,
                                                   const uint64_t *__restrict__ evk,
                                                   uint64_t *__restrict__ ip,
                                                   const PrimeConst *__restrict__ pcs, uint32_t log_n,
                                                   uint32_t nl, uint32_t L, uint32_t K, uint32_t alpha, uint32_t gx,
                                                   uint32_t gy, const IpFold &fold = IpFold()) {
    const uint32_t m = gy;
    const size_t n = ((size_t)gx * kEw + threadIdx.x) * V;
    const uint32_t g = m < nl ? m : L + (m - nl);
    const PrimeConst pc = pcs[g];
    const uint32_t dn = (nl + alpha - 1) / alpha;
    const size_t key_poly = (size_t)(L + K) << log_n;
    // HMult / HRotate sources of the Q-limbs (the P-limbs belong to no digit)
    uint64_t own[V], ad0[V], ad1[V];
#pragma unroll
    for (int v = 0; v < V; ++v) own[v] = ad0[v] = ad1[v] = 0;
    if (fold.mode != 0 && m < nl) {
        const size_t lo = (size_t)m << log_n, poly = (size_t)nl << log_n;
        if (fold.mode == 1) {
            uint64_t x0[V], x1[V], y0[V], y1[V];
            load_v<V>(fold.a + lo + n, x0);
            load_v<V>(fold.a + poly + lo + n, x1);
            load_v<V>(fold.b + lo + n, y0);
            load_v<V>(fold.b + poly + lo + n, y1);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                MacAcc s2, s0, s1;
                s2.mac(x1[v], y1[v]);
                s0.mac(x0[v], y0[v]);
                s1.mac(x0[v], y1[v]);
                s1.mac(x1[v], y0[v]);
                own[v] = reduce128(s2.value(), pc.q, pc.r64, pc.r64_p, pc.one_p);
                ad0[v] = reduce128(s0.value(), pc.q, pc.r64, pc.r64_p, pc.one_p);
                ad1[v] = reduce128(s1.value(), pc.q, pc.r64, pc.r64_p, pc.one_p);
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const size_t src = lo + galois_src((uint32_t)(n + v), fold.galois, log_n);
                own[v] = fold.a[poly + src];
                ad0[v] = fold.a[src];
            }
        }
    }
    u128 acc0[V], acc1[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc0[v] = acc1[v] = u128{0, 0};
#pragma unroll 4
    for (uint32_t j = 0; j < dn; ++j) {
        const uint32_t start = j * alpha;
        const uint32_t s = min(alpha, nl - start);
        uint64_t src[V];
        if (m >= start && m < start + s) {
            if (fold.mode != 0) {
#pragma unroll
                for (int v = 0; v < V; ++v) src[v] = own[v];
            } else {
                load_v<V>(d + ((size_t)m << log_n) + n, src);
            }
        } else {
            const uint32_t tt = m < start ? m : m - s;
            load_v<V>(ext + (((size_t)j * (nl + K - alpha) + tt) << log_n) + n, src);
        }
        const uint64_t *kj = evk + (size_t)(2 * j) * key_poly + ((size_t)g << log_n) + n;
        uint64_t k0[V], k1[V];
        load_v<V>(kj, k0);
        load_v<V>(kj + key_poly, k1);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            mac(acc0[v], src[v], k0[v]);
            mac(acc1[v], src[v], k1[v]);
        }
    }
    const size_t out_poly = (size_t)(nl + K) << log_n;
    uint64_t r0[V], r1[V];
    const uint64_t q2 = 2 * pc.q;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        // [0, 4q): the Shoup product by P^-1 takes any 64-bit input, the other
        // outputs are made canonical below
        r0[v] = reduce128_lazy(acc0[v], pc.q, pc.r64, pc.r64_p, pc.one_p);
        r1[v] = reduce128_lazy(acc1[v], pc.q, pc.r64, pc.r64_p, pc.one_p);
    }
    if (fold.pinv && m < nl) {
        const uint64_t pinv = fold.pinv[2 * m], pinv_p = fold.pinv[2 * m + 1];
        const size_t lo = (size_t)m << log_n;
        uint64_t a0[V], a1[V];
        if (fold.mode == 0) {
            if (fold.add0) load_v<V>(fold.add0 + lo + n, a0);
            if (fold.add1) load_v<V>(fold.add1 + lo + n, a1);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            r0[v] = shoup(r0[v], pinv, pinv_p, pc.q);
            r1[v] = shoup(r1[v], pinv, pinv_p, pc.q);
            if (fold.mode == 1) {
                r0[v] = addmod(r0[v], ad0[v], pc.q);
                r1[v] = addmod(r1[v], ad1[v], pc.q);
            } else if (fold.mode == 2) {
                r0[v] = addmod(r0[v], ad0[v], pc.q);
            } else {
                if (fold.add0) r0[v] = addmod(r0[v], a0[v], pc.q);
                if (fold.add1) r1[v] = addmod(r1[v], a1[v], pc.q);
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            r0[v] = csub(csub(r0[v], q2), pc.q);
            r1[v] = csub(csub(r1[v], q2), pc.q);
        }
    }
    store_v<V>(ip + ((size_t)m << log_n) + n, r0);
    store_v<V>(ip + out_poly + ((size_t)m << log_n) + n, r1);
}

// ModDown conversion of one chunk of Q targets from KP special primes
// (compile-time), centred digits.
template <int KP>
__device__ __forceinline__ void moddown_conv_k(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
                                               const PrimeConst *__restrict__ pcs, const uint64_t *__restrict__ tab,
                                               uint32_t i0, uint32_t nl, uint32_t L, uint32_t log_n) {
    const uint64_t *cross = tab + 2 * KP;
    const uint64_t *negp = tab + 2 * KP + (size_t)KP * L + 2 * (size_t)L;
    uint32_t yl[KP], yh[KP];
    uint64_t cnt = 0;
#pragma unroll
    for (int a = 0; a < KP; ++a) {
        const uint64_t p = pcs[L + a].q;
        const uint64_t y = shoup(src[(size_t)a << log_n], tab[2 * a], tab[2 * a + 1], p);
        cnt += y > (p >> 1) ? 1u : 0u;
        yl[a] = (uint32_t)y & 0x3fffffffu;
        yh[a] = (uint32_t)(y >> 30);
    }
#pragma unroll
    for (int k = 0; k < kConvChunk; ++k) {
        const uint32_t i = i0 + k;
        if (i < nl) {
            const PrimeConst pc = pcs[i];
            const uint64_t *ci = cross + (size_t)i * KP;
            MacAcc acc;
            acc.add(cnt * negp[i]);
#pragma unroll
            for (int a = 0; a < KP; ++a) acc.mac_split(yl[a], yh[a], ci[a]);
            dst[(size_t)i << log_n] = reduce128_lazy(acc.value(), pc.q, pc.r64, pc.r64_p, pc.one_p);
        }
    }
}

// ModDown base conversion P -> Q_l with centred digits, gy = polynomial *
// moddown_chunks + chunk.  ip = [2][nl + K][N] with the K P-limbs already in
// the coefficient domain; conv = [2][nl][N] coefficient domain, residues in
// [0, 4q) (a forward NTT follows).
__device__ __forceinline__ void moddown_bconv_unit(const uint64_t *__restrict__ ip, uint64_t *__restrict__ conv,
                                                   const PrimeConst *__restrict__ pcs,
                                                   const uint64_t *__restrict__ tab, uint32_t log_n,
                                                   uint32_t nl, uint32_t L, uint32_t K, uint32_t gx, uint32_t gy) {
    const uint32_t nch = moddown_chunks(nl);
    const uint32_t c = gy / nch, ch = gy - c * nch;
    const uint32_t i0 = ch * kConvChunk;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const uint64_t *src = ip + (((size_t)c * (nl + K) + nl) << log_n) + n;
    uint64_t *dst = conv + (((size_t)c * nl) << log_n) + n;
    switch (K) {
        case 1: moddown_conv_k<1>(src, dst, pcs, tab, i0, nl, L, log_n); break;
        case 2: moddown_conv_k<2>(src, dst, pcs, tab, i0, nl, L, log_n); break;
        case 3: moddown_conv_k<3>(src, dst, pcs, tab, i0, nl, L, log_n); break;
        case 4: moddown_conv_k<4>(src, dst, pcs, tab, i0, nl, L, log_n); break;
        case 5: moddown_conv_k<5>(src, dst, pcs, tab, i0, nl, L, log_n); break;
        case 6: moddown_conv_k<6>(src, dst, pcs, tab, i0, nl, L, log_n); break;
        case 7: moddown_conv_k<7>(src, dst, pcs, tab, i0, nl, L, log_n); break;
        default: moddown_conv_k<8>(src, dst, pcs, tab, i0, nl, L, log_n); break;
    }
}

// out[c][i] = (ip[c][i] - conv[c][i]) * P^-1 mod q_i  (+ add_c[i] when add_c != null).
// grid.y = c * nl + i.  add_c may alias out (same element is read then written).
__device__ __forceinline__ void moddown_tail_unit(const uint64_t *__restrict__ ip,
                                                           const uint64_t *__restrict__ conv, const uint64_t *add0,
                                                           const uint64_t *add1, uint64_t *out,
                                                           const PrimeConst *__restrict__ pcs,
                                                           const uint64_t *__restrict__ pinv, uint32_t log_n,
                                                           uint32_t nl, uint32_t K, uint32_t gx, uint32_t gy) {
    const uint32_t c = gy / nl, i = gy - c * nl;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const PrimeConst pc = pcs[i];
    const uint64_t x = ip[(((size_t)c * (nl + K) + i) << log_n) + n];
    const size_t off = (((size_t)c * nl + i) << log_n) + n;
    uint64_t r = shoup(submod(x, conv[off], pc.q), pinv[2 * i], pinv[2 * i + 1], pc.q);
    const uint64_t *add = c == 0 ? add0 : add1;
    if (add) r = addmod(r, add[((size_t)i << log_n) + n], pc.q);
    out[off] = r;
}

// Rescale / modulus switch, step 1: the last limb (coefficient domain, [2][N])
// lifted from its centred representative into every remaining prime:
// lift = [2][nl-1][N].  KEEP_T (BGV): the lifted value is t [x t^-1]_{q_l}, so
// that the difference is 0 mod t as well as mod q_l.
template <bool KEEP_T>
__device__ __forceinline__ void rescale_lift_unit(const uint64_t *__restrict__ last, uint64_t *__restrict__ lift,
                                                           const PrimeConst *__restrict__ pcs,
                                                           const uint64_t *__restrict__ tab, uint32_t log_n,
                                                           uint32_t nl, uint32_t L, uint32_t gx, uint32_t gy) {
    const uint32_t l = nl - 1;
    const uint32_t c = gy / l, i = gy - c * l;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const PrimeConst pl = pcs[l];
    const PrimeConst pc = pcs[i];
    uint64_t x = last[((size_t)c << log_n) + n];
    if (KEEP_T) x = shoup(x, pl.tinv, pl.tinv_p, pl.q);
    uint64_t r = barrett64(x, pc.mu1, pc.mu0, pc.q);
    if (x > (pl.q >> 1)) r = addmod(r, tab[((size_t)l * L + i) * 3 + 2], pc.q);
    if (KEEP_T) r = shoup(r, pc.tmod, pc.tmod_p, pc.q);
    lift[(((size_t)c * l + i) << log_n) + n] = r;
}

// Rescale, step 2: out[c][i] = (in[c][i] - lift[c][i]) * q_l^-1 mod q_i.  grid.y = c * (nl-1) + i.
// out may equal lift.
__device__ __forceinline__ void rescale_tail_unit(const uint64_t *__restrict__ in, const uint64_t *lift,
                                                           uint64_t *out, const PrimeConst *__restrict__ pcs,
                                                           const uint64_t *__restrict__ tab, uint32_t log_n,
                                                           uint32_t nl, uint32_t L, uint32_t gx, uint32_t gy) {
    const uint32_t l = nl - 1;
    const uint32_t c = gy / l, i = gy - c * l;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const PrimeConst pc = pcs[i];
    const uint64_t *t = tab + ((size_t)l * L + i) * 3;
    const size_t off = (((size_t)c * l + i) << log_n) + n;
    const uint64_t x = in[(((size_t)c * nl + i) << log_n) + n];
    out[off] = shoup(submod(x, lift[off], pc.q), t[0], t[1], pc.q);
}

// sigma_g in the NTT domain: out[k] = in[k'] with 2 brv(k') + 1 = (2 brv(k) + 1) g mod 2N.
// grid.y = polynomial * nl + limb (the permutation is the same on every limb).
__device__ __forceinline__ void automorphism_unit(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                           uint32_t galois, uint32_t log_n, uint32_t gx, uint32_t gy) {
    const uint32_t k = gx * kEw + threadIdx.x;
    const size_t base = (size_t)gy << log_n;
    out[base + k] = in[base + galois_src(k, galois, log_n)];
}

}  // namespace rf

namespace rf {

// Element-wise residue operations (the paper's lower-tier add / sub / multiply,
// II and III-A, one thread per residue).  OP: 0 add, 1 sub, 2 multiply by a
// signed integer constant, 3 add a signed integer constant (polynomial 0 only,
// polynomial 1 copied), 4 multiply by a plaintext polynomial [nl][N].
// gy = polynomial * nl + limb.
template <int OP>
__device__ __forceinline__ void ewise_unit(const uint64_t *a, const uint64_t *b, int64_t k, uint64_t *out,
                                           const PrimeConst *__restrict__ pcs, uint32_t log_n, uint32_t nl,
                                           uint32_t gx, uint32_t gy) {
    const uint32_t poly = gy / nl, i = gy - poly * nl;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const size_t off = ((size_t)gy << log_n) + n;
    const PrimeConst pc = pcs[i];
    const uint64_t x = a[off];
    uint64_t r;
    if constexpr (OP == 0) {
        r = addmod(x, b[off], pc.q);
    } else if constexpr (OP == 1) {
        r = submod(x, b[off], pc.q);
    } else if constexpr (OP == 4) {
        r = mulmod(x, b[((size_t)i << log_n) + n], pc.mu1, pc.mu0, pc.q);
    } else {
        const uint64_t mag = k < 0 ? (uint64_t)0 - (uint64_t)k : (uint64_t)k;
        uint64_t km = barrett64(mag, pc.mu1, pc.mu0, pc.q);
        if (k < 0 && km) km = pc.q - km;
        if constexpr (OP == 2) r = mulmod(x, km, pc.mu1, pc.mu0, pc.q);
        else r = poly == 0 ? addmod(x, km, pc.q) : x;
    }
    out[off] = r;
}

}  // namespace rf

namespace rf {

// Exact sum of (yh 2^30 + yl)[i] * coef(i) for i < n <= NMAX (pre-split
// operands and coefficients below 2^60), in groups of 8 products (MacAcc).
template <int NMAX, typename F>
__device__ __forceinline__ u128 dot_split(const uint32_t *yl, const uint32_t *yh, F coef, int n) {
    u128 total = {0, 0};
#pragma unroll
    for (int g = 0; g < (NMAX + 7) / 8; ++g) {
        MacAcc acc;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = g * 8 + k;
            if (i < NMAX && i < n) acc.mac_split(yl[i], yh[i], coef(i));
        }
        add_wide(total, acc.value());
    }
    return total;
}

// Conversions of the BEHZ multiplication, each split over groups of
// kBehzGroup output limbs so that a launch has several threads per
// coefficient (one thread per coefficient and every output limb left 1.5-2
// waves per SIMD, each running thousands of dependent instructions); the
// per-coefficient inputs of a group are recomputed by each group.  Measured
// at N = 2^15, 14 + 15 limbs, BFV HMult+Relin: groups of 4, 8 and 16 took
// 348, 343 and 374 us (16: one group, 3 waves per SIMD).
constexpr int kBehzGroup = 8;

__host__ __device__ inline uint32_t behz_groups(uint32_t limbs) { return (limbs + kBehzGroup - 1) / kBehzGroup; }

// BEHZ step 1 for one coefficient-domain polynomial (a0, a1, b0, b1):
// fast conversion of [m~ x]_q to B_sk, then the small Montgomery reduction
// by m~ = 2^32: with y_i = [x_i m~ (Q/q_i)^-1]_{q_i} and r = -(sum_i y_i
// [Q/q_i]_{m~}) Q^-1 mod m~ taken centred, out_m = (sum_i y_i [Q/q_i]_m + r Q)
// m~^-1 mod bsk_m (the factor m~^-1 is folded into the tables).  gy =
// poly * behz_groups(nb + 1) + group; the group's outputs are m = kBehzGroup
// group + k.  ext = [poly][L + nb + 1][N]: the q part is a copy of x (written
// by group 0), then b_0..b_{nb-1}, m_sk.  Prime indices: q_i = i, bsk_m =
// kb + m.
__device__ __forceinline__ void behz_extend_unit(const uint64_t *a, const uint64_t *b, uint64_t *ext,
                                                 const PrimeConst *__restrict__ pcs, const uint64_t *__restrict__ tab,
                                                 BehzLayout o, uint32_t kb, uint32_t log_n, uint32_t gx, uint32_t gy) {
    const uint32_t L = o.L, nb = o.nb, W = L + nb + 1;
    const uint32_t ng = behz_groups(nb + 1);
    const uint32_t poly = gy / ng, m0 = (gy - poly * ng) * kBehzGroup;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const size_t psz = (size_t)L << log_n;
    const uint64_t *x = (poly < 2 ? a : b) + (poly & 1) * psz + n;
    uint64_t *dst = ext + (((size_t)poly * W) << log_n) + n;
    uint32_t yl[kMaxBfvLimbs], yh[kMaxBfvLimbs];
    uint32_t acc_mt = 0;
#pragma unroll
    for (int i = 0; i < kMaxBfvLimbs; ++i) {
        yl[i] = yh[i] = 0;
        if (i < (int)L) {
            const uint64_t xi = x[(size_t)i << log_n];
            if (m0 == 0) dst[(size_t)i << log_n] = xi;
            const uint64_t y = shoup(xi, tab[o.ext_factor + 2 * i], tab[o.ext_factor + 2 * i + 1], pcs[i].q);
            yl[i] = (uint32_t)y & 0x3fffffffu;
            yh[i] = (uint32_t)(y >> 30);
            acc_mt += (uint32_t)y * (uint32_t)tab[o.cross_q_mt + i];
        }
    }
    // r = -x~_{m~} Q^-1 mod 2^32, centred
    const uint32_t r32 = acc_mt * (uint32_t)tab[o.neg_qinv_mt];
    const bool neg = r32 >= 0x80000000u;
    const uint64_t rmag = neg ? (uint64_t)(0x100000000ull - r32) : (uint64_t)r32;
#pragma unroll
    for (int k = 0; k < kBehzGroup; ++k) {
        const uint32_t m = m0 + k;
        if (m <= nb) {
            const PrimeConst pc = pcs[kb + m];
            const uint64_t *cm = tab + o.ext_cross + (size_t)m * L;
            const u128 acc = dot_split<kMaxBfvLimbs>(yl, yh, [&](int i) { return cm[i]; }, L);
            const uint64_t v = reduce128(acc, pc.q, pc.r64, pc.r64_p, pc.one_p);
            const uint64_t rq = shoup(rmag, tab[o.ext_q + 2 * m], tab[o.ext_q + 2 * m + 1], pc.q);
            dst[(size_t)(L + m) << log_n] = neg ? submod(v, rq, pc.q) : addmod(v, rq, pc.q);
        }
    }
}

// Fast floor into B_sk of polynomial gy / behz_groups(nb + 1), outputs
// m = kBehzGroup (gy % behz_groups(nb + 1)) + k: f_m = (t d_m - conv_m) Q^-1
// mod bsk_m with conv_m = sum_i [d_i t (Q/q_i)^-1]_{q_i} [Q/q_i]_m, into
// f [3][nb+1][N].
__device__ __forceinline__ void behz_floor_unit(const uint64_t *tens, uint64_t *f, const PrimeConst *__restrict__ pcs,
                                                const uint64_t *__restrict__ tab, BehzLayout o, uint32_t kb,
                                                uint32_t log_n, uint32_t gx, uint32_t gy) {
    const uint32_t L = o.L, nb = o.nb, W = L + nb + 1;
    const uint32_t ng = behz_groups(nb + 1);
    const uint32_t poly = gy / ng, m0 = (gy - poly * ng) * kBehzGroup;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const uint64_t *d = tens + (((size_t)poly * W) << log_n) + n;
    uint32_t zl[kMaxBfvLimbs], zh[kMaxBfvLimbs];
#pragma unroll
    for (int i = 0; i < kMaxBfvLimbs; ++i) {
        zl[i] = zh[i] = 0;
        if (i < (int)L) {
            const uint64_t z = shoup(d[(size_t)i << log_n], tab[o.floor_factor + 2 * i],
                                     tab[o.floor_factor + 2 * i + 1], pcs[i].q);
            zl[i] = (uint32_t)z & 0x3fffffffu;
            zh[i] = (uint32_t)(z >> 30);
        }
    }
#pragma unroll
    for (int k = 0; k < kBehzGroup; ++k) {
        const uint32_t m = m0 + k;
        if (m <= nb) {
            const PrimeConst pc = pcs[kb + m];
            const uint64_t *cm = tab + o.floor_cross + (size_t)m * L;
            const u128 acc = dot_split<kMaxBfvLimbs>(zl, zh, [&](int i) { return cm[i]; }, L);
            const uint64_t conv = reduce128(acc, pc.q, pc.r64, pc.r64_p, pc.one_p);
            const uint64_t td = shoup(d[(size_t)(L + m) << log_n], tab[o.t_bsk + 2 * m], tab[o.t_bsk + 2 * m + 1],
                                      pc.q);
            f[(((size_t)poly * (nb + 1) + m) << log_n) + n] =
                shoup(submod(td, conv, pc.q), tab[o.qinv_bsk + 2 * m], tab[o.qinv_bsk + 2 * m + 1], pc.q);
        }
    }
}

// Shenoy-Kumaresan conversion B_sk -> q of polynomial gy / behz_groups(L),
// outputs i = kBehzGroup (gy % behz_groups(L)) + k: w_j = f_j (M/b_j)^-1 mod
// b_j, alpha from the m_sk residue (centred), out_i = sum_j w_j [M/b_j]_{q_i}
// - alpha M mod q_i; polynomials 0, 1 to out01 [2][L][N], 2 to out2 [L][N].
__device__ __forceinline__ void behz_sk_unit(const uint64_t *f, uint64_t *out01, uint64_t *out2,
                                             const PrimeConst *__restrict__ pcs, const uint64_t *__restrict__ tab,
                                             BehzLayout o, uint32_t kb, uint32_t log_n, uint32_t gx, uint32_t gy) {
    const uint32_t L = o.L, nb = o.nb;
    const uint32_t ng = behz_groups(L);
    const uint32_t poly = gy / ng, i0 = (gy - poly * ng) * kBehzGroup;
    const size_t n = (size_t)gx * kEw + threadIdx.x;
    const uint64_t *fp = f + (((size_t)poly * (nb + 1)) << log_n) + n;
    uint32_t wl[kMaxBfvLimbs], wh[kMaxBfvLimbs];
#pragma unroll
    for (int j = 0; j < kMaxBfvLimbs; ++j) {
        wl[j] = wh[j] = 0;
        if (j < (int)nb) {
            const uint64_t w = shoup(fp[(size_t)j << log_n], tab[o.sk_factor + 2 * j], tab[o.sk_factor + 2 * j + 1],
                                     pcs[kb + j].q);
            wl[j] = (uint32_t)w & 0x3fffffffu;
            wh[j] = (uint32_t)(w >> 30);
        }
    }
    const u128 acc_msk = dot_split<kMaxBfvLimbs>(wl, wh, [&](int j) { return tab[o.cross_b_msk + j]; }, nb);
    const PrimeConst pm = pcs[kb + nb];
    const uint64_t fmsk = fp[(size_t)nb << log_n];
    const uint64_t cmsk = reduce128(acc_msk, pm.q, pm.r64, pm.r64_p, pm.one_p);
    const uint64_t alpha = shoup(submod(cmsk, fmsk, pm.q), tab[o.minv_msk], tab[o.minv_msk + 1], pm.q);
    const bool neg = alpha > (pm.q >> 1);
    const uint64_t amag = neg ? pm.q - alpha : alpha;
    uint64_t *out = (poly < 2 ? out01 + (((size_t)poly * L) << log_n) : out2) + n;
#pragma unroll
    for (int k = 0; k < kBehzGroup; ++k) {
        const uint32_t i = i0 + k;
        if (i < L) {
            const PrimeConst pc = pcs[i];
            const uint64_t *ci = tab + o.sk_cross + (size_t)i * nb;
            const u128 acc = dot_split<kMaxBfvLimbs>(wl, wh, [&](int j) { return ci[j]; }, nb);
            const uint64_t r = reduce128(acc, pc.q, pc.r64, pc.r64_p, pc.one_p);
            // amag < m_sk < 2^64: one Shoup product by [M]_{q_i}
            const uint64_t am = shoup(amag, tab[o.m_q + 2 * i], tab[o.m_q + 2 * i + 1], pc.q);
            out[(size_t)i << log_n] = neg ? addmod(r, am, pc.q) : submod(r, am, pc.q);
        }
    }
}

}  // namespace rf
