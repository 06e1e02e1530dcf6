/*
 * Plain, slow arithmetic core of the CPU oracle (test infrastructure only:
 * nothing in the product library links or loads this file).
 *
 * Every residue is a uint64_t in [0, q).  Every modular product is the
 * definition (a * b) mod q evaluated on a 128-bit integer with the C `%`
 * operator: no Barrett, Shoup or Montgomery forms, no lazy ranges.
 *
 * The NTT follows the textbook negacyclic transform over R_q = Z_q[X]/(X^N+1)
 * (the ring of the paper's notation section): output index i holds
 * a(psi^(2*brv(i)+1)), psi a primitive 2N-th root of unity mod q and brv the
 * log2(N)-bit reversal.  It is computed with the radix-2 Cooley-Tukey
 * recursion (decimation in time, powers of psi merged into the twiddles); the
 * inverse runs the Gentleman-Sande butterflies in the opposite order and
 * scales by N^-1.  The Python side pins both against the O(N^2) definition.
 */
#include <stdint.h>
#include <stdlib.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a * b) % q);
}

static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a + b) % q);
}

static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a + q - b) % q);
}

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

static uint32_t bitrev(uint32_t x, int bits) {
    uint32_t r = 0;
    for (int i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

uint64_t orc_mulmod(uint64_t a, uint64_t b, uint64_t q) { return mulmod(a, b, q); }
uint64_t orc_powmod(uint64_t b, uint64_t e, uint64_t q) { return powmod(b, e, q); }

/* table[k] = root^(brv(k)) for k < n */
static uint64_t *brv_power_table(int log_n, uint64_t root, uint64_t q) {
    uint32_t n = 1u << log_n;
    uint64_t *pw = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t *tw = (uint64_t *)malloc(sizeof(uint64_t) * n);
    pw[0] = 1 % q;
    for (uint32_t e = 1; e < n; e++) pw[e] = mulmod(pw[e - 1], root, q);
    for (uint32_t k = 0; k < n; k++) tw[k] = pw[bitrev(k, log_n)];
    free(pw);
    return tw;
}

/* Forward negacyclic NTT of one limb, in place; psi is a primitive 2N-th root mod q. */
void orc_ntt_fwd(uint64_t *a, int log_n, uint64_t q, uint64_t psi) {
    uint32_t n = 1u << log_n;
    uint64_t *tw = brv_power_table(log_n, psi, q);
    for (uint32_t m = 1, t = n / 2; m < n; m *= 2, t /= 2) {
        for (uint32_t i = 0; i < m; i++) {
            uint64_t w = tw[m + i];
            for (uint32_t j = 2 * i * t; j < 2 * i * t + t; j++) {
                uint64_t u = a[j];
                uint64_t v = mulmod(a[j + t], w, q);
                a[j] = addmod(u, v, q);
                a[j + t] = submod(u, v, q);
            }
        }
    }
    free(tw);
}

/* Inverse of orc_ntt_fwd, in place. */
void orc_ntt_inv(uint64_t *a, int log_n, uint64_t q, uint64_t psi) {
    uint32_t n = 1u << log_n;
    uint64_t psi_inv = powmod(psi, q - 2, q);
    uint64_t *tw = brv_power_table(log_n, psi_inv, q);
    for (uint32_t m = n / 2, t = 1; m >= 1; m /= 2, t *= 2) {
        for (uint32_t i = 0; i < m; i++) {
            uint64_t w = tw[m + i];
            for (uint32_t j = 2 * i * t; j < 2 * i * t + t; j++) {
                uint64_t u = a[j];
                uint64_t v = a[j + t];
                a[j] = addmod(u, v, q);
                a[j + t] = mulmod(submod(u, v, q), w, q);
            }
        }
    }
    uint64_t n_inv = powmod(n % q, q - 2, q);
    for (uint32_t j = 0; j < n; j++) a[j] = mulmod(a[j], n_inv, q);
    free(tw);
}

/* Element-wise operations on one limb of n residues. */
void orc_mul(const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n, uint64_t q) {
    for (uint64_t j = 0; j < n; j++) out[j] = mulmod(a[j], b[j], q);
}
void orc_add(const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n, uint64_t q) {
    for (uint64_t j = 0; j < n; j++) out[j] = addmod(a[j], b[j], q);
}
void orc_sub(const uint64_t *a, const uint64_t *b, uint64_t *out, uint64_t n, uint64_t q) {
    for (uint64_t j = 0; j < n; j++) out[j] = submod(a[j], b[j], q);
}
void orc_mul_scalar(const uint64_t *a, uint64_t c, uint64_t *out, uint64_t n, uint64_t q) {
    for (uint64_t j = 0; j < n; j++) out[j] = mulmod(a[j], c, q);
}

/*
 * Fast base conversion from the basis {in_mod[i]} to the basis {out_mod[m]},
 * with no correction of the overflow:
 *   y_i   = x_i * in_factor[i] mod in_mod[i]
 *   out_m = sum_i y_i * cross[i * n_out + m]  mod out_mod[m]
 * With centred != 0 each y_i is first taken to its representative in
 * (-in_mod[i]/2, in_mod[i]/2] (a signed integer) before the sum.
 * x is [n_in][n], out is [n_out][n].
 */
void orc_bconv(const uint64_t *x, int n_in, const uint64_t *in_mod, const uint64_t *in_factor,
               int n_out, const uint64_t *out_mod, const uint64_t *cross, uint64_t *out,
               uint64_t n, int centred) {
    __int128 *y = (__int128 *)malloc(sizeof(__int128) * (size_t)n_in);
    for (uint64_t j = 0; j < n; j++) {
        for (int i = 0; i < n_in; i++) {
            uint64_t r = mulmod(x[(size_t)i * n + j], in_factor[i], in_mod[i]);
            y[i] = (__int128)r;
            if (centred && r > in_mod[i] / 2) y[i] -= (__int128)in_mod[i];
        }
        for (int m = 0; m < n_out; m++) {
            __int128 mod = (__int128)out_mod[m];
            uint64_t s = 0;
            for (int i = 0; i < n_in; i++) {
                uint64_t yi = (uint64_t)(((y[i] % mod) + mod) % mod);
                s = addmod(s, mulmod(yi, cross[(size_t)i * n_out + m], out_mod[m]), out_mod[m]);
            }
            out[(size_t)m * n + j] = s;
        }
    }
    free(y);
}

/*
 * Automorphism a(X) -> a(X^g) of one limb in the coefficient domain (g odd):
 * coefficient j moves to g*j mod 2N and changes sign when that index is >= N.
 */
void orc_automorphism_coeff(const uint64_t *a, uint64_t *out, int log_n, uint64_t g, uint64_t q) {
    uint64_t n = 1ull << log_n;
    for (uint64_t j = 0; j < n; j++) {
        uint64_t k = (uint64_t)(((u128)j * g) % (2 * n));
        if (k < n) out[k] = a[j];
        else out[k - n] = submod(0, a[j], q);
    }
}
