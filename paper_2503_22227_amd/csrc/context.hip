// Context creation: every table the kernels read is derived here, on the host,
// from the primes the caller passes (the paper's "pre-computed elements" of the
// middle tier, section III), and uploaded once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ntt_dev.hpp"
#include "rf_internal.hpp"

namespace {

typedef unsigned __int128 u128h;

uint64_t mulmod_h(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128h)a * b) % q); }

uint64_t powmod_h(uint64_t b, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod_h(r, b, q);
        b = mulmod_h(b, b, q);
        e >>= 1;
    }
    return r;
}

uint64_t inv_h(uint64_t a, uint64_t q) { return powmod_h(a % q, q - 2, q); }  // q prime

// Deterministic Miller-Rabin for 64-bit integers (bases 2..37).
bool is_prime_h(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : bases)
        if (n % p == 0) return n == p;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++s;
    }
    for (uint64_t a : bases) {
        uint64_t x = powmod_h(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod_h(x, x, n);
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

uint64_t shoup_companion(uint64_t w, uint64_t q) { return (uint64_t)(((u128h)w << 64) / q); }
// companion of the NTT twiddles, scaled by 2^62 (shoup62_lazy)
uint64_t shoup_companion62(uint64_t w, uint64_t q) { return (uint64_t)(((u128h)w << 62) / q); }

uint32_t bitrev_h(uint32_t x, int bits) {
    uint32_t r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

// psi_max = g^((q-1)/(2 nmax)) for the smallest g >= 2 with psi_max^nmax = -1.
uint64_t root_2n(uint64_t q, uint64_t nmax) {
    for (uint64_t g = 2;; ++g) {
        uint64_t psi = powmod_h(g, (q - 1) / (2 * nmax), q);
        if (powmod_h(psi, nmax, q) == q - 1) return psi;
    }
}

template <typename T>
int upload(T **dst, const std::vector<T> &src) {
    size_t bytes = src.size() * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    if (hipMalloc((void **)dst, bytes) != hipSuccess) return rf::fail(RF_EHIP, "hipMalloc of a context table failed");
    if (!src.empty() && hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return rf::fail(RF_EHIP, "hipMemcpy of a context table failed");
    return RF_OK;
}

}  // namespace

namespace rf {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

const char *last_error() { return g_last_error.c_str(); }

}  // namespace rf

static void free_tables(rf_ctx *c) {
    (void)hipFree(c->d_pc);
    (void)hipFree(c->d_pc_md);
    (void)hipFree(c->d_pc_mu);
    (void)hipFree(c->d_tw_fwd);
    (void)hipFree(c->d_tw_inv);
    (void)hipFree(c->d_tw_fwd_rows);
    (void)hipFree(c->d_tw_inv_rows);
    (void)hipFree(c->d_modup);
    (void)hipFree(c->d_moddown);
    (void)hipFree(c->d_moddown_t);
    (void)hipFree(c->d_rescale);
    (void)hipFree(c->d_pmaps);
    (void)hipFree(c->d_behz);
    (void)hipFree(c->d_pmap_qb);
    (void)hipFree(c->d_client);
    (void)hipFree(c->d_garner);
    (void)hipFree(c->d_zeta);
    (void)hipFree(c->d_slot_idx);
}

extern "C" int rf_ctx_create(const rf_params *p, int device, rf_ctx **out) {
    using namespace rf;
    if (!p || !out) return fail(RF_EINVAL, "rf_ctx_create: null argument");
    *out = nullptr;
    if (p->scheme < RF_CKKS || p->scheme > RF_BGV) return fail(RF_EINVAL, "unknown scheme");
    if (p->log_n < 12 || p->log_n > 16) return fail(RF_EUNSUPPORTED, "log_n must be in [12, 16]");
    if (p->log_nmax < p->log_n || p->log_nmax > 20) return fail(RF_EINVAL, "log_nmax must be in [log_n, 20]");
    if (p->n_q < 1 || p->n_p < 1 || !p->q || !p->p) return fail(RF_EINVAL, "need at least one q and one p prime");
    if (p->n_q + p->n_p > (uint32_t)kMaxPrimes) return fail(RF_EUNSUPPORTED, "too many primes");
    if (p->alpha < 1 || p->alpha > (uint32_t)kMaxAlpha) return fail(RF_EUNSUPPORTED, "alpha must be in [1, 8]");
    if (p->n_p > 8) return fail(RF_EUNSUPPORTED, "at most 8 special primes");
    if (p->scheme != RF_CKKS && (p->t < 2 || p->t >= (1ull << 32)))
        return fail(RF_EINVAL, "BFV/BGV need a plaintext modulus 2 <= t < 2^32");
    if (p->scheme == RF_BFV) {
        if (p->n_b < 1 || !p->b || p->m_sk == 0) return fail(RF_EINVAL, "BFV needs an auxiliary base B and m_sk");
        if (p->n_b > (uint32_t)kMaxBfvLimbs || p->n_q > (uint32_t)kMaxBfvLimbs)
            return fail(RF_EUNSUPPORTED, "BFV: at most 24 Q-primes and 24 auxiliary primes");
    }
    if (p->n_q + p->n_p + (p->scheme == RF_BFV ? p->n_b + 1 : 0) > (uint32_t)kMaxPrimes)
        return fail(RF_EUNSUPPORTED, "too many primes");

    rf_ctx *c = new rf_ctx();
    c->device = device;
    c->scheme = p->scheme;
    c->log_n = p->log_n;
    c->log_nmax = p->log_nmax;
    c->n = 1u << p->log_n;
    c->L = p->n_q;
    c->K = p->n_p;
    c->alpha = p->alpha;
    c->dnum = (c->L + c->alpha - 1) / c->alpha;
    c->t = p->t;
    for (uint32_t i = 0; i < c->L; ++i) c->primes.push_back(p->q[i]);
    for (uint32_t i = 0; i < c->K; ++i) c->primes.push_back(p->p[i]);
    if (c->scheme == RF_BFV) {
        c->nb = p->n_b;
        for (uint32_t i = 0; i < c->nb; ++i) c->primes.push_back(p->b[i]);
        c->primes.push_back(p->m_sk);
    }
    const uint64_t nmax = 1ull << c->log_nmax;
    const uint32_t N = c->n;
    const uint32_t NP = (uint32_t)c->primes.size();
    for (uint32_t g = 0; g < NP; ++g) {
        uint64_t q = c->primes[g];
        if (q >= (1ull << 60) || q < 3 || (q - 1) % (2 * nmax) != 0 || !is_prime_h(q)) {
            delete c;
            return fail(RF_EINVAL, "prime " + std::to_string(g) + " is not an NTT-friendly prime below 2^60");
        }
        for (uint32_t h = 0; h < g; ++h)
            if (c->primes[h] == q) {
                delete c;
                return fail(RF_EINVAL, "primes must be distinct");
            }
        uint64_t psi_max = root_2n(q, nmax);
        c->psi.push_back(powmod_h(psi_max, nmax / N, q));
    }

    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return fail(RF_EHIP, "hipSetDevice failed");
    }

    // per-prime constants and twiddle tables
    std::vector<PrimeConst> pc(NP);
    std::vector<TwPair> twf((size_t)NP * N), twi((size_t)NP * N);
    std::vector<TwPair> twrf, twri;
    if (c->log_n > 12) {
        // the row-pass layout must be a permutation of each stage block
        const int A = ntt_split_a((int)c->log_n), B = (int)c->log_n - A;
        for (int dir = 0; dir < 2; ++dir) {
            std::vector<uint8_t> seen(N, 0);
            for (int s = 0; s < B; ++s)
                for (uint32_t r = 0; r < (1u << A); ++r)
                    for (uint32_t j = 0; j < (1u << s); ++j) {
                        const uint32_t k = row_tw_index(A, B, dir == 0, r, s, j);
                        if (k < (1u << (A + s)) || k >= (2u << (A + s)) || seen[k]) {
                            delete c;
                            return fail(RF_EINVAL, "internal: row twiddle layout is not a permutation");
                        }
                        seen[k] = 1;
                    }
        }
        twrf.assign((size_t)NP * N, TwPair{0, 0});
        twri.assign((size_t)NP * N, TwPair{0, 0});
    }
    std::vector<uint64_t> pw(N), pwi(N);
    for (uint32_t g = 0; g < NP; ++g) {
        uint64_t q = c->primes[g];
        u128h mu = (~(u128h)0) / q;  // floor((2^128 - 1) / q) = floor(2^128 / q) for q not a power of 2
        pc[g].q = q;
        pc[g].mu1 = (uint64_t)(mu >> 64);
        pc[g].mu0 = (uint64_t)mu;
        uint64_t ninv = inv_h(N, q);
        pc[g].ninv = ninv;
        pc[g].ninv_p = shoup_companion(ninv, q);
        pc[g].r64 = (uint64_t)(((u128h)1 << 64) % q);
        pc[g].r64_p = shoup_companion(pc[g].r64, q);
        pc[g].one_p = shoup_companion(1, q);
        uint64_t psi = c->psi[g], psi_inv = inv_h(psi, q);
        pw[0] = pwi[0] = 1;
        for (uint32_t e = 1; e < N; ++e) {
            pw[e] = mulmod_h(pw[e - 1], psi, q);
            pwi[e] = mulmod_h(pwi[e - 1], psi_inv, q);
        }
        for (uint32_t k = 0; k < N; ++k) {
            uint32_t r = bitrev_h(k, c->log_n);
            TwPair &f = twf[(size_t)g * N + k];
            f.w = pw[r];
            f.wp = shoup_companion62(f.w, q);
            TwPair &b = twi[(size_t)g * N + k];
            b.w = pwi[r];
            b.wp = shoup_companion62(b.w, q);
        }
        if (c->log_n > 12) {
            // row-pass layout: entry (r, s, j) of the natural table moves to row_tw_index
            const int A = ntt_split_a((int)c->log_n), B = (int)c->log_n - A;
            for (int s = 0; s < B; ++s)
                for (uint32_t r = 0; r < (1u << A); ++r)
                    for (uint32_t j = 0; j < (1u << s); ++j) {
                        const size_t nat = ((size_t)1 << (A + s)) + ((size_t)r << s) + j;
                        twrf[(size_t)g * N + row_tw_index(A, B, true, r, s, j)] = twf[(size_t)g * N + nat];
                        twri[(size_t)g * N + row_tw_index(A, B, false, r, s, j)] = twi[(size_t)g * N + nat];
                    }
        }
        uint64_t wl = mulmod_h(twi[(size_t)g * N + 1].w, ninv, q);
        pc[g].wlast = wl;
        pc[g].wlast_p = shoup_companion(wl, q);
        pc[g].tmod = pc[g].tmod_p = pc[g].tinv = pc[g].tinv_p = 0;
        if (c->t > 1) {
            pc[g].tmod = c->t % q;
            pc[g].tmod_p = shoup_companion(pc[g].tmod, q);
            pc[g].tinv = inv_h(c->t, q);
            pc[g].tinv_p = shoup_companion(pc[g].tinv, q);
        }
    }

    // ModUp: for every digit j and every digit size s (a truncated last digit at a lower level)
    const uint32_t A = c->alpha;
    const uint32_t NQP = c->L + c->K;  // the key-switching basis Q u P
    c->modup_stride = 2 * (size_t)A + (size_t)A * NQP;
    std::vector<uint64_t> mu((size_t)c->dnum * A * c->modup_stride, 0);
    for (uint32_t j = 0; j < c->dnum; ++j) {
        for (uint32_t s = 1; s <= A; ++s) {
            uint32_t start = j * A;
            if (start + s > c->L) continue;
            uint64_t *blk = mu.data() + modup_block(c, j, s);
            for (uint32_t i = 0; i < s; ++i) {
                uint64_t qi = c->primes[start + i];
                uint64_t prod = 1;  // (Q_j / q_i) mod q_i
                for (uint32_t h = 0; h < s; ++h)
                    if (h != i) prod = mulmod_h(prod, c->primes[start + h] % qi, qi);
                uint64_t f = inv_h(prod, qi);
                blk[2 * i] = f;
                blk[2 * i + 1] = shoup_companion(f, qi);
                for (uint32_t g = 0; g < NQP; ++g) {
                    uint64_t m = c->primes[g];
                    uint64_t v = 1;
                    for (uint32_t h = 0; h < s; ++h)
                        if (h != i) v = mulmod_h(v, c->primes[start + h] % m, m);
                    blk[2 * A + (size_t)g * A + i] = v;  // target-major: a target's constants are contiguous
                }
            }
        }
    }

    // ModDown: P = p_0 ... p_{k-1} to every q_i
    std::vector<uint64_t> md(moddown_negp_off(c) + c->L, 0);
    for (uint32_t a = 0; a < c->K; ++a) {
        uint64_t pa = c->primes[c->L + a];
        uint64_t prod = 1;
        for (uint32_t h = 0; h < c->K; ++h)
            if (h != a) prod = mulmod_h(prod, c->primes[c->L + h] % pa, pa);
        uint64_t f = inv_h(prod, pa);
        md[2 * a] = f;
        md[2 * a + 1] = shoup_companion(f, pa);
        for (uint32_t i = 0; i < c->L; ++i) {
            uint64_t qi = c->primes[i];
            uint64_t v = 1;
            for (uint32_t h = 0; h < c->K; ++h)
                if (h != a) v = mulmod_h(v, c->primes[c->L + h] % qi, qi);
            md[moddown_cross_off(c) + (size_t)i * c->K + a] = v;  // target-major
        }
    }
    for (uint32_t i = 0; i < c->L; ++i) {
        uint64_t qi = c->primes[i];
        uint64_t P = 1;
        for (uint32_t h = 0; h < c->K; ++h) P = mulmod_h(P, c->primes[c->L + h] % qi, qi);
        uint64_t pinv = inv_h(P, qi);
        md[moddown_pinv_off(c) + 2 * i] = pinv;
        md[moddown_pinv_off(c) + 2 * i + 1] = shoup_companion(pinv, qi);
        md[moddown_negp_off(c) + i] = (qi - P) % qi;
    }

    // ModDown that keeps the message mod t: delta = t * conv(centred [y t^-1 (P/p)^-1]_p), folded
    // into the same table layout (factor * t^-1, cross * t, (q_i - [t P]_{q_i}))
    std::vector<uint64_t> mdt;
    if (c->t > 1) {
        mdt = md;
        for (uint32_t a = 0; a < c->K; ++a) {
            uint64_t pa = c->primes[c->L + a];
            uint64_t f = mulmod_h(md[2 * a], inv_h(c->t % pa, pa), pa);
            mdt[2 * a] = f;
            mdt[2 * a + 1] = shoup_companion(f, pa);
            for (uint32_t i = 0; i < c->L; ++i) {
                uint64_t qi = c->primes[i];
                size_t o = moddown_cross_off(c) + (size_t)i * c->K + a;
                mdt[o] = mulmod_h(md[o], c->t % qi, qi);
            }
        }
        for (uint32_t i = 0; i < c->L; ++i) {
            uint64_t qi = c->primes[i];
            uint64_t P = 1;
            for (uint32_t h = 0; h < c->K; ++h) P = mulmod_h(P, c->primes[c->L + h] % qi, qi);
            mdt[moddown_negp_off(c) + i] = (qi - mulmod_h(P, c->t % qi, qi)) % qi;
        }
    }

    // INTT constants of the special primes with the ModDown input factor folded
    // into the last stage, so the INTT of the P-limbs yields [y (P/p_a)^-1]_{p_a}
    std::vector<PrimeConst> pc_md = pc;
    for (uint32_t a = 0; a < c->K; ++a) {
        PrimeConst &e = pc_md[c->L + a];
        const uint64_t pa = e.q;
        const uint64_t f = (c->scheme == RF_BGV ? mdt : md)[2 * a];
        e.ninv = mulmod_h(e.ninv, f, pa);
        e.ninv_p = shoup_companion(e.ninv, pa);
        e.wlast = mulmod_h(e.wlast, f, pa);
        e.wlast_p = shoup_companion(e.wlast, pa);
    }

    // INTT constants of every level with the ModUp input factor of each Q-limb
    // folded into the last stage (the factor of limb i depends on the size of
    // its digit, which the level truncates)
    const size_t npc = (size_t)c->L + c->K;
    std::vector<PrimeConst> pc_mu((size_t)c->L * npc);
    for (uint32_t nl = 1; nl <= c->L; ++nl) {
        PrimeConst *row = pc_mu.data() + (size_t)(nl - 1) * npc;
        std::copy(pc.begin(), pc.begin() + npc, row);
        for (uint32_t i = 0; i < nl; ++i) {
            const uint32_t j = i / A, start = j * A, sz = std::min(A, nl - start);
            const uint64_t f = mu[modup_block(c, j, sz) + 2 * (i - start)];
            PrimeConst &e = row[i];
            e.ninv = mulmod_h(e.ninv, f, e.q);
            e.ninv_p = shoup_companion(e.ninv, e.q);
            e.wlast = mulmod_h(e.wlast, f, e.q);
            e.wlast_p = shoup_companion(e.wlast, e.q);
        }
    }

    // Rescale: drop q_l (l >= 1) into every q_i, i < l
    std::vector<uint64_t> rs((size_t)c->L * c->L * 3, 0);
    for (uint32_t l = 1; l < c->L; ++l) {
        uint64_t ql = c->primes[l];
        for (uint32_t i = 0; i < l; ++i) {
            uint64_t qi = c->primes[i];
            uint64_t inv = inv_h(ql % qi, qi);
            rs[rescale_off(c, l, i)] = inv;
            rs[rescale_off(c, l, i) + 1] = shoup_companion(inv, qi);
            rs[rescale_off(c, l, i) + 2] = (qi - ql % qi) % qi;
        }
    }

    // ModUp extension prime maps per level nl: for each digit, the basis Q_l u P minus the digit
    std::vector<uint32_t> pm;
    c->modup_levels.assign(c->L + 1, ModupLevel{0, 0, 0});
    c->tuning.assign(c->L + 1, kDefaultTuning);
    for (uint32_t nl = 1; nl <= c->L; ++nl) {
        ModupLevel lv;
        lv.dnum = (nl + A - 1) / A;
        lv.pmap_off = (uint32_t)pm.size();
        for (uint32_t j = 0; j < lv.dnum; ++j) {
            uint32_t start = j * A, s = std::min(A, nl - start);
            for (uint32_t g = 0; g < nl; ++g)
                if (g < start || g >= start + s) pm.push_back(g);
            for (uint32_t g = 0; g < c->K; ++g) pm.push_back(c->L + g);
        }
        lv.ext_limbs = (uint32_t)pm.size() - lv.pmap_off;
        c->modup_levels[nl] = lv;
    }

    // BFV: BEHZ tables and the prime map of q u B_sk
    std::vector<uint64_t> bz;
    std::vector<uint32_t> pmqb;
    if (c->scheme == RF_BFV) {
        const uint32_t L = c->L, nb = c->nb, KB = c->L + c->K;  // index of b_0 in `primes`
        BehzLayout &o = c->behz;
        o.L = L;
        o.nb = nb;
        uint32_t at = 0;
        auto take = [&at](uint32_t n) { uint32_t r = at; at += n; return r; };
        o.ext_factor = take(2 * L);
        o.ext_cross = take((nb + 1) * L);
        o.ext_q = take(2 * (nb + 1));
        o.cross_q_mt = take(L);
        o.neg_qinv_mt = take(1);
        o.floor_factor = take(2 * L);
        o.floor_cross = take((nb + 1) * L);
        o.t_bsk = take(2 * (nb + 1));
        o.qinv_bsk = take(2 * (nb + 1));
        o.sk_factor = take(2 * nb);
        o.sk_cross = take(L * nb);
        o.cross_b_msk = take(nb);
        o.minv_msk = take(2);
        o.m_q = take(2 * L);
        o.total = at;
        bz.assign(at, 0);
        const uint64_t mt_mask = 0xffffffffull;
        auto bsk = [&](uint32_t m) { return c->primes[KB + m]; };  // m in [0, nb]: b_0..b_{nb-1}, m_sk
        // products of the Q-primes other than q_i, modulo a target (64-bit arithmetic)
        auto qhat_mod = [&](uint32_t i, uint64_t m) {
            uint64_t v = 1 % m;
            for (uint32_t h = 0; h < L; ++h)
                if (h != i) v = mulmod_h(v, c->primes[h] % m, m);
            return v;
        };
        auto qhat_mt = [&](uint32_t i) {  // mod 2^32
            uint64_t v = 1;
            for (uint32_t h = 0; h < L; ++h)
                if (h != i) v = (v * (c->primes[h] & mt_mask)) & mt_mask;
            return v;
        };
        uint64_t qmt = 1;
        for (uint32_t h = 0; h < L; ++h) qmt = (qmt * (c->primes[h] & mt_mask)) & mt_mask;
        // inverse of an odd number mod 2^32 by Newton iteration
        uint64_t inv = qmt;
        for (int k = 0; k < 5; ++k) inv = (inv * (2 - qmt * inv)) & mt_mask;
        bz[o.neg_qinv_mt] = (0x100000000ull - inv) & mt_mask;
        for (uint32_t i = 0; i < L; ++i) {
            uint64_t qi = c->primes[i];
            uint64_t qh_inv = inv_h(qhat_mod(i, qi), qi);
            uint64_t f = mulmod_h((1ull << 32) % qi, qh_inv, qi);
            bz[o.ext_factor + 2 * i] = f;
            bz[o.ext_factor + 2 * i + 1] = shoup_companion(f, qi);
            uint64_t ff = mulmod_h(c->t % qi, qh_inv, qi);
            bz[o.floor_factor + 2 * i] = ff;
            bz[o.floor_factor + 2 * i + 1] = shoup_companion(ff, qi);
            for (uint32_t m = 0; m <= nb; ++m) {
                const uint64_t bm = bsk(m), qh = qhat_mod(i, bm);
                bz[o.floor_cross + m * L + i] = qh;
                bz[o.ext_cross + m * L + i] = mulmod_h(qh, inv_h((1ull << 32) % bm, bm), bm);
            }
            bz[o.cross_q_mt + i] = qhat_mt(i);
        }
        for (uint32_t m = 0; m <= nb; ++m) {
            uint64_t bm = bsk(m);
            uint64_t qm = 1;
            for (uint32_t h = 0; h < L; ++h) qm = mulmod_h(qm, c->primes[h] % bm, bm);
            const uint64_t qmt = mulmod_h(qm, inv_h((1ull << 32) % bm, bm), bm);
            bz[o.ext_q + 2 * m] = qmt;
            bz[o.ext_q + 2 * m + 1] = shoup_companion(qmt, bm);
            uint64_t tm = c->t % bm;
            bz[o.t_bsk + 2 * m] = tm;
            bz[o.t_bsk + 2 * m + 1] = shoup_companion(tm, bm);
            uint64_t qi = inv_h(qm, bm);
            bz[o.qinv_bsk + 2 * m] = qi;
            bz[o.qinv_bsk + 2 * m + 1] = shoup_companion(qi, bm);
        }
        auto mhat_mod = [&](uint32_t j, uint64_t m) {  // (M / b_j) mod m
            uint64_t v = 1 % m;
            for (uint32_t h = 0; h < nb; ++h)
                if (h != j) v = mulmod_h(v, bsk(h) % m, m);
            return v;
        };
        const uint64_t msk = bsk(nb);
        for (uint32_t j = 0; j < nb; ++j) {
            uint64_t bj = bsk(j);
            uint64_t f = inv_h(mhat_mod(j, bj), bj);
            bz[o.sk_factor + 2 * j] = f;
            bz[o.sk_factor + 2 * j + 1] = shoup_companion(f, bj);
            for (uint32_t i = 0; i < L; ++i) bz[o.sk_cross + i * nb + j] = mhat_mod(j, c->primes[i]);
            bz[o.cross_b_msk + j] = mhat_mod(j, msk);
        }
        uint64_t mm = 1;
        for (uint32_t h = 0; h < nb; ++h) mm = mulmod_h(mm, bsk(h) % msk, msk);
        uint64_t minv = inv_h(mm, msk);
        bz[o.minv_msk] = minv;
        bz[o.minv_msk + 1] = shoup_companion(minv, msk);
        for (uint32_t i = 0; i < L; ++i) {
            uint64_t qi = c->primes[i], v = 1;
            for (uint32_t h = 0; h < nb; ++h) v = mulmod_h(v, bsk(h) % qi, qi);
            bz[o.m_q + 2 * i] = v;
            bz[o.m_q + 2 * i + 1] = shoup_companion(v, qi);
        }
        for (uint32_t i = 0; i < L; ++i) pmqb.push_back(i);
        for (uint32_t m = 0; m <= nb; ++m) pmqb.push_back(KB + m);
    }

    // Client-side tables.  [P]_{p_g} for the P [i in D_j] s' term of key
    // generation (0 on the special primes); floor(Q_L / t) mod p_g for BFV
    // encryption, = -[Q_L]_t t^-1 mod q_g since q_g divides Q_L.
    std::vector<uint64_t> cl((size_t)NP * 4, 0);
    {
        uint64_t qt = 0;
        if (c->scheme == RF_BFV) {
            qt = 1 % c->t;
            for (uint32_t h = 0; h < c->L; ++h) qt = mulmod_h(qt, c->primes[h] % c->t, c->t);
        }
        for (uint32_t g = 0; g < NP; ++g) {
            const uint64_t q = c->primes[g];
            uint64_t pm = 1 % q;
            for (uint32_t a = 0; a < c->K; ++a) pm = mulmod_h(pm, c->primes[c->L + a] % q, q);
            if (g >= c->L && g < c->L + c->K) pm = 0;
            cl[4 * g] = pm;
            cl[4 * g + 1] = shoup_companion(pm, q);
            if (c->scheme == RF_BFV && g < c->L) {
                const uint64_t d = mulmod_h((q - qt % q) % q, inv_h(c->t % q, q), q);
                cl[4 * g + 2] = d;
                cl[4 * g + 3] = shoup_companion(d, q);
            }
        }
    }
    // q_i^-1 mod q_j (i < j): balanced mixed-radix digits of the CRT composition
    std::vector<uint64_t> gar((size_t)c->L * c->L * 2, 0);
    for (uint32_t i = 0; i < c->L; ++i)
        for (uint32_t j = i + 1; j < c->L; ++j) {
            const uint64_t qj = c->primes[j];
            const uint64_t v = inv_h(c->primes[i] % qj, qj);
            gar[((size_t)i * c->L + j) * 2] = v;
            gar[((size_t)i * c->L + j) * 2 + 1] = shoup_companion(v, qj);
        }
    // CKKS: zeta^k = exp(i pi k / N) for k < 2N and the slot positions of the
    // canonical embedding: slot j is the evaluation at zeta^(5^j)
    std::vector<double> zeta;
    std::vector<uint32_t> slot_idx;
    if (c->scheme == RF_CKKS) {
        zeta.resize(4 * (size_t)N);
        const long double pi = 3.141592653589793238462643383279502884L;
        for (uint32_t k = 0; k < 2 * N; ++k) {
            const long double ang = pi * (long double)k / (long double)N;
            zeta[2 * k] = (double)cosl(ang);
            zeta[2 * k + 1] = (double)sinl(ang);
        }
        slot_idx.resize(N / 2);
        uint64_t x = 1;
        for (uint32_t j = 0; j < N / 2; ++j) {
            slot_idx[j] = (uint32_t)((x - 1) / 2);
            x = x * 5 % (2 * (uint64_t)N);
        }
    }

    int rc = RF_OK;
    if ((rc = upload(&c->d_client, cl)) || (rc = upload(&c->d_garner, gar)) ||
        (!zeta.empty() && ((rc = upload(&c->d_zeta, zeta)) || (rc = upload(&c->d_slot_idx, slot_idx))))) {
        free_tables(c);
        delete c;
        return rc;
    }
    if ((!bz.empty() && ((rc = upload(&c->d_behz, bz)) || (rc = upload(&c->d_pmap_qb, pmqb)))) ||
        (rc = upload(&c->d_pc, pc)) || (rc = upload(&c->d_pc_md, pc_md)) || (rc = upload(&c->d_pc_mu, pc_mu)) ||
        (!twrf.empty() && ((rc = upload(&c->d_tw_fwd_rows, twrf)) || (rc = upload(&c->d_tw_inv_rows, twri)))) || (rc = upload(&c->d_tw_fwd, twf)) || (rc = upload(&c->d_tw_inv, twi)) ||
        (rc = upload(&c->d_modup, mu)) || (rc = upload(&c->d_moddown, md)) ||
        (!mdt.empty() && (rc = upload(&c->d_moddown_t, mdt))) || (rc = upload(&c->d_rescale, rs)) ||
        (rc = upload(&c->d_pmaps, pm))) {
        free_tables(c);
        delete c;
        return rc;
    }
    *out = c;
    return RF_OK;
}

static bool tuning_valid(const rf_tuning &t) {
    return (t.ntt_small_tile == 0 || t.ntt_small_tile == 1024 || t.ntt_small_tile == 2048) &&
           (t.ntt_small_radix == 4 || t.ntt_small_radix == 8) &&
           (t.modup_chunk == 4 || t.modup_chunk == 8 || t.modup_chunk == 16);
}

extern "C" int rf_ctx_set_tuning(rf_ctx *c, uint32_t nl, const rf_tuning *t) {
    if (!c || !t) return rf::fail(RF_EINVAL, "rf_ctx_set_tuning: null argument");
    if (nl > c->L) return rf::fail(RF_ELEVEL, "rf_ctx_set_tuning: level out of range");
    if (!tuning_valid(*t)) return rf::fail(RF_EINVAL, "rf_ctx_set_tuning: unsupported variant");
    if (nl == 0) {
        for (uint32_t l = 1; l <= c->L; ++l) c->tuning[l] = *t;
    } else {
        c->tuning[nl] = *t;
    }
    return RF_OK;
}

extern "C" int rf_ctx_get_tuning(const rf_ctx *c, uint32_t nl, rf_tuning *out) {
    if (!c || !out) return rf::fail(RF_EINVAL, "rf_ctx_get_tuning: null argument");
    if (nl < 1 || nl > c->L) return rf::fail(RF_ELEVEL, "rf_ctx_get_tuning: level out of range");
    *out = c->tuning[nl];
    return RF_OK;
}

extern "C" void rf_ctx_destroy(rf_ctx *c) {
    if (!c) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(c->device);
    free_tables(c);
    (void)hipSetDevice(prev);
    delete c;
}

extern "C" const char *rf_last_error(void) { return rf::last_error(); }

extern "C" const char *rf_version(void) { return "rnsfhe 0.1 gfx950"; }
