// Internal structures of the RNS-FHE library shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rnsfhe.h"

namespace rf {

constexpr int kMaxAlpha = 8;
constexpr int kMaxBfvLimbs = 24;  // BFV: Q-primes and auxiliary primes the BEHZ kernels hold in registers
constexpr int kMaxPrimes = 250;  // L + k, prime indices fit in a byte

// Per-prime constants, device resident.  Prime index g < L is q_g, g >= L is p_{g-L}.
struct PrimeConst {
    uint64_t q;
    uint64_t mu1, mu0;       // floor(2^128 / q) = mu1 * 2^64 + mu0
    uint64_t ninv, ninv_p;   // N^-1 mod q and its Shoup companion
    uint64_t wlast, wlast_p; // psi^-brv(1) * N^-1 (last inverse stage) and companion
    uint64_t tmod, tmod_p;   // plaintext modulus t mod q and companion (BGV/BFV; 0 for CKKS)
    uint64_t tinv, tinv_p;   // t^-1 mod q and companion
    uint64_t r64, r64_p;     // 2^64 mod q and companion
    uint64_t one_p;          // floor(2^64 / q): Shoup companion of 1
};

struct __align__(16) TwPair {
    uint64_t w, wp;  // twiddle and floor(w 2^62 / q) (the companion of shoup62_lazy)
};

// Launch description of a batched (I)NTT over limbs laid out as
// [n_polys][per_poly][N]; limb i of a polynomial uses prime pmap[i] (or prime_base + i).
struct NttBatch {
    const uint64_t *in;
    uint64_t *out;
    uint64_t in_poly_stride;   // elements between polynomials
    uint64_t out_poly_stride;
    uint32_t per_poly;
    uint32_t n_polys;
    uint32_t prime_base;
    const uint32_t *pmap;      // device array [per_poly] or nullptr
};

// Offsets (uint64 entries) of the BEHZ tables of a BFV context (L Q-primes,
// nb auxiliary primes B, B_sk = B u {m_sk}, m~ = 2^32).  The constants of one
// output limb of a conversion are contiguous (target-major), so a thread reads
// them with wide scalar loads.
struct BehzLayout {
    uint32_t L, nb;
    uint32_t ext_factor;   // [L] pairs: m~ (Q/q_i)^-1 mod q_i
    uint32_t ext_cross;    // [nb+1][L]: (Q/q_i) m~^-1 mod bsk_m
    uint32_t ext_q;        // [nb+1] pairs: Q m~^-1 mod bsk_m
    uint32_t cross_q_mt;   // [L]: Q/q_i mod 2^32
    uint32_t neg_qinv_mt;  // [1]: -Q^-1 mod 2^32
    uint32_t floor_factor; // [L] pairs: t (Q/q_i)^-1 mod q_i
    uint32_t floor_cross;  // [nb+1][L]: Q/q_i mod bsk_m
    uint32_t t_bsk;        // [nb+1] pairs: t mod bsk_m
    uint32_t qinv_bsk;     // [nb+1] pairs: Q^-1 mod bsk_m
    uint32_t sk_factor;    // [nb] pairs: (M/b_j)^-1 mod b_j
    uint32_t sk_cross;     // [L][nb]: M/b_j mod q_i
    uint32_t cross_b_msk;  // [nb]: M/b_j mod m_sk
    uint32_t minv_msk;     // [1] pair: M^-1 mod m_sk
    uint32_t m_q;          // [L] pairs: M mod q_i
    uint32_t total;
};

// Host-side layout of the ModUp extension basis at one level.
struct ModupLevel {
    uint32_t dnum;        // digits at this level
    uint32_t ext_limbs;   // sum over digits of (nl - alpha_j + k)
    uint32_t pmap_off;    // offset of this level's prime map in Context::d_pmaps
};

}  // namespace rf

struct rf_ctx {
    int device;
    int scheme;
    uint32_t log_n, log_nmax, n;
    uint32_t L, K, alpha, dnum;
    uint64_t t;
    std::vector<uint64_t> primes;  // L + K: q_0..q_{L-1}, p_0..p_{k-1}
    std::vector<uint64_t> psi;     // primitive 2N-th roots
    std::vector<rf::ModupLevel> modup_levels;  // index nl in [1, L]
    std::vector<rf_tuning> tuning;             // kernel variants per level nl in [1, L] (index 0 unused)

    // device tables (owned)
    rf::PrimeConst *d_pc = nullptr;        // [L+K]
    rf::PrimeConst *d_pc_md = nullptr;     // d_pc with the ModDown input factor [(P/p_a)^-1]_{p_a}
                                           // folded into the last inverse stage of every special prime
    rf::PrimeConst *d_pc_mu = nullptr;     // [L][L+K]: per level nl (row nl - 1), d_pc with the ModUp
                                           // input factor [(Q_j/q_i)^-1]_{q_i} of limb i < nl (digit j
                                           // at that level) folded into its last inverse stage
    rf::TwPair *d_tw_fwd = nullptr;        // [L+K][N]: psi^brv(k)
    rf::TwPair *d_tw_inv = nullptr;        // [L+K][N]: psi^-brv(k)
    rf::TwPair *d_tw_fwd_rows = nullptr;   // the same twiddles in the row-pass layout (ntt_dev.hpp)
    rf::TwPair *d_tw_inv_rows = nullptr;
    uint64_t *d_modup = nullptr;           // ModUp base-conversion constants, see context.hip
    uint64_t *d_moddown = nullptr;         // ModDown constants
    uint64_t *d_moddown_t = nullptr;       // ModDown constants keeping the message mod t (BGV)
    uint64_t *d_rescale = nullptr;         // rescale constants
    uint32_t *d_pmaps = nullptr;           // ModUp extension prime maps for every level
    // BFV: auxiliary base B and m_sk follow the special primes in `primes`
    uint32_t nb = 0;
    uint64_t *d_behz = nullptr;            // BEHZ tables (rf::BehzLayout)
    uint32_t *d_pmap_qb = nullptr;         // prime indices of q u B_sk
    rf::BehzLayout behz{};
    size_t modup_stride = 0;               // uint64 entries per (digit, size) block
    // client side (key generation, encryption, decryption, encode / decode)
    uint64_t *d_client = nullptr;          // [L+K][4]: [P]_{p_g}, companion, [floor(Q_L / t)]_{p_g} (BFV), companion
    uint64_t *d_garner = nullptr;          // [L][L][2]: (q_i^-1 mod q_j, companion) for i < j
    double *d_zeta = nullptr;              // CKKS: [2N][2] (cos, sin)(pi k / N)
    uint32_t *d_slot_idx = nullptr;        // CKKS: [N/2] (5^j mod 2N - 1) / 2
};

namespace rf {

// Defaults of rf_tuning.
constexpr rf_tuning kDefaultTuning = {256, 0, 4, 8, 0};
inline const rf_tuning &level_tuning(const rf_ctx *c, uint32_t nl) {
    return c->tuning[nl < 1 ? 1 : (nl > c->L ? c->L : nl)];
}

// What the inner product adds on the Q-limbs when the ModDown tail that follows
// is reduced to out = ip' - NTT(conv) P^-1 (the fused two-pass path):
// ip'[c][m] = ip[c][m] P^-1 + add_c[m].  pinv null: the plain inner product.
struct IpFold {
    const uint64_t *pinv = nullptr;  // pairs (P^-1 mod q_i, companion)
    // Where the digit's own residue d[m] and the addends come from:
    //   0: d and add0/add1 (nullable) as given;
    //   1 (HMult+Relin): a, b = [2][nl][N] ciphertexts in the NTT domain:
    //      d = a1 b1, add0 = a0 b0, add1 = a0 b1 + a1 b0 (the tensor), computed here;
    //   2 (HRotate): a = the input ciphertext: d = sigma_g(a1), add0 = sigma_g(a0)
    //      (g = galois), gathered here; no add1.
    uint32_t mode = 0;
    const uint64_t *add0 = nullptr, *add1 = nullptr;
    const uint64_t *a = nullptr, *b = nullptr;
    uint32_t galois = 0;
};

// Index map of sigma_g in the NTT domain (output k holds a(psi^(2 brv(k) + 1))):
// sigma_g(a)[k] = a[k'] with 2 brv(k') + 1 = (2 brv(k) + 1) g mod 2N.
__device__ __forceinline__ uint32_t galois_src(uint32_t k, uint32_t galois, uint32_t log_n) {
    const uint32_t mask2n = (2u << log_n) - 1;
    const uint32_t rk = __brev(k) >> (32 - log_n);
    const uint32_t e = ((2u * rk + 1u) * galois) & mask2n;
    return __brev((e - 1u) >> 1) >> (32 - log_n);
}

// Offsets (in uint64 entries) inside the ModUp table block of (digit j, digit size s):
//   [0, 2*alpha):            factor pairs (w, w') of [(Q_j/q_i)^-1]_{q_i}, i' < s
//   [2*alpha, ...):          cross[g][i'] = [Q_j/q_i]_{prime g}, g in [0, L+K), target-major
inline size_t modup_block(const rf_ctx *c, uint32_t j, uint32_t s) {
    return ((size_t)j * c->alpha + (s - 1)) * c->modup_stride;
}
// INTT constants of level nl whose output is the ModUp input y_i = [x_i (Q_j/q_i)^-1]_{q_i}.
inline const PrimeConst *pc_modup(const rf_ctx *c, uint32_t nl) {
    return c->d_pc_mu + (size_t)(nl - 1) * (c->L + c->K);
}
// ModDown table: [K] factor pairs (w, w') of [(P/p)^-1]_p; [L][K] cross [P/p]_{q_i} (target-major);
// [L] pairs P^-1 mod q_i; [L] (q_i - [P]_{q_i}).
inline size_t moddown_cross_off(const rf_ctx *c) { return 2 * (size_t)c->K; }
inline size_t moddown_pinv_off(const rf_ctx *c) { return 2 * (size_t)c->K + (size_t)c->K * c->L; }
inline size_t moddown_negp_off(const rf_ctx *c) { return moddown_pinv_off(c) + 2 * (size_t)c->L; }
// Rescale table, per dropped prime index l in [1, L) and i < l:
//   entry (l * L + i) * 3 + {0,1,2} = q_l^-1 mod q_i, its companion, q_i - [q_l]_{q_i}.
inline size_t rescale_off(const rf_ctx *c, uint32_t l, uint32_t i) {
    return ((size_t)l * c->L + i) * 3;
}

// Brackets one kernel launch with HIP events on its stream while profiling is
// enabled (rf_profile_enable); a no-op otherwise.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();

  private:
    int idx_;
    hipStream_t s_;
};

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// kernel launchers (kernels.hip)
// pcs: per-prime constants (null: the context's d_pc).
// tn: the level's kernel variants (null: the defaults).
int launch_ntt(const rf_ctx *c, const NttBatch &b, bool forward, hipStream_t s, const PrimeConst *pcs = nullptr,
               const rf_tuning *tn = nullptr);
// ModDown after the inner product, two-pass ring degrees only: ip = [2][nl + K][N]
// whose K P-limbs hold the INTT with d_pc_md (so already scaled by the input
// factor).  The first forward pass computes the base conversion of each Q
// target in its prologue (into conv [2][nl][N]), the last applies the tail:
// out[c][i] = (ip[c][i] - NTT(conv)) P^-1 + add_c.
// ip's Q-limbs must come from launch_inner_product with fold (P^-1 and the addends
// applied), so the tail is out[c][i] = ip[c][i] - NTT(conv)[c][i] P^-1.
int launch_ntt_fwd_moddown(const rf_ctx *c, uint64_t *conv, const uint64_t *ip, uint64_t *out, uint32_t nl,
                           hipStream_t s, const rf_tuning *tn = nullptr);
// INTT of the polynomial to key-switch (two-pass ring degrees only), with the
// step that produces it as the prologue of its first pass, into dc [nl][N]
// (coefficient domain, scaled for ModUp by pc_modup(c, nl)):
//   galois == 0 (HMult): d2 = a1 b1 of a, b ([2][nl][N]);
//   galois != 0 (HRotate): sigma_g of a's polynomial 1.
int launch_intt_first(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *dc, uint32_t galois,
                      uint32_t nl, hipStream_t s, const rf_tuning *tn = nullptr);
// Rescale / modulus switch after the INTT of the last limb (last = [2][N]),
// two-pass ring degrees only: the first forward pass lifts the last limb into
// each remaining prime in its prologue (into lift [2][nl-1][N]; KEEP_T for BGV),
// the last applies the tail out[c][i] = (in[c][i] - NTT(lift)) q_l^-1.
int launch_ntt_fwd_rescale(const rf_ctx *c, const uint64_t *last, uint64_t *lift, const uint64_t *in,
                           uint64_t *out, uint32_t nl, bool keep_t, hipStream_t s, const rf_tuning *tn = nullptr);
int launch_tensor(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *d01,
                  uint64_t *d2, uint32_t nl, hipStream_t s);
// scaled: x is an INTT taken with pc_modup(c, nl), so each limb already carries
// its digit's input factor [(Q_j/q_i)^-1]_{q_i}.
// chunk: output limbs per thread (4, 8 or 16).
int launch_modup_bconv(const rf_ctx *c, const uint64_t *x, uint64_t *ext, uint32_t nl, hipStream_t s,
                       bool scaled = false, uint32_t chunk = 8);
// fold (non-null): the Q-limbs leave as ip P^-1 + add_c with the sources fold
// names (its pinv is filled in here), for launch_ntt_fwd_moddown.
int launch_inner_product(const rf_ctx *c, const uint64_t *d_ntt, const uint64_t *ext,
                         const uint64_t *evk, uint64_t *ip, uint32_t nl, hipStream_t s,
                         const IpFold *fold = nullptr);
int launch_moddown_bconv(const rf_ctx *c, const uint64_t *ip, uint64_t *conv, uint32_t nl,
                         hipStream_t s);  // uses the t-preserving table for BGV contexts
int launch_moddown_tail(const rf_ctx *c, const uint64_t *ip, const uint64_t *conv,
                        const uint64_t *add0, const uint64_t *add1, uint64_t *out, uint32_t nl,
                        hipStream_t s);
int launch_rescale_lift(const rf_ctx *c, const uint64_t *last, uint64_t *lift, uint32_t nl,
                        bool keep_t, hipStream_t s);
int launch_rescale_tail(const rf_ctx *c, const uint64_t *in, const uint64_t *lift, uint64_t *out,
                        uint32_t nl, hipStream_t s);
int launch_ewise(const rf_ctx *c, int op, const uint64_t *a, const uint64_t *b, int64_t k, uint64_t *out,
                 uint32_t nl, uint32_t n_polys, hipStream_t s);
int launch_behz_extend(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *ext, hipStream_t s);
// BEHZ fast floor (into f [3][nb+1][N], scratch) and Shenoy-Kumaresan
// conversion of tens = [3][L+nb+1][N]: d0, d1 to out01 [2][L][N], d2 to out2 [L][N].
int launch_behz_floor_sk(const rf_ctx *c, const uint64_t *tens, uint64_t *f, uint64_t *out01, uint64_t *out2,
                         hipStream_t s);
int launch_tensor_map(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *d01, uint64_t *d2,
                      uint32_t nl, const uint32_t *pmap, hipStream_t s);
int launch_automorphism(const rf_ctx *c, const uint64_t *in, uint64_t *out, uint32_t galois,
                        uint32_t nl, uint32_t n_polys, hipStream_t s);

}  // namespace rf
