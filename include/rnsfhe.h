/*
 * rnsfhe.h -- C ABI of the MI355X (gfx950) RNS-FHE hot path.
 *
 * Citations name sections, tables and algorithms of the CAT paper
 * (arXiv 2503.22227): section II-B "RNS Representation"; III-A.2 "Multi Level
 * Memory Usage on GPU" (its "NTT & INTT" paragraph); III-A.3 "Kernel Fusion
 * and Segmentation"; III-A.4 "Data layout and Indexing"; III-B the GPU memory
 * pool; IV-C "Search-and-Average Query"; V-A "Basic FHE operators" with the
 * tables "CKKS operators", "BFV operators" and "BGV operators".
 *
 * What is computed:
 *   * RNS representation (II-B): a coefficient of R_Q, Q = q_0 ... q_l, is held
 *     as its residues mod each word-sized prime q_i ("limbs");
 *   * the negacyclic NTT and its inverse (III-A.2, "NTT & INTT");
 *   * the operators of the tables of V-A: multiply (the five-stage product of
 *     III-A.3) with relinearize, rotate, rescale and modulus switch (the level
 *     concept of II-B: one prime dropped per rescale or switch), and the
 *     client-side key generation, encode, encrypt, decrypt and decode rows.
 * The paper does not define its key switching; this library implements hybrid
 * key switching: digits of ``alpha`` consecutive Q-primes, fast base conversion
 * to Q_l u P (ModUp), inner product with the evaluation key, and division by P
 * with rounding (ModDown).
 *
 * Data layout (III-A.4: the residues of one modulus are stored contiguously,
 * one modulus after another):
 *   a polynomial with n limbs is n * N uint64 values, limb i at [i * N, (i+1) * N);
 *   a ciphertext is 2 such polynomials back to back: [poly][limb][N].
 *   Every residue is in [0, q_i).  CKKS and BGV ciphertexts rest in the NTT
 *   domain, BFV ciphertexts in the coefficient domain (the scheme of the
 *   context fixes the domain of every operand); NTT index k holds the
 *   evaluation at psi^(2 brv(k) + 1).
 *   An evaluation key is [dnum][2][L + k][N]: limbs q_0..q_{L-1} then p_0..p_{k-1},
 *   dnum = ceil(L / alpha); it serves every level by ignoring limbs q_l.. of Q.
 *
 * Memory and streams: every data pointer is DEVICE memory owned by the caller;
 * the library never allocates device memory inside an operation (the aim of
 * the memory pool of III-B).  Operations that need scratch space take a
 * caller-owned device workspace whose size is given by rf_workspace_bytes().
 * Every operation is enqueued asynchronously on the caller's HIP stream
 * (hipStream_t passed as void*; NULL = default stream); a fault inside a kernel
 * shows up at the caller's next synchronisation.  A context is immutable after
 * creation: calls on different streams may share it.  Buffers passed to one
 * call must not alias unless stated.
 *
 * Errors: every function returns RF_OK (0) or a negative RF_E* code and sets a
 * thread-local message readable with rf_last_error().  Arguments are checked on
 * the host before anything is enqueued.  No C++ exception crosses this
 * interface.
 */
#ifndef RNSFHE_H
#define RNSFHE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rf_status {
    RF_OK = 0,
    RF_EINVAL = -1,       /* null pointer, bad size or shape */
    RF_ELEVEL = -2,       /* limb count out of range or operands at different levels */
    /* -3 is not used: the context's scheme fixes the domain of every operand */
    RF_EWORKSPACE = -4,   /* workspace missing or smaller than rf_workspace_bytes() */
    RF_EHIP = -5,         /* a HIP runtime call or kernel launch failed */
    RF_EUNSUPPORTED = -6  /* parameters outside what the kernels implement */
};

enum rf_scheme { RF_CKKS = 0, RF_BFV = 1, RF_BGV = 2 };

/* Parameters of one RNS chain at one ring degree (II-B: the chain of word-sized
 * primes; V-A fixes N = 2^15 and 16 primes for its tables).  The context derives
 * every table (roots, twiddles, Shoup and Barrett constants, base-conversion
 * matrices) from these primes itself. */
typedef struct rf_params {
    int32_t scheme;          /* rf_scheme */
    uint32_t log_n;          /* ring degree N = 2^log_n, 12 <= log_n <= 16 */
    uint32_t log_nmax;       /* degree the roots refer to: psi_N = psi_max^(2^(log_nmax - log_n)),
                                psi_max = g^((q-1)/2^(log_nmax+1)) for the smallest g >= 2 with
                                psi_max^(2^log_nmax) = -1; every prime is 1 mod 2^(log_nmax+1) */
    uint32_t n_q;            /* L: ciphertext primes q_0..q_{L-1}, 1 <= L */
    const uint64_t *q;       /* host array of L primes, each < 2^60 */
    uint32_t n_p;            /* k: special primes, 1 <= k */
    const uint64_t *p;       /* host array of k primes, each < 2^60 */
    uint32_t alpha;          /* Q-primes per key-switching digit, 1 <= alpha <= 8 */
    uint64_t t;              /* plaintext modulus (BFV/BGV, 2 <= t < 2^32), 0 for CKKS */
    uint32_t n_b;            /* BFV: auxiliary base B of the BEHZ multiplication (0 otherwise) */
    const uint64_t *b;       /* host array of n_b primes, each < 2^60 */
    uint64_t m_sk;           /* BFV: the extra prime of B_sk = B u {m_sk}; m~ = 2^32 is fixed */
} rf_params;

typedef struct rf_ctx rf_ctx;

/* Create a context on HIP device `device` (the precomputed tables of the
 * middle tier, section III, and the pool set-up of IV-A); uploads its tables
 * with hipMalloc once and makes `device` current.  Returns RF_EUNSUPPORTED for
 * degrees or sizes outside the kernels' range, RF_EINVAL for a non-prime or
 * non-NTT-friendly modulus, RF_EHIP if an upload fails.  *out is owned by the
 * caller and released with rf_ctx_destroy. */
int rf_ctx_create(const rf_params *params, int device, rf_ctx **out);
void rf_ctx_destroy(rf_ctx *ctx);

/* Kernel variants of one level (the segmentation / grouping choices of
 * III-A.3 "Kernel Fusion and Segmentation", made per ring degree and limb count
 * instead of fixed).  Every variant computes the same residues: a setting
 * changes speed only, never results.
 *   ntt_small_below  an (I)NTT launch of a two-pass degree (N >= 2^13) with fewer
 *                    4096-residue tiles than this runs the small-tile passes
 *                    (more workgroups, a shorter butterfly chain per thread);
 *                    0 = never.  Default 256 (the CU count).
 *   ntt_small_tile   residues per small tile: 1024 or 2048, or 0 = 2048 when the
 *                    launch has at least half of ntt_small_below tiles, else 1024
 *                    (default 0).
 *   ntt_small_radix  residues per thread of the small tiles, i.e. butterfly
 *                    stages per LDS round: 4 (radix-4, default) or 8 (radix-8).
 *                    The 4096-residue tiles always hold 16 (radix-16 rounds).
 *   modup_chunk      ModUp base-conversion output limbs per thread (the limb
 *                    grouping of the conversion): 4, 8 (default) or 16.
 *   ntt_fused_small_below  the same threshold for the (I)NTT launches that carry a
 *                    fused step (the tensor or automorphism before the first INTT
 *                    pass, the ModDown conversion and tail, the rescale lift and
 *                    tail); their small tiles take ntt_small_tile and 4 residues per
 *                    thread.  Default 0 (always 4096-residue tiles).
 * The settings of every level start at the defaults. */
typedef struct rf_tuning {
    uint32_t ntt_small_below;
    uint32_t ntt_small_tile;
    uint32_t ntt_small_radix;
    uint32_t modup_chunk;
    uint32_t ntt_fused_small_below;
} rf_tuning;

/* Use `t` for operations at level `n_limbs` (1 <= n_limbs <= L; 0 = every
 * level).  The standalone rf_ntt / rf_intt use the level min(n_limbs, L) of
 * their window.  RF_EINVAL for a value outside the lists above.  Host state
 * only: call it while no other thread issues operations on the context. */
int rf_ctx_set_tuning(rf_ctx *ctx, uint32_t n_limbs, const rf_tuning *t);
/* The setting of level n_limbs (1 <= n_limbs <= L) into *out. */
int rf_ctx_get_tuning(const rf_ctx *ctx, uint32_t n_limbs, rf_tuning *out);

/* Operation ids for rf_workspace_bytes. */
enum rf_op {
    RF_OP_HMULT_RELIN = 1,
    RF_OP_ROTATE = 2,
    RF_OP_RESCALE = 3,
    RF_OP_KEYSWITCH = 4,
    RF_OP_MODSWITCH = 5,  /* BGV only; a CKKS modulus switch needs no workspace (size 0) */
    RF_OP_ENCODE = 6,     /* CKKS encode and decode (complex FFT scratch) */
    RF_OP_DECODE = 7
};

/* Device workspace bytes an operation needs at a level with `n_limbs` Q-limbs
 * (the memory each operator asks of the pool, III-B); 0 if the arguments are
 * invalid or the operation needs none. */
size_t rf_workspace_bytes(const rf_ctx *ctx, int op, uint32_t n_limbs);

/* Forward / inverse negacyclic NTT (III-A.2, "NTT & INTT"), in place, of
 * `n_polys` polynomials of `n_limbs` limbs each, stored back to back; limb i of
 * each polynomial is mod prime `first_limb + i` of the chain q_0..q_{L-1},
 * p_0..p_{k-1}.  Input residues must be in [0, q); outputs are in [0, q).
 * RF_ELEVEL for an empty or out-of-range limb window. */
int rf_ntt(const rf_ctx *ctx, uint64_t *data, uint32_t first_limb, uint32_t n_limbs,
           uint32_t n_polys, void *stream);
int rf_intt(const rf_ctx *ctx, uint64_t *data, uint32_t first_limb, uint32_t n_limbs,
            uint32_t n_polys, void *stream);

/* HMult+Relin: the multiply row followed by the relinearize row of the tables
 * of V-A (the five-stage product of III-A.3, then key switching):
 * out = (d0 + KS_0(d2), d1 + KS_1(d2)) with (d0, d1, d2) the tensor product of
 * a and b, rlk the relinearisation key, out must not overlap a or b.
 *   CKKS / BGV: ciphertexts with `n_limbs` Q-limbs in the NTT domain.
 *   BFV: ciphertexts with all L limbs (n_limbs == L) in the COEFFICIENT domain;
 *   (d0, d1, d2) is the BEHZ tensor: extension to B_sk with the small
 *   Montgomery reduction by m~ = 2^32, products on q u B_sk, fast floor of
 *   t d / Q and the Shenoy-Kumaresan conversion back to q (the multiply row of
 *   Table "BFV operators").
 * Workspace: rf_workspace_bytes(RF_OP_HMULT_RELIN, n_limbs). */
int rf_hmult_relin(const rf_ctx *ctx, const uint64_t *a, const uint64_t *b, const uint64_t *rlk,
                   uint64_t *out, uint32_t n_limbs, void *workspace, size_t workspace_bytes,
                   void *stream);

/* HMult+Relin for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation and results as rf_hmult_relin, with the workspace taken from a
 * static device array of 160 MiB that the library holds on every device it runs
 * on until the process ends (enough for N = 2^16 with 24 Q-primes and 4 special
 * primes at alpha = 8 or alpha = 4).  RF_EUNSUPPORTED when the operation needs
 * more scratch than that, RF_ELEVEL / RF_EINVAL as rf_hmult_relin.  Every call on
 * one device shares the array: calls that overlap on one device (other streams,
 * other threads) race, so the caller serialises them. */
int rf_hmult_relin_noalloc(const rf_ctx *ctx, const uint64_t *a, const uint64_t *b, const uint64_t *rlk,
                           uint64_t *out, uint32_t n_limbs, void *stream);

/* HRotate (the rotate and complex_conjugate rows of Table "CKKS operators",
 * rotate_rows / rotate_columns of the BFV and BGV tables):
 * out = (sigma_g(c0) + KS_0(sigma_g(c1)), KS_1(sigma_g(c1))) with
 * sigma_g : a(X) -> a(X^g), g odd in [1, 2N), and gk the key from s(X^g) to s.
 * rf_galois_element gives g for a slot rotation; g = 2N - 1 conjugates.
 *   CKKS / BGV: NTT-domain ciphertexts with `n_limbs` Q-limbs.
 *   BFV: coefficient-domain ciphertexts with all L limbs (RF_ELEVEL otherwise);
 *   the result decrypts to m(X^g) mod t, a permutation of the batched slots.
 * out must not overlap in; workspace of rf_workspace_bytes(RF_OP_ROTATE). */
int rf_rotate(const rf_ctx *ctx, const uint64_t *in, uint32_t galois_elt, const uint64_t *gk,
              uint64_t *out, uint32_t n_limbs, void *workspace, size_t workspace_bytes,
              void *stream);

/* The Galois element of a slot rotation (the rotate rows of the tables of V-A):
 * g = 5^r mod 2N rotates the CKKS slots (and the BFV/BGV columns) left by r, any
 * integer r (negative: right); with conjugate != 0 the result is (2N - 1) 5^r mod
 * 2N, which also conjugates (CKKS) or swaps the two rows (BFV/BGV). */
int rf_galois_element(const rf_ctx *ctx, int64_t rotation, int conjugate, uint32_t *galois_elt);

/* Key switching (the relinearize row of the tables of V-A, on its own) of one
 * NTT-domain polynomial d (n_limbs Q-limbs) under key evk:
 * out = (KS_0(d), KS_1(d)) into [2][n_limbs][N], or out += when accumulate != 0.
 * Workspace: rf_workspace_bytes(RF_OP_KEYSWITCH, n_limbs). */
int rf_keyswitch(const rf_ctx *ctx, const uint64_t *d, const uint64_t *evk, uint64_t *out,
                 uint32_t n_limbs, int accumulate, void *workspace, size_t workspace_bytes,
                 void *stream);

/* Rescale (the rescale row of Table "CKKS operators"; the level concept of
 * II-B): out = round(in / q_l) with q_l = q_{n_limbs-1}, in with n_limbs >= 2
 * Q-limbs, out with n_limbs - 1 (out may equal in).  RF_EUNSUPPORTED on a
 * BFV/BGV context.  Workspace: rf_workspace_bytes(RF_OP_RESCALE, n_limbs). */
int rf_rescale(const rf_ctx *ctx, const uint64_t *in, uint64_t *out, uint32_t n_limbs,
               void *workspace, size_t workspace_bytes, void *stream);

/* Modulus switch (the level concept of II-B; the mod_switch rows of the
 * tables of V-A), out with n_limbs - 1 limbs per polynomial (out may equal in):
 *   CKKS: drop the last limb (workspace unused, may be NULL);
 *   BGV:  out = (in - delta) / q_l with delta = t [in t^-1]_{q_l} (centred), so
 *         the plaintext is kept mod t up to the factor q_l^-1 mod t, which the
 *         caller multiplies into the ciphertext's correction factor.
 * With a BGV context, rf_hmult_relin / rf_rotate / rf_keyswitch use the
 * matching ModDown out = (y - delta)/P with delta = t [y t^-1]_P (centred). */
int rf_modswitch(const rf_ctx *ctx, const uint64_t *in, uint64_t *out, uint32_t n_limbs,
                 void *workspace, size_t workspace_bytes, void *stream);

/* Tensor product only (the multiply row of Table "CKKS operators", the
 * five-stage product of III-A.3): d = (a0 b0, a0 b1 + a1 b0, a1 b1), d is
 * [3][n_limbs][N] and must not overlap a or b. */
int rf_tensor(const rf_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *d,
              uint32_t n_limbs, void *stream);

/* Galois automorphism sigma_g (the permutation inside the rotate rows of the
 * tables of V-A) of `n_polys` NTT-domain polynomials of n_limbs Q-limbs (out
 * must not alias in; g odd in [1, 2N), RF_EINVAL otherwise). */
int rf_automorphism(const rf_ctx *ctx, const uint64_t *in, uint64_t *out, uint32_t galois_elt,
                    uint32_t n_limbs, uint32_t n_polys, void *stream);

/* ---- Element-wise helpers (the add / sub / multiply_plain rows of the tables
 * of V-A; the private-query circuit of IV needs them) ----
 * n_polys polynomials of n_limbs limbs, [n_polys][n_limbs][N], limb i mod q_i;
 * out may alias an input.  Every residue operation is exact mod q_i. */
/* out = a + b, a - b */
int rf_add(const rf_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t n_limbs,
           uint32_t n_polys, void *stream);
int rf_sub(const rf_ctx *ctx, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t n_limbs,
           uint32_t n_polys, void *stream);
/* out = k * a for a signed integer k (k taken mod q_i) */
int rf_mul_scalar(const rf_ctx *ctx, const uint64_t *a, int64_t k, uint64_t *out, uint32_t n_limbs,
                  uint32_t n_polys, void *stream);
/* ciphertext a = (c0, c1): out = (c0 + k, c1), k added to every residue of c0 (in the
 * NTT domain: adding the constant polynomial k) */
int rf_add_scalar(const rf_ctx *ctx, const uint64_t *a, int64_t k, uint64_t *out, uint32_t n_limbs,
                  void *stream);
/* out_p = a_p * pt for each polynomial p, pt a single [n_limbs][N] polynomial (same domain) */
int rf_mul_plain(const rf_ctx *ctx, const uint64_t *a, const uint64_t *pt, uint64_t *out, uint32_t n_limbs,
                 uint32_t n_polys, void *stream);

/* ---- Client side: key generation, encrypt, decrypt, encode, decode (the
 * create-key, encode, encrypt, decrypt and decode rows of the tables of V-A;
 * the client of IV-A runs them).  Random draws (secret, masks a, errors e) are
 * made by the caller and passed in; every step here is exact integer
 * arithmetic except encode / decode (double precision). ---- */

/* NTT-domain form of a polynomial with signed integer coefficients over every
 * prime of the chain: out [L + k][N] = NTT(x mod p_i) (II-B).  x: device int64 [N].
 * Used for the secret key s, from which every other client call works. */
int rf_key_ntt(const rf_ctx *ctx, const int64_t *x, uint64_t *out, void *stream);

/* Key-switching key generation (the create relin / galois keys rows): for each
 * digit j of the full chain,
 *   evk_j = (-a_j s + err e_j + P [i in D_j] s', a_j)   over Q_L u P, NTT domain,
 * with s' = s^2 (galois_elt == 0, relinearisation) or s(X^g) (galois_elt = g),
 * [i in D_j] = 1 on the limbs of digit j and 0 on every other limb (and no P term
 * on the P-limbs), err = t for BGV and 1 otherwise.  s_ntt [L + k][N] from
 * rf_key_ntt; a [dnum][L + k][N] uniform residues (taken as NTT-domain values);
 * e [dnum][N] int64 error coefficients; evk [dnum][2][L + k][N]. */
int rf_keygen_switch(const rf_ctx *ctx, const uint64_t *s_ntt, uint32_t galois_elt, const uint64_t *a,
                     const int64_t *e, uint64_t *evk, void *stream);

/* Secret-key encryption (the encrypt rows) at `n_limbs` Q-limbs into out [2][n_limbs][N]:
 *   CKKS: (NTT(m + e) - a s, a);  BGV: (NTT(m + t e) - a s, a)   (NTT domain, a taken as
 *         NTT-domain values);
 *   BFV:  (Delta m + e - INTT(NTT(a) s), a), Delta = floor(Q_L / t)   (coefficient domain,
 *         n_limbs == L).
 * m, e: device int64 [N] (m: encoded message coefficients, BFV/BGV in [0, t)); a: device
 * [n_limbs][N] uniform residues; s_ntt [L + k][N] from rf_key_ntt.  out must not overlap
 * the inputs. */
int rf_encrypt_sk(const rf_ctx *ctx, const int64_t *m, const int64_t *e, const uint64_t *a,
                  const uint64_t *s_ntt, uint64_t *out, uint32_t n_limbs, void *stream);

/* Decryption to the coefficients of the phase (the decrypt rows): out [n_limbs][N] =
 *   CKKS / BGV: INTT(c0 + c1 s);   BFV: c0 + INTT(NTT(c1) s)   (residues in [0, q_i)).
 * The plaintext follows by rf_crt_centered (CKKS), or by taking the centred value
 * mod t (BGV, times the inverse correction factor) or round(t x / Q) mod t (BFV)
 * on the client.  ct [2][n_limbs][N]; out must not overlap ct. */
int rf_decrypt(const rf_ctx *ctx, const uint64_t *ct, const uint64_t *s_ntt, uint64_t *out,
               uint32_t n_limbs, void *stream);

/* The centred integer of each coefficient (II-B: CRT composition) divided by
 * `scale`, as a double: x [n_limbs][N] coefficient-domain residues -> out[n] =
 * X_n / scale with X_n the representative of the residues in (-Q_l/2, Q_l/2]
 * (balanced mixed-radix digits, exact; the final sum in double precision). */
int rf_crt_centered(const rf_ctx *ctx, const uint64_t *x, double *out, uint32_t n_limbs, double scale,
                    void *stream);

/* CKKS encode (the encode row of Table "CKKS operators"): z [N/2] complex slots as
 * interleaved (re, im) doubles -> m [N] int64 = round(scale * tau^-1(z)), tau the
 * canonical embedding at zeta^(5^j), zeta = exp(i pi / N) (slot j holds
 * m(zeta^(5^j))); the result is clamped to |m| <= 2^62.  Workspace:
 * rf_workspace_bytes(RF_OP_ENCODE, 1).  RF_EUNSUPPORTED on a BFV/BGV context. */
int rf_encode_ckks(const rf_ctx *ctx, const double *z, double scale, int64_t *m, void *workspace,
                   size_t workspace_bytes, void *stream);

/* CKKS decode (the decode row): x [N] doubles (coefficients already divided by the
 * scale, e.g. from rf_crt_centered) -> z [N/2] complex slots (interleaved re, im),
 * z_j = x(zeta^(5^j)).  Workspace: rf_workspace_bytes(RF_OP_DECODE, 1). */
int rf_decode_ckks(const rf_ctx *ctx, const double *x, double *z, void *workspace, size_t workspace_bytes,
                   void *stream);

/* ---- Batched HMult+Relin (many ciphertexts, mixed ring degree and level) ----
 *
 * The paper batches per-modulus work over a stream pool (III-A.3 segmentation,
 * III-A.5 and its stream-pool ablation); here a plan fixes a list of
 * independent HMult+Relin items, each naming the context of its own ring
 * degree (contexts of one prime chain at N = 2^13..2^16 with the same alpha and
 * special primes), its operands, relinearisation key, output and limb count.
 * rf_batch_hmult_relin enqueues the chain once for the whole batch: one launch
 * per element-wise step (base conversion, inner product) over the work units of
 * every item, and one launch per NTT pass and ring degree present;
 * rf_batch_graph_launch replays the same launches captured once in a hipGraph.
 * Every item's output is bit-identical to rf_hmult_relin on the same operands.
 * The plan owns a small device job table (allocated by rf_batch_create, never
 * during execution) and refers to the caller's workspace, which must stay valid
 * and untouched by other work while the plan is in use; two launches of one
 * plan must not overlap.  Operands, keys and outputs are caller-owned device
 * memory, outputs must not alias inputs. */
typedef struct rf_batch rf_batch;

typedef struct rf_batch_item {
    const rf_ctx *ctx;      /* context of this item's ring degree */
    const uint64_t *a;      /* [2][n_limbs][N], NTT domain */
    const uint64_t *b;      /* [2][n_limbs][N], NTT domain */
    const uint64_t *rlk;    /* [dnum][2][L + k][N] relinearisation key of ctx */
    uint64_t *out;          /* [2][n_limbs][N] */
    uint32_t n_limbs;       /* Q-limbs of this item, 1 <= n_limbs <= L */
} rf_batch_item;

/* Workspace bytes for a batch (0 if the items are invalid). */
size_t rf_batch_workspace_bytes(const rf_batch_item *items, uint32_t n_items);
/* Build a plan (copies the item list; uploads the job tables).  RF_EINVAL /
 * RF_ELEVEL / RF_EUNSUPPORTED for invalid items, RF_EWORKSPACE for a short
 * workspace, RF_EHIP if the upload fails. */
int rf_batch_create(const rf_batch_item *items, uint32_t n_items, void *workspace,
                    size_t workspace_bytes, rf_batch **out);
void rf_batch_destroy(rf_batch *plan);
/* Tuning knob (the stream-pool size ablation of V-C is the paper's analogue):
 * number of workgroups of launch `stage` (0..12), each walking a contiguous
 * range of work units; 0 = one workgroup per work unit.  Invalidates a
 * captured graph. */
int rf_batch_set_grid(rf_batch *plan, uint32_t stage, uint32_t workgroups);
/* Limb grouping of the batched ModUp conversion: output limbs per thread,
 * 4, 8 (default) or 16 (modup_chunk of rf_tuning).  Waits for the device to
 * be idle, rebuilds and uploads the job tables and invalidates a captured
 * graph; RF_EINVAL for another value. */
int rf_batch_set_modup_chunk(rf_batch *plan, uint32_t chunk);
/* Work units of launch `stage` (or a negative RF_E* code). */
int rf_batch_stage_units(const rf_batch *plan, uint32_t stage);
/* Enqueue the batch on `stream`. */
int rf_batch_hmult_relin(rf_batch *plan, void *stream);
/* Same, through a hipGraph captured on the first call (and after a grid change). */
int rf_batch_graph_launch(rf_batch *plan, void *stream);

/* Measurement support (the per-stage timings of III-B and V-C).  While enabled,
 * every kernel launch of the library is bracketed by two HIP events recorded on
 * the launch's own stream (a few microseconds of overhead per launch).
 * rf_profile_read waits for the recorded events, writes one line
 * "kernel_name launches total_ms" per kernel into buf (NUL-terminated,
 * truncated to len), clears the records and returns the full text length (or a
 * negative RF_E* code).  Process-wide, thread-safe. */
int rf_profile_enable(int on);
int rf_profile_read(char *buf, size_t len);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *rf_last_error(void);

/* Library version string. */
const char *rf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RNSFHE_H */
