// C ABI entry points: argument checks, workspace layout and the kernel chains
// of HMult+Relin, HRotate, key switching and rescale.
#include <hip/hip_runtime.h>

#include "rf_internal.hpp"

using namespace rf;

namespace {

// Key-switching workspace at level nl, in limbs of N residues:
//   d_coeff [nl] | ext [ext_limbs] | ip [2][nl+K] | conv [2][nl]
struct KsLayout {
    size_t d_coeff, ext, ip, conv, total;
};

KsLayout ks_layout(const rf_ctx *c, uint32_t nl) {
    KsLayout l;
    const size_t N = c->n;
    l.d_coeff = 0;
    l.ext = l.d_coeff + (size_t)nl * N;
    l.ip = l.ext + (size_t)c->modup_levels[nl].ext_limbs * N;
    l.conv = l.ip + 2 * (size_t)(nl + c->K) * N;
    l.total = l.conv + 2 * (size_t)nl * N;
    return l;
}

int check_level(const rf_ctx *c, uint32_t nl, uint32_t min_limbs = 1) {
    if (!c) return fail(RF_EINVAL, "null context");
    if (nl < min_limbs || nl > c->L) return fail(RF_ELEVEL, "limb count out of range for this chain");
    return RF_OK;
}

int check_ws(const rf_ctx *c, int op, uint32_t nl, void *ws, size_t ws_bytes) {
    size_t need = rf_workspace_bytes(c, op, nl);
    if (!ws || ws_bytes < need)
        return fail(RF_EWORKSPACE, "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(need));
    return RF_OK;
}

// Whether [a, a + na) and [b, b + nb) (in uint64 residues) share memory.
bool overlaps(const uint64_t *a, size_t na, const uint64_t *b, size_t nb) { return a < b + nb && b < a + na; }

// Set the context's device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

NttBatch batch(const uint64_t *in, uint64_t *out, uint64_t in_stride, uint64_t out_stride, uint32_t per_poly,
               uint32_t n_polys, uint32_t prime_base, const uint32_t *pmap) {
    NttBatch b;
    b.in = in;
    b.out = out;
    b.in_poly_stride = in_stride;
    b.out_poly_stride = out_stride;
    b.per_poly = per_poly;
    b.n_polys = n_polys;
    b.prime_base = prime_base;
    b.pmap = pmap;
    return b;
}

// (KS_0(d), KS_1(d)) into out [2][nl][N]; add0/add1 (nullable) are added.
// fused (two-pass ring degrees only): d is not materialised; the workspace's
// d_coeff region already holds INTT(d) (launch_intt_first) and the inner
// product takes d's residues and the addends from fused's sources.
// d_coeff_in (nullable): d in the coefficient domain, given by the caller
// (BFV's fast floor produces it), which replaces the INTT of d.
int keyswitch_core(const rf_ctx *c, const uint64_t *d, const uint64_t *evk, uint64_t *out, uint32_t nl,
                   const uint64_t *add0, const uint64_t *add1, uint64_t *ws, hipStream_t s,
                   const IpFold *fused = nullptr, const uint64_t *d_coeff_in = nullptr) {
    const KsLayout l = ks_layout(c, nl);
    const size_t N = c->n;
    const ModupLevel &lv = c->modup_levels[nl];
    uint64_t *d_coeff = ws + l.d_coeff, *ext = ws + l.ext, *ip = ws + l.ip, *conv = ws + l.conv;
    int rc;
    // ModUp: INTT of d, base conversion of each digit, NTT of the new limbs.
    // Two-pass ring degrees: the INTT folds in the conversion's input factor
    // (pc_modup; launch_intt_first does the same for the fused callers).
    const rf_tuning &tn = level_tuning(c, nl);
    const bool scaled = c->log_n > 12 && !d_coeff_in;
    if (!fused && !d_coeff_in &&
        (rc = launch_ntt(c, batch(d, d_coeff, 0, 0, nl, 1, 0, nullptr), false, s, scaled ? pc_modup(c, nl) : nullptr,
                         &tn)))
        return rc;
    if ((rc = launch_modup_bconv(c, d_coeff_in ? d_coeff_in : d_coeff, ext, nl, s, scaled, tn.modup_chunk))) return rc;
    if ((rc = launch_ntt(c, batch(ext, ext, 0, 0, lv.ext_limbs, 1, 0, c->d_pmaps + lv.pmap_off), true, s, nullptr, &tn)))
        return rc;
    // ModDown: INTT of the P-limbs, base conversion to Q_l, NTT, subtract and scale by P^-1
    const uint64_t ip_stride = (uint64_t)(nl + c->K) * N;
    const NttBatch pl = batch(ip + (size_t)nl * N, ip + (size_t)nl * N, ip_stride, ip_stride, c->K, 2, c->L, nullptr);
    if (c->log_n > 12) {
        // the inner product applies P^-1 and the addends to its Q-limbs; the INTT
        // of the P-limbs folds in the conversion's input factor; the conversion
        // runs in the first pass of the NTT and the tail in its last pass
        IpFold f;
        if (fused) {
            f = *fused;
        } else {
            f.add0 = add0;
            f.add1 = add1;
        }
        if ((rc = launch_inner_product(c, d, ext, evk, ip, nl, s, &f))) return rc;
        if ((rc = launch_ntt(c, pl, false, s, c->d_pc_md, &tn))) return rc;
        return launch_ntt_fwd_moddown(c, conv, ip, out, nl, s, &tn);
    }
    // inner product with the key over Q_l u P
    if ((rc = launch_inner_product(c, d, ext, evk, ip, nl, s))) return rc;
    if ((rc = launch_ntt(c, pl, false, s, nullptr, &tn))) return rc;
    if ((rc = launch_moddown_bconv(c, ip, conv, nl, s))) return rc;
    if ((rc = launch_ntt(c, batch(conv, conv, (uint64_t)nl * N, (uint64_t)nl * N, nl, 2, 0, nullptr), true, s, nullptr,
                         &tn)))
        return rc;
    return launch_moddown_tail(c, ip, conv, add0, add1, out, nl, s);
}

}  // namespace

// BFV HMult+Relin workspace, in limbs of N residues (W = L + nb + 1):
//   ext [4][W] | tens [3][W] | d2 [L] | ks_out [2][L] | key-switch workspace
static size_t bfv_ws_limbs(const rf_ctx *c) {
    const size_t W = c->L + c->nb + 1;
    return 7 * W + 3 * (size_t)c->L + ks_layout(c, c->L).total / c->n;
}

extern "C" size_t rf_workspace_bytes(const rf_ctx *c, int op, uint32_t nl) {
    if (!c || nl < 1 || nl > c->L) return 0;
    const size_t N = c->n;
    if (c->scheme == RF_BFV && op == RF_OP_HMULT_RELIN) return nl == c->L ? bfv_ws_limbs(c) * N * 8 : 0;
    switch (op) {
        case RF_OP_KEYSWITCH: return ks_layout(c, nl).total * 8;
        case RF_OP_HMULT_RELIN: return (ks_layout(c, nl).total + (size_t)nl * N) * 8;
        // BFV: the NTT of the coefficient-domain input comes first
        case RF_OP_ROTATE: return (ks_layout(c, nl).total + (size_t)(c->scheme == RF_BFV ? 3 : 1) * nl * N) * 8;
        case RF_OP_RESCALE: return nl < 2 ? 0 : (2 + 2 * (size_t)(nl - 1)) * N * 8;
        case RF_OP_MODSWITCH: return (nl < 2 || c->scheme != RF_BGV) ? 0 : (2 + 2 * (size_t)(nl - 1)) * N * 8;
        // two buffers of N complex doubles (the FFT's ping-pong)
        case RF_OP_ENCODE: case RF_OP_DECODE: return c->scheme == RF_CKKS ? 32 * N : 0;
        default: return 0;
    }
}

extern "C" int rf_ntt(const rf_ctx *c, uint64_t *data, uint32_t first, uint32_t nl, uint32_t np, void *stream) {
    if (!c || !data) return fail(RF_EINVAL, "rf_ntt: null argument");
    if (nl == 0 || np == 0 || first + nl > c->L + c->K) return fail(RF_ELEVEL, "rf_ntt: limb range");
    DeviceGuard g(c->device);
    const uint64_t stride = (uint64_t)nl * c->n;
    return launch_ntt(c, batch(data, data, stride, stride, nl, np, first, nullptr), true, (hipStream_t)stream, nullptr,
                      &level_tuning(c, nl));
}

extern "C" int rf_intt(const rf_ctx *c, uint64_t *data, uint32_t first, uint32_t nl, uint32_t np, void *stream) {
    if (!c || !data) return fail(RF_EINVAL, "rf_intt: null argument");
    if (nl == 0 || np == 0 || first + nl > c->L + c->K) return fail(RF_ELEVEL, "rf_intt: limb range");
    DeviceGuard g(c->device);
    const uint64_t stride = (uint64_t)nl * c->n;
    return launch_ntt(c, batch(data, data, stride, stride, nl, np, first, nullptr), false, (hipStream_t)stream, nullptr,
                      &level_tuning(c, nl));
}

extern "C" int rf_tensor(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *d, uint32_t nl,
                         void *stream) {
    int rc;
    if ((rc = check_level(c, nl))) return rc;
    if (!a || !b || !d) return fail(RF_EINVAL, "rf_tensor: null argument");
    DeviceGuard g(c->device);
    return launch_tensor(c, a, b, d, d + 2 * (size_t)nl * c->n, nl, (hipStream_t)stream);
}

extern "C" int rf_keyswitch(const rf_ctx *c, const uint64_t *d, const uint64_t *evk, uint64_t *out, uint32_t nl,
                            int accumulate, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_level(c, nl))) return rc;
    if (!d || !evk || !out) return fail(RF_EINVAL, "rf_keyswitch: null argument");
    if ((rc = check_ws(c, RF_OP_KEYSWITCH, nl, ws, ws_bytes))) return rc;
    DeviceGuard g(c->device);
    const size_t poly = (size_t)nl * c->n;
    return keyswitch_core(c, d, evk, out, nl, accumulate ? out : nullptr, accumulate ? out + poly : nullptr,
                          (uint64_t *)ws, (hipStream_t)stream);
}

// BFV: BEHZ tensor on q u B_sk, then relinearisation of d2 (coefficient domain in and out).
static int bfv_hmult_relin(const rf_ctx *c, const uint64_t *a, const uint64_t *b, const uint64_t *rlk, uint64_t *out,
                           uint64_t *ws, hipStream_t s) {
    int rc;
    const size_t N = c->n, L = c->L;
    const uint32_t W = c->L + c->nb + 1;
    uint64_t *ext = ws;                       // [4][W][N]: a0, a1, b0, b1 on q u B_sk
    uint64_t *tens = ext + 4 * (size_t)W * N; // [3][W][N]
    uint64_t *d2 = tens + 3 * (size_t)W * N;  // [L][N]
    uint64_t *ks = d2 + L * N;                // [2][L][N]
    uint64_t *ks_ws = ks + 2 * L * N;
    const uint64_t wstride = (uint64_t)W * N;
    const rf_tuning &tn = level_tuning(c, c->L);
    if ((rc = launch_behz_extend(c, a, b, ext, s))) return rc;
    if ((rc = launch_ntt(c, batch(ext, ext, wstride, wstride, W, 4, 0, c->d_pmap_qb), true, s, nullptr, &tn))) return rc;
    if ((rc = launch_tensor_map(c, ext, ext + 2 * wstride, tens, tens + 2 * wstride, W, c->d_pmap_qb, s))) return rc;
    if ((rc = launch_ntt(c, batch(tens, tens, wstride, wstride, W, 3, 0, c->d_pmap_qb), false, s, nullptr, &tn))) return rc;
    // the fast floor's B_sk residues go through the extension region, free after the tensor
    if ((rc = launch_behz_floor_sk(c, tens, ext, out, d2, s))) return rc;
    // the key switch takes d2 in both domains: the NTT (into the free tensor
    // region) for its inner product, the coefficients for its ModUp
    uint64_t *d2n = tens;
    if ((rc = launch_ntt(c, batch(d2, d2n, 0, 0, c->L, 1, 0, nullptr), true, s, nullptr, &tn))) return rc;
    if ((rc = keyswitch_core(c, d2n, rlk, ks, c->L, nullptr, nullptr, ks_ws, s, nullptr, d2))) return rc;
    if ((rc = launch_ntt(c, batch(ks, ks, L * N, L * N, c->L, 2, 0, nullptr), false, s, nullptr, &tn))) return rc;
    return launch_ewise(c, 0, out, ks, 0, out, c->L, 2, s);
}

extern "C" int rf_hmult_relin(const rf_ctx *c, const uint64_t *a, const uint64_t *b, const uint64_t *rlk,
                              uint64_t *out, uint32_t nl, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_level(c, nl))) return rc;
    if (!a || !b || !rlk || !out) return fail(RF_EINVAL, "rf_hmult_relin: null argument");
    const size_t ct = 2 * (size_t)nl * c->n;
    if (overlaps(out, ct, a, ct) || overlaps(out, ct, b, ct))
        return fail(RF_EINVAL, "rf_hmult_relin: out overlaps an input");
    if ((rc = check_ws(c, RF_OP_HMULT_RELIN, nl, ws, ws_bytes))) return rc;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (c->scheme == RF_BFV) {
        if (nl != c->L) return fail(RF_ELEVEL, "rf_hmult_relin: BFV ciphertexts carry all L limbs");
        return bfv_hmult_relin(c, a, b, rlk, out, (uint64_t *)ws, s);
    }
    const size_t poly = (size_t)nl * c->n;
    uint64_t *d2 = (uint64_t *)ws;
    uint64_t *ks_ws = d2 + poly;
    if (c->log_n > 12) {
        // d2 = a1 b1 is formed by the first pass of its INTT and, with d0 and d1,
        // by the inner product
        if ((rc = launch_intt_first(c, a, b, ks_ws + ks_layout(c, nl).d_coeff, 0, nl, s, &level_tuning(c, nl))))
            return rc;
        IpFold f;
        f.mode = 1;
        f.a = a;
        f.b = b;
        return keyswitch_core(c, nullptr, rlk, out, nl, nullptr, nullptr, ks_ws, s, &f);
    }
    if ((rc = launch_tensor(c, a, b, out, d2, nl, s))) return rc;
    return keyswitch_core(c, d2, rlk, out, nl, out, out + poly, ks_ws, s);
}

// HRotate of an NTT-domain ciphertext (CKKS, BGV) into out; ws holds the
// automorphism of polynomial 1 and the key-switch workspace.
static int rotate_ntt(const rf_ctx *c, const uint64_t *in, uint32_t galois, const uint64_t *gk, uint64_t *out,
                      uint32_t nl, uint64_t *ws, hipStream_t s) {
    int rc;
    const size_t poly = (size_t)nl * c->n;
    uint64_t *d = ws;
    uint64_t *ks_ws = d + poly;
    if (c->log_n > 12) {
        // sigma_g(a1) is gathered by the first pass of its INTT and, with sigma_g(a0),
        // by the inner product
        if ((rc = launch_intt_first(c, in, nullptr, ks_ws + ks_layout(c, nl).d_coeff, galois, nl, s,
                                    &level_tuning(c, nl))))
            return rc;
        IpFold f;
        f.mode = 2;
        f.a = in;
        f.galois = galois;
        return keyswitch_core(c, nullptr, gk, out, nl, nullptr, nullptr, ks_ws, s, &f);
    }
    if ((rc = launch_automorphism(c, in, out, galois, nl, 1, s))) return rc;
    if ((rc = launch_automorphism(c, in + poly, d, galois, nl, 1, s))) return rc;
    return keyswitch_core(c, d, gk, out, nl, out, nullptr, ks_ws, s);
}

extern "C" int rf_rotate(const rf_ctx *c, const uint64_t *in, uint32_t galois, const uint64_t *gk, uint64_t *out,
                         uint32_t nl, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_level(c, nl))) return rc;
    if (!in || !gk || !out) return fail(RF_EINVAL, "rf_rotate: null argument");
    if (overlaps(out, 2 * (size_t)nl * c->n, in, 2 * (size_t)nl * c->n))
        return fail(RF_EINVAL, "rf_rotate: out overlaps in");
    if ((galois & 1u) == 0 || galois >= 2u * c->n) return fail(RF_EINVAL, "rf_rotate: Galois element must be odd and < 2N");
    if (c->scheme == RF_BFV && nl != c->L) return fail(RF_ELEVEL, "rf_rotate: BFV ciphertexts carry all L limbs");
    if ((rc = check_ws(c, RF_OP_ROTATE, nl, ws, ws_bytes))) return rc;
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (c->scheme != RF_BFV) return rotate_ntt(c, in, galois, gk, out, nl, (uint64_t *)ws, s);
    // BFV rests in the coefficient domain.  NTT(sigma_g(a)) is a fixed
    // permutation of NTT(a), so rotating the NTT of the input and transforming
    // the result back applies sigma_g (and the key switch) to the coefficients.
    const size_t poly = (size_t)nl * c->n;
    uint64_t *x = (uint64_t *)ws;
    if ((rc = launch_ntt(c, batch(in, x, poly, poly, nl, 2, 0, nullptr), true, s, nullptr, &level_tuning(c, nl)))) return rc;
    if ((rc = rotate_ntt(c, x, galois, gk, out, nl, x + 2 * poly, s))) return rc;
    return launch_ntt(c, batch(out, out, poly, poly, nl, 2, 0, nullptr), false, s, nullptr, &level_tuning(c, nl));
}

extern "C" int rf_galois_element(const rf_ctx *c, int64_t r, int conjugate, uint32_t *out) {
    if (!c || !out) return fail(RF_EINVAL, "rf_galois_element: null argument");
    // 5 has order N/2 in (Z/2NZ)^*: reduce r mod N/2 (a negative r rotates right)
    const uint64_t two_n = 2ull * c->n, half = c->n / 2;
    int64_t e = r % (int64_t)half;
    if (e < 0) e += (int64_t)half;
    uint64_t g = 1, b = 5;
    for (uint64_t k = (uint64_t)e; k; k >>= 1) {
        if (k & 1) g = g * b % two_n;
        b = b * b % two_n;
    }
    if (conjugate) g = g * (two_n - 1) % two_n;
    *out = (uint32_t)g;
    return RF_OK;
}

extern "C" int rf_automorphism(const rf_ctx *c, const uint64_t *in, uint64_t *out, uint32_t galois, uint32_t nl,
                               uint32_t np, void *stream) {
    int rc;
    if ((rc = check_level(c, nl))) return rc;
    if (!in || !out || np == 0) return fail(RF_EINVAL, "rf_automorphism: bad argument");
    if (out == in) return fail(RF_EINVAL, "rf_automorphism: out aliases in");
    if ((galois & 1u) == 0 || galois >= 2u * c->n) return fail(RF_EINVAL, "Galois element must be odd and < 2N");
    DeviceGuard g(c->device);
    return launch_automorphism(c, in, out, galois, nl, np, (hipStream_t)stream);
}

// Divide by the last prime q_l with rounding, keeping the message mod t when
// keep_t (BGV modulus switch): out = (in - lift(last limb)) * q_l^-1.
static int divide_last(const rf_ctx *c, const uint64_t *in, uint64_t *out, uint32_t nl, void *ws, bool keep_t,
                       hipStream_t s) {
    int rc;
    const size_t N = c->n;
    uint64_t *last = (uint64_t *)ws;         // [2][N]
    uint64_t *lift = last + 2 * N;           // [2][nl-1][N]
    const uint64_t in_stride = (uint64_t)nl * N;
    const rf_tuning &tn = level_tuning(c, nl);
    if ((rc = launch_ntt(c, batch(in + (size_t)(nl - 1) * N, last, in_stride, N, 1, 2, nl - 1, nullptr), false, s,
                         nullptr, &tn)))
        return rc;
    // out has a smaller polynomial stride than in: when they overlap, compute in
    // the workspace and copy the result over.
    const bool overlap = (const void *)out < (const void *)(in + 2 * (size_t)nl * N) &&
                         (const void *)in < (const void *)(out + 2 * (size_t)(nl - 1) * N);
    if (c->log_n > 12) {
        // the lift runs in the first pass of the NTT and the tail in its last pass
        if (!overlap) return launch_ntt_fwd_rescale(c, last, lift, in, out, nl, keep_t, s, &tn);
        if ((rc = launch_ntt_fwd_rescale(c, last, lift, in, lift, nl, keep_t, s, &tn))) return rc;
    } else {
        if ((rc = launch_rescale_lift(c, last, lift, nl, keep_t, s))) return rc;
        if ((rc = launch_ntt(c, batch(lift, lift, (uint64_t)(nl - 1) * N, (uint64_t)(nl - 1) * N, nl - 1, 2, 0,
                                      nullptr), true, s, nullptr, &tn)))
            return rc;
        if (!overlap) return launch_rescale_tail(c, in, lift, out, nl, s);
        if ((rc = launch_rescale_tail(c, in, lift, lift, nl, s))) return rc;
    }
    if (hipMemcpyAsync(out, lift, 2 * (size_t)(nl - 1) * N * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(RF_EHIP, "copy of the divided ciphertext");
    return RF_OK;
}

extern "C" int rf_rescale(const rf_ctx *c, const uint64_t *in, uint64_t *out, uint32_t nl, void *ws, size_t ws_bytes,
                          void *stream) {
    int rc;
    if ((rc = check_level(c, nl, 2))) return rc;
    if (c->scheme != RF_CKKS) return fail(RF_EUNSUPPORTED, "rf_rescale: CKKS only (use rf_modswitch for BGV)");
    if (!in || !out) return fail(RF_EINVAL, "rf_rescale: null argument");
    if ((rc = check_ws(c, RF_OP_RESCALE, nl, ws, ws_bytes))) return rc;
    DeviceGuard g(c->device);
    return divide_last(c, in, out, nl, ws, false, (hipStream_t)stream);
}

extern "C" int rf_modswitch(const rf_ctx *c, const uint64_t *in, uint64_t *out, uint32_t nl, void *ws,
                            size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_level(c, nl, 2))) return rc;
    if (!in || !out) return fail(RF_EINVAL, "rf_modswitch: null argument");
    DeviceGuard g(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (c->scheme == RF_BGV) {
        if ((rc = check_ws(c, RF_OP_MODSWITCH, nl, ws, ws_bytes))) return rc;
        return divide_last(c, in, out, nl, ws, true, s);
    }
    if (c->scheme != RF_CKKS) return fail(RF_EUNSUPPORTED, "rf_modswitch: CKKS or BGV");
    const size_t N = c->n;
    const size_t limb = N * 8;
    // limb by limb in increasing address order: each copy moves data to a lower
    // address, so with out == in no limb is overwritten before it is read
    for (uint32_t p = 0; p < 2; ++p)
        for (uint32_t i = 0; i + 1 < nl; ++i) {
            const uint64_t *src = in + ((size_t)p * nl + i) * N;
            uint64_t *dst = out + ((size_t)p * (nl - 1) + i) * N;
            if (src == dst) continue;
            if (hipMemcpyAsync(dst, src, limb, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(RF_EHIP, "rf_modswitch: copy");
        }
    return RF_OK;
}

static int ewise_entry(const rf_ctx *c, int op, const uint64_t *a, const uint64_t *b, int64_t k, uint64_t *out,
                       uint32_t nl, uint32_t np, void *stream, const char *name) {
    int rc;
    if ((rc = check_level(c, nl))) return rc;
    if (!a || !out || np == 0 || ((op == 0 || op == 1 || op == 4) && !b))
        return fail(RF_EINVAL, std::string(name) + ": bad argument");
    DeviceGuard g(c->device);
    return launch_ewise(c, op, a, b, k, out, nl, np, (hipStream_t)stream);
}

extern "C" int rf_add(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t nl, uint32_t np,
                      void *stream) {
    return ewise_entry(c, 0, a, b, 0, out, nl, np, stream, "rf_add");
}

extern "C" int rf_sub(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t nl, uint32_t np,
                      void *stream) {
    return ewise_entry(c, 1, a, b, 0, out, nl, np, stream, "rf_sub");
}

extern "C" int rf_mul_scalar(const rf_ctx *c, const uint64_t *a, int64_t k, uint64_t *out, uint32_t nl, uint32_t np,
                             void *stream) {
    return ewise_entry(c, 2, a, nullptr, k, out, nl, np, stream, "rf_mul_scalar");
}

extern "C" int rf_add_scalar(const rf_ctx *c, const uint64_t *a, int64_t k, uint64_t *out, uint32_t nl,
                             void *stream) {
    return ewise_entry(c, 3, a, nullptr, k, out, nl, 2, stream, "rf_add_scalar");
}

extern "C" int rf_mul_plain(const rf_ctx *c, const uint64_t *a, const uint64_t *p, uint64_t *out, uint32_t nl,
                            uint32_t np, void *stream) {
    return ewise_entry(c, 4, a, p, 0, out, nl, np, stream, "rf_mul_plain");
}
