// Client side on the GPU: key generation, secret-key encryption, decryption,
// CRT composition and CKKS encode / decode (the create-key, encode, encrypt,
// decrypt and decode rows of the operator tables of section V-A; the client
// of the query framework, IV-A).  Random draws come in as arguments; the
// integer steps are exact, encode / decode run in double precision.
//
// Kernels are one thread per coefficient (grid.x over N in blocks of kCl,
// grid.y over limbs, grid.z over polynomials) except the FFT stages (one
// thread per butterfly).
#include <hip/hip_runtime.h>

#include "ks_dev.hpp"
#include "rf_internal.hpp"

namespace rf {

constexpr int kCl = 256;
constexpr uint32_t kMaxCrtLimbs = 32;
constexpr int kCrtThreads = 128;

// Representative in [0, q) of a signed 64-bit integer.
__device__ __forceinline__ uint64_t signed_mod(int64_t v, const PrimeConst &pc) {
    const uint64_t mag = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
    const uint64_t r = barrett64(mag, pc.mu1, pc.mu0, pc.q);
    return (v < 0 && r) ? pc.q - r : r;
}

// Lift flags: the x term times floor(Q_L / t) (BFV message), the y term times t
// (BGV error), the x term times t (BGV key error).
enum LiftMode { kLiftXDelta = 1, kLiftYT = 2, kLiftXT = 4 };

// out[z][i][n] = x[z][n] (times the mode's factor) + y[z][n] (likewise) mod p_{first+i}.
__global__ __launch_bounds__(kCl) void lift_kernel(const int64_t *__restrict__ x, const int64_t *__restrict__ y,
                                                   size_t in_stride, uint64_t *__restrict__ out, size_t out_stride,
                                                   const PrimeConst *__restrict__ pcs, const uint64_t *__restrict__ cl,
                                                   uint32_t first, uint32_t log_n, int mode) {
    const uint32_t i = blockIdx.y, z = blockIdx.z, g = first + i;
    const size_t n = (size_t)blockIdx.x * kCl + threadIdx.x;
    const PrimeConst pc = pcs[g];
    uint64_t r = signed_mod(x[z * in_stride + n], pc);
    if (mode & kLiftXDelta) r = shoup(r, cl[4 * g + 2], cl[4 * g + 3], pc.q);
    if (mode & kLiftXT) r = shoup(r, pc.tmod, pc.tmod_p, pc.q);
    if (y) {
        uint64_t e = signed_mod(y[z * in_stride + n], pc);
        if (mode & kLiftYT) e = shoup(e, pc.tmod, pc.tmod_p, pc.q);
        r = addmod(r, e, pc.q);
    }
    out[z * out_stride + ((size_t)i << log_n) + n] = r;
}

// SUB: out = x - a s; otherwise out = x + a s (limb i mod q_i, s limb i of [L+K][N]).
template <bool SUB>
__global__ __launch_bounds__(kCl) void fma_s_kernel(const uint64_t *x, const uint64_t *__restrict__ a,
                                                    const uint64_t *__restrict__ s, uint64_t *out,
                                                    const PrimeConst *__restrict__ pcs, uint32_t log_n) {
    const uint32_t i = blockIdx.y;
    const size_t off = ((size_t)i << log_n) + (size_t)blockIdx.x * kCl + threadIdx.x;
    const PrimeConst pc = pcs[i];
    const uint64_t as = mulmod(a[off], s[off], pc.mu1, pc.mu0, pc.q);
    out[off] = SUB ? submod(x[off], as, pc.q) : addmod(x[off], as, pc.q);
}

// Switching-key assembly of digit j = blockIdx.z on limb m = blockIdx.y of Q_L u P:
// evk[j][0][m] (holding NTT(err e_j) on entry) += -a_j s + [m in D_j] [P]_{q_m} s',
// s' = s^2 (galois 0) or sigma_g(s); evk[j][1][m] = a_j.
__global__ __launch_bounds__(kCl) void keygen_kernel(uint64_t *evk, const uint64_t *__restrict__ a,
                                                     const uint64_t *__restrict__ s, const PrimeConst *__restrict__ pcs,
                                                     const uint64_t *__restrict__ cl, uint32_t galois, uint32_t log_n,
                                                     uint32_t L, uint32_t K, uint32_t alpha) {
    const uint32_t m = blockIdx.y, j = blockIdx.z;
    const uint32_t n = blockIdx.x * kCl + threadIdx.x;
    const size_t limbs = (size_t)(L + K) << log_n;
    const size_t off = ((size_t)m << log_n) + n;
    const PrimeConst pc = pcs[m];
    uint64_t *b = evk + 2 * (size_t)j * limbs;
    const uint64_t aj = a[(size_t)j * limbs + off];
    const uint64_t sm = s[off];
    uint64_t v = submod(b[off], mulmod(aj, sm, pc.mu1, pc.mu0, pc.q), pc.q);
    if (m < L && m >= j * alpha && m < j * alpha + alpha) {
        const uint64_t sf = galois ? s[((size_t)m << log_n) + galois_src(n, galois, log_n)]
                                   : mulmod(sm, sm, pc.mu1, pc.mu0, pc.q);
        v = addmod(v, shoup(sf, cl[4 * m], cl[4 * m + 1], pc.q), pc.q);
    }
    b[off] = v;
    b[limbs + off] = aj;
}

// Balanced mixed-radix digits of each coefficient, X = sum_i v_i q_0 .. q_{i-1}
// with v_i in (-q_i/2, q_i/2]: a complete residue system, so X is the centred
// representative mod Q_l.  Horner in double from the top digit, then / scale.
__global__ __launch_bounds__(kCrtThreads) void crt_centered_kernel(const uint64_t *__restrict__ x, double *out,
                                                                   const PrimeConst *__restrict__ pcs,
                                                                   const uint64_t *__restrict__ gar, uint32_t L,
                                                                   uint32_t nl, uint32_t log_n, double scale) {
    __shared__ int64_t v[kMaxCrtLimbs][kCrtThreads];
    const size_t n = (size_t)blockIdx.x * kCrtThreads + threadIdx.x;
    const int tid = threadIdx.x;
    for (uint32_t j = 0; j < nl; ++j) {
        const PrimeConst pc = pcs[j];
        uint64_t t = x[((size_t)j << log_n) + n];
        for (uint32_t i = 0; i < j; ++i) {
            const uint64_t *gi = gar + ((size_t)i * L + j) * 2;
            t = shoup(submod(t, signed_mod(v[i][tid], pc), pc.q), gi[0], gi[1], pc.q);
        }
        v[j][tid] = t > (pc.q >> 1) ? (int64_t)t - (int64_t)pc.q : (int64_t)t;
    }
    double acc = (double)v[nl - 1][tid];
    for (int i = (int)nl - 2; i >= 0; --i) acc = fma(acc, (double)pcs[i].q, (double)v[i][tid]);
    out[n] = acc / scale;
}

// One radix-2 stage of a Stockham FFT of N points (natural order in and out):
// butterfly j combines in[j] and in[j + N/2] with the twiddle
// exp(sign 2 pi i k / (2 Ns)) = zeta^(+-k N / Ns), k = j mod Ns.
__global__ __launch_bounds__(kCl) void fft_stage_kernel(const double2 *__restrict__ in, double2 *__restrict__ out,
                                                        const double2 *__restrict__ zeta, uint32_t log_n, uint32_t Ns,
                                                        int sign) {
    const uint32_t N = 1u << log_n;
    const uint32_t j = blockIdx.x * kCl + threadIdx.x;
    const double2 v0 = in[j], x1 = in[j + N / 2];
    const uint32_t k = j & (Ns - 1);
    uint32_t e = (uint32_t)(((uint64_t)k * N / Ns) & (2 * N - 1));
    if (sign < 0) e = (2 * N - e) & (2 * N - 1);
    const double2 w = zeta[e];
    const double2 v1 = make_double2(x1.x * w.x - x1.y * w.y, x1.x * w.y + x1.y * w.x);
    const uint32_t d = (j / Ns) * 2 * Ns + k;
    out[d] = make_double2(v0.x + v1.x, v0.y + v1.y);
    out[d + Ns] = make_double2(v0.x - v1.x, v0.y - v1.y);
}

// Decode, before the FFT: y_i = x_i zeta^i (the negacyclic twist).
__global__ __launch_bounds__(kCl) void decode_pre_kernel(const double *__restrict__ x, double2 *__restrict__ y,
                                                         const double2 *__restrict__ zeta) {
    const uint32_t i = blockIdx.x * kCl + threadIdx.x;
    const double2 w = zeta[i];
    y[i] = make_double2(x[i] * w.x, x[i] * w.y);
}

// Decode, after the FFT: slot j = V[(5^j mod 2N - 1) / 2].
__global__ __launch_bounds__(kCl) void decode_post_kernel(const double2 *__restrict__ V, double2 *__restrict__ z,
                                                          const uint32_t *__restrict__ slot_idx) {
    const uint32_t j = blockIdx.x * kCl + threadIdx.x;
    z[j] = V[slot_idx[j]];
}

// Encode, before the FFT: the value at zeta^(2t+1) for every t: z_j at
// 2t+1 = 5^j mod 2N, its conjugate at 2N - 5^j (t' = N - 1 - t).
__global__ __launch_bounds__(kCl) void encode_pre_kernel(const double2 *__restrict__ z, double2 *__restrict__ u,
                                                         const uint32_t *__restrict__ slot_idx, uint32_t N) {
    const uint32_t j = blockIdx.x * kCl + threadIdx.x;
    const double2 v = z[j];
    const uint32_t t = slot_idx[j];
    u[t] = v;
    u[N - 1 - t] = make_double2(v.x, -v.y);
}

// Encode, after the FFT: m_i = round(Re(zeta^-i U_i) scale / N), clamped to |m| <= 2^62.
__global__ __launch_bounds__(kCl) void encode_post_kernel(const double2 *__restrict__ U, int64_t *__restrict__ m,
                                                          const double2 *__restrict__ zeta, uint32_t N, double factor) {
    const uint32_t i = blockIdx.x * kCl + threadIdx.x;
    const double2 w = zeta[(2 * N - i) & (2 * N - 1)];
    const double2 x = U[i];
    double re = rint((w.x * x.x - w.y * x.y) * factor);
    const double lim = 4611686018427387904.0;  // 2^62
    re = fmin(fmax(re, -lim), lim);
    m[i] = (int64_t)re;
}

}  // namespace rf

using namespace rf;

namespace {

bool overlaps_bytes(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return RF_OK;
}

struct Dev {
    int prev = -1;
    explicit Dev(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) (void)hipSetDevice(d);
    }
    ~Dev() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

NttBatch plain_batch(uint64_t *d, uint64_t stride, uint32_t per_poly, uint32_t n_polys) {
    NttBatch b;
    b.in = d;
    b.out = d;
    b.in_poly_stride = stride;
    b.out_poly_stride = stride;
    b.per_poly = per_poly;
    b.n_polys = n_polys;
    b.prime_base = 0;
    b.pmap = nullptr;
    return b;
}

int lift(const rf_ctx *c, const int64_t *x, const int64_t *y, size_t in_stride, uint64_t *out, size_t out_stride,
         uint32_t first, uint32_t nlimbs, uint32_t npolys, int mode, hipStream_t s) {
    ProfScope prof("client_lift", s);
    hipLaunchKernelGGL(lift_kernel, dim3(c->n / kCl, nlimbs, npolys), dim3(kCl), 0, s, x, y, in_stride, out,
                       out_stride, c->d_pc, c->d_client, first, c->log_n, mode);
    return check_launch("lift");
}

// FFT of N complex values from buf0 with ping-pong into buf1; returns the buffer holding the result.
double2 *fft(const rf_ctx *c, double2 *buf0, double2 *buf1, int sign, hipStream_t s) {
    ProfScope prof("client_fft", s);
    for (uint32_t Ns = 1; Ns < c->n; Ns <<= 1) {
        hipLaunchKernelGGL(fft_stage_kernel, dim3(c->n / 2 / kCl), dim3(kCl), 0, s, buf0, buf1,
                           (const double2 *)c->d_zeta, c->log_n, Ns, sign);
        double2 *t = buf0;
        buf0 = buf1;
        buf1 = t;
    }
    return buf0;
}

}  // namespace

extern "C" int rf_key_ntt(const rf_ctx *c, const int64_t *x, uint64_t *out, void *stream) {
    if (!c || !x || !out) return fail(RF_EINVAL, "rf_key_ntt: null argument");
    Dev g(c->device);
    hipStream_t s = (hipStream_t)stream;
    const uint32_t all = c->L + c->K;
    int rc;
    if ((rc = lift(c, x, nullptr, 0, out, 0, 0, all, 1, 0, s))) return rc;
    return launch_ntt(c, plain_batch(out, 0, all, 1), true, s);
}

extern "C" int rf_keygen_switch(const rf_ctx *c, const uint64_t *s_ntt, uint32_t galois, const uint64_t *a,
                                const int64_t *e, uint64_t *evk, void *stream) {
    if (!c || !s_ntt || !a || !e || !evk) return fail(RF_EINVAL, "rf_keygen_switch: null argument");
    if (galois != 0 && ((galois & 1u) == 0 || galois >= 2u * c->n))
        return fail(RF_EINVAL, "rf_keygen_switch: Galois element must be 0 (relinearisation) or odd and < 2N");
    const uint32_t all = c->L + c->K;
    const size_t limbs = (size_t)all * c->n;
    const size_t key_bytes = (size_t)c->dnum * 2 * limbs * 8;
    if (overlaps_bytes(evk, key_bytes, s_ntt, limbs * 8) || overlaps_bytes(evk, key_bytes, a, c->dnum * limbs * 8))
        return fail(RF_EINVAL, "rf_keygen_switch: evk overlaps an input");
    Dev g(c->device);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    // NTT(err e_j) into polynomial 0 of every digit
    if ((rc = lift(c, e, nullptr, c->n, evk, 2 * limbs, 0, all, c->dnum, c->scheme == RF_BGV ? kLiftXT : 0, s)))
        return rc;
    if ((rc = launch_ntt(c, plain_batch(evk, 2 * limbs, all, c->dnum), true, s))) return rc;
    {
        ProfScope prof("client_keygen", s);
        hipLaunchKernelGGL(keygen_kernel, dim3(c->n / kCl, all, c->dnum), dim3(kCl), 0, s, evk, a, s_ntt, c->d_pc,
                           c->d_client, galois, c->log_n, c->L, c->K, c->alpha);
    }
    return check_launch("keygen");
}

extern "C" int rf_encrypt_sk(const rf_ctx *c, const int64_t *m, const int64_t *e, const uint64_t *a,
                             const uint64_t *s_ntt, uint64_t *out, uint32_t nl, void *stream) {
    if (!c || !m || !e || !a || !s_ntt || !out) return fail(RF_EINVAL, "rf_encrypt_sk: null argument");
    if (nl < 1 || nl > c->L) return fail(RF_ELEVEL, "rf_encrypt_sk: limb count out of range");
    if (c->scheme == RF_BFV && nl != c->L) return fail(RF_ELEVEL, "rf_encrypt_sk: BFV ciphertexts carry all L limbs");
    const size_t poly = (size_t)nl * c->n;
    if (overlaps_bytes(out, 2 * poly * 8, a, poly * 8) ||
        overlaps_bytes(out, 2 * poly * 8, s_ntt, (size_t)(c->L + c->K) * c->n * 8) ||
        overlaps_bytes(out, 2 * poly * 8, m, c->n * 8) || overlaps_bytes(out, 2 * poly * 8, e, c->n * 8))
        return fail(RF_EINVAL, "rf_encrypt_sk: out overlaps an input");
    Dev g(c->device);
    hipStream_t s = (hipStream_t)stream;
    uint64_t *c0 = out, *c1 = out + poly;
    int rc;
    if (c->scheme == RF_BFV) {
        // c1 <- Delta m + e; c0 <- INTT(NTT(a) s); c0 <- c1 - c0; c1 <- a
        if ((rc = lift(c, m, e, 0, c1, 0, 0, nl, 1, kLiftXDelta, s))) return rc;
        if (hipMemcpyAsync(c0, a, poly * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return fail(RF_EHIP, "rf_encrypt_sk: copy");
        if ((rc = launch_ntt(c, plain_batch(c0, 0, nl, 1), true, s))) return rc;
        if ((rc = launch_ewise(c, 4, c0, s_ntt, 0, c0, nl, 1, s))) return rc;
        if ((rc = launch_ntt(c, plain_batch(c0, 0, nl, 1), false, s))) return rc;
        if ((rc = launch_ewise(c, 1, c1, c0, 0, c0, nl, 1, s))) return rc;
    } else {
        // c0 <- NTT(m + err e) - a s
        if ((rc = lift(c, m, e, 0, c0, 0, 0, nl, 1, c->scheme == RF_BGV ? kLiftYT : 0, s))) return rc;
        if ((rc = launch_ntt(c, plain_batch(c0, 0, nl, 1), true, s))) return rc;
        {
            ProfScope prof("client_encrypt", s);
            hipLaunchKernelGGL(fma_s_kernel<true>, dim3(c->n / kCl, nl), dim3(kCl), 0, s, c0, a, s_ntt, c0, c->d_pc,
                               c->log_n);
        }
        if ((rc = check_launch("encrypt"))) return rc;
    }
    if (hipMemcpyAsync(c1, a, poly * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(RF_EHIP, "rf_encrypt_sk: copy");
    return RF_OK;
}

extern "C" int rf_decrypt(const rf_ctx *c, const uint64_t *ct, const uint64_t *s_ntt, uint64_t *out, uint32_t nl,
                          void *stream) {
    if (!c || !ct || !s_ntt || !out) return fail(RF_EINVAL, "rf_decrypt: null argument");
    if (nl < 1 || nl > c->L) return fail(RF_ELEVEL, "rf_decrypt: limb count out of range");
    if (c->scheme == RF_BFV && nl != c->L) return fail(RF_ELEVEL, "rf_decrypt: BFV ciphertexts carry all L limbs");
    const size_t poly = (size_t)nl * c->n;
    if (overlaps_bytes(out, poly * 8, ct, 2 * poly * 8)) return fail(RF_EINVAL, "rf_decrypt: out overlaps ct");
    Dev g(c->device);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if (c->scheme == RF_BFV) {
        // c0 + INTT(NTT(c1) s)
        if (hipMemcpyAsync(out, ct + poly, poly * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return fail(RF_EHIP, "rf_decrypt: copy");
        if ((rc = launch_ntt(c, plain_batch(out, 0, nl, 1), true, s))) return rc;
        if ((rc = launch_ewise(c, 4, out, s_ntt, 0, out, nl, 1, s))) return rc;
        if ((rc = launch_ntt(c, plain_batch(out, 0, nl, 1), false, s))) return rc;
        return launch_ewise(c, 0, out, ct, 0, out, nl, 1, s);
    }
    {
        ProfScope prof("client_decrypt", s);
        hipLaunchKernelGGL(fma_s_kernel<false>, dim3(c->n / kCl, nl), dim3(kCl), 0, s, ct, ct + poly, s_ntt, out,
                           c->d_pc, c->log_n);
    }
    if ((rc = check_launch("decrypt"))) return rc;
    return launch_ntt(c, plain_batch(out, 0, nl, 1), false, s);
}

extern "C" int rf_crt_centered(const rf_ctx *c, const uint64_t *x, double *out, uint32_t nl, double scale,
                               void *stream) {
    if (!c || !x || !out) return fail(RF_EINVAL, "rf_crt_centered: null argument");
    if (nl < 1 || nl > c->L) return fail(RF_ELEVEL, "rf_crt_centered: limb count out of range");
    if (nl > kMaxCrtLimbs) return fail(RF_EUNSUPPORTED, "rf_crt_centered: at most 32 limbs");
    if (!(scale > 0.0)) return fail(RF_EINVAL, "rf_crt_centered: scale must be positive");
    if (overlaps_bytes(out, (size_t)c->n * 8, x, (size_t)nl * c->n * 8))
        return fail(RF_EINVAL, "rf_crt_centered: out overlaps x");
    Dev g(c->device);
    hipStream_t s = (hipStream_t)stream;
    {
        ProfScope prof("client_crt", s);
        hipLaunchKernelGGL(crt_centered_kernel, dim3(c->n / kCrtThreads), dim3(kCrtThreads), 0, s, x, out, c->d_pc,
                           c->d_garner, c->L, nl, c->log_n, scale);
    }
    return check_launch("crt_centered");
}

extern "C" int rf_encode_ckks(const rf_ctx *c, const double *z, double scale, int64_t *m, void *ws, size_t ws_bytes,
                              void *stream) {
    if (!c || !z || !m) return fail(RF_EINVAL, "rf_encode_ckks: null argument");
    if (c->scheme != RF_CKKS) return fail(RF_EUNSUPPORTED, "rf_encode_ckks: CKKS contexts only");
    if (!(scale > 0.0)) return fail(RF_EINVAL, "rf_encode_ckks: scale must be positive");
    const size_t need = rf_workspace_bytes(c, RF_OP_ENCODE, 1);
    if (!ws || ws_bytes < need) return fail(RF_EWORKSPACE, "rf_encode_ckks: workspace too small");
    Dev g(c->device);
    hipStream_t s = (hipStream_t)stream;
    double2 *b0 = (double2 *)ws, *b1 = b0 + c->n;
    {
        ProfScope prof("client_encode", s);
        hipLaunchKernelGGL(encode_pre_kernel, dim3(c->n / 2 / kCl), dim3(kCl), 0, s, (const double2 *)z, b0,
                           c->d_slot_idx, c->n);
    }
    double2 *U = fft(c, b0, b1, -1, s);
    {
        ProfScope prof("client_encode", s);
        hipLaunchKernelGGL(encode_post_kernel, dim3(c->n / kCl), dim3(kCl), 0, s, U, m, (const double2 *)c->d_zeta,
                           c->n, scale / (double)c->n);
    }
    return check_launch("encode");
}

extern "C" int rf_decode_ckks(const rf_ctx *c, const double *x, double *z, void *ws, size_t ws_bytes, void *stream) {
    if (!c || !x || !z) return fail(RF_EINVAL, "rf_decode_ckks: null argument");
    if (c->scheme != RF_CKKS) return fail(RF_EUNSUPPORTED, "rf_decode_ckks: CKKS contexts only");
    const size_t need = rf_workspace_bytes(c, RF_OP_DECODE, 1);
    if (!ws || ws_bytes < need) return fail(RF_EWORKSPACE, "rf_decode_ckks: workspace too small");
    Dev g(c->device);
    hipStream_t s = (hipStream_t)stream;
    double2 *b0 = (double2 *)ws, *b1 = b0 + c->n;
    {
        ProfScope prof("client_decode", s);
        hipLaunchKernelGGL(decode_pre_kernel, dim3(c->n / kCl), dim3(kCl), 0, s, x, b0, (const double2 *)c->d_zeta);
    }
    double2 *V = fft(c, b0, b1, +1, s);
    {
        ProfScope prof("client_decode", s);
        hipLaunchKernelGGL(decode_post_kernel, dim3(c->n / 2 / kCl), dim3(kCl), 0, s, V, (double2 *)z,
                           c->d_slot_idx);
    }
    return check_launch("decode");
}
