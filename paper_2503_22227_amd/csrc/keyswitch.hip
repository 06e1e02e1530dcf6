// Element-wise and base-conversion kernels of HMult+Relin, HRotate and rescale.
//
// All kernels are one thread per coefficient of one limb (grid.x covers N in
// blocks of 256, grid.y enumerates limbs or digits), read and write whole
// 128-byte lines per wavefront, and take their per-prime constants from the
// context tables; indices that are uniform across a workgroup (limb, digit,
// target prime) come from blockIdx so the compiler keeps them in SGPRs and
// reads the constants with scalar loads.
//
// Key switching is the hybrid method (the paper's relinearize/rotate rows do
// not name one):
//   ModUp        y_i = [x_i (Q_j/q_i)^-1]_{q_i},  out_m = sum_{i in D_j} y_i [Q_j/q_i]_m
//   inner prod.  (sum_j ext_j evk_{j,0}, sum_j ext_j evk_{j,1}) on Q_l u P
//   ModDown      y_p = [x_p (P/p)^-1]_p taken in (-p/2, p/2],
//                conv_i = sum_p y_p [P/p]_{q_i}, out_i = (x_i - NTT(conv_i)) P^-1
// Sums of products are accumulated exactly in 128 bits and reduced once.
#include <hip/hip_runtime.h>

#include "ks_dev.hpp"

namespace rf {

__global__ __launch_bounds__(kEw) void tensor_kernel(const uint64_t *__restrict__ a, const uint64_t *__restrict__ b,
                                                     uint64_t *__restrict__ d01, uint64_t *__restrict__ d2,
                                                     const PrimeConst *__restrict__ pcs, uint32_t log_n, uint32_t nl,
                                                     const uint32_t *pmap) {
    tensor_unit(a, b, d01, d2, pcs, log_n, nl, pmap, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kEw) void behz_extend_kernel(const uint64_t *a, const uint64_t *b, uint64_t *ext,
                                                          const PrimeConst *__restrict__ pcs,
                                                          const uint64_t *__restrict__ tab, BehzLayout o, uint32_t kb,
                                                          uint32_t log_n) {
    behz_extend_unit(a, b, ext, pcs, tab, o, kb, log_n, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kEw) void behz_floor_kernel(const uint64_t *tens, uint64_t *f,
                                                         const PrimeConst *__restrict__ pcs,
                                                         const uint64_t *__restrict__ tab, BehzLayout o, uint32_t kb,
                                                         uint32_t log_n) {
    behz_floor_unit(tens, f, pcs, tab, o, kb, log_n, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kEw) void behz_sk_kernel(const uint64_t *f, uint64_t *out01, uint64_t *out2,
                                                      const PrimeConst *__restrict__ pcs,
                                                      const uint64_t *__restrict__ tab, BehzLayout o, uint32_t kb,
                                                      uint32_t log_n) {
    behz_sk_unit(f, out01, out2, pcs, tab, o, kb, log_n, blockIdx.x, blockIdx.y);
}

template <bool SCALED, int CH>
__global__ __launch_bounds__(kEw) void modup_bconv_kernel(const uint64_t *__restrict__ x, uint64_t *__restrict__ ext,
                                                          const PrimeConst *__restrict__ pcs,
                                                          const uint64_t *__restrict__ tab, size_t tab_stride,
                                                          uint32_t log_n, uint32_t nl, uint32_t L, uint32_t K,
                                                          uint32_t alpha) {
    modup_bconv_unit<SCALED, CH>(x, ext, pcs, tab, tab_stride, log_n, nl, L, K, alpha, blockIdx.x, blockIdx.y);
}

template <int V>
__global__ __launch_bounds__(kEw) void inner_product_kernel(const uint64_t *__restrict__ d,
                                                            const uint64_t *__restrict__ ext,
                                                            const uint64_t *__restrict__ evk,
                                                            uint64_t *__restrict__ ip,
                                                            const PrimeConst *__restrict__ pcs, uint32_t log_n,
                                                            uint32_t nl, uint32_t L, uint32_t K, uint32_t alpha,
                                                            IpFold fold) {
    inner_product_unit<V>(d, ext, evk, ip, pcs, log_n, nl, L, K, alpha, blockIdx.x, blockIdx.y, fold);
}

__global__ __launch_bounds__(kEw) void moddown_bconv_kernel(const uint64_t *__restrict__ ip, uint64_t *__restrict__ conv,
                                                            const PrimeConst *__restrict__ pcs,
                                                            const uint64_t *__restrict__ tab, uint32_t log_n,
                                                            uint32_t nl, uint32_t L, uint32_t K) {
    moddown_bconv_unit(ip, conv, pcs, tab, log_n, nl, L, K, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kEw) void moddown_tail_kernel(const uint64_t *__restrict__ ip,
                                                           const uint64_t *__restrict__ conv, const uint64_t *add0,
                                                           const uint64_t *add1, uint64_t *out,
                                                           const PrimeConst *__restrict__ pcs,
                                                           const uint64_t *__restrict__ pinv, uint32_t log_n,
                                                           uint32_t nl, uint32_t K) {
    moddown_tail_unit(ip, conv, add0, add1, out, pcs, pinv, log_n, nl, K, blockIdx.x, blockIdx.y);
}

template <bool KEEP_T>
__global__ __launch_bounds__(kEw) void rescale_lift_kernel(const uint64_t *__restrict__ last, uint64_t *__restrict__ lift,
                                                           const PrimeConst *__restrict__ pcs,
                                                           const uint64_t *__restrict__ tab, uint32_t log_n,
                                                           uint32_t nl, uint32_t L) {
    rescale_lift_unit<KEEP_T>(last, lift, pcs, tab, log_n, nl, L, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kEw) void rescale_tail_kernel(const uint64_t *__restrict__ in, const uint64_t *lift,
                                                           uint64_t *out, const PrimeConst *__restrict__ pcs,
                                                           const uint64_t *__restrict__ tab, uint32_t log_n,
                                                           uint32_t nl, uint32_t L) {
    rescale_tail_unit(in, lift, out, pcs, tab, log_n, nl, L, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kEw) void automorphism_kernel(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                           uint32_t galois, uint32_t log_n) {
    automorphism_unit(in, out, galois, log_n, blockIdx.x, blockIdx.y);
}

template <int OP>
__global__ __launch_bounds__(kEw) void ewise_kernel(const uint64_t *a, const uint64_t *b, int64_t k, uint64_t *out,
                                                    const PrimeConst *__restrict__ pcs, uint32_t log_n, uint32_t nl) {
    ewise_unit<OP>(a, b, k, out, pcs, log_n, nl, blockIdx.x, blockIdx.y);
}

static int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return RF_OK;
}

static dim3 ew_grid(const rf_ctx *c, uint32_t y) { return dim3(c->n / kEw, y); }

int launch_tensor(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *d01, uint64_t *d2, uint32_t nl,
                  hipStream_t s) {
    ProfScope prof("tensor", s);
    hipLaunchKernelGGL(tensor_kernel, ew_grid(c, nl), dim3(kEw), 0, s, a, b, d01, d2, c->d_pc, c->log_n, nl,
                       (const uint32_t *)nullptr);
    return check_launch("tensor");
}

int launch_tensor_map(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *d01, uint64_t *d2,
                      uint32_t nl, const uint32_t *pmap, hipStream_t s) {
    ProfScope prof("tensor", s);
    hipLaunchKernelGGL(tensor_kernel, ew_grid(c, nl), dim3(kEw), 0, s, a, b, d01, d2, c->d_pc, c->log_n, nl, pmap);
    return check_launch("tensor");
}

int launch_behz_extend(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *ext, hipStream_t s) {
    ProfScope prof("behz_extend", s);
    hipLaunchKernelGGL(behz_extend_kernel, ew_grid(c, 4 * behz_groups(c->nb + 1)), dim3(kEw), 0, s, a, b, ext, c->d_pc,
                       c->d_behz, c->behz,
                       c->L + c->K, c->log_n);
    return check_launch("behz_extend");
}

int launch_behz_floor_sk(const rf_ctx *c, const uint64_t *tens, uint64_t *f, uint64_t *out01, uint64_t *out2,
                         hipStream_t s) {
    const uint32_t kb = c->L + c->K;
    {
        ProfScope prof("behz_floor", s);
        hipLaunchKernelGGL(behz_floor_kernel, ew_grid(c, 3 * behz_groups(c->nb + 1)), dim3(kEw), 0, s, tens, f,
                           c->d_pc, c->d_behz, c->behz, kb, c->log_n);
    }
    ProfScope prof("behz_sk", s);
    hipLaunchKernelGGL(behz_sk_kernel, ew_grid(c, 3 * behz_groups(c->L)), dim3(kEw), 0, s, f, out01, out2, c->d_pc,
                       c->d_behz, c->behz, kb, c->log_n);
    return check_launch("behz_floor_sk");
}

int launch_modup_bconv(const rf_ctx *c, const uint64_t *x, uint64_t *ext, uint32_t nl, hipStream_t s, bool scaled,
                       uint32_t chunk) {
    const uint32_t dn = (nl + c->alpha - 1) / c->alpha;
    if (chunk != 4 && chunk != 8 && chunk != 16) return fail(RF_EINVAL, "modup_bconv: chunk of 4, 8 or 16 limbs");
    ProfScope prof("modup_bconv", s);
    const dim3 grid = ew_grid(c, dn * modup_chunks(nl, c->K, chunk));
#define RF_MU(SC, CH)                                                                                            \
    hipLaunchKernelGGL((modup_bconv_kernel<SC, CH>), grid, dim3(kEw), 0, s, x, ext, c->d_pc, c->d_modup,          \
                       c->modup_stride, c->log_n, nl, c->L, c->K, c->alpha)
    if (scaled) {
        if (chunk == 4) RF_MU(true, 4);
        else if (chunk == 16) RF_MU(true, 16);
        else RF_MU(true, 8);
    } else {
        if (chunk == 4) RF_MU(false, 4);
        else if (chunk == 16) RF_MU(false, 16);
        else RF_MU(false, 8);
    }
#undef RF_MU
    return check_launch("modup_bconv");
}

int launch_inner_product(const rf_ctx *c, const uint64_t *d, const uint64_t *ext, const uint64_t *evk, uint64_t *ip,
                         uint32_t nl, hipStream_t s, const IpFold *fold) {
    ProfScope prof("inner_product", s);
    IpFold f;
    if (fold) {
        f = *fold;
        f.pinv = c->d_moddown + moddown_pinv_off(c);
    }
    hipLaunchKernelGGL(inner_product_kernel<kIpVec>, dim3(c->n / (kEw * kIpVec), nl + c->K), dim3(kEw), 0, s, d, ext,
                       evk, ip, c->d_pc, c->log_n, nl, c->L, c->K, c->alpha, f);
    return check_launch("inner_product");
}

int launch_moddown_bconv(const rf_ctx *c, const uint64_t *ip, uint64_t *conv, uint32_t nl, hipStream_t s) {
    ProfScope prof("moddown_bconv", s);
    const uint64_t *tab = c->scheme == RF_BGV ? c->d_moddown_t : c->d_moddown;
    hipLaunchKernelGGL(moddown_bconv_kernel, ew_grid(c, 2 * moddown_chunks(nl)), dim3(kEw), 0, s, ip, conv, c->d_pc, tab,
                       c->log_n, nl, c->L, c->K);
    return check_launch("moddown_bconv");
}

int launch_moddown_tail(const rf_ctx *c, const uint64_t *ip, const uint64_t *conv, const uint64_t *add0,
                        const uint64_t *add1, uint64_t *out, uint32_t nl, hipStream_t s) {
    ProfScope prof("moddown_tail", s);
    hipLaunchKernelGGL(moddown_tail_kernel, ew_grid(c, 2 * nl), dim3(kEw), 0, s, ip, conv, add0, add1, out, c->d_pc,
                       c->d_moddown + moddown_pinv_off(c), c->log_n, nl, c->K);
    return check_launch("moddown_tail");
}

int launch_rescale_lift(const rf_ctx *c, const uint64_t *last, uint64_t *lift, uint32_t nl, bool keep_t,
                        hipStream_t s) {
    ProfScope prof("rescale_lift", s);
    if (keep_t)
        hipLaunchKernelGGL(rescale_lift_kernel<true>, ew_grid(c, 2 * (nl - 1)), dim3(kEw), 0, s, last, lift, c->d_pc,
                           c->d_rescale, c->log_n, nl, c->L);
    else
        hipLaunchKernelGGL(rescale_lift_kernel<false>, ew_grid(c, 2 * (nl - 1)), dim3(kEw), 0, s, last, lift,
                           c->d_pc, c->d_rescale, c->log_n, nl, c->L);
    return check_launch("rescale_lift");
}

int launch_rescale_tail(const rf_ctx *c, const uint64_t *in, const uint64_t *lift, uint64_t *out, uint32_t nl,
                        hipStream_t s) {
    ProfScope prof("rescale_tail", s);
    hipLaunchKernelGGL(rescale_tail_kernel, ew_grid(c, 2 * (nl - 1)), dim3(kEw), 0, s, in, lift, out, c->d_pc,
                       c->d_rescale, c->log_n, nl, c->L);
    return check_launch("rescale_tail");
}

int launch_automorphism(const rf_ctx *c, const uint64_t *in, uint64_t *out, uint32_t galois, uint32_t nl,
                        uint32_t n_polys, hipStream_t s) {
    ProfScope prof("automorphism", s);
    hipLaunchKernelGGL(automorphism_kernel, ew_grid(c, nl * n_polys), dim3(kEw), 0, s, in, out, galois, c->log_n);
    return check_launch("automorphism");
}

int launch_ewise(const rf_ctx *c, int op, const uint64_t *a, const uint64_t *b, int64_t k, uint64_t *out,
                 uint32_t nl, uint32_t n_polys, hipStream_t s) {
    ProfScope prof("elementwise", s);
    const dim3 g = ew_grid(c, nl * n_polys);
    switch (op) {
        case 0: hipLaunchKernelGGL(ewise_kernel<0>, g, dim3(kEw), 0, s, a, b, k, out, c->d_pc, c->log_n, nl); break;
        case 1: hipLaunchKernelGGL(ewise_kernel<1>, g, dim3(kEw), 0, s, a, b, k, out, c->d_pc, c->log_n, nl); break;
        case 2: hipLaunchKernelGGL(ewise_kernel<2>, g, dim3(kEw), 0, s, a, b, k, out, c->d_pc, c->log_n, nl); break;
        case 3: hipLaunchKernelGGL(ewise_kernel<3>, g, dim3(kEw), 0, s, a, b, k, out, c->d_pc, c->log_n, nl); break;
        case 4: hipLaunchKernelGGL(ewise_kernel<4>, g, dim3(kEw), 0, s, a, b, k, out, c->d_pc, c->log_n, nl); break;
        default: return fail(RF_EINVAL, "unknown element-wise op");
    }
    return check_launch("elementwise");
}

}  // namespace rf
