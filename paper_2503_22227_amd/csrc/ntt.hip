// Negacyclic NTT / INTT kernels of single operations; the device code is in
// ntt_dev.hpp (shared with the batched kernels).
#include <hip/hip_runtime.h>

#include "ntt_dev.hpp"

namespace rf {

struct LimbView {
    const uint64_t *in;
    uint64_t *out;
    uint32_t g;  // prime index
};

__device__ __forceinline__ LimbView limb_view(const NttBatch &b, int log_n) {
    const uint32_t limb = blockIdx.y;
    const uint32_t poly = limb / b.per_poly, li = limb - poly * b.per_poly;
    LimbView v;
    v.g = b.pmap ? (uint32_t)b.pmap[li] : b.prime_base + li;
    v.in = b.in + (size_t)poly * b.in_poly_stride + ((size_t)li << log_n);
    v.out = b.out + (size_t)poly * b.out_poly_stride + ((size_t)li << log_n);
    return v;
}

template <int A, int B, bool FWD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesCols))) void ntt_cols_kernel(NttBatch b, const TwPair *__restrict__ tw_all,
                                                            const PrimeConst *__restrict__ pcs) {
    __shared__ uint64_t lds[(1 << A) * (kTile / (1 << A) + 1)];
    const LimbView v = limb_view(b, A + B);
    const PrimeConst pc = pcs[v.g];
    ntt_cols_unit<A, B, FWD>(lds, v.in, v.out, tw_all + ((size_t)v.g << (A + B)), pc, blockIdx.x);
}

template <int A, int B, bool FWD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesRows))) void ntt_rows_kernel(NttBatch b, const TwPair *__restrict__ tw_all,
                                                            const PrimeConst *__restrict__ pcs) {
    __shared__ uint64_t lds[(1 << B) * (kTile / (1 << B) + 1)];
    const LimbView v = limb_view(b, A + B);
    const PrimeConst pc = pcs[v.g];
    ntt_rows_unit<A, B, FWD>(lds, v.in, v.out, tw_all + ((size_t)v.g << (A + B)), pc, blockIdx.x);
}

// Last forward pass of NTT(conv) with the ModDown tail: limb (c, i) of conv
// [2][nl][N] -> out[c][i] = (ip[c][i] - NTT(conv)[c][i]) P^-1 (+ add_c[i]).
template <int A, int B>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesRows))) void ntt_rows_moddown_kernel(
    const uint64_t *conv, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs, const uint64_t *ip,
    const uint64_t *add0, const uint64_t *add1, uint64_t *out, const uint64_t *__restrict__ pinv, uint32_t nl,
    uint32_t K) {
    __shared__ uint64_t lds[(1 << B) * (kTile / (1 << B) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t c = blockIdx.y / nl, i = blockIdx.y - c * nl;
    const PrimeConst pc = pcs[i];
    const uint64_t *add = c == 0 ? add0 : add1;
    ModdownTailEpi epi{ip + (((size_t)c * (nl + K) + i) << LOGN), add ? add + ((size_t)i << LOGN) : nullptr,
                       out + (((size_t)c * nl + i) << LOGN), pinv[2 * i], pinv[2 * i + 1], pc.q};
    ntt_rows_unit_epi<A, B, true>(lds, conv + (((size_t)c * nl + i) << LOGN), tw_all + ((size_t)i << LOGN), pc,
                                  blockIdx.x, epi);
}

// Last forward pass of NTT(lift) with the rescale tail: limb (c, i) of lift
// [2][l][N] -> out[c][i] = (in[c][i] - NTT(lift)[c][i]) q_l^-1, l = nl - 1.
template <int A, int B>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesRows))) void ntt_rows_rescale_kernel(
    const uint64_t *lift, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs, const uint64_t *in,
    uint64_t *out, const uint64_t *__restrict__ tab, uint32_t nl, uint32_t L) {
    __shared__ uint64_t lds[(1 << B) * (kTile / (1 << B) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t l = nl - 1;
    const uint32_t c = blockIdx.y / l, i = blockIdx.y - c * l;
    const PrimeConst pc = pcs[i];
    const uint64_t *t = tab + ((size_t)l * L + i) * 3;
    RescaleTailEpi epi{in + (((size_t)c * nl + i) << LOGN), out + (((size_t)c * l + i) << LOGN), t[0], t[1], pc.q};
    ntt_rows_unit_epi<A, B, true>(lds, lift + (((size_t)c * l + i) << LOGN), tw_all + ((size_t)i << LOGN), pc,
                                  blockIdx.x, epi);
}

// Whole limb in one workgroup (N = 2^LOGN <= 4096).
template <int LOGN, bool FWD>
__global__ __launch_bounds__(kThreads) void ntt_single_kernel(NttBatch b, const TwPair *__restrict__ tw_all,
                                                              const PrimeConst *__restrict__ pcs) {
    constexpr int S = 1 << LOGN;
    constexpr int NT = S / kElems;
    __shared__ uint64_t lds[S];
    const LimbView v = limb_view(b, LOGN);
    const PrimeConst pc = pcs[v.g];
    const TwPair *tw = tw_all + ((size_t)v.g << LOGN);
    if (threadIdx.x < NT) {
#pragma unroll
        for (int r = 0; r < kElems; ++r) lds[threadIdx.x + r * NT] = v.in[threadIdx.x + r * NT];
    }
    __syncthreads();
    ntt_rounds<LOGN, FWD, !FWD>(lds, 1, 0, threadIdx.x < NT ? threadIdx.x : 0, 1u, tw, pc);
    if (threadIdx.x < NT) {
        const uint64_t q2 = 2 * pc.q;
#pragma unroll
        for (int r = 0; r < kElems; ++r) {
            uint64_t x = lds[threadIdx.x + r * NT];
            x = FWD ? csub(csub(x, q2), pc.q) : csub(x, pc.q);
            v.out[threadIdx.x + r * NT] = x;
        }
    }
}

template <int A, int B>
static void launch_two_pass(const rf_ctx *c, const NttBatch &b, bool forward, hipStream_t s) {
    const uint32_t limbs = b.per_poly * b.n_polys;
    const dim3 block(kThreads);
    const dim3 grid_cols((1u << B) / (kTile >> A), limbs);
    const dim3 grid_rows((1u << A) / (kTile >> B), limbs);
    NttBatch b2 = b;
    b2.in = b.out;
    b2.in_poly_stride = b.out_poly_stride;
    if (forward) {
        {
            ProfScope p("ntt_fwd_cols", s);
            hipLaunchKernelGGL((ntt_cols_kernel<A, B, true>), grid_cols, block, 0, s, b, c->d_tw_fwd, c->d_pc);
        }
        ProfScope p("ntt_fwd_rows", s);
        hipLaunchKernelGGL((ntt_rows_kernel<A, B, true>), grid_rows, block, 0, s, b2, c->d_tw_fwd, c->d_pc);
    } else {
        {
            ProfScope p("ntt_inv_rows", s);
            hipLaunchKernelGGL((ntt_rows_kernel<A, B, false>), grid_rows, block, 0, s, b, c->d_tw_inv, c->d_pc);
        }
        ProfScope p("ntt_inv_cols", s);
        hipLaunchKernelGGL((ntt_cols_kernel<A, B, false>), grid_cols, block, 0, s, b2, c->d_tw_inv, c->d_pc);
    }
}

template <int A, int B>
static void launch_cols_fwd(const rf_ctx *c, const NttBatch &b, hipStream_t s) {
    ProfScope p("ntt_fwd_cols", s);
    hipLaunchKernelGGL((ntt_cols_kernel<A, B, true>), dim3((1u << B) / (kTile >> A), b.per_poly * b.n_polys),
                       dim3(kThreads), 0, s, b, c->d_tw_fwd, c->d_pc);
}

int launch_ntt_fwd_moddown(const rf_ctx *c, uint64_t *conv, const uint64_t *ip, const uint64_t *add0,
                           const uint64_t *add1, uint64_t *out, uint32_t nl, hipStream_t s) {
    const uint64_t stride = (uint64_t)nl * c->n;
    NttBatch b{conv, conv, stride, stride, nl, 2, 0, nullptr};
    const uint64_t *pinv = c->d_moddown + moddown_pinv_off(c);
    const dim3 g(c->n / kTile, 2 * nl);
#define RF_MD(A, B)                                                                                             \
    {                                                                                                            \
        launch_cols_fwd<A, B>(c, b, s);                                                                          \
        ProfScope p("ntt_fwd_rows_moddown", s);                                                                  \
        hipLaunchKernelGGL((ntt_rows_moddown_kernel<A, B>), g, dim3(kThreads), 0, s, conv, c->d_tw_fwd, c->d_pc, ip, \
                           add0, add1, out, pinv, nl, c->K);                                                     \
    }
    switch (c->log_n) {
        case 13: RF_MD(7, 6) break;
        case 14: RF_MD(7, 7) break;
        case 15: RF_MD(8, 7) break;
        case 16: RF_MD(8, 8) break;
        default: return fail(RF_EUNSUPPORTED, "fused ModDown NTT: ring degree");
    }
#undef RF_MD
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RF_EHIP, std::string("NTT launch: ") + hipGetErrorString(e));
    return RF_OK;
}

int launch_ntt_fwd_rescale(const rf_ctx *c, uint64_t *lift, const uint64_t *in, uint64_t *out, uint32_t nl,
                           hipStream_t s) {
    const uint32_t l = nl - 1;
    const uint64_t stride = (uint64_t)l * c->n;
    NttBatch b{lift, lift, stride, stride, l, 2, 0, nullptr};
    const dim3 g(c->n / kTile, 2 * l);
#define RF_RS(A, B)                                                                                              \
    {                                                                                                            \
        launch_cols_fwd<A, B>(c, b, s);                                                                          \
        ProfScope p("ntt_fwd_rows_rescale", s);                                                                  \
        hipLaunchKernelGGL((ntt_rows_rescale_kernel<A, B>), g, dim3(kThreads), 0, s, lift, c->d_tw_fwd, c->d_pc, in, \
                           out, c->d_rescale, nl, c->L);                                                         \
    }
    switch (c->log_n) {
        case 13: RF_RS(7, 6) break;
        case 14: RF_RS(7, 7) break;
        case 15: RF_RS(8, 7) break;
        case 16: RF_RS(8, 8) break;
        default: return fail(RF_EUNSUPPORTED, "fused rescale NTT: ring degree");
    }
#undef RF_RS
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RF_EHIP, std::string("NTT launch: ") + hipGetErrorString(e));
    return RF_OK;
}

int launch_ntt(const rf_ctx *c, const NttBatch &b, bool forward, hipStream_t s) {
    const uint32_t limbs = b.per_poly * b.n_polys;
    if (limbs == 0) return RF_OK;
    if (limbs > 65535) return fail(RF_EUNSUPPORTED, "too many limbs in one NTT launch");
    switch (c->log_n) {
        case 12: {
            ProfScope p(forward ? "ntt_fwd_single" : "ntt_inv_single", s);
            if (forward)
                hipLaunchKernelGGL((ntt_single_kernel<12, true>), dim3(1, limbs), dim3(kThreads), 0, s, b,
                                   c->d_tw_fwd, c->d_pc);
            else
                hipLaunchKernelGGL((ntt_single_kernel<12, false>), dim3(1, limbs), dim3(kThreads), 0, s, b,
                                   c->d_tw_inv, c->d_pc);
            break;
        }
        case 13: launch_two_pass<7, 6>(c, b, forward, s); break;
        case 14: launch_two_pass<7, 7>(c, b, forward, s); break;
        case 15: launch_two_pass<8, 7>(c, b, forward, s); break;
        case 16: launch_two_pass<8, 8>(c, b, forward, s); break;
        default: return fail(RF_EUNSUPPORTED, "ring degree");
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RF_EHIP, std::string("NTT launch: ") + hipGetErrorString(e));
    return RF_OK;
}

}  // namespace rf
