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

// grid.y runs over the limbs with the polynomials interleaved (limb li of every
// polynomial, then limb li + 1, ...): the tiles that share a prime's twiddles
// are launched back to back, 16 workgroups apart at N = 2^16, which places them
// on the same XCD (workgroups are dealt to the 8 XCDs in turn), so the second
// reads the twiddles from that XCD's L2.
//
// The limb index is uniform across the workgroup: held in a scalar register, so
// the prime map and the prime's constants are read with scalar loads instead of
// a vector load whose latency would delay the tile's own loads.
__device__ __forceinline__ LimbView limb_view(const NttBatch &b, int log_n, uint32_t limb) {
    const uint32_t li = __builtin_amdgcn_readfirstlane(limb / b.n_polys), poly = limb - li * b.n_polys;
    LimbView v;
    v.g = b.pmap ? b.pmap[li] : b.prime_base + li;
    v.in = b.in + (size_t)poly * b.in_poly_stride + ((size_t)li << log_n);
    v.out = b.out + (size_t)poly * b.out_poly_stride + ((size_t)li << log_n);
    return v;
}

template <int A, int B, bool FWD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesCols))) void ntt_cols_kernel(NttBatch b, const TwPair *__restrict__ tw_all,
                                                            const PrimeConst *__restrict__ pcs) {
    __shared__ uint64_t lds[(1 << A) * (kTile / (1 << A) + 1)];
    const uint32_t tile = blockIdx.x;
    const LimbView v = limb_view(b, A + B, blockIdx.y);
    const PrimeConst pc = pcs[v.g];
    ntt_cols_unit<A, B, FWD>(lds, v.in, v.out, tw_all + ((size_t)v.g << (A + B)), pc, tile);
}

template <int A, int B, bool FWD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesRows))) void ntt_rows_kernel(NttBatch b, const TwPair *__restrict__ tw_all,
                                                            const PrimeConst *__restrict__ pcs) {
    __shared__ uint64_t lds[(1 << B) * (kTile / (1 << B) + 1)];
    const uint32_t tile = blockIdx.x;
    const LimbView v = limb_view(b, A + B, blockIdx.y);
    const PrimeConst pc = pcs[v.g];
    ntt_rows_unit<A, B, FWD>(lds, v.in, v.out, tw_all + ((size_t)v.g << (A + B)), pc, tile);
}

// Prologue of the first pass of NTT(conv): the ModDown conversion of target i
// of polynomial c from the K P-limbs of ip[c] ([2][nl + K][N]).
template <int KP, int LOGN>
__device__ __forceinline__ ModdownPro<KP> moddown_pro(const uint64_t *ip, const PrimeConst *__restrict__ pcs,
                                                      const PrimeConst &pc, const uint64_t *__restrict__ cross,
                                                      const uint64_t *__restrict__ negp, uint32_t c, uint32_t i,
                                                      uint32_t nl, uint32_t L, uint32_t K) {
    ModdownPro<KP> pro;
    pro.src = ip + (((size_t)c * (nl + K) + nl) << LOGN);
    pro.stride = (size_t)1 << LOGN;
    pro.K = K;
#pragma unroll
    for (int a = 0; a < KP; ++a) {
        pro.half[a] = a < (int)K ? pcs[L + a].q >> 1 : 0;
        pro.cross[a] = a < (int)K ? cross[(size_t)i * K + a] : 0;
    }
    pro.negp = negp[i];
    pro.q = pc.q;
    pro.r64 = pc.r64;
    pro.r64_p = pc.r64_p;
    pro.one_p = pc.one_p;
    return pro;
}

// Prologue of the first pass of NTT(lift): the lift of polynomial c's last
// limb (last [2][N], dropped prime l = nl - 1) into prime i.
template <bool KEEP_T, int LOGN>
__device__ __forceinline__ LiftPro<KEEP_T> lift_pro(const uint64_t *last, const PrimeConst *__restrict__ pcs,
                                                    const PrimeConst &pc, const uint64_t *__restrict__ tab,
                                                    uint32_t c, uint32_t i, uint32_t nl, uint32_t L) {
    const uint32_t l = nl - 1;
    const PrimeConst pl = pcs[l];
    LiftPro<KEEP_T> pro;
    pro.last = last + ((size_t)c << LOGN);
    pro.ql = pl.q;
    pro.ql_half = pl.q >> 1;
    pro.tinv = pl.tinv;
    pro.tinv_p = pl.tinv_p;
    pro.q = pc.q;
    pro.one_p = pc.one_p;
    pro.corr = tab[((size_t)l * L + i) * 3 + 2];
    pro.tmod = pc.tmod;
    pro.tmod_p = pc.tmod_p;
    return pro;
}

// First forward pass of NTT(conv) with the ModDown base conversion as its
// prologue: limb (c, i) of conv [2][nl][N] from the K P-limbs of ip[c].
template <int A, int B, int KP>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(KP == 8 ? kNttWavesCols : kNttWavesFused))) void ntt_cols_moddown_kernel(
    const uint64_t *ip, uint64_t *conv, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs,
    const uint64_t *__restrict__ cross, const uint64_t *__restrict__ negp, uint32_t nl, uint32_t L, uint32_t K) {
    __shared__ uint64_t lds[(1 << A) * (kTile / (1 << A) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t tile = blockIdx.x;
    const uint32_t c = blockIdx.y & 1, i = blockIdx.y >> 1;  // polynomials interleaved
    const PrimeConst pc = pcs[i];
    const ModdownPro<KP> pro = moddown_pro<KP, LOGN>(ip, pcs, pc, cross, negp, c, i, nl, L, K);
    ntt_cols_unit_pro<A, B, true, B == 8>(lds, conv + (((size_t)c * nl + i) << LOGN), tw_all + ((size_t)i << LOGN), pc,
                                  tile, pro);
}

// First forward pass of NTT(lift) with the rescale lift as its prologue: limb
// (c, i) of lift [2][l][N], l = nl - 1, from the last limb last[c].
template <int A, int B, bool KEEP_T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesFused))) void ntt_cols_lift_kernel(
    const uint64_t *last, uint64_t *lift, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs,
    const uint64_t *__restrict__ tab, uint32_t nl, uint32_t L) {
    __shared__ uint64_t lds[(1 << A) * (kTile / (1 << A) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t l = nl - 1;
    const uint32_t tile = blockIdx.x;
    const uint32_t c = blockIdx.y & 1, i = blockIdx.y >> 1;  // polynomials interleaved
    const PrimeConst pc = pcs[i];
    const LiftPro<KEEP_T> pro = lift_pro<KEEP_T, LOGN>(last, pcs, pc, tab, c, i, nl, L);
    ntt_cols_unit_pro<A, B, true, B == 8>(lds, lift + (((size_t)c * l + i) << LOGN), tw_all + ((size_t)i << LOGN), pc,
                                  tile, pro);
}

// Last forward pass of NTT(conv) with the ModDown tail: limb (c, i) of conv
// [2][nl][N] -> out[c][i] = (ip[c][i] - NTT(conv)[c][i]) P^-1 (+ add_c[i]).
template <int A, int B>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(B == 8 ? kNttWavesFused : kNttWavesCols))) void ntt_rows_moddown_kernel(
    const uint64_t *conv, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs, const uint64_t *ip,
    uint64_t *out, const uint64_t *__restrict__ pinv, uint32_t nl, uint32_t K) {
    __shared__ uint64_t lds[(1 << B) * (kTile / (1 << B) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t tile = blockIdx.x;
    const uint32_t c = blockIdx.y & 1, i = blockIdx.y >> 1;  // polynomials interleaved
    const PrimeConst pc = pcs[i];
    const ModdownFoldEpi epi{ip + (((size_t)c * (nl + K) + i) << LOGN), out + (((size_t)c * nl + i) << LOGN),
                             pinv[2 * i], pinv[2 * i + 1], pc.q};
    ntt_rows_unit_epi<A, B, true, B == 8>(lds, conv + (((size_t)c * nl + i) << LOGN), tw_all + ((size_t)i << LOGN), pc,
                                  tile, epi);
}

// First inverse pass of INTT(d2) with d2 = a1 b1 as its prologue: limb i of a, b
// ([2][nl][N], NTT domain); the row pass goes to dc [nl][N].
template <int A, int B>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesRows))) void ntt_inv_rows_tensor_kernel(
    const uint64_t *a, const uint64_t *b, uint64_t *dc, const TwPair *__restrict__ tw_all,
    const PrimeConst *__restrict__ pcs, uint32_t nl) {
    __shared__ uint64_t lds[(1 << B) * (kTile / (1 << B) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t tile = blockIdx.x, i = blockIdx.y;
    const PrimeConst pc = pcs[i];
    const size_t li = (size_t)i << LOGN, poly = (size_t)nl << LOGN;
    const TensorPro pro{a + poly + li, b + poly + li, pc.q, pc.r64, pc.r64_p, pc.one_p};
    ntt_rows_unit_pe<A, B, false>(lds, pro, tw_all + li, pc, tile, StoreEpi{dc + li});
}

// First inverse pass of INTT(sigma_g(a1)) with the automorphism as its
// prologue: limb i of a1 ([nl][N], NTT domain) permuted, row pass into dc.
template <int A, int B>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesRows))) void ntt_inv_rows_gather_kernel(
    const uint64_t *a1, uint64_t *dc, uint32_t galois, const TwPair *__restrict__ tw_all,
    const PrimeConst *__restrict__ pcs) {
    __shared__ uint64_t lds[(1 << B) * (kTile / (1 << B) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t tile = blockIdx.x, i = blockIdx.y;
    const PrimeConst pc = pcs[i];
    const size_t li = (size_t)i << LOGN;
    const GatherPro pro{a1 + li, galois, (uint32_t)LOGN};
    ntt_rows_unit_pe<A, B, false>(lds, pro, tw_all + li, pc, tile, StoreEpi{dc + li});
}

// Last forward pass of NTT(lift) with the rescale tail: limb (c, i) of lift
// [2][l][N] -> out[c][i] = (in[c][i] - NTT(lift)[c][i]) q_l^-1, l = nl - 1.
template <int A, int B>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(B == 8 ? kNttWavesFused : kNttWavesCols))) void ntt_rows_rescale_kernel(
    const uint64_t *lift, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs, const uint64_t *in,
    uint64_t *out, const uint64_t *__restrict__ tab, uint32_t nl, uint32_t L) {
    __shared__ uint64_t lds[(1 << B) * (kTile / (1 << B) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t l = nl - 1;
    const uint32_t tile = blockIdx.x;
    const uint32_t c = blockIdx.y & 1, i = blockIdx.y >> 1;  // polynomials interleaved
    const PrimeConst pc = pcs[i];
    const uint64_t *t = tab + ((size_t)l * L + i) * 3;
    RescaleTailEpi epi{in + (((size_t)c * nl + i) << LOGN), out + (((size_t)c * l + i) << LOGN), t[0], t[1], pc.q};
    ntt_rows_unit_epi<A, B, true, B == 8>(lds, lift + (((size_t)c * l + i) << LOGN), tw_all + ((size_t)i << LOGN), pc,
                                  tile, epi);
}

// Whole limb in one workgroup (N = 2^LOGN <= 4096).
template <int LOGN, bool FWD>
__global__ __launch_bounds__(kThreads) void ntt_single_kernel(NttBatch b, const TwPair *__restrict__ tw_all,
                                                              const PrimeConst *__restrict__ pcs) {
    constexpr int S = 1 << LOGN;
    constexpr int NT = S / kElems;
    __shared__ uint64_t lds[S];
    const LimbView v = limb_view(b, LOGN, blockIdx.y);
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

// A pass of a launch with few limbs (ntt_cols_small / ntt_rows_small): one
// workgroup per TILE residues of a limb, E residues per thread.
// Tile of a small column pass.  Its U = TILE / 2^A columns are narrower than
// a 128-byte line (G = 16 / U tiles share each line of a row), and workgroups
// are dealt to the 8 XCDs in turn, each with its own L2: dispatch order
// w = blockIdx.x is mapped so that the G tiles of one line group go to the
// same XCD one after another (w, w + 8, ...), and the line is read from HBM
// once instead of G times.  Identity when the grid is not a multiple of 8 G.
template <int TILE, int A>
__device__ __forceinline__ int xcd_grouped_tile() {
    constexpr int U = TILE >> A, G = U >= 16 ? 1 : 16 / U;
    const int w = blockIdx.x;
    if (G == 1 || gridDim.x % (8 * G) != 0) return w;
    const int x = w & 7, r = w >> 3;
    return ((r / G) * 8 + x) * G + r % G;
}

template <int A, int B, bool FWD, bool COLS, int TILE, int E>
__global__ __launch_bounds__(TILE / E) void ntt_small_kernel(NttBatch b, const TwPair *__restrict__ tw_all,
                                                             const PrimeConst *__restrict__ pcs) {
    constexpr int S = COLS ? (1 << A) : (1 << B);
    __shared__ uint64_t lds[S * (TILE / S + 1)];
    const LimbView v = limb_view(b, A + B, blockIdx.y);
    const PrimeConst pc = pcs[v.g];
    const TwPair *tw = tw_all + ((size_t)v.g << (A + B));
    if constexpr (COLS) ntt_cols_small<A, B, FWD, TILE, E>(lds, v.in, v.out, tw, pc, xcd_grouped_tile<TILE, A>());
    else ntt_rows_small<A, B, FWD, TILE, E>(lds, v.in, v.out, tw, pc, blockIdx.x);
}

// Default residues per thread of the few-limb passes (4 measured faster than 8:
// the 8-limb inverse passes at N = 2^16 took 10.3 / 10.9 us against 10.8 / 12.7
// us); rf_tuning picks per level.
constexpr int kSmallE = 4;

// The passes of the fused ModDown, rescale and first-INTT launches on small
// tiles (the same prologues and epilogues as their 4096-tile kernels; natural
// twiddle tables, strict butterflies in both passes of a limb).
template <int A, int B, int TILE, int KP>
__global__ __launch_bounds__(TILE / kSmallE) void ntt_small_cols_moddown_kernel(
    const uint64_t *ip, uint64_t *conv, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs,
    const uint64_t *__restrict__ cross, const uint64_t *__restrict__ negp, uint32_t nl, uint32_t L, uint32_t K) {
    __shared__ uint64_t lds[(1 << A) * (TILE / (1 << A) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t c = blockIdx.y & 1, i = blockIdx.y >> 1;
    const PrimeConst pc = pcs[i];
    const ModdownPro<KP> pro = moddown_pro<KP, LOGN>(ip, pcs, pc, cross, negp, c, i, nl, L, K);
    ntt_cols_small_pro<A, B, true, TILE, kSmallE>(lds, pro, conv + (((size_t)c * nl + i) << LOGN),
                                                  tw_all + ((size_t)i << LOGN), pc, xcd_grouped_tile<TILE, A>());
}

template <int A, int B, int TILE>
__global__ __launch_bounds__(TILE / kSmallE) void ntt_small_rows_moddown_kernel(
    const uint64_t *conv, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs, const uint64_t *ip,
    uint64_t *out, const uint64_t *__restrict__ pinv, uint32_t nl, uint32_t K) {
    __shared__ uint64_t lds[(1 << B) * (TILE / (1 << B) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t c = blockIdx.y & 1, i = blockIdx.y >> 1;
    const PrimeConst pc = pcs[i];
    const ModdownFoldEpi epi{ip + (((size_t)c * (nl + K) + i) << LOGN), out + (((size_t)c * nl + i) << LOGN),
                             pinv[2 * i], pinv[2 * i + 1], pc.q};
    ntt_rows_small_pe<A, B, true, TILE, kSmallE>(lds, LoadPro{conv + (((size_t)c * nl + i) << LOGN)},
                                                 tw_all + ((size_t)i << LOGN), pc, blockIdx.x, epi);
}

template <int A, int B, int TILE, bool KEEP_T>
__global__ __launch_bounds__(TILE / kSmallE) void ntt_small_cols_lift_kernel(
    const uint64_t *last, uint64_t *lift, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs,
    const uint64_t *__restrict__ tab, uint32_t nl, uint32_t L) {
    __shared__ uint64_t lds[(1 << A) * (TILE / (1 << A) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t l = nl - 1;
    const uint32_t c = blockIdx.y & 1, i = blockIdx.y >> 1;
    const PrimeConst pc = pcs[i];
    const LiftPro<KEEP_T> pro = lift_pro<KEEP_T, LOGN>(last, pcs, pc, tab, c, i, nl, L);
    ntt_cols_small_pro<A, B, true, TILE, kSmallE>(lds, pro, lift + (((size_t)c * l + i) << LOGN),
                                                  tw_all + ((size_t)i << LOGN), pc, xcd_grouped_tile<TILE, A>());
}

template <int A, int B, int TILE>
__global__ __launch_bounds__(TILE / kSmallE) void ntt_small_rows_rescale_kernel(
    const uint64_t *lift, const TwPair *__restrict__ tw_all, const PrimeConst *__restrict__ pcs, const uint64_t *in,
    uint64_t *out, const uint64_t *__restrict__ tab, uint32_t nl, uint32_t L) {
    __shared__ uint64_t lds[(1 << B) * (TILE / (1 << B) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t l = nl - 1;
    const uint32_t c = blockIdx.y & 1, i = blockIdx.y >> 1;
    const PrimeConst pc = pcs[i];
    const uint64_t *t = tab + ((size_t)l * L + i) * 3;
    const RescaleTailEpi epi{in + (((size_t)c * nl + i) << LOGN), out + (((size_t)c * l + i) << LOGN), t[0], t[1],
                             pc.q};
    ntt_rows_small_pe<A, B, true, TILE, kSmallE>(lds, LoadPro{lift + (((size_t)c * l + i) << LOGN)},
                                                 tw_all + ((size_t)i << LOGN), pc, blockIdx.x, epi);
}

// First pass of INTT(d2) (galois == 0: d2 = a1 b1 of a, b) or of INTT(sigma_g(a1))
// on small tiles, into dc [nl][N].
template <int A, int B, int TILE>
__global__ __launch_bounds__(TILE / kSmallE) void ntt_small_inv_rows_first_kernel(
    const uint64_t *a, const uint64_t *b, uint64_t *dc, uint32_t galois, const TwPair *__restrict__ tw_all,
    const PrimeConst *__restrict__ pcs, uint32_t nl) {
    __shared__ uint64_t lds[(1 << B) * (TILE / (1 << B) + 1)];
    constexpr int LOGN = A + B;
    const uint32_t i = blockIdx.y;
    const PrimeConst pc = pcs[i];
    const size_t li = (size_t)i << LOGN, poly = (size_t)nl << LOGN;
    if (galois) {
        const GatherPro pro{a + poly + li, galois, (uint32_t)LOGN};
        ntt_rows_small_pe<A, B, false, TILE, kSmallE>(lds, pro, tw_all + li, pc, blockIdx.x, StoreEpi{dc + li});
    } else {
        const TensorPro pro{a + poly + li, b + poly + li, pc.q, pc.r64, pc.r64_p, pc.one_p};
        ntt_rows_small_pe<A, B, false, TILE, kSmallE>(lds, pro, tw_all + li, pc, blockIdx.x, StoreEpi{dc + li});
    }
}


template <int A, int B, int TILE, int E>
static void launch_two_pass_small(const rf_ctx *c, const NttBatch &b, bool forward, hipStream_t s,
                                  const PrimeConst *pcs) {
    const uint32_t limbs = b.per_poly * b.n_polys;
    const dim3 grid((1u << (A + B)) / TILE, limbs), block(TILE / E);
    NttBatch b2 = b;
    b2.in = b.out;
    b2.in_poly_stride = b.out_poly_stride;
    if (forward) {
        {
            ProfScope p("ntt_fwd_cols_small", s);
            hipLaunchKernelGGL((ntt_small_kernel<A, B, true, true, TILE, E>), grid, block, 0, s, b, c->d_tw_fwd, pcs);
        }
        ProfScope p("ntt_fwd_rows_small", s);
        hipLaunchKernelGGL((ntt_small_kernel<A, B, true, false, TILE, E>), grid, block, 0, s, b2, c->d_tw_fwd, pcs);
    } else {
        {
            ProfScope p("ntt_inv_rows_small", s);
            hipLaunchKernelGGL((ntt_small_kernel<A, B, false, false, TILE, E>), grid, block, 0, s, b, c->d_tw_inv,
                               pcs);
        }
        ProfScope p("ntt_inv_cols_small", s);
        hipLaunchKernelGGL((ntt_small_kernel<A, B, false, true, TILE, E>), grid, block, 0, s, b2, c->d_tw_inv, pcs);
    }
}

template <int A, int B>
static void launch_two_pass(const rf_ctx *c, const NttBatch &b, bool forward, hipStream_t s,
                            const PrimeConst *pcs, const rf_tuning &tn) {
    const uint32_t limbs = b.per_poly * b.n_polys;
    const uint32_t tiles = limbs << (A + B - 12);
    if (tiles < tn.ntt_small_below) {
        const bool big = tn.ntt_small_tile == 2048 || (tn.ntt_small_tile == 0 && tiles * 2 >= tn.ntt_small_below);
        if (tn.ntt_small_radix == 8) {
            if (big) launch_two_pass_small<A, B, 2048, 8>(c, b, forward, s, pcs);
            else launch_two_pass_small<A, B, 1024, 8>(c, b, forward, s, pcs);
        } else {
            if (big) launch_two_pass_small<A, B, 2048, kSmallE>(c, b, forward, s, pcs);
            else launch_two_pass_small<A, B, 1024, kSmallE>(c, b, forward, s, pcs);
        }
        return;
    }
    const dim3 block(kThreads);
    const dim3 grid_cols((1u << B) / (kTile >> A), limbs);
    const dim3 grid_rows((1u << A) / (kTile >> B), limbs);
    NttBatch b2 = b;
    b2.in = b.out;
    b2.in_poly_stride = b.out_poly_stride;
    if (forward) {
        {
            ProfScope p("ntt_fwd_cols", s);
            hipLaunchKernelGGL((ntt_cols_kernel<A, B, true>), grid_cols, block, 0, s, b, c->d_tw_fwd, pcs);
        }
        ProfScope p("ntt_fwd_rows", s);
        hipLaunchKernelGGL((ntt_rows_kernel<A, B, true>), grid_rows, block, 0, s, b2, c->d_tw_fwd_rows, pcs);
    } else {
        {
            ProfScope p("ntt_inv_rows", s);
            hipLaunchKernelGGL((ntt_rows_kernel<A, B, false>), grid_rows, block, 0, s, b, c->d_tw_inv_rows, pcs);
        }
        ProfScope p("ntt_inv_cols", s);
        hipLaunchKernelGGL((ntt_cols_kernel<A, B, false>), grid_cols, block, 0, s, b2, c->d_tw_inv, pcs);
    }
}

// Small-tile size of a fused launch of `limbs` limbs, or 0 for the 4096-residue
// tiles (launch_two_pass's rule with the fused launches' threshold).
static int small_tile_of(const rf_ctx *c, uint32_t limbs, const rf_tuning *tn) {
    const rf_tuning &t = tn ? *tn : kDefaultTuning;
    const uint32_t tiles = limbs * (c->n / kTile);
    if (c->log_n < 13 || tiles >= t.ntt_fused_small_below) return 0;
    return t.ntt_small_tile == 2048 || (t.ntt_small_tile == 0 && tiles * 2 >= t.ntt_fused_small_below) ? 2048 : 1024;
}

int launch_ntt_fwd_moddown(const rf_ctx *c, uint64_t *conv, const uint64_t *ip, uint64_t *out, uint32_t nl,
                           hipStream_t s, const rf_tuning *tn) {
    const uint64_t *tab = c->scheme == RF_BGV ? c->d_moddown_t : c->d_moddown;
    const uint64_t *cross = tab + moddown_cross_off(c), *negp = tab + moddown_negp_off(c);
    const uint64_t *pinv = c->d_moddown + moddown_pinv_off(c);
    const dim3 g(c->n / kTile, 2 * nl);
    const int st = small_tile_of(c, 2 * nl, tn);
    if (st) {
#define RF_SMDK(A, B, T, KP)                                                                                     \
    hipLaunchKernelGGL((ntt_small_cols_moddown_kernel<A, B, T, KP>), dim3(c->n / T, 2 * nl), dim3(T / kSmallE), 0, s, \
                       ip, conv, c->d_tw_fwd, c->d_pc, cross, negp, nl, c->L, c->K)
#define RF_SMD(A, B, T)                                                                                          \
    {                                                                                                            \
        {                                                                                                        \
            ProfScope p("ntt_fwd_cols_moddown_small", s);                                                        \
            switch (c->K) {                                                                                      \
                case 1: RF_SMDK(A, B, T, 1); break;                                                              \
                case 2: RF_SMDK(A, B, T, 2); break;                                                              \
                case 3: RF_SMDK(A, B, T, 3); break;                                                              \
                case 4: RF_SMDK(A, B, T, 4); break;                                                              \
                default: RF_SMDK(A, B, T, 8); break;                                                             \
            }                                                                                                    \
        }                                                                                                        \
        ProfScope p("ntt_fwd_rows_moddown_small", s);                                                            \
        hipLaunchKernelGGL((ntt_small_rows_moddown_kernel<A, B, T>), dim3(c->n / T, 2 * nl), dim3(T / kSmallE), 0, s, \
                           conv, c->d_tw_fwd, c->d_pc, ip, out, pinv, nl, c->K);                                 \
    }
#define RF_SMDT(A, B) \
    if (st == 2048) RF_SMD(A, B, 2048) else RF_SMD(A, B, 1024)
        switch (c->log_n) {
            case 13: RF_SMDT(7, 6) break;
            case 14: RF_SMDT(7, 7) break;
            case 15: RF_SMDT(8, 7) break;
            default: RF_SMDT(8, 8) break;
        }
#undef RF_SMDT
#undef RF_SMD
#undef RF_SMDK
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(RF_EHIP, std::string("NTT launch: ") + hipGetErrorString(e));
        return RF_OK;
    }
#define RF_MDK(A, B, KP)                                                                                         \
    hipLaunchKernelGGL((ntt_cols_moddown_kernel<A, B, KP>), dim3((1u << B) / (kTile >> A), 2 * nl), dim3(kThreads), \
                       0, s, ip, conv, c->d_tw_fwd, c->d_pc, cross, negp, nl, c->L, c->K)
#define RF_MD(A, B)                                                                                              \
    {                                                                                                            \
        {                                                                                                        \
            ProfScope p("ntt_fwd_cols_moddown", s);                                                              \
            switch (c->K) {                                                                                      \
                case 1: RF_MDK(A, B, 1); break;                                                                  \
                case 2: RF_MDK(A, B, 2); break;                                                                  \
                case 3: RF_MDK(A, B, 3); break;                                                                  \
                case 4: RF_MDK(A, B, 4); break;                                                                  \
                default: RF_MDK(A, B, 8); break;                                                                 \
            }                                                                                                    \
        }                                                                                                        \
        ProfScope p("ntt_fwd_rows_moddown", s);                                                                  \
        hipLaunchKernelGGL((ntt_rows_moddown_kernel<A, B>), g, dim3(kThreads), 0, s, conv, c->d_tw_fwd_rows, c->d_pc, ip, \
                           out, pinv, nl, c->K);                                                                 \
    }
    switch (c->log_n) {
        case 13: RF_MD(7, 6) break;
        case 14: RF_MD(7, 7) break;
        case 15: RF_MD(8, 7) break;
        case 16: RF_MD(8, 8) break;
        default: return fail(RF_EUNSUPPORTED, "fused ModDown NTT: ring degree");
    }
#undef RF_MD
#undef RF_MDK
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RF_EHIP, std::string("NTT launch: ") + hipGetErrorString(e));
    return RF_OK;
}

int launch_ntt_fwd_rescale(const rf_ctx *c, const uint64_t *last, uint64_t *lift, const uint64_t *in,
                           uint64_t *out, uint32_t nl, bool keep_t, hipStream_t s, const rf_tuning *tn) {
    const uint32_t l = nl - 1;
    const dim3 g(c->n / kTile, 2 * l);
    const int st = small_tile_of(c, 2 * l, tn);
    if (st) {
#define RF_SRS(A, B, T)                                                                                          \
    {                                                                                                            \
        const dim3 gs(c->n / T, 2 * l), bs(T / kSmallE);                                                         \
        {                                                                                                        \
            ProfScope p("ntt_fwd_cols_lift_small", s);                                                           \
            if (keep_t)                                                                                          \
                hipLaunchKernelGGL((ntt_small_cols_lift_kernel<A, B, T, true>), gs, bs, 0, s, last, lift,        \
                                   c->d_tw_fwd, c->d_pc, c->d_rescale, nl, c->L);                                \
            else                                                                                                 \
                hipLaunchKernelGGL((ntt_small_cols_lift_kernel<A, B, T, false>), gs, bs, 0, s, last, lift,       \
                                   c->d_tw_fwd, c->d_pc, c->d_rescale, nl, c->L);                                \
        }                                                                                                        \
        ProfScope p("ntt_fwd_rows_rescale_small", s);                                                            \
        hipLaunchKernelGGL((ntt_small_rows_rescale_kernel<A, B, T>), gs, bs, 0, s, lift, c->d_tw_fwd, c->d_pc, in, \
                           out, c->d_rescale, nl, c->L);                                                         \
    }
#define RF_SRST(A, B) \
    if (st == 2048) RF_SRS(A, B, 2048) else RF_SRS(A, B, 1024)
        switch (c->log_n) {
            case 13: RF_SRST(7, 6) break;
            case 14: RF_SRST(7, 7) break;
            case 15: RF_SRST(8, 7) break;
            default: RF_SRST(8, 8) break;
        }
#undef RF_SRST
#undef RF_SRS
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(RF_EHIP, std::string("NTT launch: ") + hipGetErrorString(e));
        return RF_OK;
    }
#define RF_RS(A, B)                                                                                              \
    {                                                                                                            \
        {                                                                                                        \
            ProfScope p("ntt_fwd_cols_lift", s);                                                                 \
            const dim3 gc((1u << B) / (kTile >> A), 2 * l);                                                      \
            if (keep_t)                                                                                          \
                hipLaunchKernelGGL((ntt_cols_lift_kernel<A, B, true>), gc, dim3(kThreads), 0, s, last, lift,     \
                                   c->d_tw_fwd, c->d_pc, c->d_rescale, nl, c->L);                                \
            else                                                                                                 \
                hipLaunchKernelGGL((ntt_cols_lift_kernel<A, B, false>), gc, dim3(kThreads), 0, s, last, lift,    \
                                   c->d_tw_fwd, c->d_pc, c->d_rescale, nl, c->L);                                \
        }                                                                                                        \
        ProfScope p("ntt_fwd_rows_rescale", s);                                                                  \
        hipLaunchKernelGGL((ntt_rows_rescale_kernel<A, B>), g, dim3(kThreads), 0, s, lift, c->d_tw_fwd_rows, c->d_pc, in, \
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

int launch_intt_first(const rf_ctx *c, const uint64_t *a, const uint64_t *b, uint64_t *dc, uint32_t galois,
                      uint32_t nl, hipStream_t s, const rf_tuning *tn) {
    const uint64_t N = c->n;
    const int st = small_tile_of(c, nl, tn);
    if (st) {
#define RF_SIF(A, B, T)                                                                                          \
    {                                                                                                            \
        const dim3 gs(c->n / T, nl), bs(T / kSmallE);                                                            \
        {                                                                                                        \
            ProfScope p(galois ? "ntt_inv_rows_gather_small" : "ntt_inv_rows_tensor_small", s);                  \
            hipLaunchKernelGGL((ntt_small_inv_rows_first_kernel<A, B, T>), gs, bs, 0, s, a, b, dc, galois,      \
                               c->d_tw_inv, c->d_pc, nl);                                                        \
        }                                                                                                        \
        NttBatch bc{dc, dc, 0, 0, nl, 1, 0, nullptr};                                                            \
        ProfScope p("ntt_inv_cols_small", s);                                                                    \
        hipLaunchKernelGGL((ntt_small_kernel<A, B, false, true, T, kSmallE>), gs, bs, 0, s, bc, c->d_tw_inv,     \
                           pc_modup(c, nl));                                                                     \
    }
#define RF_SIFT(A, B) \
    if (st == 2048) RF_SIF(A, B, 2048) else RF_SIF(A, B, 1024)
        switch (c->log_n) {
            case 13: RF_SIFT(7, 6) break;
            case 14: RF_SIFT(7, 7) break;
            case 15: RF_SIFT(8, 7) break;
            default: RF_SIFT(8, 8) break;
        }
#undef RF_SIFT
#undef RF_SIF
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(RF_EHIP, std::string("NTT launch: ") + hipGetErrorString(e));
        return RF_OK;
    }
#define RF_IF(A, B)                                                                                              \
    {                                                                                                            \
        const dim3 gr((1u << A) / (kTile >> B), nl);                                                             \
        if (galois) {                                                                                            \
            ProfScope p("ntt_inv_rows_gather", s);                                                               \
            hipLaunchKernelGGL((ntt_inv_rows_gather_kernel<A, B>), gr, dim3(kThreads), 0, s, a + (size_t)nl * N, dc, \
                               galois, c->d_tw_inv_rows, c->d_pc);                                                    \
        } else {                                                                                                 \
            ProfScope p("ntt_inv_rows_tensor", s);                                                               \
            hipLaunchKernelGGL((ntt_inv_rows_tensor_kernel<A, B>), gr, dim3(kThreads), 0, s, a, b, dc,           \
                               c->d_tw_inv_rows, c->d_pc, nl);                                                        \
        }                                                                                                        \
        NttBatch bc{dc, dc, 0, 0, nl, 1, 0, nullptr};                                                            \
        ProfScope p("ntt_inv_cols", s);                                                                          \
        hipLaunchKernelGGL((ntt_cols_kernel<A, B, false>), dim3((1u << B) / (kTile >> A), nl), dim3(kThreads), 0, \
                           s, bc, c->d_tw_inv, pc_modup(c, nl));                                                 \
    }
    switch (c->log_n) {
        case 13: RF_IF(7, 6) break;
        case 14: RF_IF(7, 7) break;
        case 15: RF_IF(8, 7) break;
        case 16: RF_IF(8, 8) break;
        default: return fail(RF_EUNSUPPORTED, "fused first INTT: ring degree");
    }
#undef RF_IF
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RF_EHIP, std::string("NTT launch: ") + hipGetErrorString(e));
    return RF_OK;
}

int launch_ntt(const rf_ctx *c, const NttBatch &b, bool forward, hipStream_t s, const PrimeConst *pcs,
               const rf_tuning *tn) {
    const uint32_t limbs = b.per_poly * b.n_polys;
    if (!pcs) pcs = c->d_pc;
    const rf_tuning &t = tn ? *tn : kDefaultTuning;
    if (limbs == 0) return RF_OK;
    if (limbs > 65535) return fail(RF_EUNSUPPORTED, "too many limbs in one NTT launch");
    switch (c->log_n) {
        case 12: {
            ProfScope p(forward ? "ntt_fwd_single" : "ntt_inv_single", s);
            if (forward)
                hipLaunchKernelGGL((ntt_single_kernel<12, true>), dim3(1, limbs), dim3(kThreads), 0, s, b,
                                   c->d_tw_fwd, pcs);
            else
                hipLaunchKernelGGL((ntt_single_kernel<12, false>), dim3(1, limbs), dim3(kThreads), 0, s, b,
                                   c->d_tw_inv, pcs);
            break;
        }
        case 13: launch_two_pass<7, 6>(c, b, forward, s, pcs, t); break;
        case 14: launch_two_pass<7, 7>(c, b, forward, s, pcs, t); break;
        case 15: launch_two_pass<8, 7>(c, b, forward, s, pcs, t); break;
        case 16: launch_two_pass<8, 8>(c, b, forward, s, pcs, t); break;
        default: return fail(RF_EUNSUPPORTED, "ring degree");
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(RF_EHIP, std::string("NTT launch: ") + hipGetErrorString(e));
    return RF_OK;
}

}  // namespace rf
