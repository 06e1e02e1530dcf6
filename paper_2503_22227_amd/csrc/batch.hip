// Batched HMult+Relin over many ciphertexts of different ring degrees and
// levels.  The chain is the single-operation one: INTT of d2 = a1 b1 (formed
// in the first pass), ModUp conversion, NTT, inner product (which forms d0, d1
// and the own-digit d2 residues itself and leaves its Q-limbs as
// ip P^-1 + d_c), INTT of the P-limbs (with the conversion's input factor in
// its last stage), NTT of the ModDown conversion (computed in the first pass,
// the tail out = ip' - NTT(conv) P^-1 in the last).  The tensor,
// ModDown-conversion and tail steps keep their stage numbers with no work
// units.
//
// Launches: each element-wise step (ModUp conversion, inner product) is ONE
// launch over the work units of every item; each NTT pass is one launch per
// ring degree present (one transform shape per kernel keeps the unrolled
// rounds free of register spills).  By default a workgroup takes one work
// unit; rf_batch_set_grid gives a launch a fixed number of workgroups, each
// walking a contiguous range of units (a persistent form the autotuner can
// pick).
//
// Work units: an NTT pass unit is one 4096-residue tile of one limb
// (N / 4096 tiles per limb); an element-wise unit is 256 coefficients of one
// limb, digit or polynomial.  The units of a step are numbered item after
// item (prefix sums in the job tables); a workgroup finds the item of its
// first unit by binary search and then walks forward, so the per-unit
// overhead is a compare.  Mixed ring degrees are dispatched per unit to the
// matching template instantiation of the shared device code (ntt_dev.hpp,
// ks_dev.hpp), so an item's results are bit-identical to the single-operation
// path.  The launch sequence can be captured once in a hipGraph and replayed;
// the job tables are device data, so the graph does not depend on anything but
// the plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ks_dev.hpp"
#include "ntt_dev.hpp"

namespace rf {

enum BatchStage {
    kTensor = 0,
    kInttD0, kInttD1,       // INTT of d2: row pass, column pass
    kModupConv,
    kNttExt0, kNttExt1,     // NTT of the ModUp output: column pass, row pass
    kInnerProduct,
    kInttP0, kInttP1,       // INTT of the P-limbs
    kModdownConv,
    kNttConv0, kNttConv1,   // NTT of the ModDown conversion
    kTail,
    kStages
};

struct KsJob {
    const uint64_t *a, *b, *evk;
    uint64_t *out;
    uint64_t *d2, *d_coeff, *ext, *ip, *conv;
    const PrimeConst *pcs;
    const uint64_t *modup_tab;
    uint64_t modup_stride;
    const uint64_t *moddown_tab;
    const uint64_t *pinv;
    uint32_t log_n, nl, L, K, alpha;
    uint32_t unit_begin[kStages];
};

struct NttJob {
    NttBatch b;
    const TwPair *tw_all;   // natural table (column passes)
    const TwPair *tw_rows;  // row-pass layout (row passes)
    const PrimeConst *pcs;
    uint32_t log_n;
    uint32_t unit_begin;
    // prologue of the INTT of d2: the item's ciphertexts a, b ([2][nl][N])
    const uint64_t *ct_a, *ct_b;
    // ModDown in NTT(conv): conversion from the P-limbs of ip in the first pass,
    // tail out = ip' - NTT(conv) P^-1 in the last
    const uint64_t *ip;
    uint64_t *out;
    const uint64_t *pinv, *md_cross, *md_negp;
    uint32_t nl, K, L;
};

template <typename J>
__device__ __forceinline__ uint32_t unit_begin_of(const J &j, int stage);
template <>
__device__ __forceinline__ uint32_t unit_begin_of<KsJob>(const KsJob &j, int stage) {
    return j.unit_begin[stage];
}
template <>
__device__ __forceinline__ uint32_t unit_begin_of<NttJob>(const NttJob &j, int) {
    return j.unit_begin;
}

// The pointers of a job table address device memory, but loaded from the table
// they are generic pointers, and every access through one would be a flat
// instruction (counted by both the vector-memory and the LDS/scalar wait
// counters, so each use waits for both).  A job is copied with its pointers'
// bits re-typed as global-address-space pointers, which lets the compiler emit
// global loads and stores.
template <typename T>
__device__ __forceinline__ T *gptr(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

__device__ __forceinline__ KsJob global_job(const KsJob &J) {
    KsJob g = J;
    g.a = gptr(J.a);
    g.b = gptr(J.b);
    g.evk = gptr(J.evk);
    g.out = gptr(J.out);
    g.d2 = gptr(J.d2);
    g.d_coeff = gptr(J.d_coeff);
    g.ext = gptr(J.ext);
    g.ip = gptr(J.ip);
    g.conv = gptr(J.conv);
    g.pcs = gptr(J.pcs);
    g.modup_tab = gptr(J.modup_tab);
    g.moddown_tab = gptr(J.moddown_tab);
    g.pinv = gptr(J.pinv);
    return g;
}

__device__ __forceinline__ NttJob global_job(const NttJob &J) {
    NttJob g = J;
    g.b.in = gptr(J.b.in);
    g.b.out = gptr(J.b.out);
    g.b.pmap = gptr(J.b.pmap);
    g.tw_all = gptr(J.tw_all);
    g.tw_rows = gptr(J.tw_rows);
    g.pcs = gptr(J.pcs);
    g.ct_a = gptr(J.ct_a);
    g.ct_b = gptr(J.ct_b);
    g.ip = gptr(J.ip);
    g.out = gptr(J.out);
    g.pinv = gptr(J.pinv);
    g.md_cross = gptr(J.md_cross);
    g.md_negp = gptr(J.md_negp);
    return g;
}

// Last job whose first unit is <= u (jobs sorted by unit_begin).
template <typename J>
__device__ __forceinline__ uint32_t find_job(const J *jobs, uint32_t njobs, uint32_t u, int stage) {
    uint32_t lo = 0, hi = njobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (unit_begin_of(jobs[mid], stage) <= u) lo = mid;
        else hi = mid;
    }
    return lo;
}

// CH: ModUp conversion output limbs per thread (kModupConv only).
template <int STAGE, int CH = kModupChunk>
__global__ __launch_bounds__(kEw) void ks_batched_kernel(const KsJob *__restrict__ jobs, uint32_t njobs,
                                                         uint32_t total, uint32_t per_wg) {
    const uint32_t u0 = blockIdx.x * per_wg;
    const uint32_t u1 = min(total, u0 + per_wg);
    if (u0 >= u1) return;
    uint32_t j = find_job(jobs, njobs, u0, STAGE);
    for (uint32_t u = u0; u < u1; ++u) {
        while (j + 1 < njobs && jobs[j + 1].unit_begin[STAGE] <= u) ++j;
        const KsJob J = global_job(jobs[j]);
        const uint32_t local = u - J.unit_begin[STAGE];
        const uint32_t cshift = J.log_n - 8;  // N / 256 blocks per row
        const uint32_t gy = local >> cshift, gx = local & ((1u << cshift) - 1);
        if constexpr (STAGE == kTensor) {
            tensor_unit(J.a, J.b, J.out, J.d2, J.pcs, J.log_n, J.nl, nullptr, gx, gy);
        } else if constexpr (STAGE == kModupConv) {
            modup_bconv_unit<true, CH>(J.d_coeff, J.ext, J.pcs, J.modup_tab, J.modup_stride, J.log_n, J.nl, J.L, J.K, J.alpha,
                             gx, gy);
        } else if constexpr (STAGE == kInnerProduct) {
            IpFold f;
            f.pinv = J.pinv;
            f.mode = 1;
            f.a = J.a;
            f.b = J.b;
            inner_product_unit<1>(J.d2, J.ext, J.evk, J.ip, J.pcs, J.log_n, J.nl, J.L, J.K, J.alpha, gx, gy, f);
        } else if constexpr (STAGE == kModdownConv) {
            moddown_bconv_unit(J.ip, J.conv, J.pcs, J.moddown_tab, J.log_n, J.nl, J.L, J.K, gx, gy);
        } else if constexpr (STAGE == kTail) {
            const size_t poly = (size_t)J.nl << J.log_n;
            moddown_tail_unit(J.ip, J.conv, J.out, J.out + poly, J.out, J.pcs, J.pinv, J.log_n, J.nl, J.K, gx, gy);
        }
    }
}

// First pass of NTT(conv) of target li of polynomial poly with the ModDown
// conversion from the item's P-limbs as its prologue (KP: see ModdownPro).
template <int A, int B, int KP>
__device__ __forceinline__ void moddown_cols_pass(uint64_t *lds, const NttJob &J, uint32_t poly, uint32_t li,
                                                  uint64_t *out, const TwPair *tw, const PrimeConst &pc, uint32_t tile) {
    constexpr int LOGN = A + B;
    ModdownPro<KP> pro;
    pro.src = J.ip + (((size_t)poly * (J.nl + J.K) + J.nl) << LOGN);
    pro.stride = (size_t)1 << LOGN;
    pro.K = J.K;
#pragma unroll
    for (int a = 0; a < KP; ++a) {
        pro.half[a] = a < (int)J.K ? J.pcs[J.L + a].q >> 1 : 0;
        pro.cross[a] = a < (int)J.K ? J.md_cross[(size_t)li * J.K + a] : 0;
    }
    pro.negp = J.md_negp[li];
    pro.q = pc.q;
    pro.r64 = pc.r64;
    pro.r64_p = pc.r64_p;
    pro.one_p = pc.one_p;
    ntt_cols_unit_pro<A, B, true>(lds, out, tw, pc, tile, pro);
}

// One pass of a batched (I)NTT over the items of one ring degree 2^(A+B) (the
// plan launches each NTT step once per ring degree present: one transform
// shape per kernel keeps the unrolled rounds free of register spills).
// FIRST = the pass that reads b.in (forward: columns; inverse: rows); the
// second pass works in place on b.out.  TAIL (the forward row pass of
// NTT(conv)) writes the ModDown result instead.  PRO: the first pass computes
// its input: 1 = d2 from a, b (INTT of d2), 2 / 3 = the ModDown conversion
// (NTT of conv) from 4 / up to 8 special primes.  Units [unit0, unit0 + total) of the step; jobs = the items of the
// ring degree, whose unit_begin values are absolute.
template <int A, int B, bool FWD, bool FIRST, bool TAIL, int PRO>
__device__ __forceinline__ void ntt_batched_unit(uint64_t *lds, const NttJob &J, uint32_t u) {
    constexpr int LOGN = A + B;
    constexpr bool COLS = FWD == FIRST;
    const uint32_t local = u - J.unit_begin;
    constexpr uint32_t tshift = LOGN - 12;  // N / 4096 tiles per limb
    const uint32_t limb = local >> tshift, tile = local & ((1u << tshift) - 1);
    const uint32_t poly = limb / J.b.per_poly, li = limb - poly * J.b.per_poly;
    const uint32_t g = J.b.pmap ? (uint32_t)J.b.pmap[li] : J.b.prime_base + li;
    const uint64_t *base_in = FIRST ? J.b.in : J.b.out;
    const uint64_t in_stride = FIRST ? J.b.in_poly_stride : J.b.out_poly_stride;
    const uint64_t *in = base_in + (size_t)poly * in_stride + ((size_t)li << LOGN);
    uint64_t *out = J.b.out + (size_t)poly * J.b.out_poly_stride + ((size_t)li << LOGN);
    const PrimeConst pc = J.pcs[g];
    const TwPair *tw = (COLS ? J.tw_all : J.tw_rows) + ((size_t)g << LOGN);
    if constexpr (PRO == 1) {
        // first pass of INTT(d2): d2 = a1 b1 of limb li
        const size_t poly1 = ((size_t)J.nl + li) << LOGN;
        const TensorPro pro{J.ct_a + poly1, J.ct_b + poly1, pc.q, pc.r64, pc.r64_p, pc.one_p};
        ntt_rows_unit_pe<A, B, false>(lds, pro, tw, pc, tile, StoreEpi{out});
    } else if constexpr (PRO == 2 || PRO == 3) {
        // first pass of NTT(conv): ModDown conversion of target li of polynomial
        // poly (2: 4 special primes; 3: any K <= 8).  One variant per kernel: both
        // behind a runtime switch cost the register allocation of the larger.
        moddown_cols_pass<A, B, PRO == 2 ? 4 : 8>(lds, J, poly, li, out, tw, pc, tile);
    } else if constexpr (TAIL) {
        // limb li of polynomial poly of conv [2][nl][N]: ModDown tail into out
        const size_t lo = ((size_t)poly * (J.nl + J.K) + li) << LOGN;
        const size_t oo = ((size_t)poly * J.nl + li) << LOGN;
        const ModdownFoldEpi epi{J.ip + lo, J.out + oo, J.pinv[2 * li], J.pinv[2 * li + 1], pc.q};
        ntt_rows_unit_epi<A, B, true>(lds, in, tw, pc, tile, epi);
    } else if constexpr (COLS) {
        ntt_cols_unit<A, B, FWD>(lds, in, out, tw, pc, tile);
    } else {
        ntt_rows_unit<A, B, FWD>(lds, in, out, tw, pc, tile);
    }
}

// One pass of a batched (I)NTT over the items of one ring degree 2^(A+B) (the
// plan launches each NTT step once per ring degree present: one transform
// shape per kernel keeps the unrolled rounds free of register spills).
// FIRST = the pass that reads b.in (forward: columns; inverse: rows); the
// second pass works in place on b.out.  TAIL (the forward row pass of
// NTT(conv)) writes the ModDown result instead.  PRO: the first pass computes
// its input: 1 = d2 from a, b (INTT of d2), 2 / 3 = the ModDown conversion
// (NTT of conv) from 4 / up to 8 special primes.  Units [unit0, unit0 + total) of the step; jobs = the items of the
// ring degree, whose unit_begin values are absolute.  LOOP: workgroups walk
// per_wg consecutive units; otherwise each takes one unit (per_wg == 1).
template <int A, int B, bool FWD, bool FIRST, bool TAIL, int PRO, bool LOOP>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNttWavesCols))) void ntt_batched_kernel(
    const NttJob *__restrict__ jobs, uint32_t njobs, uint32_t unit0, uint32_t total, uint32_t per_wg) {
    constexpr bool COLS = FWD == FIRST;
    __shared__ uint64_t lds[COLS ? (1 << A) * (kTile / (1 << A) + 1) : (1 << B) * (kTile / (1 << B) + 1)];
    static_assert(!TAIL || (FWD && !FIRST), "the tail follows the forward row pass");
    static_assert(PRO == 0 || FIRST, "prologues belong to the first pass");
    if constexpr (!LOOP) {
        if (blockIdx.x >= total) return;
        const uint32_t u = unit0 + blockIdx.x;
        ntt_batched_unit<A, B, FWD, FIRST, TAIL, PRO>(lds, global_job(jobs[find_job(jobs, njobs, u, 0)]), u);
    } else {
        const uint32_t u0 = unit0 + blockIdx.x * per_wg;
        const uint32_t u1 = unit0 + min(total, (blockIdx.x + 1) * per_wg);
        if (u0 >= u1) return;
        uint32_t j = find_job(jobs, njobs, u0, 0);
        for (uint32_t u = u0; u < u1; ++u) {
            while (j + 1 < njobs && jobs[j + 1].unit_begin <= u) ++j;
            ntt_batched_unit<A, B, FWD, FIRST, TAIL, PRO>(lds, global_job(jobs[j]), u);
        }
    }
}

}  // namespace rf

using namespace rf;

struct rf_batch {
    int device = 0;
    uint32_t n_items = 0;
    // items sorted by ring degree; group: [job0, job1) with one log_n, and the
    // first unit / unit count of every step inside the group
    struct Group {
        uint32_t log_n, job0, job1;
        bool k4;  // every item has 4 special primes (the specialised ModDown prologue)
        uint32_t unit0[kStages], units[kStages];
    };
    std::vector<Group> groups;
    KsJob *d_jobs = nullptr;
    NttJob *d_ntt[4] = {nullptr, nullptr, nullptr, nullptr};  // INTT d2, NTT ext, INTT P, NTT conv
    uint32_t total[kStages] = {0};
    uint32_t grid[kStages] = {0};  // workgroups per launch; 0 = one per unit
    uint32_t modup_chunk = kModupChunk;  // ModUp output limbs per thread
    std::vector<rf_batch_item> items;    // the item list, to rebuild the tables
    uint64_t *ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture_stream = nullptr;
};

namespace {

size_t item_ws_limbs(const rf_ctx *c, uint32_t nl) {
    const ModupLevel &lv = c->modup_levels[nl];
    return (size_t)nl + (size_t)nl + lv.ext_limbs + 2 * (size_t)(nl + c->K) + 2 * (size_t)nl;
}

int validate(const rf_batch_item *items, uint32_t n) {
    if (!items || n == 0) return fail(RF_EINVAL, "rf_batch: no items");
    const rf_ctx *c0 = items[0].ctx;
    for (uint32_t i = 0; i < n; ++i) {
        const rf_batch_item &it = items[i];
        const rf_ctx *c = it.ctx;
        if (!c || !it.a || !it.b || !it.rlk || !it.out) return fail(RF_EINVAL, "rf_batch: null pointer in an item");
        if (c->scheme != RF_CKKS && c->scheme != RF_BGV) return fail(RF_EUNSUPPORTED, "rf_batch: CKKS or BGV");
        if (c->log_n < 13 || c->log_n > 16) return fail(RF_EUNSUPPORTED, "rf_batch: ring degree 2^13..2^16");
        if (it.n_limbs < 1 || it.n_limbs > c->L) return fail(RF_ELEVEL, "rf_batch: limb count out of range");
        if (c->device != c0->device) return fail(RF_EINVAL, "rf_batch: items on different devices");
        if (it.out == it.a || it.out == it.b) return fail(RF_EINVAL, "rf_batch: out aliases an input");
    }
    return RF_OK;
}

uint32_t stage_units(const rf_ctx *c, uint32_t nl, int stage, uint32_t chunk) {
    const uint32_t chunks = c->n / kEw, tiles = c->n / kTile;
    const uint32_t dn = (nl + c->alpha - 1) / c->alpha;
    switch (stage) {
        case kTensor: return 0;  // formed by the INTT of d2 and the inner product
        case kInttD0: case kInttD1: return nl * tiles;
        case kModupConv: return dn * modup_chunks(nl, c->K, chunk) * chunks;
        case kNttExt0: case kNttExt1: return c->modup_levels[nl].ext_limbs * tiles;
        case kInnerProduct: return (nl + c->K) * chunks;
        case kInttP0: case kInttP1: return 2 * c->K * tiles;
        case kModdownConv: return 0;  // computed in the first pass of NTT(conv)
        case kNttConv0: case kNttConv1: return 2 * nl * tiles;
        case kTail: return 0;  // applied by the last pass of NTT(conv)
    }
    return 0;
}

int enqueue(rf_batch *p, hipStream_t s, bool profile) {
    static const char *names[kStages] = {"batch_tensor", "batch_ntt_inv_rows_tensor", "batch_ntt_inv_cols",
                                         "batch_modup_bconv", "batch_ntt_fwd_cols", "batch_ntt_fwd_rows",
                                         "batch_inner_product", "batch_ntt_inv_rows", "batch_ntt_inv_cols",
                                         "batch_moddown_bconv", "batch_ntt_fwd_cols_moddown", "batch_ntt_fwd_rows_moddown",
                                         "batch_moddown_tail"};
    for (int st = 0; st < kStages; ++st) {
        const uint32_t total = p->total[st];
        if (total == 0) continue;
        ProfScope prof(profile ? names[st] : nullptr, s);
        const bool ntt_step = st != kTensor && st != kModupConv && st != kInnerProduct && st != kModdownConv &&
                              st != kTail;
        if (!ntt_step) {
            const uint32_t g = p->grid[st] == 0 ? total : std::min(total, p->grid[st]);
            const uint32_t per = (total + g - 1) / g;
            const uint32_t blocks = (total + per - 1) / per;
            const uint32_t nj = p->n_items;
            switch (st) {
                case kTensor: hipLaunchKernelGGL(ks_batched_kernel<kTensor>, blocks, kEw, 0, s, p->d_jobs, nj, total, per); break;
                case kModupConv:
                    if (p->modup_chunk == 4)
                        hipLaunchKernelGGL((ks_batched_kernel<kModupConv, 4>), blocks, kEw, 0, s, p->d_jobs, nj, total, per);
                    else if (p->modup_chunk == 16)
                        hipLaunchKernelGGL((ks_batched_kernel<kModupConv, 16>), blocks, kEw, 0, s, p->d_jobs, nj, total, per);
                    else
                        hipLaunchKernelGGL((ks_batched_kernel<kModupConv, 8>), blocks, kEw, 0, s, p->d_jobs, nj, total, per);
                    break;
                case kInnerProduct: hipLaunchKernelGGL(ks_batched_kernel<kInnerProduct>, blocks, kEw, 0, s, p->d_jobs, nj, total, per); break;
                case kModdownConv: hipLaunchKernelGGL(ks_batched_kernel<kModdownConv>, blocks, kEw, 0, s, p->d_jobs, nj, total, per); break;
                case kTail: hipLaunchKernelGGL(ks_batched_kernel<kTail>, blocks, kEw, 0, s, p->d_jobs, nj, total, per); break;
            }
        } else {
            // one launch per ring degree; the step's workgroups are shared out in
            // proportion to the units of each degree
            for (const rf_batch::Group &G : p->groups) {
                const uint32_t units = G.units[st];
                if (units == 0) continue;
                uint32_t g = units;
                if (p->grid[st] != 0)
                    g = std::max(1u, std::min(units, (uint32_t)(((uint64_t)p->grid[st] * units + total - 1) / total)));
                const uint32_t per = (units + g - 1) / g;
                const uint32_t blocks = (units + per - 1) / per;
                const int k = st == kInttD0 || st == kInttD1 ? 0 : st == kNttExt0 || st == kNttExt1 ? 1
                            : st == kInttP0 || st == kInttP1 ? 2 : 3;
                const NttJob *jobs = p->d_ntt[k] + G.job0;
                const uint32_t nj = G.job1 - G.job0, u0 = G.unit0[st];
#define RF_BLK(A, B, FWD, FIRST, TAIL, PRO)                                                                      \
    if (per == 1)                                                                                                \
        hipLaunchKernelGGL((ntt_batched_kernel<A, B, FWD, FIRST, TAIL, PRO, false>), blocks, kThreads, 0, s, jobs, \
                           nj, u0, units, per);                                                                  \
    else                                                                                                         \
        hipLaunchKernelGGL((ntt_batched_kernel<A, B, FWD, FIRST, TAIL, PRO, true>), blocks, kThreads, 0, s, jobs, \
                           nj, u0, units, per)
#define RF_BL(A, B)                                                                                              \
    switch (st) {                                                                                                \
        case kInttD0: RF_BLK(A, B, false, true, false, 1); break;                                                \
        case kInttD1: RF_BLK(A, B, false, false, false, 0); break;                                               \
        case kNttExt0: RF_BLK(A, B, true, true, false, 0); break;                                                \
        case kNttExt1: RF_BLK(A, B, true, false, false, 0); break;                                               \
        case kInttP0: RF_BLK(A, B, false, true, false, 0); break;                                                \
        case kInttP1: RF_BLK(A, B, false, false, false, 0); break;                                               \
        case kNttConv0:                                                                                          \
            if (G.k4) {                                                                                          \
                RF_BLK(A, B, true, true, false, 2);                                                              \
            } else {                                                                                             \
                RF_BLK(A, B, true, true, false, 3);                                                              \
            }                                                                                                    \
            break;                                                                                               \
        case kNttConv1: RF_BLK(A, B, true, false, true, 0); break;                                               \
    }
                switch (G.log_n) {
                    case 16: RF_BL(8, 8) break;
                    case 15: RF_BL(8, 7) break;
                    case 14: RF_BL(7, 7) break;
                    default: RF_BL(7, 6) break;
                }
#undef RF_BL
#undef RF_BLK
            }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(RF_EHIP, std::string("batched launch: ") + hipGetErrorString(e));
    }
    return RF_OK;
}

void drop_graph(rf_batch *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

// Job tables of a plan from its items, workspace and ModUp chunk: the
// element-wise jobs, the four NTT job lists and the ring-degree groups.
void build_tables(rf_batch *p, std::vector<KsJob> &jobs, std::vector<NttJob> (&ntt)[4]) {
    const rf_batch_item *items = p->items.data();
    const uint32_t n = (uint32_t)p->items.size();
    jobs.assign(n, KsJob{});
    for (auto &v : ntt) v.assign(n, NttJob{});
    uint32_t acc[kStages] = {0};
    uint64_t *w = p->ws;
    // items in order of ring degree (the NTT steps run one launch per degree)
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return items[x].ctx->log_n < items[y].ctx->log_n; });
    std::vector<rf_batch::Group> groups;
    for (uint32_t i = 0; i < n; ++i) {
        const rf_batch_item &it = items[order[i]];
        const rf_ctx *c = it.ctx;
        if (groups.empty() || groups.back().log_n != c->log_n) {
            if (!groups.empty()) {
                groups.back().job1 = i;
                for (int st = 0; st < kStages; ++st) groups.back().units[st] = acc[st] - groups.back().unit0[st];
            }
            rf_batch::Group G{};
            G.log_n = c->log_n;
            G.job0 = i;
            G.k4 = true;
            for (int st = 0; st < kStages; ++st) G.unit0[st] = acc[st];
            groups.push_back(G);
        }
        if (c->K != 4) groups.back().k4 = false;
        const uint32_t nl = it.n_limbs;
        const size_t N = c->n;
        const ModupLevel &lv = c->modup_levels[nl];
        KsJob &J = jobs[i];
        J.a = it.a;
        J.b = it.b;
        J.evk = it.rlk;
        J.out = it.out;
        J.d2 = w;
        J.d_coeff = J.d2 + (size_t)nl * N;
        J.ext = J.d_coeff + (size_t)nl * N;
        J.ip = J.ext + (size_t)lv.ext_limbs * N;
        J.conv = J.ip + 2 * (size_t)(nl + c->K) * N;
        w = J.conv + 2 * (size_t)nl * N;
        J.pcs = c->d_pc;
        J.modup_tab = c->d_modup;
        J.modup_stride = c->modup_stride;
        J.moddown_tab = c->scheme == RF_BGV ? c->d_moddown_t : c->d_moddown;
        J.pinv = c->d_moddown + moddown_pinv_off(c);
        J.log_n = c->log_n;
        J.nl = nl;
        J.L = c->L;
        J.K = c->K;
        J.alpha = c->alpha;
        for (int st = 0; st < kStages; ++st) {
            J.unit_begin[st] = acc[st];
            acc[st] += stage_units(c, nl, st, p->modup_chunk);
        }
        const uint64_t ipstride = (uint64_t)(nl + c->K) * N;
        NttBatch bd{J.d2, J.d_coeff, 0, 0, nl, 1, 0, nullptr};
        NttBatch be{J.ext, J.ext, 0, 0, lv.ext_limbs, 1, 0, c->d_pmaps + lv.pmap_off};
        NttBatch bp{J.ip + (size_t)nl * N, J.ip + (size_t)nl * N, ipstride, ipstride, c->K, 2, c->L, nullptr};
        NttBatch bc{J.conv, J.conv, (uint64_t)nl * N, (uint64_t)nl * N, nl, 2, 0, nullptr};
        const NttBatch bs[4] = {bd, be, bp, bc};
        const int first_stage[4] = {kInttD0, kNttExt0, kInttP0, kNttConv0};
        for (int k = 0; k < 4; ++k) {
            ntt[k][i].b = bs[k];
            ntt[k][i].tw_all = (k == 1 || k == 3) ? c->d_tw_fwd : c->d_tw_inv;
            ntt[k][i].tw_rows = (k == 1 || k == 3) ? c->d_tw_fwd_rows : c->d_tw_inv_rows;
            // the INTT of d2 folds the ModUp input factor, the INTT of the P-limbs the
            // ModDown input factor into its last stage
            ntt[k][i].pcs = k == 0 ? pc_modup(c, nl) : k == 2 ? c->d_pc_md : c->d_pc;
            ntt[k][i].log_n = c->log_n;
            ntt[k][i].unit_begin = J.unit_begin[first_stage[k]];
            ntt[k][i].ct_a = it.a;
            ntt[k][i].ct_b = it.b;
            ntt[k][i].ip = J.ip;
            ntt[k][i].out = J.out;
            ntt[k][i].pinv = J.pinv;
            ntt[k][i].md_cross = J.moddown_tab + moddown_cross_off(c);
            ntt[k][i].md_negp = J.moddown_tab + moddown_negp_off(c);
            ntt[k][i].nl = nl;
            ntt[k][i].K = c->K;
            ntt[k][i].L = c->L;
        }
    }
    groups.back().job1 = n;
    for (int st = 0; st < kStages; ++st) groups.back().units[st] = acc[st] - groups.back().unit0[st];
    p->groups = groups;
    for (int st = 0; st < kStages; ++st) p->total[st] = acc[st];
}

// Rebuild and upload the job tables (the device buffers exist already).
int upload_tables(rf_batch *p) {
    std::vector<KsJob> jobs;
    std::vector<NttJob> ntt[4];
    build_tables(p, jobs, ntt);
    const uint32_t n = p->n_items;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    // a launch of the plan still in flight reads the old tables
    bool ok = hipDeviceSynchronize() == hipSuccess &&
              hipMemcpy(p->d_jobs, jobs.data(), sizeof(KsJob) * n, hipMemcpyHostToDevice) == hipSuccess;
    for (int k = 0; k < 4 && ok; ++k)
        ok = hipMemcpy(p->d_ntt[k], ntt[k].data(), sizeof(NttJob) * n, hipMemcpyHostToDevice) == hipSuccess;
    (void)hipSetDevice(prev);
    return ok ? RF_OK : fail(RF_EHIP, "batch plan: upload of the job tables");
}

}  // namespace

extern "C" size_t rf_batch_workspace_bytes(const rf_batch_item *items, uint32_t n) {
    if (validate(items, n)) return 0;
    size_t limbs = 0;
    for (uint32_t i = 0; i < n; ++i) limbs += item_ws_limbs(items[i].ctx, items[i].n_limbs) * items[i].ctx->n;
    return limbs * 8;
}

extern "C" int rf_batch_create(const rf_batch_item *items, uint32_t n, void *ws, size_t ws_bytes, rf_batch **out) {
    int rc;
    if (!out) return fail(RF_EINVAL, "rf_batch_create: null out");
    *out = nullptr;
    if ((rc = validate(items, n))) return rc;
    const size_t need = rf_batch_workspace_bytes(items, n);
    if (!ws || ws_bytes < need)
        return fail(RF_EWORKSPACE, "rf_batch_create: workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                       std::to_string(need));
    rf_batch *p = new rf_batch();
    p->device = items[0].ctx->device;
    p->n_items = n;
    p->items.assign(items, items + n);
    p->ws = (uint64_t *)ws;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    bool ok = hipMalloc((void **)&p->d_jobs, sizeof(KsJob) * n) == hipSuccess;
    for (int k = 0; k < 4 && ok; ++k) ok = hipMalloc((void **)&p->d_ntt[k], sizeof(NttJob) * n) == hipSuccess;
    (void)hipSetDevice(prev);
    if (!ok || upload_tables(p) != RF_OK) {
        rf_batch_destroy(p);
        return fail(RF_EHIP, "rf_batch_create: allocation or upload of the job tables");
    }
    *out = p;
    return RF_OK;
}

extern "C" void rf_batch_destroy(rf_batch *p) {
    if (!p) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    drop_graph(p);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    (void)hipFree(p->d_jobs);
    for (auto *d : p->d_ntt) (void)hipFree(d);
    (void)hipSetDevice(prev);
    delete p;
}

extern "C" int rf_batch_set_grid(rf_batch *p, uint32_t stage, uint32_t workgroups) {
    if (!p || stage >= (uint32_t)kStages) return fail(RF_EINVAL, "rf_batch_set_grid: bad stage");
    if (p->grid[stage] != workgroups) {
        p->grid[stage] = workgroups;
        drop_graph(p);
    }
    return RF_OK;
}

extern "C" int rf_batch_set_modup_chunk(rf_batch *p, uint32_t chunk) {
    if (!p) return fail(RF_EINVAL, "rf_batch_set_modup_chunk: null plan");
    if (chunk != 4 && chunk != 8 && chunk != 16) return fail(RF_EINVAL, "rf_batch_set_modup_chunk: 4, 8 or 16");
    if (p->modup_chunk == chunk) return RF_OK;
    p->modup_chunk = chunk;
    drop_graph(p);
    return upload_tables(p);
}

extern "C" int rf_batch_stage_units(const rf_batch *p, uint32_t stage) {
    if (!p || stage >= (uint32_t)kStages) return fail(RF_EINVAL, "rf_batch_stage_units: bad stage");
    return (int)p->total[stage];
}

extern "C" int rf_batch_hmult_relin(rf_batch *p, void *stream) {
    if (!p) return fail(RF_EINVAL, "rf_batch_hmult_relin: null plan");
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != p->device) (void)hipSetDevice(p->device);
    int rc = enqueue(p, (hipStream_t)stream, true);
    if (prev != p->device) (void)hipSetDevice(prev);
    return rc;
}

extern "C" int rf_batch_graph_launch(rf_batch *p, void *stream) {
    if (!p) return fail(RF_EINVAL, "rf_batch_graph_launch: null plan");
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != p->device) (void)hipSetDevice(p->device);
    int rc = RF_OK;
    if (!p->exec) {
        if (!p->capture_stream && hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess)
            rc = fail(RF_EHIP, "rf_batch_graph_launch: stream");
        if (!rc && hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            rc = fail(RF_EHIP, "rf_batch_graph_launch: begin capture");
        if (!rc) {
            int erc = enqueue(p, p->capture_stream, false);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(p->capture_stream, &g);
            if (erc) rc = erc;
            else if (e != hipSuccess || !g) rc = fail(RF_EHIP, "rf_batch_graph_launch: end capture");
            else {
                p->graph = g;
                if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
                    drop_graph(p);
                    rc = fail(RF_EHIP, "rf_batch_graph_launch: instantiate");
                }
            }
            if (rc && g && !p->graph) (void)hipGraphDestroy(g);
        }
    }
    if (!rc && hipGraphLaunch(p->exec, (hipStream_t)stream) != hipSuccess)
        rc = fail(RF_EHIP, "rf_batch_graph_launch: launch");
    if (prev != p->device) (void)hipSetDevice(prev);
    return rc;
}
