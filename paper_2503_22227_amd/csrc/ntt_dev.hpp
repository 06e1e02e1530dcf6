// Device code of the negacyclic NTT shared by the single-operation kernels
// (ntt.hip) and the persistent batched kernels (batch.hip).
// Negacyclic NTT / INTT for gfx950 (the paper's butterfly-method NTT, III-A).
//
// Convention: forward output index k holds a(psi^(2 brv(k) + 1)).  The forward
// transform is the radix-2 Cooley-Tukey recursion with psi merged into the
// twiddles: stage st (0-based) pairs j and j + N/2^(st+1) with twiddle
// psi^brv(2^st + j / (N/2^st)).  The inverse runs Gentleman-Sande butterflies
// with psi^-brv(.) from the smallest distance up and folds N^-1 into its last
// stage.
//
// Decomposition: a limb of N = 2^(A+B) residues is seen as a 2^A x 2^B matrix
// (row p, column c at index p 2^B + c).  The first A forward stages only mix
// elements of one column; the last B only mix elements of one row.  So the
// forward transform is a column pass then a row pass, the inverse a row pass
// then a column pass, each a size-2^A or 2^B sub-transform that lives in LDS:
//   * a workgroup owns a 4096-residue tile (32 KiB + padding): 16 columns x
//     256 rows, or 16 rows x 256, so every global access of a wavefront is a
//     run of whole 128-byte lines;
//   * inside the tile every thread holds kElems = 16 residues in registers and
//     performs up to 4 butterfly stages on them (a radix-16 round), then the
//     tile is exchanged through LDS for the next round, so a pass of up to 8
//     stages takes two rounds (256-thread workgroups; 8 residues per thread
//     with radix-8 rounds was measured no faster on MI355X);
//   * values stay in Harvey's lazy ranges ([0, 4q) forward, [0, 2q) inverse)
//     between stages and passes and are reduced to [0, q) at the last store.
// N <= 4096 is done in one pass by one workgroup per limb.
#pragma once
#include <hip/hip_runtime.h>

#include "modarith.hpp"
#include "rf_internal.hpp"

namespace rf {

constexpr int kTile = 4096;
constexpr int kElems = 16;                         // residues per thread
constexpr int kElemsLog = 4;                       // stages per round
constexpr int kThreads = kTile / kElems;           // threads per workgroup

// Twiddle layout of the row passes.  A row pass of N = 2^(A+B) works on 2^A rows
// of S = 2^B residues, a tile of U = 4096 / S consecutive rows per workgroup,
// T = S / kElems threads per row.  At local stage s (0..B-1) row r uses the
// twiddles j < 2^s of psi^(+-brv(2^(A+s) + r 2^s + j)).  In the round whose
// butterflies only depend on e (the first forward round, the last inverse
// round) j is the same for the T threads of a row; in the other round thread t
// of a row uses j = t R + k, k < R = kElems 2^s / S.  The row table stores them
// so that one wave instruction (consecutive rows u of a tile, then threads t)
// reads consecutive entries:
//   uniform stage: 2^(A+s) + (r_hi 2^s + j) U + u
//   ranged stage:  2^(A+s) + ((r_hi R + k) T + t) U + u,   r = r_hi U + u.
// The entries below 2^A are unused.  A ranged stage is, forward: s >= kElemsLog
// (the stages after the first round); inverse: s >= B - kElemsLog (the stages
// of the first round).
__host__ __device__ constexpr bool row_tw_ranged(int B, bool fwd, int s) {
    return fwd ? s >= kElemsLog : s >= B - kElemsLog;
}

__host__ __device__ inline uint32_t row_tw_index(int A, int B, bool fwd, uint32_t r, int s, uint32_t j) {
    const uint32_t U = (uint32_t)kTile >> B, T = (1u << B) / kElems;
    const uint32_t r_hi = r / U, u = r % U;
    if (!row_tw_ranged(B, fwd, s)) return (1u << (A + s)) + ((r_hi << s) + j) * U + u;
    const uint32_t R = ((uint32_t)kElems << s) >> B;
    const uint32_t t = j / R, k = j % R;
    return (1u << (A + s)) + ((r_hi * R + k) * T + t) * U + u;
}

// Butterflies with twiddle w and its 2^62-scaled companion wp (shoup62_lazy);
// nq = 2^64 - q.
//
// LZ (primes below kLazyPrimeBound): no correction of the sum.  Forward
// (Cooley-Tukey), x grows by less than 2q per stage, so after all stages of
// both passes of N <= 2^16 every value stays below 36q < 2^56; inverse
// (Gentleman-Sande), values at most double per stage, so at local stage k of a
// pass (inputs below 2^(k+1) q) the difference is formed as x - y + off with
// off = 2^(k+1) q, and each pass starts from inputs below 2q (the row pass
// reduces its output once, see ntt_rows_compute).  Strict: Harvey's ranges,
// inputs and outputs below 4q (forward) or 2q (inverse), off = 2q.
template <bool LZ>
__device__ __forceinline__ void ct_bfly(uint64_t &x, uint64_t &y, uint64_t w, uint64_t wp, uint64_t nq,
                                        uint64_t q2) {
    uint64_t xr = LZ ? x : (x >= q2 ? x - q2 : x);  // strict: [0, 2q)
    uint64_t t = shoup62_lazy(y, w, wp, nq);         // [0, 2q); y < 2^62
    x = xr + t;
    y = xr - t + q2;
}

template <bool LZ>
__device__ __forceinline__ void gs_bfly(uint64_t &x, uint64_t &y, uint64_t w, uint64_t wp, uint64_t nq,
                                        uint64_t q2, uint64_t off) {
    uint64_t s = x + y;
    if (!LZ) s = s >= q2 ? s - q2 : s;
    uint64_t d = x - y + off;                 // off >= any y of this stage
    x = s;
    y = shoup62_lazy(d, w, wp, nq);           // [0, 2q)
}

__device__ __forceinline__ void gs_bfly_last(uint64_t &x, uint64_t &y, const PrimeConst &pc, uint64_t off) {
    uint64_t s = x + y;
    uint64_t d = x - y + off;
    x = shoup_lazy(s, pc.ninv, pc.ninv_p, pc.q);
    y = shoup_lazy(d, pc.wlast, pc.wlast_p, pc.q);
}

// Transforms of primes below this bound skip the sum corrections (LZ above).
constexpr uint64_t kLazyPrimeBound = 1ull << 50;

// Table index of twiddle j of local stage s: the natural index (tw_base << s) + j
// (column passes, ROW_A == 0) or the row-pass layout above, with tw_base = 2^A + r
// and t the thread's index within its row.
template <int S_LOG, int ROW_A, bool FWD>
__device__ __forceinline__ uint32_t row_or_natural(uint32_t tw_base, int s, int t, uint32_t j) {
    if constexpr (ROW_A == 0) {
        return (tw_base << s) + j;
    } else {
        constexpr uint32_t U = (uint32_t)kTile >> S_LOG, T = (1u << S_LOG) / kElems;
        const uint32_t r = tw_base - (1u << ROW_A);
        const uint32_t r_hi = r / U, uu = r % U;
        if (!row_tw_ranged(S_LOG, FWD, s)) return (1u << (ROW_A + s)) + ((r_hi << s) + j) * U + uu;
        const uint32_t R = ((uint32_t)kElems << s) >> S_LOG;
        return (1u << (ROW_A + s)) + ((r_hi * R + (j - (uint32_t)t * R)) * T + (uint32_t)t) * U + uu;
    }
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// Where a round takes its twiddles: loads from the table as each stage needs
// them (kTwLoad); kTwPrefetch only loads the pairs every round of the pass will
// use into a register array (no butterflies, no LDS access), so that all of
// them are in flight together with the tile's own loads; kTwCached then takes
// them from that array.  A pass with few residues per thread (the small-tile
// passes) otherwise waits one table latency after every round's barrier.
constexpr int kTwLoad = 0, kTwPrefetch = 1, kTwCached = 2;

// Register slots of the prefetched twiddles of a pass of S_LOG stages with E
// residues per thread: round r, group gi, stage c, element e at
// SLOT0(r) + (gi C + c) 2^C + e, each round taking E C slots.  Slots a round
// does not use are never written or read.
__host__ __device__ constexpr int tw_slots(int S_LOG, int E) { return E * S_LOG; }

// One round of C butterfly stages of a size-2^S_LOG sub-transform held in LDS
// (element p of sub-transform u at lds[p * ldu + u]).  Thread t of the
// sub-transform owns E residues (kElems unless stated): E / 2^C groups of 2^C
// residues spaced by the round's smallest distance 2^DL.
//
// IN_REGS / OUT_REGS: the round takes its residues from regs / leaves them in
// regs (group gi, element e at regs[gi * 2^C + e]) instead of LDS.  TW, SLOT0,
// cache: the twiddle source above.
template <int S_LOG, int ST0, int C, bool FWD, bool SCALE_LAST, int ROW_A, bool IN_REGS = false,
          bool OUT_REGS = false, bool LZ = false, int E = kElems, int TW = kTwLoad, int SLOT0 = 0>
__device__ __forceinline__ void ntt_round(uint64_t *lds, int ldu, int u, int t, uint32_t tw_base,
                                          const TwPair *__restrict__ tw, const PrimeConst &pc,
                                          uint64_t *regs = nullptr, TwPair *cache = nullptr) {
    constexpr int G = 1 << C;
    constexpr int NG = E / G;
    constexpr int DL = FWD ? (S_LOG - ST0 - C) : ST0;
    constexpr bool RUN = TW != kTwPrefetch;
    const uint64_t q = pc.q, q2 = 2 * q, nq = 0 - q;
    // twiddle (slot, table index): fetched, loaded or taken from the cache
    auto twiddle = [&](int slot, uint32_t idx) -> TwPair {
        if constexpr (TW == kTwPrefetch) {
            cache[slot] = tw[idx];
            return TwPair{};
        } else if constexpr (TW == kTwCached) {
            return cache[slot];
        } else {
            return tw[idx];
        }
    };
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        const int grp = t * NG + gi;
        const int lo = grp & ((1 << DL) - 1);
        const int hi = grp >> DL;
        const int base = (hi << (DL + C)) + lo;
        uint64_t v[G];
        if constexpr (RUN) {
#pragma unroll
            for (int e = 0; e < G; ++e) v[e] = IN_REGS ? regs[gi * G + e] : lds[(base + (e << DL)) * ldu + u];
        }
        if constexpr (FWD) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int st = ST0 + c;
                const int h = G >> (c + 1);
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    if (e & h) continue;
                    // in the first round every group starts below 2^DL, so the twiddle
                    // index depends on e only (uniform across the sub-transform)
                    const uint32_t j = ST0 == 0 ? (uint32_t)(e >> (C - c))
                                                : (uint32_t)((base + (e << DL)) >> (S_LOG - st));
                    const TwPair w = twiddle(SLOT0 + (gi * C + c) * G + e,
                                             row_or_natural<S_LOG, ROW_A, true>(tw_base, st, t, j));
                    if constexpr (RUN) ct_bfly<LZ>(v[e], v[e + h], w.w, w.wp, nq, q2);
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int us = ST0 + c;
                const int h = 1 << c;
                const uint64_t off = LZ ? q << (us + 1) : q2;
#pragma unroll
                for (int e = 0; e < G; ++e) {
                    if (e & h) continue;
                    if (SCALE_LAST && us == S_LOG - 1) {
                        if constexpr (RUN) gs_bfly_last(v[e], v[e + h], pc, off);
                    } else {
                        // in the last round every group starts below 2^DL: index from e only
                        const uint32_t lo_part = ST0 + C == S_LOG ? (uint32_t)(e >> (c + 1))
                                                                  : (uint32_t)((base + (e << DL)) >> (us + 1));
                        const TwPair w = twiddle(SLOT0 + (gi * C + c) * G + e,
                                                 row_or_natural<S_LOG, ROW_A, false>(tw_base, S_LOG - us - 1, t,
                                                                                     lo_part));
                        if constexpr (RUN) gs_bfly<LZ>(v[e], v[e + h], w.w, w.wp, nq, q2, off);
                    }
                }
            }
        }
        if constexpr (RUN) {
#pragma unroll
            for (int e = 0; e < G; ++e) {
                if constexpr (OUT_REGS) regs[gi * G + e] = v[e];
                else lds[(base + (e << DL)) * ldu + u] = v[e];
            }
        }
    }
}

// Rounds of a size-2^S_LOG sub-transform from stage ST0 on: radix-E rounds,
// the last one shorter when log2(E) does not divide S_LOG.  With kTwPrefetch
// only the twiddle loads run (no barriers).
template <int S_LOG, int ST0, bool FWD, bool SCALE_LAST, int ROW_A, bool LZ = false, int E = kElems,
          int TW = kTwLoad, int SLOT0 = 0>
__device__ __forceinline__ void ntt_rounds_from(uint64_t *lds, int ldu, int u, int t, uint32_t tw_base,
                                                const TwPair *__restrict__ tw, const PrimeConst &pc,
                                                TwPair *cache = nullptr) {
    constexpr int CL = ilog2(E);
    constexpr int C = (S_LOG - ST0) < CL ? (S_LOG - ST0) : CL;
    constexpr bool LAST = ST0 + C == S_LOG;
    ntt_round<S_LOG, ST0, C, FWD, SCALE_LAST && LAST, ROW_A, false, false, LZ, E, TW, SLOT0>(
        lds, ldu, u, t, tw_base, tw, pc, nullptr, cache);
    if constexpr (TW != kTwPrefetch) __syncthreads();
    if constexpr (!LAST)
        ntt_rounds_from<S_LOG, ST0 + C, FWD, SCALE_LAST, ROW_A, LZ, E, TW, SLOT0 + E * C>(lds, ldu, u, t, tw_base,
                                                                                        tw, pc, cache);
}

// ROW_A: 0 for the natural twiddle table; A for a row pass reading the row table
// (which needs exactly two rounds of kElems residues: S_LOG in (kElemsLog, 2 kElemsLog]).
template <int S_LOG, bool FWD, bool SCALE_LAST, int ROW_A = 0, bool LZ = false, int E = kElems, int TW = kTwLoad>
__device__ __forceinline__ void ntt_rounds(uint64_t *lds, int ldu, int u, int t, uint32_t tw_base,
                                           const TwPair *__restrict__ tw, const PrimeConst &pc,
                                           TwPair *cache = nullptr) {
    static_assert(S_LOG >= 5 && S_LOG <= 12, "sub-transform size");
    static_assert(ROW_A == 0 || (E == kElems && S_LOG > kElemsLog && S_LOG <= 2 * kElemsLog),
                  "row table: two rounds of kElems residues");
    ntt_rounds_from<S_LOG, 0, FWD, SCALE_LAST, ROW_A, LZ, E, TW, 0>(lds, ldu, u, t, tw_base, tw, pc, cache);
}

// Plain load of a pass (no prologue).
struct LoadPro {
    const uint64_t *in;
    __device__ __forceinline__ uint64_t operator()(size_t idx) const { return in[idx]; }
};

// Final store of a pass: out[idx] = x.  Passes take the store as a functor, so
// an element-wise step that follows the transform (the ModDown or rescale
// tail) runs in the pass's epilogue instead of another kernel.
struct StoreEpi {
    static constexpr bool kPrefetch = false;
    uint64_t *out;
    __device__ __forceinline__ void operator()(size_t idx, uint64_t x) const { out[idx] = x; }
};

// Passes of launches with few limbs (the INTT of the special-prime limbs before
// ModDown, the INTT of the dropped limb before a rescale): a tile of TILE
// residues (fewer than kTile) and E residues per thread (fewer than kElems), so
// such a launch has enough workgroups for every CU and a shorter chain of
// dependent butterflies per thread; twiddles from the natural table.  Columns:
// U = TILE / 2^A columns of 2^A rows; rows: U rows of 2^B.  Values in the same
// ranges as the kTile passes (forward columns lazy below 4q, forward rows in
// [0, q); inverse rows lazy below 2q, inverse columns in [0, q)).  Ends with a
// barrier.
template <int A, int B, bool FWD, int TILE, int E, typename Pro>
__device__ __forceinline__ void ntt_cols_small_pro(uint64_t *lds, const Pro &pro, uint64_t *out,
                                                   const TwPair *__restrict__ tw, const PrimeConst &pc, int tile) {
    constexpr int U = TILE >> A, LDU = U + 1, NT = TILE / E;
    static_assert(U >= 1 && NT >= 64, "small column tile");
    const int col0 = tile * U;
    uint64_t vin[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int idx = threadIdx.x + r * NT;
        vin[r] = pro(((size_t)(idx / U) << B) + col0 + idx % U);
    }
    TwPair twc[tw_slots(A, E)];
    ntt_rounds<A, FWD, !FWD, 0, false, E, kTwPrefetch>(lds, LDU, threadIdx.x % U, threadIdx.x / U, 1u, tw, pc, twc);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int idx = threadIdx.x + r * NT;
        lds[(idx / U) * LDU + idx % U] = vin[r];
    }
    __syncthreads();
    ntt_rounds<A, FWD, !FWD, 0, false, E, kTwCached>(lds, LDU, threadIdx.x % U, threadIdx.x / U, 1u, tw, pc, twc);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int idx = threadIdx.x + r * NT;
        const uint64_t x = lds[(idx / U) * LDU + idx % U];
        out[((size_t)(idx / U) << B) + col0 + idx % U] = FWD ? x : csub(x, pc.q);
    }
    __syncthreads();
}

template <int A, int B, bool FWD, int TILE, int E>
__device__ __forceinline__ void ntt_cols_small(uint64_t *lds, const uint64_t *in, uint64_t *out,
                                               const TwPair *__restrict__ tw, const PrimeConst &pc, int tile) {
    ntt_cols_small_pro<A, B, FWD, TILE, E>(lds, LoadPro{in}, out, tw, pc, tile);
}

// The result for limb index idx (forward: in [0, q); inverse: lazy in [0, 2q))
// goes through epi(idx, value), or, when Epi::kPrefetch, through
// epi.finish(idx, value, epi.operand(idx)) with the operand loaded at the start.
template <int A, int B, bool FWD, int TILE, int E, typename Pro, typename Epi>
__device__ __forceinline__ void ntt_rows_small_pe(uint64_t *lds, const Pro &pro, const TwPair *__restrict__ tw,
                                                  const PrimeConst &pc, int tile, const Epi &epi) {
    constexpr int S = 1 << B, U = TILE >> B, LDU = U + 1, NT = TILE / E;
    static_assert(U >= 1 && NT >= 64, "small row tile");
    const int row0 = tile * U;
    uint64_t vin[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int idx = threadIdx.x + r * NT;
        vin[r] = pro(((size_t)(row0 + (idx >> B)) << B) + (idx & (S - 1)));
    }
    // an epilogue that reads an operand of its own (the ModDown and rescale
    // tails) has it loaded here, with the tile, instead of after the last
    // barrier: a few registers in a pass of E residues per thread
    uint64_t opnd[E];
    if constexpr (Epi::kPrefetch) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int idx = threadIdx.x + r * NT;
            opnd[r] = epi.operand(((size_t)(row0 + (idx >> B)) << B) + (idx & (S - 1)));
        }
    }
    const int u = threadIdx.x % U;
    TwPair twc[tw_slots(B, E)];
    ntt_rounds<B, FWD, false, 0, false, E, kTwPrefetch>(lds, LDU, u, threadIdx.x / U, (1u << A) + row0 + u, tw, pc,
                                                        twc);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int idx = threadIdx.x + r * NT;
        lds[(idx & (S - 1)) * LDU + (idx >> B)] = vin[r];
    }
    __syncthreads();
    ntt_rounds<B, FWD, false, 0, false, E, kTwCached>(lds, LDU, u, threadIdx.x / U, (1u << A) + row0 + u, tw, pc,
                                                      twc);
    const uint64_t q2 = 2 * pc.q;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int idx = threadIdx.x + r * NT;
        const uint64_t x = lds[(idx & (S - 1)) * LDU + (idx >> B)];
        const size_t gi = ((size_t)(row0 + (idx >> B)) << B) + (idx & (S - 1));
        const uint64_t v = FWD ? csub(csub(x, q2), pc.q) : x;
        if constexpr (Epi::kPrefetch) epi.finish(gi, v, opnd[r]);
        else epi(gi, v);
    }
    __syncthreads();
}

template <int A, int B, bool FWD, int TILE, int E>
__device__ __forceinline__ void ntt_rows_small(uint64_t *lds, const uint64_t *in, uint64_t *out,
                                               const TwPair *__restrict__ tw, const PrimeConst &pc, int tile) {
    ntt_rows_small_pe<A, B, FWD, TILE, E>(lds, LoadPro{in}, tw, pc, tile, StoreEpi{out});
}

// Column pass: sub-transforms are columns (2^A rows, stride 2^B), tile
// `tile` covers 4096 / 2^A consecutive columns.  Forward: the first A stages
// (output lazy in [0, 4q)); inverse: the last A stages with the N^-1 scaling
// (output in [0, q)).  The input residue of limb index idx is pro(idx) (a
// plain load, or an element-wise step that precedes the transform: forward
// inputs may lie anywhere in [0, 4q)).
//
// A pass is split into its loads (ntt_cols_load: the kElems input residues of
// this thread, in registers, prologue included) and the rest
// (ntt_cols_compute): the prologue's temporaries are dead before the transform
// starts, which keeps the multi-pass batched kernels within their register
// budget.
template <int A, int B, bool FWD, typename Pro>
__device__ __forceinline__ void ntt_cols_load(uint64_t (&regs)[kElems], int tile, const Pro &pro) {
    static_assert(A > kElemsLog && A <= 2 * kElemsLog, "two rounds");
    constexpr int U = kTile >> A;
    constexpr int C2 = A - kElemsLog;  // stages of the second round
    const int col0 = tile * U;
    const int u = threadIdx.x % U, t = threadIdx.x / U;
    if constexpr (FWD) {
        // The first forward round works on rows t + e 2^(A-4) of column u, the
        // order in which the tile arrives: it starts from registers.
#pragma unroll
        for (int e = 0; e < kElems; ++e) regs[e] = pro(((size_t)(t + (e << C2)) << B) + col0 + u);
    } else {
#pragma unroll
        for (int r = 0; r < kTile / kThreads; ++r) {
            const int idx = threadIdx.x + r * kThreads;
            regs[r] = pro(((size_t)(idx / U) << B) + col0 + idx % U);
        }
    }
}

// Ends with a barrier, so lds may be reused at once.  LZ: see ct_bfly; the
// forward output is then lazy below (4 + 2A) q.
template <int A, int B, bool FWD, bool LZ>
__device__ __forceinline__ void ntt_cols_compute_t(uint64_t *lds, uint64_t *out, const TwPair *__restrict__ tw,
                                                   const PrimeConst &pc, int tile, uint64_t (&regs)[kElems]) {
    constexpr int S = 1 << A;
    constexpr int U = kTile / S;
    constexpr int LDU = U + 1;
    constexpr int C2 = A - kElemsLog;
    const int col0 = tile * U;
    const int u = threadIdx.x % U, t = threadIdx.x / U;
    if constexpr (FWD) {
        ntt_round<A, 0, kElemsLog, true, false, 0, true, false, LZ>(lds, LDU, u, t, 1u, tw, pc, regs);
        __syncthreads();
        ntt_round<A, kElemsLog, C2, true, false, 0, false, false, LZ>(lds, LDU, u, t, 1u, tw, pc);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kTile / kThreads; ++r) {
            const int idx = threadIdx.x + r * kThreads;
            const int row = idx / U, col = idx % U;
            out[((size_t)row << B) + col0 + col] = lds[row * LDU + col];
        }
    } else {
#pragma unroll
        for (int r = 0; r < kTile / kThreads; ++r) {
            const int idx = threadIdx.x + r * kThreads;
            lds[(idx / U) * LDU + idx % U] = regs[r];
        }
        __syncthreads();
        ntt_round<A, 0, kElemsLog, false, false, 0, false, false, LZ>(lds, LDU, u, t, 1u, tw, pc);
        __syncthreads();
        // The last inverse round leaves rows grp + 16 e (grp = t NG + gi) of
        // column u in registers, the order of a coalesced store.
        ntt_round<A, kElemsLog, C2, false, true, 0, false, true, LZ>(lds, LDU, u, t, 1u, tw, pc, regs);
        constexpr int G = 1 << C2, NG = kElems / G;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi)
#pragma unroll
            for (int e = 0; e < G; ++e) {
                const int row = t * NG + gi + (e << kElemsLog);
                out[((size_t)row << B) + col0 + u] = csub(regs[gi * G + e], pc.q);
            }
    }
    __syncthreads();
}

// LZOK: the butterflies skip the sum corrections for primes below
// kLazyPrimeBound (the prime is uniform across the workgroup: a scalar
// branch).  Worth it only in passes whose prologue or epilogue adds ALU work
// (the two code paths cost registers, so occupancy); the forward column and
// row passes of a limb must agree on it (the column output range differs).
template <int A, int B, bool FWD, bool LZOK = false>
__device__ __forceinline__ void ntt_cols_compute(uint64_t *lds, uint64_t *out, const TwPair *__restrict__ tw,
                                                 const PrimeConst &pc, int tile, uint64_t (&regs)[kElems]) {
    if (LZOK && pc.q < kLazyPrimeBound) ntt_cols_compute_t<A, B, FWD, true>(lds, out, tw, pc, tile, regs);
    else ntt_cols_compute_t<A, B, FWD, false>(lds, out, tw, pc, tile, regs);
}

template <int A, int B, bool FWD, bool LZOK = false, typename Pro>
__device__ __forceinline__ void ntt_cols_unit_pro(uint64_t *lds, uint64_t *out, const TwPair *__restrict__ tw,
                                                  const PrimeConst &pc, int tile, const Pro &pro) {
    uint64_t regs[kElems];
    ntt_cols_load<A, B, FWD>(regs, tile, pro);
    ntt_cols_compute<A, B, FWD, LZOK>(lds, out, tw, pc, tile, regs);
}

template <int A, int B, bool FWD>
__device__ __forceinline__ void ntt_cols_unit(uint64_t *lds, const uint64_t *in, uint64_t *out,
                                              const TwPair *__restrict__ tw, const PrimeConst &pc, int tile) {
    ntt_cols_unit_pro<A, B, FWD>(lds, out, tw, pc, tile, LoadPro{in});
}

// Rescale / modulus-switch lift as the prologue of the NTT of the lifted limb:
// the last limb x (coefficient domain, in [0, q_l)) taken from its centred
// representative into prime q: [x]_q, + (q - [q_l]_q) when x > q_l / 2, lazy in
// [0, 3q).  KEEP_T (BGV): x is first replaced by [x t^-1]_{q_l} and the result
// multiplied by t (lazy in [0, 2q)), so the lift is 0 mod t as well.
template <bool KEEP_T>
struct LiftPro {
    const uint64_t *last;
    uint64_t ql, ql_half, tinv, tinv_p;  // dropped prime q_l, t^-1 mod q_l
    uint64_t q, one_p, corr, tmod, tmod_p;
    __device__ __forceinline__ uint64_t operator()(size_t idx) const {
        uint64_t x = last[idx];
        if (KEEP_T) x = shoup(x, tinv, tinv_p, ql);
        uint64_t r = x - mulhi64(x, one_p) * q;
        if (x > ql_half) r += corr;
        if (KEEP_T) r = shoup_lazy(r, tmod, tmod_p, q);
        return r;
    }
};

// ModDown base conversion P -> q_i as the prologue of the NTT of target i:
// the K P-limbs y_a (coefficient domain, already multiplied by the input
// factor [(P/p_a)^-1]_{p_a}) give sum_a y_a [P/p_a]_{q_i} + cnt (q_i - [P]_{q_i})
// with cnt the number of y_a above p_a / 2 (centred digits), lazy in [0, 4q).
// KP: the number of special primes K, or 8 for any K <= 8 (runtime K).
template <int KP>
struct ModdownPro {
    const uint64_t *src;  // P-limb 0 of the polynomial; limb a at src + a * stride
    size_t stride;
    uint32_t K;
    uint64_t half[KP], cross[KP];
    uint64_t negp, q, r64, r64_p, one_p;
    __device__ __forceinline__ uint64_t operator()(size_t idx) const {
        MacAcc acc;
        uint64_t cnt = 0;
#pragma unroll
        for (int a = 0; a < KP; ++a) {
            if (KP < 8 || a < (int)K) {
                const uint64_t y = src[a * stride + idx];
                cnt += y > half[a] ? 1u : 0u;
                acc.mac(y, cross[a]);
            }
        }
        acc.add(cnt * negp);
        return reduce128_lazy(acc.value(), q, r64, r64_p, one_p);
    }
};

// Row pass: sub-transforms are rows (2^B contiguous residues), tile `tile`
// covers 4096 / 2^B consecutive rows.  Forward: the last B stages (output in
// [0, q)); inverse: the first B stages (output lazy in [0, 2q)).  The result
// for limb index idx goes through epi(idx, value).  Split into loads and the
// rest like the column pass.
template <int A, int B, typename Pro>
__device__ __forceinline__ void ntt_rows_load(uint64_t (&regs)[kElems], int tile, const Pro &pro) {
    constexpr int S = 1 << B;
    constexpr int U = kTile / S;
    const int row0 = tile * U;
#pragma unroll
    for (int r = 0; r < kTile / kThreads; ++r) {
        const int idx = threadIdx.x + r * kThreads;
        regs[r] = pro(((size_t)(row0 + (idx >> B)) << B) + (idx & (S - 1)));
    }
}

template <int A, int B, bool FWD, bool LZ, typename Epi>
__device__ __forceinline__ void ntt_rows_compute_t(uint64_t *lds, const TwPair *__restrict__ tw, const PrimeConst &pc,
                                                   int tile, const Epi &epi, uint64_t (&regs)[kElems]) {
    constexpr int S = 1 << B;
    constexpr int U = kTile / S;
    constexpr int LDU = U + 1;
    const int row0 = tile * U;
#pragma unroll
    for (int r = 0; r < kTile / kThreads; ++r) {
        const int idx = threadIdx.x + r * kThreads;
        lds[(idx & (S - 1)) * LDU + (idx >> B)] = regs[r];
    }
    __syncthreads();
    const int u = threadIdx.x % U, t = threadIdx.x / U;
    ntt_rounds<B, FWD, false, A, LZ>(lds, LDU, u, t, (1u << A) + row0 + u, tw, pc);
    const uint64_t q2 = 2 * pc.q;
#pragma unroll
    for (int r = 0; r < kTile / kThreads; ++r) {
        const int idx = threadIdx.x + r * kThreads;
        const int row = idx >> B, p = idx & (S - 1);
        uint64_t x = lds[p * LDU + row];
        // LZ values lie below 2^59: one Shoup reduction by 1 brings them to [0, 2q)
        if (LZ) x -= mulhi64(x, pc.one_p) * pc.q;
        if (FWD) x = csub(LZ ? x : csub(x, q2), pc.q);
        epi(((size_t)(row0 + row) << B) + p, x);
    }
    __syncthreads();
}

// LZOK: as for ntt_cols_compute.
template <int A, int B, bool FWD, typename Epi, bool LZOK = false>
__device__ __forceinline__ void ntt_rows_compute(uint64_t *lds, const TwPair *__restrict__ tw, const PrimeConst &pc,
                                                 int tile, const Epi &epi, uint64_t (&regs)[kElems]) {
    if (LZOK && pc.q < kLazyPrimeBound) ntt_rows_compute_t<A, B, FWD, true>(lds, tw, pc, tile, epi, regs);
    else ntt_rows_compute_t<A, B, FWD, false>(lds, tw, pc, tile, epi, regs);
}

template <int A, int B, bool FWD, bool LZOK = false, typename Pro, typename Epi>
__device__ __forceinline__ void ntt_rows_unit_pe(uint64_t *lds, const Pro &pro, const TwPair *__restrict__ tw,
                                                 const PrimeConst &pc, int tile, const Epi &epi) {
    uint64_t regs[kElems];
    ntt_rows_load<A, B>(regs, tile, pro);
    ntt_rows_compute<A, B, FWD, Epi, LZOK>(lds, tw, pc, tile, epi, regs);
}

template <int A, int B, bool FWD, bool LZOK = false, typename Epi>
__device__ __forceinline__ void ntt_rows_unit_epi(uint64_t *lds, const uint64_t *in, const TwPair *__restrict__ tw,
                                                  const PrimeConst &pc, int tile, const Epi &epi) {
    ntt_rows_unit_pe<A, B, FWD, LZOK>(lds, LoadPro{in}, tw, pc, tile, epi);
}

template <int A, int B, bool FWD>
__device__ __forceinline__ void ntt_rows_unit(uint64_t *lds, const uint64_t *in, uint64_t *out,
                                              const TwPair *__restrict__ tw, const PrimeConst &pc, int tile) {
    ntt_rows_unit_epi<A, B, FWD>(lds, in, tw, pc, tile, StoreEpi{out});
}

// HMult: d2 = a1 b1 mod q as the prologue of the INTT of d2 (the inner product
// computes d0, d1 and its own d2 residues from a and b itself), lazy in
// [0, 2q), the range the inverse butterflies accept.
struct TensorPro {
    const uint64_t *a1, *b1;  // limb i of a1, b1
    uint64_t q, r64, r64_p, one_p;
    __device__ __forceinline__ uint64_t operator()(size_t idx) const {
        MacAcc s2;
        s2.mac(a1[idx], b1[idx]);
        return csub(reduce128_lazy(s2.value(), q, r64, r64_p, one_p), 2 * q);
    }
};

// HRotate: sigma_g(a1) as the prologue of its INTT.
struct GatherPro {
    const uint64_t *in;  // limb i of a1
    uint32_t galois, log_n;
    __device__ __forceinline__ uint64_t operator()(size_t idx) const {
        return in[galois_src((uint32_t)idx, galois, log_n)];
    }
};

// ModDown tail as the epilogue of the last forward pass of NTT(conv):
// out = (ip - NTT(conv)) * P^-1 mod q (+ add).  add may alias out.
struct ModdownTailEpi {
    static constexpr bool kPrefetch = false;
    const uint64_t *ip;
    const uint64_t *add;
    uint64_t *out;
    uint64_t pinv, pinv_p, q;
    __device__ __forceinline__ void operator()(size_t idx, uint64_t conv) const {
        uint64_t r = shoup(submod(ip[idx], conv, q), pinv, pinv_p, q);
        if (add) r = addmod(r, add[idx], q);
        out[idx] = r;
    }
};

// The same tail when the inner product already left ip' = ip P^-1 + add:
// out = ip' - NTT(conv) P^-1 mod q (one stream read besides the transform).
struct ModdownFoldEpi {
    // the small-tile row pass loads ip with its tile (operand), then finish
    static constexpr bool kPrefetch = true;
    const uint64_t *ip;
    uint64_t *out;
    uint64_t pinv, pinv_p, q;
    __device__ __forceinline__ void operator()(size_t idx, uint64_t conv) const { finish(idx, conv, ip[idx]); }
    __device__ __forceinline__ uint64_t operand(size_t idx) const { return ip[idx]; }
    __device__ __forceinline__ void finish(size_t idx, uint64_t conv, uint64_t ipv) const {
        out[idx] = submod(ipv, shoup(conv, pinv, pinv_p, q), q);
    }
};

// Rescale / modulus-switch tail as the epilogue of the NTT of the lifted limb:
// out = (in - NTT(lift)) * q_l^-1 mod q.
struct RescaleTailEpi {
    static constexpr bool kPrefetch = true;  // as ModdownFoldEpi
    const uint64_t *in;
    uint64_t *out;
    uint64_t qlinv, qlinv_p, q;
    __device__ __forceinline__ void operator()(size_t idx, uint64_t lift) const { finish(idx, lift, in[idx]); }
    __device__ __forceinline__ uint64_t operand(size_t idx) const { return in[idx]; }
    __device__ __forceinline__ void finish(size_t idx, uint64_t lift, uint64_t inv) const {
        out[idx] = shoup(submod(inv, lift, q), qlinv, qlinv_p, q);
    }
};

// Waves per SIMD the NTT kernels are compiled for.  Measured on MI355X at
// N = 2^16: 4 (a 128-VGPR cap, four workgroups per CU) gains nothing on the row
// pass and makes the column pass spill, so the passes are built for 3.
#ifndef RF_NTT_WAVES_COLS
#define RF_NTT_WAVES_COLS 3
#endif
#ifndef RF_NTT_WAVES_ROWS
#define RF_NTT_WAVES_ROWS 3
#endif
constexpr int kNttWavesCols = RF_NTT_WAVES_COLS;
constexpr int kNttWavesRows = RF_NTT_WAVES_ROWS;
// The forward passes with the ModDown conversion / tail and the rescale lift /
// tail (the lazy butterflies, two code paths): held to 4 waves per SIMD so
// that they share the CUs with a concurrent stream as the other passes do.
#ifndef RF_NTT_WAVES_FUSED
#define RF_NTT_WAVES_FUSED 4
#endif
constexpr int kNttWavesFused = RF_NTT_WAVES_FUSED;

// LDS words a column or row unit needs (the largest tile: 2^8 x 17 padded).
constexpr int kNttLdsWords = 256 * 17;

// Split of log2(N) into the column pass (A stages) and the row pass (B stages).
__host__ __device__ constexpr int ntt_split_a(int log_n) { return (log_n + 1) / 2; }

}  // namespace rf
