// tile.hip -- the BF16 selection score of many queries at once, on MFMA.
//
// When a batch of queries opens a large share of the forest's leaves, the
// candidate tiles of different queries overlap heavily: at 10,000 queries
// over 10^6 points with ~57% of the points candidates of each query, every
// 64-point tile is a candidate tile of essentially every query block.  The
// scores ||x||^2 - 2 q.x of a (128-query x 64-point) tile are then one
// MFMA product (v_mfma_f32_16x16x32_bf16, FP32 accumulation), computed once
// for the block instead of once per query from gathered rows.  The forest
// decides which of those scores count: a score enters a query's best list
// only if the point is set in that query's visited bitmap (its candidate
// set, Sec. 2.3).  The result is the reduced-precision selection of the
// per-query path, followed by the same FP32 re-rank and FP64 tie re-check.
//
//   k_open_transpose  opened-leaf words (32 leaves of one query each) -> one
//                    row per (tree, leaf) of the bits of the queries that
//                    opened it, in chunks of up to 1024 queries.
//   k_expand_points  one row per point: the OR of the rows of the m leaves
//                    holding it = the queries having the point as candidate.
//   k_tile_bf16      grid (query blocks of 128, point splits): the waves work in
//                    pairs on 32 queries each, one wave of a pair holding the
//                    BF16 rows' even k steps and the other the odd ones in
//                    registers as MFMA A operands, so every B fragment read
//                    from LDS feeds two MFMAs; 64-point x 256-k stages of X
//                    stream into three LDS buffers with direct global->LDS
//                    loads (two stages in flight) as B operands.  After a tile
//                    the two waves swap half their partial sums through LDS,
//                    and each finishes 16 queries after the next tile's first
//                    barrier: the epilogue masks by the candidate bits and
//                    keeps, per query and split, the `cap` best (score, id)
//                    pairs in registers, ordered across the 16 lanes that
//                    hold that query's row of the MFMA result (three each).
//                    The splits of a query block share bounds on its cap-th
//                    best score (a full list's worst, and each split's
//                    ceil(cap / nsplit)-th best) that let them skip points.
//   k_merge_rerank   one workgroup per query: best `kk` over the splits, then
//                    FP32 compensated re-rank and FP64 tie re-check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"
#include "rank.h"

namespace gf {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTWaves = 8;
constexpr int kTThreads = kTWaves * kWave;
constexpr int kTQ = kTWaves * 16;     // queries per workgroup (32 per wave pair)
constexpr int kTP = 64;               // points per tile
constexpr int kSlots = 3;             // list entries per lane and query (x 16 lanes)
// Tiles between publications of the shared bounds: the atomics are
// vector-memory operations, so the next stage's wait for its loads also
// waits for them, and publishing after every tile's inserts cost more than
// the pruning it bought.
constexpr int kPublishTiles = 16;
constexpr int kExpandThreads = 1024;
constexpr int kXcds = 8;              // XCDs of an MI355X (32 CUs each)

// Order-preserving map of float scores to uint32 (a < b <=> key(a) < key(b)).
__device__ __forceinline__ uint32_t score_key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_score(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// List entries as 64-bit keys: the score's key above the id with its sign bit
// flipped, so that one unsigned comparison is the (score, id) order.  Scores
// are finite and never -0 (a score is a norm minus twice a product, and x - x
// rounds to +0), so the key order is the order entry_before uses.  Key 0
// precedes every entry (the end mark) and kEmpty follows every entry.
constexpr uint64_t kEmpty = ~uint64_t{0};
__device__ __forceinline__ uint64_t entry_key(float s, int id) {
    return (uint64_t(score_key(s)) << 32) | (uint32_t(id) ^ 0x80000000u);
}
__device__ __forceinline__ float entry_score(uint64_t k) { return key_score(uint32_t(k >> 32)); }
__device__ __forceinline__ int entry_id(uint64_t k) { return int(uint32_t(k) ^ 0x80000000u); }

// DPP moves within a quarter-wave (a DPP row): lane c takes lane c + 1
// (c = 15 takes lane 0), and every lane takes lane 0.
__device__ __forceinline__ uint32_t row_next(uint32_t v) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x12F, 0xF, 0xF, false));   // row_ror:15
}
__device__ __forceinline__ uint32_t row_first(uint32_t v) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x150, 0xF, 0xF, false));   // row_newbcast:0
}
__device__ __forceinline__ uint64_t row_next(uint64_t v) {
    return (uint64_t(row_next(uint32_t(v >> 32))) << 32) | row_next(uint32_t(v));
}
__device__ __forceinline__ uint64_t row_first(uint64_t v) {
    return (uint64_t(row_first(uint32_t(v >> 32))) << 32) | row_first(uint32_t(v));
}

// Offer every lane's entry key with cand set to the list of its quarter-wave.
// The 16 lanes 16u..16u+15 share one query's list, kept in order across the
// lanes: position p = 16 j + c (slot j of lane c) holds the entry of rank
// cap - 1 - p, so position 0 is the worst and position cap - 1 the best;
// positions from cap on hold key 0, which precedes every entry and never
// moves.  Each round the four quarters take their lowest pending candidate;
// where it precedes the worst entry (position 0, lane 0 of the quarter), the
// positions below its place take their successor's entry (the worst drops
// out) and its place takes the candidate, all in registers.
__device__ __forceinline__ void quarter_offer(bool cand, uint64_t key, uint64_t (&v)[kSlots]) {
    const int lane = threadIdx.x & (kWave - 1);
    const int quarter = lane >> 4, col = lane & 15;
    uint64_t m = __ballot(cand);
    while (m) {
        const uint32_t qm = uint32_t(m >> (16 * quarter)) & 0xFFFFu;
        const int src = 16 * quarter + (qm ? __builtin_ctz(qm) : 0);
        const uint64_t c = (uint64_t(uint32_t(__shfl(int(key >> 32), src))) << 32) |
                           uint32_t(__shfl(int(uint32_t(key)), src));
        const bool go = (qm != 0) & (c < row_first(v[0]));
        // the entry one position up: the next lane's, or for lane 15 lane 0's
        // of the next slot; past the last slot the end mark
        uint64_t n[kSlots];
#pragma unroll
        for (int j = 0; j < kSlots; ++j) n[j] = row_next(v[j]);
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            const uint64_t u = col < 15 ? n[j] : (j + 1 < kSlots ? n[j + 1] : uint64_t{0});
            const bool keep = (!go) | (v[j] < c);
            v[j] = keep ? v[j] : (u < c ? c : u);
        }
        m &= ~__ballot((qm != 0) & (lane == src));   // each quarter's candidate is done
    }
}

// s_waitcnt immediates (gfx9 encoding: vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[5:4] at 15:14)
constexpr int kWaitVm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | (((n >> 4) & 3) << 14); }
// the same with every LDS access of this wave complete as well (lgkmcnt 0)
constexpr int kWaitVmLds(int n) { return (n & 15) | (7 << 4) | (((n >> 4) & 3) << 14); }

constexpr int kKS = 256;                               // k (bf16 elements) per pipeline stage
constexpr int kNBuf = 3;                               // LDS stages (prefetch distance kNBuf - 1)
constexpr int kStageBytes = kTP * kKS * 2;             // 64 rows x 512 B = 32 KB
constexpr int kUnits = kKS / 8;                        // 16-byte units per staged row
constexpr int kRowsPerInst = kWave / kUnits;           // rows per 1 KB wave instruction
constexpr int kDmaPerWave = kStageBytes / 1024 / kTWaves;   // 4
static_assert(kRowsPerInst * kUnits == kWave && kDmaPerWave * kTWaves * 1024 == kStageBytes, "stage shape");
// epilogue operands per tile (dwords): 4 candidate words per point, the
// points' norms, the block's 128 rows of shared bounds (kBoundWords each)
constexpr int kEpiVis = 0, kEpiNorm = 4 * kTP, kEpiThr = 5 * kTP;
constexpr int kEpi = 5 * kTP + kBoundWords * kTQ;
static_assert(kBoundWords == 4, "one 16-byte load per query's bound row");

typedef __attribute__((address_space(3))) uint32_t lds_u32;

__device__ __forceinline__ uint32_t lds_offset(const void* p) {
    return uint32_t(uintptr_t((const lds_u32*)p));   // generic -> LDS address space
}

__device__ __forceinline__ const void* uniform_ptr(const void* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return reinterpret_cast<const void*>((uint64_t(hi) << 32) | lo);
}

// Direct global -> LDS loads (gfx950 global_load_lds_*): every lane of the
// wave reads `size` bytes at its own global address and the wave writes them
// contiguously at LDS address m0 + lane * size.  They are issued from inline
// assembly so that the compiler does not wait for them before unrelated LDS
// reads; the kernel waits for them itself (s_waitcnt vmcnt) before a barrier.
// dma_16s addresses a uniform base plus a 32-bit per-lane byte offset.
__device__ __forceinline__ void dma_16s(const void* base, uint32_t voff, uint32_t lds) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
                 :: "v"(voff), "s"(base), "{m0}"(__builtin_amdgcn_readfirstlane(lds)) : "memory");
}
__device__ __forceinline__ void dma_16(const void* g, uint32_t lds) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :: "v"(g), "{m0}"(__builtin_amdgcn_readfirstlane(lds)) : "memory");
}
__device__ __forceinline__ void dma_4(const void* g, uint32_t lds) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dword %0, off"
                 :: "v"(g), "{m0}"(__builtin_amdgcn_readfirstlane(lds)) : "memory");
}
// Device-scope variants (sc1: served by L2, not a CU cache) for values that
// other workgroups update with atomics during the kernel.
__device__ __forceinline__ void dma_4_dev(const void* g, uint32_t lds) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dword %0, off sc1"
                 :: "v"(g), "{m0}"(__builtin_amdgcn_readfirstlane(lds)) : "memory");
}
__device__ __forceinline__ void dma_16_dev(const void* g, uint32_t lds) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off sc1"
                 :: "v"(g), "{m0}"(__builtin_amdgcn_readfirstlane(lds)) : "memory");
}

// KSTEPS k steps of 32 (the row length rounded up; steps past the row have
// zero A operands), in stages of kKS per tile.  Waves w and w + 4 form pair
// w & 3 over queries 32 (w & 3) .. + 32 of the block; wave half = w >> 2
// holds the k steps of parity `half` of both 16-query groups.
template <int KSTEPS>
__global__ __launch_bounds__(kTThreads) void k_tile_bf16(TileArgs a) {
    static_assert(KSTEPS % 2 == 0, "the k steps split evenly between the waves of a pair");
    constexpr int kSteps = kKS / 32;
    constexpr int kHalf = kSteps / 2;            // k steps per wave and stage
    constexpr int KH = KSTEPS / 2;               // k steps per wave and tile
    constexpr int NC = (KSTEPS + kSteps - 1) / kSteps;
    // X stages: row r of a stage holds its kUnits k units (16 B each) at
    // positions unit ^ (r & 15), so the contiguous 1 KB writes of the direct
    // loads and the 16-row B-operand reads are both free of bank conflicts.
    __shared__ __attribute__((aligned(1024))) uint16_t xs[kNBuf * kStageBytes / 2];
    __shared__ __attribute__((aligned(1024))) uint32_t epi[2][kEpi];
    // partial sums handed to the other wave of the pair: [wave][block][lane]
    __shared__ __attribute__((aligned(16))) f4 xch[kTWaves * 4 * kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int pair = wave & 3, half = wave >> 2;
    const int quarter = lane >> 4, col = lane & 15;
    // Workgroups are dispatched to the XCDs round-robin (workgroup i to XCD
    // i % kXcds).  Each XCD takes a consecutive run of the (split, query
    // block) list instead, so the workgroups sharing an L2 stream the same
    // split's rows at about the same time.
    int qblk, split;
    {
        const int nqb = (a.nq + kTQ - 1) / kTQ;
        const int total = nqb * a.nsplit;
        const int i = int(blockIdx.x), x = i % kXcds, j = i / kXcds;
        const int base = total / kXcds, rem = total % kXcds;
        const int L = (x < rem) ? x * (base + 1) + j : rem * (base + 1) + (x - rem) * base + j;
        split = L / nqb;
        qblk = L - split * nqb;
    }
    const int qp = qblk * kTQ + pair * 32;       // the pair's first query
    const int q0 = qp + 16 * half;               // the 16 queries this wave finishes
    const int ks = int(a.ld16 / 32);

    // A operands: group g's query row qp + 16 (g ^ half) + col (group 0 is
    // the one this wave finishes), k step S = 2 j + half, elements
    // k = 32 S + 8 quarter .. + 8
    bf16x8 qa[2][KH];
    {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int qrow = qp + 16 * (g ^ half) + col;
#pragma unroll
            for (int j = 0; j < KH; ++j) {
                const int S = 2 * j + half;
                if (qrow < a.nq && S < ks) {
                    const uint4 v = *reinterpret_cast<const uint4*>(a.Q16 + int64_t(qrow) * a.ld16 +
                                                                    32 * S + 8 * quarter);
                    qa[g][j] = __builtin_bit_cast(bf16x8, v);
                } else {
                    qa[g][j] = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
                }
            }
        }
    }
    // the A operands are complete before any direct load is issued, so the
    // compiler has no pending load of its own to wait for inside the loop
    __builtin_amdgcn_s_waitcnt(kWaitVm(0));
    // the lists of this lane's four queries: kSlots positions each (position
    // 16 j + col in slot j), in registers, ordered from the worst entry at
    // position 0.  Positions from the capacity on hold the end mark 0, which
    // precedes every entry, so a list keeps its cap best.
    uint64_t lk[4][kSlots];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < kSlots; ++j) lk[i][j] = 16 * j + col >= a.cap ? uint64_t{0} : kEmpty;

    const int64_t pb = int64_t(split) * a.split_pts;
    const int npts = int((pb + a.split_pts < a.n) ? a.split_pts : a.n - pb);
    const int ntile = (npts + kTP - 1) / kTP;
    const uint32_t xs0 = lds_offset(xs), epib = lds_offset(epi);
    const void* xbase = uniform_ptr(a.X16 + pb * a.ld16);
    const uint32_t rowbytes = uint32_t(a.ld16) * 2u;
    // this block's 128 queries: words wo .. wo + 3 of query chunk qc
    const int qc = (4 * qblk) / a.cw, wo = (4 * qblk) % a.cw;
    const uint32_t* visb = a.visT + (int64_t(qc) * a.n + pb) * a.cw + wo;

    // This wave's share of a stage: instructions inst = wave + kTWaves j each
    // load rows kRowsPerInst inst ..; lane l loads k unit
    // (l % kUnits) ^ (row & 15) of row kRowsPerInst inst + l / kUnits.  Rows
    // past the split and k past the row are clamped to valid addresses; that
    // data is never used.  Row kRowsPerInst (wave + kTWaves j) + l / kUnits is
    // 16 j rows past instruction 0's, so every instruction of a lane loads the
    // same k unit.
    static_assert(kRowsPerInst * kTWaves == 16, "instruction j loads rows 16 j past instruction 0's");
    const int drow0 = kRowsPerInst * wave + lane / kUnits;
    const uint32_t dk = uint32_t(((lane % kUnits) ^ (drow0 & 15)) * 8);
    uint32_t trow[kDmaPerWave];
    // B-operand LDS element offsets within a stage for this wave's k step j
    // (stage step 2 j + half; block b adds 16 kKS b): row col, unit
    // u = (4 (2 j + half) + quarter) ^ col.  With y = 4 half + quarter < 8,
    // u = 8 (j ^ (col >> 3)) + (y ^ (col & 7)), so steps j and j + 2 lie
    // 16 units apart and two lane offsets serve all four steps.
    static_assert(kHalf == 4, "four k steps per wave and stage");
    const int lsel0 = col * kKS + 8 * ((4 * half + quarter) ^ (col & 7)) + 64 * (col >> 3);
    const int lsel1 = col * kKS + 8 * ((4 * half + quarter) ^ (col & 7)) + 64 * (1 - (col >> 3));
    auto ldsel = [&](int j) { return ((j & 1) ? lsel1 : lsel0) + 128 * (j >> 1); };

    // issue cursor: the next stage to load is chunk ic of tile it, into ibuf
    int it = 0, ic = 0, ibuf = 0;
    auto set_rows = [&]() {
#pragma unroll
        for (int j = 0; j < kDmaPerWave; ++j) {
            const int r = it * kTP + drow0 + 16 * j;
            trow[j] = uint32_t(r < npts ? r : 0) * rowbytes;
        }
    };
    auto issue_next = [&]() {
        const uint32_t dst = xs0 + uint32_t(ibuf) * kStageBytes;
#pragma unroll
        for (int j = 0; j < kDmaPerWave; ++j) {
            const uint32_t k = uint32_t(ic * kKS) + dk;
            const uint32_t koff = k < uint32_t(a.ld16) ? 2u * k : 0u;
            dma_16s(xbase, trow[j] + koff, dst + uint32_t(wave + kTWaves * j) * 1024u);
        }
        ibuf = (ibuf + 1 == kNBuf) ? 0 : ibuf + 1;
        if (++ic == NC) {
            ic = 0;
            ++it;
            set_rows();
        }
    };
    // wave 0 loads the tile's candidate words, wave 1 its norms, waves 2 and
    // 3 the block's bound rows
    auto issue_epi = [&](int t) {
        const uint32_t epi0 = epib + 4u * kEpi * uint32_t(t & 1);   // this tile's buffer
        const int xl = t * kTP + lane;
        const int xc = xl < npts ? xl : 0;
        if (wave == 0) {
            dma_16(visb + int64_t(xc) * a.cw, epi0 + 4u * kEpiVis);
        } else if (wave == 1) {
            dma_4(a.norm16 + pb + xc, epi0 + 4u * kEpiNorm);
        } else if (wave < 4) {
            const int qq = qblk * kTQ + (wave - 2) * kWave + lane;
            dma_16_dev(a.gthr + kBoundWords * (qq < a.nq ? qq : 0),
                       epi0 + 4u * (kEpiThr + kBoundWords * (wave - 2) * kWave));
        }
    };
    set_rows();
    for (int p = 0; p < kNBuf - 1 && it < ntile; ++p) issue_next();

    const int wv = pair;                            // the pair's candidate word
    const int bit0 = 16 * half + 4 * quarter;       // bit of query q0 + 4 quarter
    f4* const xout = xch + wave * 4 * kWave + lane;
    const int xdelta = half ? -4 * 4 * kWave : 4 * 4 * kWave;   // to the partner's slot
    int buf = 0, left = ntile * NC;                  // stages not yet consumed
    // The epilogue of tile t runs after the first barrier of tile t + 1 (an
    // extra pass t = ntile has only that barrier and the last epilogue): the
    // partial-sum swap needs no barrier of its own, and the epilogue operands
    // alternate between two LDS buffers.
    f4 sum[4];
    for (int t = 0; t <= ntile; ++t) {
        f4 acc[2][4];
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[g][b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            // Loads complete in issue order.  After the current stage's
            // loads, those of min(kNBuf - 2, left - 1) later stages (and
            // possibly the epilogue loads) were issued: waiting down to that
            // many stages' worth completes the current stage for this wave,
            // and the barrier then covers every wave (and frees the previous
            // stage's buffer for reuse).
            // At a tile's first barrier the swap's LDS writes must be done as
            // well, and the previous tile's epilogue loads: with more than one
            // stage per tile a later stage's loads were issued after them, so
            // the wait covers them; with one stage per tile wait for all.
            static_assert(kNBuf == 3, "wait immediates for two stages ahead");
            asm volatile("" ::: "memory");
            if (c == 0 && (NC == 1 || left < 2)) __builtin_amdgcn_s_waitcnt(kWaitVmLds(0));
            else if (c == 0) __builtin_amdgcn_s_waitcnt(kWaitVmLds(kDmaPerWave));
            else if (left >= 2) __builtin_amdgcn_s_waitcnt(kWaitVm(kDmaPerWave));
            else __builtin_amdgcn_s_waitcnt(kWaitVm(0));
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (c == 0 && t > 0) {
                const int tp = t - 1;                          // the tile this epilogue finishes
                uint32_t* const E = epi[tp & 1];               // its operands' buffer
#pragma unroll
                for (int b = 0; b < 4; ++b) sum[b] += xout[xdelta + b * kWave];
                // epilogue: C[row 4 quarter + i][col] of block b = q(row) . x(16 b + col).
                // A point enters a query's list only if it is a candidate of the
                // query and its score is at most both the list's worst and the
                // shared bound (an upper bound on the query's cap-th best over
                // all splits, so nothing it excludes can be in the final lists); the
                // insertion re-checks the exact (score, id) order.
                uint32_t word[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int xl = tp * kTP + 16 * b + col;
                    const uint32_t w = E[kEpiVis + (16 * b + col) * 4 + wv] >> bit0;
                    word[b] = xl < npts ? w : 0u;
                    const float nx = __uint_as_float(E[kEpiNorm + 16 * b + col]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) sum[b][i] = nx - 2.0f * sum[b][i];   // scores
                }
                float lim[4], bm[4];
                bool any = false;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // the list's worst score (NaN, ignored, while the list is not full)
                    // and the shared bound
                    lim[i] = fminf(key_score(row_first(uint32_t(lk[i][0] >> 32))),
                                   key_score(E[kEpiThr + kBoundWords * (q0 - qblk * kTQ + 4 * quarter + i)]));
                    bm[i] = __builtin_inff();
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        bm[i] = (((word[b] >> i) & 1u) && sum[b][i] < bm[i]) ? sum[b][i] : bm[i];
                    any = any || bm[i] <= lim[i];
                }
                // Only queries with a candidate at or below their limit in this tile
                // go through the (rare) insertions, one score at a time.
                if (__ballot(any)) {
                    // the lane's first query, made opaque so that the addresses and
                    // tests derived from it are formed here when needed rather than
                    // held in registers across the whole loop
                    int qme = q0 + 4 * quarter;
                    asm volatile("" : "+v"(qme));
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (!__ballot(bm[i] <= lim[i])) continue;
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int x = int(pb) + tp * kTP + 16 * b + col;
                            const bool cand = ((word[b] >> i) & 1u) && sum[b][i] <= lim[i];
                            quarter_offer(cand, entry_key(sum[b][i], x), lk[i]);
                            lim[i] = fminf(lim[i], key_score(row_first(uint32_t(lk[i][0] >> 32))));
                        }
                    }
                }
                // Every kPublishTiles tiles (and at the last), publish each
                // query's bounds for the other splits: a full list's worst
                // score, and the score of its rank rpub - 1.  Global atomics
                // are counted with the stage loads by the next stage's wait,
                // so they go out in batches rather than after every insert.
                if ((tp % kPublishTiles) == kPublishTiles - 1 || tp == ntile - 1) {
                    int qme = q0 + 4 * quarter;
                    asm volatile("" : "+v"(qme));
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int q = qme + i;
                        uint32_t* br = E + kEpiThr + kBoundWords * (q - qblk * kTQ);   // its bound row
                        uint32_t* gr = a.gthr + int64_t(kBoundWords) * q;
                        const uint32_t wk = uint32_t(lk[i][0] >> 32);   // lane 0: the worst score's key
                        if (col == 0 && q < a.nq && wk < br[0]) atomicMin(gr, wk);
                        if (split < a.nrb) {
                            // Every split holds rpub entries at or below its published
                            // score, so the largest of the nrb scores has nrb rpub >= cap
                            // entries at or below it: a bound on the cap-th best too.
                            // The other splits' scores come from this tile's copy; an
                            // older (larger) score only loosens the bound.
                            // (the lane holding position rpos publishes it)
                            const int rj = a.rpos >> 4;
                            const uint32_t rk = uint32_t((rj == 0 ? lk[i][0] : (rj == 1 ? lk[i][1] : lk[i][2])) >> 32);
                            if (col == (a.rpos & 15) && q < a.nq && rk < br[1 + split]) {
                                atomicMin(gr + 1 + split, rk);
                                // this tile's copy of the row takes the new score (only
                                // this lane reads the rank words of this query), and
                                // words past nrb hold 0
                                br[1 + split] = rk;
                                const uint32_t bk = max(max(br[1], br[2]), br[3]);
                                if (bk < br[0]) atomicMin(gr, bk);
                            }
                        }
                    }
                }
            }
            if (t == ntile) break;
            const uint16_t* xb = xs + buf * (kStageBytes / 2);
            // B fragments run one k step ahead of the MFMAs that use them:
            // block b's next fragment is read as soon as both query groups'
            // MFMAs have taken the current one
            uint4 v[4];
            if (c * kHalf < KH)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    v[b] = *reinterpret_cast<const uint4*>(xb + ldsel(0) + 16 * kKS * b);
            // keep the scheduler from sinking the reads down to their uses
            __builtin_amdgcn_sched_barrier(0);
            // A wave issuing its stage's MFMAs takes issue priority over its
            // SIMD partner while that one is in its epilogue or list inserts.
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int s = 0; s < kHalf; ++s) {
                const int J = c * kHalf + s;
                if (J < KH) {
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
#pragma unroll
                        for (int g = 0; g < 2; ++g)
                            acc[g][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                qa[g][J], __builtin_bit_cast(bf16x8, v[b]), acc[g][b], 0, 0, 0);
                        if (s + 1 < kHalf && J + 1 < KH)
                            v[b] = *reinterpret_cast<const uint4*>(xb + ldsel(s + 1) + 16 * kKS * b);
                    }
                }
                if (s == 0) {
                    // the next loads go out once the MFMA pipe is busy (their
                    // buffer has been free since the barrier)
                    if (it < ntile) issue_next();
                    if (c == 0) issue_epi(t);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            __builtin_amdgcn_s_setprio(0);
            buf = (buf + 1 == kNBuf) ? 0 : buf + 1;
            --left;
        }
        if (t == ntile) break;
        // Swap: this wave hands its partial sums of the other group to its
        // partner, which adds them after the next tile's first barrier, so
        // each score is (even k steps) + (odd k steps) in FP32 whichever wave
        // finishes it.  The partner reads this wave's slot before it reaches
        // the following barrier, and this wave writes it again only after
        // that barrier (with one stage per tile, after an extra barrier).
        if constexpr (NC == 1) {
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            xout[b * kWave] = acc[1][b];
            sum[b] = acc[0][b];
        }
    }
    __builtin_amdgcn_s_waitcnt(kWaitVm(0));
    // the cap best of each query in this split (padding entries written empty)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = q0 + 4 * quarter + i;
        if (q < a.nq) {
            const int64_t base = (int64_t(q) * a.nsplit + split) * kTileList;
#pragma unroll
            for (int j = 0; j < kSlots; ++j) {
                const uint64_t e = lk[i][j];
                const bool pad = e == 0 || e == kEmpty;
                a.part_s[base + col * kSlots + j] = pad ? __builtin_inff() : entry_score(e);
                a.part_i[base + col * kSlots + j] = pad ? 0x7FFFFFFF : entry_id(e);
            }
        }
    }
}

}  // namespace

// Point groups each workgroup of the expansion handles in turn (fewer,
// longer-lived workgroups than one per group).
constexpr int kExpandRepeat = 8;
// Leaf words each workgroup of the transpose handles (one LDS tile each).
constexpr int kTransposeWords = 4;

// Opened leaves, query-major words -> per-leaf rows of query bits.  One
// workgroup of 32 cw threads per (kTransposeWords leaf words from f0, query
// chunk): thread i reads query (chunk 32 cw + i)'s words f0.. (32 leaves
// each), all loads in flight; each half-wave transposes its
// 32 queries x 32 leaves bit matrix, so that lane x (or 32 + x) holds leaf
// x's word of the wave's low (or high) 32 queries; the 32 rows of cw words
// are written whole.  The transpose is five butterfly stages: at width j the
// lanes l and l ^ j swap the off-diagonal j x j blocks of each 2j x 2j block
// (the lane with bit j clear keeps its low halves and takes the partner's
// low halves into its high ones, the other the reverse).
__global__ __launch_bounds__(1024) void k_open_transpose(ExpandArgs a) {
    __shared__ uint32_t tile[kTransposeWords][32 * 32];
    const int64_t words = int64_t(a.m) * a.W;
    const int64_t f0 = int64_t(blockIdx.x) * kTransposeWords;
    const int chunk = blockIdx.y;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int q = chunk * 32 * a.cw + int(threadIdx.x);
    uint32_t bits[kTransposeWords];
#pragma unroll
    for (int u = 0; u < kTransposeWords; ++u)
        bits[u] = (q < a.nq && f0 + u < words) ? a.leafbits[(f0 + u) * a.nq + q] : 0u;
    if (f0 == 0 && q < a.nq) {
        // shared bound +inf; no rank scores yet (words past nrb: 0, no split)
        a.gthr[int64_t(kBoundWords) * q] = 0xFF800000u;
        for (int u = 1; u < kBoundWords; ++u) a.gthr[int64_t(kBoundWords) * q + u] = u <= a.nrb ? 0xFFFFFFFFu : 0u;
    }
    constexpr uint32_t kLow[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int u = 0; u < kTransposeWords; ++u) {
        uint32_t mine = bits[u];
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            const int j = 16 >> s;
            const uint32_t lo = kLow[s];
            const uint32_t y = uint32_t(__shfl_xor(int(mine), j));
            mine = (lane & j) ? ((mine & ~lo) | ((y & ~lo) >> j)) : ((mine & lo) | ((y & lo) << j));
        }
        tile[u][(lane & 31) * a.cw + 2 * wave + (lane >> 5)] = mine;
    }
    __syncthreads();
    const int leaf = int(threadIdx.x) / a.cw, word = int(threadIdx.x) % a.cw;
    const int64_t nleaf = int64_t{1} << a.H;
#pragma unroll
    for (int u = 0; u < kTransposeWords; ++u) {
        const int64_t f = f0 + u;
        const int64_t tree = f / a.W;
        const int64_t lt = (f % a.W) * 32 + leaf;
        if (f < words && lt < nleaf)
            a.openT[((int64_t(chunk) * a.m + tree) * nleaf + lt) * a.cw + word] = tile[u][leaf * a.cw + word];
    }
}

// Point-major candidate sets: row x of chunk c is the OR over the trees of
// the rows of the leaves holding x.  Thread (x, w) of a 256-thread group
// covers 256 / cw points at a time, kExpandRepeat times.  Points are taken
// in tree 0's leaf order, so the points of one tree-0 leaf run together and
// that tree's row is read from memory once and then from L2.
__global__ __launch_bounds__(256) void k_expand_points(ExpandArgs a) {
    const int per = 256 / a.cw;
    const int w = int(threadIdx.x) % a.cw;
    const int chunk = blockIdx.y;
    const int64_t rows = int64_t(a.m) << a.H;
    const uint32_t* op = a.openT + int64_t(chunk) * rows * a.cw + w;
    // Workgroups go to the XCDs round-robin; each XCD takes a consecutive run
    // of point groups instead, so that neighbouring groups (points of nearby
    // leaves, which share leaves in the other trees too) meet in one L2.
    int64_t gblk;
    {
        const int64_t total = gridDim.x, i = blockIdx.x, x = i % kXcds, j = i / kXcds;
        const int64_t base = total / kXcds, rem = total % kXcds;
        gblk = (x < rem) ? x * (base + 1) + j : rem * (base + 1) + (x - rem) * base + j;
    }
    for (int rep = 0; rep < kExpandRepeat; ++rep) {
        const int64_t i = (gblk * kExpandRepeat + rep) * per + threadIdx.x / a.cw;
        if (i >= a.n) return;
        const int64_t x = a.order[i];
        const uint32_t* lf = a.leafof + x * a.m;
        // eight trees at a time: the leaf indices, then the rows, all in flight
        uint32_t v = 0;
        for (int j0 = 0; j0 < a.m; j0 += 8) {
            uint32_t r[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) r[j] = j0 + j < a.m ? lf[j0 + j] : 0u;
            uint32_t o[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) o[j] = j0 + j < a.m ? op[int64_t(r[j]) * a.cw] : 0u;
#pragma unroll
            for (int j = 0; j < 8; ++j) v |= o[j];
        }
        a.visT[(int64_t(chunk) * a.n + x) * a.cw + w] = v;
    }
}

// Best kk over the splits' lists, then the final ranking of the query.
constexpr int kMergeMax = 512;   // the workgroup: up to this many list entries are ranked at once
__global__ __launch_bounds__(kMergeMax) void k_merge_rerank(MergeArgs a) {
    __shared__ float md[kWave];
    __shared__ int mi[kWave];
    __shared__ float mr[kWave];
    const int q = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    WaveList L;
    L.init();
    const int64_t tot = int64_t(a.nsplit) * kTileList;
    const float* ps = a.part_s + int64_t(q) * tot;
    const int* pi = a.part_i + int64_t(q) * tot;
    if (tot <= int64_t(blockDim.x)) {
        // every entry at once: thread e takes the rank of entry e among the
        // filled ones by (score, id); ids are distinct (each point lies in
        // one split), so the ranks below kk give the kk best in order
        __shared__ float es[kMergeMax];
        __shared__ int ei[kMergeMax];
        const int t = int(threadIdx.x);
        float sv = __builtin_inff();
        int iv = 0x7FFFFFFF;
        if (t < tot) { sv = ps[t]; iv = pi[t]; }
        if (t < kMergeMax) { es[t] = sv; ei[t] = iv; }
        if (t < kWave) { md[t] = __builtin_inff(); mi[t] = 0x7FFFFFFF; }
        __syncthreads();
        if (sv < __builtin_inff()) {
            int rank = 0;
            for (int f = 0; f < int(tot); ++f)
                if (es[f] < __builtin_inff() && entry_before(es[f], ei[f], sv, iv)) ++rank;
            if (rank < a.kk) { md[rank] = sv; mi[rank] = iv; }
        }
        __syncthreads();
        if (wave == 0) {
            L.d = lane < a.kk ? md[lane] : __builtin_inff();
            L.id = lane < a.kk ? mi[lane] : 0x7FFFFFFF;
        }
    } else {
        // each wave keeps the kk best of every blockDim.x / kWave-th run of
        // kWave entries; then the waves' lists (at most kMergeMax entries)
        // are ranked at once as above
        __shared__ float es[kMergeMax];
        __shared__ int ei[kMergeMax];
        const int nw = int(blockDim.x) / kWave;
        for (int64_t e0 = int64_t(wave) * kWave; e0 < tot; e0 += int64_t(nw) * kWave) {
            const int64_t e = e0 + lane;
            const float s = e < tot ? ps[e] : __builtin_inff();
            const int id = e < tot ? pi[e] : 0x7FFFFFFF;
            const float td = L.thr_d(a.kk);
            const int tid = L.thr_id(a.kk);
            uint64_t m = __ballot(s < __builtin_inff() && entry_before(s, id, td, tid));
            while (m) {
                const int src = __builtin_ctzll(m);
                m &= m - 1;
                L.offer(__shfl(s, src), __shfl(id, src), a.kk);
            }
        }
        const int t = int(threadIdx.x);
        const float sv = lane < a.kk ? L.d : __builtin_inff();
        const int iv = lane < a.kk ? L.id : 0x7FFFFFFF;
        es[t] = sv;
        ei[t] = iv;
        if (t < kWave) { md[t] = __builtin_inff(); mi[t] = 0x7FFFFFFF; }
        __syncthreads();
        if (sv < __builtin_inff()) {
            int rank = 0;
            for (int f = 0; f < int(blockDim.x); ++f)
                if (es[f] < __builtin_inff() && entry_before(es[f], ei[f], sv, iv)) ++rank;
            if (rank < a.kk) { md[rank] = sv; mi[rank] = iv; }
        }
        __syncthreads();
        if (wave == 0) {
            L.d = lane < a.kk ? md[lane] : __builtin_inff();
            L.id = lane < a.kk ? mi[lane] : 0x7FFFFFFF;
        }
    }
    __syncthreads();
    finish_query(a.rerank, a.kk, a.k, q, a.Q + int64_t(q) * a.ldq, a.X32, a.ld32, a.d, md, mi, mr, L,
                 a.ids, a.dists);
}

// Candidate bits of the tile path, back in query-major form: bit j of word
// w of query q is set when point 32 w + j is a candidate of q in visT (the
// rows k_tile_bf16 masks its scores with).  Thread per (query, word).
__global__ __launch_bounds__(256) void k_vis_to_query_bits(const uint32_t* __restrict__ visT, int nq,
                                                           int64_t n, int cw, int64_t nbmw,
                                                           uint32_t* __restrict__ bits) {
    const int q = blockIdx.y;
    const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= nq || w >= nbmw) return;
    const int chunk = q / (32 * cw), word = (q >> 5) % cw, bit = q & 31;
    uint32_t out = 0;
    for (int j = 0; j < 32; ++j) {
        const int64_t x = w * 32 + j;
        if (x < n) out |= ((visT[(int64_t(chunk) * n + x) * cw + word] >> bit) & 1u) << j;
    }
    bits[int64_t(q) * nbmw + w] = out;
}

// Candidates per query: the population count of its bit row.
__global__ __launch_bounds__(256) void k_count_bits(const uint32_t* __restrict__ bits, int64_t nbmw,
                                                    int64_t* __restrict__ count) {
    __shared__ int64_t part[256 / kWave];
    const int q = blockIdx.x;
    int64_t c = 0;
    for (int64_t w = threadIdx.x; w < nbmw; w += blockDim.x) c += __popc(bits[int64_t(q) * nbmw + w]);
    for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_down(c, o);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int i = 0; i < int(blockDim.x) / kWave; ++i) t += part[i];
        count[q] = t;
    }
}

hipError_t launch_tile_expand(const ExpandArgs& e, hipStream_t st) {
    const int64_t words = int64_t(e.m) * e.W;
    if (e.cw < 4 || e.cw > 32 || (e.cw & (e.cw - 1))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_open_transpose, dim3(unsigned((words + kTransposeWords - 1) / kTransposeWords),
                                              unsigned(e.nchunk)),
                       dim3(32 * e.cw), 0, st, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int per = 256 / e.cw;
    const int64_t per_group = int64_t(per) * kExpandRepeat;
    hipLaunchKernelGGL(k_expand_points, dim3(unsigned((e.n + per_group - 1) / per_group), unsigned(e.nchunk)),
                       dim3(256), 0, st, e);
    return hipGetLastError();
}

hipError_t launch_count_bits(const uint32_t* bits, int nq, int64_t nbmw, int64_t* count, hipStream_t st) {
    if (nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_bits, dim3(unsigned(nq)), dim3(256), 0, st, bits, nbmw, count);
    return hipGetLastError();
}

hipError_t launch_tile_trace(const ExpandArgs& e, uint32_t* cand_bits, int64_t* ncand, hipStream_t st) {
    hipError_t err = launch_tile_expand(e, st);
    if (err != hipSuccess) return err;
    const int64_t nbmw = (e.n + 31) / 32;
    hipLaunchKernelGGL(k_vis_to_query_bits, dim3(unsigned((nbmw + 255) / 256), unsigned(e.nq)), dim3(256), 0,
                       st, static_cast<const uint32_t*>(e.visT), e.nq, e.n, e.cw, nbmw, cand_bits);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (ncand) {
        hipLaunchKernelGGL(k_count_bits, dim3(unsigned(e.nq)), dim3(256), 0, st,
                           static_cast<const uint32_t*>(cand_bits), nbmw, ncand);
        err = hipGetLastError();
    }
    return err;
}

hipError_t launch_tile_path(const ExpandArgs& e, const TileArgs& t, const MergeArgs& m,
                            hipStream_t st, hipEvent_t* ev) {
    if (t.cw != e.cw) return hipErrorInvalidValue;
    if (t.split_pts % kTP || t.split_pts * t.ld16 * 2 >= (int64_t{1} << 31)) return hipErrorInvalidValue;
    hipError_t err = launch_tile_expand(e, st);
    if (err != hipSuccess) return err;
    if (ev && (err = hipEventRecord(ev[0], st)) != hipSuccess) return err;
    dim3 grid(unsigned(((t.nq + kTQ - 1) / kTQ) * t.nsplit));   // 1-D: see the XCD mapping
    const int ks = int(t.ld16 / 32);
#define GF_TILE(KS) \
    else if (ks <= KS) hipLaunchKernelGGL(k_tile_bf16<KS>, grid, dim3(kTThreads), 0, st, t);
    if (ks < 1) return hipErrorInvalidValue;
    GF_TILE(4) GF_TILE(8) GF_TILE(12) GF_TILE(16) GF_TILE(20) GF_TILE(24) GF_TILE(28) GF_TILE(30)
    GF_TILE(32)
    else return hipErrorInvalidValue;
#undef GF_TILE
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (ev && (err = hipEventRecord(ev[1], st)) != hipSuccess) return err;
    return launch_merge(m, st);
}

hipError_t launch_merge(const MergeArgs& m, hipStream_t st) {
    // threads: enough to rank every list entry at once (up to kMergeMax), in whole waves
    const int64_t tot = int64_t(m.nsplit) * kTileList;
    const unsigned mthreads = unsigned(std::min<int64_t>(kMergeMax, std::max<int64_t>(256, (tot + kWave - 1) / kWave * kWave)));
    hipLaunchKernelGGL(k_merge_rerank, dim3(m.nq), dim3(mthreads), 0, st, m);
    return hipGetLastError();
}

}  // namespace gf
