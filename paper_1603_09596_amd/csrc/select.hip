// select.hip -- which leaves each query opens (Alg. 2, Sec. 2.3) on gfx950.
//
// Alg. 2 keeps one queue over all trees.  Every tree's root enters at key 0;
// popping an entry descends to a leaf, and each node passed on the way
// leaves its far child behind with key |gap|, gap being the float32
// difference of Eq. (1).  Ties go to the lower tree, then the lower node.
//
// The pop order is a sort by a static per-leaf key.  Write a leaf's chain
// as the root (key 0) followed by the far children on its root path, each
// with its own |gap|.  Its static key is the subsequence of chain entries
// strictly larger than every entry after them (the strictly decreasing
// suffix maxima), compared lexicographically by (|gap|, tree, node), a
// prefix first.  Why: (1) no entry with a smaller chain maximum can wait
// behind a popped one, so pops come in non-decreasing order of the chain
// maximum M; (2) among the leaves of maximum M, every chain entry of key M
// heads a group (the entries below it reached through keys < M), the
// queue empties one group before it pops the next head, and heads come out
// in (tree, node) order because a head found inside a group is a
// descendant, with a larger node index, of that group's head; (3) inside a
// group the same argument applies to the chain below its head.  The head of
// a leaf's group, S1, is the deepest chain entry of key M.
//
// This file computes the set of the B first leaves in that order without a
// sequential queue:
//
//   * a tree walk in which the 64 lanes of a wavefront are 64 queries walking
//     the same tree in lockstep: node loads are uniform (scalar / broadcast),
//     each lane keeps its own M and S1, and the bottom five levels are
//     expanded breadth-first in registers, 32 leaves at a time;
//   * counting walks that narrow each query's threshold to a bin of at most
//     kCollectCap leaves of the first-level key (M, tree, S1) (per-lane
//     histograms in LDS, written out per (query, tree slice) without
//     atomics).  The trees are drawn alike, so the ceil(2B/m)-th smallest M
//     of trees 0 and 1 lies close to the B-th smallest of the forest: a walk
//     over those two trees finds it in bins of 1/8 octave, and one walk over
//     every tree then counts 62 bins of 1/128 octave around it (a quarter
//     octave either way) and the keys below the window.  The estimate only
//     places the window; the counts are exact.  A query whose B-th key falls
//     outside the window, or whose bin still holds more than kCollectCap
//     leaves, continues with exact radix passes over the 64-bit first-level
//     key (7-bit digits);
//   * a final walk that marks every leaf below the bin in the query's leaf
//     bitmap and writes the bin's keys and leaf codes to per-slice offsets
//     of the query's collect buffer (again without atomics); a per-query
//     radix select over those keys finds the threshold, and where the group
//     at the threshold crosses the budget the deeper levels of the static
//     key are computed from the root paths of its leaves, one level at a
//     time, until the group no longer crosses it.
//
// First-level key layout: bits 63..32 = M as float bits (M >= 0, so the bit
// pattern orders like the value), 31..24 = tree, 23..0 = S1 (heap index).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "forest.h"
#include "kernels.h"

namespace gf {

namespace {

constexpr int kWave = 64;
constexpr int kDigitBits = 7;
constexpr int kBins = 1 << kDigitBits;   // 128

// Bins of the sample walk: eff bits >> 20 (exponent and 3 mantissa bits,
// 1/8 octave); of the window walk: eff bits >> 16 (1/128 octave).  Window
// bins 1..62 are centred on the sampled bin.
constexpr int kSampleShift = 20;
constexpr int kWindowShift = 16;
constexpr int kWinBins = 64;          // window bins 1..62 inside, 0 below
constexpr uint32_t kWindowHalf = 31;   // bin 1 lies 31 bins below the centre

// Trees walked by the sample walk: two where the forest has them (the
// estimate's spread over queries shrinks with the sampled leaves).
__host__ __device__ inline int sample_trees(int m) { return m >= 2 ? 2 : 1; }

// Walk one tree for the 64 queries of this wavefront.  Calls
// fn(chunk, M[32], S1[32]) for every group of 2^CH consecutive leaves
// (leaf index = chunk * 2^CH + x), M[] holding each leaf's chain maximum
// as the bit pattern of a float >= +0.  qd: LDS [t][64] query coordinates
// on the split set D; pe/pn: LDS [(H-CH+1)][64] path state.  With ENTRY
// false the heads S1 are not tracked (the array stays undefined).
//
// Child state from the parent's (M, S1), M >= +0, and gap g = q - v: the
// left child is the far one exactly when g >= 0 (including g = -0), with
// key |g|; the right one when g < 0, with key v - q = -g exactly.  The far
// child's M is max(M, key), and it becomes S1 when key >= M (the deepest
// entry attaining the maximum).  For M >= +0 the float maximum equals the
// signed-integer maximum of the bit patterns (a negative float is a
// negative integer, below every M), so M is formed without sign handling;
// S1's comparison uses the key's magnitude bits, so that g = -0 counts as
// key 0.
template <int CH, bool ENTRY, class Fn>
__device__ __forceinline__ void walk_tree(const uint2* __restrict__ nodes, int H,
                                          uint32_t chunk_begin, uint32_t chunk_end,
                                          const float* qd, int32_t* pe, uint32_t* pn, Fn&& fn) {
    const int lane = threadIdx.x & (kWave - 1);
    const int U = H - CH;
    constexpr int NL = 1 << CH;
    // the chunk range is the same for the whole wavefront: node indices are
    // uniform, and the nodes (read-only during the walk) are read through the
    // constant address space, so the loads are scalar
#if defined(__HIP_DEVICE_COMPILE__)
    using cnode = const __attribute__((address_space(4))) uint2;
#else
    using cnode = const uint2;
#endif
    cnode* cnodes = (cnode*)(nodes);
    const uint32_t cb = __builtin_amdgcn_readfirstlane(chunk_begin);
    const uint32_t ce = __builtin_amdgcn_readfirstlane(chunk_end);
    for (uint32_t c = cb; c < ce; ++c) {
        // Upper path: levels h0..U-1 change between chunk c-1 and chunk c.
        int h0 = (c == cb) ? 0 : (U - 1 - __builtin_ctz(c));
        if (c == cb) {
            pe[lane] = 0;
            if (ENTRY) pn[lane] = 0u;
        }
        for (int h = h0; h < U; ++h) {
            const uint32_t v = ((1u << h) - 1u) + (c >> (U - h));
            const uint2 nd = cnodes[v];
            const float qv = qd[nd.y * kWave + lane], sv = __uint_as_float(nd.x);
            const float g = qv - sv;
            const bool go_right = (c >> (U - 1 - h)) & 1u;
            const int32_t e = pe[h * kWave + lane];
            const int32_t kb = __float_as_int(go_right ? sv - qv : g);
            pe[(h + 1) * kWave + lane] = max(e, kb);
            if (ENTRY) {
                const bool near_right = !(g < 0.0f);
                uint32_t en = pn[h * kWave + lane];
                if (go_right != near_right && (kb & 0x7FFFFFFF) >= e) en = 2u * v + 1u + (go_right ? 1u : 0u);
                pn[(h + 1) * kWave + lane] = en;
            }
        }
        // Chunk subtree, breadth-first: level j holds nodes base_j + (c << j) + x.
        int32_t ef[NL];
        uint32_t en[NL];
        ef[0] = pe[U * kWave + lane];
        if (ENTRY) en[0] = pn[U * kWave + lane];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const uint32_t row = ((1u << (U + j)) - 1u) + (c << j);
            cnode* rowp = cnodes + row;
#pragma unroll
            for (int x = (1 << j) - 1; x >= 0; --x) {
                const uint2 nd = rowp[x];
                const float qv = qd[nd.y * kWave + lane], sv = __uint_as_float(nd.x);
                const float g = qv - sv;
                const int32_t e = ef[x];
                const int32_t kl = __float_as_int(g), kr = __float_as_int(sv - qv);
                ef[2 * x] = max(e, kl);
                ef[2 * x + 1] = max(e, kr);
                if (ENTRY) {
                    const bool near_right = !(g < 0.0f);
                    const uint32_t n = en[x];
                    const uint32_t v = row + uint32_t(x);
                    en[2 * x] = (near_right && (kl & 0x7FFFFFFF) >= e) ? 2u * v + 1u : n;
                    en[2 * x + 1] = (!near_right && kr >= e) ? 2u * v + 2u : n;
                }
            }
        }
        fn(c, reinterpret_cast<const uint32_t*>(ef), en);
    }
}

__device__ __forceinline__ uint32_t eff_bits(float eff) { return __float_as_uint(eff) & 0x7FFFFFFFu; }

// eff bits of a walk (already free of the sign bit)

__device__ __forceinline__ uint64_t leaf_key(uint32_t eff, uint32_t tree, uint32_t entry) {
    return (uint64_t(eff) << 32) | (uint64_t(tree) << 24) | uint64_t(entry);
}

// Shared setup of a walk kernel: stage the coordinates of the 64 queries on
// D into LDS (for the isometry variant, those of the query reflected for
// this tree).
__device__ __forceinline__ void stage_query_dims(const SelectArgs& a, int q, uint32_t tree, float* qd) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int j = 0; j < a.t; ++j) {
        float v = 0.0f;
        if (q < a.nq)
            v = a.qt ? a.qt[(int64_t(tree) * a.nq + q) * a.t + j] : a.Q[int64_t(q) * a.ldq + a.D[j]];
        qd[j * kWave + lane] = v;
    }
}

// The eight waves of a walk workgroup serve the same 64 queries (lane =
// query) and split the slice's chunks into eight consecutive ranges; they
// share the staged query coordinates and the histogram (or the collect
// counters), each keeping its own path state.  (Measured at 10,000 queries:
// selection 5.26 ms with four waves, 4.89 with eight, 5.67 with sixteen.)
constexpr int kSelWaves = 8;
constexpr int kSelThreads = kSelWaves * kWave;
constexpr int kSelMinGroups = 1024;

// Workgroups go to the XCDs round-robin; each XCD takes a consecutive run of
// (tree, slice, query group) in that order instead, so that the node rows of
// about m / 8 trees stay in its L2.
__device__ __forceinline__ void walk_ids(uint32_t& qb, uint32_t& tree, uint32_t& z) {
    const uint32_t nx = gridDim.x, ny = gridDim.y, nz = gridDim.z;
    const uint32_t total = nx * ny * nz;
    const uint32_t i = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    const uint32_t x = i % 8u, j = i / 8u, base = total / 8u, rem = total % 8u;
    const uint32_t L = (x < rem) ? x * (base + 1u) + j : rem * (base + 1u) + (x - rem) * base + j;
    qb = L % nx;
    const uint32_t r = L / nx;
    z = r % nz;
    tree = r / nz;
}

__device__ __forceinline__ void wave_chunks(uint32_t nchunks, uint32_t zi, uint32_t& cb, uint32_t& ce) {
    const uint32_t per = (nchunks + gridDim.z - 1) / gridDim.z;
    const uint32_t zb = zi * per;
    const uint32_t ze = min(nchunks, zb + per);
    const uint32_t wper = (ze > zb) ? (ze - zb + kSelWaves - 1) / kSelWaves : 0u;
    const uint32_t w = threadIdx.x / kWave;
    cb = min(ze, zb + w * wper);
    ce = min(ze, cb + wper);
}

// One counting walk (PHASE kPhSample, kPhWindow or kPhRadix) for the
// queries whose next walk it is.  The sample walk counts every leaf of its
// trees, bin 0 taking all keys at or below the window (whose top bin holds
// the bound on every eff).  The window walk counts the leaves inside its 62
// bins, keeps the number below the window in a register (bin 0) and drops
// those above it.  A radix walk counts the leaves under the fixed prefix by
// their next digit.
template <int CH, int PHASE>
__global__ __launch_bounds__(kSelThreads) void k_select_hist(SelectArgs a) {
    extern __shared__ uint32_t smem[];
    const int U = a.H - CH;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    float* qd = reinterpret_cast<float*>(smem);                          // [t][64]
    uint32_t* hist = reinterpret_cast<uint32_t*>(qd + a.t * kWave);      // [64][64] packed u16 pairs
    // path state per wave: eff, and the entry node where a walk tracks it
    constexpr int kPath = (PHASE == kPhRadix) ? 2 : 1;
    int32_t* pe = reinterpret_cast<int32_t*>(hist + (kBins / 2) * kWave) + wave * kPath * (U + 1) * kWave;
    uint32_t* pn = reinterpret_cast<uint32_t*>(pe + (U + 1) * kWave);   // [U+1][64] per wave
    // a compact radix walk serves the listed queries only
    uint32_t wqb, tree, wz;
    walk_ids(wqb, tree, wz);
    const int slot = int(wqb) * kWave + lane;
    const int q = (PHASE == kPhRadix && a.nlist > 0) ? (slot < a.nlist ? int(a.qlist[slot]) : a.nq) : slot;
    const SelState st = (q < a.nq) ? a.state[q] : SelState{};
    const bool active = (q < a.nq) && st.status == kSelSearching && st.phase == uint32_t(PHASE);
    if (!__any(active)) return;   // the same for every wave of the workgroup
    if (wave == 0) stage_query_dims(a, q, tree, qd);
    for (int b = wave; b < kBins / 2; b += kSelWaves) hist[b * kWave + lane] = 0u;
    __syncthreads();
    uint32_t cb, ce;
    wave_chunks(1u << U, wz, cb, ce);
    const uint2* nodes = a.nodes + int64_t(tree) * a.n_internal;
    auto count = [&](uint32_t dgt) {
        atomicAdd(&hist[(dgt >> 1) * kWave + lane], (dgt & 1u) ? 65536u : 1u);
    };
    if (PHASE == kPhSample) {
        const uint32_t base = st.base;
        walk_tree<CH, false>(nodes, a.H, cb, ce, qd, pe, pn,
                             [&](uint32_t, const uint32_t* ef, const uint32_t*) {
                                 if (!active) return;
#pragma unroll
                                 for (int x = 0; x < (1 << CH); ++x) {
                                     const uint32_t v = ef[x] >> kSampleShift;
                                     count(v <= base ? 0u : min(v - base, uint32_t(kBins - 1)));
                                 }
                             });
    } else if (PHASE == kPhWindow) {
        // plain 32-bit counters, kWinBins per lane: bin b = 1..kWinBins-2 holds
        // (E >> kWindowShift) == base + b, bin 0 everything below, bin
        // kWinBins-1 everything above (every leaf is counted, no branch)
        const int base = int(st.base);
        walk_tree<CH, false>(nodes, a.H, cb, ce, qd, pe, pn,
                             [&](uint32_t, const uint32_t* ef, const uint32_t*) {
                                 if (!active) return;
#pragma unroll
                                 for (int x = 0; x < (1 << CH); ++x) {
                                     const int v = int(ef[x] >> kWindowShift);
                                     const int bin = min(max(v - base, 0), kWinBins - 1);
                                     atomicAdd(&hist[bin * kWave + lane], 1u);
                                 }
                             });
    } else {
        const int cs = int(st.cs);
        if (__any(active && cs < 32 + kDigitBits)) {
            // some digit reaches below the eff bits: full keys for every lane
            const int fshift = cs > kDigitBits ? cs - kDigitBits : 0;
            const uint32_t fmask = (1u << (cs - fshift)) - 1u;
            walk_tree<CH, true>(nodes, a.H, cb, ce, qd, pe, pn,
                                [&](uint32_t, const uint32_t* ef, const uint32_t* en) {
                                    if (!active) return;
#pragma unroll
                                    for (int x = 0; x < (1 << CH); ++x) {
                                        const uint64_t K = leaf_key(ef[x], tree, en[x]);
                                        if ((K >> cs) == st.prefix) count(uint32_t(K >> fshift) & fmask);
                                    }
                                });
        } else {
            const int sh = cs - 32 - kDigitBits;
            const uint32_t base = uint32_t(st.prefix) << kDigitBits;
            walk_tree<CH, false>(nodes, a.H, cb, ce, qd, pe, pn,
                                 [&](uint32_t, const uint32_t* ef, const uint32_t*) {
                                     if (!active) return;
#pragma unroll
                                     for (int x = 0; x < (1 << CH); ++x) {
                                         const uint32_t r = (ef[x] >> sh) - base;
                                         if (r < uint32_t(kBins)) count(r);
                                     }
                                 });
        }
    }
    __syncthreads();
    if (!active) return;
    // A radix walk may run zf = gridDim.z / zsplit workgroups per slice (few
    // queries left): those add into the slice's row, which the pick that
    // sent the query here has cleared.
    const int zsplit = a.nslice / a.m;
    const int zf = (PHASE == kPhRadix) ? int(gridDim.z) / zsplit : 1;
    const int slice = int(tree) * (int(gridDim.z) / zf) + int(wz) / zf;
    uint32_t* gh = a.hist + (int64_t(q) * a.nslice + slice) * kBins;
    if (PHASE == kPhWindow) {
        for (int b = wave; b < kBins; b += kSelWaves) gh[b] = b < kWinBins ? hist[b * kWave + lane] : 0u;
        return;
    }
    for (int b = wave; b < kBins / 2; b += kSelWaves) {
        const uint32_t w = hist[b * kWave + lane];
        if (zf > 1) {
            if (w & 0xFFFFu) atomicAdd(&gh[2 * b], w & 0xFFFFu);
            if (w >> 16) atomicAdd(&gh[2 * b + 1], w >> 16);
        } else {
            gh[2 * b] = w & 0xFFFFu;
            gh[2 * b + 1] = w >> 16;
        }
    }
}

// Whether the collect walk marks the whole bin (eff-bit bins only): when more
// than half of it is opened, the finish then clears the rest, which takes
// fewer scattered updates than marking the opened part.
__device__ __forceinline__ bool premark_bin(const SelState& s) {
    const uint32_t cnt = min(s.bincount, uint32_t(kCollectCap));
    return s.cs >= 32u && 2u * (s.budget - s.below) > cnt;
}

// The final walk: marks the leaves below the query's bin and writes the
// bin's leaves to the collect buffer.  A bin fixed on eff bits alone (cs >=
// 32) stores eff bits (u32, first half of the query's key area); a bin that
// reaches into the (tree, entry) bits stores full 64-bit keys.  It is
// launched twice: FULL = false serves the workgroups whose bins are all
// eff-bit bins, FULL = true the others (rare), each with the registers its
// walk needs.
template <int CH, bool FULL>
__global__ __launch_bounds__(kSelThreads) void k_select_collect(SelectArgs a) {
    extern __shared__ uint32_t smem[];
    const int U = a.H - CH;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    float* qd = reinterpret_cast<float*>(smem);                          // [t][64]
    uint32_t* cnt = reinterpret_cast<uint32_t*>(qd + a.t * kWave);       // [64] next collect slot
    constexpr int kPath = FULL ? 2 : 1;
    int32_t* pe = reinterpret_cast<int32_t*>(cnt + kWave) + wave * kPath * (U + 1) * kWave;
    uint32_t* pn = reinterpret_cast<uint32_t*>(pe + (U + 1) * kWave);
    uint32_t wqb, tree, wz;
    walk_ids(wqb, tree, wz);
    const int q = int(wqb) * kWave + lane;
    const bool valid = q < a.nq;
    const SelState st = valid ? a.state[q] : SelState{};
    const bool all = valid && st.status == kSelAll;
    const bool ready = valid && st.status == kSelReady;
    const bool full = ready && st.cs < 32u;
    if (__any(full) != FULL) return;   // the same for every wave of the workgroup
    // this slice's share of the bin starts at coff[q][slice]; the waves take
    // slots from a shared counter (the order of the collected keys is free)
    const int slice = int(tree) * int(gridDim.z) + int(wz);
    if (wave == 0) {
        stage_query_dims(a, q, tree, qd);
        cnt[lane] = ready ? a.coff[int64_t(q) * a.nslice + slice] : 0u;
    }
    __syncthreads();
    uint32_t cb, ce;
    wave_chunks(1u << U, wz, cb, ce);
    const uint2* nodes = a.nodes + int64_t(tree) * a.n_internal;
    uint64_t* keys = a.ckey + int64_t(q) * a.ccap;
    uint32_t* effs = reinterpret_cast<uint32_t*>(keys);
    uint32_t* codes = a.ccode + int64_t(q) * a.ccap;
    if (FULL) {
        // full-key bounds for every lane: [lo, hi) is the bin, all keys of an
        // exhausted budget lie below lo = ~0
        uint64_t lo = 0, hi = 0;
        if (all) {
            lo = hi = ~0ull;
        } else if (ready) {
            lo = st.prefix << st.cs;
            hi = (st.prefix + 1ull) << st.cs;
        }
        // marked here: below the bin, or below its top where the bin is
        // premarked (an M-bit bin of a query sharing this workgroup with a
        // full-key query: the finish then only clears what it does not take)
        const uint64_t mlo = (ready && premark_bin(st)) ? hi : lo;
        walk_tree<CH, true>(nodes, a.H, cb, ce, qd, pe, pn,
                            [&](uint32_t c, const uint32_t* ef, const uint32_t* en) {
                                if (!valid) return;
                                uint32_t bits = 0;
#pragma unroll
                                for (int x = 0; x < (1 << CH); ++x) {
                                    const uint64_t K = leaf_key(ef[x], tree, en[x]);
                                    bits |= (K < mlo ? 1u : 0u) << x;
                                    if (K - lo < hi - lo) {
                                        const uint32_t pos = atomicAdd(&cnt[lane], 1u);
                                        if (pos < uint32_t(a.ccap)) {
                                            if (full)
                                                keys[pos] = K;
                                            else
                                                effs[pos] = uint32_t(K >> 32);
                                            codes[pos] = (tree << 24) | ((c << CH) + uint32_t(x));
                                        }
                                    }
                                }
                                a.leafbits[(int64_t(tree) * a.W + c) * a.nq + q] = bits;
                            });
    } else {
        // the bin as eff bits [elo, ehi); an exhausted budget takes every
        // leaf (elo above every eff)
        uint32_t elo = 0, ehi = 0;
        if (all) {
            elo = ehi = ~0u;
        } else if (ready) {
            const int r = int(st.cs) - 32;
            elo = uint32_t(st.prefix << r);
            ehi = uint32_t((st.prefix + 1ull) << r);
        }
        const uint32_t width = ehi - elo;
        // marked here: below the bin, or below its top where the bin is premarked
        const uint32_t mlo = (ready && premark_bin(st)) ? ehi : elo;
        walk_tree<CH, false>(nodes, a.H, cb, ce, qd, pe, pn,
                             [&](uint32_t c, const uint32_t* ef, const uint32_t*) {
                                 if (!valid) return;
                                 uint32_t bits = 0;
                                 // leaves from the last down: bits doubles and takes the next bit
#pragma unroll
                                 for (int x = (1 << CH) - 1; x >= 0; --x) {
                                     const uint32_t E = ef[x];
                                     bits = bits + bits + (E < mlo ? 1u : 0u);
                                     if (E - elo < width) {
                                         const uint32_t pos = atomicAdd(&cnt[lane], 1u);
                                         if (pos < uint32_t(a.ccap)) {
                                             effs[pos] = E;
                                             codes[pos] = (tree << 24) | ((c << CH) + uint32_t(x));
                                         }
                                     }
                                 }
                                 a.leafbits[(int64_t(tree) * a.W + c) * a.nq + q] = bits;
                             });
    }
}

// Head S1 of leaf `leaf` of tree `tree` for a query (coordinates on D in
// qd): the deepest entry of its chain whose |gap| equals the chain maximum
// (the root, key 0, when no far-side key reaches it).  The same float32 gaps
// as the walk.  The path follows from the leaf index alone, so all node
// loads are independent.
__device__ uint32_t head_node(const SelectArgs& a, const float* qd, uint32_t tree, uint32_t leaf) {
    const uint2* nodes = a.nodes + int64_t(tree) * a.n_internal;
    const int H = a.H;
    uint32_t en = 0;
    int32_t e = 0;
#pragma unroll
    for (int h = 0; h < 24; ++h) {   // tree depth is at most 23
        if (h < H) {
            const uint32_t v = ((1u << h) - 1u) + (leaf >> (H - h));
            const uint2 nd = nodes[v];
            const float qv = qd[nd.y], sv = __uint_as_float(nd.x);
            const float g = qv - sv;
            const bool go_right = (leaf >> (H - 1 - h)) & 1u;
            const bool near_right = !(g < 0.0f);
            const int32_t kb = __float_as_int(go_right ? sv - qv : g) & 0x7FFFFFFF;
            if (go_right != near_right && kb >= e) {
                en = 2u * v + 1u + (go_right ? 1u : 0u);
                e = kb;
            }
        }
    }
    return en;
}

// The next level of a leaf's static key below a head it shares with the
// rest of its group: the largest |gap| among the far-side nodes of its path
// strictly below the head node, and the deepest far child attaining it,
// encoded as ((|gap| bits + 1) << 24) | node; 0 when the path has no far
// side below the head (that leaf comes first: it is reached from the head
// by near descents only, and is unique).
__device__ uint64_t next_level_key(const SelectArgs& a, const float* qd, uint32_t tree, uint32_t leaf,
                                   uint32_t head) {
    const uint2* nodes = a.nodes + int64_t(tree) * a.n_internal;
    const int H = a.H;
    const int dh = 31 - __builtin_clz(head + 1u);   // depth of the head
    uint32_t best = 0, node = 0;                    // best = bits + 1 (0: none)
    for (int h = dh; h < H; ++h) {
        const uint32_t v = ((1u << h) - 1u) + (leaf >> (H - h));
        const uint2 nd = nodes[v];
        const float qv = qd[nd.y], sv = __uint_as_float(nd.x);
        const float g = qv - sv;
        const bool go_right = (leaf >> (H - 1 - h)) & 1u;
        const bool near_right = !(g < 0.0f);
        const uint32_t kb = (__float_as_uint(go_right ? sv - qv : g) & 0x7FFFFFFFu) + 1u;
        if (go_right != near_right && kb >= best) {
            best = kb;
            node = 2u * v + 1u + (go_right ? 1u : 0u);
        }
    }
    return best ? (uint64_t(best) << 24) | node : 0ull;
}

// Block-wide step of a radix select over 2^w <= 256 bins (256 threads, all
// calling): with hist[] complete, the bin holding the `left`-th smallest is
// the first whose inclusive prefix count reaches `left`.  The block finds it
// with a prefix sum over the bins (one bin per thread) and publishes the
// extended prefix, the rank left inside that bin and the bin's size in
// out[0..2]; the caller synchronises before reading them.  left = 0 gives
// bin 0, and a total below `left` the last bin with the total subtracted,
// as a bin-by-bin search would.  wsum: 4 words of LDS.
__device__ __forceinline__ void pick_bin(const uint32_t* hist, uint32_t cur, int w, uint32_t left,
                                         uint32_t* out, uint32_t* wsum) {
    const int nb = 1 << w;
    const int t = int(threadIdx.x), lane = t & (kWave - 1), wv = t / kWave;
    const uint32_t v = t < nb ? hist[t] : 0u;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    // the bins lie in the first four waves (the later ones of a wider
    // workgroup hold none)
    if (lane == kWave - 1 && wv < 4) wsum[wv] = incl;
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (int k = 0; k < 4; ++k) {
        const uint32_t ws = wsum[k];
        if (k < wv) base += ws;
        total += ws;
    }
    incl += base;
    const uint32_t excl = incl - v;
    if (left == 0u) {
        if (t == 0) { out[0] = cur << w; out[1] = 0u; out[2] = hist[0]; }
    } else if (total < left) {
        if (t == 0) { out[0] = (cur << w) | uint32_t(nb - 1); out[1] = left - total; out[2] = hist[nb - 1]; }
    } else if (t < nb && excl < left && incl >= left) {
        out[0] = (cur << w) | uint32_t(t);
        out[1] = left - excl;
        out[2] = v;
    }
}

}  // namespace

// Isometry variant (Sec. 2.1 "Rotation", Sec. 2.2): one thread per (query,
// tree), mp >= m lanes per query side by side, forms u.q in FP64 in index order,
// each product rounded before it is added (no fused multiply-add, the same
// sums as the build), then each coordinate on D of the reflected query,
// rounded once to float32.  UT is [d][m], so the lanes of one query read one
// row of it and one value of the query at each step.
__global__ void k_reflect_queries(const float* Q, int64_t ldq, int nq, int d, int m, int mp, int t,
                                  const int32_t* D, const double* UT, float* qt) {
#pragma clang fp contract(off)
    const int tree = int(threadIdx.x) % mp;
    const int q = int(blockIdx.x) * (int(blockDim.x) / mp) + int(threadIdx.x) / mp;
    if (q >= nq || tree >= m) return;
    const float* x = Q + int64_t(q) * ldq;
    double acc = 0.0;
    for (int j = 0; j < d; ++j) {
        const double prod = UT[int64_t(j) * m + tree] * double(x[j]);
        acc = acc + prod;
    }
    for (int j = 0; j < t; ++j) {
        const int s = D[j];
        const double r = (2.0 * acc) * UT[int64_t(s) * m + tree];
        qt[(int64_t(tree) * nq + q) * t + j] = float(double(x[s]) - r);
    }
}

// Per-query initialisation: budget and state.  Every gap's split value lies
// within its slot's range, and float subtraction is monotone, so no eff
// exceeds gmax = max over slots of |q - lo| and |q - hi|: the sample walk's
// bins end at gmax's bin and reach 127 bins (15.9 octaves) below it.  (The
// pass-through nodes of jittered trees, value +inf, are left out of the
// ranges: the leaves behind them have infinite keys, fall into the top bin
// and lie beyond the budget, which is capped at the trees' own leaves.)
__global__ void k_select_init(SelectArgs a, int32_t checks, const int32_t* cpq, double eps,
                              uint32_t* flags) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {   // the radix-pass flag and list count of k_select_pick
        flags[0] = 0u;
        flags[1] = 0u;
    }
    if (q >= a.nq) return;
    const int64_t c = cpq ? int64_t(cpq[q]) : int64_t(checks);
    // Alg. 2 checks leaves while l < c/(1+eps): ceil(c/(1+eps)) of them.
    int64_t B = int64_t(ceil(double(c) / (1.0 + eps)));
    const int64_t total = int64_t(a.m) << a.H;
    if (B > a.leaves) B = a.leaves;
    if (B < 0) B = 0;
    float gmax = 0.0f;
    const int ntq = a.qt ? a.m : 1;    // the isometry variant: every tree's reflected query
    for (int i = 0; i < ntq; ++i)
        for (int j = 0; j < a.t; ++j) {
            const float v = a.qt ? a.qt[(int64_t(i) * a.nq + q) * a.t + j] : a.Q[int64_t(q) * a.ldq + a.D[j]];
            const float2 r = a.drange[j];
            gmax = fmaxf(gmax, fmaxf(fabsf(v - r.x), fabsf(v - r.y)));
        }
    const uint32_t top = eff_bits(gmax) >> kSampleShift;
    SelState s{};
    s.budget = uint32_t(B);
    s.cs = 63;
    s.phase = kPhSample;
    s.base = top > uint32_t(kBins - 1) ? top - uint32_t(kBins - 1) : 0u;
    s.status = (B == total) ? kSelAll : (B == 0 ? kSelDone : kSelSearching);
    a.state[q] = s;
}

// The decision after a counting walk for one query, given the bin totals:
//   sample: place the window on the bin of the ceil(ns B/m)-th smallest eff
//           of the ns sampled trees (or go to radix passes if that bin is
//           the lowest one);
//   window: fix the 1/128-octave bin of the B-th key if it is inside the
//           window, else start radix passes from the top of the key;
//   radix:  fix the digit holding the B-th key.
// A query whose bin holds at most kCollectCap leaves is ready (ready_bin is
// set to the bin).  Returns whether the query's next walk is a radix pass; such queries set
// flags[0] and are listed in qlist at positions counted in flags[1].
__device__ bool pick_one(const SelectArgs& a, int phase, SelState s, const uint32_t* tot,
                         uint32_t* flags, int& ready_bin) {
    const int q = blockIdx.x;
    const uint32_t ns = uint32_t(sample_trees(a.m));
    // the sample covers ns of the m trees: aim at the same share of its leaves
    const uint32_t target = (phase == kPhSample)
                                ? uint32_t((uint64_t(s.budget) * ns + uint32_t(a.m) - 1u) / uint32_t(a.m))
                                : s.budget;
    uint32_t cum = s.below;
    int dgt = kBins - 1;
    for (int b = 0; b < kBins; ++b) {
        if (cum + tot[b] >= target) { dgt = b; break; }
        cum += tot[b];
    }
    bool radix = false;
    if (phase == kPhSample) {
        if (dgt == 0) {
            s.phase = kPhRadix;
            radix = true;
        } else {
            // centre: the target's place inside the sampled bin, by its rank
            // there (linear in the bin's 16 window bins)
            constexpr int kRatio = kSampleShift - kWindowShift;
            const uint32_t within =
                min(uint32_t((uint64_t(target - cum) << kRatio) / max(tot[dgt], 1u)), (1u << kRatio) - 1u);
            const uint32_t centre = ((s.base + uint32_t(dgt)) << kRatio) + within;
            s.base = (centre > kWindowHalf ? centre - kWindowHalf : 1u) - 1u;
            s.phase = kPhWindow;
        }
    } else if (phase == kPhWindow && (dgt == 0 || dgt >= kWinBins - 1)) {
        // outside the window: radix passes from the top (cs 63, prefix 0, below 0)
        s.phase = kPhRadix;
        radix = true;
    } else {
        if (phase == kPhWindow) {
            s.prefix = uint64_t(s.base) + uint64_t(dgt);   // eff bits >> kWindowShift
            s.cs = 32u + kWindowShift;
            s.phase = kPhRadix;
        } else {
            const uint32_t shift = s.cs > uint32_t(kDigitBits) ? s.cs - kDigitBits : 0u;
            s.prefix = (s.prefix << (s.cs - shift)) | uint64_t(dgt);
            s.cs = shift;
        }
        s.below = cum;
        s.bincount = tot[dgt];
        if (s.bincount <= uint32_t(kCollectCap) || s.cs == 0u) {
            s.status = kSelReady;
            ready_bin = dgt;
        } else {
            radix = true;
        }
    }
    if (radix) {
        atomicOr(&flags[0], 1u);
        // the list holds nq entries; a pass adds each query at most once,
        // and the count starts at 0 (k_select_init, or a reset per pass)
        const uint32_t slot = atomicAdd(&flags[1], 1u);
        if (slot < uint32_t(a.nq)) a.qlist[slot] = uint32_t(q);
    }
    a.state[q] = s;
    return radix;
}

// After a counting walk: for the queries it served, sum each bin over the
// slices (one workgroup per query, blockDim.x / kBins threads per bin, at
// most kPickParts, each taking every blockDim.x / kBins-th slice) and move
// the query on (pick_one).  A query that
// is ready gets the offsets at which each slice writes its share of the bin:
// an exclusive prefix sum over the slices (in wave 0).
constexpr int kPickParts = 4;
static_assert(kPickThreads == kPickParts * kBins, "kPickParts threads per bin");
__global__ __launch_bounds__(kPickThreads) void k_select_pick(SelectArgs a, int phase, uint32_t* flags) {
    __shared__ uint32_t part[kPickParts][kBins];
    __shared__ uint32_t tot[kBins];
    __shared__ int again, rbin;
    const int q = blockIdx.x;
    const SelState s = a.state[q];
    if (s.status != kSelSearching || s.phase != uint32_t(phase)) return;
    uint32_t* h = a.hist + int64_t(q) * a.nslice * kBins;
    const int b = int(threadIdx.x) % kBins, pp = int(threadIdx.x) / kBins;
    const int parts = int(blockDim.x) / kBins;
    // the sample walk writes the first ns * (nslice / ns) slices
    const int ns = sample_trees(a.m);
    const int nsl = (phase == kPhSample) ? ns * (a.nslice / ns) : a.nslice;
    uint32_t sum = 0;
#pragma unroll 8
    for (int sl = pp; sl < nsl; sl += parts) sum += h[int64_t(sl) * kBins + b];
    part[pp][b] = sum;
    __syncthreads();
    if (pp == 0) {
        uint32_t t = 0;
        for (int i = 0; i < parts; ++i) t += part[i][b];
        tot[b] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int rb = -1;
        again = pick_one(a, phase, s, tot, flags, rb) ? 1 : 0;
        rbin = rb;
    }
    __syncthreads();
    if (rbin >= 0 && threadIdx.x < kWave) {
        // lane l of wave 0 takes a run of consecutive slices
        const int lane = int(threadIdx.x);
        const int per = (a.nslice + kWave - 1) / kWave;
        const int s0 = min(a.nslice, lane * per), s1 = min(a.nslice, s0 + per);
        uint32_t loc = 0;
#pragma unroll 8
        for (int sl = s0; sl < s1; ++sl) loc += h[int64_t(sl) * kBins + rbin];
        uint32_t inc = loc;   // inclusive scan of the runs over the lanes
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t v = __shfl_up(inc, o);
            if (lane >= o) inc += v;
        }
        uint32_t off = inc - loc;
        for (int sl = s0; sl < s1; ++sl) {
            a.coff[int64_t(q) * a.nslice + sl] = off;
            off += h[int64_t(sl) * kBins + rbin];
        }
    }
    // a query that goes on to a radix pass gets cleared rows (that pass may
    // add into them); each thread clears the slices of bin b it has read
    if (again)
        for (int sl = pp; sl < a.nslice; sl += parts) h[int64_t(sl) * kBins + b] = 0u;
}

// Resolve the bin: exactly (B - below) of the collected leaves are taken
// (marked in the leaf bitmap), those first in the static order.
//   eff-bit bins: a radix select (8-bit digits) over the M bits finds the
//   threshold M*.  If the leaves at M* are not all taken, their (tree, S1)
//   are recomputed from the root paths and a second radix select orders
//   them; the group at the threshold (tree, S1), if it still crosses the
//   budget, goes to the deeper levels.
//   full-key bins: a radix select over the 64-bit first-level keys, then
//   the deeper levels for the group at the threshold key.
// Deeper levels: each leaf of the group gets the next element of its static
// key below the group's head (next_level_key), a radix select over those
// 56-bit values splits the group, and the part at the threshold, if it
// still crosses the budget, repeats one level further down.  A head is
// deeper at every level, so at most H levels run.
constexpr int kFinishUnroll = 4;

namespace {

// Radix select over up to 56-bit values of the collected slots for which
// get(i, v) returns true: finds the value kstar holding the need-th
// smallest (1-based), the rank left of the need-th inside kstar's group and
// that group's size.  All 256 threads call it.
template <class Get>
__device__ void select56(uint32_t cnt, uint32_t need, Get get, uint32_t* hist, uint32_t* pub,
                         uint32_t* wsum, uint64_t* sh_prefix, uint64_t& kstar, uint32_t& left,
                         uint32_t& ties) {
    uint64_t prefix = 0;
    left = need;
    ties = 0;
    for (int shift = 48; shift >= 0; shift -= 8) {
        if (threadIdx.x < 256) hist[threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
            uint64_t v;
            if (get(i, v) && (shift == 48 || (v >> (shift + 8)) == prefix))
                atomicAdd(&hist[(v >> shift) & 255u], 1u);
        }
        __syncthreads();
        pick_bin(hist, 0u, 8, left, pub, wsum);
        __syncthreads();
        if (threadIdx.x == 0) *sh_prefix = (prefix << 8) | pub[0];
        left = pub[1];
        ties = pub[2];
        __syncthreads();
        prefix = *sh_prefix;
        __syncthreads();
    }
    kstar = prefix;
}

}  // namespace

__global__ __launch_bounds__(kFinishThreadsMax) void k_select_finish(SelectArgs a) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t pub[3];
    __shared__ uint32_t wsum[4];
    __shared__ float qd[kMaxT];
    __shared__ uint64_t sh_prefix;
    __shared__ uint32_t sh_need;
    const int q = blockIdx.x;
    const SelState s = a.state[q];
    if (s.status != kSelReady) return;
    const int64_t cap = a.ccap;
    const uint32_t cnt = min(s.bincount, uint32_t(cap));
    const uint32_t need = s.budget - s.below;
    const uint32_t* codes = a.ccode + int64_t(q) * cap;
    auto mark = [&](uint32_t code) {
        const uint32_t tree = code >> 24, leaf = code & 0xFFFFFFu;
        atomicOr(&a.leafbits[(int64_t(tree) * a.W + (leaf >> 5)) * a.nq + q], 1u << (leaf & 31u));
    };
    auto clear = [&](uint32_t code) {
        const uint32_t tree = code >> 24, leaf = code & 0xFFFFFFu;
        atomicAnd(&a.leafbits[(int64_t(tree) * a.W + (leaf >> 5)) * a.nq + q], ~(1u << (leaf & 31u)));
    };
    // the query's coordinates on D for recomputing paths (the isometry
    // variant reads each tree's reflected coordinates from qt instead)
    for (int j = threadIdx.x; j < a.t; j += blockDim.x)
        qd[j] = a.qt ? 0.0f : a.Q[int64_t(q) * a.ldq + a.D[j]];
    __syncthreads();
    auto coords = [&](uint32_t tree) -> const float* {
        return a.qt ? a.qt + (int64_t(tree) * a.nq + q) * a.t : qd;
    };
    // The deeper levels for a group sharing `head` in `tree`, of which the
    // first `left` are taken.  member(i) / store(i, v) / drop(i) access the
    // group's slots; take_i / skip_i apply a decision to slot i.
    auto deeper = [&](uint32_t tree, uint32_t head, uint32_t left, auto member, auto store, auto drop,
                      auto take_i, auto skip_i) {
        const float* cq = coords(tree);
        for (int level = 0; level < 25; ++level) {
            for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
                uint64_t v;
                if (member(i, v)) store(i, next_level_key(a, cq, tree, codes[i] & 0xFFFFFFu, head));
            }
            __syncthreads();
            uint64_t kstar;
            uint32_t l2, t2;
            select56(cnt, left, member, hist, pub, wsum, &sh_prefix, kstar, l2, t2);
            const bool done = l2 == t2;
            for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
                uint64_t v;
                if (!member(i, v)) continue;
                if (v < kstar || (v == kstar && done)) {
                    take_i(i);
                    drop(i);
                } else if (v > kstar) {
                    skip_i(i);
                    drop(i);
                }
            }
            __syncthreads();
            if (done) return;
            head = uint32_t(kstar) & 0xFFFFFFu;
            left = l2;
        }
    };
    if (s.cs < 32u) {
        uint64_t* keys = a.ckey + int64_t(q) * cap;
        if (threadIdx.x == 0) {
            sh_prefix = 0;
            sh_need = need;
        }
        __syncthreads();
        uint64_t kstar = ~0ull;
        uint32_t left = 0, ties = 0;
        if (need < cnt) {
            for (int pass = 0; pass < 8; ++pass) {
                const int shift = 56 - 8 * pass;
                if (threadIdx.x < 256) hist[threadIdx.x] = 0;
                __syncthreads();
                const uint64_t prefix = sh_prefix;
                for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
                    const uint64_t K = keys[i];
                    if (pass == 0 || (K >> (shift + 8)) == prefix)
                        atomicAdd(&hist[(K >> shift) & 255u], 1u);
                }
                __syncthreads();
                pick_bin(hist, 0u, 8, sh_need, pub, wsum);
                __syncthreads();
                left = pub[1];
                ties = pub[2];
                if (threadIdx.x == 0) {
                    sh_need = pub[1];
                    sh_prefix = (prefix << 8) | pub[0];
                }
                __syncthreads();
            }
            kstar = sh_prefix;
        }
        if (kstar == ~0ull || left == ties) {
            for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x)
                if (keys[i] <= kstar) mark(codes[i]);
            return;
        }
        // the group at kstar crosses the budget: decide the rest, then flag
        // the group's slots (bit 63) and hold their deeper keys there
        for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
            const uint64_t K = keys[i];
            if (K < kstar) mark(codes[i]);
            keys[i] = (K == kstar) ? (1ull << 63) : 0ull;
        }
        __syncthreads();
        constexpr uint64_t kFlag = 1ull << 63;
        deeper(uint32_t(kstar >> 24) & 0xFFu, uint32_t(kstar) & 0xFFFFFFu, left,
               [&](uint32_t i, uint64_t& v) { const uint64_t x = keys[i]; v = x & ~kFlag; return (x & kFlag) != 0; },
               [&](uint32_t i, uint64_t v) { keys[i] = kFlag | v; },
               [&](uint32_t i) { keys[i] = 0ull; },
               [&](uint32_t i) { mark(codes[i]); },
               [&](uint32_t) {});
        return;
    }
    uint32_t* effs = reinterpret_cast<uint32_t*>(a.ckey + int64_t(q) * cap);
    // a premarked bin (the collect walk marked all of it) clears the keys
    // above the threshold instead of marking those up to it
    const bool pre = premark_bin(s);
    // the passes over the collected keys take kFinishUnroll keys per thread at
    // a time, their loads issued before any is used
    const uint32_t bstep = blockDim.x;
    if (need >= cnt) {
        if (!pre)
            for (uint32_t i0 = threadIdx.x; i0 < cnt; i0 += kFinishUnroll * bstep) {
                uint32_t cv[kFinishUnroll];
#pragma unroll
                for (int u = 0; u < kFinishUnroll; ++u) {
                    const uint32_t i = i0 + u * bstep;
                    cv[u] = i < cnt ? codes[i] : 0u;
                }
#pragma unroll
                for (int u = 0; u < kFinishUnroll; ++u)
                    if (i0 + u * bstep < cnt) mark(cv[u]);
            }
        return;
    }
    uint32_t* tks = effs + cap;
    // the threshold M*: every collected key has (E >> r) == prefix at r = cs - 32
    uint32_t cur = uint32_t(s.prefix), left = need, ties = cnt;
    for (int r = int(s.cs) - 32; r > 0;) {
        const int w = r < 8 ? r : 8, sh = r - w;
        if (threadIdx.x < 256) hist[threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t i0 = threadIdx.x; i0 < cnt; i0 += kFinishUnroll * bstep) {
            uint32_t ev[kFinishUnroll];
#pragma unroll
            for (int u = 0; u < kFinishUnroll; ++u) {
                const uint32_t i = i0 + u * bstep;
                ev[u] = i < cnt ? effs[i] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kFinishUnroll; ++u)
                if (i0 + u * bstep < cnt && (ev[u] >> r) == cur)
                    atomicAdd(&hist[(ev[u] >> sh) & ((1u << w) - 1u)], 1u);
        }
        __syncthreads();
        pick_bin(hist, cur, w, left, pub, wsum);
        __syncthreads();
        cur = pub[0];
        left = pub[1];
        ties = pub[2];
        r = sh;
        __syncthreads();
    }
    const uint32_t estar = cur;
    if (left == ties) {
        for (uint32_t i0 = threadIdx.x; i0 < cnt; i0 += kFinishUnroll * bstep) {
            uint32_t ev[kFinishUnroll], cv[kFinishUnroll];
#pragma unroll
            for (int u = 0; u < kFinishUnroll; ++u) {
                const uint32_t i = i0 + u * bstep;
                ev[u] = i < cnt ? effs[i] : 0u;
                cv[u] = i < cnt ? codes[i] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kFinishUnroll; ++u) {
                if (i0 + u * bstep >= cnt) continue;
                const bool take = ev[u] <= estar;
                if (pre && !take) clear(cv[u]);
                if (!pre && take) mark(cv[u]);
            }
        }
        return;
    }
    // leaves at M* cross the budget: order them by (tree, S1).  Each thread
    // computes the keys of its own slots once, into the second half of the
    // query's key area, and reads back only those.
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        if (effs[i] != estar) continue;
        const uint32_t code = codes[i], tree = code >> 24;
        tks[i] = (tree << 24) | head_node(a, coords(tree), tree, code & 0xFFFFFFu);
    }
    uint32_t tcur = 0, tties = 0;
    for (int r = 32; r > 0;) {
        const int sh = r - 8;
        if (threadIdx.x < 256) hist[threadIdx.x] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
            if (effs[i] != estar) continue;
            const uint32_t tk = tks[i];
            if (r == 32 || (tk >> r) == tcur) atomicAdd(&hist[(tk >> sh) & 255u], 1u);
        }
        __syncthreads();
        pick_bin(hist, tcur, 8, left, pub, wsum);
        __syncthreads();
        tcur = pub[0];
        left = pub[1];
        tties = pub[2];
        r = sh;
        __syncthreads();
    }
    const bool done = left == tties;
    // decide every slot outside the group at (M*, tcur); flag the group's
    // slots (bit 31 of tks) and hold their deeper keys as (effs, tks & 2^24-1)
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        const uint32_t E = effs[i];
        const uint32_t tk = (E == estar) ? tks[i] : 0u;
        const bool grp = !done && E == estar && tk == tcur;
        if (!grp) {
            const bool take = E < estar || (E == estar && tk <= tcur);
            if (pre && !take) clear(codes[i]);
            if (!pre && take) mark(codes[i]);
        }
        tks[i] = grp ? 0x80000000u : 0u;
    }
    __syncthreads();
    if (done) return;
    deeper(tcur >> 24, tcur & 0xFFFFFFu, left,
           [&](uint32_t i, uint64_t& v) {
               const uint32_t lo = tks[i];
               v = (uint64_t(effs[i]) << 24) | (lo & 0xFFFFFFu);
               return (lo & 0x80000000u) != 0;
           },
           [&](uint32_t i, uint64_t v) {
               effs[i] = uint32_t(v >> 24);
               tks[i] = 0x80000000u | (uint32_t(v) & 0xFFFFFFu);
           },
           [&](uint32_t i) { tks[i] = 0u; },
           [&](uint32_t i) { if (!pre) mark(codes[i]); },
           [&](uint32_t i) { if (pre) clear(codes[i]); });
}

// Each tree is walked in ranges of at most 2^15 leaves (one workgroup per
// range), so that the packed 16-bit histogram counters cannot overflow.  For
// small batches the ranges are cut finer, down to 2^10 leaves (8 chunks of 32
// per wave), until a walk has kSelMinGroups workgroups: a single query
// otherwise walks each tree on one CU.
int select_slices_per_tree(int H, int m, int nq) {
    int z = 1;
    while ((int64_t{1} << H) / z > 32768) z <<= 1;
    const int64_t groups = int64_t((nq + kWave - 1) / kWave) * m;
    while (groups * z < kSelMinGroups && (int64_t{1} << H) / z > 1024) z <<= 1;
    return z;
}

hipError_t launch_select_walk(const SelectArgs& a, int phase, bool collect, hipStream_t st,
                              int zfine) {
    const int CH = a.H < 5 ? a.H : 5;
    const int U = a.H - CH;
    // staged query dims, histogram or collect counters, path state (eff, plus
    // the entry node in walks that may need full keys)
    auto lds_of = [&](bool entry) {
        return size_t(a.t) * kWave * 4 + (collect ? size_t(kWave) * 4 : size_t(kBins / 2) * kWave * 4) +
               size_t(kSelWaves) * (entry ? 2 : 1) * (U + 1) * kWave * 4;
    };
    if (lds_of(true) > 160 * 1024) return hipErrorInvalidValue;
    const int zsplit = select_slices_per_tree(a.H, a.m, a.nq);
    if (a.nslice != a.m * zsplit) return hipErrorInvalidValue;
    // the sample walk covers the first sample_trees(m) trees, in as many
    // slices as a full walk has
    const bool sample = !collect && phase == kPhSample;
    const int ns = sample_trees(a.m);
    const bool fine = !collect && phase == kPhRadix && zfine > 1;
    const int nserved = (!collect && phase == kPhRadix && a.nlist > 0) ? a.nlist : a.nq;
    dim3 grid((nserved + kWave - 1) / kWave, sample ? ns : a.m,
              sample ? a.nslice / ns : (fine ? zsplit * zfine : zsplit));
    auto go = [&](const void* fn, bool entry) {
        const size_t lds = lds_of(entry);
        if (lds > 65536)
            (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        void* args[] = {const_cast<SelectArgs*>(&a)};
        return hipLaunchKernel(fn, grid, dim3(kSelThreads), args, lds, st);
    };
#define GF_WALK(CHV)                                                                         \
    case CHV:                                                                                \
        if (collect) {                                                                       \
            const hipError_t e = go(reinterpret_cast<const void*>(&k_select_collect<CHV, false>), false); \
            if (e != hipSuccess) return e;                                                   \
            return go(reinterpret_cast<const void*>(&k_select_collect<CHV, true>), true);        \
        }                                                                                    \
        if (phase == kPhSample)                                                              \
            return go(reinterpret_cast<const void*>(&k_select_hist<CHV, kPhSample>), false);     \
        if (phase == kPhWindow)                                                              \
            return go(reinterpret_cast<const void*>(&k_select_hist<CHV, kPhWindow>), false);     \
        return go(reinterpret_cast<const void*>(&k_select_hist<CHV, kPhRadix>), true);
    switch (CH) {
        GF_WALK(0) GF_WALK(1) GF_WALK(2) GF_WALK(3) GF_WALK(4) GF_WALK(5)
        default: return hipErrorInvalidValue;
    }
#undef GF_WALK
}

}  // namespace gf
