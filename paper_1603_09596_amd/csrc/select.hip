// select.hip -- which leaves each query opens (Alg. 2, Sec. 2.3) on gfx950.
//
// The queue of Alg. 2 pops entries in the order of the key
//     (eff, tree, node),  eff = max(eff of the entry being descended, |gap|),
// where gap is the float32 difference of Eq. (1) and every tree's root enters
// at eff 0.  Under this order a parent entry always precedes the entries it
// pushes, so the pop sequence is the sorted order of the static per-leaf key
//     K(L) = (eff(L), tree, entry(L)),
// eff(L) being the largest gap on L's root path among the nodes where L lies
// on the far side, and entry(L) the deepest such far child (the root if none).
// The first B pops are therefore the B smallest K(L) over every leaf of the
// forest, and this file computes exactly that set without a sequential queue:
//
//   * a tree walk in which the 64 lanes of a wavefront are 64 queries walking
//     the same tree in lockstep: node loads are uniform (scalar / broadcast),
//     each lane keeps its own eff and entry, and the bottom five levels are
//     expanded breadth-first in registers, 32 leaves at a time;
//   * a radix select on the 64-bit key K (7-bit digits, per-lane histograms
//     in LDS, written out per (query, tree slice) without atomics) that
//     narrows each query's threshold to a bin of at most kCollectCap leaves;
//   * a final walk that marks every leaf below the bin in the query's leaf
//     bitmap and writes the bin's keys to per-slice offsets of the query's
//     collect buffer (again without atomics); a per-query radix select over
//     those keys (8-bit digits, LDS histogram) finds the exact B-th key.
//
// Key layout: bits 63..32 = eff as float bits (eff >= 0, so the bit pattern
// orders like the value), 31..24 = tree, 23..0 = entry node (heap index).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace gf {

namespace {

constexpr int kWave = 64;
constexpr int kDigitBits = 7;
constexpr int kBins = 1 << kDigitBits;   // 128

__device__ __forceinline__ int digit_shift(int pass) { return 56 - kDigitBits * pass; }

// Walk one tree for the 64 queries of this wavefront.  Calls
// fn(chunk, eff[32], entry[32]) for every group of 2^CH consecutive leaves
// (leaf index = chunk * 2^CH + x).  qd: LDS [t][64] query coordinates on the
// split set D; pe/pn: LDS [(H-CH+1)][64] path state.  With ENTRY false the
// entry nodes are not tracked (en[] stays undefined).
//
// Child eff from the parent's eff e >= 0 and gap g: the left child is the far
// one exactly when g >= 0, so its eff is max(e, g) (which is e when g < 0),
// and the right child's is max(e, -g).  Such a value may be -0 where the true
// eff is 0; keys use the eff bits without the sign bit.
template <int CH, bool ENTRY, class Fn>
__device__ __forceinline__ void walk_tree(const uint2* __restrict__ nodes, int H,
                                          uint32_t chunk_begin, uint32_t chunk_end,
                                          const float* qd, float* pe, uint32_t* pn, Fn&& fn) {
    const int lane = threadIdx.x & (kWave - 1);
    const int U = H - CH;
    constexpr int NI = (1 << CH) - 1;
    constexpr int NL = 1 << CH;
    for (uint32_t c = chunk_begin; c < chunk_end; ++c) {
        // Upper path: levels h0..U-1 change between chunk c-1 and chunk c.
        int h0 = (c == chunk_begin) ? 0 : (U - 1 - __builtin_ctz(c));
        if (c == chunk_begin) {
            pe[lane] = 0.0f;
            if (ENTRY) pn[lane] = 0u;
        }
        for (int h = h0; h < U; ++h) {
            const uint32_t v = ((1u << h) - 1u) + (c >> (U - h));
            const uint2 nd = nodes[v];
            const float g = qd[nd.y * kWave + lane] - __uint_as_float(nd.x);
            const bool go_right = (c >> (U - 1 - h)) & 1u;
            const float e = pe[h * kWave + lane];
            pe[(h + 1) * kWave + lane] = go_right ? fmaxf(e, -g) : fmaxf(e, g);
            if (ENTRY) {
                const bool near_right = !(g < 0.0f);
                uint32_t en = pn[h * kWave + lane];
                if (go_right != near_right) en = 2u * v + 1u + (go_right ? 1u : 0u);
                pn[(h + 1) * kWave + lane] = en;
            }
        }
        // Chunk subtree: lane i < NI fetches its i-th node (breadth-first).
        uint32_t mval = 0, mslot = 0;
        if (lane < NI) {
            const int j = 31 - __clz(lane + 1);
            const uint32_t x = uint32_t(lane + 1) - (1u << j);
            const uint32_t v = ((1u << (U + j)) - 1u) + (c << j) + x;
            const uint2 nd = nodes[v];
            mval = nd.x;
            mslot = nd.y;
        }
        float ef[NL];
        uint32_t en[NL];
        ef[0] = pe[U * kWave + lane];
        if (ENTRY) en[0] = pn[U * kWave + lane];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
#pragma unroll
            for (int x = (1 << j) - 1; x >= 0; --x) {
                const int i = (1 << j) - 1 + x;
                const float val = __uint_as_float(__builtin_amdgcn_readlane(mval, i));
                const uint32_t slot = __builtin_amdgcn_readlane(mslot, i);
                const float g = qd[slot * kWave + lane] - val;
                const float e = ef[x];
                ef[2 * x] = fmaxf(e, g);
                ef[2 * x + 1] = fmaxf(e, -g);
                if (ENTRY) {
                    const bool near_right = !(g < 0.0f);
                    const uint32_t n = en[x];
                    const uint32_t v = ((1u << (U + j)) - 1u) + (c << j) + uint32_t(x);
                    en[2 * x] = near_right ? 2u * v + 1u : n;
                    en[2 * x + 1] = near_right ? n : 2u * v + 2u;
                }
            }
        }
        fn(c, ef, en);
    }
}

__device__ __forceinline__ uint32_t eff_bits(float eff) { return __float_as_uint(eff) & 0x7FFFFFFFu; }

__device__ __forceinline__ uint64_t leaf_key(float eff, uint32_t tree, uint32_t entry) {
    return (uint64_t(eff_bits(eff)) << 32) | (uint64_t(tree) << 24) | uint64_t(entry);
}

// Shared setup of a walk kernel: stage q_D of the 64 queries into LDS.
__device__ __forceinline__ void stage_query_dims(const SelectArgs& a, int q, float* qd) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int j = 0; j < a.t; ++j)
        qd[j * kWave + lane] = (q < a.nq) ? a.Q[int64_t(q) * a.ldq + a.D[j]] : 0.0f;
}

// The four waves of a walk workgroup serve the same 64 queries (lane =
// query) and split the slice's chunks into four consecutive ranges; they
// share the staged query coordinates and the histogram (or the collect
// counters), each keeping its own path state.
constexpr int kSelWaves = 4;
constexpr int kSelThreads = kSelWaves * kWave;

__device__ __forceinline__ void wave_chunks(uint32_t nchunks, uint32_t& cb, uint32_t& ce) {
    const uint32_t per = (nchunks + gridDim.z - 1) / gridDim.z;
    const uint32_t zb = blockIdx.z * per;
    const uint32_t ze = min(nchunks, zb + per);
    const uint32_t wper = (ze > zb) ? (ze - zb + kSelWaves - 1) / kSelWaves : 0u;
    const uint32_t w = threadIdx.x / kWave;
    cb = min(ze, zb + w * wper);
    ce = min(ze, cb + wper);
}

template <int CH>
__global__ __launch_bounds__(kSelThreads) void k_select_hist(SelectArgs a, int pass) {
    extern __shared__ uint32_t smem[];
    const int U = a.H - CH;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    float* qd = reinterpret_cast<float*>(smem);                          // [t][64]
    uint32_t* hist = reinterpret_cast<uint32_t*>(qd + a.t * kWave);      // [64][64] packed u16 pairs
    float* pe = reinterpret_cast<float*>(hist + (kBins / 2) * kWave) + wave * 2 * (U + 1) * kWave;
    uint32_t* pn = reinterpret_cast<uint32_t*>(pe + (U + 1) * kWave);   // [U+1][64] per wave
    const int q = blockIdx.x * kWave + lane;
    const uint32_t tree = blockIdx.y;
    const SelState st = (q < a.nq) ? a.state[q] : SelState{};
    const bool active = (q < a.nq) && st.status == kSelSearching;
    if (!__any(active)) return;   // the same for every wave of the workgroup
    if (wave == 0) stage_query_dims(a, q, qd);
    for (int b = wave; b < kBins / 2; b += kSelWaves) hist[b * kWave + lane] = 0u;
    __syncthreads();
    const int shift = digit_shift(pass);
    const uint64_t prefix = st.prefix;
    uint32_t cb, ce;
    wave_chunks(1u << U, cb, ce);
    const uint2* nodes = a.nodes + int64_t(tree) * a.n_internal;
    auto count = [&](uint32_t dgt) {
        atomicAdd(&hist[(dgt >> 1) * kWave + lane], (dgt & 1u) ? 65536u : 1u);
    };
    if (shift >= 32) {
        // the digit and the fixed prefix lie within the eff bits
        const int s32 = shift - 32;
        const uint32_t pfx = uint32_t(prefix);
        walk_tree<CH, false>(nodes, a.H, cb, ce, qd, pe, pn,
                             [&](uint32_t, const float* ef, const uint32_t*) {
                                 if (!active) return;
#pragma unroll
                                 for (int x = 0; x < (1 << CH); ++x) {
                                     const uint32_t E = eff_bits(ef[x]);
                                     if ((E >> (s32 + kDigitBits)) == pfx)
                                         count((E >> s32) & (kBins - 1));
                                 }
                             });
    } else {
        walk_tree<CH, true>(nodes, a.H, cb, ce, qd, pe, pn,
                            [&](uint32_t, const float* ef, const uint32_t* en) {
                                if (!active) return;
#pragma unroll
                                for (int x = 0; x < (1 << CH); ++x) {
                                    const uint64_t K = leaf_key(ef[x], tree, en[x]);
                                    if ((K >> (shift + kDigitBits)) == prefix)
                                        count(uint32_t(K >> shift) & (kBins - 1));
                                }
                            });
    }
    __syncthreads();
    if (!active) return;
    const int slice = int(tree) * int(gridDim.z) + int(blockIdx.z);
    uint32_t* gh = a.hist + (int64_t(q) * a.nslice + slice) * kBins;
    for (int b = wave; b < kBins / 2; b += kSelWaves) {
        const uint32_t w = hist[b * kWave + lane];
        gh[2 * b] = w & 0xFFFFu;
        gh[2 * b + 1] = w >> 16;
    }
}

template <int CH>
__global__ __launch_bounds__(kSelThreads) void k_select_collect(SelectArgs a) {
    extern __shared__ uint32_t smem[];
    const int U = a.H - CH;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    float* qd = reinterpret_cast<float*>(smem);                          // [t][64]
    uint32_t* cnt = reinterpret_cast<uint32_t*>(qd + a.t * kWave);       // [64] next collect slot
    float* pe = reinterpret_cast<float*>(cnt + kWave) + wave * 2 * (U + 1) * kWave;
    uint32_t* pn = reinterpret_cast<uint32_t*>(pe + (U + 1) * kWave);
    const int q = blockIdx.x * kWave + lane;
    const uint32_t tree = blockIdx.y;
    const SelState st = (q < a.nq) ? a.state[q] : SelState{};
    const bool all = st.status == kSelAll;
    // Bin [lo, hi): the key range still undecided after the last pass.
    const int shift = digit_shift(int(st.pass) - 1);
    const uint64_t lo = st.pass ? (st.prefix << shift) : 0ull;
    const uint64_t hi = st.pass ? ((st.prefix + 1ull) << shift) : 0ull;
    // this slice's share of the bin starts at coff[q][slice]; the waves take
    // slots from a shared counter (the order of the collected keys is free)
    const int slice = int(tree) * int(gridDim.z) + int(blockIdx.z);
    if (wave == 0) {
        stage_query_dims(a, q, qd);
        cnt[lane] = (q < a.nq && st.status == kSelReady) ? a.coff[int64_t(q) * a.nslice + slice] : 0u;
    }
    __syncthreads();
    uint32_t cb, ce;
    wave_chunks(1u << U, cb, ce);
    const uint2* nodes = a.nodes + int64_t(tree) * a.n_internal;
    walk_tree<CH, true>(nodes, a.H, cb, ce, qd, pe, pn,
                        [&](uint32_t c, const float* ef, const uint32_t* en) {
                            if (q >= a.nq) return;
                            uint32_t bits = 0;
#pragma unroll
                            for (int x = 0; x < (1 << CH); ++x) {
                                const uint64_t K = leaf_key(ef[x], tree, en[x]);
                                if (all || K < lo) {
                                    bits |= 1u << x;
                                } else if (K < hi) {
                                    const uint32_t pos = atomicAdd(&cnt[lane], 1u);
                                    if (pos < uint32_t(kCollectCap)) {
                                        const int64_t o = int64_t(q) * kCollectCap + pos;
                                        a.ckey[o] = K;
                                        a.ccode[o] = (tree << 24) | ((c << CH) + uint32_t(x));
                                    }
                                }
                            }
                            a.leafbits[(int64_t(tree) * a.W + c) * a.nq + q] = bits;
                        });
}

}  // namespace

// Per-query initialisation: budget, state, histogram.
__global__ void k_select_init(SelectArgs a, int32_t checks, const int32_t* cpq, double eps) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nq) return;
    const int64_t c = cpq ? int64_t(cpq[q]) : int64_t(checks);
    // Alg. 2 checks leaves while l < c/(1+eps): ceil(c/(1+eps)) of them.
    int64_t B = int64_t(ceil(double(c) / (1.0 + eps)));
    const int64_t total = int64_t(a.m) << a.H;
    if (B > total) B = total;
    if (B < 0) B = 0;
    SelState s{};
    s.budget = uint32_t(B);
    s.status = (B == total) ? kSelAll : (B == 0 ? kSelDone : kSelSearching);
    a.state[q] = s;
}

// After a histogram pass: fix the digit holding the B-th smallest key (one
// workgroup of 128 threads per query: thread b sums bin b over the slices),
// and the offsets at which each slice will write its share of that bin.
__global__ __launch_bounds__(kBins) void k_select_pick(SelectArgs a, int pass,
                                                       uint32_t* any_searching) {
    __shared__ uint32_t tot[kBins];
    const int q = blockIdx.x;
    SelState s = a.state[q];
    if (s.status != kSelSearching) return;
    const uint32_t* h = a.hist + int64_t(q) * a.nslice * kBins;
    uint32_t sum = 0;
    for (int sl = 0; sl < a.nslice; ++sl) sum += h[int64_t(sl) * kBins + threadIdx.x];
    tot[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x != 0) return;
    uint32_t cum = s.below;
    int dgt = kBins - 1;
    for (int b = 0; b < kBins; ++b) {
        if (cum + tot[b] >= s.budget) { dgt = b; break; }
        cum += tot[b];
    }
    s.below = cum;
    s.bincount = tot[dgt];
    s.prefix = (s.prefix << kDigitBits) | uint64_t(dgt);
    s.pass = uint32_t(pass + 1);
    if (s.bincount <= uint32_t(kCollectCap) || s.pass == uint32_t(kMaxPasses)) {
        s.status = kSelReady;
        uint32_t off = 0;
        for (int sl = 0; sl < a.nslice; ++sl) {
            a.coff[int64_t(q) * a.nslice + sl] = off;
            off += h[int64_t(sl) * kBins + dgt];
        }
    } else {
        atomicOr(any_searching, 1u);
    }
    a.state[q] = s;
}

// Resolve the bin: a radix select (8-bit digits, from the top) over the
// collected keys finds the (B - below)-th smallest; every collected leaf with
// a key up to it is marked.  Keys are distinct, so exactly B leaves end up
// marked in total.
__global__ __launch_bounds__(256) void k_select_finish(SelectArgs a) {
    __shared__ uint32_t hist[256];
    __shared__ uint64_t sh_prefix;
    __shared__ uint32_t sh_need;
    const int q = blockIdx.x;
    const SelState s = a.state[q];
    if (s.status != kSelReady) return;
    const uint32_t cnt = min(s.bincount, uint32_t(kCollectCap));
    const uint64_t* keys = a.ckey + int64_t(q) * kCollectCap;
    const uint32_t* codes = a.ccode + int64_t(q) * kCollectCap;
    if (threadIdx.x == 0) {
        sh_prefix = 0;
        sh_need = s.budget - s.below;
    }
    __syncthreads();
    uint64_t kstar = ~0ull;
    if (sh_need < cnt) {
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            hist[threadIdx.x] = 0;
            __syncthreads();
            const uint64_t prefix = sh_prefix;
            for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
                const uint64_t K = keys[i];
                if (pass == 0 || (K >> (shift + 8)) == prefix)
                    atomicAdd(&hist[(K >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t need = sh_need, d = 255;
                for (uint32_t b = 0; b < 256; ++b) {
                    if (hist[b] >= need) { d = b; break; }
                    need -= hist[b];
                }
                sh_need = need;
                sh_prefix = (prefix << 8) | d;
            }
            __syncthreads();
        }
        kstar = sh_prefix;
    }
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        if (keys[i] <= kstar) {
            const uint32_t tree = codes[i] >> 24, leaf = codes[i] & 0xFFFFFFu;
            atomicOr(&a.leafbits[(int64_t(tree) * a.W + (leaf >> 5)) * a.nq + q], 1u << (leaf & 31u));
        }
    }
}

// Each tree is walked in ranges of at most 2^15 leaves (one workgroup per
// range), so that the packed 16-bit histogram counters cannot overflow.
int select_slices_per_tree(int H) {
    int z = 1;
    while ((int64_t{1} << H) / z > 32768) z <<= 1;
    return z;
}

hipError_t launch_select_walk(const SelectArgs& a, int pass, bool collect, hipStream_t st) {
    const int CH = a.H < 5 ? a.H : 5;
    const int U = a.H - CH;
    const size_t lds = size_t(a.t) * kWave * 4 + (collect ? size_t(kWave) * 4 : size_t(kBins / 2) * kWave * 4) +
                       size_t(kSelWaves) * 2 * (U + 1) * kWave * 4;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int zsplit = select_slices_per_tree(a.H);
    if (a.nslice != a.m * zsplit) return hipErrorInvalidValue;
    dim3 grid((a.nq + kWave - 1) / kWave, a.m, zsplit);
#define GF_WALK(CHV)                                                                         \
    case CHV:                                                                                \
        if (collect) {                                                                       \
            if (lds > 65536)                                                                 \
                (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_select_collect<CHV>), \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)); \
            hipLaunchKernelGGL(k_select_collect<CHV>, grid, dim3(kSelThreads), lds, st, a);  \
        } else {                                                                             \
            if (lds > 65536)                                                                 \
                (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_select_hist<CHV>), \
                                          hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)); \
            hipLaunchKernelGGL(k_select_hist<CHV>, grid, dim3(kSelThreads), lds, st, a, pass); \
        }                                                                                    \
        break;
    switch (CH) {
        GF_WALK(0) GF_WALK(1) GF_WALK(2) GF_WALK(3) GF_WALK(4) GF_WALK(5)
        default: return hipErrorInvalidValue;
    }
#undef GF_WALK
    return hipGetLastError();
}

}  // namespace gf
