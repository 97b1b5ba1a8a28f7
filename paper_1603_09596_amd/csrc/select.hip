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
//     in LDS) that narrows each query's threshold to a bin of at most
//     kCollectCap leaves;
//   * a final walk that marks every leaf below the bin in the query's leaf
//     bitmap and collects the bin, which a per-query sort resolves.
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
// split set D; pe/pn: LDS [(H-CH+1)][64] path state.
template <int CH, class Fn>
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
            pn[lane] = 0u;
        }
        for (int h = h0; h < U; ++h) {
            const uint32_t v = ((1u << h) - 1u) + (c >> (U - h));
            const uint2 nd = nodes[v];
            const float g = qd[nd.y * kWave + lane] - __uint_as_float(nd.x);
            const bool go_right = (c >> (U - 1 - h)) & 1u;
            const bool near_right = !(g < 0.0f);
            float e = pe[h * kWave + lane];
            uint32_t en = pn[h * kWave + lane];
            if (go_right != near_right) {
                e = fmaxf(e, fabsf(g));
                en = 2u * v + 1u + (go_right ? 1u : 0u);
            }
            pe[(h + 1) * kWave + lane] = e;
            pn[(h + 1) * kWave + lane] = en;
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
        en[0] = pn[U * kWave + lane];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
#pragma unroll
            for (int x = (1 << j) - 1; x >= 0; --x) {
                const int i = (1 << j) - 1 + x;
                const float val = __uint_as_float(__builtin_amdgcn_readlane(mval, i));
                const uint32_t slot = __builtin_amdgcn_readlane(mslot, i);
                const float g = qd[slot * kWave + lane] - val;
                const bool near_right = !(g < 0.0f);
                const float e = ef[x];
                const uint32_t n = en[x];
                const float efar = fmaxf(e, fabsf(g));
                const uint32_t v = ((1u << (U + j)) - 1u) + (c << j) + uint32_t(x);
                ef[2 * x] = near_right ? efar : e;
                en[2 * x] = near_right ? 2u * v + 1u : n;
                ef[2 * x + 1] = near_right ? e : efar;
                en[2 * x + 1] = near_right ? n : 2u * v + 2u;
            }
        }
        fn(c, ef, en);
    }
}

__device__ __forceinline__ uint64_t leaf_key(float eff, uint32_t tree, uint32_t entry) {
    return (uint64_t(__float_as_uint(eff)) << 32) | (uint64_t(tree) << 24) | uint64_t(entry);
}

// Shared setup of a walk kernel: stage q_D of the 64 queries into LDS.
__device__ __forceinline__ void stage_query_dims(const SelectArgs& a, int q, float* qd) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int j = 0; j < a.t; ++j)
        qd[j * kWave + lane] = (q < a.nq) ? a.Q[int64_t(q) * a.ldq + a.D[j]] : 0.0f;
}

template <int CH>
__global__ __launch_bounds__(64) void k_select_hist(SelectArgs a, int pass) {
    extern __shared__ uint32_t smem[];
    float* qd = reinterpret_cast<float*>(smem);                 // [t][64]
    float* pe = qd + a.t * kWave;                               // [U+1][64]
    uint32_t* pn = reinterpret_cast<uint32_t*>(pe + (a.H - CH + 1) * kWave);
    uint32_t* hist = pn + (a.H - CH + 1) * kWave;               // [64][64] packed u16 pairs
    const int lane = threadIdx.x;
    const int q = blockIdx.x * kWave + lane;
    const uint32_t tree = blockIdx.y;
    const SelState st = (q < a.nq) ? a.state[q] : SelState{};
    const bool active = (q < a.nq) && st.status == kSelSearching;
    if (!__any(active)) return;
    stage_query_dims(a, q, qd);
    for (int b = 0; b < kBins / 2; ++b) hist[b * kWave + lane] = 0u;
    const int shift = digit_shift(pass);
    const uint64_t prefix = st.prefix;
    const uint32_t nchunks = 1u << (a.H - CH);
    const uint32_t per = (nchunks + gridDim.z - 1) / gridDim.z;
    const uint32_t cb = blockIdx.z * per;
    const uint32_t ce = min(nchunks, cb + per);
    const uint2* nodes = a.nodes + int64_t(tree) * a.n_internal;
    walk_tree<CH>(nodes, a.H, cb, ce, qd, pe, pn,
                  [&](uint32_t, const float* ef, const uint32_t* en) {
                      if (!active) return;
#pragma unroll
                      for (int x = 0; x < (1 << CH); ++x) {
                          const uint64_t K = leaf_key(ef[x], tree, en[x]);
                          if ((K >> (shift + kDigitBits)) == prefix) {
                              const uint32_t dgt = uint32_t(K >> shift) & (kBins - 1);
                              atomicAdd(&hist[(dgt >> 1) * kWave + lane], (dgt & 1u) ? 65536u : 1u);
                          }
                      }
                  });
    if (!active) return;
    uint32_t* gh = a.hist + int64_t(q) * kBins;
    for (int b = 0; b < kBins / 2; ++b) {
        const uint32_t w = hist[b * kWave + lane];
        if (w & 0xFFFFu) atomicAdd(&gh[2 * b], w & 0xFFFFu);
        if (w >> 16) atomicAdd(&gh[2 * b + 1], w >> 16);
    }
}

template <int CH>
__global__ __launch_bounds__(64) void k_select_collect(SelectArgs a) {
    extern __shared__ uint32_t smem[];
    float* qd = reinterpret_cast<float*>(smem);
    float* pe = qd + a.t * kWave;
    uint32_t* pn = reinterpret_cast<uint32_t*>(pe + (a.H - CH + 1) * kWave);
    const int lane = threadIdx.x;
    const int q = blockIdx.x * kWave + lane;
    const uint32_t tree = blockIdx.y;
    const SelState st = (q < a.nq) ? a.state[q] : SelState{};
    stage_query_dims(a, q, qd);
    const bool all = st.status == kSelAll;
    // Bin [lo, hi): the key range still undecided after the last pass.
    const int shift = digit_shift(int(st.pass) - 1);
    const uint64_t lo = st.pass ? (st.prefix << shift) : 0ull;
    const uint64_t hi = st.pass ? ((st.prefix + 1ull) << shift) : 0ull;
    const uint32_t nchunks = 1u << (a.H - CH);
    const uint32_t per = (nchunks + gridDim.z - 1) / gridDim.z;
    const uint32_t cb = blockIdx.z * per;
    const uint32_t ce = min(nchunks, cb + per);
    const uint2* nodes = a.nodes + int64_t(tree) * a.n_internal;
    uint32_t* col_n = a.ncollect;
    walk_tree<CH>(nodes, a.H, cb, ce, qd, pe, pn,
                  [&](uint32_t c, const float* ef, const uint32_t* en) {
                      if (q >= a.nq) return;
                      uint32_t bits = 0;
#pragma unroll
                      for (int x = 0; x < (1 << CH); ++x) {
                          const uint64_t K = leaf_key(ef[x], tree, en[x]);
                          if (all || K < lo) {
                              bits |= 1u << x;
                          } else if (K < hi) {
                              const uint32_t slot = atomicAdd(&col_n[q], 1u);
                              if (slot < uint32_t(kCollectCap)) {
                                  const int64_t o = int64_t(q) * kCollectCap + slot;
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
    a.ncollect[q] = 0;
    for (int b = 0; b < kBins; ++b) a.hist[int64_t(q) * kBins + b] = 0;
}

// After a histogram pass: fix the digit holding the B-th smallest key.
__global__ void k_select_pick(SelectArgs a, int pass, uint32_t* any_searching) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nq) return;
    SelState s = a.state[q];
    if (s.status != kSelSearching) return;
    uint32_t* h = a.hist + int64_t(q) * kBins;
    uint32_t cum = s.below;
    int dgt = kBins - 1;
    for (int b = 0; b < kBins; ++b) {
        if (cum + h[b] >= s.budget) { dgt = b; break; }
        cum += h[b];
    }
    s.below = cum;
    s.bincount = h[dgt];
    s.prefix = (s.prefix << kDigitBits) | uint64_t(dgt);
    s.pass = uint32_t(pass + 1);
    if (s.bincount <= uint32_t(kCollectCap) || s.pass == uint32_t(kMaxPasses)) {
        s.status = kSelReady;
    } else {
        atomicOr(any_searching, 1u);
    }
    for (int b = 0; b < kBins; ++b) h[b] = 0;
    a.state[q] = s;
}

// Resolve the bin: sort the collected keys, mark the first budget-below.
__global__ __launch_bounds__(256) void k_select_finish(SelectArgs a) {
    __shared__ uint64_t key[kCollectCap];
    __shared__ uint32_t code[kCollectCap];
    const int q = blockIdx.x;
    const SelState s = a.state[q];
    if (s.status != kSelReady) return;
    const uint32_t cnt = min(a.ncollect[q], uint32_t(kCollectCap));
    const uint32_t take = s.budget - s.below;
    uint32_t np2 = 1;
    while (np2 < cnt) np2 <<= 1;
    for (uint32_t i = threadIdx.x; i < np2; i += blockDim.x) {
        if (i < cnt) {
            key[i] = a.ckey[int64_t(q) * kCollectCap + i];
            code[i] = a.ccode[int64_t(q) * kCollectCap + i];
        } else {
            key[i] = ~0ull;
            code[i] = 0;
        }
    }
    __syncthreads();
    for (uint32_t size = 2; size <= np2; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < np2; i += blockDim.x) {
                const uint32_t j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    if ((key[i] > key[j]) == up) {
                        const uint64_t tk = key[i]; key[i] = key[j]; key[j] = tk;
                        const uint32_t tc = code[i]; code[i] = code[j]; code[j] = tc;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < take && i < cnt; i += blockDim.x) {
        const uint32_t tree = code[i] >> 24, leaf = code[i] & 0xFFFFFFu;
        atomicOr(&a.leafbits[(int64_t(tree) * a.W + (leaf >> 5)) * a.nq + q], 1u << (leaf & 31u));
    }
}

hipError_t launch_select_walk(const SelectArgs& a, int pass, bool collect, hipStream_t st) {
    const int CH = a.H < 5 ? a.H : 5;
    const int U = a.H - CH;
    const size_t lds = size_t(a.t) * kWave * 4 + size_t(U + 1) * kWave * 8 +
                       (collect ? 0 : size_t(kBins / 2) * kWave * 4);
    // split each tree into ranges of at most 2^15 leaves (16-bit counters)
    const uint32_t nchunks = 1u << U;
    uint32_t zsplit = 1;
    while ((uint64_t(nchunks) << CH) / zsplit > 32768u) zsplit <<= 1;
    dim3 grid((a.nq + kWave - 1) / kWave, a.m, zsplit);
#define GF_WALK(CHV)                                                                       \
    case CHV:                                                                              \
        if (collect)                                                                       \
            hipLaunchKernelGGL(k_select_collect<CHV>, grid, dim3(kWave), lds, st, a);      \
        else                                                                               \
            hipLaunchKernelGGL(k_select_hist<CHV>, grid, dim3(kWave), lds, st, a, pass);   \
        break;
    switch (CH) {
        GF_WALK(0) GF_WALK(1) GF_WALK(2) GF_WALK(3) GF_WALK(4) GF_WALK(5)
        default: return hipErrorInvalidValue;
    }
#undef GF_WALK
    return hipGetLastError();
}

}  // namespace gf
