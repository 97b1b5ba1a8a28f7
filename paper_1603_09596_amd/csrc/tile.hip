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
//   k_expand        one workgroup per query: opened leaves -> visited bitmap
//                   (LDS), written out as [nq][vw] words.
//   k_tile_bf16     grid (query blocks of 128, point splits): each wave keeps
//                   its 16 queries' BF16 rows in registers as MFMA A operands;
//                   64-point x 256-k tiles of X stream through LDS (double
//                   buffered) as B operands; the epilogue masks by the visited
//                   bits and keeps, per query and split, the 48 best (score,
//                   id) pairs in registers of the 16 lanes that hold that
//                   query's row of the MFMA result.
//   k_merge_rerank  one workgroup per query: best `kk` over the splits, then
//                   FP32 compensated re-rank and FP64 tie re-check.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "rank.h"

namespace gf {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTWaves = 8;
constexpr int kTThreads = kTWaves * kWave;
constexpr int kTQ = kTWaves * 16;     // queries per workgroup
constexpr int kTP = 64;               // points per tile
constexpr int kKC = 256;              // k (bf16 elements) per LDS stage
constexpr int kRowPad = kKC + 8;      // LDS row stride in elements (528 B)
constexpr int kSlots = 3;             // list entries per lane and query (x 16 lanes)
constexpr int kExpandThreads = 1024;

// Lexicographic maximum of (s, i) over the 16 lanes of a quarter-wave.
__device__ __forceinline__ void quarter_max(float& s, int& i) {
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) {
        const float os = __shfl_xor(s, o);
        const int oi = __shfl_xor(i, o);
        if (entry_before(s, i, os, oi)) { s = os; i = oi; }
    }
}

// Offer every lane's (sc, id) with cand set to the list of its quarter-wave.
// The 16 lanes 16u..16u+15 share one query's list of 48 entries in LDS
// (lane c owns entries 3c..3c+2, unsorted) and keep its current worst entry
// (ts, ti) in registers.  The four quarters insert in parallel; a candidate
// replaces the worst entry when it precedes it.
__device__ __forceinline__ void quarter_offer(bool cand, float sc, int id, float* rs, int* ri,
                                              float& ts, int& ti) {
    const int lane = threadIdx.x & (kWave - 1);
    const int quarter = lane >> 4, col = lane & 15;
    uint64_t m = __ballot(cand);
    while (m) {
        const uint32_t qm = uint32_t(m >> (16 * quarter)) & 0xFFFFu;
        const int src = 16 * quarter + (qm ? __builtin_ctz(qm) : 0);
        const float cs = __shfl(sc, src);
        const int ci = __shfl(id, src);
        const bool ins = qm != 0 && entry_before(cs, ci, ts, ti);
        float vs[kSlots];
        int vi[kSlots];
        int slot = -1;
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            vs[j] = rs[col * kSlots + j];
            vi[j] = ri[col * kSlots + j];
            if (vs[j] == ts && vi[j] == ti) slot = j;
        }
        const uint64_t hb = __ballot(ins && slot >= 0);
        const uint32_t hq = uint32_t(hb >> (16 * quarter)) & 0xFFFFu;
        if (ins && hq && col == __builtin_ctz(hq)) {
#pragma unroll
            for (int j = 0; j < kSlots; ++j)
                if (j == slot) {
                    vs[j] = cs; vi[j] = ci;
                    rs[col * kSlots + j] = cs;
                    ri[col * kSlots + j] = ci;
                }
        }
        float ws = vs[0];
        int wi = vi[0];
#pragma unroll
        for (int j = 1; j < kSlots; ++j)
            if (entry_before(ws, wi, vs[j], vi[j])) { ws = vs[j]; wi = vi[j]; }
        quarter_max(ws, wi);
        if (ins) { ts = ws; ti = wi; }
        uint64_t low = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t mq = (m >> (16 * u)) & 0xFFFFull;
            low |= (mq & (~mq + 1)) << (16 * u);
        }
        m &= ~low;
    }
}

template <int KSTEPS>
__global__ __launch_bounds__(kTThreads) void k_tile_bf16(TileArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[2][kTP * kRowPad];
    __shared__ float lst_s[kTWaves * 16 * kTileList];   // per wave: 16 queries x 48 entries
    __shared__ int lst_i[kTWaves * 16 * kTileList];
    __shared__ uint32_t epi_vis[2 * kTQ];    // visited words of the tile: [query][half]
    __shared__ float epi_norm[kTP];          // squared norms of the tile's points
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int quarter = lane >> 4, col = lane & 15;
    const int q0 = blockIdx.x * kTQ + wave * 16;
    const int ks = int(a.ld16 / 32);
    const int nchunks = int((a.ld16 + kKC - 1) / kKC);

    // A operands: query row q0 + col, elements k = 32 s + 8 quarter .. + 8
    bf16x8 qa[KSTEPS];
    {
        const int qrow = q0 + col;
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s) {
            if (qrow < a.nq && s < ks) {
                const uint4 v = *reinterpret_cast<const uint4*>(a.Q16 + int64_t(qrow) * a.ld16 +
                                                                32 * s + 8 * quarter);
                qa[s] = __builtin_bit_cast(bf16x8, v);
            } else {
                qa[s] = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
            }
        }
    }
    // list of query row r of this wave: lst_*[(wave * 16 + r) * 48 ..]
    float ts[4];
    int ti[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        ts[i] = __builtin_inff();
        ti[i] = 0x7FFFFFFF;
        const int base = (wave * 16 + 4 * quarter + i) * kTileList + col * kSlots;
#pragma unroll
        for (int j = 0; j < kSlots; ++j) { lst_s[base + j] = __builtin_inff(); lst_i[base + j] = 0x7FFFFFFF; }
    }

    const int64_t pb = int64_t(blockIdx.y) * a.split_pts;
    const int64_t pe = (pb + a.split_pts < a.n) ? pb + a.split_pts : a.n;
    const int64_t ntile = (pe > pb) ? (pe - pb + kTP - 1) / kTP : 0;
    constexpr int kMaxChunks = (KSTEPS * 32 + kKC - 1) / kKC;

    // X tiles stream through two LDS buffers; stage s (tile s / nchunks,
    // chunk s % nchunks) is computed from buffer s & 1 while stage s + 1 is
    // being fetched, across tile boundaries too.
    auto load_chunk = [&](int64_t p0, int c, uint4 (&r)[4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = threadIdx.x + kTThreads * j;   // 16-byte unit, 32 per row
            const int row = e >> 5, c16 = e & 31;
            const int64_t x = p0 + row;
            const int64_t k = int64_t(c) * kKC + c16 * 8;
            r[j] = (x < pe && k < a.ld16)
                       ? *reinterpret_cast<const uint4*>(a.X16 + x * a.ld16 + k)
                       : make_uint4(0, 0, 0, 0);
        }
    };
    auto store_chunk = [&](int buf, const uint4 (&r)[4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = threadIdx.x + kTThreads * j;
            const int row = e >> 5, c16 = e & 31;
            *reinterpret_cast<uint4*>(&xs[buf][row * kRowPad + c16 * 8]) = r[j];
        }
    };
    if (ntile > 0) {
        uint4 r[4];
        load_chunk(pb, 0, r);
        store_chunk(0, r);
    }
    __syncthreads();
    int stage = 0;
    for (int64_t t = 0; t < ntile; ++t) {
        const int64_t p0 = pb + t * kTP;
        // operands of this tile's epilogue, fetched ahead of the MFMA loop
        // (one per thread): the visited words of the 128 queries for points
        // p0..p0+31 and p0+32..p0+63, and the squared norms of the 64 points
        uint32_t pre = 0;
        {
            const int tid = threadIdx.x;
            if (tid < 2 * kTQ) {
                const int qq = blockIdx.x * kTQ + (tid >> 1);
                const int64_t x = p0 + 32 * (tid & 1);
                pre = (qq < a.nq && x < pe) ? a.vis[int64_t(qq) * a.vw + (x >> 5)] : 0u;
            } else if (tid < 2 * kTQ + kTP) {
                const int64_t x = p0 + (tid - 2 * kTQ);
                pre = (x < pe) ? __float_as_uint(a.norm16[x]) : 0u;
            }
        }
        f4 acc[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < kMaxChunks; ++c) {
            if (c < nchunks) {
                const bool last = (c + 1 == nchunks);
                const bool more = !last || (t + 1 < ntile);
                uint4 nxt[4];
                if (more) load_chunk(last ? p0 + kTP : p0, last ? 0 : c + 1, nxt);
                const uint16_t* xb = xs[stage & 1];
#pragma unroll
                for (int s = 0; s < kKC / 32; ++s) {
                    const int S = c * (kKC / 32) + s;
                    if (S < KSTEPS && S < ks) {
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const uint4 v = *reinterpret_cast<const uint4*>(
                                xb + (16 * b + col) * kRowPad + 32 * s + 8 * quarter);
                            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                qa[S], __builtin_bit_cast(bf16x8, v), acc[b], 0, 0, 0);
                        }
                    }
                }
                if (more) store_chunk((stage + 1) & 1, nxt);
                __syncthreads();
                ++stage;
            }
        }
        if (threadIdx.x < 2 * kTQ) epi_vis[threadIdx.x] = pre;
        else if (threadIdx.x < 2 * kTQ + kTP) epi_norm[threadIdx.x - 2 * kTQ] = __uint_as_float(pre);
        __syncthreads();
        // epilogue: C[row 4 quarter + i][col] of block b = q(row) . x(16 b + col)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t x = p0 + 16 * b + col;
            const bool xin = x < pe;
            const float nxb = epi_norm[16 * b + col];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = q0 + 4 * quarter + i;
                bool cand = false;
                float sc = __builtin_inff();
                const uint32_t vword = epi_vis[2 * (wave * 16 + 4 * quarter + i) + (b >> 1)];
                if (xin && q < a.nq && ((vword >> (x & 31)) & 1u)) {
                    sc = nxb - 2.0f * acc[b][i];
                    cand = entry_before(sc, int(x), ts[i], ti[i]);
                }
                const int rbase = (wave * 16 + 4 * quarter + i) * kTileList;
                quarter_offer(cand, sc, int(x), lst_s + rbase, lst_i + rbase, ts[i], ti[i]);
            }
        }
    }
    // the 48 best of each query in this split
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = q0 + 4 * quarter + i;
        if (q < a.nq) {
            const int64_t base = (int64_t(q) * a.nsplit + blockIdx.y) * kTileList;
            const int rbase = (wave * 16 + 4 * quarter + i) * kTileList;
#pragma unroll
            for (int j = 0; j < kSlots; ++j) {
                a.part_s[base + col * kSlots + j] = lst_s[rbase + col * kSlots + j];
                a.part_i[base + col * kSlots + j] = lst_i[rbase + col * kSlots + j];
            }
        }
    }
}

}  // namespace

// Opened leaves -> visited bitmap of one query, written to vis[q][0 .. vw).
__global__ __launch_bounds__(kExpandThreads) void k_expand(ExpandArgs a) {
    extern __shared__ uint32_t smem[];
    uint32_t* bm = smem;                                   // [vw]
    const int q = blockIdx.x;
    for (int64_t i = threadIdx.x; i < a.vw; i += kExpandThreads) bm[i] = 0u;
    __syncthreads();
    expand_opened_leaves(bm, a.leafbits, q, a.nq, a.m, a.W, a.H, a.permp, a.pp, threadIdx.x,
                         kExpandThreads);
    __syncthreads();
    for (int64_t i = threadIdx.x; i < a.vw; i += kExpandThreads) a.vis[int64_t(q) * a.vw + i] = bm[i];
}

// Best kk over the splits' lists, then the final ranking of the query.
__global__ __launch_bounds__(512) void k_merge_rerank(MergeArgs a) {
    __shared__ float md[kWave];
    __shared__ int mi[kWave];
    __shared__ float mr[kWave];
    const int q = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    WaveList L;
    L.init();
    if (wave == 0) {
        const int64_t tot = int64_t(a.nsplit) * kTileList;
        const float* ps = a.part_s + int64_t(q) * tot;
        const int* pi = a.part_i + int64_t(q) * tot;
        for (int64_t e0 = 0; e0 < tot; e0 += kWave) {
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
        if (lane < a.kk) {
            md[lane] = L.d;
            mi[lane] = L.id;
        }
    }
    __syncthreads();
    finish_query(true, a.kk, a.k, q, a.Q + int64_t(q) * a.ldq, a.X32, a.ld32, a.d, md, mi, mr, L,
                 a.ids, a.dists);
}

size_t expand_lds_bytes(int64_t vw) { return size_t(vw) * 4; }

hipError_t launch_tile_path(const ExpandArgs& e, const TileArgs& t, const MergeArgs& m,
                            hipStream_t st, hipEvent_t* ev) {
    const size_t lds = expand_lds_bytes(e.vw);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_expand),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_expand, dim3(e.nq), dim3(kExpandThreads), lds, st, e);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (ev && (err = hipEventRecord(ev[0], st)) != hipSuccess) return err;
    dim3 grid((t.nq + kTQ - 1) / kTQ, t.nsplit);
    const int ks = int(t.ld16 / 32);
    if (ks <= 4) hipLaunchKernelGGL(k_tile_bf16<4>, grid, dim3(kTThreads), 0, st, t);
    else if (ks <= 8) hipLaunchKernelGGL(k_tile_bf16<8>, grid, dim3(kTThreads), 0, st, t);
    else if (ks <= 16) hipLaunchKernelGGL(k_tile_bf16<16>, grid, dim3(kTThreads), 0, st, t);
    else if (ks <= 24) hipLaunchKernelGGL(k_tile_bf16<24>, grid, dim3(kTThreads), 0, st, t);
    else if (ks <= 30) hipLaunchKernelGGL(k_tile_bf16<30>, grid, dim3(kTThreads), 0, st, t);
    else if (ks <= 32) hipLaunchKernelGGL(k_tile_bf16<32>, grid, dim3(kTThreads), 0, st, t);
    else return hipErrorInvalidValue;
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (ev && (err = hipEventRecord(ev[1], st)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_merge_rerank, dim3(m.nq), dim3(512), 0, st, m);
    return hipGetLastError();
}

}  // namespace gf
