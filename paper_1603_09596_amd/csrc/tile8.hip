// tile8.hip -- the FP8 (e4m3, per-row scale) selection score of many
// queries at once, on MFMA, for wide rows.
//
// At d = 10,000 a query's candidates (Sec. 2.3) are a few percent of the
// points, yet gathering them row by row reads 10 KB per candidate from HBM,
// while the dense product of a 256-query block with a 256-point tile pair
// costs 1.3 GFLOP on the FP8 matrix cores (5 PFLOP/s): scoring every pair of
// a block is cheaper than gathering the pairs that count.  The forest then
// decides which scores are kept, through the per-point candidate words of
// the tile path's expansion, and only those are written out, compacted:
//
//   k_cand_masks   per (query, tile of 128 points): the 128-bit mask of the
//                  tile's points that are candidates of the query, from the
//                  per-point words of query bits (ballots over the points);
//   k_cand_prefix  per query: the exclusive prefix count of its candidates
//                  over the tiles, so that every candidate has its own slot;
//   k_tile_fp8     grid (query blocks of 256, point splits of an even number
//                  of tiles): A (queries) and B (points) stream through LDS
//                  by direct loads in 64-byte k stages, four buffers with
//                  three in flight; each wave computes 64 queries x 128
//                  points of the 256 x 256 block as 2 x 4 blocks of 32 x 32
//                  with v_mfma_scale_f32_32x32x64_f8f6f4 (neutral scales,
//                  FP32 accumulation); the epilogue forms
//                  ||x||^2 - 2 s_q s_x q.x for the candidates only and writes
//                  (score, id) to the query's slots;
//   k_topk_select  per query: a radix select over the (score, id) keys of its
//                  candidates keeps the kk best, handed to the tile path's
//                  merge, FP32 compensated re-rank and FP64 tie re-check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace gf {

namespace {

constexpr int kW = 64;                 // wavefront
constexpr int kQB = kTile8Queries;     // queries per workgroup
constexpr int kTP8 = 128;              // points per tile
constexpr int kT8Threads = 512;        // 8 waves, each 64 queries x 128 points
constexpr int kXcd8 = 8;               // XCDs of an MI355X

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Order-preserving map of float scores to uint32 (a < b <=> key(a) < key(b)).
__device__ __forceinline__ uint32_t fkey(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ int popc128_below(uint64_t m0, uint64_t m1, int xl) {
    if (xl < 64) return __popcll(m0 & ((uint64_t{1} << xl) - 1u));
    return __popcll(m0) + __popcll(m1 & ((uint64_t{1} << (xl - 64)) - 1u));
}

}  // namespace

// One workgroup of 128 threads per (tile, word of 32 queries): thread x
// holds the word of point 128 T + x; 32 ballots give the 32 queries' masks
// over the tile's halves.  Ragged tails (points past n, queries past nq)
// are zero or skipped.
__global__ __launch_bounds__(128) void k_cand_masks(const uint32_t* __restrict__ visT, int nq,
                                                    int64_t n, int cw, int ntiles,
                                                    uint64_t* __restrict__ masks) {
    const int T = blockIdx.x, gw = blockIdx.y;
    const int c = gw / cw, w = gw % cw;
    const int64_t x = int64_t(T) * kTP8 + threadIdx.x;
    const uint32_t word = x < n ? visT[(int64_t(c) * n + x) * cw + w] : 0u;
    const int lane = threadIdx.x & (kW - 1), half = threadIdx.x / kW;
#pragma unroll 4
    for (int b = 0; b < 32; ++b) {
        const uint64_t m = __ballot((word >> b) & 1u);
        const int q = gw * 32 + b;
        if (lane == 0 && q < nq) masks[(int64_t(q) * ntiles + T) * 2 + half] = m;
    }
}

// One workgroup of 256 threads per query: offs[q][T] = candidates of q in
// tiles before T; total[q] = all of them.
__global__ __launch_bounds__(256) void k_cand_prefix(const uint64_t* __restrict__ masks, int ntiles,
                                                     uint32_t* __restrict__ offs,
                                                     uint32_t* __restrict__ total) {
    __shared__ uint32_t part[256];
    const int q = blockIdx.x;
    const int per = (ntiles + 255) / 256;
    const int t0 = int(threadIdx.x) * per, t1 = min(ntiles, t0 + per);
    const uint64_t* m = masks + int64_t(q) * ntiles * 2;
    uint32_t s = 0;
    for (int t = t0; t < t1; ++t) s += uint32_t(__popcll(m[2 * t]) + __popcll(m[2 * t + 1]));
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int i = 0; i < 256; ++i) {
            const uint32_t v = part[i];
            part[i] = run;
            run += v;
        }
        total[q] = run;
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (int t = t0; t < t1; ++t) {
        offs[int64_t(q) * ntiles + t] = run;
        run += uint32_t(__popcll(m[2 * t]) + __popcll(m[2 * t + 1]));
    }
}

// Direct global -> LDS loads (global_load_lds_dwordx4): every lane reads 16
// bytes at base + voff and the wave writes them contiguously at LDS address
// m0 + 16 lane.  Issued from inline assembly so that the compiler does not
// wait for them before unrelated LDS reads; the kernel waits itself
// (s_waitcnt vmcnt) before the barrier that publishes a stage.
__device__ __forceinline__ void dma8_16s(const void* base, uint32_t voff, uint32_t lds) {
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
                 :: "v"(voff), "s"(base), "{m0}"(__builtin_amdgcn_readfirstlane(lds)) : "memory");
}
__device__ __forceinline__ const void* uniform8(const void* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return reinterpret_cast<const void*>((uint64_t(hi) << 32) | lo);
}
// s_waitcnt immediates (gfx9 encoding: vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[5:4] at 15:14)
constexpr int kWait8(int n) { return (n & 15) | (7 << 4) | (15 << 8) | (((n >> 4) & 3) << 14); }
typedef __attribute__((address_space(3))) uint32_t lds8_u32;
__device__ __forceinline__ uint32_t lds8_offset(const void* p) {
    return uint32_t(uintptr_t((const lds8_u32*)p));
}

constexpr int kNBuf8 = 4;                          // stage buffers (three stages in flight)
constexpr int kKS = 64;                            // k bytes per stage (one 32x32x64 MFMA depth)
constexpr int kTW8 = 2 * kTP8;                     // points per workgroup tile: two mask tiles
constexpr int kStageA8 = kQB * kKS;                // 16 KB of query rows per stage
constexpr int kStageB8 = kTW8 * kKS;               // 16 KB of point rows per stage
constexpr int kDmaA8 = kStageA8 / 1024 / (kT8Threads / kW);   // 1 KB loads per wave and stage: 2
constexpr int kDmaB8 = kStageB8 / 1024 / (kT8Threads / kW);   // 2
constexpr int kDma8 = kDmaA8 + kDmaB8;
static_assert(kDmaA8 * 1024 * (kT8Threads / kW) == kStageA8 && kDmaB8 * 1024 * (kT8Threads / kW) == kStageB8,
              "stage shape");
typedef float v16f __attribute__((ext_vector_type(16)));

// Byte offset in a stage of 16-byte unit u (0..3) of row r: rows are paired
// into 128-byte lines, row r in line r >> 1 at unit positions u + 4 (r & 1),
// XOR (r >> 1) & 7.  A direct load's lane l % 8 takes position l % 8 of line
// l / 8, and the operand reads of 8 consecutive rows (one unit each) fall on
// 8 different 16-byte bank groups.
__device__ __forceinline__ int unit_off8(int r, int u) {
    return (r >> 1) * 128 + (((u + 4 * (r & 1)) ^ ((r >> 1) & 7)) << 4);
}

// The score kernel: grid (query blocks of 256, point splits), 8 waves; wave
// w computes queries 64 (w >> 1) .. + 64 against points 128 (w & 1) .. + 128
// of each 256-point tile (two 128-point mask tiles) with
// v_mfma_scale_f32_32x32x64_f8f6f4 (neutral scales, FP32 accumulation), 2 x 4
// blocks of 32 x 32.  Both operands stream through LDS in 64-byte k stages by
// direct loads, four buffers, three stages in flight across tile boundaries.
// Workgroups are dispatched to the XCDs round-robin (workgroup i to XCD
// i % 8); each XCD takes a consecutive run of the split-major (split, query
// block) list, so the query blocks of one split run on one XCD and share its
// L2 for the split's rows.  k bytes past the row (ld8 is a multiple of 16,
// not of 64) are loaded from a valid address and zeroed in the fragments.
__global__ __launch_bounds__(kT8Threads) void k_tile_fp8(Tile8Args a) {
    __shared__ __attribute__((aligned(1024))) uint8_t sA[kNBuf8][kStageA8];
    __shared__ __attribute__((aligned(1024))) uint8_t sB[kNBuf8][kStageB8];
    __shared__ uint64_t sMask[kQB][2][2];
    __shared__ uint32_t sOff[kQB][2];
    __shared__ float sQs[kQB];
    __shared__ float sXn[kTW8], sXs[kTW8];
    const int tid = threadIdx.x, lane = tid & (kW - 1), wave = tid / kW;
    int qblk, split;
    {
        const int nqb = (a.nq + kQB - 1) / kQB;
        const int total = nqb * a.nsplit;
        const int i = int(blockIdx.x), x = i % kXcd8, j = i / kXcd8;
        const int base = total / kXcd8, rem = total % kXcd8;
        const int L = (x < rem) ? x * (base + 1) + j : rem * (base + 1) + (x - rem) * base + j;
        split = L / nqb;
        qblk = L - split * nqb;
    }
    const int q0 = qblk * kQB;
    const int t_begin = split * a.split_tiles;            // even: tiles are taken in pairs
    const int t_end = min(a.ntiles, t_begin + a.split_tiles);
    const int npair = (t_end - t_begin + 1) / 2;
    const int nk = int((a.ld8 + kKS - 1) / kKS);
    if (tid < kQB) sQs[tid] = (q0 + tid < a.nq) ? a.qscale[q0 + tid] : 0.0f;

    // MFMA operands: lane l reads row (l & 31) of each 32-row fragment, k
    // bytes 32 (l >> 5) .. + 32 of the stage (units 2 kg and 2 kg + 1)
    const int qq = wave >> 1, ph = wave & 1;
    const int fr = lane & 31, kg = lane >> 5;
    // Direct loads: instruction j of wave w writes lines 8 (w + 8 j) .. + 8
    // (rows 16 (w + 8 j) .. + 16) of a stage; lane l position l % 8 of line
    // 8 (w + 8 j) + l / 8, which holds row 2 line + s / 4, unit s % 4, with
    // s = (l % 8) ^ (line & 7).  Rows past the queries or points are clamped
    // to the block's or tile's first row; their scores are never kept.
    const int dline = lane >> 3;                          // line within the 8 of an instruction
    const int ds = (lane & 7) ^ dline;                    // (line & 7) == dline for every instruction
    const int drow = 2 * dline + (ds >> 2), du = ds & 3;  // row within the 16, unit
    const uint32_t sA0 = lds8_offset(sA), sB0 = lds8_offset(sB);
    const void* qbase = uniform8(a.Q8 + int64_t(q0) * a.ld8);
    uint32_t qoff[kDmaA8];
#pragma unroll
    for (int j = 0; j < kDmaA8; ++j) {
        const int r = 16 * (wave + 8 * j) + drow;
        qoff[j] = uint32_t(q0 + r < a.nq ? r : 0) * uint32_t(a.ld8);
    }
    // issue cursor: the next stage to load is stage ic of tile pair ip, into ibuf
    int ip = 0, ic = 0, ibuf = 0;
    const int nstages = npair * nk;
    auto issue_next = [&]() {
        const uint32_t k = uint32_t(ic * kKS) + 16u * uint32_t(du);
        const uint32_t koff = k < uint32_t(a.ld8) ? k : 0u;
#pragma unroll
        for (int j = 0; j < kDmaA8; ++j)
            dma8_16s(qbase, qoff[j] + koff, sA0 + uint32_t(ibuf * kStageA8 + (wave + 8 * j) * 1024));
        const int64_t x0 = int64_t(t_begin + 2 * ip) * kTP8;
        const void* xbase = uniform8(a.X8 + x0 * a.ld8);
#pragma unroll
        for (int j = 0; j < kDmaB8; ++j) {
            const int r = 16 * (wave + 8 * j) + drow;
            const uint32_t xo = uint32_t(x0 + r < a.n ? r : 0) * uint32_t(a.ld8);
            dma8_16s(xbase, xo + koff, sB0 + uint32_t(ibuf * kStageB8 + (wave + 8 * j) * 1024));
        }
        ibuf = (ibuf + 1 == kNBuf8) ? 0 : ibuf + 1;
        if (++ic == nk) {
            ic = 0;
            ++ip;
        }
    };
    int issued = 0;
    for (; issued < kNBuf8 - 1 && issued < nstages; ++issued) issue_next();

    int buf = 0, consumed = 0;
    for (int P = 0; P < npair; ++P) {
        const int T = t_begin + 2 * P;
        const int64_t x0 = int64_t(T) * kTP8;
        v16f acc[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = v16f{};
        for (int kc = 0; kc < nk; ++kc) {
            // Loads complete in issue order: waiting down to the stages issued
            // after this one completes this stage for this wave, and the
            // barrier then covers every wave and frees the buffer of the stage
            // before for reuse.
            asm volatile("" ::: "memory");
            const int ahead = issued - consumed - 1;
            if (ahead >= 2) __builtin_amdgcn_s_waitcnt(kWait8(2 * kDma8));
            else if (ahead == 1) __builtin_amdgcn_s_waitcnt(kWait8(kDma8));
            else __builtin_amdgcn_s_waitcnt(kWait8(0));
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (issued < nstages) {
                issue_next();
                ++issued;
            }
            const uint8_t* A = sA[buf];
            const uint8_t* B = sB[buf];
            // fragments: 32 k bytes of the lane's row; bytes past the row are zero
            const bool lo_in = kc * kKS + 32 * kg < a.ld8;
            const bool hi_in = kc * kKS + 32 * kg + 16 < a.ld8;
            v8i fa[2], fb[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int r = 64 * qq + 32 * i + fr;
                uint4 lo = *reinterpret_cast<const uint4*>(&A[unit_off8(r, 2 * kg)]);
                uint4 hi = *reinterpret_cast<const uint4*>(&A[unit_off8(r, 2 * kg + 1)]);
                if (!lo_in) lo = make_uint4(0, 0, 0, 0);
                if (!hi_in) hi = make_uint4(0, 0, 0, 0);
                fa[i] = v8i{int(lo.x), int(lo.y), int(lo.z), int(lo.w), int(hi.x), int(hi.y), int(hi.z), int(hi.w)};
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 128 * ph + 32 * j + fr;
                const uint4 lo = *reinterpret_cast<const uint4*>(&B[unit_off8(r, 2 * kg)]);
                const uint4 hi = *reinterpret_cast<const uint4*>(&B[unit_off8(r, 2 * kg + 1)]);
                fb[j] = v8i{int(lo.x), int(lo.y), int(lo.z), int(lo.w), int(hi.x), int(hi.y), int(hi.z), int(hi.w)};
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[i], fb[j], acc[i][j],
                                                                                0, 0, 0, 127, 0, 127);
            buf = (buf + 1 == kNBuf8) ? 0 : buf + 1;
            ++consumed;
        }
        // epilogue operands of this tile pair: the block's masks and offsets
        // of both mask tiles, the points' norms and scales.  The previous
        // pair's epilogue finished reading them before this pair's first
        // stage barrier.
        if (tid < kQB) {
            const int q = q0 + tid;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const bool in = q < a.nq && T + h < t_end;
                const int64_t mi = (int64_t(q) * a.ntiles + T + h) * 2;
                sMask[tid][h][0] = in ? a.masks[mi] : 0;
                sMask[tid][h][1] = in ? a.masks[mi + 1] : 0;
                sOff[tid][h] = in ? a.offs[int64_t(q) * a.ntiles + T + h] : 0;
            }
        } else {
            const int xl = tid - kQB;                      // 256 threads for the 256 points
            const int64_t x = x0 + xl;
            const bool in = x < a.n && T + (xl >> 7) < t_end;
            sXn[xl] = in ? a.norm8[x] : 0.0f;
            sXs[xl] = in ? a.scale8[x] : 0.0f;
        }
        __syncthreads();
        // C[row][col] of block (i, j): lane l holds column l % 32 and, in
        // element e, row 8 (e / 4) + 4 (l / 32) + e % 4: query
        // 64 qq + 32 i + row, point 128 ph + 32 j + l % 32 of the pair.  The
        // lane's first row is made opaque, so that the addresses derived from
        // it are formed here rather than held in registers across the loop.
        int qrow = 64 * qq + 4 * kg;
        asm volatile("" : "+v"(qrow));
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int ql = qrow + 32 * i + 8 * (e >> 2) + (e & 3);
                const int h = ph;                           // the wave's points lie in mask tile ph
                const uint64_t m0 = sMask[ql][h][0], m1 = sMask[ql][h][1];
                if (!(m0 | m1)) continue;
                const int64_t slot0 = int64_t(q0 + ql) * a.cap + sOff[ql][h];
                const float qs2 = 2.0f * sQs[ql];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int xt = 32 * j + fr;             // point within mask tile h
                    const bool cand = ((xt < 64 ? (m0 >> xt) : (m1 >> (xt - 64))) & 1u) != 0;
                    if (cand) {
                        const int xl = kTP8 * h + xt;
                        const int64_t slot = slot0 + popc128_below(m0, m1, xt);
                        a.out_s[slot] = sXn[xl] - qs2 * sXs[xl] * acc[i][j][e];
                        a.out_i[slot] = int(x0 + xl);
                    }
                }
            }
    }
    __builtin_amdgcn_s_waitcnt(kWait8(0));
}

// The kk best (score, id) of each query among its candidates: a radix select
// over the 64-bit keys (order-preserving score bits, id) in eight 8-bit
// digits; keys are distinct (ids are), so exactly min(kk, count) entries are
// at or below the threshold.  They go to the first kk slots of the query's
// list, the rest of its kTileList slots hold (+inf, max id).
__global__ __launch_bounds__(256) void k_topk_select(const float* __restrict__ out_s,
                                                     const int* __restrict__ out_i,
                                                     const uint32_t* __restrict__ total, int64_t cap,
                                                     int kk, float* __restrict__ part_s,
                                                     int* __restrict__ part_i) {
    __shared__ uint32_t hist[256];
    __shared__ uint64_t sh_prefix;
    __shared__ uint32_t sh_left, sh_pos;
    const int q = blockIdx.x;
    const uint32_t cnt = min(total[q], uint32_t(cap));
    const float* s = out_s + int64_t(q) * cap;
    const int* id = out_i + int64_t(q) * cap;
    auto key = [&](uint32_t i) { return (uint64_t(fkey(s[i])) << 32) | uint32_t(id[i]); };
    uint64_t kstar = ~0ull;
    if (cnt > uint32_t(kk)) {
        if (threadIdx.x == 0) {
            sh_prefix = 0;
            sh_left = uint32_t(kk);
        }
        __syncthreads();
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            hist[threadIdx.x] = 0;
            __syncthreads();
            const uint64_t prefix = sh_prefix;
            for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
                const uint64_t K = key(i);
                if (pass == 0 || (K >> (shift + 8)) == prefix) atomicAdd(&hist[(K >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t left = sh_left, b = 0;
                for (; b < 255u && hist[b] < left; ++b) left -= hist[b];
                sh_left = left;
                sh_prefix = (prefix << 8) | b;
            }
            __syncthreads();
        }
        kstar = sh_prefix;
    }
    if (threadIdx.x == 0) sh_pos = 0;
    __syncthreads();
    float* ps = part_s + int64_t(q) * kTileList;
    int* pi = part_i + int64_t(q) * kTileList;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        if (key(i) <= kstar) {
            const uint32_t p = atomicAdd(&sh_pos, 1u);
            if (p < uint32_t(kTileList)) {
                ps[p] = s[i];
                pi[p] = id[i];
            }
        }
    }
    __syncthreads();
    for (uint32_t p = sh_pos + threadIdx.x; p < uint32_t(kTileList); p += blockDim.x) {
        ps[p] = __builtin_inff();
        pi[p] = 0x7FFFFFFF;
    }
}

int tile8_ntiles(int64_t n) { return int((n + kTP8 - 1) / kTP8); }

hipError_t launch_tile8(const Tile8Args& t, int nqw, hipStream_t st, hipEvent_t* ev) {
    if (t.cw < 4 || t.cw > 32 || t.ld8 % 16 || t.ntiles != tile8_ntiles(t.n) || t.split_tiles < 2 ||
        t.split_tiles % 2 || t.nsplit * t.split_tiles < t.ntiles)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cand_masks, dim3(unsigned(t.ntiles), unsigned(nqw)), dim3(128), 0, st,
                       t.visT, t.nq, t.n, t.cw, t.ntiles, t.masks);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_cand_prefix, dim3(unsigned(t.nq)), dim3(256), 0, st,
                       static_cast<const uint64_t*>(t.masks), t.ntiles, t.offs, t.total);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (ev && (err = hipEventRecord(ev[0], st)) != hipSuccess) return err;
    const int nqb = (t.nq + kQB - 1) / kQB;
    hipLaunchKernelGGL(k_tile_fp8, dim3(unsigned(nqb * t.nsplit)), dim3(kT8Threads), 0, st, t);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if (ev && (err = hipEventRecord(ev[1], st)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_topk_select, dim3(unsigned(t.nq)), dim3(256), 0, st,
                       static_cast<const float*>(t.out_s), static_cast<const int*>(t.out_i),
                       static_cast<const uint32_t*>(t.total), t.cap, t.kk, t.part_s, t.part_i);
    return hipGetLastError();
}

}  // namespace gf
