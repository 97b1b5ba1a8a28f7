// scan.hip -- candidates, distances and the k best of every query on gfx950
// (Alg. 2 "descend at a leaf" and the visited array of Sec. 2.3; the
// squared-norm expansion of Sec. 3 "Distance computation").
//
// One workgroup of 8 wavefronts per query:
//   1. expansion: every opened leaf's point ids are OR-ed into a visited
//      bitmap of n bits held in LDS, so each candidate appears once however
//      many trees reach it;
//   2. scan: the waves walk the bitmap in point-id order (16 words at a time
//      per wave), gather the candidate rows with 16-byte loads and reduce each
//      row's distance across the lanes that share it; walking ids in order
//      keeps the row gathers monotone in address, so concurrent queries on
//      the chip stream through the same region of X;
//   3. each wave keeps its best `kk` (distance, id) pairs, one per lane,
//      sorted; the eight lists are merged at the end;
//   4. reduced-precision forms: the merged `kk` candidates are measured again
//      on the FP32 rows with a compensated sum (two-sum / two-product), then
//      ranked; every form: the distances within 1e-5 relative of the k-th
//      are measured once more in FP64 and the tie group is re-ranked by
//      (FP64 distance, id).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "kernels.h"
#include "rank.h"

namespace gf {

namespace {

constexpr int kWaves = 8;
constexpr int kThreads = kWave * kWaves;
constexpr int kListWords = 16;                // bitmap words per wave step
constexpr int kListCap = kListWords * 32;     // ids per wave step

template <int LPR>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int o = LPR / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ------------------------------------------------------------- row scoring

template <int FORM>
struct Chunk;   // one 16-byte slice of a row in the given storage form

template <>
struct Chunk<kFormFP32> {
    using T = float4;
    static constexpr int kElems = 4;
    __device__ static float score(const float4& q, const float4& x) {
        const float a = q.x - x.x, b = q.y - x.y, c = q.z - x.z, e = q.w - x.w;
        return fmaf(a, a, fmaf(b, b, fmaf(c, c, e * e)));
    }
};

template <>
struct Chunk<kFormBF16> {
    using T = uint4;
    static constexpr int kElems = 8;
    typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
    __device__ static float dot2(uint32_t a, uint32_t b, float acc) {
        return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf2, a),
                                               __builtin_bit_cast(bf2, b), acc, false);
    }
    __device__ static float score(const uint4& q, const uint4& x) {
        float acc = dot2(q.x, x.x, 0.0f);
        acc = dot2(q.y, x.y, acc);
        acc = dot2(q.z, x.z, acc);
        return dot2(q.w, x.w, acc);
    }
};

template <>
struct Chunk<kFormFP8> {
    using T = uint4;
    static constexpr int kElems = 16;
    __device__ static float dot4(uint32_t a, uint32_t b, float acc) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 a0 = __builtin_amdgcn_cvt_pk_f32_fp8(a, false);
        const f2 a1 = __builtin_amdgcn_cvt_pk_f32_fp8(a, true);
        const f2 b0 = __builtin_amdgcn_cvt_pk_f32_fp8(b, false);
        const f2 b1 = __builtin_amdgcn_cvt_pk_f32_fp8(b, true);
        acc = fmaf(a0.x, b0.x, acc);
        acc = fmaf(a0.y, b0.y, acc);
        acc = fmaf(a1.x, b1.x, acc);
        return fmaf(a1.y, b1.y, acc);
    }
    __device__ static float score(const uint4& q, const uint4& x) {
        float acc = dot4(q.x, x.x, 0.0f);
        acc = dot4(q.y, x.y, acc);
        acc = dot4(q.z, x.z, acc);
        return dot4(q.w, x.w, acc);
    }
    // x (16 codes of chunk ci) against the decoded query held in LDS as four
    // planes: plane i holds values 4i .. 4i+3 of every chunk, so lanes
    // reading consecutive chunks read consecutive 16-byte words
    __device__ static float score_lds(const float4* qp, int64_t ci, int64_t nch, const uint4& x) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        const uint32_t w[4] = {x.x, x.y, x.z, x.w};
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const f2 lo = __builtin_amdgcn_cvt_pk_f32_fp8(w[i], false);
            const f2 hi = __builtin_amdgcn_cvt_pk_f32_fp8(w[i], true);
            const float4 qq = qp[i * nch + ci];
            acc = fmaf(lo.x, qq.x, acc);
            acc = fmaf(lo.y, qq.y, acc);
            acc = fmaf(hi.x, qq.z, acc);
            acc = fmaf(hi.y, qq.w, acc);
        }
        return acc;
    }
};

// ------------------------------------------------------------------ kernel

template <int FORM, int LPR, int CPL>
__global__ __launch_bounds__(kThreads) void k_scan(ScanArgs a) {
    using C = Chunk<FORM>;
    using T = typename C::T;
    constexpr int G = kWave / LPR;     // rows per load instruction
    // CPL <= 0: rows wider than the register-resident tiles; each lane
    // streams its chunks.  CPL == -1 (FP32, BF16) reads the query from a copy
    // in LDS, so the row stream cannot evict it from L2; CPL == 0 reads it
    // from global memory, for rows whose copy would not fit beside the bitmap.
    constexpr bool kStream = (CPL <= 0);
    constexpr bool kQStage = (CPL < 0);
    static_assert(!(kQStage && FORM == kFormFP8), "the FP8 query is always decoded into LDS");
    constexpr int CPLR = kStream ? 1 : CPL;
    constexpr int U = kStream ? 1 : ((FORM == kFormFP8 && CPL > 8) ? 1 : 2);
    extern __shared__ uint32_t smem[];
    const int q = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    // this workgroup's slice of the id range: bitmap words [w_lo, w_lo + nbmw)
    const int64_t nbmw_all = (a.n + 31) / 32;
    const int64_t w_lo = int64_t(blockIdx.y) * a.slice_words;
    const int64_t nbmw = a.nslice > 1 ? min(a.slice_words, nbmw_all - w_lo) : nbmw_all;
    const int64_t nbmw_pad = (nbmw + kListWords - 1) / kListWords * kListWords;
    uint32_t* bm = smem;                                        // [nbmw_pad]
    uint32_t* lists = bm + nbmw_pad;                            // [kWaves][kListCap]
    float* mg_d = reinterpret_cast<float*>(lists + kWaves * kListCap);   // [kWaves][64]
    int* mg_i = reinterpret_cast<int*>(mg_d + kWaves * kWave);           // [kWaves][64]
    float* rr_d = reinterpret_cast<float*>(mg_i + kWaves * kWave);       // [64]
    float* q8f = rr_d + kWave;          // [ld8] decoded FP8 query, or the staged FP32 / BF16 query

    // 1. visited bitmap <- union of the opened leaves (this slice's words of
    // the query's bitmap, when one was built beforehand)
    if (a.gbits) {
        const uint32_t* g = a.gbits + int64_t(q) * nbmw_all + w_lo;
        for (int64_t i = threadIdx.x; i < nbmw_pad; i += kThreads) bm[i] = i < nbmw ? g[i] : 0u;
    } else {
        for (int64_t i = threadIdx.x; i < nbmw_pad; i += kThreads) bm[i] = 0u;
        __syncthreads();
        expand_opened_leaves(bm, a.leafbits, q, a.nq, a.m, a.W, a.H, a.permp, a.pp, threadIdx.x,
                             kThreads, w_lo, w_lo + nbmw);
    }
    __syncthreads();
    if (a.cand_bits) {
        // this slice's words of the query's row of the candidate bitmap
        for (int64_t i = threadIdx.x; i < nbmw; i += kThreads)
            a.cand_bits[int64_t(q) * nbmw_all + w_lo + i] = bm[i];
    }
    if (a.ncand) {
        uint32_t cnt = 0;
        for (int64_t i = threadIdx.x; i < nbmw; i += kThreads) cnt += __popc(bm[i]);
        for (int o = kWave / 2; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o);
        if (lane == 0) mg_i[wave] = int(cnt);
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t tot = 0;
            for (int w = 0; w < kWaves; ++w) tot += mg_i[w];
            a.ncand[q] = tot;
        }
        __syncthreads();
    }

    // 2./3. scan the candidates in id order, keep the best kk per wave
    const int sub = lane % LPR;
    const int grp = lane / LPR;
    const int64_t nchunks_row = (FORM == kFormFP32) ? (a.ld32 / 4)
                              : (FORM == kFormBF16) ? (a.ld16 / 8) : (a.ld8 / 16);
    const T* Xb = (FORM == kFormFP32) ? reinterpret_cast<const T*>(a.X32)
                : (FORM == kFormBF16) ? reinterpret_cast<const T*>(a.X16)
                                      : reinterpret_cast<const T*>(a.X8);
    const T* Qrow = (FORM == kFormFP32) ? reinterpret_cast<const T*>(a.Q + int64_t(q) * a.ldq)
                  : (FORM == kFormBF16) ? reinterpret_cast<const T*>(a.Q16 + int64_t(q) * a.ld16)
                                        : reinterpret_cast<const T*>(a.Q8 + int64_t(q) * a.ld8);
    constexpr int QREG = (FORM == kFormFP8 || kStream) ? 1 : CPL;
    T qv[QREG];
    if constexpr (FORM == kFormFP8) {
        // the e4m3 query, decoded once into LDS (same conversion as the rows)
        typedef float f2 __attribute__((ext_vector_type(2)));
        const uint32_t* q8w = reinterpret_cast<const uint32_t*>(a.Q8 + int64_t(q) * a.ld8);
        for (int64_t i = threadIdx.x; i < a.ld8 / 4; i += kThreads) {
            const uint32_t wv = q8w[i];
            const f2 lo = __builtin_amdgcn_cvt_pk_f32_fp8(wv, false);
            const f2 hi = __builtin_amdgcn_cvt_pk_f32_fp8(wv, true);
            // word i = values 4i .. 4i+3 = plane i % 4 of chunk i / 4
            reinterpret_cast<float4*>(q8f)[(i & 3) * (a.ld8 / 16) + (i >> 2)] =
                make_float4(lo.x, lo.y, hi.x, hi.y);
        }
        __syncthreads();
        qv[0] = T{};
    } else if constexpr (kQStage) {
        T* qt = reinterpret_cast<T*>(q8f);
        for (int64_t i = threadIdx.x; i < nchunks_row; i += kThreads) qt[i] = Qrow[i];
        __syncthreads();
        qv[0] = T{};
    } else if constexpr (kStream) {
        qv[0] = T{};
    } else {
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const int64_t ci = sub + int64_t(j) * LPR;
            qv[j] = (ci < nchunks_row) ? Qrow[ci] : T{};
        }
    }
    const T* Qsrc = kQStage ? reinterpret_cast<const T*>(q8f) : Qrow;
    const float4* q8p = reinterpret_cast<const float4*>(q8f);   // FP8: the planes of the decoded query
    float qn = 0.0f, qs = 0.0f;
    if (FORM != kFormFP32) qn = a.qnorm[q];
    if (FORM == kFormFP8) qs = a.qscale8[q];

    WaveList L;
    L.init();
    const int kk = a.kk;
    uint32_t* list = lists + wave * kListCap;
    const int64_t nsteps = nbmw_pad / kListWords;
    for (int64_t step = wave; step < nsteps; step += kWaves) {
        uint32_t w = (lane < kListWords) ? bm[step * kListWords + lane] : 0u;
        const int cnt = __popc(w);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < kListWords; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        const int total = __shfl(incl, kListWords - 1);
        if (total == 0) continue;
        int pos = incl - cnt;
        const uint32_t base = uint32_t(w_lo + step * kListWords + lane) * 32u;
        while (w) {
            list[pos++] = base + uint32_t(__builtin_ctz(w));
            w &= w - 1;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int r0 = 0; r0 < total; r0 += G * U) {
            int rid[U];
            T xv[U][CPLR];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int slot = r0 + u * G + grp;
                rid[u] = (slot < total) ? int(list[slot]) : -1;
                if constexpr (!kStream) {
                    const T* xr = Xb + int64_t(rid[u] < 0 ? 0 : rid[u]) * nchunks_row;
#pragma unroll
                    for (int j = 0; j < CPL; ++j) {
                        const int64_t ci = sub + int64_t(j) * LPR;
                        xv[u][j] = (rid[u] >= 0 && ci < nchunks_row) ? xr[ci] : T{};
                    }
                }
            }
            float dist[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                float acc = 0.0f;
                if constexpr (kStream) {
                    if (rid[u] >= 0) {
                        const T* xr = Xb + int64_t(rid[u]) * nchunks_row;
                        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
                        int64_t ci = sub;
                        for (; ci + 3 * LPR < nchunks_row; ci += 4 * LPR) {
                            const T x0 = xr[ci], x1 = xr[ci + LPR], x2 = xr[ci + 2 * LPR],
                                    x3 = xr[ci + 3 * LPR];
                            if constexpr (FORM == kFormFP8) {
                                a0 += C::score_lds(q8p, ci, nchunks_row, x0);
                                a1 += C::score_lds(q8p, ci + LPR, nchunks_row, x1);
                                a2 += C::score_lds(q8p, ci + 2 * LPR, nchunks_row, x2);
                                a3 += C::score_lds(q8p, ci + 3 * LPR, nchunks_row, x3);
                            } else {
                                a0 += C::score(Qsrc[ci], x0);
                                a1 += C::score(Qsrc[ci + LPR], x1);
                                a2 += C::score(Qsrc[ci + 2 * LPR], x2);
                                a3 += C::score(Qsrc[ci + 3 * LPR], x3);
                            }
                        }
                        for (; ci < nchunks_row; ci += LPR) {
                            if constexpr (FORM == kFormFP8) a0 += C::score_lds(q8p, ci, nchunks_row, xr[ci]);
                            else a0 += C::score(Qsrc[ci], xr[ci]);
                        }
                        acc = (a0 + a1) + (a2 + a3);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < CPL; ++j) {
                        if constexpr (FORM == kFormFP8) {
                            const int64_t ci = sub + int64_t(j) * LPR;
                            if (ci < nchunks_row) acc += C::score_lds(q8p, ci, nchunks_row, xv[u][j]);
                        } else {
                            acc += C::score(qv[QREG > 1 ? j : 0], xv[u][j]);
                        }
                    }
                }
                acc = group_sum<LPR>(acc);
                if (FORM == kFormBF16 && rid[u] >= 0)
                    acc = a.norm16[rid[u]] - 2.0f * acc + qn;
                if (FORM == kFormFP8 && rid[u] >= 0)
                    acc = a.norm8[rid[u]] - 2.0f * (a.scale8[rid[u]] * qs) * acc + qn;
                dist[u] = acc;
            }
            const float td = L.thr_d(kk);
            const int ti = L.thr_id(kk);
            bool any_q = false;
#pragma unroll
            for (int u = 0; u < U; ++u)
                any_q |= (sub == 0 && rid[u] >= 0 && entry_before(dist[u], rid[u], td, ti));
            if (!__any(any_q)) continue;
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int idc = __builtin_amdgcn_readlane(rid[u], g * LPR);
                    if (idc < 0) continue;
                    const float dc = __int_as_float(
                        __builtin_amdgcn_readlane(__float_as_int(dist[u]), g * LPR));
                    L.offer(dc, idc, kk);
                }
            }
        }
    }

    // merge the per-wave lists into wave 0
    if (lane < kk) {
        mg_d[wave * kWave + lane] = L.d;
        mg_i[wave * kWave + lane] = L.id;
    }
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < kWaves; ++w)
            for (int e = 0; e < kk; ++e) {
                const float dc = mg_d[w * kWave + e];
                if (!(dc < __builtin_inff())) break;
                L.offer(dc, mg_i[w * kWave + e], kk);
            }
        if (lane < kk) {
            mg_d[lane] = L.d;
            mg_i[lane] = L.id;
        }
        if (a.nslice > 1) {
            // a slice hands its kk best (in order) to the merge
            // (lane e holds entry e of the sorted list; kTileList <= kWave)
            const int64_t base = (int64_t(q) * a.nslice + blockIdx.y) * kTileList;
            if (lane < kTileList) {
                const bool have = lane < kk && L.d < __builtin_inff();
                a.part_s[base + lane] = have ? L.d : __builtin_inff();
                a.part_i[base + lane] = have ? L.id : 0x7FFFFFFF;
            }
        }
    }
    if (a.nslice > 1) return;
    __syncthreads();

    finish_query(FORM != kFormFP32, kk, a.k, q, a.Q + int64_t(q) * a.ldq, a.X32, a.ld32, a.d,
                 mg_d, mg_i, rr_d, L, a.ids, a.dists);
}

}  // namespace

namespace {

template <int FORM>
hipError_t launch_form(const ScanArgs& a, hipStream_t st, size_t lds) {
    const int64_t nchunks_row = (FORM == kFormFP32) ? (a.ld32 / 4)
                              : (FORM == kFormBF16) ? (a.ld16 / 8) : (a.ld8 / 16);
    dim3 grid(a.nq, a.nslice > 1 ? a.nslice : 1), block(kThreads);
#define GF_TRY(LPRV, CPLV)                                                                   \
    if (nchunks_row <= int64_t(LPRV) * CPLV) {                                               \
        hipError_t e = hipFuncSetAttribute(                                                  \
            reinterpret_cast<const void*>(&k_scan<FORM, LPRV, CPLV>),                        \
            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));                           \
        if (e != hipSuccess) return e;                                                       \
        hipLaunchKernelGGL((k_scan<FORM, LPRV, CPLV>), grid, block, lds, st, a);             \
        return hipGetLastError();                                                            \
    }
    GF_TRY(8, 4)
    GF_TRY(16, 4)
    GF_TRY(8, 16)
    GF_TRY(16, 16)
    GF_TRY(64, 8)
    GF_TRY(64, 16)
#undef GF_TRY
    if constexpr (FORM != kFormFP8) {
        // wide rows: stage the query in LDS when it fits beside the bitmap
        // (GF_SCAN_WIDE_QUERY=global keeps it in global memory, as for rows
        // whose copy would not fit; both give the same sums)
        const size_t lq = lds + size_t(nchunks_row) * 16;
        const char* wq = std::getenv("GF_SCAN_WIDE_QUERY");
        if (lq <= 160 * 1024 && !(wq && std::strcmp(wq, "global") == 0)) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scan<FORM, 64, -1>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lq));
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_scan<FORM, 64, -1>), grid, block, lq, st, a);
            return hipGetLastError();
        }
    }
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scan<FORM, 64, 0>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_scan<FORM, 64, 0>), grid, block, lds, st, a);
    return hipGetLastError();
}

}  // namespace

size_t scan_lds_bytes_words(int64_t words, int form, int64_t ld8) {
    const int64_t nbmw_pad = (words + kListWords - 1) / kListWords * kListWords;
    // bitmap + per-wave id lists + merge area + re-rank staging (+ FP8 query)
    return size_t(nbmw_pad) * 4 + size_t(kWaves) * kListCap * 4 + size_t(kWaves) * kWave * 8 +
           size_t(kWave) * 4 + (form == kFormFP8 ? size_t(ld8) * 4 : 0);
}

size_t scan_lds_bytes(int64_t n, int form, int64_t ld8) {
    return scan_lds_bytes_words((n + 31) / 32, form, ld8);
}

bool scan_supported(int64_t n, int form, int64_t ld8) {
    return scan_lds_bytes(n, form, ld8) <= 160 * 1024;
}

int64_t scan_max_slice_words(int form, int64_t ld8) {
    const size_t fixed = scan_lds_bytes_words(0, form, ld8);
    if (fixed + size_t(kListWords) * 4 > 160 * 1024) return 0;
    return int64_t((160 * 1024 - fixed) / 4) / kListWords * kListWords;
}

namespace {

__global__ __launch_bounds__(256) void k_zero_words(uint32_t* p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
        p[i] = 0u;
}

// One thread per leaf of the forest (x) and query (y): an opened leaf's point
// ids go into the query's row of the bitmap.
__global__ __launch_bounds__(256) void k_mark_candidates(ScanArgs a, uint32_t* gbits) {
    const int q = int(blockIdx.y);
    const int64_t leaf = int64_t(blockIdx.x) * 256 + threadIdx.x;   // word leaf / 32, bit leaf % 32
    const int64_t f = leaf >> 5;
    if (f >= int64_t(a.m) * a.W) return;
    if (!((a.leafbits[f * a.nq + q] >> (leaf & 31)) & 1u)) return;
    const int64_t nleaf = int64_t(1) << a.H;
    const int64_t tree = f / a.W, lt = (f % a.W) * 32 + (leaf & 31);
    if (lt >= nleaf) return;
    const uint4* row = reinterpret_cast<const uint4*>(a.permp + (tree * nleaf + lt) * a.pp);
    uint32_t* g = gbits + int64_t(q) * ((a.n + 31) / 32);
    for (int c = 0; c < a.pp / 4; ++c) {
        const uint4 v = row[c];
        const uint32_t ids[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (ids[e] != 0xFFFFFFFFu) atomicOr(&g[ids[e] >> 5], 1u << (ids[e] & 31u));
    }
}

}  // namespace

hipError_t launch_mark_candidates(const ScanArgs& a, uint32_t* gbits, hipStream_t st) {
    if (a.nq <= 0) return hipSuccess;
    if (a.nq > kMarkMaxQueries || a.pp % 4) return hipErrorInvalidValue;
    const int64_t words = int64_t(a.nq) * ((a.n + 31) / 32);
    const int64_t zb = std::min<int64_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_words, dim3(unsigned(zb)), dim3(256), 0, st, gbits, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t leaves = int64_t(a.m) * a.W * 32;
    hipLaunchKernelGGL(k_mark_candidates, dim3(unsigned((leaves + 255) / 256), unsigned(a.nq)), dim3(256), 0,
                       st, a, gbits);
    return hipGetLastError();
}

hipError_t launch_scan(const ScanArgs& a, int form, hipStream_t st) {
    if (a.nslice > 1 && (a.slice_words % kListWords || a.ncand ||
                         a.slice_words * a.nslice < (a.n + 31) / 32 || !a.part_s || !a.part_i))
        return hipErrorInvalidValue;
    const size_t lds = a.nslice > 1 ? scan_lds_bytes_words(a.slice_words, form, a.ld8)
                                    : scan_lds_bytes(a.n, form, a.ld8);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    switch (form) {
        case kFormFP32: return launch_form<kFormFP32>(a, st, lds);
        case kFormBF16: return launch_form<kFormBF16>(a, st, lds);
        case kFormFP8: return launch_form<kFormFP8>(a, st, lds);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gf
