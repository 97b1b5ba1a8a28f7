// rank.h -- wavefront-level best-k lists, exact re-measurement of selected
// candidates, and the final ranking of a query (shared by the scan kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gf {

constexpr int kWave = 64;
constexpr float kTieBand = 1e-5f;   // relative band around the k-th distance re-checked in FP64

__device__ __forceinline__ bool entry_before(float da, int ia, float db, int ib) {
    return da < db || (da == db && ia < ib);
}

// Sorted best-kk list spread over lanes 0..kk-1 of a wavefront.
struct WaveList {
    float d;
    int id;
    __device__ __forceinline__ void init() { d = __builtin_inff(); id = 0x7FFFFFFF; }
    __device__ __forceinline__ float thr_d(int kk) const {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), kk - 1));
    }
    __device__ __forceinline__ int thr_id(int kk) const { return __builtin_amdgcn_readlane(id, kk - 1); }
    // Insert a wave-uniform (dc, ic) known to beat the current kk-th entry.
    __device__ __forceinline__ void insert(float dc, int ic, int kk) {
        const int lane = threadIdx.x & (kWave - 1);
        const bool before = lane < kk && entry_before(d, id, dc, ic);
        const int pos = __popcll(__ballot(before));
        const float pd = __shfl_up(d, 1);
        const int pi = __shfl_up(id, 1);
        if (lane < kk) {
            if (lane > pos) { d = pd; id = pi; }
            else if (lane == pos) { d = dc; id = ic; }
        }
    }
    __device__ __forceinline__ void offer(float dc, int ic, int kk) {
        const float td = thr_d(kk);
        const int ti = thr_id(kk);
        if (entry_before(dc, ic, td, ti)) insert(dc, ic, kk);
    }
};

// Compensated FP32 squared distance of one row, computed by a whole wave:
// (q - x) split exactly into s + e (two-sum), s^2 split exactly into p + r
// (two-product with FMA), the p's summed with two-sum and every rounding
// error collected in a second accumulator (Ogita, Rump, Oishi 2005).
// Each lane takes j = lane, lane + 64, ... in order; the loads of kRowUnroll
// steps are issued before any is used (a position past d reads as zero, and
// a zero term leaves sum and err exactly as they were).
constexpr int kRowUnroll = 8;

__device__ __forceinline__ float row_dist_fp32_comp(const float* q, const float* x, int d) {
    const int lane = threadIdx.x & (kWave - 1);
    float sum = 0.0f, err = 0.0f;
    for (int j0 = lane; j0 < d; j0 += kRowUnroll * kWave) {
        float qa[kRowUnroll], xb[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const int j = j0 + u * kWave;
            qa[u] = j < d ? q[j] : 0.0f;
            xb[u] = j < d ? x[j] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const float a = qa[u], b = -xb[u];
            const float s = a + b;
            const float bb = s - a;
            const float e = (a - (s - bb)) + (b - bb);
            const float p = s * s;
            const float r = fmaf(s, s, -p);
            const float t = sum + p;
            const float tp = t - sum;
            err += ((sum - (t - tp)) + (p - tp)) + r + fmaf(2.0f * s, e, e * e);
            sum = t;
        }
    }
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        const float os = __shfl_xor(sum, o);
        const float oe = __shfl_xor(err, o);
        const float t = sum + os;
        const float tp = t - sum;
        err = err + oe + ((sum - (t - tp)) + (os - tp));
        sum = t;
    }
    return sum + err;
}

__device__ __forceinline__ double row_dist_fp64(const float* q, const float* x, int d) {
    const int lane = threadIdx.x & (kWave - 1);
    double acc = 0.0;
    for (int j0 = lane; j0 < d; j0 += kRowUnroll * kWave) {
        float qa[kRowUnroll], xb[kRowUnroll];
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const int j = j0 + u * kWave;
            qa[u] = j < d ? q[j] : 0.0f;
            xb[u] = j < d ? x[j] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kRowUnroll; ++u) {
            const double diff = double(qa[u]) - double(xb[u]);
            acc = fma(diff, diff, acc);
        }
    }
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    return acc;
}

// Re-rank the list by (FP64 distance, id) inside the band of the k-th place.
__device__ __forceinline__ void refine_ties(WaveList& L, int kk, int k, const float* q, const float* X32,
                            int64_t ld32, int d) {
    const int lane = threadIdx.x & (kWave - 1);
    const float dk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(L.d), k - 1));
    double key = double(L.d);
    if (dk < __builtin_inff()) {
        const float lo = dk * (1.0f - kTieBand), hi = dk * (1.0f + kTieBand);
        const bool inband = lane < kk && L.d >= lo && L.d <= hi && L.d < __builtin_inff();
        uint64_t band = __ballot(inband);
        while (band) {
            const int b = __builtin_ctzll(band);
            band &= band - 1;
            const int id = __builtin_amdgcn_readlane(L.id, b);
            const double d64 = row_dist_fp64(q, X32 + int64_t(id) * ld32, d);
            if (lane == b) key = d64;
        }
    }
    // bitonic sort of the 64 lanes by (key, id); lanes >= kk carry +inf
    int id = L.id;
    if (lane >= kk) { key = __builtin_inf(); id = 0x7FFFFFFF; }
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const double ok = __shfl_xor(key, stride);
            const int oid = __shfl_xor(id, stride);
            const bool up = (lane & size) == 0;
            const bool lower = (lane & stride) == 0;
            const bool other_first = ok < key || (ok == key && oid < id);
            const bool take = (lower == up) ? other_first : !other_first;
            if (take) { key = ok; id = oid; }
        }
    }
    L.d = float(key);
    L.id = id;
}

// Final steps of one query, run by a whole workgroup once the best `kk`
// candidates of the selection score sit in lds_d / lds_i (and, for wave 0,
// in L, sorted).  Reduced-precision forms (rerank = true): every wave
// re-measures some of them on the FP32 rows (compensated), wave 0 ranks them
// again.  Then wave 0 re-checks the k-th place tie band in FP64 and writes
// the k best (padding with -1 / +inf).  Contains __syncthreads.
__device__ __forceinline__ void finish_query(bool rerank, int kk, int k, int q, const float* qf,
                                             const float* X32, int64_t ld32, int d,
                                             float* lds_d, int* lds_i, float* lds_rr, WaveList& L,
                                             int32_t* ids, float* dists) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    if (rerank) {
        for (int e = wave; e < kk; e += nwaves) {
            const int id = lds_i[e];
            float dv = __builtin_inff();
            if (lds_d[e] < __builtin_inff()) dv = row_dist_fp32_comp(qf, X32 + int64_t(id) * ld32, d);
            if (lane == 0) lds_rr[e] = dv;
        }
        __syncthreads();
        // order the re-measured entries: thread e takes the rank of entry e
        // among them by (distance, id) (ids are distinct, so ranks are too)
        const int t = int(threadIdx.x);
        float dv = __builtin_inff();
        int iv = 0x7FFFFFFF, rank = kk;
        if (t < kk) {
            dv = lds_rr[t];
            iv = lds_i[t];
            if (dv < __builtin_inff()) {
                rank = 0;
                for (int f = 0; f < kk; ++f) {
                    const float fd = lds_rr[f];
                    if (fd < __builtin_inff() && entry_before(fd, lds_i[f], dv, iv)) ++rank;
                }
            }
        }
        __syncthreads();
        if (t < kk) { lds_d[t] = __builtin_inff(); lds_i[t] = 0x7FFFFFFF; }
        __syncthreads();
        if (rank < kk) { lds_d[rank] = dv; lds_i[rank] = iv; }
        __syncthreads();
        if (wave == 0) {
            L.d = lane < kk ? lds_d[lane] : __builtin_inff();
            L.id = lane < kk ? lds_i[lane] : 0x7FFFFFFF;
        }
    }
    if (wave == 0) {
        refine_ties(L, kk, k, qf, X32, ld32, d);
        if (lane < k) {
            const bool have = L.d < __builtin_inff();
            ids[int64_t(q) * k + lane] = have ? L.id : -1;
            dists[int64_t(q) * k + lane] = have ? L.d : __builtin_inff();
        }
    }
}

// OR the point ids of every opened leaf of query q into the LDS bitmap bm.
// Threads take whole words (32 leaves of one tree) of the query's leaf
// bitmap, strided by `stride`; each opened leaf is one padded row of pp ids
// (16-byte aligned, unused slots 0xFFFFFFFF), read as 16-byte vectors, two
// leaves in flight at a time.  leafbits: [m][W][nq] words.  Only ids whose
// bitmap word lies in [w_lo, w_hi) are kept, at word (id / 32) - w_lo (a
// slice of the id range).
__device__ __forceinline__ void expand_opened_leaves(uint32_t* bm, const uint32_t* leafbits, int q,
                                                     int nq, int m, int W, int H,
                                                     const uint32_t* permp, int pp, int first,
                                                     int stride, int64_t w_lo = 0,
                                                     int64_t w_hi = int64_t(1) << 62) {
    const int64_t nwords = int64_t(m) * W;
    const int64_t nleaf = int64_t(1) << H;      // leaves per tree (rows per tree in permp)
    const int pp4 = pp / 4;
    for (int64_t f = first; f < nwords; f += stride) {
        uint32_t bits = leafbits[f * nq + q];
        const int64_t tree = f / W;
        const int64_t leaf0 = (f % W) * 32;
        while (bits) {
            const int ja = __builtin_ctz(bits);
            bits &= bits - 1;
            int jb = -1;
            if (bits) { jb = __builtin_ctz(bits); bits &= bits - 1; }
            const uint4* ra = reinterpret_cast<const uint4*>(permp + ((tree * nleaf) + leaf0 + ja) * pp);
            const uint4* rb = reinterpret_cast<const uint4*>(permp + ((tree * nleaf) + leaf0 + (jb < 0 ? ja : jb)) * pp);
            for (int c = 0; c < pp4; c += 8) {
                uint4 va[8], vb[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const bool ok = c + i < pp4;
                    va[i] = ok ? ra[c + i] : make_uint4(~0u, ~0u, ~0u, ~0u);
                    vb[i] = (ok && jb >= 0) ? rb[c + i] : make_uint4(~0u, ~0u, ~0u, ~0u);
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint32_t ids[8] = {va[i].x, va[i].y, va[i].z, va[i].w,
                                             vb[i].x, vb[i].y, vb[i].z, vb[i].w};
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int64_t wd = int64_t(ids[e] >> 5);
                        if (ids[e] != 0xFFFFFFFFu && wd >= w_lo && wd < w_hi)
                            atomicOr(&bm[wd - w_lo], 1u << (ids[e] & 31u));
                    }
                }
            }
        }
    }
}

}  // namespace gf
