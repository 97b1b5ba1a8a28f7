// build.hip -- the forest build on the GPU (Alg. 1 and Alg. 3; Sec. 3
// "Median, variances" and "Parallelization").
//
//   k_col_welford    per-dimension (mean, M2) over row chunks with Knuth's
//                    online update (Alg. 3), one thread per column, FP64
//   k_col_combine    the chunks' triples combined in chunk order (Chan,
//                    Golub, LeVeque): V = M2 / (n - 1)
//   k_reflect_dots   u_i . x in FP64, index order, per (tree, point), for the
//                    isometry variant
//   k_level          one workgroup per node of one level of every tree: the
//                    node's split dimension from the generator, the split
//                    coordinates of its points, a radix select of the item of
//                    rank floor(|P|/2) under (coordinate, tie key, id), and a
//                    stable partition of its ids around that item
//   k_sort_leaves    every leaf's ids in ascending order
//
// The median item of a node is unique (the order is strict: ids differ), so
// the partition, the split value (the smallest coordinate on the right) and,
// once the leaves are sorted, every array equal the host build's bit for bit
// whatever order the items had inside a node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "forest.h"

namespace gf {

namespace {

constexpr int kBuildThreads = 256;
constexpr int kMaxDeviceLeaf = 4096;         // ids per leaf sorted in LDS
constexpr uint64_t kStreamSplitDim = 1;      // generator streams shared with the host build
constexpr uint64_t kStreamTieKey = 2;

// splitmix64 output function (Steele, Lea, Flood 2014) and the keyed draw
// built from it: the same published function as the host build's.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t stream, uint64_t tree, uint64_t idx) {
    uint64_t h = mix64(seed);
    h = mix64(h ^ stream);
    h = mix64(h ^ tree);
    return mix64(h ^ idx);
}

// Order-preserving uint32 image of a finite float, with -0 and +0 equal
// (they compare equal as floats).
__device__ __forceinline__ uint32_t coord_key(float x) {
    uint32_t u = __float_as_uint(x);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(kBuildThreads) void k_col_welford(const float* __restrict__ X, int64_t ld,
                                                              int64_t n, int d, int nchunk,
                                                              double* __restrict__ pmean,
                                                              double* __restrict__ pm2) {
#pragma clang fp contract(off)
    const int c = int(blockIdx.x) * kBuildThreads + int(threadIdx.x);
    const int ch = int(blockIdx.y);
    if (c >= d) return;
    const int64_t a = n * ch / nchunk, b = n * (ch + 1) / nchunk;
    double mu = 0.0, v = 0.0;
    for (int64_t i = a; i < b; ++i) {
        const double alpha = 1.0 / double(i - a + 1);
        const double x = double(X[i * ld + c]);
        const double delta = x - mu;
        mu += alpha * delta;
        v += delta * (x - mu);
    }
    pmean[int64_t(ch) * d + c] = mu;
    pm2[int64_t(ch) * d + c] = v;
}

__global__ __launch_bounds__(kBuildThreads) void k_col_combine(const double* __restrict__ pmean,
                                                              const double* __restrict__ pm2,
                                                              int64_t n, int d, int nchunk,
                                                              double* __restrict__ V,
                                                              double* __restrict__ M) {
#pragma clang fp contract(off)
    const int c = int(blockIdx.x) * kBuildThreads + int(threadIdx.x);
    if (c >= d) return;
    if (n < 2) { V[c] = 0.0; M[c] = 0.0; return; }
    double mu = pmean[c], v = pm2[c];
    double na = double(n / nchunk);   // rows of chunk 0: floor(n / nchunk)
    for (int ch = 1; ch < nchunk; ++ch) {
        const double nb = double(n * (ch + 1) / nchunk - n * ch / nchunk);
        if (nb == 0.0) continue;
        const double nt = na + nb;
        const double delta = pmean[int64_t(ch) * d + c] - mu;
        mu += delta * nb / nt;
        v += pm2[int64_t(ch) * d + c] + delta * delta * na * nb / nt;
        na = nt;
    }
    V[c] = v / double(n - 1);
    M[c] = mu;
}

// t = u . x of every (tree, point): products rounded, then added in index
// order, no fused multiply-add (the host build's reflector_dot).
__global__ __launch_bounds__(kBuildThreads) void k_reflect_dots(const float* __restrict__ X, int64_t ld,
                                                               int64_t n, int d, int m,
                                                               const double* __restrict__ U,
                                                               double* __restrict__ tdot) {
#pragma clang fp contract(off)
    const int64_t i = int64_t(blockIdx.x) * kBuildThreads + threadIdx.x;
    const int tree = int(blockIdx.y);
    if (i >= n || tree >= m) return;
    const float* x = X + i * ld;
    const double* u = U + int64_t(tree) * d;
    double acc = 0.0;
    for (int j = 0; j < d; ++j) {
        const double prod = u[j] * double(x[j]);
        acc = acc + prod;
    }
    tdot[int64_t(tree) * n + i] = acc;
}

// ids[tree][i] = i: every tree starts from the identity order
__global__ __launch_bounds__(kBuildThreads) void k_iota(uint32_t* __restrict__ ids, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kBuildThreads + threadIdx.x;
    if (i < n) ids[int64_t(blockIdx.y) * n + i] = uint32_t(i);
}

struct LevelArgs {
    const float* X;
    int64_t ld, n;
    int d, m, t, h;
    int64_t nint;             // internal nodes per tree
    uint64_t seed;
    const int32_t* D;         // [t]
    const double* U;          // [m][d] reflectors, or null
    const double* tdot;       // [m][n] u . x, or null
    const uint32_t* node_off; // [nint] first position of each node's segment
    const uint32_t* node_len; // [nint]
    const uint32_t* ids_in;   // [m][n] positions of this level
    uint32_t* ids_out;        // [m][n] positions of the next level
    uint32_t* keys;           // [m][n] coordinate keys (scratch)
    uint8_t* slot_out;        // [m][nint]
    float* val_out;           // [m][nint]
};

// Exclusive digit search over a 256-bin LDS histogram: the digit whose
// cumulative range holds `rank`, and rank minus the items below it.  Run by
// the first wave; each lane scans four bins.
__device__ __forceinline__ void pick_digit(const uint32_t* hist, uint32_t rank, uint32_t* out) {
    const int lane = threadIdx.x;
    uint32_t c[4], s = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) { c[j] = hist[4 * lane + j]; s += c[j]; }
    // inclusive prefix of the lane sums over the wave
    uint32_t incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    uint32_t below = incl - s;
    if (rank >= below && rank < incl) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (rank < below + c[j]) {
                out[0] = uint32_t(4 * lane + j);
                out[1] = rank - below;
                out[2] = c[j];
                break;
            }
            below += c[j];
        }
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_level(LevelArgs a) {
#pragma clang fp contract(off)
    __shared__ uint32_t hist[256];
    __shared__ uint32_t pick[3];
    __shared__ uint32_t wsum[2][NT / 64];
    const int tid = int(threadIdx.x);
    const int64_t per = int64_t(1) << a.h;
    const int tree = int(int64_t(blockIdx.x) / per);
    const int64_t v = per - 1 + int64_t(blockIdx.x) % per;
    const int64_t o = a.node_off[v];
    const int64_t len = a.node_len[v];
    const uint64_t r = draw(a.seed, kStreamSplitDim, uint64_t(tree), uint64_t(v));
    const int slot = int(r % uint64_t(a.t));
    const int s = a.D[slot];
    const uint32_t* ids = a.ids_in + int64_t(tree) * a.n + o;
    uint32_t* keys = a.keys + int64_t(tree) * a.n + o;
    // split coordinates of the node's points (reflected in the isometry variant)
    for (int64_t i = tid; i < len; i += NT) {
        uint32_t id = ids[i];
        if (id >= uint32_t(a.n)) id = 0;   // never taken when the levels above partitioned correctly
        float x = a.X[int64_t(id) * a.ld + s];
        if (a.U) {
            const double r2 = (2.0 * a.tdot[int64_t(tree) * a.n + id]) * a.U[int64_t(tree) * a.d + s];
            x = float(double(x) - r2);
        }
        keys[i] = coord_key(x);
    }
    __syncthreads();

    // radix select of the item of rank nl: first on the coordinate key, then
    // (only among items tied with it) on the tie key, then on the id
    const uint32_t nl = uint32_t(len / 2);
    uint32_t rank = nl;
    uint32_t xk = 0;              // coordinate key of the median item
    uint64_t tk = 0;              // its tie key (when needed)
    uint32_t ik = 0;              // its id (when needed)
    int depth = 0;                // 1: ties on the coordinate, 2: also on the tie key
    uint32_t tied = 0;
    for (int pass = 0; pass < 4; ++pass) {
        const int sh = 24 - 8 * pass;
        for (int b = tid; b < 256; b += NT) hist[b] = 0;
        __syncthreads();
        for (int64_t i = tid; i < len; i += NT) {
            const uint32_t k = keys[i];
            if (pass == 0 || (k >> (sh + 8)) == (xk >> (sh + 8))) atomicAdd(&hist[(k >> sh) & 255u], 1u);
        }
        __syncthreads();
        if (tid < 64) pick_digit(hist, rank, pick);
        __syncthreads();
        xk |= pick[0] << sh;
        rank = pick[1];
        tied = pick[2];
        __syncthreads();
    }
    if (tied > 1) {
        depth = 1;
        for (int pass = 0; pass < 8; ++pass) {
            const int sh = 56 - 8 * pass;
            for (int b = tid; b < 256; b += NT) hist[b] = 0;
            __syncthreads();
            for (int64_t i = tid; i < len; i += NT) {
                if (keys[i] != xk) continue;
                const uint64_t k = draw(a.seed, kStreamTieKey, uint64_t(tree), uint64_t(ids[i]));
                if (pass == 0 || (k >> (sh + 8)) == (tk >> (sh + 8)))
                    atomicAdd(&hist[uint32_t(k >> sh) & 255u], 1u);
            }
            __syncthreads();
            if (tid < 64) pick_digit(hist, rank, pick);
            __syncthreads();
            tk |= uint64_t(pick[0]) << sh;
            rank = pick[1];
            tied = pick[2];
            __syncthreads();
        }
        if (tied > 1) {
            depth = 2;
            for (int pass = 0; pass < 4; ++pass) {
                const int sh = 24 - 8 * pass;
                for (int b = tid; b < 256; b += NT) hist[b] = 0;
                __syncthreads();
                for (int64_t i = tid; i < len; i += NT) {
                    if (keys[i] != xk) continue;
                    const uint32_t id = ids[i];
                    if (draw(a.seed, kStreamTieKey, uint64_t(tree), uint64_t(id)) != tk) continue;
                    if (pass == 0 || (id >> (sh + 8)) == (ik >> (sh + 8))) atomicAdd(&hist[(id >> sh) & 255u], 1u);
                }
                __syncthreads();
                if (tid < 64) pick_digit(hist, rank, pick);
                __syncthreads();
                ik |= pick[0] << sh;
                rank = pick[1];
                __syncthreads();
            }
        }
    }

    // stable partition: items before the median item go left (positions
    // o .. o + nl), the others right, each side in chunk order
    uint32_t* out = a.ids_out + int64_t(tree) * a.n + o;
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t lbase = 0, rbase = 0;
    for (int64_t c0 = 0; c0 < len; c0 += NT) {
        const int64_t i = c0 + tid;
        bool left = false, pivot = false;
        uint32_t id = 0;
        if (i < len) {
            id = ids[i];
            const uint32_t k = keys[i];
            if (k < xk) {
                left = true;
            } else if (k == xk) {
                if (depth == 0) {
                    pivot = true;
                } else {
                    const uint64_t tv = draw(a.seed, kStreamTieKey, uint64_t(tree), uint64_t(id));
                    left = tv < tk || (depth > 1 && tv == tk && id < ik);
                    pivot = tv == tk && (depth == 1 || id == ik);
                }
            }
        }
        if (pivot) {
            // the split value is the median item's own coordinate (-0 and +0
            // share a key but keep their sign here)
            const uint32_t pid = id < uint32_t(a.n) ? id : 0u;
            float x = a.X[int64_t(pid) * a.ld + s];
            if (a.U) {
                const double r2 = (2.0 * a.tdot[int64_t(tree) * a.n + pid]) * a.U[int64_t(tree) * a.d + s];
                x = float(double(x) - r2);
            }
            a.val_out[int64_t(tree) * a.nint + v] = x;
        }
        const uint64_t lb = __ballot(i < len && left), rb = __ballot(i < len && !left);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const uint32_t lr = uint32_t(__popcll(lb & below)), rr = uint32_t(__popcll(rb & below));
        if (lane == 0) { wsum[0][wave] = uint32_t(__popcll(lb)); wsum[1][wave] = uint32_t(__popcll(rb)); }
        __syncthreads();
        uint32_t lw = 0, rw = 0, lt = 0, rt = 0;
        for (int w = 0; w < NT / 64; ++w) {
            if (w < wave) { lw += wsum[0][w]; rw += wsum[1][w]; }
            lt += wsum[0][w];
            rt += wsum[1][w];
        }
        if (i < len) {
            // exactly nl items precede the median item; the bounds only keep
            // a failed select inside the node's segment
            const uint32_t li = lbase + lw + lr, ri = nl + rbase + rw + rr;
            if (left) { if (li < nl) out[li] = id; }
            else if (ri < uint32_t(len)) out[ri] = id;
        }
        lbase += lt;
        rbase += rt;
        __syncthreads();
    }
    if (tid == 0) a.slot_out[int64_t(tree) * a.nint + v] = uint8_t(slot);
}

// Ids of every leaf in ascending order: one workgroup per (tree, leaf), a
// bitonic sort in LDS padded to a power of two with 0xFFFFFFFF.
__global__ __launch_bounds__(kBuildThreads) void k_sort_leaves(uint32_t* __restrict__ ids,
                                                              const uint32_t* __restrict__ leaf_off,
                                                              int64_t n, int H) {
    __shared__ uint32_t s[kMaxDeviceLeaf];
    const int64_t nleaf = int64_t(1) << H;
    const int tree = int(int64_t(blockIdx.x) / nleaf);
    const int64_t j = int64_t(blockIdx.x) % nleaf;
    const uint32_t o = leaf_off[j], len = leaf_off[j + 1] - o;
    if (len < 2) return;
    uint32_t* p = ids + int64_t(tree) * n + o;
    uint32_t np2 = 1;
    while (np2 < len) np2 <<= 1;
    for (uint32_t i = threadIdx.x; i < np2; i += kBuildThreads) s[i] = i < len ? p[i] : 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t size = 2; size <= np2; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < np2; i += kBuildThreads) {
                const uint32_t partner = i ^ stride;
                if (partner > i) {
                    const bool up = (i & size) == 0;
                    const uint32_t x = s[i], y = s[partner];
                    if ((x > y) == up) { s[i] = y; s[partner] = x; }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < len; i += kBuildThreads) p[i] = s[i];
}

template <class T>
struct DevBuf {
    T* p = nullptr;
    hipError_t alloc(size_t count) {
        return dev_malloc(reinterpret_cast<void**>(&p), std::max<size_t>(count, 1) * sizeof(T));
    }
    ~DevBuf() { dev_free(p); }
};

}  // namespace

std::string build_device_forest(const float* X32, int64_t ld32, int64_t n, int32_t d, int32_t m,
                                int32_t t, int32_t p, uint64_t seed, bool householder,
                                hipStream_t st, HostForest& F) {
    F = HostForest{};
    F.n = n; F.d = d; F.m = m; F.t = t; F.p = p; F.seed = seed;
    F.H = perfect_depth(n, p);
    if (F.H > 23) return "tree depth above 23 (n/leaf too large)";
    const int H = F.H;
    const int64_t nint = (int64_t{1} << H) - 1;
    const int64_t nleaf = int64_t{1} << H;
#define GF_TRY(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return std::string(#expr) + ": " + hipGetErrorString(e_); \
    } while (0)

    // node segments: sizes split floor / ceil level by level, the same in
    // every tree; leaves last
    std::vector<uint32_t> noff(size_t(std::max<int64_t>(nint, 1))), nlen(noff.size());
    std::vector<int64_t> size{n}, off{0};
    for (int h = 0; h < H; ++h) {
        std::vector<int64_t> ns, no;
        for (size_t j = 0; j < size.size(); ++j) {
            const int64_t v = (int64_t{1} << h) - 1 + int64_t(j);
            noff[v] = uint32_t(off[j]);
            nlen[v] = uint32_t(size[j]);
            ns.push_back(size[j] / 2); no.push_back(off[j]);
            ns.push_back(size[j] - size[j] / 2); no.push_back(off[j] + size[j] / 2);
        }
        size.swap(ns);
        off.swap(no);
    }
    std::vector<uint32_t> lo(nleaf + 1);     // the same in every tree
    lo[0] = 0;
    uint32_t maxleaf = 0;
    for (int64_t j = 0; j < nleaf; ++j) {
        lo[j + 1] = uint32_t(lo[j] + size[j]);
        maxleaf = std::max(maxleaf, uint32_t(size[j]));
    }
    F.leaf_off.resize(size_t(m) * (nleaf + 1));
    for (int32_t tr = 0; tr < m; ++tr) std::copy(lo.begin(), lo.end(), F.leaf_off.begin() + size_t(tr) * (nleaf + 1));
    F.real_leaves = int64_t(m) * nleaf;
    if (maxleaf > uint32_t(kMaxDeviceLeaf)) return "leaves above 4096 points are built on the host only";

    // V, M: column moments on the device; D and the near-tie guard from them
    const int nchunk = int(std::min<int64_t>(256, std::max<int64_t>(1, n / 1024)));
    DevBuf<double> pmean, pm2, dV, dM;
    GF_TRY(pmean.alloc(size_t(nchunk) * d));
    GF_TRY(pm2.alloc(size_t(nchunk) * d));
    GF_TRY(dV.alloc(d));
    GF_TRY(dM.alloc(d));
    const unsigned cblk = unsigned((d + kBuildThreads - 1) / kBuildThreads);
    hipLaunchKernelGGL(k_col_welford, dim3(cblk, unsigned(nchunk)), dim3(kBuildThreads), 0, st, X32, ld32,
                       n, d, nchunk, pmean.p, pm2.p);
    GF_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_col_combine, dim3(cblk), dim3(kBuildThreads), 0, st, pmean.p, pm2.p, n, d, nchunk,
                       dV.p, dM.p);
    GF_TRY(hipGetLastError());
    std::vector<double> V(d), M(d);
    GF_TRY(hipMemcpyAsync(V.data(), dV.p, size_t(d) * 8, hipMemcpyDeviceToHost, st));
    GF_TRY(hipMemcpyAsync(M.data(), dM.p, size_t(d) * 8, hipMemcpyDeviceToHost, st));
    GF_TRY(hipStreamSynchronize(st));
    std::string err = select_dims(V, M, n, t, F.D);
    if (!err.empty()) return err;

    DevBuf<int32_t> dD;
    GF_TRY(dD.alloc(t));
    GF_TRY(hipMemcpyAsync(dD.p, F.D.data(), size_t(t) * 4, hipMemcpyHostToDevice, st));
    DevBuf<double> dU, tdot;
    if (householder) {
        F.U.resize(size_t(m) * d);
        for (int32_t tr = 0; tr < m; ++tr) householder_vector(seed, tr, d, F.U.data() + size_t(tr) * d);
        GF_TRY(dU.alloc(F.U.size()));
        GF_TRY(hipMemcpyAsync(dU.p, F.U.data(), F.U.size() * 8, hipMemcpyHostToDevice, st));
        GF_TRY(tdot.alloc(size_t(m) * n));
        hipLaunchKernelGGL(k_reflect_dots, dim3(unsigned((n + kBuildThreads - 1) / kBuildThreads), unsigned(m)),
                           dim3(kBuildThreads), 0, st, X32, ld32, n, d, m, dU.p, tdot.p);
        GF_TRY(hipGetLastError());
    }

    // levels: ping-pong id arrays, identity order to start
    DevBuf<uint32_t> idsA, idsB, keys, dnoff, dnlen, dlo;
    DevBuf<uint8_t> dslot;
    DevBuf<float> dval;
    GF_TRY(idsA.alloc(size_t(m) * n));
    GF_TRY(idsB.alloc(size_t(m) * n));
    GF_TRY(keys.alloc(size_t(m) * n));
    GF_TRY(dnoff.alloc(noff.size()));
    GF_TRY(dnlen.alloc(nlen.size()));
    GF_TRY(dlo.alloc(lo.size()));
    GF_TRY(dslot.alloc(size_t(m) * std::max<int64_t>(nint, 1)));
    GF_TRY(dval.alloc(size_t(m) * std::max<int64_t>(nint, 1)));
    GF_TRY(hipMemcpyAsync(dnoff.p, noff.data(), noff.size() * 4, hipMemcpyHostToDevice, st));
    GF_TRY(hipMemcpyAsync(dnlen.p, nlen.data(), nlen.size() * 4, hipMemcpyHostToDevice, st));
    GF_TRY(hipMemcpyAsync(dlo.p, lo.data(), lo.size() * 4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_iota, dim3(unsigned((n + kBuildThreads - 1) / kBuildThreads), unsigned(m)),
                       dim3(kBuildThreads), 0, st, idsA.p, n);
    GF_TRY(hipGetLastError());
    uint32_t* cur = idsA.p;
    uint32_t* nxt = idsB.p;
    for (int h = 0; h < H; ++h) {
        LevelArgs la{X32, ld32, n, d, m, t, h, nint, seed, dD.p, householder ? dU.p : nullptr,
                     householder ? tdot.p : nullptr, dnoff.p, dnlen.p, cur, nxt, keys.p, dslot.p, dval.p};
        // workgroup size by the level's largest node
        const int64_t big = (n + (int64_t{1} << h) - 1) >> h;
        const dim3 grid(unsigned(int64_t(m) << h));
        if (big >= 65536) hipLaunchKernelGGL(k_level<1024>, grid, dim3(1024), 0, st, la);
        else if (big >= 1024) hipLaunchKernelGGL(k_level<256>, grid, dim3(256), 0, st, la);
        else hipLaunchKernelGGL(k_level<64>, grid, dim3(64), 0, st, la);
        GF_TRY(hipGetLastError());
        std::swap(cur, nxt);
    }
    hipLaunchKernelGGL(k_sort_leaves, dim3(unsigned(int64_t(m) * nleaf)), dim3(kBuildThreads), 0, st, cur,
                       dlo.p, n, H);
    GF_TRY(hipGetLastError());

    F.perm.resize(size_t(m) * n);
    F.split_slot.assign(size_t(m) * nint, 0);
    F.split_val.assign(size_t(m) * nint, 0.0f);
    F.split_dim.assign(size_t(m) * nint, 0);
    GF_TRY(hipMemcpyAsync(F.perm.data(), cur, F.perm.size() * 4, hipMemcpyDeviceToHost, st));
    if (nint > 0) {
        GF_TRY(hipMemcpyAsync(F.split_slot.data(), dslot.p, F.split_slot.size(), hipMemcpyDeviceToHost, st));
        GF_TRY(hipMemcpyAsync(F.split_val.data(), dval.p, F.split_val.size() * 4, hipMemcpyDeviceToHost, st));
    }
    GF_TRY(hipStreamSynchronize(st));
    for (size_t i = 0; i < F.split_slot.size(); ++i) F.split_dim[i] = F.D[F.split_slot[i]];
#undef GF_TRY
    return {};
}

}  // namespace gf
