// kernels.h -- argument blocks and launchers of the query-path kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gf {

// ---------------------------------------------------------------- selection

// A bin of the first-level key is resolved by the final per-query select
// once it holds at most kCollectCap leaves.  The narrowest bin, one key,
// holds one group: the leaves below a head at depth >= 1, at most 2^(H-1),
// so the collect buffer per query holds max(kCollectCap, 2^(H-1)) slots.
constexpr int kCollectCap = 32768;
inline int64_t collect_capacity(int H) {
    return H - 1 > 15 ? (int64_t{1} << (H - 1)) : int64_t{kCollectCap};
}
constexpr int kMaxPasses = 9;       // 63 significant key bits / 7-bit digits

enum : uint32_t { kSelSearching = 0, kSelReady = 1, kSelAll = 2, kSelDone = 3 };

// Counting walks of the selection, in launch order: a sample walk over tree
// 0 that estimates each query's threshold, one walk over every tree that
// counts a window of bins around the estimate, then radix passes for the
// queries whose window missed or whose bin is still too large.
enum : int { kPhSample = 0, kPhWindow = 1, kPhRadix = 2 };

struct SelState {
    uint64_t prefix;      // key bits above bit cs, fixed so far (K >> cs)
    uint32_t cs;          // bits of the key below the fixed prefix
    uint32_t phase;       // next counting walk that serves this query
    uint32_t base;        // sample / window walks: bin b >= 1 holds (E >> shift) == base + b
    uint32_t below;       // leaves whose key is below the current bin
    uint32_t budget;      // B of this query
    uint32_t status;
    uint32_t bincount;    // leaves inside the current bin
    uint32_t pad;
};

struct SelectArgs {
    const float* Q;        // [nq][ldq] device
    int64_t ldq;
    int nq;
    int m, H, t;
    int64_t n_internal;    // 2^H - 1
    int W;                 // leaf-bitmap words per tree
    const uint2* nodes;    // [m][n_internal]
    const int32_t* D;      // [t]
    const float2* drange;  // [t] smallest and largest split value on each slot of D
    int64_t leaves;        // leaves of the trees themselves: the budget's cap (below
                           // m 2^H for jittered trees, whose padding leaves stay closed)
    int nslice;            // m * (leaf ranges per tree)
    SelState* state;       // [nq]
    uint32_t* hist;        // [nq][nslice][128]
    uint32_t* coff;        // [nq][nslice] collect offsets
    int64_t ccap;          // collect slots per query: collect_capacity(H)
    uint64_t* ckey;        // [nq][ccap] keys (or M bits and tie keys, as two u32 halves)
    uint32_t* ccode;       // [nq][ccap]
    uint32_t* leafbits;    // [m][W][nq]  (word-major, query fastest)
    uint32_t* qlist;       // [nq] queries sent to the next radix pass, in flags[1] order
    int nlist;             // > 0: a radix walk serves qlist[0 .. nlist) only
    const float* qt;       // [m][nq][t] reflected query coordinates on D (isometry
                           // variant), or null: tree i then reads qt, else Q[q][D[j]]
};

// Isometry variant: qt[i][q][j] = float32(q_s - (2 u_i.q) u_i[s]) for s = D[j],
// with u_i.q summed in FP64 in index order (the build's definition).  UT is
// [d][m] (u_i[j] at UT[j m + i]); blocks of blockDim.x threads serve
// blockDim.x / mp queries, mp >= m a power of two dividing blockDim.x.
__global__ void k_reflect_queries(const float* Q, int64_t ldq, int nq, int d, int m, int mp, int t,
                                  const int32_t* D, const double* UT, float* qt);

// Also clears flags[0..1] (the radix-pass flags of k_select_pick).
__global__ void k_select_init(SelectArgs a, int32_t checks, const int32_t* cpq, double eps,
                              uint32_t* flags);
// flags[0]: set when some query goes on to a radix pass; flags[1]: how many.
// One workgroup per query: pick_threads(nslice) threads, at most kPickThreads.
constexpr int kPickThreads = 512;
inline int pick_threads(int nslice) { return nslice > 64 ? kPickThreads : 128; }
__global__ void k_select_pick(SelectArgs a, int phase, uint32_t* flags);
// leaf ranges per tree of the counting and collect walks (nslice = m times it)
int select_slices_per_tree(int H, int m, int nq);
// One workgroup per query, of finish_threads(nq) threads (256 or more; the
// histograms have 256 bins): small batches give each query more threads
// (measured: 230 -> 103 us at 128 queries with 1,024; 5.39 -> 5.25 ms of
// selection at 10,000 queries with 512 instead of 256, 5.88 with 1,024).
constexpr int kFinishThreadsMax = 1024;
inline int finish_threads(int nq) { return nq < 1024 ? kFinishThreadsMax : 512; }
__global__ void k_select_finish(SelectArgs a);
// phase: kPhSample / kPhWindow / kPhRadix for a counting walk (ignored with
// collect).  zfine > 1 splits each slice of a radix walk over zfine
// workgroups (for few remaining queries: shorter walks per workgroup).
hipError_t launch_select_walk(const SelectArgs& a, int phase, bool collect, hipStream_t st,
                              int zfine = 1);

// --------------------------------------------------------------------- scan

enum : int { kFormFP32 = 0, kFormBF16 = 1, kFormFP8 = 2 };

struct ScanArgs {
    int nq, k, kk;          // kk: list length kept per query (>= k)
    int64_t n;
    int d;
    int m, W, H;
    const uint32_t* leafbits;   // [m][W][nq]
    const uint32_t* permp;      // [m][2^H][pp] padded leaf rows
    int pp;
    const float* Q;             // [nq][ldq] FP32 queries (device)
    int64_t ldq;
    const float* X32;           // [n][ld32]
    int64_t ld32;
    // reduced-precision copies
    const uint16_t* X16; int64_t ld16; const float* norm16;
    const uint8_t* X8; int64_t ld8; const float* scale8; const float* norm8;
    const uint16_t* Q16;        // [nq][ld16] bf16 queries
    const uint8_t* Q8;          // [nq][ld8] e4m3 queries
    const float* qscale8;       // [nq]
    const float* qnorm;         // [nq] squared norm of the reduced query
    // outputs
    int32_t* ids;               // [nq][k]
    float* dists;               // [nq][k]
    uint32_t* cand_bits;        // [nq][ceil(n/32)] or null
    int64_t* ncand;             // [nq] or null
    // Slices: with nslice > 1 each query's id range is cut into nslice
    // slices of slice_words bitmap words (a multiple of 16), one workgroup
    // each; a slice writes its kk best to part_s / part_i
    // [nq][nslice][kTileList] (rest +inf) for the merge, instead of
    // finishing the query (cand_bits / ncand need nslice = 1).
    int nslice;
    int64_t slice_words;
    float* part_s;
    int* part_i;
    // [nq][ceil(n/32)] candidate bitmap built beforehand by
    // launch_mark_candidates (small sliced batches), or null: each slice
    // then expands the opened leaves itself
    const uint32_t* gbits;
};

// Scan kernel launch: one workgroup per query.  Returns hipErrorInvalidValue
// when the (form, d) combination has no instantiation.
hipError_t launch_scan(const ScanArgs& a, int form, hipStream_t st);
// LDS of a scan workgroup whose bitmap covers `words` words (ceil(n/32) unsliced).
size_t scan_lds_bytes_words(int64_t words, int form, int64_t ld8);
// Most bitmap words one scan workgroup's LDS holds (a multiple of 16), 0
// when not even one step fits (FP8 rows too wide to stage the query).  Id
// ranges above it are cut into slices of at most this many words.
int64_t scan_max_slice_words(int form, int64_t ld8);
// Candidate bitmap of each query, [nq][ceil(n/32)], from the opened leaves
// (cleared first), for the sliced scan of a small batch: one pass over the
// opened leaves instead of one per slice.
constexpr int kMarkMaxQueries = 64;
hipError_t launch_mark_candidates(const ScanArgs& a, uint32_t* gbits, hipStream_t st);
// Number of set bits of each query's row of an [nq][nbmw] bitmap.
hipError_t launch_count_bits(const uint32_t* bits, int nq, int64_t nbmw, int64_t* count, hipStream_t st);
size_t scan_lds_bytes(int64_t n, int form, int64_t ld8);
bool scan_supported(int64_t n, int form, int64_t ld8);

// ------------------------------------------------------- tile (MFMA) path

constexpr int kTileList = 48;   // best scores kept per (query, point split)
constexpr int kBoundWords = 4;   // per query: the shared bound and up to 3 splits' rank scores

// Candidate sets in point-major form for the tile path.  Queries are grouped
// in chunks of 32 cw (cw words of query bits per row, cw a power of two in
// [4, 32]); bit (q & 31) of word (q >> 5) % cw of a row belongs to query q.
struct ExpandArgs {
    int nq, m, W, H;
    int64_t n;
    int cw, nchunk;
    const uint32_t* leafbits;   // [m][W][nq] opened leaves, query fastest
    const uint32_t* leafof;     // [n][m] tree * 2^H + leaf holding each point
    const uint32_t* order;      // [n] point ids in tree 0's leaf order (the expansion's order)
    uint32_t* openT;            // [nchunk][m 2^H][cw] queries that opened each leaf
    uint32_t* visT;             // [nchunk][n][cw] queries having each point as candidate
    uint32_t* gthr;             // [nq][kBoundWords]: word 0 set to the bits of +inf
                                // here, words 1..nrb to 0xFFFFFFFF (no rank score
                                // yet), the rest to 0
    int nrb;                    // the tile kernel's rank-score splits (0: none)
};

struct TileArgs {
    int nq;
    int64_t n, ld16;
    int cw;
    const uint16_t* Q16;        // [nq][ld16]
    const uint16_t* X16;        // [n][ld16]
    const float* norm16;        // [n]
    const uint32_t* visT;       // [nchunk][n][cw]
    // [nq][kBoundWords]: word 0 holds the order-preserving bits of an upper
    // bound on the query's cap-th best score; words 1..nrb the splits' rank
    // scores (2 <= nsplit <= kBoundWords - 1 gives nrb = nsplit, else 0):
    // split s's rpub-th best, rpub = ceil(cap / nsplit), so that the largest
    // of the nrb is a bound as well, and is published to word 0.
    uint32_t* gthr;
    int cap;                    // list capacity per (query, split): the merge's kk, <= kTileList
    int nsplit;
    int nrb, rpos;              // rpos = cap - rpub: the list position of rank rpub - 1
    int64_t split_pts;          // points per split, multiple of 64, split_pts * ld16 * 2 < 2^31
    float* part_s;              // [nq][nsplit][kTileList]
    int* part_i;
};

struct MergeArgs {
    int nq, k, kk, d, nsplit;
    bool rerank;                // re-measure the kk in compensated FP32 (reduced-precision scores)
    const float* part_s;
    const int* part_i;
    const float* Q;             // [nq][ldq] FP32 queries
    int64_t ldq;
    const float* X32;
    int64_t ld32;
    int32_t* ids;
    float* dists;
};

// FP8 tile path (wide rows): dense FP8 MFMA scores of 128-query blocks
// against 128-point tiles, kept only for each query's candidates, written
// compactly per query, then the kk best per query.
constexpr int kTile8Queries = 256;   // queries per FP8 tile workgroup
struct Tile8Args {
    int nq;
    int64_t n, ld8;             // ld8: a multiple of 16
    int cw;                     // query words per chunk of visT
    int ntiles;                 // ceil(n / 128)
    int nsplit, split_tiles;    // point splits of split_tiles tiles each
    int64_t cap;                // candidate slots per query (>= its candidate count)
    int kk;                     // best entries kept per query (<= kTileList)
    const uint8_t* Q8;          // [nq][ld8] e4m3 queries
    const uint8_t* X8;          // [n][ld8] e4m3 points
    const float* qscale;        // [nq]
    const float* norm8;         // [n] ||dequantised x||^2
    const float* scale8;        // [n]
    const uint32_t* visT;       // [nchunk][n][cw] from the expansion
    uint64_t* masks;            // [nq][ntiles][2] candidate points of each tile
    uint32_t* offs;             // [nq][ntiles] candidates of the query before each tile
    uint32_t* total;            // [nq]
    float* out_s;               // [nq][cap] candidate scores, compacted
    int* out_i;                 // [nq][cap]
    float* part_s;              // [nq][kTileList] the kk best (rest +inf)
    int* part_i;
};
int tile8_ntiles(int64_t n);
// masks, prefix, scores and the per-query selection (nqw = ceil(nq / 32));
// ev (may be null) gets marks before and after the score kernel.
hipError_t launch_tile8(const Tile8Args& t, int nqw, hipStream_t st, hipEvent_t* ev);
// The tile path's merge of per-split lists, FP32 re-rank and FP64 ties.
hipError_t launch_merge(const MergeArgs& m, hipStream_t st);

// The expansion alone: openT and visT from the opened-leaf bits.
hipError_t launch_tile_expand(const ExpandArgs& e, hipStream_t st);
// The expansion, then visT in query-major form (cand_bits [nq][ceil(n/32)])
// and, if ncand is not null, each query's candidate count.
hipError_t launch_tile_trace(const ExpandArgs& e, uint32_t* cand_bits, int64_t* ncand, hipStream_t st);
// Records ev[0] after the expansion and ev[1] after the tile kernel (ev may
// be null).
hipError_t launch_tile_path(const ExpandArgs& e, const TileArgs& t, const MergeArgs& m,
                            hipStream_t st, hipEvent_t* ev);

// --------------------------------------------------------- data conversion

__global__ void k_to_bf16(const float* X, int64_t n, int d, int64_t ldx, uint16_t* Y,
                          int64_t ldy, float* norm);
__global__ void k_to_fp8(const float* X, int64_t n, int d, int64_t ldx, uint8_t* Y,
                         int64_t ldy, float* scale, float* norm);
__global__ void k_pad_rows(const float* X, int64_t n, int d, float* Y, int64_t ldy);
__global__ void k_check_finite(const float* X, int64_t n, int d, int64_t ld, uint32_t* bad);
__global__ void k_leafbits_to_query_major(const uint32_t* src, int nq, int64_t words,
                                          uint32_t* dst);
__global__ void k_e4m3_decode_both(float* hw, float* sw);
__global__ void k_e4m3_encode(const float* x, int n, uint8_t* y);

}  // namespace gf
