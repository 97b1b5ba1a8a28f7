// capi.hip -- the C ABI (include/geraf.h): validation, device memory, and
// the order of the query-path launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "forest.h"
#include "kernels.h"

namespace {

thread_local std::string g_last_error;
// Phase times of the last gf_query / gf_query_trace call on this thread (ms):
// query prep, leaf selection, then either the row scan (expansion +
// distances + best-k + re-rank) or the tile path's expansion, MFMA tile
// kernel and merge/re-rank; summed over the call's batches.
constexpr int kPhases = 5;
thread_local double g_phase_ms[kPhases] = {0.0, 0.0, 0.0, 0.0, 0.0};
thread_local int32_t g_path = 0;
thread_local int64_t g_batches = 0;

gf_status fail(gf_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

// out-of-memory (the runtime's, or the cap below) reports GF_ENOMEM
#define GF_HIP(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? GF_ENOMEM : GF_EHIP,                 \
                        std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

// Device memory held by the library, against an optional cap: the
// environment variable GF_MAX_DEVICE_BYTES (read at every allocation), when
// set to a positive byte count, makes any allocation that would take the
// library's total above it fail with hipErrorOutOfMemory (GF_ENOMEM).
std::mutex g_alloc_mutex;
std::unordered_map<void*, size_t> g_alloc_size;
size_t g_alloc_total = 0;

size_t device_cap() {
    const char* e = std::getenv("GF_MAX_DEVICE_BYTES");
    if (!e || !*e) return 0;
    char* end = nullptr;
    const unsigned long long v = std::strtoull(e, &end, 10);
    return (end && *end == '\0') ? size_t(v) : 0;
}

bool exceeds_cap(size_t more) {
    const size_t cap = device_cap();
    std::lock_guard<std::mutex> lock(g_alloc_mutex);
    return cap != 0 && g_alloc_total + more > cap;
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct DevFree {
    void operator()(void* p) const { gf::dev_free(p); }
};

bool is_device_ptr(const void* p) {
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged ||
           attr.isManaged;
}

bool all_finite_host(const float* X, int64_t count) {
    const unsigned nw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<char> ok(nw, 1);
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nw; ++w)
        th.emplace_back([&, w] {
            int64_t a = count * w / nw, b = count * (w + 1) / nw;
            for (int64_t i = a; i < b; ++i)
                if (!std::isfinite(X[i])) { ok[w] = 0; return; }
        });
    for (auto& t : th) t.join();
    for (char c : ok)
        if (!c) return false;
    return true;
}

// rows [n][d] -> dst [n][ld] in host memory, zero-padded, with host threads
// for large copies (about one per 4 MB, at most 16).
void pad_rows(float* dst, const float* src, int64_t n, int32_t d, int32_t ld) {
    const size_t bytes = size_t(n) * size_t(ld) * 4;
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const unsigned nw = unsigned(std::max<size_t>(1, std::min<size_t>(hw, bytes >> 22)));
    auto part = [=](unsigned w) {
        for (int64_t i = n * w / nw; i < n * (w + 1) / nw; ++i) {
            std::memcpy(dst + i * ld, src + i * d, size_t(d) * 4);
            if (ld > d) std::memset(dst + i * ld + d, 0, size_t(ld - d) * 4);
        }
    };
    if (nw == 1) { part(0); return; }
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nw; ++w) th.emplace_back(part, w);
    for (auto& x : th) x.join();
}

// X (pageable host memory) -> dst [n][ld] on the device, rows zero-padded
// to ld.  Pageable sources are copied slowly by the runtime, so the rows go
// through two pinned buffers: host threads fill one while the other is
// copied.  Returns the first HIP error, after the stream has drained.
hipError_t upload_rows(float* dst, const float* Xh, int64_t n, int32_t d, int32_t ld, hipStream_t st) {
    const size_t row_bytes = size_t(ld) * 4;
    const int64_t rows_per = std::min<int64_t>(n, std::max<int64_t>(1, int64_t((size_t{128} << 20) / row_bytes)));
    const int64_t nchunk = (n + rows_per - 1) / rows_per;
    const int nbuf = nchunk > 1 ? 2 : 1;
    void* buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t err = hipSuccess;
    for (int b = 0; b < nbuf && err == hipSuccess; ++b) {
        err = hipHostMalloc(&buf[b], size_t(rows_per) * row_bytes, hipHostMallocDefault);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&ev[b], hipEventDisableTiming);
    }
    for (int64_t c = 0; c < nchunk && err == hipSuccess; ++c) {
        const int b = int(c % nbuf);
        if (c >= nbuf && (err = hipEventSynchronize(ev[b])) != hipSuccess) break;   // buffer free again
        const int64_t r0 = c * rows_per, rows = std::min(rows_per, n - r0);
        float* hb = static_cast<float*>(buf[b]);
        pad_rows(hb, Xh + r0 * d, rows, d, ld);
        err = hipMemcpyAsync(dst + r0 * ld, hb, size_t(rows) * row_bytes, hipMemcpyHostToDevice, st);
        if (err == hipSuccess) err = hipEventRecord(ev[b], st);
    }
    const hipError_t sync = hipStreamSynchronize(st);
    if (err == hipSuccess) err = sync;
    for (int b = 0; b < 2; ++b) {
        if (ev[b]) (void)hipEventDestroy(ev[b]);
        if (buf[b]) (void)hipHostFree(buf[b]);
    }
    return err;
}

// Host query rows -> dst [rows][ld] on the device through the forest's
// pinned staging buffer (grown on demand).  The stream is drained first, so
// the buffer is free to refill; the caller synchronises before the next use.
hipError_t stage_host_rows(gf_forest* F, float* dst, const float* src, int64_t rows, int32_t d,
                           int32_t ld, hipStream_t st) {
    const size_t bytes = size_t(rows) * size_t(ld) * 4;
    hipError_t err = hipStreamSynchronize(st);
    if (err != hipSuccess) return err;
    if (bytes > F->hstage_bytes) {
        if (F->hstage) (void)hipHostFree(F->hstage);
        F->hstage = nullptr;
        F->hstage_bytes = 0;
        if ((err = hipHostMalloc(&F->hstage, bytes, hipHostMallocDefault)) != hipSuccess) return err;
        F->hstage_bytes = bytes;
    }
    pad_rows(static_cast<float*>(F->hstage), src, rows, d, ld);
    return hipMemcpyAsync(dst, F->hstage, bytes, hipMemcpyHostToDevice, st);
}

void free_forest_device(gf_forest* F) {
    void* ptrs[] = {F->X32, F->X16, F->norm16, F->X8, F->scale8, F->norm8,
                    F->nodes, F->perm, F->leaf_off, F->permp, F->leafof, F->D, F->drange, F->U, F->ws};
    for (void* p : ptrs)
        gf::dev_free(p);
    F->X32 = nullptr; F->X16 = nullptr; F->norm16 = nullptr; F->X8 = nullptr;
    F->scale8 = nullptr; F->norm8 = nullptr; F->nodes = nullptr; F->perm = nullptr;
    F->leaf_off = nullptr; F->permp = nullptr; F->leafof = nullptr; F->D = nullptr; F->drange = nullptr;
    F->U = nullptr;
    if (F->hstage) (void)hipHostFree(F->hstage);
    F->hstage = nullptr;
    F->hstage_bytes = 0;
    F->ws = nullptr;
    F->ws_bytes = 0;
}

// Bump allocator over the forest's grow-only workspace.
struct Carve {
    size_t off = 0;
    template <class T>
    size_t take(size_t count) {
        off = (off + 255) & ~size_t(255);
        size_t at = off;
        off += count * sizeof(T);
        return at;
    }
};

struct Workspace {
    float* Qp; uint16_t* Q16; uint8_t* Q8; float* qscale; float* qnorm; int32_t* cpq;
    gf::SelState* state; uint32_t* hist; uint32_t* coff; uint64_t* ckey; uint32_t* ccode;
    uint32_t* leafbits; uint32_t* flags; uint32_t* qlist; int32_t* ids; float* dists;
    uint32_t* openT; uint32_t* visT; uint32_t* gthr; float* part_s; int* part_i;   // tile paths only
    uint64_t* masks8; uint32_t* offs8; uint32_t* total8; float* out_s8; int* out_i8;   // FP8 tile path
    float* qt;   // [m][nb][t] reflected query coordinates (isometry variant only)
    uint32_t* gbits;   // [nb][ceil(n/32)] candidate bitmap of a small sliced row scan
};

// Split of the points for the tile path: enough (query block, split)
// workgroups to fill the chip several times over, each split small enough
// for 32-bit byte offsets into its rows; and the query chunking of the
// point-major candidate sets.
struct TilePlan {
    int nsplit = 0;
    int64_t split_pts = 0;
    int cw = 0, nchunk = 0;
    // FP8 tile path: tiles of 128 points, splits of split_tiles tiles, and
    // the candidate slots per query
    int ntiles8 = 0, nsplit8 = 0, split_tiles8 = 0;
    int64_t cap8 = 0;
};

// The tile kernels run one workgroup per CU at a time, so the batch takes
// ceil(qblocks * ns / CUs) rounds of 1/ns of the work each, plus a fixed
// cost per round (start-up, list fill and write-out: about 0.4% of one
// workgroup's pass over all the points, measured at 10^6 x 960).  Among the
// split counts within 2% of the least such time the smallest wins: every
// split fills and merges its own per-query list, and with 2 or 3 splits the
// splits also share a rank bound.
int64_t pick_splits(int64_t qblocks, int64_t max_splits, int64_t cus) {
    auto cost = [&](int64_t s) {
        const double rounds = double((qblocks * s + cus - 1) / cus);
        return rounds * (1.0 / double(s) + 0.004);
    };
    double best = 1e300;
    for (int64_t s = 1; s <= max_splits; ++s) best = std::min(best, cost(s));
    for (int64_t s = 1; s <= max_splits; ++s)
        if (cost(s) <= 1.02 * best) return s;
    return 1;
}

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

TilePlan tile_plan(const gf_forest* F, int nb, int form = gf::kFormBF16, int64_t checks_max = 0) {
    TilePlan p;
    if (form == gf::kFormFP8) {
        // one workgroup per CU at a time, each a block of kTile8Queries
        // queries and a split of the tiles: the split count with the least
        // time in whole rounds
        const int64_t qblocks = (nb + gf::kTile8Queries - 1) / gf::kTile8Queries;
        const int64_t tiles = gf::tile8_ntiles(F->host.n);
        const int64_t ns = pick_splits(qblocks, std::min<int64_t>((tiles + 1) / 2, 512), device_cus());
        p.ntiles8 = int(tiles);
        // the score kernel takes the 128-point tiles in pairs: splits of an
        // even number of tiles (the last may be odd)
        p.split_tiles8 = int(((tiles + ns - 1) / ns + 1) / 2 * 2);
        p.nsplit8 = int((tiles + p.split_tiles8 - 1) / p.split_tiles8);
        p.cap8 = std::max<int64_t>(1, std::min<int64_t>(F->host.n, std::max<int64_t>(1, checks_max) *
                                                                         int64_t(std::max(1, F->maxleaf))));
    }
    const int64_t qblocks = (nb + 127) / 128;
    const int64_t tiles = (F->host.n + 63) / 64;
    const int64_t max_tiles = ((int64_t{1} << 31) - 1) / (int64_t(F->ld16) * 2 * 64);
    int64_t ns = pick_splits(qblocks, std::min<int64_t>(tiles, 256), device_cus());
    // GF_TILE_SPLITS=s forces the split count (tests: the result does not depend on it)
    const char* senv = std::getenv("GF_TILE_SPLITS");
    if (senv && std::atoi(senv) > 0) ns = std::min<int64_t>(tiles, std::atoi(senv));
    if ((tiles + ns - 1) / ns > max_tiles) ns = (tiles + max_tiles - 1) / max_tiles;
    p.split_pts = ((tiles + ns - 1) / ns) * 64;
    p.nsplit = int((F->host.n + p.split_pts - 1) / p.split_pts);
    const int64_t nqw = (nb + 31) / 32;
    p.cw = 4;
    while (p.cw < 32 && p.cw < nqw) p.cw <<= 1;
    p.nchunk = int((nqw + p.cw - 1) / p.cw);
    return p;
}

// Offsets of a batch's workspace (nb queries, bytes from a 256-aligned base).
struct WsLayout {
    size_t oQp = 0, oQ16 = 0, oQ8 = 0, oqs = 0, oqn = 0, ocpq = 0, ost = 0, ohist = 0, onc = 0;
    size_t ock = 0, occ = 0, olb = 0, ofl = 0, oql = 0, oids = 0, odst = 0, oqt = 0;
    size_t oopen = 0, ovis = 0, othr = 0, ops = 0, opi = 0;
    size_t omask = 0, ooff = 0, otot = 0, oos = 0, ooi = 0;
    size_t ogb = 0;
    size_t need = 0;   // bytes
};

WsLayout ws_layout(const gf_forest* F, int nb, int k, int form, bool tile, int64_t checks_max = 0,
                   int scan_nslice = 1) {
    const int64_t W = std::max<int64_t>(1, (int64_t{1} << F->host.H) / 32);
    Carve c;
    WsLayout L;
    L.oQp = c.take<float>(size_t(nb) * F->ld32);
    L.oQ16 = form == gf::kFormBF16 ? c.take<uint16_t>(size_t(nb) * F->ld16) : 0;
    L.oQ8 = form == gf::kFormFP8 ? c.take<uint8_t>(size_t(nb) * F->ld8) : 0;
    L.oqs = c.take<float>(nb);
    L.oqn = c.take<float>(nb);
    L.ocpq = c.take<int32_t>(nb);
    L.ost = c.take<gf::SelState>(nb);
    const int nslice = F->host.m * gf::select_slices_per_tree(F->host.H, F->host.m, nb);
    L.ohist = c.take<uint32_t>(size_t(nb) * nslice * 128);
    L.onc = c.take<uint32_t>(size_t(nb) * nslice);
    const int64_t ccap = gf::collect_capacity(F->host.H);
    L.ock = c.take<uint64_t>(size_t(nb) * ccap);
    L.occ = c.take<uint32_t>(size_t(nb) * ccap);
    L.olb = c.take<uint32_t>(size_t(nb) * F->host.m * W);
    L.ofl = c.take<uint32_t>(8);
    L.oql = c.take<uint32_t>(nb);
    L.oids = c.take<int32_t>(size_t(nb) * k);
    L.odst = c.take<float>(size_t(nb) * k);
    L.oqt = F->U ? c.take<float>(size_t(nb) * F->host.m * F->host.t) : 0;
    if (tile) {
        const TilePlan tp = tile_plan(F, nb, form, checks_max);
        L.oopen = c.take<uint32_t>(size_t(tp.nchunk) * F->host.m * (size_t{1} << F->host.H) * tp.cw);
        L.ovis = c.take<uint32_t>(size_t(tp.nchunk) * F->host.n * tp.cw);
        // per query the shared bound and the splits' rank scores
        L.othr = c.take<uint32_t>(size_t(nb) * gf::kBoundWords);
        const size_t lists = form == gf::kFormFP8 ? 1 : size_t(tp.nsplit);
        L.ops = c.take<float>(size_t(nb) * lists * gf::kTileList);
        L.opi = c.take<int>(size_t(nb) * lists * gf::kTileList);
        if (form == gf::kFormFP8) {
            L.omask = c.take<uint64_t>(size_t(nb) * tp.ntiles8 * 2);
            L.ooff = c.take<uint32_t>(size_t(nb) * tp.ntiles8);
            L.otot = c.take<uint32_t>(nb);
            L.oos = c.take<float>(size_t(nb) * tp.cap8);
            L.ooi = c.take<int>(size_t(nb) * tp.cap8);
        }
    } else if (scan_nslice > 1) {
        // the sliced row scan's per-slice lists, and for a small batch the
        // candidate bitmap every slice reads its words of
        L.ops = c.take<float>(size_t(nb) * scan_nslice * gf::kTileList);
        L.opi = c.take<int>(size_t(nb) * scan_nslice * gf::kTileList);
        if (nb <= gf::kMarkMaxQueries) L.ogb = c.take<uint32_t>(size_t(nb) * ((F->host.n + 31) / 32));
    }
    L.need = c.off + 256;
    return L;
}

void ws_bind(const gf_forest* F, const WsLayout& L, char* b, int form, bool tile, Workspace& w) {
    w.Qp = reinterpret_cast<float*>(b + L.oQp);
    w.Q16 = form == gf::kFormBF16 ? reinterpret_cast<uint16_t*>(b + L.oQ16) : nullptr;
    w.Q8 = form == gf::kFormFP8 ? reinterpret_cast<uint8_t*>(b + L.oQ8) : nullptr;
    w.qscale = reinterpret_cast<float*>(b + L.oqs);
    w.qnorm = reinterpret_cast<float*>(b + L.oqn);
    w.cpq = reinterpret_cast<int32_t*>(b + L.ocpq);
    w.state = reinterpret_cast<gf::SelState*>(b + L.ost);
    w.hist = reinterpret_cast<uint32_t*>(b + L.ohist);
    w.coff = reinterpret_cast<uint32_t*>(b + L.onc);
    w.ckey = reinterpret_cast<uint64_t*>(b + L.ock);
    w.ccode = reinterpret_cast<uint32_t*>(b + L.occ);
    w.leafbits = reinterpret_cast<uint32_t*>(b + L.olb);
    w.flags = reinterpret_cast<uint32_t*>(b + L.ofl);
    w.qlist = reinterpret_cast<uint32_t*>(b + L.oql);
    w.ids = reinterpret_cast<int32_t*>(b + L.oids);
    w.dists = reinterpret_cast<float*>(b + L.odst);
    w.qt = F->U ? reinterpret_cast<float*>(b + L.oqt) : nullptr;
    w.openT = tile ? reinterpret_cast<uint32_t*>(b + L.oopen) : nullptr;
    w.visT = tile ? reinterpret_cast<uint32_t*>(b + L.ovis) : nullptr;
    w.gthr = tile ? reinterpret_cast<uint32_t*>(b + L.othr) : nullptr;
    w.part_s = (tile || L.ops) ? reinterpret_cast<float*>(b + L.ops) : nullptr;
    w.part_i = (tile || L.opi) ? reinterpret_cast<int*>(b + L.opi) : nullptr;
    const bool t8 = tile && form == gf::kFormFP8;
    w.masks8 = t8 ? reinterpret_cast<uint64_t*>(b + L.omask) : nullptr;
    w.offs8 = t8 ? reinterpret_cast<uint32_t*>(b + L.ooff) : nullptr;
    w.total8 = t8 ? reinterpret_cast<uint32_t*>(b + L.otot) : nullptr;
    w.out_s8 = t8 ? reinterpret_cast<float*>(b + L.oos) : nullptr;
    w.out_i8 = t8 ? reinterpret_cast<int*>(b + L.ooi) : nullptr;
    w.gbits = L.ogb ? reinterpret_cast<uint32_t*>(b + L.ogb) : nullptr;
}

gf_status get_workspace(gf_forest* F, int nb, int k, int form, bool tile, Workspace& w,
                        int64_t checks_max = 0, int nslice = 1) {
    const WsLayout L = ws_layout(F, nb, k, form, tile, checks_max, nslice);
    if (L.need > F->ws_bytes) {
        gf::dev_free(F->ws);
        F->ws = nullptr;
        F->ws_bytes = 0;
        if (gf::dev_malloc(&F->ws, L.need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GF_ENOMEM, "device workspace allocation of " + std::to_string(L.need) +
                                       " bytes failed");
        }
        F->ws_bytes = L.need;
    }
    ws_bind(F, L, static_cast<char*>(F->ws), form, tile, w);
    return GF_OK;
}

constexpr int kMaxBatch = 16384;

// Queries per batch: kMaxBatch, fewer for trees deeper than 16 levels, whose
// collect buffers grow with the largest group of leaves (so the batch's
// collect area stays at what 16,384 queries take at depth <= 16, 6 GiB).
int max_batch(const gf_forest* F) {
    const int64_t per = gf::collect_capacity(F->host.H);
    return int(std::max<int64_t>(1, std::min<int64_t>(kMaxBatch, int64_t{kMaxBatch} * gf::kCollectCap / per)));
}

struct QueryJob {
    const float* Q;            // caller's rows (host or device)
    bool q_dev;
    const int32_t* cpq;        // caller's budgets (host or device) or null
    bool cpq_dev;
    int64_t nq;
    int32_t k, checks;
    double checks_mean;        // mean budget over the queries (the path rule's estimate)
    int64_t checks_max;        // largest budget (bounds a query's candidates)
    double eps;
    int form, kk;
    // outputs (host or device), any may be null
    int32_t* ids; float* dists; bool out_dev;
    uint32_t* leaf_bits; uint32_t* cand_bits; int64_t* ncand; bool trace_dev;
    int path = -1;             // -1 by rule, 0 rows, 1 tile (when eligible)
    bool trace_tile = false;   // trace: candidates as the tile path builds them
    int slice_mult = 1;        // row path: slices per query times this (autotuner)
};

// Whether a batch takes the tile path (BF16 scores of whole query blocks on
// MFMA, masked by each query's candidate bitmap) instead of per-query row
// gathers.  The tile path computes nb * n scores at MFMA rate; the gather
// path reads every candidate's row from HBM.  It pays off once each query's
// candidates are more than ~1/256 of the points and the batch is large
// enough to amortise scoring every point (16 queries for BF16, 512 for FP8,
// measured).  GF_SCAN_PATH=rows|tile forces a path.
//
// The FP8 form has a tile path of its own (tile8.hip) for wide rows: dense
// FP8 scores of 128-query blocks against 128-point tiles, the candidates'
// scores compacted per query.  Its product reads every row once per query
// block at 5 PFLOP/s where the gathers read each candidate's row at HBM
// rate; it pays off from about 1/192 of the points per query.
bool tile_eligible(const gf_forest* F, const QueryJob& J) {
    if (J.leaf_bits || J.cand_bits || J.ncand || !F->leafof) return false;
    if (J.kk > gf::kTileList) return false;   // lists of kTileList entries per query
    if (J.form == gf::kFormBF16) return F->ld16 <= 1024;   // A operands of one wave pair in registers
    return J.form == gf::kFormFP8;
}

bool use_tile_path(const gf_forest* F, const QueryJob& J, int nb) {
    if (J.path >= 0) return J.path == 1 && tile_eligible(F, J);
    if (!tile_eligible(F, J)) return false;
    const char* env = std::getenv("GF_SCAN_PATH");
    if (env && std::strcmp(env, "rows") == 0) return false;
    if (env && std::strcmp(env, "tile") == 0) return true;
    // batch sizes from which the tile path measured faster, with the splits
    // of pick_splits (1M x 960 BF16: 1.19 vs 1.42 ms at 2 queries, 0.86 vs
    // 0.79 at 1; 200k x 10,000 FP8: 1.72 vs 1.78 ms at 32 queries, 1.52 vs
    // 1.02 at 8)
    if (nb < (J.form == gf::kFormFP8 ? 32 : 2)) return false;
    const double leaf_pts = double(F->host.n) * F->host.m / double(F->host.real_leaves);
    const double cand_est = J.checks_mean * leaf_pts * 0.5;
    return cand_est * (J.form == gf::kFormFP8 ? 192.0 : 256.0) >= double(F->host.n);
}

// Slices of the row scan.  One workgroup per query leaves most of the
// device idle for small batches (a single query would stream its candidate
// rows through one CU), so below two workgroups per CU each query's id range
// is cut into slices, one workgroup each, whose best lists the tile path's
// merge combines.  Traces keep one slice (they read the whole bitmap), and so
// do re-rank depths above the merge's list length.  GF_SCAN_SLICES=<count>
// forces a count (for tests).
struct ScanSlices {
    int nslice = 1;
    int64_t words = 0;   // bitmap words per slice (a multiple of 16)
};

ScanSlices scan_slices(const gf_forest* F, const QueryJob& J, int nb) {
    ScanSlices r;
    const int64_t nbmw = (F->host.n + 31) / 32;
    // id ranges above one workgroup's bitmap are always sliced (traces
    // included: each slice writes its words of the candidate rows)
    const int64_t wmax = gf::scan_max_slice_words(J.form, F->ld8);
    if (wmax > 0 && nbmw > wmax) {
        const int64_t ns = (nbmw + wmax - 1) / wmax;
        int64_t words = (nbmw + ns - 1) / ns;
        words = (words + 15) / 16 * 16;
        r.nslice = int((nbmw + words - 1) / words);
        r.words = words;
        return r;
    }
    if (J.cand_bits || J.ncand || J.kk > gf::kTileList) return r;
    int64_t want = 1;
    const char* env = std::getenv("GF_SCAN_SLICES");
    if (env && std::atoi(env) > 0) {
        want = std::atoi(env);
    } else {
        const int64_t cus = device_cus();
        if (int64_t(nb) < 2 * cus) want = std::min<int64_t>(256, (2 * cus + nb - 1) / nb);
        want = std::min<int64_t>(256, want * std::max(1, J.slice_mult));
    }
    if (want <= 1) return r;
    int64_t words = (nbmw + want - 1) / want;
    words = std::max<int64_t>(64, (words + 15) / 16 * 16);   // at least 2,048 ids per slice
    const int64_t ns = (nbmw + words - 1) / words;
    if (ns <= 1) return r;
    r.nslice = int(ns);
    r.words = words;
    return r;
}

gf::SelectArgs make_select_args(const gf_forest* F, int nb, const Workspace& w, int64_t W) {
    const gf::HostForest& h = F->host;
    gf::SelectArgs sa{};
    sa.Q = w.Qp; sa.ldq = F->ld32; sa.nq = nb; sa.m = h.m; sa.H = h.H; sa.t = h.t;
    sa.n_internal = (int64_t{1} << h.H) - 1; sa.W = int(W); sa.nodes = F->nodes; sa.D = F->D;
    sa.drange = F->drange;
    sa.leaves = h.real_leaves;
    sa.nslice = h.m * gf::select_slices_per_tree(h.H, h.m, nb);
    sa.state = w.state; sa.hist = w.hist; sa.coff = w.coff; sa.ckey = w.ckey;
    sa.ccap = gf::collect_capacity(h.H);
    sa.ccode = w.ccode; sa.leafbits = w.leafbits; sa.qlist = w.qlist; sa.nlist = 0;
    sa.qt = F->U ? w.qt : nullptr;
    return sa;
}

// a2: the opened leaves.  With `more` a host flag ends the radix passes
// early; without it every pass is launched.
gf_status launch_selection(const gf_forest* F, const QueryJob& J, int nb, const Workspace& w,
                           int64_t W, const int32_t* cpq, bool early_exit, hipStream_t st) {
    const gf::SelectArgs sa = make_select_args(F, nb, w, W);
    if (F->U) {
        // isometry variant: each tree's reflected query coordinates on D,
        // the trees of a query on neighbouring lanes
        int mp = 1;
        while (mp < F->host.m) mp <<= 1;                 // m <= 255, so mp <= 256
        const int qpb = 256 / mp;
        hipLaunchKernelGGL(gf::k_reflect_queries, dim3((nb + qpb - 1) / qpb), dim3(256), 0, st,
                           static_cast<const float*>(w.Qp), int64_t(F->ld32), nb, F->host.d,
                           F->host.m, mp, F->host.t, static_cast<const int32_t*>(F->D),
                           static_cast<const double*>(F->U), w.qt);
        GF_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(gf::k_select_init, dim3((nb + 255) / 256), dim3(256), 0, st, sa,
                       J.checks, cpq, J.eps, w.flags + 1);
    GF_HIP(hipGetLastError());
    // sample walk, window walk, then radix passes while some query needs one.
    // flags[1]: any query left for a radix pass, flags[2]: how many.  With
    // the host readback, a pass for a few queries splits each tree finer.
    uint32_t more[2] = {1u, uint32_t(nb)};
    for (int step = 0; step < gf::kMaxPasses + 2 && more[0]; ++step) {
        const int phase = step == 0 ? gf::kPhSample : (step == 1 ? gf::kPhWindow : gf::kPhRadix);
        // the flags collect the window walk's queries and those the sample
        // walk sent straight to radix passes
        if (early_exit && phase != gf::kPhWindow) GF_HIP(hipMemsetAsync(w.flags + 1, 0, 8, st));
        // few queries left: a compact walk over the listed queries, each
        // tree split finer
        const bool sparse = early_exit && phase == gf::kPhRadix && int64_t(more[1]) * 16 <= nb;
        gf::SelectArgs sw = sa;
        if (sparse) sw.nlist = int(more[1]);
        GF_HIP(gf::launch_select_walk(sw, phase, false, st, sparse ? 16 : 1));
        hipLaunchKernelGGL(gf::k_select_pick, dim3(nb), dim3(gf::pick_threads(sa.nslice)), 0, st, sa, phase,
                           w.flags + 1);
        GF_HIP(hipGetLastError());
        if (early_exit && phase != gf::kPhSample) {
            GF_HIP(hipMemcpyAsync(more, w.flags + 1, 8, hipMemcpyDeviceToHost, st));
            GF_HIP(hipStreamSynchronize(st));
        }
    }
    GF_HIP(gf::launch_select_walk(sa, 0, true, st));
    hipLaunchKernelGGL(gf::k_select_finish, dim3(nb), dim3(gf::finish_threads(nb)), 0, st, sa);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

gf::ScanArgs make_scan_args(const gf_forest* F, const QueryJob& J, int64_t q0, int nb,
                            const Workspace& w, int64_t W) {
    const gf::HostForest& h = F->host;
    gf::ScanArgs ca{};
    ca.nq = nb; ca.k = J.k; ca.kk = J.kk; ca.n = h.n; ca.d = h.d; ca.m = h.m; ca.W = int(W); ca.H = h.H;
    ca.leafbits = w.leafbits; ca.permp = F->permp; ca.pp = F->pp;
    ca.Q = w.Qp; ca.ldq = F->ld32; ca.X32 = F->X32; ca.ld32 = F->ld32;
    ca.X16 = F->X16; ca.ld16 = F->ld16; ca.norm16 = F->norm16;
    ca.X8 = F->X8; ca.ld8 = F->ld8; ca.scale8 = F->scale8; ca.norm8 = F->norm8;
    ca.Q16 = w.Q16; ca.Q8 = w.Q8; ca.qscale8 = w.qscale; ca.qnorm = w.qnorm;
    ca.ids = J.out_dev && J.ids ? J.ids + q0 * J.k : w.ids;
    ca.dists = J.out_dev && J.dists ? J.dists + q0 * J.k : w.dists;
    return ca;
}

gf::ExpandArgs make_expand_args(const gf_forest* F, int nb, const Workspace& w, int64_t W) {
    const gf::HostForest& h = F->host;
    const TilePlan tp = tile_plan(F, nb);
    gf::ExpandArgs ea{};
    ea.nq = nb; ea.m = h.m; ea.W = int(W); ea.H = h.H; ea.n = h.n;
    ea.cw = tp.cw; ea.nchunk = tp.nchunk;
    ea.leafbits = w.leafbits; ea.leafof = F->leafof; ea.openT = w.openT; ea.visT = w.visT;
    ea.order = F->perm;   // tree 0's row of perm: every point once, leaf by leaf
    ea.gthr = w.gthr;
    return ea;
}

// a3-a6 on the tile path; ev (may be null) gets the expansion and tile marks.
gf_status launch_tile(gf_forest* F, const QueryJob& J, int nb, const Workspace& w, int64_t W,
                      const gf::ScanArgs& ca, hipStream_t st, hipEvent_t* ev) {
    const gf::HostForest& h = F->host;
    const TilePlan tp = tile_plan(F, nb, J.form, J.checks_max);
    const gf::ExpandArgs ea = make_expand_args(F, nb, w, W);
    if (J.form == gf::kFormFP8) {
        GF_HIP(gf::launch_tile_expand(ea, st));
        gf::Tile8Args t8{};
        t8.nq = nb; t8.n = h.n; t8.ld8 = F->ld8; t8.cw = tp.cw; t8.ntiles = tp.ntiles8;
        t8.nsplit = tp.nsplit8; t8.split_tiles = tp.split_tiles8; t8.cap = tp.cap8; t8.kk = J.kk;
        t8.Q8 = w.Q8; t8.X8 = F->X8; t8.qscale = w.qscale; t8.norm8 = F->norm8; t8.scale8 = F->scale8;
        t8.visT = w.visT; t8.masks = w.masks8; t8.offs = w.offs8; t8.total = w.total8;
        t8.out_s = w.out_s8; t8.out_i = w.out_i8; t8.part_s = w.part_s; t8.part_i = w.part_i;
        // phase marks: expansion with the masks and offsets, then the score kernel
        GF_HIP(gf::launch_tile8(t8, (nb + 31) / 32, st, ev));
        gf::MergeArgs ma{};
        ma.nq = nb; ma.k = J.k; ma.kk = J.kk; ma.d = h.d; ma.nsplit = 1; ma.rerank = true;
        ma.part_s = w.part_s; ma.part_i = w.part_i; ma.Q = w.Qp; ma.ldq = F->ld32;
        ma.X32 = F->X32; ma.ld32 = F->ld32; ma.ids = ca.ids; ma.dists = ca.dists;
        GF_HIP(gf::launch_merge(ma, st));
        return GF_OK;
    }
    gf::TileArgs ta{};
    ta.nq = nb; ta.n = h.n; ta.ld16 = F->ld16; ta.cw = tp.cw; ta.Q16 = w.Q16; ta.X16 = F->X16;
    ta.norm16 = F->norm16; ta.visT = w.visT; ta.gthr = w.gthr; ta.cap = J.kk; ta.nsplit = tp.nsplit;
    ta.split_pts = tp.split_pts; ta.part_s = w.part_s; ta.part_i = w.part_i;
    // rank scores: each of 2 or 3 splits publishes its ceil(kk / nsplit)-th best
    ta.nrb = (tp.nsplit >= 2 && tp.nsplit < gf::kBoundWords) ? tp.nsplit : 0;
    ta.rpos = ta.nrb ? J.kk - (J.kk + tp.nsplit - 1) / tp.nsplit : 0;
    gf::ExpandArgs eb = ea;
    eb.nrb = ta.nrb;
    gf::MergeArgs ma{};
    ma.nq = nb; ma.k = J.k; ma.kk = J.kk; ma.d = h.d; ma.nsplit = tp.nsplit; ma.rerank = true;
    ma.part_s = w.part_s; ma.part_i = w.part_i; ma.Q = w.Qp; ma.ldq = F->ld32;
    ma.X32 = F->X32; ma.ld32 = F->ld32; ma.ids = ca.ids; ma.dists = ca.dists;
    GF_HIP(gf::launch_tile_path(eb, ta, ma, st, ev));
    return GF_OK;
}

// a3-a6 on the row path: the scan, and for a sliced scan the merge of the
// slices' lists (re-ranked in FP32 for the reduced-precision forms, as the
// unsliced scan does).
gf_status launch_rows(const gf_forest* F, const QueryJob& J, int nb, const Workspace& w,
                      gf::ScanArgs ca, const ScanSlices& sl, hipStream_t st) {
    int64_t* ncand = nullptr;
    if (sl.nslice > 1) {
        ca.nslice = sl.nslice;
        ca.slice_words = sl.words;
        ca.part_s = w.part_s;
        ca.part_i = w.part_i;
        // candidate counts of a sliced trace: summed from the bitmap rows
        ncand = ca.ncand;
        ca.ncand = nullptr;
        if (ncand && !ca.cand_bits) return fail(GF_EINTERNAL, "sliced trace without a bitmap");
        if (w.gbits) {
            GF_HIP(gf::launch_mark_candidates(ca, w.gbits, st));
            ca.gbits = w.gbits;
        }
    }
    GF_HIP(gf::launch_scan(ca, J.form, st));
    if (ncand) GF_HIP(gf::launch_count_bits(ca.cand_bits, nb, (F->host.n + 31) / 32, ncand, st));
    if (sl.nslice > 1) {
        gf::MergeArgs ma{};
        ma.nq = nb; ma.k = J.k; ma.kk = J.kk; ma.d = F->host.d; ma.nsplit = sl.nslice;
        ma.rerank = J.form != gf::kFormFP32;
        ma.part_s = w.part_s; ma.part_i = w.part_i; ma.Q = w.Qp; ma.ldq = F->ld32;
        ma.X32 = F->X32; ma.ld32 = F->ld32; ma.ids = ca.ids; ma.dists = ca.dists;
        GF_HIP(gf::launch_merge(ma, st));
    }
    return GF_OK;
}

// The reduced query copies (BF16 / FP8 rows and norms) from the padded rows.
gf_status launch_query_forms(const gf_forest* F, const QueryJob& J, int nb, const Workspace& w,
                             hipStream_t st) {
    const gf::HostForest& h = F->host;
    if (J.form == gf::kFormBF16) {
        hipLaunchKernelGGL(gf::k_to_bf16, dim3((nb + 3) / 4), dim3(256), 0, st, w.Qp, int64_t(nb),
                           h.d, int64_t(F->ld32), w.Q16, int64_t(F->ld16), w.qnorm);
        GF_HIP(hipGetLastError());
    } else if (J.form == gf::kFormFP8) {
        hipLaunchKernelGGL(gf::k_to_fp8, dim3((nb + 3) / 4), dim3(256), 0, st, w.Qp, int64_t(nb),
                           h.d, int64_t(F->ld32), w.Q8, int64_t(F->ld8), w.qscale, w.qnorm);
        GF_HIP(hipGetLastError());
    }
    return GF_OK;
}

// Graph-mode batch: device Q, budgets and outputs, queries already checked
// finite; nothing waits on the host and no memset is issued, so every
// launch can be captured into a graph.  The query rows are padded by a
// kernel and all radix passes are launched (once each query's bin is
// settled a pass finds no active query and its workgroups return at once).
gf_status run_batch_graph(gf_forest* F, const QueryJob& J, int64_t q0, int nb, hipStream_t st,
                          const Workspace& w, bool tile, int64_t W, const ScanSlices& sl) {
    const gf::HostForest& h = F->host;
    {
        const int64_t tot = int64_t(nb) * F->ld32;
        hipLaunchKernelGGL(gf::k_pad_rows, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st,
                           J.Q + q0 * h.d, int64_t(nb), h.d, w.Qp, int64_t(F->ld32));
        GF_HIP(hipGetLastError());
    }
    gf_status s = launch_query_forms(F, J, nb, w, st);
    if (s != GF_OK) return s;
    const int32_t* cpq = nullptr;
    if (J.cpq) {
        GF_HIP(hipMemcpyAsync(w.cpq, J.cpq + q0, size_t(nb) * 4, hipMemcpyDeviceToDevice, st));
        cpq = w.cpq;
    }
    s = launch_selection(F, J, nb, w, W, cpq, false, st);
    if (s != GF_OK) return s;
    const gf::ScanArgs ca = make_scan_args(F, J, q0, nb, w, W);
    if (tile) return launch_tile(F, J, nb, w, W, ca, st, nullptr);
    return launch_rows(F, J, nb, w, ca, sl, st);
}

// Runs the whole query path for queries [q0, q0 + nb); graph mode as above.
// With `scratch` (device memory the caller sized with ws_layout for the row
// path) the batch allocates nothing: no workspace growth, no staging, no
// events; Q, budgets and outputs are then device buffers.
gf_status run_batch(gf_forest* F, const QueryJob& J, int64_t q0, int nb, hipStream_t st,
                    bool graph = false, char* scratch = nullptr) {
    const gf::HostForest& h = F->host;
    Workspace w;
    const bool tile = !scratch && (J.trace_tile || use_tile_path(F, J, nb));
    const ScanSlices sl = tile ? ScanSlices{} : scan_slices(F, J, nb);
    if (scratch) {
        ws_bind(F, ws_layout(F, nb, J.k, J.form, false, 0, sl.nslice), scratch, J.form, false, w);
    } else {
        gf_status s0 = get_workspace(F, nb, J.k, J.form, tile, w, J.checks_max, sl.nslice);
        if (s0 != GF_OK) return s0;
    }
    gf_status s = GF_OK;
    const int64_t W = std::max<int64_t>(1, (int64_t{1} << h.H) / 32);
    if (graph) return run_batch_graph(F, J, q0, nb, st, w, tile, W, sl);

    // phase marks (none in the allocation-free mode)
    hipEvent_t ev[6] = {};
    const bool timed = scratch == nullptr;
    struct EvGuard { hipEvent_t* e; ~EvGuard() { for (int i = 0; i < 6; ++i) if (e[i]) (void)hipEventDestroy(e[i]); } } evg{ev};
    if (timed)
        for (auto& e : ev) GF_HIP(hipEventCreate(&e));
    auto mark_phase = [&](int i) -> hipError_t { return timed ? hipEventRecord(ev[i], st) : hipSuccess; };
    GF_HIP(mark_phase(0));
    // a1: query prep -- padded FP32 rows, finiteness, reduced copies
    if (J.q_dev) {
        GF_HIP(hipMemsetAsync(w.Qp, 0, size_t(nb) * F->ld32 * 4, st));
        GF_HIP(hipMemcpy2DAsync(w.Qp, size_t(F->ld32) * 4, J.Q + q0 * h.d, size_t(h.d) * 4,
                                size_t(h.d) * 4, nb, hipMemcpyDeviceToDevice, st));
    } else {
        // pageable host rows would be copied slowly by the runtime
        GF_HIP(stage_host_rows(F, w.Qp, J.Q + q0 * h.d, nb, h.d, F->ld32, st));
    }
    GF_HIP(hipMemsetAsync(w.flags, 0, 8 * 4, st));
    {
        const int64_t tot = int64_t(nb) * h.d;
        hipLaunchKernelGGL(gf::k_check_finite, dim3((tot + 255) / 256), dim3(256), 0, st,
                           w.Qp, int64_t(nb), h.d, int64_t(F->ld32), w.flags);
        GF_HIP(hipGetLastError());
    }
    s = launch_query_forms(F, J, nb, w, st);
    if (s != GF_OK) return s;
    const int32_t* cpq = nullptr;
    if (J.cpq) {
        GF_HIP(hipMemcpyAsync(w.cpq, J.cpq + q0, size_t(nb) * 4,
                              J.cpq_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
        cpq = w.cpq;
    }
    uint32_t bad = 0;
    GF_HIP(hipMemcpyAsync(&bad, w.flags, 4, hipMemcpyDeviceToHost, st));
    GF_HIP(hipStreamSynchronize(st));
    if (bad) return fail(GF_EINVAL, "Q contains a non-finite value");

    // a2: leaf selection
    GF_HIP(mark_phase(1));
    s = launch_selection(F, J, nb, w, W, cpq, true, st);
    if (s != GF_OK) return s;

    // a3-a6: candidates, distances, best k, re-rank, ties
    const int64_t nbmw = (h.n + 31) / 32;
    gf::ScanArgs ca = make_scan_args(F, J, q0, nb, w, W);
    ca.cand_bits = (J.cand_bits && J.trace_dev) ? J.cand_bits + q0 * nbmw : nullptr;
    ca.ncand = (J.ncand && J.trace_dev) ? J.ncand + q0 : nullptr;
    std::unique_ptr<uint32_t, DevFree> tmp_bits;
    std::unique_ptr<int64_t, DevFree> tmp_nc;
    if ((J.cand_bits && !J.trace_dev) || ((J.trace_tile || sl.nslice > 1) && !ca.cand_bits && J.ncand)) {
        uint32_t* p = nullptr;
        GF_HIP(gf::dev_malloc((void**)&p, size_t(nb) * nbmw * 4));
        tmp_bits.reset(p);
        ca.cand_bits = p;
    }
    if (J.ncand && !J.trace_dev) {
        int64_t* p = nullptr;
        GF_HIP(gf::dev_malloc((void**)&p, size_t(nb) * 8));
        tmp_nc.reset(p);
        ca.ncand = p;
    }
    GF_HIP(mark_phase(2));
    if (J.trace_tile) {
        // the tile path's own candidate words, turned back into query rows
        if (ca.cand_bits)
            GF_HIP(gf::launch_tile_trace(make_expand_args(F, nb, w, W), ca.cand_bits, ca.ncand, st));
        else
            GF_HIP(gf::launch_tile_expand(make_expand_args(F, nb, w, W), st));
        GF_HIP(mark_phase(3));
        GF_HIP(mark_phase(4));
    } else if (tile) {
        s = launch_tile(F, J, nb, w, W, ca, st, timed ? ev + 3 : nullptr);
        if (s != GF_OK) return s;
    } else {
        s = launch_rows(F, J, nb, w, ca, sl, st);
        if (s != GF_OK) return s;
        GF_HIP(mark_phase(3));
        GF_HIP(mark_phase(4));
    }
    GF_HIP(mark_phase(5));

    // outputs
    if (J.ids && !J.out_dev)
        GF_HIP(hipMemcpyAsync(J.ids + q0 * J.k, w.ids, size_t(nb) * J.k * 4, hipMemcpyDeviceToHost, st));
    if (J.dists && !J.out_dev)
        GF_HIP(hipMemcpyAsync(J.dists + q0 * J.k, w.dists, size_t(nb) * J.k * 4, hipMemcpyDeviceToHost, st));
    if (J.cand_bits && !J.trace_dev)
        GF_HIP(hipMemcpyAsync(J.cand_bits + q0 * nbmw, ca.cand_bits, size_t(nb) * nbmw * 4,
                              hipMemcpyDeviceToHost, st));
    if (J.ncand && !J.trace_dev)
        GF_HIP(hipMemcpyAsync(J.ncand + q0, ca.ncand, size_t(nb) * 8, hipMemcpyDeviceToHost, st));
    if (J.leaf_bits) {
        const int64_t words = int64_t(h.m) * W;
        uint32_t* dst = J.leaf_bits + q0 * words;
        std::unique_ptr<uint32_t, DevFree> tmp;
        if (!J.trace_dev) {
            uint32_t* p = nullptr;
            GF_HIP(gf::dev_malloc((void**)&p, size_t(nb) * words * 4));
            tmp.reset(p);
            dst = p;
        }
        const int64_t tot = words * nb;
        hipLaunchKernelGGL(gf::k_leafbits_to_query_major, dim3((tot + 255) / 256), dim3(256), 0, st,
                           w.leafbits, nb, words, dst);
        GF_HIP(hipGetLastError());
        if (!J.trace_dev) {
            GF_HIP(hipMemcpyAsync(J.leaf_bits + q0 * words, dst, size_t(tot) * 4,
                                  hipMemcpyDeviceToHost, st));
            GF_HIP(hipStreamSynchronize(st));
        }
    }
    GF_HIP(hipStreamSynchronize(st));
    for (int i = 0; timed && i < kPhases; ++i) {
        float ms = 0.0f;
        GF_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
        g_phase_ms[i] += ms;
    }
    g_path = tile ? 1 : 0;
    g_batches += 1;
    return GF_OK;
}

gf_status run_query(gf_forest* F, QueryJob& J, hipStream_t st) {
    GF_HIP(hipSetDevice(F->device));
    std::lock_guard<std::mutex> lock(F->ws_mutex);
    for (double& x : g_phase_ms) x = 0.0;
    g_batches = 0;
    const int mb = max_batch(F);
    for (int64_t q0 = 0; q0 < J.nq; q0 += mb) {
        const int nb = int(std::min<int64_t>(mb, J.nq - q0));
        gf_status s = run_batch(F, J, q0, nb, st);
        if (s != GF_OK) return s;
    }
    return GF_OK;
}

gf_status validate_query_common(const gf_forest* F, const float* Q, int64_t nq, int32_t checks,
                                const int32_t* cpq, double eps) {
    if (!F) return fail(GF_EINVAL, "forest is NULL");
    if (nq < 0) return fail(GF_EINVAL, "nq < 0");
    if (nq > 0 && !Q) return fail(GF_EINVAL, "Q is NULL");
    if (!cpq && checks < 1) return fail(GF_EINVAL, "checks < 1");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(GF_EINVAL, "eps must be finite and >= 0");
    return GF_OK;
}

// Validation and setup shared by gf_query and gf_query_multi: parameters
// first (no HIP call), then where each buffer lives.
// With noalloc (gf_query_noalloc) every buffer must be device memory and
// device budgets are used as they are (not read back).
gf_status prepare_job(const gf_forest* Fc, const float* Q, int64_t nq, int32_t k, int32_t checks,
                      const int32_t* checks_per_query, double eps, int32_t form, int32_t rerank,
                      int32_t* ids, float* dists, QueryJob& J, bool noalloc = false) {
    gf_status s = validate_query_common(Fc, Q, nq, checks, checks_per_query, eps);
    if (s != GF_OK) return s;
    if (k < 1 || k > gf::kMaxK) return fail(GF_EINVAL, "k must be in [1, 64]");
    if (nq > 0 && (!ids || !dists)) return fail(GF_EINVAL, "ids or dists is NULL");
    if (form != GF_FORM_FP32 && form != GF_FORM_BF16 && form != GF_FORM_FP8)
        return fail(GF_EINVAL, "unknown form");
    const gf_forest* F = Fc;
    if (form == GF_FORM_BF16 && !F->X16) return fail(GF_EINVAL, "forest was built without GF_KEEP_BF16");
    if (form == GF_FORM_FP8 && !F->X8) return fail(GF_EINVAL, "forest was built without GF_KEEP_FP8");
    int kk;
    if (form == GF_FORM_FP32) {
        kk = std::min(gf::kMaxK, k + 8);
    } else {
        if (rerank == 0) rerank = std::min(gf::kMaxK, 4 * k);
        if (rerank < k || rerank > gf::kMaxK) return fail(GF_EINVAL, "rerank must be in [k, 64]");
        kk = rerank;
    }
    if (gf::scan_max_slice_words(form, F->ld8) == 0)
        return fail(GF_EUNSUPPORTED, "d too large to stage the FP8 query in the scan's LDS");
    if (!gf::scan_supported(F->host.n, form, F->ld8) && kk > gf::kTileList)
        return fail(GF_EUNSUPPORTED, "n above one workgroup's visited bitmap (sliced id ranges) "
                                     "needs at most 48 list entries per query (k <= 40 in FP32)");
    J = QueryJob{};
    J.nq = nq; J.k = k; J.checks = checks; J.eps = eps; J.form = form; J.kk = kk;
    J.ids = ids; J.dists = dists;
    if (nq == 0) return GF_OK;
    J.Q = Q; J.q_dev = is_device_ptr(Q);
    J.cpq = checks_per_query; J.cpq_dev = checks_per_query && is_device_ptr(checks_per_query);
    J.checks_mean = double(checks);
    J.checks_max = checks;
    if (noalloc) {
        if (!J.q_dev || !is_device_ptr(ids) || !is_device_ptr(dists) || (checks_per_query && !J.cpq_dev))
            return fail(GF_EINVAL, "gf_query_noalloc takes device buffers for Q, budgets and outputs");
        J.out_dev = true;
        return GF_OK;
    }
    if (checks_per_query) {
        // every budget >= 1, and their mean for the path rule (device
        // budgets are read back once here)
        std::vector<int32_t> staged;
        const int32_t* c = checks_per_query;
        if (J.cpq_dev) {
            staged.resize(size_t(nq));
            GF_HIP(hipMemcpy(staged.data(), checks_per_query, size_t(nq) * 4, hipMemcpyDeviceToHost));
            c = staged.data();
        }
        double sum = 0.0;
        int64_t mx = 1;
        for (int64_t i = 0; i < nq; ++i) {
            if (c[i] < 1) return fail(GF_EINVAL, "checks_per_query has a value < 1");
            sum += double(c[i]);
            mx = std::max<int64_t>(mx, c[i]);
        }
        J.checks_mean = sum / double(nq);
        J.checks_max = mx;
    }
    J.out_dev = is_device_ptr(ids);
    if (J.out_dev != is_device_ptr(dists)) return fail(GF_EINVAL, "ids and dists must both be host or both device");
    return GF_OK;
}

// ------------------------------------------------------- multi-index launch

std::atomic<int64_t> g_graphs_built{0}, g_graphs_reused{0}, g_tuned{0};
std::atomic<uint64_t> g_next_uid{1};

// Instantiated graphs of earlier calls, keyed by everything the captured
// launches depend on: each batch's forest (by unique id), buffers, sizes,
// parameters and path, and the workspace address it was carved from.
struct GraphEntry {
    std::vector<uint64_t> key;
    std::vector<uint64_t> uids;
    hipGraphExec_t exec = nullptr;
};
std::mutex g_graph_mutex;
std::vector<GraphEntry> g_graphs;   // most recent last
constexpr size_t kGraphCache = 16;

void drop_graphs_of(uint64_t uid) {
    std::lock_guard<std::mutex> lock(g_graph_mutex);
    for (size_t i = 0; i < g_graphs.size();) {
        const auto& u = g_graphs[i].uids;
        if (std::find(u.begin(), u.end(), uid) != u.end()) {
            (void)hipGraphExecDestroy(g_graphs[i].exec);
            g_graphs.erase(g_graphs.begin() + i);
        } else {
            ++i;
        }
    }
}

struct MultiBatch {
    gf_forest* F;
    int job;
    int64_t q0;
    int nb;
    bool tile;
    int slice_mult;
};

// Launch variants the autotuner measures: the row path with 1, 2 or 4 times
// the rule's slices per query, and the tile path where the job has one.
constexpr int kTuneVariants = 4;

// Batch-size class of the autotuner (powers of two).
int size_class(int nb) {
    int c = 0;
    while ((1 << c) < nb) ++c;
    return c;
}

gf_status run_multi(const gf_job* jobs, int32_t njobs, uint32_t flags, hipStream_t st) {
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(GF_EINVAL, "jobs is NULL or njobs < 0");
    if (flags & ~uint32_t(GF_MULTI_AUTOTUNE | GF_MULTI_EAGER)) return fail(GF_EINVAL, "unknown bits in flags");
    for (int i = 0; i < njobs; ++i) {
        const gf_job& j = jobs[i];
        gf_status s = validate_query_common(j.forest, j.Q, j.nq, j.checks, j.checks_per_query, j.eps);
        if (s != GF_OK) return s;
    }
    std::vector<QueryJob> J(size_t(std::max(njobs, 0)));
    std::vector<gf_forest*> Fs;
    for (int i = 0; i < njobs; ++i) {
        const gf_job& j = jobs[i];
        gf_status s = prepare_job(j.forest, j.Q, j.nq, j.k, j.checks, j.checks_per_query, j.eps,
                                  j.form, j.rerank, j.ids, j.dists, J[i]);
        if (s != GF_OK) return s;
        if (j.nq == 0) continue;
        if (!J[i].q_dev || !J[i].out_dev || (J[i].cpq && !J[i].cpq_dev))
            return fail(GF_EINVAL, "gf_query_multi takes device buffers for Q, budgets and outputs");
        gf_forest* F = const_cast<gf_forest*>(j.forest);
        if (!Fs.empty() && F->device != Fs[0]->device)
            return fail(GF_EINVAL, "all forests of one gf_query_multi call must be on one device");
        Fs.push_back(F);
    }
    if (Fs.empty()) return GF_OK;
    std::sort(Fs.begin(), Fs.end());
    Fs.erase(std::unique(Fs.begin(), Fs.end()), Fs.end());
    GF_HIP(hipSetDevice(Fs[0]->device));
    std::vector<std::unique_lock<std::mutex>> locks;
    for (gf_forest* F : Fs) locks.emplace_back(F->ws_mutex);   // address order

    // Every query row finite (one readback for the whole call).
    {
        // a 4-byte flag from a per-device pool: taken for this call, returned
        // at its end, reused by later calls (the pool only grows to the
        // number of calls running at once)
        static std::mutex flag_mutex;
        static std::map<int, std::vector<uint32_t*>> pool;
        const int dev = Fs[0]->device;
        uint32_t* flag = nullptr;
        {
            std::lock_guard<std::mutex> lock(flag_mutex);
            std::vector<uint32_t*>& free_list = pool[dev];
            if (!free_list.empty()) {
                flag = free_list.back();
                free_list.pop_back();
            }
        }
        if (!flag) GF_HIP(gf::dev_malloc((void**)&flag, 4));
        struct FlagBack {
            uint32_t* f; int dev;
            ~FlagBack() { std::lock_guard<std::mutex> lock(flag_mutex); pool[dev].push_back(f); }
        } flag_back{flag, dev};
        GF_HIP(hipMemsetAsync(flag, 0, 4, st));
        for (int i = 0; i < njobs; ++i) {
            if (jobs[i].nq == 0) continue;
            const int64_t tot = jobs[i].nq * int64_t(jobs[i].forest->host.d);
            hipLaunchKernelGGL(gf::k_check_finite, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st,
                               jobs[i].Q, jobs[i].nq, jobs[i].forest->host.d,
                               int64_t(jobs[i].forest->host.d), flag);
            GF_HIP(hipGetLastError());
        }
        uint32_t bad = 0;
        GF_HIP(hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, st));
        GF_HIP(hipStreamSynchronize(st));
        if (bad) return fail(GF_EINVAL, "Q contains a non-finite value");
    }

    // Batches, and the path of each: by rule, or measured once per
    // (forest, form, batch-size class, re-rank depth) when autotuning.
    std::vector<MultiBatch> B;
    for (int i = 0; i < njobs; ++i) {
        gf_forest* F = const_cast<gf_forest*>(jobs[i].forest);
        const int mb = max_batch(F);
        for (int64_t q0 = 0; q0 < jobs[i].nq; q0 += mb) {
            const int nb = int(std::min<int64_t>(mb, jobs[i].nq - q0));
            QueryJob Jb = J[i];
            bool tile = use_tile_path(F, Jb, nb);
            int mult = 1;
            if (flags & GF_MULTI_AUTOTUNE) {
                const uint64_t key = (uint64_t(Jb.form) << 40) | (uint64_t(size_class(nb)) << 32) | uint64_t(Jb.kk);
                auto it = F->tuned.find(key);
                if (it == F->tuned.end()) {
                    float ms[kTuneVariants];
                    int best = 0;
                    hipEvent_t e0, e1;
                    GF_HIP(hipEventCreate(&e0));
                    GF_HIP(hipEventCreate(&e1));
                    gf_status s = GF_OK;
                    for (int v = 0; v < kTuneVariants && s == GF_OK; ++v) {
                        ms[v] = 1e30f;
                        if (v == 3 && !tile_eligible(F, Jb)) continue;
                        Jb.path = v == 3 ? 1 : 0;
                        Jb.slice_mult = v == 3 ? 1 : (1 << v);
                        // the workspace may grow for this variant: not inside the timing
                        Workspace wtmp;
                        const ScanSlices sl = v == 3 ? ScanSlices{} : scan_slices(F, Jb, nb);
                        s = get_workspace(F, nb, Jb.k, Jb.form, v == 3, wtmp, Jb.checks_max, sl.nslice);
                        for (int rep = 0; rep < 2 && s == GF_OK; ++rep) {   // first run warms up
                            (void)hipEventRecord(e0, st);
                            s = run_batch(F, Jb, q0, nb, st, true);
                            (void)hipEventRecord(e1, st);
                            (void)hipEventSynchronize(e1);
                        }
                        (void)hipEventElapsedTime(&ms[v], e0, e1);
                        if (ms[v] < ms[best]) best = v;
                    }
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    if (s != GF_OK) return s;
                    it = F->tuned.emplace(key, best).first;
                    g_tuned.fetch_add(1);
                }
                tile = it->second == 3;
                mult = tile ? 1 : (1 << it->second);
            }
            B.push_back(MultiBatch{F, i, q0, nb, tile, mult});
        }
    }
    // Grow every workspace to its largest batch before any capture.
    for (const MultiBatch& b : B) {
        Workspace w;
        QueryJob Jb = J[b.job];
        Jb.slice_mult = b.slice_mult;
        const ScanSlices sl = b.tile ? ScanSlices{} : scan_slices(b.F, Jb, b.nb);
        gf_status s = get_workspace(b.F, b.nb, J[b.job].k, J[b.job].form, b.tile, w, J[b.job].checks_max,
                                    sl.nslice);
        if (s != GF_OK) return s;
    }
    auto launch_all = [&](hipStream_t s_) -> gf_status {
        for (const MultiBatch& b : B) {
            QueryJob Jb = J[b.job];
            Jb.path = b.tile ? 1 : 0;
            Jb.slice_mult = b.slice_mult;
            gf_status s = run_batch(b.F, Jb, b.q0, b.nb, s_, true);
            if (s != GF_OK) return s;
        }
        return GF_OK;
    };
    if (flags & GF_MULTI_EAGER) {
        gf_status s = launch_all(st);
        if (s != GF_OK) return s;
        GF_HIP(hipStreamSynchronize(st));
        return GF_OK;
    }
    std::vector<uint64_t> key;
    std::vector<uint64_t> uids;
    for (const MultiBatch& b : B) {
        const gf_job& j = jobs[b.job];
        const uint64_t vals[] = {b.F->uid, uint64_t(uintptr_t(b.F->ws)), uint64_t(b.F->ws_bytes),
                                 uint64_t(uintptr_t(j.Q)), uint64_t(uintptr_t(j.checks_per_query)),
                                 uint64_t(uintptr_t(j.ids)), uint64_t(uintptr_t(j.dists)),
                                 uint64_t(b.q0), uint64_t(b.nb), uint64_t(j.k), uint64_t(uint32_t(j.checks)),
                                 uint64_t(J[b.job].kk), uint64_t(j.form), uint64_t(b.tile),
                                 uint64_t(b.slice_mult),
                                 uint64_t(std::llround(j.eps * 1e12))};
        key.insert(key.end(), std::begin(vals), std::end(vals));
        uids.push_back(b.F->uid);
    }
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_graph_mutex);
        for (size_t i = 0; i < g_graphs.size(); ++i) {
            if (g_graphs[i].key == key) {
                exec = g_graphs[i].exec;
                std::rotate(g_graphs.begin() + i, g_graphs.begin() + i + 1, g_graphs.end());
                break;
            }
        }
    }
    if (exec) {
        g_graphs_reused.fetch_add(1);
    } else {
        // Capture on streams of our own (the caller's may be the null
        // stream, which cannot be captured); the graph runs on the caller's.
        // The batches of each forest form one branch of the graph (they
        // share the forest's workspace); branches of different forests run
        // concurrently, up to kBranches at a time.
        constexpr int kBranches = 8;
        static thread_local hipStream_t cap = nullptr;
        static thread_local hipStream_t br[kBranches] = {};
        static thread_local hipEvent_t fork = nullptr, join[kBranches] = {};
        static thread_local int cap_dev = -1;
        if (cap_dev != Fs[0]->device) {
            GF_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            GF_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
            for (int i = 0; i < kBranches; ++i) {
                GF_HIP(hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking));
                GF_HIP(hipEventCreateWithFlags(&join[i], hipEventDisableTiming));
            }
            cap_dev = Fs[0]->device;
        }
        const int nbr = std::min<int>(kBranches, int(Fs.size()));
        GF_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        gf_status s = GF_OK;
        hipError_t eb = hipEventRecord(fork, cap);
        for (int i = 0; i < nbr && eb == hipSuccess; ++i) eb = hipStreamWaitEvent(br[i], fork, 0);
        for (const MultiBatch& b : B) {
            if (eb != hipSuccess || s != GF_OK) break;
            const int g = int(std::lower_bound(Fs.begin(), Fs.end(), b.F) - Fs.begin()) % nbr;
            QueryJob Jb = J[b.job];
            Jb.path = b.tile ? 1 : 0;
            Jb.slice_mult = b.slice_mult;
            s = run_batch(b.F, Jb, b.q0, b.nb, br[g], true);
        }
        for (int i = 0; i < nbr && eb == hipSuccess; ++i) {
            eb = hipEventRecord(join[i], br[i]);
            if (eb == hipSuccess) eb = hipStreamWaitEvent(cap, join[i], 0);
        }
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(cap, &graph);
        if (s == GF_OK && eb != hipSuccess) s = fail(GF_EHIP, std::string("graph branches: ") + hipGetErrorString(eb));
        if (s != GF_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        GF_HIP(ec);
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        GF_HIP(ei);
        g_graphs_built.fetch_add(1);
        std::lock_guard<std::mutex> lock(g_graph_mutex);
        if (g_graphs.size() >= kGraphCache) {
            (void)hipGraphExecDestroy(g_graphs.front().exec);
            g_graphs.erase(g_graphs.begin());
        }
        g_graphs.push_back(GraphEntry{key, uids, exec});
    }
    GF_HIP(hipGraphLaunch(exec, st));
    GF_HIP(hipStreamSynchronize(st));
    return GF_OK;
}

// Streaming read of n16 16-byte words, nothing written: what the memory
// system delivers to a plain read stream on this device, the ceiling beside
// the rooflines' 8 TB/s.  Workgroups take contiguous spans of 16 x 256
// words (64 KB) in turn, each thread with its sixteen non-temporal loads in
// flight; the block that owns the last, partial span reads it word by word.  The XOR of the
// data keeps the loads; the sink (external, so it cannot be proven unread)
// is written only if it hits a constant.
constexpr int kProbeUnroll = 16;
}  // namespace

namespace gf {

hipError_t dev_malloc(void** p, size_t bytes) {
    *p = nullptr;
    const size_t cap = device_cap();
    std::lock_guard<std::mutex> lock(g_alloc_mutex);
    if (cap != 0 && g_alloc_total + bytes > cap) return hipErrorOutOfMemory;
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    g_alloc_size[*p] = bytes;
    g_alloc_total += bytes;
    return hipSuccess;
}

void dev_free(void* p) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mutex);
        auto it = g_alloc_size.find(p);
        if (it != g_alloc_size.end()) {
            g_alloc_total -= it->second;
            g_alloc_size.erase(it);
        }
    }
    (void)hipFree(p);
}

size_t dev_bytes_held() {
    std::lock_guard<std::mutex> lock(g_alloc_mutex);
    return g_alloc_total;
}

}  // namespace gf
__device__ uint32_t gf_probe_sink;
namespace {
__global__ __launch_bounds__(256) void k_read_probe(const uint4* __restrict__ p, int64_t n16) {
    const int64_t span = int64_t(blockDim.x) * kProbeUnroll;
    const int64_t step = int64_t(gridDim.x) * span;
    int64_t base = int64_t(blockIdx.x) * span;
    uint32_t acc = 0;
    typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));
    const v4u32* q = reinterpret_cast<const v4u32*>(p);
    for (; base + span <= n16; base += step) {
        v4u32 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
            v[u] = __builtin_nontemporal_load(q + base + u * int64_t(blockDim.x) + threadIdx.x);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (int64_t i = base + threadIdx.x; i < n16; i += blockDim.x) {
        const uint4 a = p[i];
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    if (acc == 0x9E3779B9u) gf_probe_sink = acc;
}

}  // namespace

// ------------------------------------------------- allocation-free queries
// The workspace of gf_query_noalloc: one file-scope device array, a copy on
// every GPU the library runs on, held until the process ends.  In host code
// its name is only a stand-in: the device address of each GPU's copy comes
// from hipGetSymbolAddress, taken once per device with that device current
// (scratch_base), and only that address is handed to kernels and copies.
constexpr size_t kNoAllocScratchBytes = size_t{128} << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;                  // guards g_scratch_ptr
char* g_scratch_ptr[kMaxDevices] = {};       // device address of each GPU's copy
std::mutex g_scratch_call[kMaxDevices];      // one call at a time per GPU

// Device address of the current device's copy of `scratch` (dev current).
gf_status scratch_base(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(GF_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GF_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return GF_OK;
}

}  // namespace

extern "C" {

const char* gf_last_error(void) { return g_last_error.c_str(); }

gf_status gf_query_noalloc(const gf_forest* Fc, const float* Q, int64_t nq, int32_t k,
                           int32_t checks, const int32_t* checks_per_query, double eps,
                           int32_t form, int32_t rerank, int32_t* ids, float* dists, void* stream) {
    QueryJob J{};
    gf_status s = prepare_job(Fc, Q, nq, k, checks, checks_per_query, eps, form, rerank, ids, dists,
                              J, true);
    if (s != GF_OK || nq == 0) return s;
    gf_forest* F = const_cast<gf_forest*>(Fc);
    J.path = 0;
    // the largest batch whose row-path workspace fits the scratch array
    auto need = [&](int b) {
        return ws_layout(F, b, J.k, J.form, false, 0, scan_slices(F, J, b).nslice).need;
    };
    const size_t one = need(1);
    if (one > kNoAllocScratchBytes)
        return fail(GF_EUNSUPPORTED, "one query's workspace (" + std::to_string(one) +
                                         " bytes) exceeds the 128 MiB scratch of gf_query_noalloc");
    const size_t per = ws_layout(F, 2, J.k, J.form, false).need - ws_layout(F, 1, J.k, J.form, false).need + 256;
    int nb = int(std::min<int64_t>(max_batch(F), int64_t((kNoAllocScratchBytes - one) / per) + 1));
    while (nb > 1 && need(nb) > kNoAllocScratchBytes) --nb;
    GF_HIP(hipSetDevice(F->device));
    char* base = nullptr;
    if ((s = scratch_base(F->device, &base)) != GF_OK) return s;
    std::lock_guard<std::mutex> lock(g_scratch_call[F->device]);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    for (int64_t q0 = 0; q0 < nq; q0 += nb) {
        const int b = int(std::min<int64_t>(nb, nq - q0));
        if ((s = run_batch(F, J, q0, b, st, false, base)) != GF_OK) return s;
    }
    return GF_OK;
}

const char* gf_version(void) { return "geraf-gfx950 0.1"; }

int64_t gf_device_bytes(void) { return int64_t(gf::dev_bytes_held()); }

gf_status gf_last_query_timing(double* phase_ms, int32_t nphase, int32_t* path, int64_t* batches) {
    if (nphase < 0 || (nphase > 0 && !phase_ms)) return fail(GF_EINVAL, "bad phase buffer");
    for (int i = 0; i < nphase; ++i) phase_ms[i] = i < kPhases ? g_phase_ms[i] : 0.0;
    if (path) *path = g_path;
    if (batches) *batches = g_batches;
    return GF_OK;
}

gf_status gf_build_forest(const float* X, int64_t n, int32_t d, int32_t m, int32_t t, int32_t leaf,
                          uint64_t seed, uint32_t forms, void* stream, gf_forest** out) {
    return gf_build_forest_ex(X, n, d, m, t, leaf, seed, forms, 0u, stream, out);
}

gf_status gf_build_forest_ex(const float* X, int64_t n, int32_t d, int32_t m, int32_t t,
                             int32_t leaf, uint64_t seed, uint32_t forms, uint32_t variants,
                             void* stream, gf_forest** out) {
    if (!out) return fail(GF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!X) return fail(GF_EINVAL, "X is NULL");
    if (n < 1 || n >= (int64_t{1} << 31)) return fail(GF_EINVAL, "n must be in [1, 2^31)");
    if (d < 1) return fail(GF_EINVAL, "d < 1");
    if (m < 1 || m > 255) return fail(GF_EINVAL, "m must be in [1, 255]");
    if (t < 1 || t > d) return fail(GF_EINVAL, "t must be in [1, d]");
    if (t > gf::kMaxT) return fail(GF_EUNSUPPORTED, "t above 64");
    if (leaf < 1) return fail(GF_EINVAL, "leaf < 1");
    if (forms & ~(GF_KEEP_BF16 | GF_KEEP_FP8 | GF_BUILD_DEVICE)) return fail(GF_EINVAL, "unknown bits in forms");
    if (variants & ~(GF_VARIANT_HOUSEHOLDER | GF_VARIANT_JITTER | GF_VARIANT_JITTER_EXACT))
        return fail(GF_EINVAL, "unknown bits in variants");
    const int jitter = (variants & GF_VARIANT_JITTER_EXACT) ? 2 : (variants & GF_VARIANT_JITTER) ? 1 : 0;
    if (jitter && (variants & GF_VARIANT_HOUSEHOLDER))
        return fail(GF_EUNSUPPORTED, "split-value jitter with the isometry variant");
    if (jitter && (forms & GF_BUILD_DEVICE))
        return fail(GF_EUNSUPPORTED, "split-value jitter is built on the host only");
    if (gf::perfect_depth(n, leaf) > 23) return fail(GF_EUNSUPPORTED, "tree depth above 23");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // GF_BUILD_TIMING=1 prints the wall time of each build phase to stderr
    const char* tenv = std::getenv("GF_BUILD_TIMING");
    const bool timing = tenv && tenv[0] == '1';
    auto tprev = std::chrono::steady_clock::now();
    auto phase = [&](const char* what) {
        if (!timing) return;
        (void)hipStreamSynchronize(st);
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[gf_build_forest] %-28s %8.3f s\n", what,
                     std::chrono::duration<double>(now - tprev).count());
        tprev = now;
    };

    // the FP32 rows alone must fit under the device-memory cap (checked
    // before any HIP call)
    if (exceeds_cap(size_t(n) * size_t(round_up(d, 4)) * 4))
        return fail(GF_ENOMEM, "the FP32 rows exceed GF_MAX_DEVICE_BYTES");
    const bool on_device = (forms & GF_BUILD_DEVICE) != 0;
    const bool reflect = (variants & GF_VARIANT_HOUSEHOLDER) != 0;
    const bool xdev = is_device_ptr(X);
    // host rows: the host build reads them; device rows are checked on the
    // device when the build runs there
    std::vector<float> staged;
    const float* Xh = xdev ? nullptr : X;
    if (xdev && !on_device) {
        staged.resize(size_t(n) * d);
        GF_HIP(hipMemcpy(staged.data(), X, staged.size() * 4, hipMemcpyDeviceToHost));
        Xh = staged.data();
    }
    if (Xh && !all_finite_host(Xh, n * int64_t(d))) return fail(GF_EINVAL, "X contains a non-finite value");
    phase("stage + finiteness check");

    std::unique_ptr<gf_forest> F(new gf_forest());
    if (!on_device) {
        std::string err = gf::build_host_forest(Xh, n, d, m, t, leaf, seed, reflect, F->host, jitter);
        if (!err.empty())
            return fail(err.rfind("near-tie", 0) == 0 ? GF_EINVAL
                        : err.rfind("a jittered tree", 0) == 0 ? GF_EUNSUPPORTED
                        : GF_EINTERNAL, err);
        phase("host trees");
    }
    GF_HIP(hipGetDevice(&F->device));
    F->uid = g_next_uid.fetch_add(1);
    const gf::HostForest& h = F->host;
    F->ld32 = int32_t(round_up(d, 4));
    F->ld16 = int32_t(round_up(d, 32));   // multiple of one MFMA k step (32 bf16)
    F->ld8 = int32_t(round_up(d, 16));
    auto cleanup = [&](gf_status s) { free_forest_device(F.get()); return s; };

#define GF_HIP_B(expr)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return cleanup(fail(e_ == hipErrorOutOfMemory ? GF_ENOMEM : GF_EHIP,         \
                                std::string(#expr) + ": " + hipGetErrorString(e_)));     \
    } while (0)

    GF_HIP_B(gf::dev_malloc((void**)&F->X32, size_t(n) * F->ld32 * 4));
    if (xdev) {
        // X is already on the device: copy the rows into the padded layout
        if (F->ld32 > d) GF_HIP_B(hipMemsetAsync(F->X32, 0, size_t(n) * F->ld32 * 4, st));
        GF_HIP_B(hipMemcpy2DAsync(F->X32, size_t(F->ld32) * 4, X, size_t(d) * 4, size_t(d) * 4, n,
                                  hipMemcpyDeviceToDevice, st));
    } else {
        GF_HIP_B(upload_rows(F->X32, Xh, n, d, F->ld32, st));
    }
    if (!Xh) {
        // device rows that were not staged: every value finite
        uint32_t* flag = nullptr;
        GF_HIP_B(gf::dev_malloc((void**)&flag, 4));
        uint32_t bad = 0;
        hipError_t e = hipMemsetAsync(flag, 0, 4, st);
        const int64_t tot = n * int64_t(d);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(gf::k_check_finite, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st,
                               F->X32, n, d, int64_t(F->ld32), flag);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        gf::dev_free(flag);
        GF_HIP_B(e);
        if (bad) return cleanup(fail(GF_EINVAL, "X contains a non-finite value"));
    }
    phase("X upload");
    if (on_device) {
        std::string err = gf::build_device_forest(F->X32, F->ld32, n, d, m, t, leaf, seed, reflect, st,
                                                  F->host);
        if (!err.empty()) {
            const gf_status code = err.rfind("near-tie", 0) == 0 ? GF_EINVAL
                                   : err.rfind("leaves above", 0) == 0 ? GF_EUNSUPPORTED
                                   : GF_EHIP;
            return cleanup(fail(code, err));
        }
        phase("device trees");
    }
    const int64_t nint = (int64_t{1} << h.H) - 1;
    std::vector<uint2> nodes(size_t(m) * std::max<int64_t>(nint, 1));
    for (int64_t i = 0; i < int64_t(m) * nint; ++i) {
        uint32_t bits;
        std::memcpy(&bits, &h.split_val[i], 4);
        nodes[i] = make_uint2(bits, h.split_slot[i]);
    }
    GF_HIP_B(gf::dev_malloc((void**)&F->nodes, nodes.size() * sizeof(uint2)));
    GF_HIP_B(hipMemcpyAsync(F->nodes, nodes.data(), nodes.size() * sizeof(uint2), hipMemcpyHostToDevice, st));
    GF_HIP_B(gf::dev_malloc((void**)&F->perm, h.perm.size() * 4));
    GF_HIP_B(hipMemcpyAsync(F->perm, h.perm.data(), h.perm.size() * 4, hipMemcpyHostToDevice, st));
    GF_HIP_B(gf::dev_malloc((void**)&F->leaf_off, h.leaf_off.size() * 4));
    GF_HIP_B(hipMemcpyAsync(F->leaf_off, h.leaf_off.data(), h.leaf_off.size() * 4, hipMemcpyHostToDevice, st));
    {
        // leaf rows padded to pp ids (pow2 >= the largest leaf, >= 4)
        const int64_t nleaf = int64_t{1} << h.H;
        uint32_t maxleaf = 0;
        for (int32_t tr = 0; tr < m; ++tr) {
            const uint32_t* lo = h.leaf_off.data() + size_t(tr) * (nleaf + 1);
            for (int64_t j = 0; j < nleaf; ++j) maxleaf = std::max(maxleaf, lo[j + 1] - lo[j]);
        }
        int32_t pp = 4;
        while (uint32_t(pp) < maxleaf) pp <<= 1;
        F->pp = pp;
        F->maxleaf = int32_t(maxleaf);
        std::vector<uint32_t> padded(size_t(m) * nleaf * pp, 0xFFFFFFFFu);
        for (int32_t tr = 0; tr < m; ++tr) {
            const uint32_t* lo = h.leaf_off.data() + size_t(tr) * (nleaf + 1);
            for (int64_t j = 0; j < nleaf; ++j)
                for (uint32_t i = lo[j]; i < lo[j + 1]; ++i)
                    padded[(size_t(tr) * nleaf + j) * pp + (i - lo[j])] = h.perm[size_t(tr) * n + i];
        }
        GF_HIP_B(gf::dev_malloc((void**)&F->permp, padded.size() * 4));
        GF_HIP_B(hipMemcpy(F->permp, padded.data(), padded.size() * 4, hipMemcpyHostToDevice));
    }
    phase("nodes, perm, padded leaves");
    GF_HIP_B(gf::dev_malloc((void**)&F->D, size_t(t) * 4));
    GF_HIP_B(hipMemcpyAsync(F->D, h.D.data(), size_t(t) * 4, hipMemcpyHostToDevice, st));
    {
        // range of the split values on each slot of D (0, 0 for an unused slot)
        std::vector<float2> rng(size_t(t), make_float2(0.0f, 0.0f));
        std::vector<char> used(size_t(t), 0);
        for (int64_t i = 0; i < int64_t(m) * nint; ++i) {
            const int j = h.split_slot[i];
            const float v = h.split_val[i];
            if (!std::isfinite(v)) continue;   // pass-through node of a jittered tree
            if (!used[j]) { rng[j] = make_float2(v, v); used[j] = 1; }
            rng[j].x = std::min(rng[j].x, v);
            rng[j].y = std::max(rng[j].y, v);
        }
        GF_HIP_B(gf::dev_malloc((void**)&F->drange, size_t(t) * sizeof(float2)));
        GF_HIP_B(hipMemcpy(F->drange, rng.data(), size_t(t) * sizeof(float2), hipMemcpyHostToDevice));
    }
    if (!h.U.empty()) {
        // device copy transposed to [d][m]: the trees of one query read one row
        std::vector<double> ut(h.U.size());
        for (int32_t tr = 0; tr < m; ++tr)
            for (int32_t j = 0; j < d; ++j) ut[size_t(j) * m + tr] = h.U[size_t(tr) * d + j];
        GF_HIP_B(gf::dev_malloc((void**)&F->U, ut.size() * sizeof(double)));
        GF_HIP_B(hipMemcpy(F->U, ut.data(), ut.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (forms & (GF_KEEP_BF16 | GF_KEEP_FP8)) {
        // leaf of every point in every tree, point-major (tile paths)
        const int64_t nleaf = int64_t{1} << h.H;
        std::vector<uint32_t> lof(size_t(n) * m);
        for (int32_t tr = 0; tr < m; ++tr) {
            const uint32_t* lo = h.leaf_off.data() + size_t(tr) * (nleaf + 1);
            for (int64_t j = 0; j < nleaf; ++j)
                for (uint32_t i = lo[j]; i < lo[j + 1]; ++i)
                    lof[size_t(h.perm[size_t(tr) * n + i]) * m + tr] = uint32_t(tr * nleaf + j);
        }
        GF_HIP_B(gf::dev_malloc((void**)&F->leafof, lof.size() * 4));
        GF_HIP_B(hipMemcpy(F->leafof, lof.data(), lof.size() * 4, hipMemcpyHostToDevice));
        phase("leaf of each point");
    }
    if (forms & GF_KEEP_BF16) {
        GF_HIP_B(gf::dev_malloc((void**)&F->X16, size_t(n) * F->ld16 * 2));
        GF_HIP_B(gf::dev_malloc((void**)&F->norm16, size_t(n) * 4));
        hipLaunchKernelGGL(gf::k_to_bf16, dim3((n + 3) / 4), dim3(256), 0, st, F->X32, n, d,
                           int64_t(F->ld32), F->X16, int64_t(F->ld16), F->norm16);
        GF_HIP_B(hipGetLastError());
    }
    if (forms & GF_KEEP_FP8) {
        GF_HIP_B(gf::dev_malloc((void**)&F->X8, size_t(n) * F->ld8));
        GF_HIP_B(gf::dev_malloc((void**)&F->scale8, size_t(n) * 4));
        GF_HIP_B(gf::dev_malloc((void**)&F->norm8, size_t(n) * 4));
        hipLaunchKernelGGL(gf::k_to_fp8, dim3((n + 3) / 4), dim3(256), 0, st, F->X32, n, d,
                           int64_t(F->ld32), F->X8, int64_t(F->ld8), F->scale8, F->norm8);
        GF_HIP_B(hipGetLastError());
    }
    GF_HIP_B(hipStreamSynchronize(st));
    phase("reduced-precision copies");
#undef GF_HIP_B
    *out = F.release();
    return GF_OK;
}

gf_status gf_free_forest(gf_forest* F) {
    if (!F) return GF_OK;
    (void)hipSetDevice(F->device);
    drop_graphs_of(F->uid);
    free_forest_device(F);
    delete F;
    return GF_OK;
}

gf_status gf_forest_info(const gf_forest* F, int64_t* n, int32_t* d, int32_t* m, int32_t* t,
                         int32_t* leaf, int32_t* H) {
    if (!F) return fail(GF_EINVAL, "forest is NULL");
    if (n) *n = F->host.n;
    if (d) *d = F->host.d;
    if (m) *m = F->host.m;
    if (t) *t = F->host.t;
    if (leaf) *leaf = F->host.p;
    if (H) *H = F->host.H;
    return GF_OK;
}

gf_status gf_export_tree(const gf_forest* F, int32_t* D, int32_t* split_dim, float* split_val,
                         uint32_t* perm, uint32_t* leaf_off) {
    if (!F) return fail(GF_EINVAL, "forest is NULL");
    const gf::HostForest& h = F->host;
    if (D) std::memcpy(D, h.D.data(), h.D.size() * 4);
    if (split_dim) std::memcpy(split_dim, h.split_dim.data(), h.split_dim.size() * 4);
    if (split_val) std::memcpy(split_val, h.split_val.data(), h.split_val.size() * 4);
    if (perm) std::memcpy(perm, h.perm.data(), h.perm.size() * 4);
    if (leaf_off) std::memcpy(leaf_off, h.leaf_off.data(), h.leaf_off.size() * 4);
    return GF_OK;
}

gf_status gf_query(const gf_forest* Fc, const float* Q, int64_t nq, int32_t k, int32_t checks,
                   const int32_t* checks_per_query, double eps, int32_t form, int32_t rerank,
                   int32_t* ids, float* dists, void* stream) {
    QueryJob J{};
    gf_status s = prepare_job(Fc, Q, nq, k, checks, checks_per_query, eps, form, rerank, ids, dists, J);
    if (s != GF_OK || nq == 0) return s;
    return run_query(const_cast<gf_forest*>(Fc), J, static_cast<hipStream_t>(stream));
}

gf_status gf_query_multi(const gf_job* jobs, int32_t njobs, uint32_t flags, void* stream) {
    return run_multi(jobs, njobs, flags, static_cast<hipStream_t>(stream));
}

gf_status gf_multi_stats(int64_t* graphs_built, int64_t* graphs_reused, int64_t* tuned) {
    if (graphs_built) *graphs_built = g_graphs_built.load();
    if (graphs_reused) *graphs_reused = g_graphs_reused.load();
    if (tuned) *tuned = g_tuned.load();
    return GF_OK;
}

gf_status gf_query_trace(const gf_forest* Fc, const float* Q, int64_t nq, int32_t checks,
                         const int32_t* checks_per_query, double eps, uint32_t* leaf_bits,
                         uint32_t* cand_bits, int64_t* ncand, void* stream) {
    return gf_query_trace_ex(Fc, Q, nq, checks, checks_per_query, eps, GF_TRACE_ROWS, leaf_bits,
                             cand_bits, ncand, stream);
}

gf_status gf_query_trace_ex(const gf_forest* Fc, const float* Q, int64_t nq, int32_t checks,
                            const int32_t* checks_per_query, double eps, int32_t path,
                            uint32_t* leaf_bits, uint32_t* cand_bits, int64_t* ncand, void* stream) {
    gf_status s = validate_query_common(Fc, Q, nq, checks, checks_per_query, eps);
    if (s != GF_OK) return s;
    if (path != GF_TRACE_ROWS && path != GF_TRACE_TILE) return fail(GF_EINVAL, "unknown trace path");
    gf_forest* F = const_cast<gf_forest*>(Fc);
    if (path == GF_TRACE_TILE && !F->leafof)
        return fail(GF_EINVAL, "the tile path's trace needs a forest built with GF_KEEP_BF16");
    if (path == GF_TRACE_ROWS && gf::scan_max_slice_words(GF_FORM_FP32, F->ld8) == 0)
        return fail(GF_EUNSUPPORTED, "the row scan does not fit the LDS");
    if (nq == 0) return GF_OK;
    QueryJob J{};
    J.Q = Q; J.q_dev = is_device_ptr(Q);
    J.cpq = checks_per_query; J.cpq_dev = checks_per_query && is_device_ptr(checks_per_query);
    if (checks_per_query && !J.cpq_dev) {
        for (int64_t i = 0; i < nq; ++i)
            if (checks_per_query[i] < 1) return fail(GF_EINVAL, "checks_per_query has a value < 1");
    }
    J.nq = nq; J.k = 1; J.checks = checks; J.eps = eps; J.form = GF_FORM_FP32; J.kk = 1;
    J.leaf_bits = leaf_bits; J.cand_bits = cand_bits; J.ncand = ncand;
    J.trace_tile = path == GF_TRACE_TILE;
    const void* any = leaf_bits ? (const void*)leaf_bits : cand_bits ? (const void*)cand_bits : (const void*)ncand;
    J.trace_dev = any && is_device_ptr(any);
    return run_query(F, J, static_cast<hipStream_t>(stream));
}

gf_status gf_hbm_probe(const void* buf, int64_t bytes, int32_t reps, double* read_gb_s,
                       void* stream) {
    if (!buf || bytes < 16 || reps < 1 || !read_gb_s)
        return fail(GF_EINVAL, "buf, bytes >= 16, reps >= 1 and read_gb_s are required");
    if (reinterpret_cast<uintptr_t>(buf) % 16 != 0) return fail(GF_EINVAL, "buf must be 16-byte aligned");
    if (!is_device_ptr(buf)) return fail(GF_EINVAL, "buf must be device memory");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n16 = bytes / 16;
    const dim3 grid(2048), block(256);
    hipEvent_t ev[2];
    GF_HIP(hipEventCreate(&ev[0]));
    struct EvGuard { hipEvent_t* e; int n; ~EvGuard() { for (int i = 0; i < n; ++i) (void)hipEventDestroy(e[i]); } } evg{ev, 1};
    GF_HIP(hipEventCreate(&ev[1]));
    evg.n = 2;
    const uint4* p = static_cast<const uint4*>(buf);
    hipLaunchKernelGGL(k_read_probe, grid, block, 0, st, p, n16);   // warm-up
    GF_HIP(hipGetLastError());
    GF_HIP(hipEventRecord(ev[0], st));
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_read_probe, grid, block, 0, st, p, n16);
    GF_HIP(hipGetLastError());
    GF_HIP(hipEventRecord(ev[1], st));
    GF_HIP(hipEventSynchronize(ev[1]));
    float ms = 0.0f;
    GF_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
    *read_gb_s = double(reps) * double(n16) * 16.0 / (double(ms) / 1e3) / 1e9;
    return GF_OK;
}

gf_status gf_fp8_tables(float* hw_decode, float* def_decode, const float* enc_in, int32_t n_enc,
                        uint8_t* enc_out) {
    if (!hw_decode || !def_decode || n_enc < 0 || (n_enc > 0 && (!enc_in || !enc_out)))
        return fail(GF_EINVAL, "bad arguments");
    float *dh = nullptr, *ds = nullptr, *din = nullptr;
    uint8_t* dout = nullptr;
    GF_HIP(gf::dev_malloc((void**)&dh, 256 * 4));
    GF_HIP(gf::dev_malloc((void**)&ds, 256 * 4));
    hipLaunchKernelGGL(gf::k_e4m3_decode_both, dim3(1), dim3(256), 0, 0, dh, ds);
    GF_HIP(hipGetLastError());
    GF_HIP(hipMemcpy(hw_decode, dh, 256 * 4, hipMemcpyDeviceToHost));
    GF_HIP(hipMemcpy(def_decode, ds, 256 * 4, hipMemcpyDeviceToHost));
    gf::dev_free(dh);
    gf::dev_free(ds);
    if (n_enc > 0) {
        GF_HIP(gf::dev_malloc((void**)&din, size_t(n_enc) * 4));
        GF_HIP(gf::dev_malloc((void**)&dout, size_t(n_enc)));
        GF_HIP(hipMemcpy(din, enc_in, size_t(n_enc) * 4, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(gf::k_e4m3_encode, dim3((n_enc + 255) / 256), dim3(256), 0, 0, din, n_enc, dout);
        GF_HIP(hipGetLastError());
        GF_HIP(hipMemcpy(enc_out, dout, size_t(n_enc), hipMemcpyDeviceToHost));
        gf::dev_free(din);
        gf::dev_free(dout);
    }
    return GF_OK;
}

}  // extern "C"
