// forest.h -- internal types of the kd-GeRaF library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/geraf.h"

namespace gf {

// Maximum size of the top-variance set D (query-side staging of q_D).
constexpr int kMaxT = 64;
// Largest k and re-rank depth (one list slot per lane of a wavefront).
constexpr int kMaxK = 64;

// Host-side forest arrays produced by the build (Alg. 1).
struct HostForest {
    int64_t n = 0;
    int32_t d = 0, m = 0, t = 0, p = 0, H = 0;
    uint64_t seed = 0;
    std::vector<int32_t> D;           // [t] ascending
    std::vector<int32_t> split_dim;   // [m][2^H - 1] column index
    std::vector<uint8_t> split_slot;  // [m][2^H - 1] index into D
    std::vector<float> split_val;     // [m][2^H - 1]
    std::vector<uint32_t> perm;       // [m][n] leaf-ordered point ids
    std::vector<uint32_t> leaf_off;   // [m][2^H + 1] leaf j of tree i: perm[i][off[i][j] .. off[i][j+1])
    std::vector<double> U;            // [m][d] reflectors of the isometry variant, or empty
    int jitter = 0;                   // split-value jitter: 0 none, 1 approximate, 2 exact diameter
    int64_t real_leaves = 0;          // leaves of the trees themselves (m 2^H without jitter)
};

// Device memory of the library: hipMalloc / hipFree that keep a running
// total, and refuse (hipErrorOutOfMemory) any allocation that would take it
// above GF_MAX_DEVICE_BYTES when that environment variable is set.
hipError_t dev_malloc(void** p, size_t bytes);
void dev_free(void* p);
size_t dev_bytes_held();

// Counter-based RNG (splitmix64 output function, keyed).
uint64_t splitmix64(uint64_t x);
uint64_t keyed_draw(uint64_t seed, uint64_t stream, uint64_t tree, uint64_t idx);

int32_t perfect_depth(int64_t n, int32_t p);

// Builds the host arrays; X is host memory [n][d].  With householder, tree i
// splits the reflected coordinates float32((I - 2 u_i u_i') x) (Sec. 2.1
// "Rotation", Sec. 2.2).  jitter (1 approximate, 2 exact diameter) perturbs
// every split value (Sec. 2.1 "Split value"): the trees are then built to
// whatever depth their nodes need and padded to a perfect layout (see
// forest_build.cpp).  Returns an empty string on success, else the error.
std::string build_host_forest(const float* X, int64_t n, int32_t d, int32_t m, int32_t t,
                              int32_t p, uint64_t seed, bool householder, HostForest& out,
                              int jitter = 0);

// D <- the t columns of largest variance V (variance descending, lower index
// first among equals), in ascending index order.  Returns the near-tie error
// when the t-th and (t+1)-th variances differ by at most 1e-12 of the larger
// of their mean squares V + M^2, else an empty string.
std::string select_dims(const std::vector<double>& V, const std::vector<double>& M, int64_t n,
                        int32_t t, std::vector<int32_t>& D);

// The same arrays built on the GPU (build.hip) from the device rows X32
// [n][ld32]: FP64 column moments on the device, then every tree level by
// level.  Equal to build_host_forest's arrays bit for bit, D included unless
// the near-tie guard decides differently on the two evaluations of V (only
// possible within a few ulps of its 1e-12 bound).  Leaves above 4096 points
// are refused.  Returns an empty string on success, else the error.
std::string build_device_forest(const float* X32, int64_t ld32, int64_t n, int32_t d, int32_t m,
                                int32_t t, int32_t p, uint64_t seed, bool householder,
                                hipStream_t st, HostForest& out);

// Reflector of tree `tree`: w_j uniform in [-1, 1) from the top 53 bits of
// keyed_draw(seed, 4, tree, j), normalised in FP64 (squares summed in index
// order).
void householder_vector(uint64_t seed, int32_t tree, int32_t d, double* u);

}  // namespace gf

// Device-resident forest (the opaque handle of the ABI).
struct gf_forest {
    gf::HostForest host;
    int device = 0;
    int32_t ld32 = 0;       // FP32 row stride (floats), multiple of 4
    int32_t ld16 = 0;       // BF16 row stride (elements), multiple of 8
    int32_t ld8 = 0;        // FP8 row stride (bytes), multiple of 16
    float* X32 = nullptr;           // [n][ld32]
    uint16_t* X16 = nullptr;        // [n][ld16] bfloat16 bits
    float* norm16 = nullptr;        // [n] ||bf16(x)||^2
    uint8_t* X8 = nullptr;          // [n][ld8] e4m3 bytes
    float* scale8 = nullptr;        // [n] per-row scale
    float* norm8 = nullptr;         // [n] ||dequant(x)||^2
    uint2* nodes = nullptr;         // [m][2^H - 1] {float bits of value, slot in D}
    uint32_t* perm = nullptr;       // [m][n]
    uint32_t* leaf_off = nullptr;   // [2^H + 1]
    uint32_t* permp = nullptr;      // [m][2^H][pp] leaf rows padded with 0xFFFFFFFF
    int32_t pp = 0;                 // ids per padded leaf row: pow2 >= max leaf size, >= 4
    uint32_t* leafof = nullptr;     // [n][m] tree * 2^H + leaf of each point (BF16 / FP8 forms)
    int32_t maxleaf = 0;            // points in the largest leaf
    int32_t* D = nullptr;           // [t]
    float2* drange = nullptr;       // [t] smallest and largest split value per slot of D
    double* U = nullptr;            // [d][m] reflectors, transposed (isometry variant), or null
    // Grow-only scratch for queries.  Calls on one forest are serialised by
    // this mutex (concurrent queries on one forest wait for each other).
    std::mutex ws_mutex;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // Grow-only pinned host buffer that stages host query rows (same mutex).
    void* hstage = nullptr;
    size_t hstage_bytes = 0;
    uint64_t uid = 0;               // unique per forest built in this process
    // path choices measured by the multi-index autotuner, keyed by
    // (form, batch-size class, re-rank depth): 0 rows, 1 tile
    std::map<uint64_t, int> tuned;
};
