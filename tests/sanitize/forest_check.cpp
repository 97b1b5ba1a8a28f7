// Sanitizer driver for the library's host forest build (forest_build.cpp):
// plain, reflected and jittered (both diameters) forests on small random data
// under AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status 0 when
// every build succeeds, each tree's ids are a permutation, the per-tree leaf
// offsets are monotone and cover the ids, and jittered leaves hold at most
// `leaf` points.  Compiled (host code only) and run by tests/test_sanitizers.py.
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_1603_09596_amd/csrc/forest.h"

static bool check(const gf::HostForest& F) {
    const int64_t nleaf = int64_t{1} << F.H;
    for (int32_t tr = 0; tr < F.m; ++tr) {
        std::vector<char> seen(F.n, 0);
        for (int64_t i = 0; i < F.n; ++i) {
            const uint32_t id = F.perm[size_t(tr) * F.n + i];
            if (id >= F.n || seen[id]) return false;
            seen[id] = 1;
        }
        const uint32_t* lo = F.leaf_off.data() + size_t(tr) * (nleaf + 1);
        if (lo[0] != 0 || lo[nleaf] != uint32_t(F.n)) return false;
        for (int64_t j = 0; j < nleaf; ++j) {
            if (lo[j + 1] < lo[j]) return false;
            if (F.jitter && lo[j + 1] - lo[j] > uint32_t(F.p)) return false;
        }
    }
    return true;
}

int main() {
    const int64_t n = 900;
    const int32_t d = 13, m = 3, t = 4, p = 6;
    std::mt19937 rng(3);
    std::uniform_real_distribution<float> U(-2.0f, 2.0f);
    std::vector<float> X(size_t(n) * d);
    for (float& x : X) x = U(rng);
    int code = 0;
    for (int variant = 0; variant < 4 && !code; ++variant) {
        gf::HostForest F;
        const bool reflect = variant == 1;
        const int jitter = variant >= 2 ? variant - 1 : 0;
        const std::string err = gf::build_host_forest(X.data(), n, d, m, t, p, 11, reflect, F, jitter);
        if (!err.empty()) { std::fprintf(stderr, "build %d: %s\n", variant, err.c_str()); code = 10 + variant; }
        else if (!check(F)) code = 20 + variant;
    }
    if (!code) std::puts("forest build sanitizer check passed");
    return code;
}
