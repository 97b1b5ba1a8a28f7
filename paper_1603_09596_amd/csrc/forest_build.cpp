// forest_build.cpp -- host-side construction of the randomized k-d forest
// (Alg. 1, Sec. 2.2; storage of Sec. 3 "Tree structure").
//
// Each tree is built level by level over one permutation array: at depth h
// every node owns a contiguous segment of it, and splitting a node is a
// selection (std::nth_element) of its floor(|P|/2) smallest points under the
// order (coordinate in the split dimension, per-tree random key, id), which
// is the paper's median split with its "shuffling" tie-break made
// deterministic.  Trees are independent and are built by separate threads
// (Sec. 3 "Parallelization").
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <thread>

#include "forest.h"

namespace gf {

uint64_t splitmix64(uint64_t x) {
    // splitmix64 output function (Steele, Lea, Flood 2014): advance by the
    // golden-ratio increment, then two xor-shift-multiply rounds.
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

uint64_t keyed_draw(uint64_t seed, uint64_t stream, uint64_t tree, uint64_t idx) {
    uint64_t h = splitmix64(seed);
    h = splitmix64(h ^ stream);
    h = splitmix64(h ^ tree);
    return splitmix64(h ^ idx);
}

int32_t perfect_depth(int64_t n, int32_t p) {
    int32_t H = 0;
    while (((n + (int64_t{1} << H) - 1) >> H) > p) ++H;
    return H;
}

namespace {

constexpr uint64_t kStreamSplitDim = 1;
constexpr uint64_t kStreamTieKey = 2;
constexpr uint64_t kStreamJitter = 3;
constexpr uint64_t kStreamReflector = 4;
constexpr int32_t kMaxDepth = 23;

// u . x in FP64: each product rounded, then added in index order (no fused
// multiply-add, so the device reproduces it bit for bit).
double reflector_dot(const double* u, const float* x, int32_t d) {
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        const double prod = u[j] * double(x[j]);
        acc = acc + prod;
    }
    return acc;
}

// Coordinate s of (I - 2uu') x given t = u . x, rounded once to float32.
float reflected(float xs, double t, double us) {
#pragma clang fp contract(off)
    const double r = (2.0 * t) * us;
    return float(double(xs) - r);
}

unsigned worker_count(int64_t jobs) {
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    return static_cast<unsigned>(std::min<int64_t>(hw, std::max<int64_t>(1, jobs)));
}

// Per-dimension variance with Knuth's online update (Alg. 3), run over a
// block of rows per thread; the per-block (count, mean, M2) triples are then
// combined pairwise (Chan, Golub, LeVeque).
void column_variance(const float* X, int64_t n, int32_t d, std::vector<double>& V,
                     std::vector<double>& M) {
    V.assign(d, 0.0);
    M.assign(d, 0.0);
    if (n < 2) return;
    const unsigned nw = worker_count(n / 4096 + 1);
    std::vector<std::vector<double>> mean(nw, std::vector<double>(d, 0.0));
    std::vector<std::vector<double>> m2(nw, std::vector<double>(d, 0.0));
    std::vector<int64_t> cnt(nw, 0);
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nw; ++w) {
        th.emplace_back([&, w] {
            int64_t a = n * w / nw, b = n * (w + 1) / nw;
            double* mu = mean[w].data();
            double* v = m2[w].data();
            for (int64_t i = a; i < b; ++i) {
                const double alpha = 1.0 / double(i - a + 1);
                const float* x = X + i * d;
                for (int32_t j = 0; j < d; ++j) {
                    double delta = double(x[j]) - mu[j];
                    mu[j] += alpha * delta;
                    v[j] += delta * (double(x[j]) - mu[j]);
                }
            }
            cnt[w] = b - a;
        });
    }
    for (auto& t : th) t.join();
    std::vector<double> mu = mean[0], v = m2[0];
    double na = double(cnt[0]);
    for (unsigned w = 1; w < nw; ++w) {
        double nb = double(cnt[w]);
        if (nb == 0) continue;
        double nt = na + nb;
        for (int32_t j = 0; j < d; ++j) {
            double delta = mean[w][j] - mu[j];
            mu[j] += delta * nb / nt;
            v[j] += m2[w][j] + delta * delta * na * nb / nt;
        }
        na = nt;
    }
    for (int32_t j = 0; j < d; ++j) V[j] = v[j] / double(n - 1);
    M = mu;
}

// Whether the top-t set is not determined by the data: the t-th and
// (t+1)-th largest variances (order: variance descending, index ascending)
// differ by at most 1e-12 of the larger mean square V + mean^2 of the two
// columns, the scale of the rounding error of any FP64 evaluation.  Two
// correct evaluations (this online update, a two-pass sum) could then rank
// them differently.  n < 2 (V = 0 by definition) and columns of mean square
// 0 are exact.
bool dims_ambiguous(const std::vector<double>& V, const std::vector<double>& M,
                    const std::vector<int32_t>& order, int64_t n, int32_t t) {
    const int32_t d = int32_t(V.size());
    if (n < 2 || t >= d) return false;
    const int32_t a = order[t - 1], b = order[t];
    const double scale = std::max(V[a] + M[a] * M[a], V[b] + M[b] * M[b]);
    if (!(scale > 0.0)) return false;
    return V[a] - V[b] <= 1e-12 * scale;
}

struct Item {
    float x;
    uint64_t key;
    uint32_t id;
};

inline bool item_less(const Item& a, const Item& b) {
    if (a.x < b.x) return true;      // float order: -0 and +0 compare equal
    if (b.x < a.x) return false;
    if (a.key != b.key) return a.key < b.key;
    return a.id < b.id;
}

void build_tree(const float* X, int64_t n, int32_t d, const HostForest& F, int32_t tree,
                std::vector<int32_t>& split_dim, std::vector<uint8_t>& split_slot,
                std::vector<float>& split_val, uint32_t* ids) {
    const int32_t H = F.H;
    const int64_t nint = (int64_t{1} << H) - 1;
    std::vector<uint64_t> tie(n);
    for (int64_t i = 0; i < n; ++i) tie[i] = keyed_draw(F.seed, kStreamTieKey, tree, uint64_t(i));
    // isometry variant: u . x of every point under this tree's reflector
    const double* u = F.U.empty() ? nullptr : F.U.data() + size_t(tree) * d;
    std::vector<double> tdot(u ? n : 0);
    for (int64_t i = 0; i < int64_t(tdot.size()); ++i) tdot[i] = reflector_dot(u, X + i * d, d);
    for (int64_t i = 0; i < n; ++i) ids[i] = uint32_t(i);
    std::vector<Item> items;
    // sizes/offsets of the nodes of the current level
    std::vector<int64_t> size{n}, off{0};
    for (int32_t h = 0; h < H; ++h) {
        std::vector<int64_t> nsize, noff;
        nsize.reserve(size.size() * 2);
        noff.reserve(size.size() * 2);
        for (size_t j = 0; j < size.size(); ++j) {
            const int64_t v = (int64_t{1} << h) - 1 + int64_t(j);
            const int64_t len = size[j], o = off[j];
            const uint64_t r = keyed_draw(F.seed, kStreamSplitDim, tree, uint64_t(v));
            const int32_t slot = int32_t(r % uint64_t(F.t));
            const int32_t s = F.D[slot];
            items.resize(len);
            for (int64_t a = 0; a < len; ++a) {
                uint32_t id = ids[o + a];
                const float xs = X[int64_t(id) * d + s];
                items[a] = Item{u ? reflected(xs, tdot[id], u[s]) : xs, tie[id], id};
            }
            const int64_t nl = len / 2;
            std::nth_element(items.begin(), items.begin() + nl, items.end(), item_less);
            for (int64_t a = 0; a < len; ++a) ids[o + a] = items[a].id;
            const int64_t slotpos = int64_t(tree) * nint + v;
            split_dim[slotpos] = s;
            split_slot[slotpos] = uint8_t(slot);
            split_val[slotpos] = items[nl].x;   // smallest coordinate on the right
            nsize.push_back(nl);
            noff.push_back(o);
            nsize.push_back(len - nl);
            noff.push_back(o + nl);
        }
        size.swap(nsize);
        off.swap(noff);
    }
    for (size_t j = 0; j < size.size(); ++j) std::sort(ids + off[j], ids + off[j] + size[j]);
}


// ---------------------------------------------------------------- split-value jitter
//
// Sec. 2.1 "Split value": a node splits at its median plus delta, delta
// uniform in [-3 Delta / sqrt(d), 3 Delta / sqrt(d)] with Delta the diameter
// of the node's points, drawn at every node; nodes split until they hold at
// most p points.  Readings (the paper leaves them open): the exact Delta is
// the largest pairwise distance, the approximate one the largest distance
// from the node's point of smallest id (between Delta/2 and Delta);
// distances are FP64 sums of squares in index order and one IEEE square
// root; delta = w ((3 Delta) / sqrt(d)), w in [-1, 1) from the top 53 bits of
// keyed_draw(seed, 3, tree, node); the value is float32(median + delta) and
// points with coordinate below it go left; a value that would leave a side
// empty is replaced by the median split of the plain build.
//
// The trees are stored in the perfect layout of depth H = the deepest leaf
// over all trees: a node keeps its heap index, every internal position below
// a leaf passes everything left (value +inf, slot 0), and the leaf's points
// sit in the leftmost leaf below it; the other leaves there are empty.  A
// query descends a pass-through node to the left as well, and the right
// side's gap is infinite, so the queue meets the trees' own leaves in their
// own order and the empty ones last; the budget is capped at the number of
// the trees' own leaves so that those are never opened.

struct JNode {           // a node being split: heap index, depth, id range
    int64_t heap;
    int32_t depth;
    int64_t off, len;
};
struct JSplit { int64_t heap; uint8_t slot; float value; };
struct JLeaf { int64_t heap; int32_t depth; int64_t off, len; };

double node_sq_dist(const float* a, const float* b, int32_t d) {
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        const double e = double(a[j]) - double(b[j]);
        acc = acc + e * e;
    }
    return acc;
}

double node_diameter(const float* X, int32_t d, const uint32_t* ids, int64_t len, bool exact) {
    double far2 = 0.0;
    if (exact) {
        for (int64_t i = 0; i + 1 < len; ++i)
            for (int64_t j = i + 1; j < len; ++j)
                far2 = std::max(far2, node_sq_dist(X + int64_t(ids[i]) * d, X + int64_t(ids[j]) * d, d));
    } else {
        const uint32_t a = *std::min_element(ids, ids + len);
        for (int64_t i = 0; i < len; ++i)
            far2 = std::max(far2, node_sq_dist(X + int64_t(a) * d, X + int64_t(ids[i]) * d, d));
    }
    return std::sqrt(far2);
}

// One tree: splits and leaves, ids reordered in place; returns the deepest
// leaf's depth, or -1 past the depth limit.
int32_t build_tree_jitter(const float* X, int64_t n, int32_t d, const HostForest& F, int32_t tree,
                          bool exact, uint32_t* ids, std::vector<JSplit>& splits,
                          std::vector<JLeaf>& leaves) {
#pragma clang fp contract(off)
    std::vector<uint64_t> tie(n);
    for (int64_t i = 0; i < n; ++i) tie[i] = keyed_draw(F.seed, kStreamTieKey, tree, uint64_t(i));
    for (int64_t i = 0; i < n; ++i) ids[i] = uint32_t(i);
    std::vector<Item> items;
    std::vector<JNode> todo{JNode{0, 0, 0, n}};
    int32_t deepest = 0;
    while (!todo.empty()) {
        const JNode nd = todo.back();
        todo.pop_back();
        uint32_t* seg = ids + nd.off;
        if (nd.len <= F.p) {
            std::sort(seg, seg + nd.len);
            leaves.push_back(JLeaf{nd.heap, nd.depth, nd.off, nd.len});
            deepest = std::max(deepest, nd.depth);
            continue;
        }
        if (nd.depth >= kMaxDepth) return -1;
        const uint64_t r = keyed_draw(F.seed, kStreamSplitDim, tree, uint64_t(nd.heap));
        const int32_t slot = int32_t(r % uint64_t(F.t));
        const int32_t s = F.D[slot];
        items.resize(nd.len);
        for (int64_t a = 0; a < nd.len; ++a) items[a] = Item{X[int64_t(seg[a]) * d + s], tie[seg[a]], seg[a]};
        std::sort(items.begin(), items.end(), item_less);
        const int64_t half = nd.len / 2;
        const float median = items[half].x;
        const double range = (3.0 * node_diameter(X, d, seg, nd.len, exact)) / std::sqrt(double(d));
        const uint64_t rw = keyed_draw(F.seed, kStreamJitter, tree, uint64_t(nd.heap));
        const double w = double(rw >> 11) * 0x1p-53 * 2.0 - 1.0;
        float value = float(double(median) + w * range);
        // items are in coordinate order: those below the value come first
        int64_t nl = std::partition_point(items.begin(), items.end(),
                                          [&](const Item& it) { return it.x < value; }) - items.begin();
        if (nl == 0 || nl == nd.len) {
            value = median;
            nl = half;
        }
        for (int64_t a = 0; a < nd.len; ++a) seg[a] = items[a].id;
        splits.push_back(JSplit{nd.heap, uint8_t(slot), value});
        todo.push_back(JNode{2 * nd.heap + 2, nd.depth + 1, nd.off + nl, nd.len - nl});
        todo.push_back(JNode{2 * nd.heap + 1, nd.depth + 1, nd.off, nl});
    }
    return deepest;
}

std::string build_jitter_forest(const float* X, int64_t n, int32_t d, bool exact, HostForest& F) {
    const int32_t m = F.m;
    F.perm.resize(size_t(m) * n);
    std::vector<std::vector<JSplit>> splits(m);
    std::vector<std::vector<JLeaf>> leaves(m);
    std::vector<int32_t> deep(m, 0);
    const unsigned nw = worker_count(m);
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nw; ++w) {
        th.emplace_back([&, w] {
            for (int32_t tree = int32_t(w); tree < m; tree += int32_t(nw))
                deep[tree] = build_tree_jitter(X, n, d, F, tree, exact, F.perm.data() + size_t(tree) * n,
                                               splits[tree], leaves[tree]);
        });
    }
    for (auto& x : th) x.join();
    int32_t H = 0;
    for (int32_t tree = 0; tree < m; ++tree) {
        if (deep[tree] < 0) return "a jittered tree needs more than 23 levels";
        H = std::max(H, deep[tree]);
    }
    F.H = H;
    const int64_t nint = (int64_t{1} << H) - 1;
    const int64_t nleaf = int64_t{1} << H;
    // pass-through nodes everywhere, then each tree's own splits
    F.split_slot.assign(size_t(m) * nint, 0);
    F.split_val.assign(size_t(m) * nint, std::numeric_limits<float>::infinity());
    F.split_dim.assign(size_t(m) * nint, F.D[0]);
    F.leaf_off.assign(size_t(m) * (nleaf + 1), 0);
    F.real_leaves = 0;
    for (int32_t tree = 0; tree < m; ++tree) {
        for (const JSplit& sp : splits[tree]) {
            const size_t at = size_t(tree) * nint + size_t(sp.heap);
            F.split_slot[at] = sp.slot;
            F.split_val[at] = sp.value;
            F.split_dim[at] = F.D[sp.slot];
        }
        // a leaf of depth h at heap index v sits at layout leaf (v - 2^h + 1) << (H - h);
        // the ids are in leaf order, so an empty layout leaf starts where the next
        // occupied one does
        std::vector<int64_t> start(nleaf, -1);
        for (const JLeaf& lf : leaves[tree])
            start[((lf.heap - ((int64_t{1} << lf.depth) - 1)) << (H - lf.depth))] = lf.off;
        uint32_t* lo = F.leaf_off.data() + size_t(tree) * (nleaf + 1);
        lo[nleaf] = uint32_t(n);
        for (int64_t j = nleaf - 1; j >= 0; --j) lo[j] = start[j] >= 0 ? uint32_t(start[j]) : lo[j + 1];
        F.real_leaves += int64_t(leaves[tree].size());
    }
    return {};
}

}  // namespace

std::string select_dims(const std::vector<double>& V, const std::vector<double>& M, int64_t n,
                        int32_t t, std::vector<int32_t>& D) {
    // the t dimensions of largest variance (lower index first among equal
    // variances), kept in ascending index order
    const int32_t d = int32_t(V.size());
    std::vector<int32_t> order(d);
    for (int32_t j = 0; j < d; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return V[a] > V[b]; });
    if (dims_ambiguous(V, M, order, n, t))
        return "near-tie in D: the t-th and (t+1)-th largest variances are within rounding of "
               "each other (columns " + std::to_string(order[t - 1]) + " and " +
               std::to_string(order[t]) + ")";
    D.assign(order.begin(), order.begin() + t);
    std::sort(D.begin(), D.end());
    return {};
}

void householder_vector(uint64_t seed, int32_t tree, int32_t d, double* u) {
#pragma clang fp contract(off)
    double ss = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        const uint64_t r = keyed_draw(seed, kStreamReflector, uint64_t(tree), uint64_t(j));
        const double w = double(r >> 11) * 0x1p-53 * 2.0 - 1.0;   // exact
        u[j] = w;
        const double sq = w * w;
        ss = ss + sq;
    }
    const double nrm = std::sqrt(ss);
    for (int32_t j = 0; j < d; ++j) u[j] = u[j] / nrm;
}

std::string build_host_forest(const float* X, int64_t n, int32_t d, int32_t m, int32_t t,
                              int32_t p, uint64_t seed, bool householder, HostForest& F, int jitter) {
    F = HostForest{};
    F.n = n; F.d = d; F.m = m; F.t = t; F.p = p; F.seed = seed;
    F.jitter = jitter;
    F.H = perfect_depth(n, p);
    if (!jitter && F.H > 23) return "tree depth above 23 (n/leaf too large)";
    if (householder) {
        F.U.resize(size_t(m) * d);
        for (int32_t tr = 0; tr < m; ++tr) householder_vector(seed, tr, d, F.U.data() + size_t(tr) * d);
    }
    const int64_t nint = (int64_t{1} << F.H) - 1;
    const int64_t nleaf = int64_t{1} << F.H;

    // V <- variances; D <- the t dimensions of largest variance
    std::vector<double> V, M;
    column_variance(X, n, d, V, M);
    std::string err = select_dims(V, M, n, t, F.D);
    if (!err.empty()) return err;
    if (jitter) return build_jitter_forest(X, n, d, jitter == 2, F);

    // Leaf offsets: node sizes split floor/ceil, so they depend on n only.
    std::vector<int64_t> size{n};
    for (int32_t h = 0; h < F.H; ++h) {
        std::vector<int64_t> nx;
        nx.reserve(size.size() * 2);
        for (int64_t s : size) { nx.push_back(s / 2); nx.push_back(s - s / 2); }
        size.swap(nx);
    }
    // the same offsets in every tree
    F.leaf_off.resize(size_t(m) * (nleaf + 1));
    for (int32_t tr = 0; tr < m; ++tr) {
        uint32_t* lo = F.leaf_off.data() + size_t(tr) * (nleaf + 1);
        lo[0] = 0;
        for (int64_t j = 0; j < nleaf; ++j) lo[j + 1] = uint32_t(lo[j] + size[j]);
    }
    F.real_leaves = int64_t(m) * nleaf;

    F.split_dim.assign(size_t(m) * nint, 0);
    F.split_slot.assign(size_t(m) * nint, 0);
    F.split_val.assign(size_t(m) * nint, 0.0f);
    F.perm.resize(size_t(m) * n);
    const unsigned nw = worker_count(m);
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nw; ++w) {
        th.emplace_back([&, w] {
            for (int32_t tree = int32_t(w); tree < m; tree += int32_t(nw))
                build_tree(X, n, d, F, tree, F.split_dim, F.split_slot, F.split_val,
                           F.perm.data() + size_t(tree) * n);
        });
    }
    for (auto& x : th) x.join();
    return {};
}

}  // namespace gf
