/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for the kd-GeRaF
 * build and query (Avrithis, Emiris, Samaras, "High-dimensional approximate
 * nearest neighbor: k-d Generalized Randomized Forests", arXiv 1603.09596).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library: everything below
 * (RNG, variance, split rule, priority queue, distances) is written out here
 * on its own, from the paper and from the fixed readings listed in the design
 * notes.
 *
 * Floating point: FP64 throughout, except the one place the method's result
 * is defined in float32 (the split-plane gap, see gap_f32()).
 *
 * Contents
 *   orc_splitmix64 / orc_draw  counter-based RNG: the published splitmix64
 *                              output function (Steele, Lea, Flood 2014),
 *                              keyed by (seed, stream, tree, index).
 *   orc_variance               per-dimension sample variance, two-pass FP64
 *                              (the plain definition; the paper computes the
 *                              same quantity with Knuth's online update,
 *                              Sec. 3 "Median, variances", Alg. 3).
 *   orc_top_dims               the t dimensions of largest variance (Alg. 1).
 *   orc_depth                  depth of the perfect tree (Sec. 3 "Tree
 *                              structure": trees are perfect).
 *   orc_householder            the per-tree reflector of the isometry variant
 *                              (Sec. 2.1 "Rotation", Sec. 2.2): P = I - 2uu'.
 *   orc_build                  Alg. 1: m trees, split dimension drawn from the
 *                              top-t set, split at the median, per-tree random
 *                              tie key ("shuffling", Sec. 2.1); optionally on
 *                              the reflected coordinates of each tree.
 *   orc_search                 Alg. 2 + Sec. 2.3: one shared min-priority
 *                              queue over all trees, no backtracking, stop
 *                              after B leaves, visited array so no point is
 *                              measured twice, k best by squared distance.
 *   orc_build_jitter           Alg. 1 with the split-value jitter of Sec. 2.1
 *                              ("Split value"): median plus a uniform delta
 *                              scaled by the node's diameter; trees are then
 *                              not perfect and are stored as explicit nodes.
 *   orc_search_jitter          Alg. 2 over those explicit trees.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENEARTIE (-3)   /* D is not determined by the data (see orc_dims_ambiguous) */

/* ------------------------------------------------------------------------ */
/* RNG: splitmix64 output function; stream ids: 1 split dim, 2 tie key.      */
/* ------------------------------------------------------------------------ */

uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_draw(uint64_t seed, uint64_t stream, uint64_t tree, uint64_t idx)
{
    uint64_t h = orc_splitmix64(seed);
    h = orc_splitmix64(h ^ stream);
    h = orc_splitmix64(h ^ tree);
    return orc_splitmix64(h ^ idx);
}

/* ------------------------------------------------------------------------ */
/* Variance and the top-t dimension set D (Alg. 1, first two steps).         */
/* ------------------------------------------------------------------------ */

/* Sample variance of every column, denominator n-1 (Alg. 3 returns v/(n-1));
 * fewer than two points give 0 (Alg. 3, first line).  Two passes: mean, then
 * the sum of squared deviations, each summed in row order in FP64. */
int orc_variance(const float *X, int64_t n, int32_t d, double *V)
{
    if (!X || !V || n < 0 || d < 1) return ORC_EINVAL;
    if (n < 2) {
        for (int32_t j = 0; j < d; ++j) V[j] = 0.0;
        return ORC_OK;
    }
    double *mean = (double *)calloc((size_t)d, sizeof(double));
    if (!mean) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < d; ++j) mean[j] += (double)X[i * d + j];
    for (int32_t j = 0; j < d; ++j) { mean[j] /= (double)n; V[j] = 0.0; }
    for (int64_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < d; ++j) {
            double dev = (double)X[i * d + j] - mean[j];
            V[j] += dev * dev;
        }
    for (int32_t j = 0; j < d; ++j) V[j] /= (double)(n - 1);
    free(mean);
    return ORC_OK;
}

/* The t columns of largest variance; equal variances go to the lower index.
 * Returned sorted by column index, ascending (only the set matters for the
 * method; the ascending order fixes how a random draw maps to a column). */
int orc_top_dims(const double *V, int32_t d, int32_t t, int32_t *D)
{
    if (!V || !D || t < 1 || t > d) return ORC_EINVAL;
    unsigned char *taken = (unsigned char *)calloc((size_t)d, 1);
    if (!taken) return ORC_ENOMEM;
    for (int32_t r = 0; r < t; ++r) {
        int32_t best = -1;
        for (int32_t j = 0; j < d; ++j) {
            if (taken[j]) continue;
            if (best < 0 || V[j] > V[best]) best = j;   /* strict: lower index wins ties */
        }
        taken[best] = 1;
    }
    int32_t w = 0;
    for (int32_t j = 0; j < d; ++j)
        if (taken[j]) D[w++] = j;
    free(taken);
    return ORC_OK;
}

/* Whether D is ill-determined.  The variance is defined exactly but any
 * FP64 evaluation of it is rounded (this file sums two passes; Alg. 3 uses
 * Knuth's online update), and the rounding error scales with the column's
 * mean square, V + mean^2.  When the t-th and (t+1)-th largest variances
 * differ by no more than 1e-12 of the larger mean square of the two columns,
 * two correct evaluations may rank them differently, so the top-t set is
 * not a property of the data: the build refuses such input rather than pick
 * one side silently.  Columns of mean square 0 (all zero) and n < 2 (V = 0
 * by definition) are exact and never ambiguous.  Returns 1 if ambiguous. */
int orc_dims_ambiguous(const float *X, int64_t n, int32_t d, int32_t t, const double *V)
{
    if (!X || !V || t < 1 || t > d) return 0;
    if (n < 2 || t == d) return 0;
    /* the t-th and (t+1)-th largest variances, ties to the lower index */
    unsigned char *taken = (unsigned char *)calloc((size_t)d, 1);
    if (!taken) return 0;
    int32_t rank_t = -1, rank_t1 = -1;
    for (int32_t r = 0; r <= t; ++r) {
        int32_t best = -1;
        for (int32_t j = 0; j < d; ++j) {
            if (taken[j]) continue;
            if (best < 0 || V[j] > V[best]) best = j;
        }
        taken[best] = 1;
        if (r == t - 1) rank_t = best;
        if (r == t) rank_t1 = best;
    }
    free(taken);
    double ms[2] = {0.0, 0.0};
    int32_t cols[2] = {rank_t, rank_t1};
    for (int c = 0; c < 2; ++c) {
        double sum = 0.0;
        for (int64_t i = 0; i < n; ++i) sum += (double)X[i * d + cols[c]];
        double mean = sum / (double)n;
        ms[c] = V[cols[c]] + mean * mean;
    }
    double scale = ms[0] > ms[1] ? ms[0] : ms[1];
    if (!(scale > 0.0)) return 0;
    return (V[rank_t] - V[rank_t1]) <= 1e-12 * scale;
}

/* Perfect-tree depth: the smallest H with ceil(n / 2^H) <= p.  A node of s
 * points splits into floor(s/2) and ceil(s/2), so every node at depth h holds
 * floor(n/2^h) or ceil(n/2^h) points and all leaves (depth H) hold <= p. */
int32_t orc_depth(int64_t n, int32_t p)
{
    if (n < 1 || p < 1) return -1;
    int32_t H = 0;
    for (;;) {
        int64_t pow2 = (int64_t)1 << H;
        int64_t ceil_sz = (n + pow2 - 1) / pow2;
        if (ceil_sz <= p) return H;
        ++H;
    }
}

/* ------------------------------------------------------------------------ */
/* Isometry variant (Sec. 2.1 "Rotation", Sec. 2.2): each tree is built on   */
/* the points reflected by its own Householder matrix P = I - 2uu', and the  */
/* query is reflected the same way before that tree is descended; distances */
/* stay between the original points and query.                              */
/* ------------------------------------------------------------------------ */

/* u of tree `tree`: w_j uniform in [-1, 1) from the top 53 bits of
 * draw(seed, 4, tree, j), then u = w / ||w|| (FP64, the squares summed in
 * index order, IEEE sqrt and division). */
int orc_householder(uint64_t seed, int32_t tree, int32_t d, double *u)
{
    if (!u || d < 1) return ORC_EINVAL;
    double s = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        double w = (double)(orc_draw(seed, 4, (uint64_t)tree, (uint64_t)j) >> 11) * 0x1p-53 * 2.0 - 1.0;
        u[j] = w;
        s = s + w * w;
    }
    if (!(s > 0.0)) return ORC_EINVAL;
    double nrm = sqrt(s);
    for (int32_t j = 0; j < d; ++j) u[j] = u[j] / nrm;
    return ORC_OK;
}

/* u . x in FP64: each product rounded, then added in index order. */
static double dot_u(const double *u, const float *x, int32_t d)
{
    double t = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        double p = u[j] * (double)x[j];
        t = t + p;
    }
    return t;
}

/* Coordinate s of Px = x - 2 (u.x) u given t = u.x: the FP64 value
 * x_s - (2t) u_s, rounded once to float32. */
static float reflect_coord(float x_s, double t, double u_s)
{
    double r = (2.0 * t) * u_s;
    return (float)((double)x_s - r);
}

/* ------------------------------------------------------------------------ */
/* Build (Alg. 1).                                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    float x;        /* coordinate in the split dimension */
    uint64_t key;   /* per-tree random tie key ("shuffling") */
    uint32_t id;
} orc_item;

static int cmp_item(const void *pa, const void *pb)
{
    const orc_item *a = (const orc_item *)pa, *b = (const orc_item *)pb;
    if (a->x < b->x) return -1;     /* float compare: -0 equals +0 */
    if (a->x > b->x) return 1;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->id < b->id) ? -1 : (a->id > b->id);
}

static int cmp_u32(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    return (a < b) ? -1 : (a > b);
}

typedef struct {
    const float *X; int64_t n; int32_t d; int32_t t; int32_t H;
    uint64_t seed; const int32_t *D;
    int32_t *split_dim; float *split_val; uint32_t *perm; uint32_t *leaf_off;
    uint64_t *tiekey;     /* n entries, scratch for one tree */
    orc_item *items;      /* n entries, scratch for one tree */
    int32_t tree;
    const double *U;      /* [m][d] reflectors, or NULL (no isometry) */
    double *tdot;         /* n entries: u . x of every point, for one tree */
} orc_build_ctx;

/* Recursive build of node v (heap index, root 0) at the given depth, whose
 * points are ids[0 .. len).  The points are reordered in place so that the
 * left child gets the first floor(len/2) of them. */
static void build_node(orc_build_ctx *c, int64_t v, int32_t depth,
                       uint32_t *ids, int64_t len, int64_t offset)
{
    const int64_t n_internal = ((int64_t)1 << c->H) - 1;
    if (depth == c->H) {                                     /* leaf(X) */
        int64_t leaf = v - n_internal;
        qsort(ids, (size_t)len, sizeof(uint32_t), cmp_u32);  /* ids ascending */
        if (c->tree == 0) c->leaf_off[leaf] = (uint32_t)offset;
        return;
    }
    /* s <- one of the dimensions D at random */
    int32_t s = c->D[orc_draw(c->seed, 1, (uint64_t)c->tree, (uint64_t)v) % (uint64_t)c->t];
    /* v <- median of X in dimension s: rank split at floor(len/2), ties
     * resolved by the tree's random key, then by id. */
    for (int64_t i = 0; i < len; ++i) {
        const float xs = c->X[(int64_t)ids[i] * c->d + s];
        c->items[i].x = c->U ? reflect_coord(xs, c->tdot[ids[i]], c->U[(int64_t)c->tree * c->d + s])
                             : xs;
        c->items[i].key = c->tiekey[ids[i]];
        c->items[i].id = ids[i];
    }
    qsort(c->items, (size_t)len, sizeof(orc_item), cmp_item);
    for (int64_t i = 0; i < len; ++i) ids[i] = c->items[i].id;
    int64_t nl = len / 2;
    float value = c->items[nl].x;        /* smallest coordinate on the right */
    int64_t node_slot = (int64_t)c->tree * n_internal + v;
    c->split_dim[node_slot] = s;
    c->split_val[node_slot] = value;
    build_node(c, 2 * v + 1, depth + 1, ids, nl, offset);
    build_node(c, 2 * v + 2, depth + 1, ids + nl, len - nl, offset + nl);
}

typedef struct {
    orc_build_ctx base;
    int32_t first_tree, tree_step, m;
    int status;
} orc_build_job;

static void *build_worker(void *arg)
{
    orc_build_job *job = (orc_build_job *)arg;
    orc_build_ctx c = job->base;
    c.tiekey = (uint64_t *)malloc((size_t)c.n * sizeof(uint64_t));
    c.items = (orc_item *)malloc((size_t)c.n * sizeof(orc_item));
    c.tdot = c.U ? (double *)malloc((size_t)c.n * sizeof(double)) : NULL;
    if (!c.tiekey || !c.items || (c.U && !c.tdot)) { job->status = ORC_ENOMEM; goto done; }
    for (int32_t tr = job->first_tree; tr < job->m; tr += job->tree_step) {
        c.tree = tr;
        if (c.U)
            for (int64_t i = 0; i < c.n; ++i)
                c.tdot[i] = dot_u(c.U + (int64_t)tr * c.d, c.X + i * c.d, c.d);
        for (int64_t i = 0; i < c.n; ++i)
            c.tiekey[i] = orc_draw(c.seed, 2, (uint64_t)tr, (uint64_t)i);
        uint32_t *ids = c.perm + (int64_t)tr * c.n;
        for (int64_t i = 0; i < c.n; ++i) ids[i] = (uint32_t)i;
        build_node(&c, 0, 0, ids, c.n, 0);
    }
    job->status = ORC_OK;
done:
    free(c.tiekey);
    free(c.items);
    free(c.tdot);
    return NULL;
}

/* Alg. 1.  Outputs (caller-allocated):
 *   D[t]                          the top-variance dimensions, ascending
 *   split_dim[m][2^H - 1]         column index of every internal node
 *   split_val[m][2^H - 1]         split value of every internal node
 *   perm[m][n]                    per tree, the point ids of leaf 0, leaf 1, ...
 *                                 (each leaf ascending by id)
 *   leaf_off[2^H + 1]             leaf j holds perm[tree][leaf_off[j] .. leaf_off[j+1])
 *                                 (identical for every tree: sizes depend on n only)
 * Internal node v has children 2v+1 (left) and 2v+2 (right).  U = NULL
 * builds on the points themselves, as the paper runs it (Sec. 4); otherwise
 * U[m][d] holds each tree's reflector u (orc_householder) and tree i splits
 * the coordinates of P_i x, rounded to float32, while D stays the top-variance
 * set of X itself.  Split-value jitter (Sec. 2.1) is not built. */
int orc_build(const float *X, int64_t n, int32_t d, int32_t m, int32_t t,
              int32_t p, uint64_t seed, int32_t nthreads,
              int32_t *D, int32_t *split_dim, float *split_val,
              uint32_t *perm, uint32_t *leaf_off, const double *U)
{
    if (!X || n < 1 || n > 0xFFFFFFFFLL || d < 1 || m < 1 || t < 1 || t > d || p < 1)
        return ORC_EINVAL;
    int32_t H = orc_depth(n, p);
    double *V = (double *)malloc((size_t)d * sizeof(double));
    if (!V) return ORC_ENOMEM;
    int st = orc_variance(X, n, d, V);
    if (st == ORC_OK && orc_dims_ambiguous(X, n, d, t, V)) st = ORC_ENEARTIE;
    if (st == ORC_OK) st = orc_top_dims(V, d, t, D);
    free(V);
    if (st != ORC_OK) return st;
    leaf_off[(int64_t)1 << H] = (uint32_t)n;

    if (nthreads < 1) nthreads = 1;
    if (nthreads > m) nthreads = m;
    orc_build_job *jobs = (orc_build_job *)calloc((size_t)nthreads, sizeof(orc_build_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return ORC_ENOMEM; }
    for (int32_t w = 0; w < nthreads; ++w) {
        orc_build_ctx b = {X, n, d, t, H, seed, D, split_dim, split_val, perm, leaf_off,
                           NULL, NULL, 0, U, NULL};
        jobs[w].base = b;
        jobs[w].first_tree = w;
        jobs[w].tree_step = nthreads;
        jobs[w].m = m;
        pthread_create(&th[w], NULL, build_worker, &jobs[w]);
    }
    for (int32_t w = 0; w < nthreads; ++w) {
        pthread_join(th[w], NULL);
        if (jobs[w].status != ORC_OK) st = jobs[w].status;
    }
    free(jobs);
    free(th);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Search (Alg. 2, Sec. 2.3).                                                */
/* ------------------------------------------------------------------------ */

/* The signed gap of Eq. (1), f(q)_s - v with f the identity.  Query and split
 * value are float32, and the gap is defined as their float32 difference.  It
 * is formed here as the FP64 difference rounded once to float32, which equals
 * the IEEE float32 subtraction (53 >= 2*24 + 2, so the double rounding is
 * innocuous), then widened back: FP64 comparisons of these keys are exact. */
static double gap_f32(float q_s, float v)
{
    return (double)(float)((double)q_s - (double)v);
}

/* Leaves to check: the loop of Alg. 2 runs while l < c/(1+eps), i.e.
 * ceil(c/(1+eps)) times, and never more than the forest has leaves. */
int64_t orc_budget(int64_t c, double eps, int64_t total_leaves)
{
    double b = ceil((double)c / (1.0 + eps));
    int64_t B = (int64_t)b;
    if (B > total_leaves) B = total_leaves;
    if (B < 0) B = 0;
    return B;
}

/* node: heap index (the tie order); idx: the node's own index in an
 * explicit tree (the jittered trees below), unused for perfect trees. */
typedef struct { double key; int32_t tree; int32_t node; int32_t idx; } orc_entry;

static int entry_less(const orc_entry *a, const orc_entry *b)
{
    if (a->key != b->key) return a->key < b->key;
    if (a->tree != b->tree) return a->tree < b->tree;
    return a->node < b->node;
}

typedef struct { orc_entry *a; int64_t size, cap; } orc_heap;

static int heap_push(orc_heap *h, orc_entry e)
{
    if (h->size == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        orc_entry *na = (orc_entry *)realloc(h->a, (size_t)nc * sizeof(orc_entry));
        if (!na) return ORC_ENOMEM;
        h->a = na; h->cap = nc;
    }
    int64_t i = h->size++;
    h->a[i] = e;
    while (i > 0) {
        int64_t par = (i - 1) / 2;
        if (!entry_less(&h->a[i], &h->a[par])) break;
        orc_entry tmp = h->a[i]; h->a[i] = h->a[par]; h->a[par] = tmp;
        i = par;
    }
    return ORC_OK;
}

static orc_entry heap_pop(orc_heap *h)
{
    orc_entry top = h->a[0];
    h->a[0] = h->a[--h->size];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < h->size && entry_less(&h->a[l], &h->a[s])) s = l;
        if (r < h->size && entry_less(&h->a[r], &h->a[s])) s = r;
        if (s == i) break;
        orc_entry tmp = h->a[i]; h->a[i] = h->a[s]; h->a[s] = tmp;
        i = s;
    }
    return top;
}

typedef struct { double dist; uint32_t id; } orc_cand;

static int cmp_cand(const void *pa, const void *pb)
{
    const orc_cand *a = (const orc_cand *)pa, *b = (const orc_cand *)pb;
    if (a->dist < b->dist) return -1;
    if (a->dist > b->dist) return 1;
    return (a->id < b->id) ? -1 : (a->id > b->id);
}

typedef struct {
    /* forest */
    const float *X; int64_t n; int32_t d; int32_t m; int32_t H;
    const int32_t *split_dim; const float *split_val;
    const uint32_t *perm; const uint32_t *leaf_off;
    /* queries */
    const float *Q; int64_t nq; int32_t k; int64_t B; int32_t eff_key;
    /* outputs */
    int32_t *ids; double *dists;
    uint32_t *opened; double *opened_key;
    int64_t *ncand; uint32_t *cand; int64_t cand_cap;
    /* threading */
    int64_t q_first, q_step;
    int status;
    const double *U;      /* [m][d] reflectors of the isometry variant, or NULL */
} orc_search_job;

/* One query through Alg. 2.  Queue entries are (key, tree, node) triples
 * ordered lexicographically (key as FP64, then tree, then heap index): a
 * deterministic total order, so ties resolve the same way every run.
 *
 * Readings of the paper taken here:
 *   - every tree's root enters the queue with key 0, so the first m pops
 *     descend each tree once and check its home leaf ("all visited nodes
 *     are stored in Q"); every checked leaf counts against the budget;
 *   - the key of a pushed child is |gap| at the node where it was left
 *     behind (Alg. 2 inserts the far child with the absolute signed
 *     distance of Eq. 1; Sec. 2.3).  With eff_key != 0 it is instead
 *     max(key of the entry being descended, |gap|), a variant kept only as
 *     a diagnostic: it opens the same leaves except where keys tie;
 *   - gap < 0 descends left and stores the right child; gap >= 0 (including
 *     a zero gap) descends right and stores the left child;
 *   - distances are squared Euclidean, summed in FP64;
 *   - the k best are the k smallest (distance, id) pairs, ascending, padded
 *     with id -1 / +inf when fewer than k points were checked. */
static int search_one(const orc_search_job *J, int64_t qi, unsigned char *visited,
                      uint32_t *touched, orc_cand *cands, orc_heap *heap, double *tq)
{
    const float *q = J->Q + qi * J->d;
    const int64_t n_internal = ((int64_t)1 << J->H) - 1;
    int64_t ntouched = 0;
    if (J->U)   /* u_i . q per tree: the query is reflected before descending tree i */
        for (int32_t tr = 0; tr < J->m; ++tr) tq[tr] = dot_u(J->U + (int64_t)tr * J->d, q, J->d);
    heap->size = 0;
    for (int32_t tr = 0; tr < J->m; ++tr) {
        orc_entry root = {0.0, tr, 0, 0};
        if (heap_push(heap, root) != ORC_OK) return ORC_ENOMEM;
    }
    int64_t checked = 0;
    while (checked < J->B && heap->size > 0) {
        orc_entry e = heap_pop(heap);
        int64_t v = e.node;
        const int32_t *sd = J->split_dim + (int64_t)e.tree * n_internal;
        const float *sv = J->split_val + (int64_t)e.tree * n_internal;
        while (v < n_internal) {                         /* descend(q, N, check) */
            const int32_t s = sd[v];
            const float qs = J->U ? reflect_coord(q[s], tq[e.tree], J->U[(int64_t)e.tree * J->d + s])
                                  : q[s];
            double g = gap_f32(qs, sv[v]);
            int64_t near_child, far_child;
            if (g < 0.0) { near_child = 2 * v + 1; far_child = 2 * v + 2; }
            else         { near_child = 2 * v + 2; far_child = 2 * v + 1; }
            double ag = fabs(g);
            orc_entry child;
            child.key = J->eff_key ? (ag > e.key ? ag : e.key) : ag;
            child.tree = e.tree;
            child.node = (int32_t)far_child;
            if (heap_push(heap, child) != ORC_OK) return ORC_ENOMEM;
            v = near_child;
        }
        int64_t leaf = v - n_internal;
        if (J->opened) J->opened[qi * J->B + checked] = ((uint32_t)e.tree << 24) | (uint32_t)leaf;
        if (J->opened_key) J->opened_key[qi * J->B + checked] = e.key;
        const uint32_t *pts = J->perm + (int64_t)e.tree * J->n;
        for (uint32_t a = J->leaf_off[leaf]; a < J->leaf_off[leaf + 1]; ++a) {
            uint32_t id = pts[a];
            if (visited[id]) continue;               /* never measure a point twice */
            visited[id] = 1;
            const float *x = J->X + (int64_t)id * J->d;
            double acc = 0.0;
            for (int32_t j = 0; j < J->d; ++j) {
                double diff = (double)q[j] - (double)x[j];
                acc += diff * diff;
            }
            cands[ntouched].dist = acc;
            cands[ntouched].id = id;
            touched[ntouched++] = id;
        }
        ++checked;
    }
    /* the k best, ascending by (distance, id) */
    if (J->ncand) J->ncand[qi] = ntouched;
    if (J->cand) {
        int64_t w = ntouched < J->cand_cap ? ntouched : J->cand_cap;
        uint32_t *dst = J->cand + qi * J->cand_cap;
        for (int64_t a = 0; a < w; ++a) dst[a] = touched[a];
        qsort(dst, (size_t)w, sizeof(uint32_t), cmp_u32);
    }
    qsort(cands, (size_t)ntouched, sizeof(orc_cand), cmp_cand);
    for (int32_t r = 0; r < J->k; ++r) {
        if (r < ntouched) {
            J->ids[qi * J->k + r] = (int32_t)cands[r].id;
            J->dists[qi * J->k + r] = cands[r].dist;
        } else {
            J->ids[qi * J->k + r] = -1;
            J->dists[qi * J->k + r] = INFINITY;
        }
    }
    for (int64_t a = 0; a < ntouched; ++a) visited[touched[a]] = 0;
    return ORC_OK;
}

static void *search_worker(void *arg)
{
    orc_search_job *J = (orc_search_job *)arg;
    int64_t max_pts = 0;
    for (int64_t j = 0; j < ((int64_t)1 << J->H); ++j) {
        int64_t sz = (int64_t)J->leaf_off[j + 1] - (int64_t)J->leaf_off[j];
        if (sz > max_pts) max_pts = sz;
    }
    int64_t cap = J->B * max_pts;
    if (cap > J->n) cap = J->n;
    unsigned char *visited = (unsigned char *)calloc((size_t)J->n, 1);
    uint32_t *touched = (uint32_t *)malloc((size_t)(cap + 1) * sizeof(uint32_t));
    orc_cand *cands = (orc_cand *)malloc((size_t)(cap + 1) * sizeof(orc_cand));
    orc_heap heap = {NULL, 0, 0};
    double *tq = (double *)malloc((size_t)J->m * sizeof(double));
    J->status = ORC_OK;
    if (!visited || !touched || !cands || !tq) J->status = ORC_ENOMEM;
    for (int64_t qi = J->q_first; J->status == ORC_OK && qi < J->nq; qi += J->q_step)
        J->status = search_one(J, qi, visited, touched, cands, &heap, tq);
    free(visited); free(touched); free(cands); free(heap.a); free(tq);
    return NULL;
}

/* Alg. 2 for nq queries (threads split the queries; each query is searched
 * sequentially, as in the paper).  Outputs (caller-allocated):
 *   ids[nq][k] int32, dists[nq][k] FP64 squared distances;
 *   opened[nq][B] (tree << 24 | leaf) in pop order and opened_key[nq][B]
 *   (may be NULL); ncand[nq] and cand[nq][cand_cap] = the checked point ids,
 *   ascending (may be NULL).  B = orc_budget(c, eps, m * 2^H).  U: the
 *   forest's reflectors (orc_build) or NULL. */
int orc_search(const float *X, int64_t n, int32_t d, int32_t m, int32_t H,
               const int32_t *split_dim, const float *split_val,
               const uint32_t *perm, const uint32_t *leaf_off,
               const float *Q, int64_t nq, int32_t k, int64_t c, double eps,
               int32_t eff_key, int32_t nthreads,
               int32_t *ids, double *dists, uint32_t *opened, double *opened_key,
               int64_t *ncand, uint32_t *cand, int64_t cand_cap, const double *U)
{
    if (!X || !Q || !ids || !dists || n < 1 || d < 1 || m < 1 || H < 0 || H > 23 ||
        m > 255 || nq < 0 || k < 1 || c < 0 || !(eps >= 0.0))
        return ORC_EINVAL;
    int64_t B = orc_budget(c, eps, (int64_t)m << H);
    if (nthreads < 1) nthreads = 1;
    if (nq < nthreads) nthreads = nq > 0 ? (int32_t)nq : 1;
    orc_search_job *jobs = (orc_search_job *)calloc((size_t)nthreads, sizeof(orc_search_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) { free(jobs); free(th); return ORC_ENOMEM; }
    int st = ORC_OK;
    for (int32_t w = 0; w < nthreads; ++w) {
        orc_search_job J = {X, n, d, m, H, split_dim, split_val, perm, leaf_off,
                            Q, nq, k, B, eff_key, ids, dists, opened, opened_key,
                            ncand, cand, cand_cap, w, nthreads, ORC_OK, U};
        jobs[w] = J;
        pthread_create(&th[w], NULL, search_worker, &jobs[w]);
    }
    for (int32_t w = 0; w < nthreads; ++w) {
        pthread_join(th[w], NULL);
        if (jobs[w].status != ORC_OK) st = jobs[w].status;
    }
    free(jobs);
    free(th);
    return st;
}


/* ------------------------------------------------------------------------ */
/* Split-value jitter (Sec. 2.1 "Split value"): a node's split value is its  */
/* median plus delta, delta uniform in [-3 Delta/sqrt(d), 3 Delta/sqrt(d)],   */
/* Delta the diameter of the node's point set, drawn at every node.  Nodes   */
/* then split unevenly, so the recursion of Alg. 1 stops where a node holds  */
/* at most p points, at whatever depth.                                      */
/*                                                                          */
/* Readings taken here (the paper leaves them open):                        */
/*   - the exact diameter is the largest pairwise distance; the approximate */
/*     one is the largest distance from the node's point of smallest id,    */
/*     which lies between half the diameter and the diameter;               */
/*   - distances are Euclidean, squares summed in FP64 in index order, then */
/*     the IEEE square root of the largest;                                 */
/*   - delta = w * ((3 Delta) / sqrt(d)) with w uniform in [-1, 1) from the  */
/*     top 53 bits of draw(seed, 3, tree, node), node the heap index;       */
/*   - the split value is (float)(median + delta), the median being the      */
/*     coordinate of the item of rank floor(|P|/2) under (coordinate, tie   */
/*     key, id) as in the plain build; points with coordinate < value go    */
/*     left, the rest right (the side a query with that coordinate takes);  */
/*   - when that leaves a side empty, the node splits at the median as in   */
/*     the plain build (left = the floor(|P|/2) first items, value = the    */
/*     median), so every split makes progress;                              */
/*   - a node of at most p points is a leaf; depth above 23 is refused.     */
/* ------------------------------------------------------------------------ */

#define ORC_EDEPTH (-4)
#define ORC_MAXDEPTH 23

static double sqdist_pts(const float *X, int32_t d, uint32_t a, uint32_t b)
{
    const float *x = X + (int64_t)a * d, *y = X + (int64_t)b * d;
    double acc = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        double diff = (double)x[j] - (double)y[j];
        acc = acc + diff * diff;
    }
    return acc;
}

static double node_diameter(const float *X, int32_t d, const uint32_t *ids, int64_t len, int exact)
{
    double best = 0.0;
    if (exact) {
        for (int64_t i = 0; i < len; ++i)
            for (int64_t j = i + 1; j < len; ++j) {
                double s2 = sqdist_pts(X, d, ids[i], ids[j]);
                if (s2 > best) best = s2;
            }
    } else {
        uint32_t anchor = ids[0];
        for (int64_t i = 1; i < len; ++i)
            if (ids[i] < anchor) anchor = ids[i];
        for (int64_t i = 0; i < len; ++i) {
            double s2 = sqdist_pts(X, d, anchor, ids[i]);
            if (s2 > best) best = s2;
        }
    }
    return sqrt(best);
}

/* Explicit trees: node i of tree tr at [tr * ncap + i]; root 0; dim -1 marks
 * a leaf holding perm[tr][off .. off + len) (ascending ids). */
typedef struct {
    const float *X; int64_t n; int32_t d; int32_t t; int32_t p; int32_t exact;
    uint64_t seed; const int32_t *D; int32_t tree; int64_t ncap;
    int32_t *dim; float *val; int32_t *left; int32_t *right; int32_t *heap;
    int32_t *depth; uint32_t *off; uint32_t *len;
    uint32_t *perm;
    orc_item *items; uint64_t *tiekey;
    int64_t nnodes; int32_t maxdepth; int status;
} orc_jctx;

static int32_t jitter_node(orc_jctx *c, int64_t hv, int32_t dep, uint32_t *ids, int64_t len, int64_t offset)
{
    int64_t me = c->nnodes++;
    int64_t at = (int64_t)c->tree * c->ncap + me;
    c->heap[at] = (int32_t)hv;
    c->depth[at] = dep;
    if (dep > c->maxdepth) c->maxdepth = dep;
    if (len <= c->p) {                                       /* leaf(X) */
        qsort(ids, (size_t)len, sizeof(uint32_t), cmp_u32);
        c->dim[at] = -1; c->val[at] = 0.0f; c->left[at] = -1; c->right[at] = -1;
        c->off[at] = (uint32_t)offset; c->len[at] = (uint32_t)len;
        return (int32_t)me;
    }
    if (dep >= ORC_MAXDEPTH) { c->status = ORC_EDEPTH; return (int32_t)me; }
    int32_t s = c->D[orc_draw(c->seed, 1, (uint64_t)c->tree, (uint64_t)hv) % (uint64_t)c->t];
    for (int64_t i = 0; i < len; ++i) {
        c->items[i].x = c->X[(int64_t)ids[i] * c->d + s];
        c->items[i].key = c->tiekey[ids[i]];
        c->items[i].id = ids[i];
    }
    qsort(c->items, (size_t)len, sizeof(orc_item), cmp_item);
    int64_t half = len / 2;
    float median = c->items[half].x;
    double delta_range = (3.0 * node_diameter(c->X, c->d, ids, len, c->exact)) / sqrt((double)c->d);
    double w = (double)(orc_draw(c->seed, 3, (uint64_t)c->tree, (uint64_t)hv) >> 11) * 0x1p-53 * 2.0 - 1.0;
    float value = (float)((double)median + w * delta_range);
    int64_t nl = 0;
    for (int64_t i = 0; i < len; ++i) nl += (c->items[i].x < value);
    if (nl == 0 || nl == len) {            /* an empty side: the plain median split */
        value = median;
        nl = half;
    }
    /* the items are sorted by coordinate, so the first nl are those below value */
    for (int64_t i = 0; i < len; ++i) ids[i] = c->items[i].id;
    c->dim[at] = s;
    c->val[at] = value;
    c->off[at] = 0; c->len[at] = 0;
    int32_t l = jitter_node(c, 2 * hv + 1, dep + 1, ids, nl, offset);
    int32_t r = jitter_node(c, 2 * hv + 2, dep + 1, ids + nl, len - nl, offset + nl);
    c->left[at] = l;
    c->right[at] = r;
    return (int32_t)me;
}

/* Alg. 1 with split-value jitter.  Outputs (caller-allocated, ncap >= 2n - 1
 * nodes per tree):
 *   D[t]; for every tree tr and node i < nnodes[tr], at [tr * ncap + i]:
 *   dim (-1 for a leaf), val, left, right (explicit node indices), heap (the
 *   node's heap index: root 0, children 2h+1 and 2h+2), depth, and for a
 *   leaf its range off/len in perm[tr]; *H = the largest leaf depth.
 * exact: 1 exact diameter, 0 approximate (see the readings above).
 * Returns ORC_EDEPTH when a tree would need more than 23 levels. */
int orc_build_jitter(const float *X, int64_t n, int32_t d, int32_t m, int32_t t,
                     int32_t p, uint64_t seed, int32_t exact, int64_t ncap,
                     int32_t *D, int32_t *dim, float *val, int32_t *left, int32_t *right,
                     int32_t *heap, int32_t *depth, uint32_t *off, uint32_t *len,
                     uint32_t *perm, int64_t *nnodes, int32_t *H)
{
    if (!X || n < 1 || n > 0xFFFFFFFFLL || d < 1 || m < 1 || t < 1 || t > d || p < 1 ||
        ncap < 2 * n - 1)
        return ORC_EINVAL;
    double *V = (double *)malloc((size_t)d * sizeof(double));
    if (!V) return ORC_ENOMEM;
    int st = orc_variance(X, n, d, V);
    if (st == ORC_OK && orc_dims_ambiguous(X, n, d, t, V)) st = ORC_ENEARTIE;
    if (st == ORC_OK) st = orc_top_dims(V, d, t, D);
    free(V);
    if (st != ORC_OK) return st;
    orc_jctx c;
    memset(&c, 0, sizeof(c));
    c.X = X; c.n = n; c.d = d; c.t = t; c.p = p; c.exact = exact; c.seed = seed; c.D = D;
    c.ncap = ncap; c.dim = dim; c.val = val; c.left = left; c.right = right; c.heap = heap;
    c.depth = depth; c.off = off; c.len = len; c.perm = perm;
    c.items = (orc_item *)malloc((size_t)n * sizeof(orc_item));
    c.tiekey = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    if (!c.items || !c.tiekey) { free(c.items); free(c.tiekey); return ORC_ENOMEM; }
    *H = 0;
    for (int32_t tr = 0; tr < m && c.status == ORC_OK; ++tr) {
        c.tree = tr;
        c.nnodes = 0;
        c.maxdepth = 0;
        for (int64_t i = 0; i < n; ++i) c.tiekey[i] = orc_draw(seed, 2, (uint64_t)tr, (uint64_t)i);
        uint32_t *ids = perm + (int64_t)tr * n;
        for (int64_t i = 0; i < n; ++i) ids[i] = (uint32_t)i;
        jitter_node(&c, 0, 0, ids, n, 0);
        nnodes[tr] = c.nnodes;
        if (c.maxdepth > *H) *H = c.maxdepth;
    }
    free(c.items);
    free(c.tiekey);
    return c.status;
}

/* Alg. 2 over the explicit trees of orc_build_jitter: the same queue, keys
 * and tie order (key, tree, heap index) as orc_search.  Opened leaves are
 * reported as (tree << 24 | j << (H - depth)), j = heap - (2^depth - 1): a
 * leaf's position at depth H when every leaf above depth H is put in place
 * of the leftmost leaf below it.  B = orc_budget(c, eps, leaves of all the
 * trees); ids/dists/opened/opened_key/ncand/cand as in orc_search. */
int orc_search_jitter(const float *X, int64_t n, int32_t d, int32_t m, int32_t H, int64_t ncap,
                      const int32_t *dim, const float *val, const int32_t *left,
                      const int32_t *right, const int32_t *heap, const int32_t *depth,
                      const uint32_t *off, const uint32_t *len, const uint32_t *perm,
                      const int64_t *nnodes,
                      const float *Q, int64_t nq, int32_t k, int64_t c, double eps,
                      int32_t *ids, double *dists, uint32_t *opened, double *opened_key,
                      int64_t *ncand, uint32_t *cand, int64_t cand_cap)
{
    if (!X || !Q || !ids || !dists || n < 1 || d < 1 || m < 1 || m > 255 || H < 0 ||
        H > ORC_MAXDEPTH || nq < 0 || k < 1 || c < 0 || !(eps >= 0.0))
        return ORC_EINVAL;
    int64_t leaves = 0;
    for (int32_t tr = 0; tr < m; ++tr)
        for (int64_t i = 0; i < nnodes[tr]; ++i) leaves += (dim[(int64_t)tr * ncap + i] < 0);
    int64_t B = orc_budget(c, eps, leaves);
    unsigned char *visited = (unsigned char *)calloc((size_t)n, 1);
    orc_cand *cands = (orc_cand *)malloc((size_t)n * sizeof(orc_cand));
    uint32_t *touched = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    orc_heap hq = {NULL, 0, 0};
    int st = (visited && cands && touched) ? ORC_OK : ORC_ENOMEM;
    for (int64_t qi = 0; st == ORC_OK && qi < nq; ++qi) {
        const float *q = Q + qi * d;
        int64_t ntouched = 0, checked = 0;
        hq.size = 0;
        for (int32_t tr = 0; tr < m && st == ORC_OK; ++tr) {
            orc_entry root = {0.0, tr, 0, 0};
            st = heap_push(&hq, root);
        }
        while (st == ORC_OK && checked < B && hq.size > 0) {
            orc_entry e = heap_pop(&hq);
            int64_t base = (int64_t)e.tree * ncap;
            int32_t i = e.idx;
            while (dim[base + i] >= 0) {                      /* descend */
                double g = gap_f32(q[dim[base + i]], val[base + i]);
                int32_t near_i = g < 0.0 ? left[base + i] : right[base + i];
                int32_t far_i = g < 0.0 ? right[base + i] : left[base + i];
                orc_entry child = {fabs(g), e.tree, heap[base + far_i], far_i};
                if ((st = heap_push(&hq, child)) != ORC_OK) break;
                i = near_i;
            }
            if (st != ORC_OK) break;
            int64_t dl = depth[base + i];
            uint32_t j = (uint32_t)((int64_t)heap[base + i] - (((int64_t)1 << dl) - 1));
            if (opened) opened[qi * B + checked] = ((uint32_t)e.tree << 24) | (j << (H - dl));
            if (opened_key) opened_key[qi * B + checked] = e.key;
            const uint32_t *pts = perm + (int64_t)e.tree * n;
            for (uint32_t a = off[base + i]; a < off[base + i] + len[base + i]; ++a) {
                uint32_t id = pts[a];
                if (visited[id]) continue;
                visited[id] = 1;
                const float *x = X + (int64_t)id * d;
                double acc = 0.0;
                for (int32_t jj = 0; jj < d; ++jj) {
                    double diff = (double)q[jj] - (double)x[jj];
                    acc += diff * diff;
                }
                cands[ntouched].dist = acc;
                cands[ntouched].id = id;
                touched[ntouched++] = id;
            }
            ++checked;
        }
        if (st != ORC_OK) break;
        if (ncand) ncand[qi] = ntouched;
        if (cand) {
            int64_t w = ntouched < cand_cap ? ntouched : cand_cap;
            uint32_t *dst = cand + qi * cand_cap;
            for (int64_t a = 0; a < w; ++a) dst[a] = touched[a];
            qsort(dst, (size_t)w, sizeof(uint32_t), cmp_u32);
        }
        qsort(cands, (size_t)ntouched, sizeof(orc_cand), cmp_cand);
        for (int32_t r = 0; r < k; ++r) {
            ids[qi * k + r] = r < ntouched ? (int32_t)cands[r].id : -1;
            dists[qi * k + r] = r < ntouched ? cands[r].dist : INFINITY;
        }
        for (int64_t a = 0; a < ntouched; ++a) visited[touched[a]] = 0;
    }
    free(visited); free(cands); free(touched); free(hq.a);
    return st;
}
