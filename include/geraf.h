/*
 * geraf.h -- C ABI of the kd-GeRaF query-path library for MI355X (gfx950).
 *
 * Method: Avrithis, Emiris, Samaras, "High-dimensional approximate nearest
 * neighbor: k-d Generalized Randomized Forests" (arXiv 1603.09596).
 *   - gf_build_forest follows Alg. 1 (Sec. 2.2) with the storage of Sec. 3
 *     ("Tree structure": perfect trees stored in arrays, points stored once)
 *     and the variance of Alg. 3.
 *   - gf_query follows Alg. 2 and Sec. 2.3 (one priority queue shared by all
 *     trees, keyed by the gap of Eq. 1, no backtracking, stop after
 *     ceil(c/(1+eps)) leaves, a visited array so no distance is computed
 *     twice, the k best by squared distance), plus the squared-norm
 *     expansion of Sec. 3 ("Distance computation") for the reduced-precision
 *     forms.
 *
 * Conventions shared by every entry point
 *   - Every function returns a gf_status; nothing throws across the ABI.  On
 *     error no output has been written and gf_last_error() (thread-local)
 *     describes the failure.  Arguments are validated before any HIP call.
 *   - Matrices are row-major float32: X is [n][d], Q is [nq][d].
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Query entry points enqueue their kernels on it and return once the
 *     results are in the caller's buffers (they synchronise the stream).
 *   - Host threads may call concurrently.  Calls on one forest share its
 *     workspace and wait for each other (a lock per forest); calls on
 *     different forests run side by side.  gf_free_forest must not overlap
 *     a call on the same forest.
 *   - Pointers marked host-or-device may point to either; the library checks
 *     with hipPointerGetAttributes and stages host buffers itself.
 *   - Distances are SQUARED Euclidean distances.  Result rows are sorted by
 *     (distance, id) ascending; missing slots (fewer than k candidates) hold
 *     id -1 and distance +inf.
 *   - Limits: 1 <= m <= 255 trees, perfect-tree depth H <= 23, n < 2^31,
 *     1 <= t <= min(d, 64), 1 <= k <= 64.
 */
#ifndef GERAF_H
#define GERAF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_forest gf_forest;   /* opaque; owned by the library */

typedef enum {
    GF_OK = 0,
    GF_EINVAL = -1,          /* invalid argument (nothing was launched) */
    GF_ENOMEM = -2,          /* host or device allocation failed, or the device
                                memory the library holds would exceed the cap
                                GF_MAX_DEVICE_BYTES (environment, bytes), when set */
    GF_EHIP = -3,            /* a HIP runtime call failed */
    GF_EUNSUPPORTED = -4,    /* valid request outside the library's limits */
    GF_EINTERNAL = -5        /* an internal consistency check failed */
} gf_status;

/* Distance forms.  FP32: direct sum of (q_j - x_j)^2 over FP32 rows.
 * BF16 / FP8 (e4m3, per-row scale): ||x||^2 - 2 q.x + ||q||^2 on the
 * reduced-precision copies with FP32 accumulation, used only to select the
 * `rerank` best candidates, which are then measured again in FP32 (direct,
 * compensated) on the FP32 rows.  In every form the distances that decide
 * the k-th place within 1e-5 relative are measured once more in FP64. */
typedef enum { GF_FORM_FP32 = 0, GF_FORM_BF16 = 1, GF_FORM_FP8 = 2 } gf_form;

/* Bits of gf_build_forest's `forms` argument: which reduced-precision copies
 * of X to keep on the device (FP32 rows are always kept), and where the trees
 * are built. */
#define GF_KEEP_BF16 (1u << 1)
#define GF_KEEP_FP8  (1u << 2)
/* Build on the GPU instead of the host (Alg. 1, Alg. 3; Sec. 3 "Median,
 * variances" and "Parallelization"): FP64 column moments (Knuth's update
 * over row chunks, combined in chunk order), then every tree level by level,
 * one workgroup per node: the node's split coordinates, a radix select of
 * the median item under (coordinate, tie key, id) and a stable partition of
 * its ids.  The arrays are bit-identical to the host build's (the median
 * item is unique under that strict order, and leaves are sorted by id);
 * D is the same set except where the near-tie guard below sits within a few
 * ulps of its bound.  GF_EUNSUPPORTED for leaves above 4096 points. */
#define GF_BUILD_DEVICE (1u << 8)

/* Build a forest of m randomized k-d trees over X (Alg. 1).
 *   X      [n][d] float32, host-or-device; read during the call only (the
 *          library keeps its own device copies).  Must be finite.
 *   m      number of trees; t size of the top-variance dimension set D;
 *   leaf   maximum points per leaf (the paper's p); every tree is perfect of
 *          depth H = min{h : ceil(n / 2^h) <= leaf};
 *   seed   key of the counter-based RNG (splitmix64 keyed by seed, stream,
 *          tree and node or point) that draws each node's split dimension
 *          from D and each tree's tie-break key per point ("shuffling").
 *   forms  GF_KEEP_* bits, and GF_BUILD_DEVICE.
 *   out    receives the new forest; release it with gf_free_forest.
 * Without GF_BUILD_DEVICE the build runs on the host (threads over trees,
 * Sec. 3 "Parallelization"); the arrays, the FP32 rows and the requested
 * reduced-precision copies are then uploaded on `stream` (host rows through
 * pinned staging buffers).  With it, the FP32 rows are uploaded first and
 * the trees are built from them on the device.
 * With the environment variable GF_BUILD_TIMING=1 each phase's wall time is
 * printed to stderr.
 * GF_EINVAL also when D is not determined by the data: the t-th and
 * (t+1)-th largest column variances differ by at most 1e-12 of the larger
 * of the two columns' mean squares (V + mean^2), the scale of FP64
 * rounding in the variance, so that another correct evaluation could pick a
 * different set (Alg. 1). */
gf_status gf_build_forest(const float *X, int64_t n, int32_t d, int32_t m, int32_t t,
                          int32_t leaf, uint64_t seed, uint32_t forms, void *stream,
                          gf_forest **out);

/* Bits of gf_build_forest_ex's `variants` argument. */
#define GF_VARIANT_HOUSEHOLDER (1u << 0)
#define GF_VARIANT_JITTER (1u << 1)          /* split-value jitter, approximate diameter */
#define GF_VARIANT_JITTER_EXACT (1u << 2)    /* split-value jitter, exact diameter */

/* gf_build_forest with randomisation variants.  variants = 0 is exactly
 * gf_build_forest.  GF_VARIANT_HOUSEHOLDER is the isometry of Sec. 2.1
 * ("Rotation") in the Householder form of Sec. 2.2: tree i gets a reflector
 * P_i = I - 2 u_i u_i', u_i drawn from the RNG (stream 4: components uniform
 * in [-1, 1), then normalised in FP64), and splits the coordinates of P_i x
 * rounded to float32, with u_i . x summed in FP64 in index order; D is still
 * the top-variance set of X.  gf_query reflects each query the same way
 * before that tree's descent and measures distances on the original points
 * and query.
 * GF_VARIANT_JITTER / GF_VARIANT_JITTER_EXACT: split-value jitter (Sec. 2.1
 * "Split value").  Each node splits at its median (the plain build's) plus
 * delta = w * (3 Delta / sqrt(d)), w uniform in [-1, 1) from the generator
 * (stream 3, keyed by tree and node), Delta the diameter of the node's
 * points: exact (largest pairwise distance, O(|P|^2 d) per node) or
 * approximate (largest distance from the node's point of smallest id,
 * between Delta/2 and Delta).  The value is float32(median + delta), points
 * below it go left; a value that leaves a side empty is replaced by the
 * median split.  Nodes split until they hold at most `leaf` points, so trees
 * are no longer perfect: they are stored in the perfect layout of depth H =
 * the deepest leaf (reported by gf_forest_info), every internal position
 * below a leaf passing all points and queries left (value +inf, slot 0) and
 * the leaf's points placed in the leftmost leaf below it.  Queries then open
 * the trees' own leaves in Alg. 2's order, and never the empty padding
 * leaves (the budget is capped at the trees' own leaves).  Built on the host
 * only (GF_EUNSUPPORTED with GF_BUILD_DEVICE or GF_VARIANT_HOUSEHOLDER, or
 * when a tree would need more than 23 levels).  Other bits are rejected with
 * GF_EINVAL. */
gf_status gf_build_forest_ex(const float *X, int64_t n, int32_t d, int32_t m, int32_t t,
                             int32_t leaf, uint64_t seed, uint32_t forms, uint32_t variants,
                             void *stream, gf_forest **out);

/* Release a forest and all its device memory.  NULL is accepted. */
gf_status gf_free_forest(gf_forest *F);

/* Shape of a built forest (any output pointer may be NULL). */
gf_status gf_forest_info(const gf_forest *F, int64_t *n, int32_t *d, int32_t *m,
                         int32_t *t, int32_t *leaf, int32_t *H);

/* Copy the host-side tree arrays out (host buffers, caller-allocated):
 *   D[t]                         the top-variance dimensions, ascending;
 *   split_dim[m][2^H - 1]        split column of each internal node;
 *   split_val[m][2^H - 1]        split value of each internal node;
 *   perm[m][n]                   per tree, point ids leaf by leaf, each leaf
 *                                ascending;
 *   leaf_off[m][2^H + 1]         leaf j of tree i = perm[i][leaf_off[i][j] ..
 *                                leaf_off[i][j+1]) (the same in every tree
 *                                unless the trees are jittered).
 * Node v has children 2v+1 (left, coordinate < value) and 2v+2 (right).
 * Any pointer may be NULL to skip that array. */
gf_status gf_export_tree(const gf_forest *F, int32_t *D, int32_t *split_dim,
                         float *split_val, uint32_t *perm, uint32_t *leaf_off);

/* Search every row of Q (Alg. 2): the leaves opened per query are the first
 * B = min(ceil(checks/(1+eps)), m * 2^H) of the shared queue's pop order
 * (every root enters at key 0; each child left behind during a descent
 * enters with its own |gap| of Eq. 1, gap = float32(q_s - v), a zero gap
 * descending right; equal keys pop the lower tree, then the lower node);
 * the candidates are the distinct points of those leaves; the result is the
 * k best candidates.
 * Two execution paths give the same candidate sets: the row path gathers
 * each query's candidate rows (for small batches each query's id range is
 * cut into slices, one workgroup each; GF_SCAN_SLICES=<count> forces a
 * count, for testing); the tile paths score blocks of queries (128 BF16, 256
 * FP8) against all points on MFMA and keep only those of each query's
 * candidates: BF16 (d <= 1024, batches of >= 2 queries whose candidates
 * exceed ~1/256 of the points) and FP8 (any d, batches of >= 32 queries whose
 * candidates exceed ~1/192 of the points).  The environment variable GF_SCAN_PATH (= rows |
 * tile) overrides the choice where a tile path is available.
 * Rows wider than 4,096 FP32 (8,192 BF16) elements are streamed against a
 * copy of the query in LDS where it fits beside the visited bitmap;
 * GF_SCAN_WIDE_QUERY=global reads it from device memory instead (same
 * results; for testing).
 *   Q                 [nq][d] float32, host-or-device, finite.  Host rows are
 *                     copied through a pinned host buffer that the forest
 *                     keeps and grows to its largest batch (at most 16,384
 *                     padded rows); gf_free_forest releases it.
 *   k                 neighbours per query (1..64).
 *   checks            the paper's c: leaves to check per query (>= 1).
 *   checks_per_query  NULL, or nq int32 budgets (host-or-device) that
 *                     replace `checks` per query.
 *   eps               >= 0; the budget becomes ceil(c / (1 + eps)).
 *   form              gf_form; BF16/FP8 need the copy kept at build time.
 *   rerank            reduced-precision forms: candidates re-measured in FP32
 *                     (k <= rerank <= 64; 0 selects 4k, capped at 64).
 *                     Ignored by GF_FORM_FP32.
 *   ids, dists        [nq][k] int32 / float32 outputs, host-or-device. */
gf_status gf_query(const gf_forest *F, const float *Q, int64_t nq, int32_t k,
                   int32_t checks, const int32_t *checks_per_query, double eps,
                   int32_t form, int32_t rerank, int32_t *ids, float *dists,
                   void *stream);

/* One search request of a gf_query_multi call: the arguments of gf_query
 * for one forest, with every buffer in device memory. */
typedef struct gf_job {
    const gf_forest *forest;
    const float *Q;                    /* [nq][d] float32, device, finite */
    int64_t nq;
    int32_t k;                         /* 1..64 */
    int32_t checks;                    /* >= 1, unless checks_per_query */
    const int32_t *checks_per_query;   /* NULL or [nq] int32 >= 1, device */
    double eps;                        /* >= 0 */
    int32_t form;                      /* gf_form */
    int32_t rerank;                    /* as for gf_query */
    int32_t *ids;                      /* [nq][k] int32, device */
    float *dists;                      /* [nq][k] float32, device */
} gf_job;

#define GF_MULTI_AUTOTUNE 1u  /* measure the launch variants per (forest, form, batch size) once */
#define GF_MULTI_EAGER 2u     /* launch kernel by kernel instead of one graph launch */

/* Run many searches, over many forests of uneven n and d and with per-query
 * budgets, as one launch (the batching the paper's Sec. 5 leaves for future
 * work).  Every job gives the same results as gf_query with the same
 * arguments and the same path; the path of each 16,384-query batch follows
 * gf_query's rule, or with GF_MULTI_AUTOTUNE the fastest launch variant as
 * measured on the first batch of each (forest, form, batch-size class,
 * rerank), a choice the forest then keeps.  The variants are the row path
 * with 1, 2 or 4 times the rule's slices of each query's id range (one
 * workgroup per slice) and, where the form has one, the tile path; they give
 * identical results.
 * All query rows are checked finite first (one readback for the call).  The
 * launches of every batch are then captured into one HIP graph, which runs on
 * `stream`: the batches of one forest in order on one branch (they share the
 * forest's workspace), the branches of different forests concurrently.  The instantiated graph is kept (up to 16 of them, by least recent
 * use) and launched again when a call repeats the same jobs, buffers and
 * paths; freeing a forest drops the graphs that use it.
 * All forests must live on the current device.  The call returns when the
 * results are in place.  Calls on a forest wait for each other (the forest's
 * workspace is shared).
 * Errors: GF_EINVAL for bad arguments, host buffers, NaN/Inf in Q; GF_EHIP
 * for HIP failures (nothing partially written is guaranteed then). */
gf_status gf_query_multi(const gf_job *jobs, int32_t njobs, uint32_t flags, void *stream);

/* gf_query for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and results as gf_query on its row path (GF_SCAN_PATH=rows), but
 * the call allocates nothing: no hipMalloc / hipFree, no events, no pinned
 * staging.  Its workspace is a static device array of 128 MiB, one copy per
 * GPU, held until the process ends; queries run in batches sized to fit it.
 *   Q, checks_per_query, ids, dists  device buffers only (GF_EINVAL for host
 *                    memory); device budgets are used as given (a budget
 *                    below 1 opens no leaf), not read back.
 *   GF_EUNSUPPORTED  when one query's workspace exceeds 128 MiB (very deep
 *                    or very many trees), or the device index is above 63.
 * Calls on one GPU share that array: the library runs them one at a time
 * (a lock per device), and each returns after its work has finished, so
 * they cannot overlap from one process; kernels that a caller enqueues on
 * its own into that memory would race.  Every call rewrites what it reads,
 * nothing is assumed zero from an earlier call.  gf_last_query_timing is
 * not updated by this call. */
gf_status gf_query_noalloc(const gf_forest *F, const float *Q, int64_t nq, int32_t k,
                           int32_t checks, const int32_t *checks_per_query, double eps,
                           int32_t form, int32_t rerank, int32_t *ids, float *dists,
                           void *stream);

/* Counters of the multi-index launch since the library was loaded: graphs
 * captured, graph launches reused from an earlier identical call, path
 * choices measured by the autotuner.  Any pointer may be NULL. */
gf_status gf_multi_stats(int64_t *graphs_built, int64_t *graphs_reused, int64_t *tuned);

/* The query path's intermediate sets, for parity checks:
 *   leaf_bits  [nq][m][W] uint32, W = max(1, 2^H / 32): bit (j % 32) of word
 *              j / 32 of tree i is set iff leaf j of tree i was opened;
 *   cand_bits  [nq][ceil(n/32)] uint32: bit i set iff point i was a
 *              candidate (the visited array after all opened leaves);
 *   ncand      [nq] int64: number of candidates.
 * All three are host-or-device; any may be NULL.  Same budget rules as
 * gf_query.  Runs the same selection kernels as gf_query, and the row
 * path's expansion: the candidate set is the visited bitmap that the row
 * scan builds (the visited array of Sec. 2.3).  Equal to
 * gf_query_trace_ex(..., GF_TRACE_ROWS, ...). */
gf_status gf_query_trace(const gf_forest *F, const float *Q, int64_t nq, int32_t checks,
                         const int32_t *checks_per_query, double eps, uint32_t *leaf_bits,
                         uint32_t *cand_bits, int64_t *ncand, void *stream);

/* Which expansion gf_query_trace_ex reports the candidates of. */
#define GF_TRACE_ROWS 0   /* the row scan's visited bitmap */
#define GF_TRACE_TILE 1   /* the tile path's per-point words of query bits */

/* gf_query_trace with the expansion chosen by `path`.  GF_TRACE_TILE runs
 * the tile path's expansion kernels (opened leaves -> per-leaf rows of
 * query bits -> per-point words of query bits, the words the MFMA tile
 * kernel masks its scores with) and returns those words turned back into
 * the per-query layout of cand_bits; it needs a forest built with
 * GF_KEEP_BF16 (GF_EINVAL otherwise).  Other values of path: GF_EINVAL. */
gf_status gf_query_trace_ex(const gf_forest *F, const float *Q, int64_t nq, int32_t checks,
                            const int32_t *checks_per_query, double eps, int32_t path,
                            uint32_t *leaf_bits, uint32_t *cand_bits, int64_t *ncand,
                            void *stream);

/* Diagnostics of the FP8 e4m3 storage format (used by the tests):
 *   hw_decode[256]   every byte decoded by the gfx950 conversion instruction
 *                    that the FP8 distance kernels use;
 *   def_decode[256]  every byte decoded from the OCP E4M3 definition (bias 7,
 *                    3 mantissa bits, subnormal step 2^-9, 0x7F/0xFF NaN);
 *   enc_in[n_enc] -> enc_out[n_enc]  the library's float -> e4m3 rounding
 *                    (nearest-even, saturating at 448).
 * Host buffers. */
gf_status gf_fp8_tables(float *hw_decode, float *def_decode, const float *enc_in,
                        int32_t n_enc, uint8_t *enc_out);

/* Measurement utility (not part of the method): the device's streaming
 * read bandwidth, the practical ceiling beside the 8 TB/s peak that the
 * row-gather rooflines are priced against.  One warm-up and then `reps`
 * launches of a kernel that reads the `bytes` (rounded down to 16) of `buf`
 * in 16-byte words, contiguous 64 KB spans per workgroup with sixteen
 * non-temporal loads in flight per thread, and writes nothing to it; *read_gb_s = bytes read / time between HIP events on `stream`, in
 * GB/s.  buf: device memory, 16-byte aligned, caller-owned, contents
 * unchanged.  GF_EINVAL for a host or misaligned buf, bytes < 16, reps < 1. */
gf_status gf_hbm_probe(const void *buf, int64_t bytes, int32_t reps, double *read_gb_s,
                       void *stream);

/* Device time of the phases of the last successful gf_query or
 * gf_query_trace on the calling thread, in milliseconds, from HIP events
 * recorded on the query's stream, summed over its batches (a call is split
 * into batches of at most 16384 queries):
 *   phase_ms[0]  query preparation (copies, conversions, finiteness check)
 *   phase_ms[1]  leaf selection (Alg. 2's queue: every radix pass)
 *   phase_ms[2]  row path: the whole scan kernel (candidate expansion,
 *                gathers, distances, best-k, re-rank, tie re-check);
 *                tile path: the candidate expansion kernel
 *   phase_ms[3]  tile path: the MFMA score kernel (0 on the row path)
 *   phase_ms[4]  tile path: merge, re-rank, tie re-check (0 on the row path)
 * Up to nphase entries are written.  *path = 0 (row path) or 1 (tile path)
 * for the last batch; *batches = number of batches.  Pointers may be NULL. */
gf_status gf_last_query_timing(double *phase_ms, int32_t nphase, int32_t *path,
                               int64_t *batches);

/* Human-readable description of the last error on the calling thread. */
const char *gf_last_error(void);

/* Library version string. */
const char *gf_version(void);

/* Bytes of device memory the library holds right now (forests, their query
 * workspaces and temporaries; not the fixed scratch of gf_query_noalloc):
 * the total that GF_MAX_DEVICE_BYTES caps.  Never fails. */
int64_t gf_device_bytes(void);

#ifdef __cplusplus
}
#endif

#endif /* GERAF_H */
