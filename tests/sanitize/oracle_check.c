/* Sanitizer driver for oracle.c: builds plain, reflected and jittered forests
 * on small random data and searches them, under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Exit status 0 when every call succeeds and the
 * results satisfy basic invariants (a permutation per tree, k sorted
 * distances).  Compiled and run by tests/test_sanitizers.py. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_build(const float *X, int64_t n, int32_t d, int32_t m, int32_t t, int32_t p,
              uint64_t seed, int32_t nthreads, int32_t *D, int32_t *split_dim, float *split_val,
              uint32_t *perm, uint32_t *leaf_off, const double *U);
int orc_search(const float *X, int64_t n, int32_t d, int32_t m, int32_t H,
               const int32_t *split_dim, const float *split_val, const uint32_t *perm,
               const uint32_t *leaf_off, const float *Q, int64_t nq, int32_t k, int64_t c,
               double eps, int32_t eff_key, int32_t nthreads, int32_t *ids, double *dists,
               uint32_t *opened, double *opened_key, int64_t *ncand, uint32_t *cand,
               int64_t cand_cap, const double *U);
int orc_householder(uint64_t seed, int32_t tree, int32_t d, double *u);
int32_t orc_depth(int64_t n, int32_t p);
int orc_build_jitter(const float *X, int64_t n, int32_t d, int32_t m, int32_t t, int32_t p,
                     uint64_t seed, int32_t exact, int64_t ncap, int32_t *D, int32_t *dim,
                     float *val, int32_t *left, int32_t *right, int32_t *heap, int32_t *depth,
                     uint32_t *off, uint32_t *len, uint32_t *perm, int64_t *nnodes, int32_t *H);
int orc_search_jitter(const float *X, int64_t n, int32_t d, int32_t m, int32_t H, int64_t ncap,
                      const int32_t *dim, const float *val, const int32_t *left,
                      const int32_t *right, const int32_t *heap, const int32_t *depth,
                      const uint32_t *off, const uint32_t *len, const uint32_t *perm,
                      const int64_t *nnodes, const float *Q, int64_t nq, int32_t k, int64_t c,
                      double eps, int32_t *ids, double *dists, uint32_t *opened,
                      double *opened_key, int64_t *ncand, uint32_t *cand, int64_t cand_cap);

static int is_perm(const uint32_t *p, int64_t n)
{
    unsigned char *seen = calloc((size_t)n, 1);
    int ok = 1;
    for (int64_t i = 0; i < n; ++i) {
        if (p[i] >= n || seen[p[i]]) { ok = 0; break; }
        seen[p[i]] = 1;
    }
    free(seen);
    return ok;
}

static int sorted_k(const double *dd, int32_t k)
{
    for (int32_t r = 1; r < k; ++r)
        if (dd[r] < dd[r - 1]) return 0;
    return 1;
}

int main(void)
{
    const int64_t n = 700, nq = 9;
    const int32_t d = 11, m = 3, t = 4, p = 5, k = 4;
    float *X = malloc(sizeof(float) * n * d), *Q = malloc(sizeof(float) * nq * d);
    srand(7);
    for (int64_t i = 0; i < n * d; ++i) X[i] = (float)(rand() % 1000) / 250.0f - 2.0f;
    for (int64_t i = 0; i < nq * d; ++i) Q[i] = (float)(rand() % 1000) / 250.0f - 2.0f;
    int32_t H = orc_depth(n, p), D[4];
    int64_t nint = ((int64_t)1 << H) - 1;
    int32_t *sd = malloc(sizeof(int32_t) * m * nint);
    float *sv = malloc(sizeof(float) * m * nint);
    uint32_t *perm = malloc(sizeof(uint32_t) * m * n), *lo = malloc(sizeof(uint32_t) * (((size_t)1 << H) + 1));
    double *U = malloc(sizeof(double) * m * d);
    int32_t *ids = malloc(sizeof(int32_t) * nq * k);
    double *dd = malloc(sizeof(double) * nq * k);
    int64_t *nc = malloc(sizeof(int64_t) * nq);
    uint32_t *cand = malloc(sizeof(uint32_t) * nq * n);
    for (int variant = 0; variant < 2; ++variant) {
        const double *u = NULL;
        if (variant) {
            for (int32_t tr = 0; tr < m; ++tr)
                if (orc_householder(5, tr, d, U + (int64_t)tr * d)) return 10;
            u = U;
        }
        if (orc_build(X, n, d, m, t, p, 99, 2, D, sd, sv, perm, lo, u)) return 11;
        for (int32_t tr = 0; tr < m; ++tr)
            if (!is_perm(perm + (int64_t)tr * n, n)) return 12;
        for (int eff = 0; eff < 2; ++eff)
            for (int64_t c = 1; c <= (m << H); c *= 7) {
                if (orc_search(X, n, d, m, H, sd, sv, perm, lo, Q, nq, k, c, 0.1, eff, 2, ids, dd,
                               NULL, NULL, nc, cand, n, u))
                    return 13;
                for (int64_t q = 0; q < nq; ++q)
                    if (!sorted_k(dd + q * k, k)) return 14;
            }
    }
    /* jitter: explicit trees, both diameters */
    const int64_t ncap = 2 * n;
    int32_t *dim = malloc(sizeof(int32_t) * m * ncap), *left = malloc(sizeof(int32_t) * m * ncap);
    int32_t *right = malloc(sizeof(int32_t) * m * ncap), *heap = malloc(sizeof(int32_t) * m * ncap);
    int32_t *dep = malloc(sizeof(int32_t) * m * ncap);
    float *val = malloc(sizeof(float) * m * ncap);
    uint32_t *off = malloc(sizeof(uint32_t) * m * ncap), *len = malloc(sizeof(uint32_t) * m * ncap);
    int64_t nn[3];
    for (int exact = 0; exact < 2; ++exact) {
        int32_t HJ = 0;
        if (orc_build_jitter(X, n, d, m, t, p, 17, exact, ncap, D, dim, val, left, right, heap, dep,
                             off, len, perm, nn, &HJ))
            return 20;
        for (int32_t tr = 0; tr < m; ++tr)
            if (!is_perm(perm + (int64_t)tr * n, n)) return 21;
        uint32_t *opened = malloc(sizeof(uint32_t) * nq * n);
        double *okey = malloc(sizeof(double) * nq * n);
        for (int64_t c = 1; c <= n; c *= 5) {
            if (orc_search_jitter(X, n, d, m, HJ, ncap, dim, val, left, right, heap, dep, off, len,
                                  perm, nn, Q, nq, k, c, 0.0, ids, dd, opened, okey, nc, cand, n))
                return 22;
            for (int64_t q = 0; q < nq; ++q)
                if (!sorted_k(dd + q * k, k)) return 23;
        }
        free(opened);
        free(okey);
    }
    free(X); free(Q); free(sd); free(sv); free(perm); free(lo); free(U); free(ids); free(dd);
    free(nc); free(cand); free(dim); free(left); free(right); free(heap); free(dep); free(val);
    free(off); free(len);
    puts("oracle sanitizer check passed");
    return 0;
}
