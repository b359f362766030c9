/* Host run of the C oracle (oracle/f2m_oracle.c) built with
 * AddressSanitizer and UndefinedBehaviorSanitizer: the GDP loop (complete
 * graph and a CSR graph, with the hand-off and without, b-matching
 * degrees), the trivial x, the certificate and the exact optimum on random
 * and tie-heavy instances.  Exit status 0 when every call succeeds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_gdp_solve(int64_t n, const int32_t *xy, const int64_t *rowptr, const int32_t *col, const int32_t *b,
                 int64_t *lam, int64_t max_iters, int64_t handoff_div, int64_t *trace, int64_t *iters, int32_t *stop,
                 int64_t *kstar, int64_t *z4, int32_t *i4, int32_t *neg, int32_t *zero);
int or_certify(int64_t n, const int32_t *xy, const int64_t *rowptr, const int32_t *col, const int32_t *b,
               const int64_t *lam, int64_t m, const int32_t *eu, const int32_t *ev, const uint8_t *ex2, int64_t *out);
int64_t or_trivial_x(int64_t n, const int32_t *xy, const int64_t *lam, int64_t cap, int32_t *eu, int32_t *ev,
                     uint8_t *ex2);
int or_exact_opt2(int64_t n, const int32_t *xy, const int64_t *rowptr, const int32_t *col, const int32_t *b,
                  int64_t *opt2, uint8_t *x2, int64_t *lam);
int or_knn(int64_t n, const int32_t *xy, int64_t k, int32_t *idx);

static uint64_t state = 88172645463325252ULL;
static uint64_t next(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

int main(void)
{
    int fails = 0;
    const int64_t sizes[] = {4, 7, 30, 120};
    for (int si = 0; si < 4; ++si) {
        for (int mode = 0; mode < 3; ++mode) {
            const int64_t n = sizes[si];
            int32_t *xy = malloc(sizeof(int32_t) * 2 * n);
            const int span = mode == 1 ? 30 : 100000;
            for (int64_t i = 0; i < 2 * n; ++i) xy[i] = (int32_t)(next() % span);
            int32_t *b = NULL;
            if (mode == 2) {
                b = malloc(sizeof(int32_t) * n);
                for (int64_t v = 0; v < n; ++v) b[v] = 1 + (int32_t)(next() % 3);
            }
            /* a CSR candidate graph: every node's 3 nearest, symmetrised by listing both directions */
            const int64_t k = n > 4 ? 3 : n - 1;
            int32_t *idx = malloc(sizeof(int32_t) * n * k);
            if (or_knn(n, xy, k, idx)) ++fails;
            int64_t *deg = calloc(n + 1, sizeof(int64_t));
            for (int64_t v = 0; v < n; ++v)
                for (int64_t j = 0; j < k; ++j) { deg[v]++; deg[idx[v * k + j]]++; }
            int64_t *rowptr = calloc(n + 1, sizeof(int64_t));
            for (int64_t v = 0; v < n; ++v) rowptr[v + 1] = rowptr[v] + deg[v];
            int32_t *col = malloc(sizeof(int32_t) * (rowptr[n] + 1));
            int64_t *at = malloc(sizeof(int64_t) * n);
            for (int64_t v = 0; v < n; ++v) at[v] = rowptr[v];
            for (int64_t v = 0; v < n; ++v)
                for (int64_t j = 0; j < k; ++j) {
                    const int32_t u = idx[v * k + j];
                    col[at[v]++] = u;
                    col[at[u]++] = (int32_t)v;
                }
            /* sort and dedupe each row, as a CSR graph needs */
            int64_t w = 0, start = 0;
            for (int64_t v = 0; v < n; ++v) {
                const int64_t a = start, e = rowptr[v + 1];
                for (int64_t i = a + 1; i < e; ++i)
                    for (int64_t j = i; j > a && col[j - 1] > col[j]; --j) { int32_t t = col[j]; col[j] = col[j - 1]; col[j - 1] = t; }
                start = e;
                rowptr[v + 1] = w;
                for (int64_t i = a; i < e; ++i)
                    if (i == a || col[i] != col[i - 1]) col[w++] = col[i];
                rowptr[v + 1] = w;
            }
            for (int graph = 0; graph < 2; ++graph) {
                for (int64_t hand = 0; hand <= 50; hand += 50) {
                    const int64_t max_iters = 400;
                    int64_t *lam = calloc(n, sizeof(int64_t));
                    int64_t *trace = malloc(sizeof(int64_t) * 8 * (max_iters + 1));
                    int64_t iters, kstar, *z4 = malloc(sizeof(int64_t) * 4 * n);
                    int32_t stop, *i4 = malloc(sizeof(int32_t) * 4 * n), *neg = malloc(sizeof(int32_t) * n),
                                  *zero = malloc(sizeof(int32_t) * n);
                    int rc = or_gdp_solve(n, xy, graph ? rowptr : NULL, graph ? col : NULL, b, lam, max_iters, hand,
                                          trace, &iters, &stop, &kstar, z4, i4, neg, zero);
                    if (rc < 0) ++fails;
                    const int64_t cap = 4 * n * n;
                    int32_t *eu = malloc(sizeof(int32_t) * cap), *ev = malloc(sizeof(int32_t) * cap);
                    uint8_t *ex = malloc(cap);
                    const int64_t m = or_trivial_x(n, xy, lam, cap, eu, ev, ex);
                    int64_t out[4];
                    if (m < 0 || or_certify(n, xy, NULL, NULL, b, lam, m, eu, ev, ex, out) < 0) ++fails;
                    free(eu); free(ev); free(ex);
                    free(lam); free(trace); free(z4); free(i4); free(neg); free(zero);
                }
            }
            if (n <= 30) {
                int64_t opt2;
                uint8_t *x2 = malloc((size_t)(n * n));
                int64_t *lam = malloc(sizeof(int64_t) * 2 * n);
                const int rc = or_exact_opt2(n, xy, NULL, NULL, b, &opt2, x2, lam);
                if (rc < 0 && rc != -3) ++fails;
                free(x2); free(lam);
            }
            free(xy); free(b); free(idx); free(deg); free(rowptr); free(col); free(at);
        }
    }
    printf("oracle sanitize failures %d\n", fails);
    return fails ? 1 : 0;
}
