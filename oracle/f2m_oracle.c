/*
 * f2m_oracle.c -- plain CPU oracle for the gradient descent procedure (GDP)
 * on the fractional 2-matching (F2M) relaxation of Euclidean TSP
 * (Antonov, arXiv 2011.08170).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the HIP library.
 *
 * Everything is exact integer arithmetic.  Notation follows the paper:
 *   c_e            edge length; for integer 2-D coordinates the TSPLIB
 *                  EUC_2D length nint(sqrt(D)), D the squared distance
 *                  (Sec. 5.1 says the input is TSPLIB coordinates).
 *   lambda_v       node multiplier of the degree row of node v (Sec. 4).
 *   v^e            adjusted length c_e - lambda_u - lambda_v   (eq. 9).
 * Fixed point: Lam = 2*lambda (int64) and Z_e = 2*v^e = 2c_e - Lam_u - Lam_v.
 *
 * GDP step (eq. 10 and Sec. 3, read as "move lambda_v to the midpoint of the
 * 2nd and 3rd shortest adjusted edges at v", damped by one half and rounded
 * half away from zero on the Lam grid):
 *   s_v      = Z_(2) + Z_(3)       (2nd and 3rd smallest of {Z_uv : u != v})
 *   dLam_v   = sign(s_v) * floor((|s_v| + 2) / 4)
 *   Lam'     = Lam + dLam          (all nodes from the same Lam: Jacobi, Sec. 5.1)
 *
 * Trivial solution (eq. 7 and Sec. 4): x_e = 1 if Z_e < 0, 1/2 if Z_e = 0,
 * 0 if Z_e > 0.  Its doubled degree at v is deg2_v = 2*neg_v + zero_v.
 *
 * Lagrangian dual bound of the degree rows (Sec. 2, eq. 4-5 with the box
 * kept):  L(lambda) = 2*sum_v lambda_v + sum_e min(0, v^e), so in doubled
 * units  dual2 = 2*L = 2*sum Lam + sum_{u<v} min(0, Z_uv).  For any feasible
 * x, c.x >= L (weak duality); equality certifies optimality.
 *
 * Rows with other right-hand sides (Sec. 3: the method applies to LP3 rows
 * with binary coefficients and an integral b_i, condition 8): every routine
 * takes an optional per-node degree b_v (NULL: 2, the F2M of Sec. 4), so the
 * problem is the fractional b-matching  sum_{e in delta(v)} x_e = b_v,
 * 0 <= x <= 1.  The row's gradient then compares positions b_v and b_v + 1
 * of its sorted adjusted lengths (Sec. 3), the step is
 * sign(s) floor((|s| + 2)/4) with s = Z_(b) + Z_(b+1), the trivial doubled
 * degree must equal 2 b_v, and the dual bound is sum_v b_v lambda_v +
 * sum_e min(0, v^e), i.e. dual2 = sum_v b_v Lam_v + sum_{u<v} min(0, Z).
 * The top four are kept per row, so b_v is 1, 2 or 3.
 *
 * Candidate graphs (Sec. 5.3: "the top N closest neighbors for each node"):
 * every routine takes an optional CSR graph (rowptr[n+1], col[]), symmetric,
 * no self loops; NULL means the complete graph.  On a graph, a row's
 * statistics run over its neighbours only, the dual bound sums over its
 * edges and the exact optimum uses its edges only.
 *
 * The exact optimum (used to pin the GDP and the finisher) comes from the
 * bipartite double cover: left copy v', right copy v'', arc v'->u'' of cost
 * c_uv and capacity 1 for every ordered pair; every copy has degree b_v (2
 * for F2M).  Its min-cost flow equals 2 * the optimum and x_e = (y_u'v'' + y_v'u'')/2
 * is an optimal F2M solution (Edmonds' half-integrality, Sec. 4).  Solved
 * here by plain successive shortest paths with node potentials on the dense
 * complete graph.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_RANGE (-2)
#define OR_ERR_INFEASIBLE (-3)
#define OR_ERR_NOMEM (-4)

/* stop reasons of the GDP loop */
#define OR_STOP_TRIVIAL 1   /* every doubled degree of the trivial x is 4 */
#define OR_STOP_FIXED 2     /* every step is zero */
#define OR_STOP_CYCLE 3     /* hash of Lam_k equals hash of Lam_{k-2} */
#define OR_STOP_CAP 4       /* iteration cap reached */
#define OR_STOP_HANDOFF 5   /* few unsatisfied nodes left: hand over to an exact finish */

/* ------------------------------------------------------------------ */
/* integer square root and the exact EUC_2D length                     */
/* ------------------------------------------------------------------ */

/* floor(sqrt(x)) for 0 <= x < 2^62: the library square root gives an
 * estimate r; the two loops then move r until r*r <= x < (r+1)*(r+1),
 * which defines floor(sqrt(x)) whatever the estimate's rounding was
 * (r stays below 2^31, so (r+1)^2 <= 2^62 cannot overflow). */
int64_t or_isqrt(int64_t x)
{
    if (x <= 0) return 0;
    int64_t r = (int64_t)sqrt((double)x);
    if (r > 2147483647) r = 2147483647;
    while (r > 0 && r * r > x) r--;
    while ((r + 1) * (r + 1) <= x) r++;
    return r;
}

/* nint(sqrt(D)): the integer k with k - 1/2 <= sqrt(D) < k + 1/2, i.e.
 * (2k-1)^2 <= 4D < (2k+1)^2, which is floor((isqrt(4D) + 1) / 2). */
int64_t or_nint_sqrt(int64_t D)
{
    return (or_isqrt(4 * D) + 1) / 2;
}

static inline int64_t sq_dist(const int32_t *xy, int64_t u, int64_t v)
{
    int64_t dx = (int64_t)xy[2 * u] - xy[2 * v];
    int64_t dy = (int64_t)xy[2 * u + 1] - xy[2 * v + 1];
    return dx * dx + dy * dy;
}

int64_t or_cost(const int32_t *xy, int64_t u, int64_t v)
{
    return or_nint_sqrt(sq_dist(xy, u, v));
}

/* Input check shared by every entry point of the oracle: each axis span
 * must be below 2^20 so that 4D < 2^43. */
int or_check_coords(const int32_t *xy, int64_t n)
{
    if (!xy || n < 0) return OR_ERR_ARG;
    if (n == 0) return OR_OK;
    int64_t mnx = xy[0], mxx = xy[0], mny = xy[1], mxy = xy[1];
    for (int64_t i = 1; i < n; i++) {
        if (xy[2 * i] < mnx) mnx = xy[2 * i];
        if (xy[2 * i] > mxx) mxx = xy[2 * i];
        if (xy[2 * i + 1] < mny) mny = xy[2 * i + 1];
        if (xy[2 * i + 1] > mxy) mxy = xy[2 * i + 1];
    }
    if (mxx - mnx >= (1 << 20) || mxy - mny >= (1 << 20)) return OR_ERR_RANGE;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* one GDP pass over a set of rows                                     */
/* ------------------------------------------------------------------ */

/* (Z, u) lexicographic order */
static inline int key_less(int64_t za, int64_t ua, int64_t zb, int64_t ub)
{
    return za < zb || (za == zb && ua < ub);
}

/* Step on the Lam grid from s = Z_(2) + Z_(3): sign(s) * floor((|s|+2)/4). */
int64_t or_step(int64_t s)
{
    if (s > 0) return (s + 2) / 4;
    if (s < 0) return -((-s + 2) / 4);
    return 0;
}

/* For every row v in rows[0..nrows): scan all u != v, keep the four
 * smallest (Z, u) in order, count Z < 0 and Z == 0, sum min(0, Z), and form
 * the step.  Outputs are indexed by position in `rows`.  z4/i4 hold four
 * entries per row (unused slots: Z = INT64_MAX, u = -1).  Requires n >= 2. */
void or_gdp_rows(int64_t n, const int32_t *xy, const int64_t *rowptr, const int32_t *col,
                 const int64_t *lam, const int32_t *b, int64_t nrows, const int64_t *rows,
                 int64_t *z4, int32_t *i4, int32_t *neg, int32_t *zero,
                 int64_t *rowneg, int64_t *step)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t v = rows[r];
        int64_t bz[4] = {INT64_MAX, INT64_MAX, INT64_MAX, INT64_MAX};
        int64_t bu[4] = {-1, -1, -1, -1};
        int64_t cn = 0, cz = 0, rn = 0;
        const int64_t m = rowptr ? rowptr[v + 1] - rowptr[v] : n;
        for (int64_t e = 0; e < m; e++) {
            const int64_t u = rowptr ? col[rowptr[v] + e] : e;
            if (u == v) continue;
            int64_t z = 2 * or_cost(xy, u, v) - lam[u] - lam[v];     /* eq. 9, doubled */
            if (z < 0) { cn++; rn += z; }
            else if (z == 0) cz++;
            if (key_less(z, u, bz[3], bu[3]) || bu[3] < 0) {
                /* insertion into the sorted list of four */
                int j = 3;
                while (j > 0 && (bu[j - 1] < 0 || key_less(z, u, bz[j - 1], bu[j - 1]))) {
                    bz[j] = bz[j - 1]; bu[j] = bu[j - 1]; j--;
                }
                bz[j] = z; bu[j] = u;
            }
        }
        for (int j = 0; j < 4; j++) { z4[4 * r + j] = bz[j]; i4[4 * r + j] = (int32_t)bu[j]; }
        neg[r] = (int32_t)cn;
        zero[r] = (int32_t)cz;
        rowneg[r] = rn;
        /* eq. 10 (Sec. 3 for a row with right-hand side b): the b-th and
         * (b+1)-th shortest adjusted edges, positions b-1 and b of the sorted
         * list counting from 0 (F2M: the 2nd and 3rd).  The row needs b+1
         * edges. */
        const int bv = b ? b[v] : 2;
        step[r] = (bu[bv] >= 0) ? or_step(bz[bv - 1] + bz[bv]) : 0;
    }
}

/* SplitMix64 output finaliser (Steele, Lea, Flood 2014). */
static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Order-independent fingerprint of a Lam vector. */
uint64_t or_hash(int64_t n, const int64_t *lam)
{
    uint64_t h = 0;
    for (int64_t v = 0; v < n; v++)
        h += mix64((uint64_t)lam[v] ^ (0x9E3779B97F4A7C15ULL * (uint64_t)(v + 1)));
    return h;
}

/* Per-iteration record, one row of int64 per iteration k:
 *  [0] k  [1] dual2  [2] #unsatisfied (Z2 > 0 or Z3 < 0)  [3] #deg2 != 4
 *  [4] max |step|  [5] #nonzero steps  [6] hash (as int64 bits)  [7] sum Lam */
#define OR_TRACE_W 8

/* Full GDP iteration at Lam: all rows, then the global statistics.
 * Outputs per node: z4, i4, neg, zero, step (n rows); rec[OR_TRACE_W]. */
/* every b_v in {1, 2, 3} (or b NULL) */
static int check_b(int64_t n, const int32_t *b)
{
    if (!b) return OR_OK;
    for (int64_t v = 0; v < n; v++)
        if (b[v] < 1 || b[v] > 3) return OR_ERR_ARG;
    return OR_OK;
}

int or_gdp_iter(int64_t n, const int32_t *xy, const int64_t *rowptr, const int32_t *col,
                const int64_t *lam, const int32_t *b, int64_t *z4, int32_t *i4, int32_t *neg, int32_t *zero,
                int64_t *step, int64_t *rec)
{
    if (check_b(n, b)) return OR_ERR_ARG;
    int64_t *rows = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *rowneg = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!rows || !rowneg) { free(rows); free(rowneg); return OR_ERR_NOMEM; }
    for (int64_t v = 0; v < n; v++) rows[v] = v;
    or_gdp_rows(n, xy, rowptr, col, lam, b, n, rows, z4, i4, neg, zero, rowneg, step);
    int64_t sl = 0, sbl = 0, sneg = 0, unsat = 0, bad = 0, mx = 0, nz = 0;
    for (int64_t v = 0; v < n; v++) {
        const int64_t bv = b ? b[v] : 2;
        sl += lam[v];
        sbl += bv * lam[v];
        sneg += rowneg[v];
        if (z4[4 * v + bv - 1] > 0 || z4[4 * v + bv] < 0) unsat++;
        if (2 * neg[v] + zero[v] != 2 * bv) bad++;
        int64_t a = step[v] < 0 ? -step[v] : step[v];
        if (a > mx) mx = a;
        if (step[v] != 0) nz++;
    }
    /* every unordered pair appears in two rows */
    rec[1] = sbl + sneg / 2;
    rec[2] = unsat; rec[3] = bad; rec[4] = mx; rec[5] = nz;
    rec[6] = (int64_t)or_hash(n, lam);
    rec[7] = sl;
    free(rows); free(rowneg);
    return OR_OK;
}

/* GDP loop from lam (in/out).  On return lam holds Lam*, the iterate the
 * loop stops on:  the current one for TRIVIAL, HANDOFF and FIXED, the
 * iterate with the largest dual2 (earliest on ties) for CYCLE and CAP.
 *   handoff_div > 0 stops at the first k with #unsatisfied * handoff_div <= n
 *   (checked right after the trivial test); 0 disables it.
 *   trace: max_iters+1 rows of OR_TRACE_W (may be NULL); *iters = number of
 *   iterations evaluated (records written); *stop = reason; *kstar = index
 *   of Lam*.  z4/i4/neg/zero describe Lam_k of the last evaluated k. */
int or_gdp_solve(int64_t n, const int32_t *xy, const int64_t *rowptr, const int32_t *col,
                 const int32_t *b, int64_t *lam, int64_t max_iters, int64_t handoff_div,
                 int64_t *trace, int64_t *iters, int32_t *stop, int64_t *kstar,
                 int64_t *z4, int32_t *i4, int32_t *neg, int32_t *zero)
{
    if (n < 4 || max_iters < 0 || handoff_div < 0 || !lam || check_b(n, b)) return OR_ERR_ARG;
    int rc = or_check_coords(xy, n);
    if (rc) return rc;
    int64_t *step = malloc(sizeof(int64_t) * (size_t)n);
    int64_t *best = malloc(sizeof(int64_t) * (size_t)n);
    if (!step || !best) { free(step); free(best); return OR_ERR_NOMEM; }
    int64_t rec[OR_TRACE_W];
    int64_t best_dual = INT64_MIN, best_k = -1;
    uint64_t h1 = 0, h2 = 0;   /* hashes of Lam_{k-1}, Lam_{k-2} */
    int64_t k = 0;
    int32_t why = 0;
    for (;; k++) {
        rc = or_gdp_iter(n, xy, rowptr, col, lam, b, z4, i4, neg, zero, step, rec);
        if (rc) break;
        rec[0] = k;
        if (trace) memcpy(trace + OR_TRACE_W * k, rec, sizeof(rec));
        if (rec[1] > best_dual) {
            best_dual = rec[1]; best_k = k;
            memcpy(best, lam, sizeof(int64_t) * (size_t)n);
        }
        uint64_t h = (uint64_t)rec[6];
        if (rec[3] == 0) { why = OR_STOP_TRIVIAL; break; }
        if (handoff_div > 0 && rec[2] * handoff_div <= n) { why = OR_STOP_HANDOFF; break; }
        if (rec[5] == 0) { why = OR_STOP_FIXED; break; }
        if (k >= 2 && h == h2) { why = OR_STOP_CYCLE; break; }
        if (k >= max_iters) { why = OR_STOP_CAP; break; }
        h2 = h1; h1 = h;
        for (int64_t v = 0; v < n; v++) lam[v] += step[v];
    }
    if (rc == OR_OK) {
        *iters = k + 1;
        *stop = why;
        if (why == OR_STOP_CYCLE || why == OR_STOP_CAP) {
            *kstar = best_k;
            memcpy(lam, best, sizeof(int64_t) * (size_t)n);
        } else {
            *kstar = k;
        }
    }
    free(step); free(best);
    return rc;
}

/* ------------------------------------------------------------------ */
/* certificate                                                          */
/* ------------------------------------------------------------------ */

static int cmp_pair(const void *a, const void *b)
{
    const int64_t *x = a, *y = b;
    return (x[0] > y[0]) - (x[0] < y[0]);
}

/* Checks an edge list x against Lam on the complete graph.
 *   out[0] primal2 = sum_e c_e * x2_e  (= 2 c.x)
 *   out[1] dual2   = 2*sum Lam + sum_{u<v} min(0, Z_uv)  (= 2 L)
 *   out[2] feasible: endpoints valid, u != v, x2 in {1,2}, no repeated
 *          pair, every node's sum of x2 equal to 2 b_v (degree b_v; 4 for F2M)
 *   out[3] certified = feasible && primal2 == dual2 */
int or_certify(int64_t n, const int32_t *xy, const int64_t *rowptr, const int32_t *col,
               const int32_t *b, const int64_t *lam, int64_t m,
               const int32_t *eu, const int32_t *ev, const uint8_t *ex2,
               int64_t *out)
{
    if (n < 3 || !xy || !lam || m < 0 || check_b(n, b)) return OR_ERR_ARG;
    int rc = or_check_coords(xy, n);
    if (rc) return rc;
    int feas = 1;
    int64_t primal = 0;
    int64_t *deg = calloc((size_t)n, sizeof(int64_t));
    int64_t *keys = malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!deg || !keys) { free(deg); free(keys); return OR_ERR_NOMEM; }
    for (int64_t e = 0; e < m; e++) {
        int64_t u = eu[e], v = ev[e];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v || (ex2[e] != 1 && ex2[e] != 2)) {
            feas = 0; keys[e] = -1 - e; continue;
        }
        if (rowptr) {
            int found = 0;
            for (int64_t q = rowptr[u]; q < rowptr[u + 1]; q++) if (col[q] == v) found = 1;
            if (!found) feas = 0;
        }
        primal += or_cost(xy, u, v) * ex2[e];
        deg[u] += ex2[e]; deg[v] += ex2[e];
        int64_t a = u < v ? u : v, b = u < v ? v : u;
        keys[e] = a * n + b;
    }
    qsort(keys, (size_t)m, sizeof(int64_t), cmp_pair);
    for (int64_t e = 1; e < m; e++) if (keys[e] == keys[e - 1]) feas = 0;
    for (int64_t v = 0; v < n; v++) if (deg[v] != 2 * (b ? b[v] : 2)) feas = 0;
    int64_t sbl = 0, sneg = 0;
    for (int64_t v = 0; v < n; v++) sbl += (b ? b[v] : 2) * lam[v];
#pragma omp parallel for reduction(+ : sneg) schedule(dynamic, 16)
    for (int64_t v = 0; v < n; v++) {
        const int64_t deg = rowptr ? rowptr[v + 1] - rowptr[v] : n;
        for (int64_t e = 0; e < deg; e++) {
            const int64_t u = rowptr ? col[rowptr[v] + e] : e;
            if (u <= v) continue;
            int64_t z = 2 * or_cost(xy, u, v) - lam[u] - lam[v];
            if (z < 0) sneg += z;
        }
    }
    out[0] = primal;
    out[1] = sbl + sneg;
    out[2] = feas;
    out[3] = feas && primal == out[1];
    free(deg); free(keys);
    return OR_OK;
}

/* Trivial x of Lam (eq. 7): every pair with Z <= 0, x2 = 2 if Z < 0 and 1
 * if Z == 0, listed as u < v in increasing (u, v) order.  Returns the edge
 * count, or -1 if more than cap edges exist. */
int64_t or_trivial_x(int64_t n, const int32_t *xy, const int64_t *lam, int64_t cap,
                     int32_t *eu, int32_t *ev, uint8_t *ex2)
{
    int64_t m = 0;
    for (int64_t u = 0; u < n; u++)
        for (int64_t v = u + 1; v < n; v++) {
            int64_t z = 2 * or_cost(xy, u, v) - lam[u] - lam[v];
            if (z > 0) continue;
            if (m >= cap) return -1;
            eu[m] = (int32_t)u; ev[m] = (int32_t)v; ex2[m] = z < 0 ? 2 : 1;
            m++;
        }
    return m;
}

/* ------------------------------------------------------------------ */
/* exact optimum: min-cost flow on the bipartite double cover           */
/* ------------------------------------------------------------------ */

/* Successive shortest paths with potentials (Dijkstra on reduced costs),
 * dense arrays, complete graph.  Node ids: left v -> v, right v -> n + v.
 * Flow y[v*n + u] in {0,1} on arc v' -> u''.  Reduced cost of v' -> u'' is
 * c_vu + pot(v') - pot(u'').  Returns 2*opt in *opt2, and optionally the
 * optimal x as x2[v*n+u] = y_vu + y_uv (u != v) and an optimal Lam: with
 * alpha_v = -pot(v'), beta_v = pot(v'') optimal duals of the double cover,
 * lambda = (alpha + beta)/2 is optimal for F2M by the symmetry of the cover,
 * so Lam_v = pot(v'') - pot(v').  x2 and lam may be NULL. */
int or_exact_opt2(int64_t n, const int32_t *xy, const int64_t *rowptr, const int32_t *col,
                  const int32_t *b, int64_t *opt2, uint8_t *x2, int64_t *lam)
{
    if (n < 2 || !xy || !opt2 || check_b(n, b)) return OR_ERR_ARG;
    int rc = or_check_coords(xy, n);
    if (rc) return rc;
    int64_t N = 2 * n;
    int64_t *c = malloc(sizeof(int64_t) * (size_t)(n * n));
    uint8_t *y = calloc((size_t)(n * n), 1);
    int64_t *pot = calloc((size_t)N, sizeof(int64_t));
    int64_t *dist = malloc(sizeof(int64_t) * (size_t)N);
    int64_t *prev = malloc(sizeof(int64_t) * (size_t)N);
    uint8_t *done = malloc((size_t)N);
    int64_t *exl = malloc(sizeof(int64_t) * (size_t)n);   /* remaining supply of v' */
    int64_t *dfr = malloc(sizeof(int64_t) * (size_t)n);   /* remaining demand of u'' */
    if (!c || !y || !pot || !dist || !prev || !done || !exl || !dfr) {
        rc = OR_ERR_NOMEM; goto out;
    }
    const int64_t INF = INT64_MAX / 4;
    for (int64_t v = 0; v < n; v++)
        for (int64_t u = 0; u < n; u++) c[v * n + u] = (u == v || rowptr) ? INF : or_cost(xy, u, v);
    if (rowptr)
        for (int64_t v = 0; v < n; v++)
            for (int64_t q = rowptr[v]; q < rowptr[v + 1]; q++) c[v * n + col[q]] = or_cost(xy, col[q], v);
    /* potentials: pot(v') = 0, pot(u'') = min_v c_vu, so every reduced cost
     * c_vu + pot(v') - pot(u'') is >= 0 */
    for (int64_t u = 0; u < n; u++) {
        int64_t mn = INF;
        for (int64_t v = 0; v < n; v++) if (c[v * n + u] < mn) mn = c[v * n + u];
        pot[n + u] = mn < INF ? mn : 0;
    }
    int64_t units = 0;   /* every copy has degree b_v: sum_v b_v augmentations */
    for (int64_t v = 0; v < n; v++) { exl[v] = b ? b[v] : 2; dfr[v] = exl[v]; units += exl[v]; }
    int64_t total = 0;
    for (int64_t it = 0; it < units; it++) {
        /* multi-source Dijkstra from every left copy with supply left */
        for (int64_t i = 0; i < N; i++) { dist[i] = INF; prev[i] = -1; done[i] = 0; }
        for (int64_t v = 0; v < n; v++) if (exl[v] > 0) dist[v] = 0;
        int64_t target = -1;
        for (;;) {
            int64_t a = -1, best = INF;
            for (int64_t i = 0; i < N; i++) if (!done[i] && dist[i] < best) { best = dist[i]; a = i; }
            if (a < 0) break;
            done[a] = 1;
            if (a >= n && dfr[a - n] > 0) { target = a; break; }
            if (a < n) {                      /* forward arcs a' -> u'' with y = 0 */
                for (int64_t u = 0; u < n; u++) {
                    if (u == a || y[a * n + u] || c[a * n + u] >= INF) continue;
                    int64_t rcst = c[a * n + u] + pot[a] - pot[n + u];
                    int64_t d = dist[a] + rcst;
                    if (d < dist[n + u]) { dist[n + u] = d; prev[n + u] = a; }
                }
            } else {                          /* backward arcs u'' -> v' with y = 1 */
                int64_t u = a - n;
                for (int64_t v = 0; v < n; v++) {
                    if (!y[v * n + u]) continue;
                    int64_t rcst = -(c[v * n + u] + pot[v] - pot[n + u]);
                    int64_t d = dist[a] + rcst;
                    if (d < dist[v]) { dist[v] = d; prev[v] = a; }
                }
            }
        }
        if (target < 0) { rc = OR_ERR_INFEASIBLE; goto out; }
        int64_t dt = dist[target];
        /* Johnson update capped at the target distance: every residual
         * reduced cost stays >= 0 and the path found becomes tight */
        for (int64_t i = 0; i < N; i++) pot[i] += (dist[i] < dt ? dist[i] : dt);
        /* augment one unit along the tree path */
        int64_t b = target;
        while (prev[b] >= 0) {
            int64_t a = prev[b];
            if (a < n) { y[a * n + (b - n)] = 1; } else { y[b * n + (a - n)] = 0; }
            b = a;
        }
        exl[b] -= 1;
        dfr[target - n] -= 1;
    }
    for (int64_t v = 0; v < n; v++)
        for (int64_t u = 0; u < n; u++) if (y[v * n + u]) total += c[v * n + u];
    (void)0;
    *opt2 = total;   /* = 2 * optimum (sum over both copies) */
    if (lam)
        for (int64_t v = 0; v < n; v++) lam[v] = pot[n + v] - pot[v];
    if (x2)
        for (int64_t v = 0; v < n; v++)
            for (int64_t u = 0; u < n; u++)
                x2[v * n + u] = (u == v) ? 0 : (uint8_t)(y[v * n + u] + y[u * n + v]);
out:
    free(c); free(y); free(pot); free(dist); free(prev); free(done); free(exl); free(dfr);
    return rc;
}

/* k nearest neighbours of every node: the k smallest (D_uv, u), u != v,
 * in that order.  idx[k*v + j]. */
int or_knn_rows(int64_t n, const int32_t *xy, int64_t k, int64_t nrows, const int64_t *rows, int32_t *idx)
{
    if (n < 2 || k < 1 || k > n - 1 || k > 64 || !xy || !idx || !rows) return OR_ERR_ARG;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        const int64_t v = rows[r];
        int64_t bd[64], bu[64];
        for (int64_t j = 0; j < k; j++) { bd[j] = INT64_MAX; bu[j] = -1; }
        for (int64_t u = 0; u < n; u++) {
            if (u == v) continue;
            int64_t d = sq_dist(xy, u, v);
            if (!(d < bd[k - 1] || (d == bd[k - 1] && u < bu[k - 1])) && bu[k - 1] >= 0) continue;
            int64_t j = k - 1;
            while (j > 0 && (bu[j - 1] < 0 || d < bd[j - 1] || (d == bd[j - 1] && u < bu[j - 1]))) {
                bd[j] = bd[j - 1]; bu[j] = bu[j - 1]; j--;
            }
            bd[j] = d; bu[j] = u;
        }
        for (int64_t j = 0; j < k; j++) idx[k * r + j] = (int32_t)bu[j];
    }
    return OR_OK;
}

int or_knn(int64_t n, const int32_t *xy, int64_t k, int32_t *idx)
{
    if (n < 2 || !idx) return OR_ERR_ARG;
    int64_t *rows = malloc(sizeof(int64_t) * (size_t)n);
    if (!rows) return OR_ERR_NOMEM;
    for (int64_t v = 0; v < n; v++) rows[v] = v;
    int rc = or_knn_rows(n, xy, k, n, rows, idx);
    free(rows);
    return rc;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
