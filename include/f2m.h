/*
 * f2m.h -- C ABI of libf2m: the gradient descent procedure (GDP) for the
 * fractional 2-matching (F2M) LP relaxation of Euclidean TSP, on one
 * MI355X (gfx950) GPU.
 *
 * Method: Antonov, "Gradient descent procedure for solving linear
 * programming relaxations of combinatorial optimization problems in
 * parallel mode on extra large scale", arXiv 2011.08170.
 *   - F2M LP: min c.x, sum_{e in delta(v)} x_e = 2 for every node v,
 *     0 <= x <= 1 (Sec. 4).
 *   - Adjusted length v^e = c_e - lambda_u - lambda_v (eq. 9).
 *   - Gradient of lambda_v from the 2nd and 3rd shortest adjusted edges at
 *     v (eq. 10); all nodes in parallel (Sec. 5.1).
 *   - Trivial solution: x_e = 1, 1/2, 0 for v^e <0, =0, >0 (eq. 7, Sec. 4).
 *   - Output: edges with value 1 and edges with value 1/2 (Sec. 5.1).
 *
 * Number formats used throughout:
 *   coordinates  int32 pairs (x, y), city i at [2i], [2i+1]; each axis span
 *                must be below 2^20.
 *   c_e          TSPLIB EUC_2D length nint(sqrt(dx^2 + dy^2)), exact.
 *   Lam          2*lambda as int64 ("lambda2"); |Lam| must stay below 2^38.
 *   Z_e          2c_e - Lam_u - Lam_v = twice the adjusted length (eq. 9).
 *   x2           2*x_e in {1, 2} (1 = one half, 2 = one).
 *   primal2      2*c.x;  dual2 = 2*L(lambda) = 2*sum Lam + sum_{u<v} min(0, Z).
 *
 * GDP rule (rule_version 1, a reading of eq. 10 and Sec. 3): per node
 *   s = Z_(2) + Z_(3) over the node's edges (2nd and 3rd smallest),
 *   dLam = sign(s) * floor((|s| + 2) / 4)  (midpoint move damped by 1/2,
 *   rounded half away from zero), every node from the same Lam (Jacobi).
 * At iteration k the loop stops, tested in this order, when every trivial
 * degree is 2 ("trivial"); when handoff_div > 0 and (#nodes with
 * Z_(2) > 0 or Z_(3) < 0) * handoff_div <= n ("handoff": the rest is left to
 * the exact finish); when every step is 0 ("fixed"); when Lam_k equals
 * Lam_{k-2} by hash ("cycle"); at k == max_iters ("cap").
 *
 * Ownership: the caller owns every input.  Host arrays inside f2m_result
 * are allocated by the library and released by f2m_result_free.  No
 * exception or abort crosses this ABI; on error the outputs are left
 * untouched and f2m_last_error(ctx) holds a message.
 *
 * Pointers: "device" arguments are HIP device pointers on the context's
 * device; "host" arguments are ordinary host memory.  Calls on one context
 * are not thread safe; use one context per host thread.
 */
#ifndef F2M_H
#define F2M_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct f2m_ctx f2m_ctx;

typedef enum f2m_status {
    F2M_OK = 0,
    F2M_NOT_CERTIFIED = 1,   /* soft: result returned, optimality not proven */
    F2M_ERR_ARG = -1,        /* null pointer, bad size, bad option */
    F2M_ERR_RANGE = -2,      /* coordinate span >= 2^20 on an axis */
    F2M_ERR_INFEASIBLE = -3, /* n < 3: no degree-2 solution exists */
    F2M_ERR_NOMEM = -4,      /* host or device allocation failed */
    F2M_ERR_DEVICE = -5,     /* HIP runtime error */
    F2M_ERR_CAPACITY = -6,   /* caller buffer too small */
    F2M_ERR_OVERFLOW = -7    /* |Lam| reached 2^38 */
} f2m_status;

/* F2M_GRAPH_KNN: the candidate graph of Sec. 5.3 -- every node joined to
 * its knn_k nearest neighbours by (squared distance, index), union-
 * symmetrised; the GDP, the finish and the certificate run on that graph,
 * and the result is also checked against the complete graph. */
enum { F2M_GRAPH_COMPLETE = 0, F2M_GRAPH_KNN = 1 };
/* F2M_WARM_MLP: Lam_0 from the warm-start network (see f2m_mlp_forward),
 * parameters in opts.mlp_theta; the GDP, the finish and the certificate
 * are unchanged, so the certified optimum equals the cold start's.
 * F2M_WARM_GRAPH (complete graph only): Lam_0 is the Lam* of a cold GDP
 * run, with the same stop rules, on the candidate graph of Sec. 5.3
 * (knn_k nearest neighbours), and the complete-graph GDP starts from it
 * with the candidate graph's final four smallest per node as its first
 * thresholds; result.warm_iterations counts the candidate-graph iterations
 * (0 when n <= knn_k: then the start is cold).  Again only iterations and
 * time change, never the certified optimum. */
enum { F2M_WARM_COLD = 0, F2M_WARM_USER = 1, F2M_WARM_MLP = 2, F2M_WARM_GRAPH = 3 };
enum { F2M_FINISH_NONE = 0, F2M_FINISH_EXACT = 1 };
/* Scan over the complete graph: F2M_SCAN_CULLED skips column tiles whose
 * bounding box is provably too far for any pair to matter (exact: same
 * results); F2M_SCAN_FULL tests every ordered pair. */
enum { F2M_SCAN_CULLED = 0, F2M_SCAN_FULL = 1 };
/* Scan kinds of the complete-graph GDP (f2m_result.scan_kind).  A list scan
 * evaluates each row's candidate list from the last building scan only; it
 * runs only while that is provably exact, so every kind gives the same bits.
 * On a list iteration the update kernel evaluates the lists and the scan
 * launch exits at once. */
enum { F2M_SCAN_KIND_FULL = 0, F2M_SCAN_KIND_BUILD = 1, F2M_SCAN_KIND_LIST = 2 };
enum { F2M_STOP_TRIVIAL = 1, F2M_STOP_FIXED = 2, F2M_STOP_CYCLE = 3, F2M_STOP_CAP = 4,
       F2M_STOP_HANDOFF = 5 };

/* Per-iteration record, F2M_TRACE_W int64 per iteration k:
 *   [0] k  [1] dual2 at Lam_k  [2] #nodes with Z_(2) > 0 or Z_(3) < 0
 *   [3] #nodes whose trivial doubled degree is not 4  [4] max |dLam|
 *   [5] #nonzero steps  [6] order-free hash of Lam_k (uint64 bits)
 *   [7] sum of Lam_k */
#define F2M_TRACE_W 8

typedef struct f2m_opts {
    uint32_t struct_size;         /* sizeof(f2m_opts) */
    uint32_t rule_version;        /* must be 1 */
    int32_t graph;                /* F2M_GRAPH_COMPLETE or F2M_GRAPH_KNN */
    int32_t knn_k;                /* neighbours per node for F2M_GRAPH_KNN: 10 or 16 */
    int32_t warm;                 /* F2M_WARM_COLD (Lam0 = 0), _USER, _MLP or _GRAPH */
    const int64_t *lambda2_init;  /* host, n entries, read when warm == USER */
    const float *mlp_theta;       /* device, F2M_MLP_PARAMS floats, read when warm == MLP */
    int64_t max_iters;            /* iteration cap (>= 0) */
    int64_t handoff_div;          /* hand-off stop (see above); 0 disables it */
    int32_t finish;               /* F2M_FINISH_EXACT: make the result exact
                                     when the trivial x does not certify */
    int32_t coords_on_device;     /* coords_xy argument is a device pointer */
    int32_t record_trace;         /* fill f2m_result.trace */
    int32_t chunk;                /* f2m_solve: iterations queued ahead of the last one the
                                     device has finished; f2m_solve_batch: iterations per
                                     replayed graph (0: auto) */
    int32_t time_kernels;         /* time every scan launch with HIP events */
    int32_t scan_mode;            /* F2M_SCAN_CULLED (default) or F2M_SCAN_FULL */
    int32_t scan_rows;            /* launch shape: rows per lane, 1, 2 or 4 (0: built-in choice) */
    int32_t scan_slices;          /* launch shape: column slices >= 1 (0: built-in choice);
                                     the shape never changes a result, only the time */
    void *hip_stream;             /* hipStream_t to run on; NULL: the context's stream */
    /* Resume (checkpoint = f2m_result.lambda2_last after a run that stopped
     * at iteration K): warm = F2M_WARM_USER with lambda2_init = Lam_K and
     * k0 = K continues the GDP at iteration K.  With resume_hash_valid the
     * hashes of Lam_{K-1} and Lam_{K-2} (trace column 6 of rows K-1, K-2)
     * arm the cycle test at once, so the records and the stop equal those
     * of the uninterrupted run; Lam* of a cycle or cap stop is then the
     * largest-dual iterate since K.  k0 = 0: a fresh run. */
    int64_t k0;                   /* 0 <= k0 <= max_iters; k0 > 0 needs warm == F2M_WARM_USER */
    uint64_t resume_hash[2];      /* hash of Lam_{k0-1}, of Lam_{k0-2} */
    int32_t resume_hash_valid;    /* 1: resume_hash holds them (needs k0 >= 2) */
    int32_t pad_opts;
    uint64_t max_device_bytes;    /* cap on the context's device workspace (0: none);
                                     a call that would pass it fails with F2M_ERR_NOMEM */
    const char *tuner_cache;      /* path of a tuner cache, or NULL.  Text, one entry per line,
                                     tab-separated: device name (f2m_device_name), mode
                                     ("culled", "full", "batch-culled", "batch-full"), size
                                     bucket (the integer nearest 2 log2 n, exactly
                                     floor(bitlength(n^4) / 2); the batch uses the total node
                                     count), rows, slices, chunk; 0 keeps the built-in value;
                                     '#' lines are comments.  f2m_solve takes the entry for
                                     its device, scan mode and n when scan_rows == scan_slices
                                     == 0 (complete graph); f2m_solve_batch when scan_slices
                                     == 0; chunk applies when opts.chunk == 0.  A missing
                                     file or entry leaves the built-in shape. */
    /* Rows with other right-hand sides (Sec. 3: binary rows, integral b; here
     * the fractional b-matching): host, n entries by label, each 1, 2 or 3,
     * or NULL for 2 everywhere (F2M).  Node v then needs degree b_v: the
     * GDP steps on the b_v-th and (b_v+1)-th smallest Z, a node is
     * unsatisfied when Z_(b) > 0 or Z_(b+1) < 0, its trivial doubled degree
     * must be 2 b_v, dual2 = sum_v b_v Lam_v + sum_e min(0, Z_e), and the
     * finish and the certificate use degree b_v.  The x is always made by the
     * exact finish (finish == EXACT; else NOT_CERTIFIED).  f2m_solve only,
     * n >= 4, cold or user warm start. */
    const int32_t *degree_b;
} f2m_opts;

typedef struct f2m_result {
    int64_t n;
    int64_t iterations;     /* GDP iterations evaluated (records) */
    int64_t kstar;          /* index of the GDP iterate the finish started from */
    int32_t stop;           /* F2M_STOP_* */
    int32_t certified;      /* primal2 == dual2 with a feasible x on the solved graph */
    int64_t *lambda2;       /* host, n: the final Lam (the certificate's duals) */
    int64_t *lambda2_gdp;   /* host, n: the GDP iterate Lam_kstar */
    int64_t n_edges;
    int32_t *edge_u;        /* host, n_edges, edge_u < edge_v */
    int32_t *edge_v;
    uint8_t *edge_x2;       /* 2 = value 1, 1 = value 1/2 */
    int64_t primal2;        /* 2 c.x of the returned x */
    int64_t dual2;          /* 2 L(lambda2) on the complete graph */
    int64_t dual2_gdp;      /* 2 L(lambda2_gdp) */
    int64_t finish_paths;   /* augmenting paths used by the exact finish */
    int64_t finish_rounds;  /* pricing rounds of the exact finish */
    int64_t trace_len;
    int64_t *trace;         /* host, trace_len * F2M_TRACE_W, or NULL */
    double seconds[6];      /* setup, warm start (network or candidate-graph GDP),
                               gdp, finish, certify, total */
    double scan_ms;         /* summed duration of the scan launches (time_kernels) */
    int64_t scan_launches;  /* scan launches timed */
    int32_t scan_rows;      /* scan launch shape: rows per lane */
    int32_t pad0;
    int64_t scan_slices;    /* scan launch shape: column slices */
    int64_t scan_pairs;     /* ordered pairs the GDP scans evaluated (culled tiles excluded) */
    int64_t finish_phases;      /* Dijkstra phases of the exact finish */
    int64_t finish_candidates;  /* candidate pairs of the exact finish at the end */
    double finish_seconds[3];   /* exact finish: pair collection (GPU), candidate build, flow */
    int64_t dual2_complete;     /* 2 L(lambda2) on the complete graph */
    int32_t certified_complete; /* x is also optimal for the complete graph */
    int32_t pad1;
    int64_t graph_nnz;          /* directed entries of the candidate graph (F2M_GRAPH_KNN, F2M_WARM_GRAPH) */
    int64_t warm_iterations;    /* GDP iterations of the F2M_WARM_GRAPH start (0 otherwise) */
    int32_t *scan_kind;         /* host, trace_len, or NULL: the scan of iteration k tested every
                                   surviving pair (F2M_SCAN_KIND_FULL), also stored candidate lists
                                   (_BUILD), or evaluated the lists only (_LIST) */
    int64_t scan_list_uses;     /* GDP scans that evaluated the candidate lists only */
    int64_t scan_list_builds;   /* GDP scans that built candidate lists */
    int64_t *lambda2_last;      /* host, n: Lam of the last evaluated iteration (the checkpoint
                                   to resume from, see f2m_opts.k0) */
    double scan_ms_kind[3];     /* scan_ms split by F2M_SCAN_KIND_* (time_kernels) */
    int64_t scan_launches_kind[3];
    int64_t scan_pairs_kind[3]; /* scan_pairs split by F2M_SCAN_KIND_* */
    double update_ms;           /* summed duration of the update launches (time_kernels); on a
                                   F2M_SCAN_KIND_LIST iteration the update evaluates the lists
                                   and the scan launch exits at once */
    double update_ms_kind[3];   /* update_ms split by the iteration's F2M_SCAN_KIND_* */
} f2m_result;

/* Fills opts with the defaults: rule 1, complete graph, cold start,
 * knn_k 10, max_iters 100000, handoff_div 50, exact finish, host coords,
 * no trace, auto chunk, culled scan, k0 0, no memory cap, no tuner cache. */
void f2m_opts_default(f2m_opts *opts);

/* Creates a context on HIP device `device` with its own stream.  defaults
 * (may be NULL: f2m_opts_default) is copied and used by every call of this
 * context that is given opts == NULL.  F2M_ERR_ARG for a bad struct_size,
 * F2M_ERR_DEVICE when the device does not exist or HIP fails. */
f2m_status f2m_create(f2m_ctx **ctx, int device, const f2m_opts *defaults);
void f2m_destroy(f2m_ctx *ctx);

/* Full solve of F2M on the complete graph of n cities (Sec. 4, 5.1):
 * GDP loop, then the trivial x (eq. 7) when every trivial degree is 2, else
 * (finish == EXACT) a primal-dual finish on the bipartite double cover
 * started from the GDP multipliers, then the certificate.
 *   coords_xy  host (or device, see opts) int32[2n]
 *   out        receives library-allocated host arrays
 * Returns F2M_OK when certified, F2M_NOT_CERTIFIED when the result holds
 * a valid bound but no proof (finish == NONE), or an error. n == 3 is
 * solved in closed form; n < 3 returns F2M_ERR_INFEASIBLE. */
f2m_status f2m_solve(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n,
                     const f2m_opts *opts, f2m_result *out);

/* Many independent instances in one batched GDP loop: every iteration is
 * one scan launch and one update launch over all instances (work items
 * instance x row block x column slice, a control block and stop test per
 * instance), a chunk of iterations is captured once as a HIP graph and
 * replayed until every instance has stopped; then each instance gets its
 * finish and certificate.  Results equal independent f2m_solve calls.
 *   coords   host int32, instance i at coords[2*offsets[i] .. 2*offsets[i+1])
 *   offsets  host int64[n_inst+1], offsets[0] = 0, every size >= 3
 *   opts     as for f2m_solve (complete graph, host coordinates); a
 *            USER warm start reads lambda2_init[offsets[i] + v]
 *   outs     host array of n_inst results (free each with f2m_result_free)
 * Returns F2M_OK when every instance is certified. */
f2m_status f2m_solve_batch(f2m_ctx *ctx, const int32_t *coords, const int64_t *offsets, int32_t n_inst,
                           const f2m_opts *opts, f2m_result *outs);

/* One GDP iteration (eq. 9, eq. 10, Jacobi) on device buffers, n >= 4:
 *   coords_xy   device int32[2n]
 *   lambda2_in  device int64[n]  (Lam_k)
 *   lambda2_out device int64[n]  (Lam_k + dLam), may not alias lambda2_in
 *   z4, i4      device int64[4n], int32[4n] or NULL: the four smallest
 *               (Z, u) of each row in (Z, u) order, entry j of node v at
 *               [4v + j]
 *   neg, zero   device int32[n] or NULL: #{Z < 0}, #{Z == 0} per node
 *   step        device int64[n] or NULL: dLam
 *   rec         host int64[F2M_TRACE_W]: the iteration record (k = 0)
 * Runs on the context's stream and waits for it. */
f2m_status f2m_gdp_step(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n,
                        const int64_t *lambda2_in, int64_t *lambda2_out,
                        int64_t *z4, int32_t *i4, int32_t *neg, int32_t *zero,
                        int64_t *step, int64_t rec[F2M_TRACE_W]);

/* f2m_gdp_step for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it):
 * the same iteration, arguments and results as f2m_gdp_step, with every
 * workspace buffer taken from one fixed device array of 32 MiB that the
 * library holds on each device it runs on until the process ends.  It
 * calls no hipMalloc, hipFree or other allocating routine.
 *   n           4 <= n <= F2M_NOALLOC_MAX_N; larger n returns
 *               F2M_ERR_CAPACITY before any work is queued
 * Every call on one device, from any context, uses the same array and
 * finds the previous call's contents there (each call initialises what it
 * reads): calls that overlap on one device race and must be serialised by
 * the caller.  Runs on the context's stream and waits for it. */
#define F2M_NOALLOC_MAX_N 131072
f2m_status f2m_gdp_step_noalloc(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n,
                                const int64_t *lambda2_in, int64_t *lambda2_out,
                                int64_t *z4, int32_t *i4, int32_t *neg, int32_t *zero,
                                int64_t *step, int64_t rec[F2M_TRACE_W]);

/* Certificate on the complete graph (weak/strong duality of Sec. 2):
 *   coords_xy device int32[2n]; lambda2 device int64[n];
 *   eu, ev, ex2 device arrays of m edges.
 *   out host int64[4]: primal2, dual2, feasible (every x2 in {1,2}, u != v,
 *   endpoints in range, no repeated pair, every doubled degree 4),
 *   certified (feasible and primal2 == dual2). */
f2m_status f2m_certify(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n,
                       const int64_t *lambda2, int64_t m, const int32_t *eu,
                       const int32_t *ev, const uint8_t *ex2, int64_t out[4]);

/* The candidate graph of F2M_GRAPH_KNN as CSR over labels: row v lists
 * every u with u among the k nearest neighbours of v or v among those of u
 * (k nearest by squared distance, then index), columns increasing.
 *   coords_xy device int32[2n]; k is 10 or 16; n > k.
 *   rowptr device int32[n+1]; col device int32[cap]; *nnz (host) receives
 *   the entry count.  F2M_ERR_CAPACITY (nnz set) when cap < nnz. */
f2m_status f2m_knn_graph(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n, int32_t k,
                         int32_t *rowptr, int32_t *col, int64_t cap, int64_t *nnz);

/* Warm-start network (not in the paper): per node v the features
 * x_v = (d_1, ..., d_16) / s, d_j the distance to the j-th nearest
 * neighbour (by squared distance, then index) and s the median of all
 * n*16 such distances; an MLP 16 -> 128 -> 128 -> 1 with ReLU, BF16
 * operands on the matrix cores and FP32 accumulation, predicts
 * y_v ~ lambda_v / s; Lam_0,v = round-half-even(2 s y_v).
 * Parameters: FP32 vector of F2M_MLP_PARAMS entries, in this order:
 * W1[128][16], b1[128], W2[128][128], b2[128], w3[128], b3. */
#define F2M_MLP_PARAMS 18817

/* coords_xy device int32[2n], n >= 17; feat device uint16[16n] (bf16,
 * row v = label v); *scale (host) receives s. */
f2m_status f2m_features(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n, uint16_t *feat, float *scale);
/* theta, feat, y device arrays; y[v] = network output for row v. */
f2m_status f2m_mlp_forward(f2m_ctx *ctx, const float *theta, const uint16_t *feat, int64_t n, float *y);
/* Gradient of the mean squared error mean_v (y_v - target_v)^2 over the n
 * rows: grad (device, F2M_MLP_PARAMS floats), *loss (host). */
f2m_status f2m_mlp_grad(f2m_ctx *ctx, const float *theta, const uint16_t *feat, const float *target, int64_t n,
                        float *grad, double *loss);
/* One AdamW step (beta1 0.9, beta2 0.999, eps 1e-8, decoupled decay wd)
 * on device arrays of F2M_MLP_PARAMS floats; step counts from 1. */
f2m_status f2m_mlp_adamw(f2m_ctx *ctx, float *theta, const float *grad, float *m, float *v, int64_t step, float lr,
                         float wd);

/* ---- Subtour-elimination rows (F2M + SEC) ------------------------------
 * The extension of Sec. 5: F2M plus rows x(delta(S_q)) >= 2 for node sets
 * S_q (2 <= |S_q| <= n - 2), delta(S) the edges with one end in S.  Such a
 * row enters the Lagrangian with a multiplier lambda_q >= 0 (Sec. 2,
 * eq. 4-5) and moves by the gradient of Sec. 3 with b = 2 over its edges,
 * then is projected back onto lambda_q >= 0.  Fixed point: M_q = 2 lambda_q
 * (int64, >= 0) and, for an edge e = {u, v},
 *   Z_e = 2c_e - Lam_u - Lam_v - sum_{q: e in delta(S_q)} M_q      (eq. 9)
 *   dual2 = 2 sum Lam + 2 sum M + sum_{u<v} min(0, Z).
 * Step of a row q: s = Z_(2) + Z_(3) over delta(S_q), M_q <- max(0, M_q +
 * sign(s) floor((|s| + 4) / 8)): the midpoint move s/2 divided by the four
 * rows that move a crossing edge at once (its two degree rows and the
 * layer's rows of its two ends), where a degree row's s/4 divides by two;
 * nodes step as in F2M, all rows from the same iterate.  Record fields as F2M_TRACE_W plus [8] sum of M_k; a row
 * is unsatisfied when Z_(2) > 0, or M_q > 0 and Z_(3) < 0; it is bad when
 * its trivial doubled crossing degree 2#(Z<0) + #(Z=0) is below 4, or
 * M_q > 0 and that degree is not 4.  The state hash indexes node v by v
 * and row q by n + q.  Stops as F2M without the hand-off: trivial, fixed,
 * cycle, cap; at cycle and cap the result is the largest-dual iterate.
 *
 * Rows are given in layers: within a layer the row sets are disjoint, so
 * an edge crosses at most two rows of a layer (the rows of its two ends).
 * row_of: device int32[nlayers * n] by label; row_of[l n + v] in [0, nrows)
 * is the row of layer l whose set holds v, -1 none.  Every row id occurs in
 * exactly one layer, on 2 .. n - 2 nodes.  delta(S) = delta(V - S), so a
 * row may be given by either side. */
#define F2M_SEC_MAX_LAYERS 8
#define F2M_SEC_TRACE_W 9

typedef struct f2m_sec_rows {
    int32_t nlayers;              /* 0 .. F2M_SEC_MAX_LAYERS */
    int32_t reserved;             /* 0 */
    int64_t nrows;                /* rows numbered 0 .. nrows - 1 */
    const int32_t *row_of;        /* device, see above (may be null when nlayers == 0) */
} f2m_sec_rows;

typedef struct f2m_sec_result {
    int64_t iterations;           /* iterations evaluated */
    int64_t kstar;                /* iteration of (Lam*, M*) */
    int32_t stop;                 /* F2M_STOP_TRIVIAL, _FIXED, _CYCLE or _CAP */
    int32_t overflow;             /* 1: stopped because |Lam| + sum M could pass 2^38 */
    int64_t dual2;                /* dual2 at (Lam*, M*) */
    int64_t primal2_last;         /* 2 c.x of the trivial x at the last iterate */
    int64_t bad_last;             /* bad rows (nodes and subtour rows) at the last iterate */
    double seconds;
    int64_t pairs_tested;         /* ordered pairs the scans tested with the float filter (the
                                     culled tiles and sub-tiles excluded), all iterations */
} f2m_sec_result;

/* GDP with subtour rows from (Lam_0, M_0).
 *   coords_xy device int32[2n], n >= 4; rows as above (nrows <= 2^31 - 1).
 *   lambda2 device int64[n] by label: in Lam_0, out Lam*.
 *   mu device int64[nrows]: in M_0 (every entry >= 0, else F2M_ERR_ARG),
 *   out M*.  max_iters >= 0.
 *   trace host int64[trace_cap][F2M_SEC_TRACE_W] or null: records of
 *   iterations 0 .. min(iterations, trace_cap) - 1.
 * Status F2M_OK (also when stopped by cycle or cap: the bound is valid for
 * any iterate), F2M_ERR_OVERFLOW when the multipliers grow past the range
 * (out->overflow set; Lam* and M* are still returned).  The context keeps
 * a device workspace of about (60 + 44 L) S + 100 + 60 L bytes per node
 * (L = nlayers rounded up to 1, 2, 4 or 8; S = column slices, 1 from
 * n = 262k up, more below so that small instances fill the GPU). */
f2m_status f2m_sec_gdp(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n, const f2m_sec_rows *rows,
                       int64_t *lambda2, int64_t *mu, int64_t max_iters, int64_t *trace, int64_t trace_cap,
                       f2m_sec_result *out);

/* Certificate of the trivial x of (Lam, M) (eq. 7 with the Z above):
 * out host int64[5] = primal2, dual2, feasible (every doubled degree 4 and
 * every row's doubled crossing degree >= 4), tight (every row with
 * M_q > 0 has crossing degree exactly 4), certified (feasible, tight and
 * primal2 == dual2: then x is optimal for F2M with these rows). */
f2m_status f2m_sec_certify(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n, const f2m_sec_rows *rows,
                           const int64_t *lambda2, const int64_t *mu, int64_t out[5]);

/* Separation: the connected components of the support of the trivial x of
 * (Lam, M) (the edges with Z <= 0).  When there are two or more, each
 * component S is a violated row x(delta(S)) = 0 < 2; it becomes a new row
 * when 2 <= |S| <= n - 2 and its cut is not already a row (given, or an
 * earlier component: with two components both give one cut).  New rows
 * are numbered rows->nrows, rows->nrows + 1, ... in order of their
 * components' smallest labels and written as one new layer:
 *   new_row_of device int32[n] by label (-1 for nodes in no new row);
 *   *new_rows (host) their count, *components (host) the component count. */
f2m_status f2m_sec_separate(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n, const f2m_sec_rows *rows,
                            const int64_t *lambda2, const int64_t *mu, int32_t *new_row_of,
                            int64_t *new_rows, int64_t *components);

/* Rounds of separation and GDP from a given Lam (e.g. an F2M solution's):
 * round r separates at the current (Lam, M), adds the new rows as layer
 * nlayers0 + r with M = 0, and runs f2m_sec_gdp from there; it ends when
 * no new row is found, after max_rounds rounds, when the layers or mu_cap
 * are full, or when the GDP overflows.
 *   lambda2 device int64[n]: in the start, out the last round's Lam*.
 *   row_of device int32[F2M_SEC_MAX_LAYERS * n]: layers 0 .. nlayers0 - 1
 *   hold given rows (nrows0 of them), the rounds append theirs.
 *   mu device int64[mu_cap]: entries 0 .. nrows0 - 1 hold their M.
 *   res host: per round r < rounds the rows added, the GDP's iterations,
 *   stop and dual2 (at its Lam*); nlayers and nrows at the end; the best
 *   dual2 over the start and every round (a lower bound on twice the
 *   shortest tour); certified: the last round's trivial x is certified. */
typedef struct f2m_sec_solve_result {
    int32_t rounds;
    int32_t nlayers;
    int64_t nrows;
    int64_t rows_added[F2M_SEC_MAX_LAYERS];
    int64_t iterations[F2M_SEC_MAX_LAYERS];
    int32_t stop[F2M_SEC_MAX_LAYERS];
    int64_t dual2[F2M_SEC_MAX_LAYERS];
    int64_t dual2_start;          /* dual2 at the start (its given rows and M) */
    int64_t best_dual2;
    int32_t certified;
    int32_t components;           /* components at the last separation */
    double seconds;
} f2m_sec_solve_result;

f2m_status f2m_sec_solve(f2m_ctx *ctx, const int32_t *coords_xy, int64_t n, int64_t *lambda2, int32_t *row_of,
                         int32_t nlayers0, int64_t nrows0, int64_t *mu, int64_t mu_cap, int32_t max_rounds,
                         int64_t max_iters, f2m_sec_solve_result *res);

void f2m_result_free(f2m_result *res);
const char *f2m_status_str(f2m_status s);
const char *f2m_last_error(const f2m_ctx *ctx);
/* Name of the context's device (hipDeviceProp_t::name; "" if unknown): the
 * device field of tuner-cache entries.  The string lives as long as ctx. */
const char *f2m_device_name(const f2m_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* F2M_H */
