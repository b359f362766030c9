// Internal interface between the HIP kernels (f2m_kernels.hip) and the host
// runtime (f2m_api.cpp).  Not part of the public ABI.
//
// Internal order.  Cities are relabelled by a Morton (Z-order) sort of their
// coordinates; "position" p in [0, n) is the sorted index, orig[p] the
// caller's label.  Scans run over positions (spatially compact row blocks
// and column tiles), while every tie-break, output and hash uses labels, so
// results do not depend on the order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f2m {

// Largest |Lam| accepted; keeps |Z| < 2^40 and every float in the scan
// filter finite.
constexpr int64_t kLamLimit = int64_t(1) << 38;
// Threshold meaning "no bound yet": larger than any |Z|.
constexpr int64_t kThetaNone = int64_t(1) << 40;
constexpr int kTraceW = 8;
// Entries kept per row: the four smallest (Z, u).
constexpr int kTop = 4;
// Columns per LDS tile; also the alignment of row blocks and slices.
constexpr int kTileCols = 256;
// Tiles are cut in sub-tiles of kSubCols positions for finer culling.  The
// per-tile arrays (boxes, maxima of h) hold kBoxStride entries per tile:
// entry 0 covers the whole tile, entry 1 + s its sub-tile s.
constexpr int kSubCols = 32;
constexpr int kSubs = kTileCols / kSubCols;
constexpr int kBoxStride = 1 + kSubs;

// Device-resident control block of the GDP loop.  A one-block control
// kernel after each update launch sums the update blocks' slots, writes the
// iteration record and takes the stop decision (see control_body).  Every
// field is 64 bits wide: the control kernel reads and writes the block as
// an array of words.
struct Ctrl {
    // loop state
    long long done;        // 1 once the loop has stopped
    long long stop;        // F2M_STOP_* or 0
    long long k_last;      // last evaluated iteration
    long long kstar;       // iterate the loop stops on
    long long best_dual2;
    long long best_k;
    unsigned long long h1, h2;   // hashes of Lam_{k-1}, Lam_{k-2}
    long long max_iters;
    long long maxabs_lam;  // max |Lam_k| of the iterate being scanned
    long long overflow;    // 1 if |Lam_{k+1}| reached kLamLimit
    long long trace_cap;
    long long dual2_last;  // dual2 of Lam_{k_last}
    long long handoff_div; // hand-off stop: #unsat * div <= n (0: off)
    unsigned long long pairs_tested;   // ordered pairs the GDP scans evaluated (all iterations)
    long long k_next;      // iteration the next update evaluates (batched, graph-replayed loops)
    long long nblocks;     // blocks of this instance's update launch (batched loops)
    // candidate lists of the culled one-row-per-lane scan (see ScanArgs::lst)
    long long list_ok;     // 1: the next scan evaluates the lists only
    long long list_d;      // sum of the max steps since the lists were built
    long long list_D;      // the next build keeps Z <= theta + 2 list_D (0: no build)
    long long list_over;   // a list overflowed in the building scan
    long long list_ms0;    // max step of iteration 0
    long long list_Dmax;   // margins above this overflowed (half the last one that did; 0: none yet)
    long long k_first;     // first iteration of this run (a resumed run starts at k0)
    long long hvalid;      // h1, h2 were given for k_first - 1, k_first - 2 (resume)
    unsigned long long pairs_kind[3];   // pairs_tested split by the scans' ScanKind
    long long list_uses;   // scans that evaluated the lists only
    long long list_builds; // scans that built lists
    long long ms_last;     // max |Lam_{k+1} - Lam_k| of the last iteration k
};

// Blocks of an update launch leave their part of the iteration record in
// their own slot of kSlotW 64-bit words, which the control kernel sums.
constexpr int kSlotW = 16;
// Kind of the scan of an iteration (UpdateArgs::scan_kind)
enum ScanKind { kScanFull = 0, kScanBuild = 1, kScanList = 2 };

// Static geometry of an instance in sorted order.
struct Geo {
    int64_t n;
    const int32_t *orig;        // position -> label
    const int32_t *pos;         // label -> position
    const float4 *box;          // per tile and sub-tile (kBoxStride per tile): xmin, xmax, ymin, ymax
    float xy2max;               // >= max over cities of x^2 + y^2 (centred)
    // by position: the right-hand side b_v of each node's degree row (1, 2
    // or 3: the b-matching of Sec. 3), or null for 2 everywhere (F2M)
    const int8_t *b = nullptr;
};

// Column records, one per position: centred coordinates, h = Lam/2 and
// q = x^2 + y^2 - h^2 (float4 {x, y, h, q}), plus the per-tile maximum of h.
struct LamView {
    const float4 *col;
    const int64_t *lam;         // Lam in sorted order
    const float *tile_hmax;     // per tile and sub-tile (kBoxStride per tile): max h
    const Ctrl *ctrl;           // maxabs_lam (and done for the GDP loop)
};

enum ScanMode { kModeGdp = 0, kModeCert = 1, kModeCollect = 2 };

struct ScanArgs {
    Geo g;
    LamView lv;
    int64_t slice_len;          // columns per slice (blockIdx.y), multiple of kTileCols
    int cull;                   // skip column tiles that cannot hold a passing pair
    int check_done;             // GDP loop: exit at once when ctrl->done
    const int64_t *lam_odd;     // batched loop: Lam_k for odd k (lv.lam holds even k)
    unsigned long long *tested; // if set: += ordered pairs evaluated (culled tiles excluded)
    const int32_t *seed;        // [j][n] positions bounding the 4th smallest Z, or null
    // GDP mode: partial results per (slice, position), structure of arrays
    int64_t *pz;                // [slice][4][n]
    int32_t *pi;                // [slice][4][n]  (labels)
    int32_t *pneg;              // [slice][n]
    int32_t *pzero;             // [slice][n]
    int64_t *prowneg;           // [slice][n]
    // certificate mode
    unsigned long long *acc;    // [0] += sum of min(0, Z) over ordered pairs
    // collect mode: pairs (Morton positions), lo < hi, with Z <= theta_row
    int64_t theta;              // threshold when no seed bound exists
    int64_t slack;              // added to the seeded bound
    unsigned long long *count;
    int2 *out;
    int64_t cap;
    // collect mode, optional: sorted keys (lo << 32 | hi, positions) of pairs
    // not to emit (the finish's candidates already known)
    const uint64_t *excl;
    int64_t nexcl;
    // GDP mode, optional: pflag[slice * nrb + row block] = 1 when the block
    // had a column tile to scan; a block without one writes no partials
    int32_t *pflag;
    int64_t nrb;                // row blocks of the launch
    // culled scan: > 0 = the number of slices, each of which scans every
    // interleave-th of the row block's surviving column tiles (over all
    // columns; slice_len is then not used); 0 = slice s scans columns
    // [s * slice_len, (s + 1) * slice_len)
    int64_t interleave;
    // GDP mode, culled, one row per lane, optional: candidate lists.  A
    // full scan with ctrl->list_D > 0 keeps, per row, every column it finds
    // with Z <= theta + 2 D (at most kLW per part, the four waves of the
    // row's block being the parts); the block writes them compacted: row p
    // of 64-row group g (slice s) has lcnt[s n + p] entries (-1: a part
    // overflowed) at lst[(s G + g) kListCap + loff[s n + p] ...], G the
    // number of groups, the group's rows one after another.  While
    // ctrl->list_ok the update evaluates only the lists (exact as long as
    // the steps since the build sum to at most D / 2) and the scan exits
    int32_t *lst;
    int32_t *lcnt;
    int32_t *loff;
    // GDP mode, culled, one row per lane, optional: each workgroup stores
    // its ordered pairs tested in tpart[slice * groups + group] (groups of
    // 64 rows) instead of adding them to *tested; k_update sums them
    unsigned long long *tpart;
};

struct UpdateArgs {
    Geo g;
    int64_t nslices;
    int64_t k;                  // iteration index
    const int64_t *pz;
    const int32_t *pi;
    const int32_t *pneg;
    const int32_t *pzero;
    const int64_t *prowneg;
    const int64_t *lam_in;      // Lam_k, sorted
    int64_t *lam_out;           // Lam_{k+1}, sorted; holds Lam_{k-1} on entry
    int64_t *lam_best;          // sorted copy of the best-dual iterate
    float4 *col;                // h, q rewritten for Lam_{k+1}
    float *tile_hmax;           // per tile and sub-tile max h of Lam_{k+1} (kBoxStride per tile)
    int64_t *z4;                // [4n] by label (4v + j)
    int32_t *i4;                // [4n] by label, entries are labels
    int32_t *seed;              // [j][n] positions of the top-4, for the next scan
    int32_t *neg;               // [n] by label, or null
    int32_t *zero;              // [n] by label, or null
    int64_t *step;              // [n] by label, or null
    Ctrl *ctrl;
    int64_t *trace;             // [trace_cap][8] or null
    // optional: the scan's flags (see ScanArgs); slices without one are skipped
    const int32_t *pflag;
    int64_t nrb;
    int64_t scan_rows;          // rows per lane of the scan (tiles per scan row block)
    int lists;                  // the scan keeps candidate lists: track their drift
    // optional: the scan's pairs tested per (slice, group of 64 rows), added
    // to ctrl->pairs_tested by the last block
    const unsigned long long *tpart;
    // per-block record slots, kSlotW words per update block
    unsigned long long *slots;
    // optional, [trace_cap]: the kind (ScanKind) of each iteration's scan
    int32_t *scan_kind;
    // optional: host-visible progress word, 2 k + (1 if the loop stopped at
    // k), written by the last block of iteration k
    long long *progress;
    // optional: the four smallest by position, z4p[j n + p] and their labels
    // i4p[j n + p] (coalesced; z4 / i4 by label may then be null)
    int64_t *z4p;
    int32_t *i4p;
    // the scan's candidate lists (ScanArgs::lst, lcnt, loff; nslices
    // segments per 64-row group): with lists set, an iteration whose
    // ctrl->list_ok holds is evaluated here from the lists (the scan exits)
    const int32_t *lst;
    const int32_t *lcnt;
    const int32_t *loff;
};

// candidate list entries per row and wave (see ScanArgs::lst); the margin
// D of a build is kListMult times the last max step, cut to half of the
// last margin whose lists overflowed, and a build is made once that step
// is at most 1/16 of iteration 0's and D is at least twice the step (lists
// built with margin D serve while the steps since sum to at most D / 2).
// Measured at n = 100k: margins of 12 steps keep a list for six
// iterations, and the lists rarely pass 24 entries per part.
constexpr int kLW = 24;
// entries of one 64-row group's list segment: 64 rows x 4 parts x kLW
constexpr int64_t kListCap = 64 * 4 * kLW;
constexpr int64_t kListMult = 12;

// Candidate graph (k nearest neighbours, union-symmetrised) in CSR over
// positions: rowptr[n+1], col (positions, increasing within a row), cost.
struct Csr {
    const int32_t *rowptr;
    const int32_t *col;
    const int32_t *cost;
    int64_t nnz;
};

struct GraphStepArgs {
    Geo g;
    Csr csr;
    int64_t k;
    const int64_t *lam_in;      // sorted
    int64_t *lam_out;           // sorted; holds Lam_{k-1} on entry
    int64_t *lam_best;
    int64_t *z4;                // [4n] by label
    int32_t *i4;                // [4n] by label
    int32_t *neg, *zero;        // by label, or null
    int64_t *step;              // by label, or null
    Ctrl *ctrl;
    int64_t *trace;
    unsigned long long *slots;  // per-block record slots, kSlotW words per block
    long long *progress;        // optional, as UpdateArgs::progress
    int64_t *z4p;               // optional, as UpdateArgs::z4p / i4p
    int32_t *i4p;
};

// Batched loop: one launch covers every instance.  Work items are tables in
// device memory; per-instance argument structs live in device memory too.
struct BatchScanItem {
    int32_t inst, row_block, slice, pad;
};
struct BatchTileItem {
    int32_t inst, block;   // update block `block` of instance `inst`
};
// Single-instance ScanArgs/UpdateArgs pointers are rebased per instance; the
// iteration index of a batched update comes from the instance's Ctrl.
hipError_t launch_scan_batch(const ScanArgs *args_dev, const BatchScanItem *items, int64_t nitems, int rows,
                             bool cull, hipStream_t st);
hipError_t launch_update_batch(const UpdateArgs *args_dev, const BatchTileItem *items, int64_t nitems,
                               hipStream_t st);
// ctrls[i].nblocks = nblocks[i]
hipError_t launch_ctrl_nblocks(Ctrl *ctrls, const int64_t *nblocks, int64_t ninst, hipStream_t st);
// out[0] = number of instances not yet done
hipError_t launch_count_active(const Ctrl *ctrls, int64_t ninst, int32_t *out, hipStream_t st);

// Launchers (f2m_kernels.hip).  All run on `st`; none synchronises.
// k nearest neighbours (K in {10, 16}) by (D, label): nbr[p*K + j] positions;
// pp / pd: the column slices' lists, knn_slices(n) * n * K entries each
int64_t knn_slices(int64_t n);
hipError_t launch_knn(const Geo &g, const float4 *col, int K, int32_t *nbr, int64_t *nbr_d, int32_t *pp,
                      int64_t *pd, hipStream_t st);
// CSR of the union-symmetrised graph; returns nnz through nnz_dev
size_t csr_temp_bytes(int64_t n, int K);
hipError_t launch_build_csr(const Geo &g, const int32_t *xy, int64_t n, int K, const int32_t *nbr, uint64_t *keys,
                            uint64_t *keys_alt, int32_t *deg, int32_t *rowptr, int32_t *col, int32_t *cost,
                            int64_t *nnz_dev, void *temp, size_t temp_bytes, int64_t cap, hipStream_t st);
hipError_t launch_graph_step(const GraphStepArgs &a, hipStream_t st);
// graph certificate dual side: acc[0] += sum over CSR entries of min(0, Z)
hipError_t launch_graph_dual(const Geo &g, const Csr &csr, const int64_t *lam_sorted, unsigned long long *acc,
                             hipStream_t st);
// pairs (Morton positions, lo < hi) of CSR edges with Z <= theta_row (theta_row =
// max(0, 4th smallest Z of the row) + slack when slack >= 0, else -1)
hipError_t launch_graph_collect(const Geo &g, const Csr &csr, const int64_t *lam_sorted, int64_t slack,
                                unsigned long long *count, int2 *out, int64_t cap, hipStream_t st);
// (lo, hi) node pairs, both ends below n -> sorted distinct keys
// lo * 2^32 + hi in keys_out;
// the distinct count lands in *count_dev; with costs non-null, costs[i] is
// the exact cost of keys_out[i] from the coordinates xy (same node order)
size_t pair_sort_temp_bytes(int64_t count);
// The distinct keys (count on the device, at most cap) that are not in the
// sorted set ex[nex], compacted into out (count in *out_count), with their
// exact costs
size_t exclude_temp_bytes(int64_t count);
hipError_t launch_exclude_keys(const uint64_t *keys, const int64_t *count_dev, int64_t cap, const uint64_t *ex,
                               int64_t nex, const int32_t *xy, uint8_t *flags, uint64_t *out, int64_t *out_count,
                               int32_t *costs, void *temp, size_t temp_bytes, hipStream_t st);
// Bulk candidate data for the exact finish from the distinct keys (count on
// the device, at most cap): exact costs, the negative-reduced-cost bits of
// the two arcs under alpha = floor(Lam/2), beta = Lam - alpha (xy and lam
// in the node order of the keys), and every node's incident pair ids in
// increasing order, each node's list followed by two free slots, as
// start[n + 1] (int32) and inc[2 * count + 2 * n]; deg[n + 1] is scratch
size_t pair_bulk_temp_bytes(int64_t count, int64_t n);
hipError_t launch_pair_bulk(const uint64_t *keys, const int64_t *count_dev, int64_t cap, const int32_t *xy,
                            const int64_t *lam, int64_t n, int32_t *costs, uint8_t *neg, int32_t *deg, int32_t *start,
                            int32_t *inc, void *temp, size_t temp_bytes, hipStream_t st);
hipError_t launch_sort_unique_pairs(const int2 *pairs, int64_t count, int64_t n, uint64_t *keys,
                                    uint64_t *keys_sorted, uint64_t *keys_out, int64_t *count_dev, void *temp,
                                    size_t temp_bytes, const int32_t *xy, int32_t *costs, hipStream_t st);
// labels: edges of x must be edges of the graph; acc[2] += violations
hipError_t launch_graph_membership(const Geo &g, const Csr &csr, int64_t m, const int32_t *eu, const int32_t *ev,
                                   unsigned long long *acc, hipStream_t st);
// CSR in label space (rows by label, columns labels increasing)
hipError_t launch_csr_to_labels(const Geo &g, const Csr &csr, int32_t *rowptr_l, int32_t *col_l, int32_t *deg_tmp,
                                hipStream_t st);
hipError_t launch_minmax(const int32_t *xy, int64_t n, int32_t *out4, hipStream_t st);

// Size of the fixed device workspace of f2m_gdp_step_noalloc, and its device
// address on the current device (f2m_noalloc.hip).
constexpr size_t kNoAllocBytes = size_t(32) << 20;
hipError_t noalloc_scratch(int device, void **ptr);
// Morton order: fills orig (position -> label) and pos (label -> position).
size_t sort_temp_bytes(int64_t n);
hipError_t launch_sort(const int32_t *xy, int64_t n, int32_t minx, int32_t miny, uint32_t *keys,
                       uint32_t *keys_alt, int32_t *ids, int32_t *orig, int32_t *pos, void *temp,
                       size_t temp_bytes, hipStream_t st);
// centred float coordinates in sorted order, tile boxes, xy2max
hipError_t launch_prep(const int32_t *xy, const int32_t *orig, int64_t n, int32_t cx, int32_t cy, float4 *col,
                       float4 *box, float *xy2max_dev, hipStream_t st);
// Lam (labels; orig null: already in Morton order) -> sorted Lam, h and q,
// tile maxima of h, max |Lam|
hipError_t launch_set_lam(const int64_t *lam_label, const int32_t *orig, int64_t n, int64_t *lam_sorted,
                          float4 *col, float *tile_hmax, Ctrl *ctrl, hipStream_t st);
hipError_t launch_unpermute(const int64_t *lam_sorted, const int32_t *orig, int64_t n, int64_t *lam_label,
                            hipStream_t st);
// copy of `bytes` bytes by a kernel (both 16-byte aligned; dst may be
// pinned host memory mapped into the device's address space)
hipError_t launch_copy_bytes(const void *src, void *dst, int64_t bytes, hipStream_t st);
// coordinates by label -> by Morton position (xy_pos[2n])
hipError_t launch_gather_xy(const int32_t *xy, const int32_t *orig, int64_t n, int32_t *xy_pos, hipStream_t st);
// edges as Morton positions -> labels (lo < hi), in place
hipError_t launch_edges_to_labels(const int32_t *orig, int64_t m, int32_t *eu, int32_t *ev, hipStream_t st);
// seeds (positions, [4][n]) from the four smallest of a previous run (labels, [n][4] by label)
hipError_t launch_seed_from_top(const int32_t *i4, const int32_t *orig, const int32_t *pos, int64_t n, int32_t *seed,
                                hipStream_t st);
hipError_t launch_seed_neighbours(int64_t n, const float4 *col, int32_t *seed, hipStream_t st);
// Loop state at the start of a run: iteration k0 first; with hvalid the
// hashes of Lam_{k0-1} (h1) and Lam_{k0-2} (h2) arm the cycle test at once.
struct CtrlStart {
    int64_t k0 = 0;
    uint64_t h1 = 0, h2 = 0;
    int hvalid = 0;
};
hipError_t launch_ctrl_init(Ctrl *ctrl, int64_t max_iters, int64_t trace_cap, int64_t handoff_div,
                            const CtrlStart &cs,
                            hipStream_t st);
hipError_t launch_scan(const ScanArgs &a, int mode, int64_t nslices, int rows_per_thread, hipStream_t st);
hipError_t launch_update(const UpdateArgs &a, hipStream_t st);
// The control of iteration k after an update (or candidate-graph step)
// launch of nblk blocks whose slots hold their parts of the record.
struct ControlArgs {
    Ctrl *ctrl;
    int64_t n, k, nblk;
    const unsigned long long *slots;
    int64_t *trace;             // or null
    int32_t *kinds;             // or null
    long long *progress;        // or null
    int lists;                  // the loop's scans keep candidate lists
};
hipError_t launch_control(const ControlArgs &a, hipStream_t st);
// batched: one block per instance (args: the instances' update arguments)
hipError_t launch_control_batch(const UpdateArgs *args_dev, int64_t ninst, hipStream_t st);
// z4[4v + j], i4[4v + j] by label from z4p[j n + p], i4p[j n + p] by position
hipError_t launch_top_to_labels(const int64_t *z4p, const int32_t *i4p, const int32_t *orig, int64_t n, int64_t *z4,
                                int32_t *i4, hipStream_t st);
hipError_t launch_extract_trivial(const int64_t *z4, const int32_t *i4, int64_t n,
                                  int32_t *slot_u, int32_t *slot_v, uint8_t *slot_x2,
                                  hipStream_t st);
hipError_t launch_compact(const int32_t *slot_u, const int32_t *slot_v, const uint8_t *slot_x2,
                          int64_t nslots, int32_t *eu, int32_t *ev, uint8_t *ex2,
                          int64_t *count_dev, int32_t *block_tmp, hipStream_t st);
int64_t compact_block_tmp_len(int64_t nslots);
hipError_t launch_cert_edges(const int32_t *xy, int64_t n, int64_t m, const int32_t *eu,
                             const int32_t *ev, const uint8_t *ex2, int32_t *deg, int32_t *cnt,
                             int32_t *nb, unsigned long long *acc, hipStream_t st);
// b by label, or null (F2M): every doubled degree must be 2 b_v; acc[3] +=
// sum_v b_v Lam_v.  nb holds kCertNb neighbour slots per node.
hipError_t launch_cert_nodes(const int64_t *lam, int64_t n, const int32_t *deg,
                             const int32_t *cnt, const int32_t *nb, unsigned long long *acc,
                             const int8_t *b, hipStream_t st);
constexpr int kCertNb = 6;
// b_pos[p] = b_label[orig[p]]
hipError_t launch_b_to_positions(const int8_t *b_label, const int32_t *orig, int64_t n, int8_t *b_pos,
                                 hipStream_t st);

}  // namespace f2m
