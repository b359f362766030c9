// Internal interface of the GDP with subtour-elimination rows between its
// kernels (f2m_sec.hip) and the host runtime (f2m_api.cpp).
//
// Rows come in layers of disjoint node sets.  For row q of layer l with set
// S_q, Z_e of an edge e = {u, v} loses M_q when e crosses delta(S_q), i.e.
// when exactly one end lies in S_q.  Within a layer an edge crosses the row
// of u (if any) and the row of v (if any) when those differ, so with
// Lam'_v = Lam_v + sum over v's rows of M
//     Z_uv = 2c_uv - Lam'_u - Lam'_v + sum_{l: row_l(u) == row_l(v) >= 0} 2 M_{row_l(u)}.
// Since every M >= 0, Z_uv >= 2c_uv - Lam'_u - Lam'_v: the complete-graph
// float filter run with Lam' in place of Lam never drops a pair it needs.
#pragma once
#include "f2m_internal.h"

namespace f2m {

constexpr int kSecMaxLayers = 8;
constexpr int kSecTraceW = 9;
constexpr int kSecSlotW = 16;

// Loop state of the GDP with subtour rows; 64-bit words only (the control
// kernel reads and writes it as an array of words).
struct SecCtrl {
    long long done, stop, k_last, kstar, best_dual2, best_k;
    unsigned long long h1, h2;   // hashes of the iterates k-1 and k-2
    long long max_iters, trace_cap, overflow;
    long long lamp_bound;        // bound of |Lam'_v| over the iterate being scanned
    long long dual2_last, primal2_last, unsat_last, node_bad_last, row_infeas_last, row_loose_last;
    long long nlayers;           // layers with rows (Lam' holds at most this many M per node)
    long long init_lmax, init_mmax;   // set-up: max |Lam_0|, max M_0
    long long bad_input;         // set-up: a row id out of range or an M_0 < 0
    unsigned long long pairs_tested;   // ordered pairs the GDP scans filter-tested (culled tiles excluded)
};

// The scan: per row (position) p over the columns of its slice, the three
// smallest (Z, column) and #Z<0, #Z==0, the sum of min(0, Z) and of x2 c
// over the pairs with Z <= 0; per layer l whose row holds p, the three
// smallest (Z, column) over the edges crossing that row and their #Z<0,
// #Z==0.  A row needs a pair only when its Z is at most theta_p, the largest
// of those lists' third values and 0; theta_p starts at the bound the seed
// columns give (any three distinct columns of a list bound its third
// smallest) and falls as the lists fill.  Column tiles and 32-column
// sub-tiles whose box is too far from the rows' box for any pair to reach
// theta (with Lam' in place of Lam) are skipped.  Support mode (theta = 0):
// every pair with Z <= 0 joins its ends' components (labels) instead.
struct SecScanArgs {
    Geo g;
    const float4 *col;           // centred coordinates by position (x, y used)
    const int64_t *lamp;         // Lam' by position
    const float *tile_h;         // per tile and sub-tile (kBoxStride per tile): max of Lam'/2
    const int32_t *rowp;         // [L][n] row of layer l holding position p, -1 none
    const int64_t *mu;           // M_k by row
    const SecCtrl *ctrl;
    const int32_t *seed;         // [(1 + L) * 3][n] seed columns (positions, -1 none) or null
    // with seed: per subtour row its three seed edges (member, column;
    // positions); they bound the row's third smallest crossing Z, so a
    // member needs no crossing edge above that bound
    const int2 *rseed;           // [nrows][3]
    int64_t slice_len;           // columns per slice (blockIdx.y), a multiple of 256
    int support;                 // 1: support mode
    // stats partials, [slice][...][n]
    int64_t *pz;                 // [S][3][n]
    int32_t *pzi;                // [S][3][n] their columns
    int32_t *pc;                 // [S][2][n]: #Z<0, #Z==0
    int64_t *prn;                // [S][n]: sum of min(0, Z)
    int64_t *ppr;                // [S][n]: sum of x2 c over Z <= 0 (x2 = 2 for Z < 0, 1 for Z == 0)
    int64_t *pxz;                // [S][L][3][n]
    int32_t *pxi;                // [S][L][3][n]
    int32_t *pxc;                // [S][L][2][n]
    unsigned long long *tpart;   // [S][row blocks]: ordered pairs filter-tested by the block
    int32_t *parent;             // support mode: union-find forest over labels
};

// Node step: merges the slices, steps Lam, records; writes the merged
// crossing statistics for the row step.
struct SecNodeArgs {
    Geo g;
    int64_t nslices, k;
    const int64_t *pz;
    const int32_t *pzi, *pc;
    const int64_t *prn, *ppr, *pxz;
    const int32_t *pxi, *pxc;
    const int32_t *rowp;
    int32_t *seed;               // out: the next scan's seed columns (SecScanArgs::seed)
    const int64_t *lam_in;       // Lam_k by position
    int64_t *lam_out;            // Lam_{k+1}; holds Lam_{k-1} on entry
    int64_t *lam_best;
    int64_t *lamp;               // out: Lam_{k+1} (the row step adds the M)
    int64_t *xz;                 // [L][3][n] merged crossing three smallest
    int32_t *xc;                 // [L][2][n]
    SecCtrl *ctrl;
    unsigned long long *slots;   // this launch's blocks: slots[blk]
};

// Row step: one wave per subtour row.
struct SecRowArgs {
    int64_t n, nrows, k;
    const int32_t *rptr;         // [nrows + 1] offsets into rmem
    const int32_t *rmem;         // members (positions), row after row
    const int32_t *rlayer;       // [nrows] layer of each row
    const int64_t *xz;
    const int32_t *xc;
    const int64_t *mu_in;        // M_k
    int64_t *mu_out;             // M_{k+1}; holds M_{k-1} on entry
    int64_t *mu_best;
    int64_t *lamp;               // += M_{k+1} of each member's rows
    const int32_t *seed;         // the node step's seeds: the columns of the members' crossing lists
    int2 *rseed;                 // out: [nrows][3] the row's three smallest crossing edges
    SecCtrl *ctrl;
    unsigned long long *slots;   // this launch's blocks
};

struct SecControlArgs {
    SecCtrl *ctrl;
    int64_t n, k, nblk;          // slots of the node and row launches together
    const unsigned long long *slots;
    int64_t *trace;              // [trace_cap][kSecTraceW] or null
    const unsigned long long *tpart;   // the scan's pairs tested, ntpart entries
    int64_t ntpart;
};

// L: the layer count the kernels are instantiated for (1, 2, 4 or 8 >= nlayers)
int sec_layers_inst(int nlayers);
hipError_t launch_sec_scan(const SecScanArgs &a, int L, int64_t nslices, hipStream_t st);
hipError_t launch_sec_node(const SecNodeArgs &a, int L, hipStream_t st);
hipError_t launch_sec_rows(const SecRowArgs &a, hipStream_t st);
hipError_t launch_sec_control(const SecControlArgs &a, hipStream_t st);
hipError_t launch_sec_ctrl_init(SecCtrl *ctrl, int64_t max_iters, int64_t trace_cap, int64_t nlayers,
                                hipStream_t st);
// rowp[l n + p] = row_of[l n + orig[p]]; counts members per row and the
// layer range of every row (lo, hi: the host checks lo == hi); flags ids
// out of range in ctrl->bad_input
// (layers nlayers .. L - 1 of rowp are set to -1)
hipError_t launch_sec_rows_in(const int32_t *row_of, const int32_t *orig, int64_t n, int nlayers, int L,
                              int64_t nrows, int32_t *rowp, int32_t *cnt, int32_t *lay_lo, int32_t *lay_hi,
                              SecCtrl *ctrl, hipStream_t st);
// rmem[rptr[q] + i] = the members of row q (positions; cur zeroed, [nrows])
hipError_t launch_sec_rows_fill(const int32_t *rowp, int64_t n, int L, const int32_t *rptr, int32_t *cur,
                                int32_t *rmem, hipStream_t st);
// lam_pos[p] = lam_label[orig[p]], lamp = lam_pos; init_lmax, init_mmax and
// bad_input (some M_0 < 0) in ctrl, then lamp_bound
hipError_t launch_sec_start(const int64_t *lam_label, const int32_t *orig, int64_t n, const int64_t *mu,
                            int64_t nrows, int64_t *lam_pos, int64_t *lamp, SecCtrl *ctrl, hipStream_t st);
// lamp += M of each member's rows (the start's Lam'); then the bound
hipError_t launch_sec_add_mu(const int32_t *rptr, const int32_t *rmem, const int64_t *mu, int64_t nrows,
                             int64_t *lamp, SecCtrl *ctrl, hipStream_t st);
// tile_h[t kBoxStride + s] = max over tile t (s = 0) or its sub-tile s - 1
// of the float Lam'/2 the scan's column records use
hipError_t launch_sec_tiles(const int64_t *lamp, int64_t n, float *tile_h, hipStream_t st);
// union-find over labels: parent[v] = v; after the support scan, comp[v] =
// the smallest label of v's component
hipError_t launch_sec_uf_init(int32_t *parent, int64_t n, hipStream_t st);
hipError_t launch_sec_uf_final(int32_t *parent, int64_t n, hipStream_t st);

}  // namespace f2m
