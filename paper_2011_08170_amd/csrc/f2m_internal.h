// Internal interface between the HIP kernels (f2m_kernels.hip) and the host
// runtime (f2m_api.cpp).  Not part of the public ABI.
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

// Device-resident control block of the GDP loop.  The update kernel's
// last block reads the accumulators, writes the iteration record, takes
// the stop decision and clears the accumulators for the next iteration.
struct Ctrl {
    // accumulators of the iteration being reduced
    unsigned long long acc_sumlam;    // sum Lam_k (two's complement)
    unsigned long long acc_rowneg;    // sum over rows of sum_u min(0, Z)
    unsigned long long acc_unsat;
    unsigned long long acc_bad;
    long long acc_maxstep;
    unsigned long long acc_nonzero;
    unsigned long long acc_hash;
    long long acc_maxabs_next;        // max |Lam_{k+1}|
    unsigned int blocks_done;
    unsigned int pad0;
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
};

// Column record of the scan, one per city: centred coordinates, half of
// Lam and q = x^2 + y^2 - h^2 (all float; x, y exact integers).
// float4 {x, y, h, q}.

struct ScanArgs {
    int64_t n;
    int64_t slice_len;          // columns per slice (blockIdx.y)
    const float4 *col;          // n
    const int64_t *lam;         // Lam_k, n
    const int32_t *seed;        // previous top-4 indices [4n] or null
    const Ctrl *ctrl;           // done flag, maxabs_lam
    float xy2max;               // max over cities of x^2 + y^2 (centred)
    // partial results per (slice, row), structure of arrays
    int64_t *pz;                // [slice][4][n]
    int32_t *pi;                // [slice][4][n]
    int32_t *pneg;              // [slice][n]
    int32_t *pzero;             // [slice][n]
    int64_t *prowneg;           // [slice][n]
};

struct UpdateArgs {
    int64_t n;
    int64_t nslices;
    int64_t k;                  // iteration index
    const int64_t *pz;
    const int32_t *pi;
    const int32_t *pneg;
    const int32_t *pzero;
    const int64_t *prowneg;
    const int64_t *lam_in;      // Lam_k
    int64_t *lam_out;           // Lam_{k+1}; holds Lam_{k-1} on entry
    int64_t *lam_best;          // copy of the best-dual iterate
    float4 *col;                // h, q rewritten for Lam_{k+1}
    int64_t *z4;                // [4n] node-major (4v + j)
    int32_t *i4;                // [4n] node-major
    int32_t *seed;              // [j][n] top-4 indices for the next scan
    int32_t *neg;               // [n] or null
    int32_t *zero;              // [n] or null
    int64_t *step;              // [n] or null
    Ctrl *ctrl;
    int64_t *trace;             // [trace_cap][8] or null
};

struct CollectArgs {
    int64_t n;
    int64_t slice_len;
    const float4 *col;
    const int64_t *lam;
    const int32_t *seed;        // [j][n] column indices bounding the 4th smallest Z, or null
    const Ctrl *ctrl;           // maxabs_lam
    float xy2max;
    int64_t theta;              // row threshold when seed is null (or a seed is missing)
    int64_t slack;              // added to the seeded threshold
    unsigned long long *count;  // pairs found (may exceed cap)
    int2 *out;                  // (u, v), u < v; both rows may report a pair
    int64_t cap;
};

struct CertScanArgs {
    int64_t n;
    int64_t slice_len;
    const float4 *col;
    const int64_t *lam;
    const Ctrl *ctrl;           // maxabs_lam
    float xy2max;
    unsigned long long *acc;    // [0] sum of min(0, Z) over ordered pairs
};

// Launchers (f2m_kernels.hip).  All run on `st`; none synchronises.
hipError_t launch_minmax(const int32_t *xy, int64_t n, int32_t *out4, hipStream_t st);
hipError_t launch_prep(const int32_t *xy, int64_t n, int32_t cx, int32_t cy, float4 *col,
                       float *xy2max_dev, hipStream_t st);
hipError_t launch_set_lam(const int64_t *lam, int64_t n, float4 *col, Ctrl *ctrl, hipStream_t st);
hipError_t launch_ctrl_init(Ctrl *ctrl, int64_t max_iters, int64_t trace_cap, int64_t handoff_div,
                            hipStream_t st);
hipError_t launch_scan(const ScanArgs &a, int64_t nslices, int rows_per_thread, hipStream_t st);
hipError_t launch_update(const UpdateArgs &a, hipStream_t st);
hipError_t launch_extract_trivial(const int64_t *z4, const int32_t *i4, int64_t n,
                                  int32_t *slot_u, int32_t *slot_v, uint8_t *slot_x2,
                                  hipStream_t st);
hipError_t launch_compact(const int32_t *slot_u, const int32_t *slot_v, const uint8_t *slot_x2,
                          int64_t nslots, int32_t *eu, int32_t *ev, uint8_t *ex2,
                          int64_t *count_dev, int32_t *block_tmp, hipStream_t st);
int64_t compact_block_tmp_len(int64_t nslots);
hipError_t launch_collect(const CollectArgs &a, int64_t nslices, hipStream_t st);
hipError_t launch_cert_scan(const CertScanArgs &a, int64_t nslices, hipStream_t st);
hipError_t launch_cert_edges(const int32_t *xy, int64_t n, int64_t m, const int32_t *eu,
                             const int32_t *ev, const uint8_t *ex2, int32_t *deg, int32_t *cnt,
                             int32_t *nb, unsigned long long *acc, hipStream_t st);
hipError_t launch_cert_nodes(const int64_t *lam, int64_t n, const int32_t *deg,
                             const int32_t *cnt, const int32_t *nb, unsigned long long *acc,
                             hipStream_t st);

}  // namespace f2m
