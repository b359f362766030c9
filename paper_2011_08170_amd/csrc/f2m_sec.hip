// HIP kernels of the GDP with subtour-elimination rows (F2M plus rows
// x(delta(S_q)) >= 2 with multipliers M_q >= 0; Sec. 2 eq. 4-5, Sec. 3 with
// b = 2, the extension of Sec. 5) for gfx950.
//
// One iteration is four launches on the context's stream:
//   k_sec_scan<L>   every ordered pair once (one row per lane, 256 columns per
//                   LDS tile, the block's own tile first), the float filter of
//                   the complete-graph scan run on Lam' (see f2m_sec.h), exact
//                   int64 Z for the pairs it passes; per row the three smallest
//                   Z, the counts and sums of its degree row, and per layer the
//                   three smallest Z and counts over the edges crossing the
//                   row's subtour row;
//   k_sec_node<L>   merges the column slices, steps Lam (eq. 10), records;
//   k_sec_rows      one wave per subtour row: merges its members' crossing
//                   statistics, steps and projects M, adds M_{k+1} to its
//                   members' Lam', records;
//   k_sec_control   one block: sums the records, trace, stop test.
// Support mode of the scan: every pair with Z <= 0 joins the components of
// its ends in a lock-free union-find over labels (the separation).
#include "f2m_sec.h"
#include "f2m_filter.h"
#include "f2m_device.h"

#include <limits.h>

namespace f2m {

namespace {

constexpr int kSB = 256;        // threads per block: rows of a scan block, columns of a tile
constexpr int kSGroup = 8;      // columns per filter test
constexpr int kRecS = 13;       // record entries (see sec_record)
constexpr unsigned long long kGolden = 0x9E3779B97F4A7C15ULL;

// the three smallest of a multiset of values, increasing
__device__ __forceinline__ void ins3(int64_t (&t)[3], int64_t z)
{
    if (z >= t[2]) return;
    t[2] = z;
    if (t[2] < t[1]) { const int64_t x = t[1]; t[1] = t[2]; t[2] = x; }
    if (t[1] < t[0]) { const int64_t x = t[0]; t[0] = t[1]; t[1] = x; }
}

// A subtour row's move: half the sum of its 2nd and 3rd smallest Z would put
// zero midway between them; an edge crossing the row also lies in the two
// degree rows and the layer's row of its other end, all moving at once, so
// the move is divided by four: sign(s) floor((|s| + 4) / 8).  (A degree row
// shares its edges with one other row: gdp_step divides by two.)
__device__ __forceinline__ int64_t row_step(int64_t s)
{
    if (s > 0) return (s + 4) >> 3;
    if (s < 0) return -((-s + 4) >> 3);
    return 0;
}

__device__ __forceinline__ int32_t uf_find(int32_t *parent, int32_t x)
{
    // parents only ever decrease (a root is linked under a smaller one), so
    // the walk ends; a stale read is still an ancestor
    for (;;) {
        const int32_t px = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (px == x) return x;
        x = px;
    }
}

// joins the components of a and b: the larger root goes under the smaller,
// so every root is its component's smallest label
__device__ __forceinline__ void uf_unite(int32_t *parent, int32_t a, int32_t b)
{
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a > b) { const int32_t x = a; a = b; b = x; }
        int32_t expect = b;
        if (__hip_atomic_compare_exchange_strong(&parent[b], &expect, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        // b was linked meanwhile: retry from its new parent
    }
}

// Record entries: 0 sum Lam_k, 1 sum M_k, 2 sum over ordered pairs of
// min(0, Z), 3 sum over ordered pairs with Z <= 0 of x2 c, 4 #unsat rows,
// 5 #bad degree rows, 6 #subtour rows below crossing degree 4, 7 #subtour
// rows with M > 0 above it, 8 max step, 9 #nonzero steps, 10 hash,
// 11 max |Lam_{k+1}|, 12 max M_{k+1}.  8, 11 and 12 are maxima.
__device__ __forceinline__ bool rec_is_max(int i) { return i == 8 || i == 11 || i == 12; }

// sums (maxes) v over the block into slots[blk * kSecSlotW + i]
__device__ __forceinline__ void sec_record(unsigned long long (&v)[kRecS], unsigned long long *slots, int64_t blk)
{
    __shared__ unsigned long long red[kSB / 64][kRecS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < kRecS; ++i) v[i] = rec_is_max(i) ? wave_max(v[i]) : wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kRecS; ++i) red[w][i] = v[i];
    }
    __syncthreads();
    if (w == 0 && lane < kRecS) {
        unsigned long long m = red[0][lane];
        for (int q = 1; q < kSB / 64; ++q) {
            const unsigned long long x = red[q][lane];
            m = rec_is_max(lane) ? (x > m ? x : m) : m + x;
        }
        slots[blk * kSecSlotW + lane] = m;
    }
}

template <int L>
__global__ __launch_bounds__(kSB) void k_sec_scan(SecScanArgs a)
{
    if (!a.support && a.ctrl->done) return;
    __shared__ float4 sc[kSB];
    __shared__ long long slp[kSB];
    __shared__ int32_t sr[L][kSB];
    __shared__ int32_t so[kSB];
    const int t = threadIdx.x;
    const int64_t n = a.g.n;
    const int64_t p = (int64_t)blockIdx.x * kSB + t;
    const int64_t sl = blockIdx.y;
    const int64_t c0 = sl * a.slice_len, c1 = min(n, c0 + a.slice_len);
    const float colmax = col_bound(a.g.xy2max, a.ctrl->lamp_bound);
    const bool live = p < n;

    Row rw;
    int64_t nz[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
    int32_t cn = 0, cz = 0;
    int64_t rn = 0, pr = 0;
    int32_t rv[L];
    int64_t mv[L];
    int64_t xz[L][3];
    int32_t xn[L], xzr[L];
    int32_t lab = 0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        rv[l] = live ? a.rowp[l * n + p] : -1;
        mv[l] = rv[l] >= 0 ? a.mu[rv[l]] : 0;
        xz[l][0] = xz[l][1] = xz[l][2] = INT64_MAX;
        xn[l] = xzr[l] = 0;
    }
    if (live) {
        const float4 cv = a.col[p];
        rw.xv = cv.x;
        rw.yv = cv.y;
        rw.lamv = a.lamp[p];
        rw.theta = a.support ? 0 : kThetaNone;
        rw.v = p;
        set_filter(rw, colmax);
        lab = a.g.orig[p];
    } else {
        rw.xv = rw.yv = 0.0f;
        rw.lamv = 0;
        rw.theta = 0;
        rw.v = -1;
        rw.a = rw.b = rw.c = 0.0f;
        rw.thr = -INFINITY;   // never passes
    }

    auto eval = [&](int c, int64_t base) {
        const int64_t u = base + c;
        if (u == p) return;
        const float4 cd = sc[c];
        if (!(filter_value(rw, cd) <= rw.thr)) return;   // theta may have dropped in this group
        const int32_t dx = (int32_t)(rw.xv - cd.x);
        const int32_t dy = (int32_t)(rw.yv - cd.y);
        const int64_t cst = nint_sqrt((int64_t)dx * dx + (int64_t)dy * dy);
        int64_t z = 2 * cst - rw.lamv - slp[c];
#pragma unroll
        for (int l = 0; l < L; ++l)
            if (rv[l] >= 0 && sr[l][c] == rv[l]) z += 2 * mv[l];
        if (a.support) {
            if (z <= 0 && p < u) uf_unite(a.parent, lab, so[c]);
            return;
        }
        if (z > rw.theta) return;
        if (z < 0) { ++cn; rn += z; pr += 2 * cst; }
        else if (z == 0) { ++cz; pr += cst; }
        ins3(nz, z);
        int64_t th = nz[2];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (rv[l] >= 0) {
                if (sr[l][c] != rv[l]) {
                    ins3(xz[l], z);
                    if (z < 0) ++xn[l];
                    else if (z == 0) ++xzr[l];
                }
                th = xz[l][2] > th ? xz[l][2] : th;
            }
        }
        th = th > 0 ? th : 0;
        th = th < kThetaNone ? th : kThetaNone;
        if (th < rw.theta) { rw.theta = th; set_filter(rw, colmax); }
    };

    const int64_t ntl = (c1 - c0 + kSB - 1) / kSB;
    // the block's own tile first (its rows' nearest columns tighten the
    // thresholds early), then the rest in order
    const int64_t own = ((int64_t)blockIdx.x * kSB - c0) / kSB;
    const int64_t start = ((int64_t)blockIdx.x * kSB >= c0 && own < ntl) ? own : (int64_t)blockIdx.x % max(ntl, (int64_t)1);
    for (int64_t i = 0; i < ntl; ++i) {
        int64_t ti = start + i;
        if (ti >= ntl) ti -= ntl;
        const int64_t base = c0 + ti * kSB;
        const int64_t cc = base + t;
        __syncthreads();
        if (cc < c1) {
            const float4 cd = a.col[cc];
            const long long lp = a.lamp[cc];
            sc[t] = col_record(cd.x, cd.y, lp);
            slp[t] = lp;
            so[t] = a.g.orig[cc];
#pragma unroll
            for (int l = 0; l < L; ++l) sr[l][t] = a.rowp[l * n + cc];
        } else {
            sc[t] = make_float4(0.0f, 0.0f, 0.0f, INFINITY);   // never passes the filter
            slp[t] = 0;
            so[t] = 0;
#pragma unroll
            for (int l = 0; l < L; ++l) sr[l][t] = -1;
        }
        __syncthreads();
        for (int g = 0; g < kSB; g += kSGroup) {
            float m = INFINITY;
#pragma unroll
            for (int q = 0; q < kSGroup; ++q) m = fminf(m, filter_value(rw, sc[g + q]));
            if (m <= rw.thr) {
                for (int q = 0; q < kSGroup; ++q) eval(g + q, base);
            }
        }
    }
    if (!live || a.support) return;
#pragma unroll
    for (int j = 0; j < 3; ++j) a.pz[(sl * 3 + j) * n + p] = nz[j];
    a.pc[(sl * 2) * n + p] = cn;
    a.pc[(sl * 2 + 1) * n + p] = cz;
    a.prn[sl * n + p] = rn;
    a.ppr[sl * n + p] = pr;
#pragma unroll
    for (int l = 0; l < L; ++l) {
#pragma unroll
        for (int j = 0; j < 3; ++j) a.pxz[((sl * L + l) * 3 + j) * n + p] = xz[l][j];
        a.pxc[((sl * L + l) * 2) * n + p] = xn[l];
        a.pxc[((sl * L + l) * 2 + 1) * n + p] = xzr[l];
    }
}

template <int L>
__global__ __launch_bounds__(kSB) void k_sec_node(SecNodeArgs a)
{
    SecCtrl *ctrl = a.ctrl;
    if (ctrl->done) return;
    const int64_t n = a.g.n;
    const int64_t p = (int64_t)blockIdx.x * kSB + threadIdx.x;
    const int64_t k = a.k;
    // Lam_{k-1} sits in lam_out until it is overwritten
    const bool copy_best = k > 0 && ctrl->best_k == k - 1;
    unsigned long long v[kRecS];
#pragma unroll
    for (int i = 0; i < kRecS; ++i) v[i] = 0;
    if (p < n) {
        int64_t nz[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
        int64_t cn = 0, cz = 0, rn = 0, pr = 0;
        int64_t xz[L][3];
        int32_t xn[L], xzr[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            xz[l][0] = xz[l][1] = xz[l][2] = INT64_MAX;
            xn[l] = xzr[l] = 0;
        }
        for (int64_t s = 0; s < a.nslices; ++s) {
#pragma unroll
            for (int j = 0; j < 3; ++j) ins3(nz, a.pz[(s * 3 + j) * n + p]);
            cn += a.pc[(s * 2) * n + p];
            cz += a.pc[(s * 2 + 1) * n + p];
            rn += a.prn[s * n + p];
            pr += a.ppr[s * n + p];
#pragma unroll
            for (int l = 0; l < L; ++l) {
#pragma unroll
                for (int j = 0; j < 3; ++j) ins3(xz[l], a.pxz[((s * L + l) * 3 + j) * n + p]);
                xn[l] += a.pxc[((s * L + l) * 2) * n + p];
                xzr[l] += a.pxc[((s * L + l) * 2 + 1) * n + p];
            }
        }
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (a.rowp[l * n + p] < 0) continue;
#pragma unroll
            for (int j = 0; j < 3; ++j) a.xz[(l * 3 + j) * n + p] = xz[l][j];
            a.xc[(l * 2) * n + p] = xn[l];
            a.xc[(l * 2 + 1) * n + p] = xzr[l];
        }
        // eq. 10 on the 2nd and 3rd smallest Z of the degree row (n >= 4)
        const int64_t lamv = a.lam_in[p];
        const int64_t st = gdp_step(nz[1] + nz[2]);
        const int64_t nxt = lamv + st;
        if (copy_best) a.lam_best[p] = a.lam_out[p];
        a.lam_out[p] = nxt;
        a.lamp[p] = nxt;
        const int64_t lab = a.g.orig[p];
        v[0] = (unsigned long long)lamv;
        v[2] = (unsigned long long)rn;
        v[3] = (unsigned long long)pr;
        v[4] = (nz[1] > 0 || nz[2] < 0) ? 1 : 0;
        v[5] = (2 * cn + cz != 4) ? 1 : 0;
        v[8] = (unsigned long long)(st < 0 ? -st : st);
        v[9] = st != 0 ? 1 : 0;
        v[10] = mix64((uint64_t)lamv ^ (kGolden * (uint64_t)(lab + 1)));
        v[11] = (unsigned long long)(nxt < 0 ? -nxt : nxt);
    }
    sec_record(v, a.slots, blockIdx.x);
}

__global__ __launch_bounds__(kSB) void k_sec_rows(SecRowArgs a)
{
    SecCtrl *ctrl = a.ctrl;
    if (ctrl->done) return;
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * (kSB / 64) + (threadIdx.x >> 6);
    const int64_t n = a.n, k = a.k;
    unsigned long long v[kRecS];
#pragma unroll
    for (int i = 0; i < kRecS; ++i) v[i] = 0;
    if (q < a.nrows) {
        const int64_t l = a.rlayer[q];
        const int32_t e0 = a.rptr[q], e1 = a.rptr[q + 1];
        int64_t tz[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
        long long neg = 0, zero = 0;
        for (int32_t e = e0 + lane; e < e1; e += 64) {
            const int64_t m = a.rmem[e];
#pragma unroll
            for (int j = 0; j < 3; ++j) ins3(tz, a.xz[(l * 3 + j) * n + m]);
            neg += a.xc[(l * 2) * n + m];
            zero += a.xc[(l * 2 + 1) * n + m];
        }
        // the wave's three smallest: merge with the partner lane's list at
        // each distance (a multiset: the merge order does not matter)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const long long u0 = __shfl_xor((long long)tz[0], o, 64);
            const long long u1 = __shfl_xor((long long)tz[1], o, 64);
            const long long u2 = __shfl_xor((long long)tz[2], o, 64);
            ins3(tz, u0);
            ins3(tz, u1);
            ins3(tz, u2);
        }
        neg = wave_sum(neg);
        zero = wave_sum(zero);
        const int64_t M = a.mu_in[q];
        const int64_t st = row_step(tz[1] + tz[2]);
        const int64_t Mn = M + st > 0 ? M + st : 0;
        const int64_t dM = Mn - M;
        if (lane == 0) {
            if (k > 0 && ctrl->best_k == k - 1) a.mu_best[q] = a.mu_out[q];
            a.mu_out[q] = Mn;
        }
        if (Mn != 0) {
            for (int32_t e = e0 + lane; e < e1; e += 64) atomicAdd((unsigned long long *)&a.lamp[a.rmem[e]], (unsigned long long)Mn);
        }
        if (lane == 0) {
            const long long d2 = 2 * neg + zero;
            const bool infeas = d2 < 4;
            v[1] = (unsigned long long)M;
            v[4] = (tz[1] > 0 || (M > 0 && tz[2] < 0)) ? 1 : 0;
            v[6] = infeas ? 1 : 0;
            v[7] = (!infeas && M > 0 && d2 != 4) ? 1 : 0;
            v[8] = (unsigned long long)(dM < 0 ? -dM : dM);
            v[9] = dM != 0 ? 1 : 0;
            v[10] = mix64((uint64_t)M ^ (kGolden * (uint64_t)(n + q + 1)));
            v[12] = (unsigned long long)Mn;
        }
    }
    sec_record(v, a.slots, blockIdx.x);
}

__global__ __launch_bounds__(kSB) void k_sec_control(SecControlArgs a)
{
    SecCtrl *c = a.ctrl;
    if (c->done) return;
    __shared__ unsigned long long red[kSB / 64][kRecS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long acc[kRecS];
#pragma unroll
    for (int i = 0; i < kRecS; ++i) acc[i] = 0;
    for (int64_t b = threadIdx.x; b < a.nblk; b += kSB) {
#pragma unroll
        for (int i = 0; i < kRecS; ++i) {
            const unsigned long long x = a.slots[b * kSecSlotW + i];
            acc[i] = rec_is_max(i) ? (x > acc[i] ? x : acc[i]) : acc[i] + x;
        }
    }
#pragma unroll
    for (int i = 0; i < kRecS; ++i) acc[i] = rec_is_max(i) ? wave_max(acc[i]) : wave_sum(acc[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kRecS; ++i) red[w][i] = acc[i];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    unsigned long long r[kRecS];
#pragma unroll
    for (int i = 0; i < kRecS; ++i) {
        r[i] = red[0][i];
        for (int q = 1; q < kSB / 64; ++q) r[i] = rec_is_max(i) ? (red[q][i] > r[i] ? red[q][i] : r[i]) : r[i] + red[q][i];
    }
    const long long k = a.k;
    const long long sl = (long long)r[0], sm = (long long)r[1], rn = (long long)r[2], pr = (long long)r[3];
    const long long un = (long long)r[4], nb = (long long)r[5], ri = (long long)r[6], rl = (long long)r[7];
    const long long ms = (long long)r[8], nz = (long long)r[9];
    const unsigned long long hh = r[10];
    const long long mlam = (long long)r[11], mmu = (long long)r[12];
    // each unordered pair sits in two degree rows
    const long long dual2 = 2 * sl + 2 * sm + rn / 2;
    const long long bad = nb + ri + rl;
    if (a.trace && k < c->trace_cap) {
        long long *rec = (long long *)a.trace + kSecTraceW * k;
        rec[0] = k; rec[1] = dual2; rec[2] = un; rec[3] = bad; rec[4] = ms;
        rec[5] = nz; rec[6] = (long long)hh; rec[7] = sl; rec[8] = sm;
    }
    if (c->best_k < 0 || dual2 > c->best_dual2) { c->best_dual2 = dual2; c->best_k = k; }
    // the next scan's filter needs |Lam'| below the limit
    const long long bound = mlam + c->nlayers * mmu;
    long long stop = 0;
    if (bad == 0) stop = 1;                                  // trivial
    else if (nz == 0) stop = 2;                              // fixed
    else if (k >= 2 && hh == (unsigned long long)c->h2) stop = 3;   // cycle
    else if (k >= c->max_iters) stop = 4;                    // cap
    else if (bound >= kLamLimit) { stop = 4; c->overflow = 1; }
    c->k_last = k;
    c->dual2_last = dual2;
    c->primal2_last = pr / 2;
    c->unsat_last = un;
    c->node_bad_last = nb;
    c->row_infeas_last = ri;
    c->row_loose_last = rl;
    if (stop) {
        c->stop = stop;
        c->kstar = (stop == 3 || stop == 4) ? c->best_k : k;
        c->done = 1;
    } else {
        c->h2 = c->h1;
        c->h1 = hh;
        c->lamp_bound = bound;
    }
}

__global__ void k_sec_ctrl_init(SecCtrl *c, int64_t max_iters, int64_t trace_cap, int64_t nlayers)
{
    *c = SecCtrl{};
    c->best_k = -1;
    c->kstar = -1;
    c->k_last = -1;
    c->max_iters = max_iters;
    c->trace_cap = trace_cap;
    c->nlayers = nlayers;
}

__global__ __launch_bounds__(kSB) void k_sec_rows_in(const int32_t *row_of, const int32_t *orig, int64_t n,
                                                     int nlayers, int L, int64_t nrows, int32_t *rowp,
                                                     int32_t *cnt, int32_t *lay_lo, int32_t *lay_hi, SecCtrl *ctrl)
{
    const int64_t p = (int64_t)blockIdx.x * kSB + threadIdx.x;
    if (p >= n) return;
    const int64_t v = orig[p];
    for (int l = 0; l < L; ++l) {
        int32_t r = l < nlayers ? row_of[l * n + v] : -1;
        if (r < -1 || r >= nrows) {
            atomicOr((unsigned long long *)&ctrl->bad_input, 1ULL);
            r = -1;
        }
        rowp[l * n + p] = r;
        if (r >= 0) {
            atomicAdd(&cnt[r], 1);
            atomicMin(&lay_lo[r], l);
            atomicMax(&lay_hi[r], l);
        }
    }
}

__global__ __launch_bounds__(kSB) void k_sec_rows_fill(const int32_t *rowp, int64_t n, int L, const int32_t *rptr,
                                                       int32_t *cur, int32_t *rmem)
{
    const int64_t p = (int64_t)blockIdx.x * kSB + threadIdx.x;
    if (p >= n) return;
    for (int l = 0; l < L; ++l) {
        const int32_t r = rowp[l * n + p];
        if (r >= 0) rmem[rptr[r] + atomicAdd(&cur[r], 1)] = (int32_t)p;
    }
}

__global__ __launch_bounds__(kSB) void k_sec_start(const int64_t *lam_label, const int32_t *orig, int64_t n,
                                                   const int64_t *mu, int64_t nrows, int64_t *lam_pos,
                                                   int64_t *lamp, SecCtrl *ctrl)
{
    const int64_t i = (int64_t)blockIdx.x * kSB + threadIdx.x;
    unsigned long long ml = 0, mm = 0;
    if (i < n) {
        const int64_t x = lam_label[orig[i]];
        lam_pos[i] = x;
        lamp[i] = x;
        ml = (unsigned long long)(x < 0 ? -x : x);
    }
    if (i < nrows) {
        const int64_t m = mu[i];
        if (m < 0) atomicOr((unsigned long long *)&ctrl->bad_input, 2ULL);
        else mm = (unsigned long long)m;
    }
    ml = wave_max(ml);
    mm = wave_max(mm);
    if ((threadIdx.x & 63) == 0) {
        if (ml) atomicMax((unsigned long long *)&ctrl->init_lmax, ml);
        if (mm) atomicMax((unsigned long long *)&ctrl->init_mmax, mm);
    }
}

__global__ __launch_bounds__(kSB) void k_sec_add_mu(const int32_t *rptr, const int32_t *rmem, const int64_t *mu,
                                                    int64_t nrows, int64_t *lamp)
{
    const int lane = threadIdx.x & 63;
    const int64_t q = (int64_t)blockIdx.x * (kSB / 64) + (threadIdx.x >> 6);
    if (q >= nrows) return;
    const int64_t m = mu[q];
    if (m == 0) return;
    for (int32_t e = rptr[q] + lane; e < rptr[q + 1]; e += 64)
        atomicAdd((unsigned long long *)&lamp[rmem[e]], (unsigned long long)m);
}

__global__ void k_sec_bound(SecCtrl *c)
{
    c->lamp_bound = c->init_lmax + c->nlayers * c->init_mmax;
}

__global__ __launch_bounds__(kSB) void k_sec_uf_init(int32_t *parent, int64_t n)
{
    const int64_t v = (int64_t)blockIdx.x * kSB + threadIdx.x;
    if (v < n) parent[v] = (int32_t)v;
}

__global__ __launch_bounds__(kSB) void k_sec_uf_final(int32_t *parent, int64_t n)
{
    const int64_t v = (int64_t)blockIdx.x * kSB + threadIdx.x;
    if (v < n) parent[v] = uf_find(parent, (int32_t)v);
}

inline unsigned blocks_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int sec_layers_inst(int nlayers)
{
    return nlayers <= 1 ? 1 : (nlayers <= 2 ? 2 : (nlayers <= 4 ? 4 : 8));
}

hipError_t launch_sec_scan(const SecScanArgs &a, int L, int64_t nslices, hipStream_t st)
{
    const dim3 grid(blocks_of(a.g.n, kSB), (unsigned)nslices);
    switch (L) {
    case 1: hipLaunchKernelGGL(k_sec_scan<1>, grid, dim3(kSB), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_sec_scan<2>, grid, dim3(kSB), 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_sec_scan<4>, grid, dim3(kSB), 0, st, a); break;
    case 8: hipLaunchKernelGGL(k_sec_scan<8>, grid, dim3(kSB), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sec_node(const SecNodeArgs &a, int L, hipStream_t st)
{
    const dim3 grid(blocks_of(a.g.n, kSB));
    switch (L) {
    case 1: hipLaunchKernelGGL(k_sec_node<1>, grid, dim3(kSB), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_sec_node<2>, grid, dim3(kSB), 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_sec_node<4>, grid, dim3(kSB), 0, st, a); break;
    case 8: hipLaunchKernelGGL(k_sec_node<8>, grid, dim3(kSB), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sec_rows(const SecRowArgs &a, hipStream_t st)
{
    if (a.nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sec_rows, dim3(blocks_of(a.nrows, kSB / 64)), dim3(kSB), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sec_control(const SecControlArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_sec_control, dim3(1), dim3(kSB), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sec_ctrl_init(SecCtrl *ctrl, int64_t max_iters, int64_t trace_cap, int64_t nlayers,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_sec_ctrl_init, dim3(1), dim3(1), 0, st, ctrl, max_iters, trace_cap, nlayers);
    return hipGetLastError();
}

hipError_t launch_sec_rows_in(const int32_t *row_of, const int32_t *orig, int64_t n, int nlayers, int L,
                              int64_t nrows, int32_t *rowp, int32_t *cnt, int32_t *lay_lo, int32_t *lay_hi,
                              SecCtrl *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_sec_rows_in, dim3(blocks_of(n, kSB)), dim3(kSB), 0, st, row_of, orig, n, nlayers, L, nrows,
                       rowp, cnt, lay_lo, lay_hi, ctrl);
    return hipGetLastError();
}

hipError_t launch_sec_rows_fill(const int32_t *rowp, int64_t n, int L, const int32_t *rptr, int32_t *cur,
                                int32_t *rmem, hipStream_t st)
{
    hipLaunchKernelGGL(k_sec_rows_fill, dim3(blocks_of(n, kSB)), dim3(kSB), 0, st, rowp, n, L, rptr, cur, rmem);
    return hipGetLastError();
}

hipError_t launch_sec_start(const int64_t *lam_label, const int32_t *orig, int64_t n, const int64_t *mu,
                            int64_t nrows, int64_t *lam_pos, int64_t *lamp, SecCtrl *ctrl, hipStream_t st)
{
    const int64_t m = n > nrows ? n : nrows;
    hipLaunchKernelGGL(k_sec_start, dim3(blocks_of(m, kSB)), dim3(kSB), 0, st, lam_label, orig, n, mu, nrows, lam_pos,
                       lamp, ctrl);
    return hipGetLastError();
}

hipError_t launch_sec_add_mu(const int32_t *rptr, const int32_t *rmem, const int64_t *mu, int64_t nrows,
                             int64_t *lamp, SecCtrl *ctrl, hipStream_t st)
{
    if (nrows > 0)
        hipLaunchKernelGGL(k_sec_add_mu, dim3(blocks_of(nrows, kSB / 64)), dim3(kSB), 0, st, rptr, rmem, mu, nrows,
                           lamp);
    hipLaunchKernelGGL(k_sec_bound, dim3(1), dim3(1), 0, st, ctrl);
    return hipGetLastError();
}

hipError_t launch_sec_uf_init(int32_t *parent, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_sec_uf_init, dim3(blocks_of(n, kSB)), dim3(kSB), 0, st, parent, n);
    return hipGetLastError();
}

hipError_t launch_sec_uf_final(int32_t *parent, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_sec_uf_final, dim3(blocks_of(n, kSB)), dim3(kSB), 0, st, parent, n);
    return hipGetLastError();
}

}  // namespace f2m
