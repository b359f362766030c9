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

// max of x over the block, returned to every thread (buf: kSB/64 floats)
__device__ __forceinline__ float block_max(float x, float *buf)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    x = wave_max(x);
    __syncthreads();
    if (lane == 0) buf[w] = x;
    __syncthreads();
    float r = buf[0];
    for (int i = 1; i < kSB / 64; ++i) r = fmaxf(r, buf[i]);
    return r;
}

// the three smallest (Z, column) of a list, increasing; empty entries are
// (INT64_MAX, INT32_MAX)
struct T3 {
    int64_t z[3];
    int32_t i[3];

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int j = 0; j < 3; ++j) { z[j] = INT64_MAX; i[j] = INT32_MAX; }
    }
    __device__ __forceinline__ static bool less(int64_t za, int32_t ia, int64_t zb, int32_t ib)
    {
        return za < zb || (za == zb && ia < ib);
    }
    __device__ __forceinline__ void ins(int64_t zz, int32_t u)
    {
        if (!less(zz, u, z[2], i[2])) return;
        z[2] = zz; i[2] = u;
        if (less(z[2], i[2], z[1], i[1])) { const int64_t a = z[1]; z[1] = z[2]; z[2] = a; const int32_t b = i[1]; i[1] = i[2]; i[2] = b; }
        if (less(z[1], i[1], z[0], i[0])) { const int64_t a = z[0]; z[0] = z[1]; z[1] = a; const int32_t b = i[0]; i[0] = i[1]; i[1] = b; }
    }
};

constexpr int kWin = 1024;   // column tiles tested for culling at a time

template <int L>
__global__ __launch_bounds__(kSB) void k_sec_scan(SecScanArgs a)
{
    if (!a.support && a.ctrl->done) return;
    __shared__ float4 sc[kSB];
    __shared__ long long slp[kSB];
    __shared__ int32_t sr[L][kSB];
    __shared__ int32_t so[kSB];
    __shared__ float redf[kSB / 64];
    __shared__ unsigned long long redu[kSB / 64];
    __shared__ unsigned int keep[kWin / 32];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t n = a.g.n;
    const int64_t rblk = blockIdx.x;
    const int64_t p = rblk * kSB + t;
    const int64_t sl = blockIdx.y;
    const int64_t c0 = sl * a.slice_len, c1 = min(n, c0 + a.slice_len);
    const float colmax = col_bound(a.g.xy2max, a.ctrl->lamp_bound);
    const bool live = p < n;

    Row rw;
    T3 nt;
    nt.clear();
    int32_t cn = 0, cz = 0;
    int64_t rn = 0, pr = 0;
    int32_t rv[L];
    int64_t mv[L];
    T3 xt[L];
    int32_t xn[L], xzr[L];
    int64_t xb[L];   // bound of the subtour row's third smallest crossing Z (INT64_MAX: none)
    int32_t lab = 0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        rv[l] = live ? a.rowp[l * n + p] : -1;
        mv[l] = rv[l] >= 0 ? a.mu[rv[l]] : 0;
        xt[l].clear();
        xn[l] = xzr[l] = 0;
        xb[l] = INT64_MAX;
    }
    if (live) {
        const float4 cv = a.col[p];
        rw.xv = cv.x;
        rw.yv = cv.y;
        rw.lamv = a.lamp[p];
        rw.theta = a.support ? 0 : kThetaNone;
        rw.v = p;
        lab = a.g.orig[p];
        if (!a.support && a.seed) {
            // Z of (p, u) from global memory
            auto zpair = [&](int64_t u) {
                const float4 cu = a.col[u];
                const int32_t dx = (int32_t)(rw.xv - cu.x), dy = (int32_t)(rw.yv - cu.y);
                int64_t z = 2 * nint_sqrt((int64_t)dx * dx + (int64_t)dy * dy) - rw.lamv - a.lamp[u];
#pragma unroll
                for (int l = 0; l < L; ++l)
                    if (rv[l] >= 0 && a.rowp[l * n + u] == rv[l]) z += 2 * mv[l];
                return z;
            };
            // each subtour row's bound from its seed edges
#pragma unroll
            for (int l = 0; l < L; ++l) {
                if (rv[l] < 0) continue;
                int64_t mx = INT64_MIN;
                int c3 = 0;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int2 e = a.rseed[(int64_t)rv[l] * 3 + j];
                    if (e.x < 0 || e.y < 0 || e.x >= n || e.y >= n) continue;
                    const float4 cm = a.col[e.x], cu = a.col[e.y];
                    const int32_t dx = (int32_t)(cm.x - cu.x), dy = (int32_t)(cm.y - cu.y);
                    int64_t z = 2 * nint_sqrt((int64_t)dx * dx + (int64_t)dy * dy) - a.lamp[e.x] - a.lamp[e.y];
#pragma unroll
                    for (int l2 = 0; l2 < L; ++l2) {
                        const int32_t r1 = a.rowp[l2 * n + e.x];
                        if (r1 >= 0 && a.rowp[l2 * n + e.y] == r1) z += 2 * a.mu[r1];
                    }
                    mx = z > mx ? z : mx;
                    ++c3;
                }
                if (c3 == 3) xb[l] = mx;
            }
            int64_t th = 0;
            bool full = true;
            int cnt = 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int64_t u = a.seed[j * n + p];
                if (u >= 0 && u < n && u != p) {
                    const int64_t z = zpair(u);
                    th = z > th ? z : th;
                    ++cnt;
                }
            }
            full = cnt == 3;
#pragma unroll
            for (int l = 0; l < L; ++l) {
                if (rv[l] < 0) continue;
                cnt = 0;
                int64_t mx = INT64_MIN;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int64_t u = a.seed[((1 + l) * 3 + j) * n + p];
                    if (u >= 0 && u < n && u != p && a.rowp[l * n + u] != rv[l]) {
                        const int64_t z = zpair(u);
                        mx = z > mx ? z : mx;
                        ++cnt;
                    }
                }
                // the own list's bound or the row's, whichever is smaller
                const int64_t b = cnt == 3 ? (mx < xb[l] ? mx : xb[l]) : xb[l];
                if (b == INT64_MAX) full = false;
                else th = b > th ? b : th;
            }
            // three distinct columns of a list bound its third smallest
            if (full) rw.theta = th < kThetaNone ? th : kThetaNone;
        }
        set_filter(rw, colmax);
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
        nt.ins(z, (int32_t)u);
        int64_t th = nt.z[2];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (rv[l] >= 0) {
                if (sr[l][c] != rv[l]) {
                    xt[l].ins(z, (int32_t)u);
                    if (z < 0) ++xn[l];
                    else if (z == 0) ++xzr[l];
                }
                const int64_t b = xt[l].z[2] < xb[l] ? xt[l].z[2] : xb[l];
                th = b > th ? b : th;
            }
        }
        th = th > 0 ? th : 0;
        th = th < kThetaNone ? th : kThetaNone;
        if (th < rw.theta) { rw.theta = th; set_filter(rw, colmax); }
    };

    // the rows' half-radius of the filter: hv = (theta + Lam' + 1) / 2
    auto hv_row = [&]() { return live ? (float)(0.5 * (double)(rw.theta + rw.lamv + 1)) : -INFINITY; };
    // boxes of the block's rows (tile rblk) and of this wave's (its two sub-tiles)
    const float4 rbox = a.g.box[rblk * kBoxStride];
    float4 wbox;
    {
        const float4 b0 = a.g.box[rblk * kBoxStride + 1 + 2 * wave], b1 = a.g.box[rblk * kBoxStride + 2 + 2 * wave];
        wbox = make_float4(fminf(b0.x, b1.x), fmaxf(b0.y, b1.y), fminf(b0.z, b1.z), fmaxf(b0.w, b1.w));
    }
    const unsigned long long lm = __ballot(live);
    unsigned long long tested = 0;   // wave-uniform

    // every row of the block against column tile gt (global tile index)
    auto scan_tile = [&](int64_t gt) {
        const int64_t base = gt * kSB;
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
        const float hvw = wave_max(hv_row());
        for (int s = 0; s < kSubs; ++s) {
            const int64_t s0 = base + s * kSubCols;
            if (s0 >= c1) break;
            if (!may_pass(a.g.box[gt * kBoxStride + 1 + s], wbox, hvw, a.tile_h[gt * kBoxStride + 1 + s])) continue;
            const int64_t cols = min((int64_t)kSubCols, c1 - s0);
            // ordered pairs: the wave's rows by the sub-tile's columns, less the diagonal
            const unsigned long long half = (s >> 1) == wave && gt == rblk
                                                ? __popcll(lm & ((s & 1) ? 0xffffffff00000000ULL : 0xffffffffULL))
                                                : 0ULL;
            tested += (unsigned long long)__popcll(lm) * (unsigned long long)cols - half;
            // the sub-tile's columns that pass the filter, as a mask (each
            // filter value computed once), then their exact evaluation
            unsigned int pm = 0;
            for (int g = s * kSubCols; g < (s + 1) * kSubCols; g += kSGroup) {
                float f[kSGroup];
                float m = INFINITY;
#pragma unroll
                for (int q = 0; q < kSGroup; ++q) {
                    f[q] = filter_value(rw, sc[g + q]);
                    m = fminf(m, f[q]);
                }
                if (m <= rw.thr) {
                    unsigned int gm = 0;
#pragma unroll
                    for (int q = 0; q < kSGroup; ++q) gm |= f[q] <= rw.thr ? (1u << q) : 0u;
                    pm |= gm << (g - s * kSubCols);
                }
            }
            while (pm) {
                const int q = __ffs(pm) - 1;
                pm &= pm - 1;
                eval(s * kSubCols + q, base);
            }
        }
    };

    const int64_t t0 = c0 / kSB, t1 = (c1 + kSB - 1) / kSB;   // the slice's tiles
    const bool own_in = rblk >= t0 && rblk < t1;
    // the block's own tile first: its rows' nearest columns tighten theta
    if (own_in) scan_tile(rblk);
    for (int64_t w0 = t0; w0 < t1; w0 += kWin) {
        const float hvb = block_max(hv_row(), redf);
        for (int j = t; j < kWin / 32; j += kSB) keep[j] = 0u;
        __syncthreads();
        for (int64_t j = t; j < kWin && w0 + j < t1; j += kSB) {
            const int64_t gt = w0 + j;
            if (gt != rblk && may_pass(a.g.box[gt * kBoxStride], rbox, hvb, a.tile_h[gt * kBoxStride]))
                atomicOr(&keep[j >> 5], 1u << (j & 31));
        }
        __syncthreads();
        const int words = (int)((min((int64_t)kWin, t1 - w0) + 31) / 32);
        for (int wd = 0; wd < words; ++wd) {
            unsigned int bits = keep[wd];   // the same in every thread
            while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1;
                scan_tile(w0 + wd * 32 + b);
            }
        }
    }
    // pairs tested by the block
    {
        if (lane == 0) redu[wave] = tested;
        __syncthreads();
        if (t == 0) {
            unsigned long long tot = 0;
            for (int w = 0; w < kSB / 64; ++w) tot += redu[w];
            if (a.tpart) a.tpart[sl * gridDim.x + rblk] = tot;
        }
    }
    if (!live || a.support) return;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        a.pz[(sl * 3 + j) * n + p] = nt.z[j];
        a.pzi[(sl * 3 + j) * n + p] = nt.i[j];
    }
    a.pc[(sl * 2) * n + p] = cn;
    a.pc[(sl * 2 + 1) * n + p] = cz;
    a.prn[sl * n + p] = rn;
    a.ppr[sl * n + p] = pr;
#pragma unroll
    for (int l = 0; l < L; ++l) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            a.pxz[((sl * L + l) * 3 + j) * n + p] = xt[l].z[j];
            a.pxi[((sl * L + l) * 3 + j) * n + p] = xt[l].i[j];
        }
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
        T3 nt;
        nt.clear();
        int64_t cn = 0, cz = 0, rn = 0, pr = 0;
        T3 xt[L];
        int32_t xn[L], xzr[L];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            xt[l].clear();
            xn[l] = xzr[l] = 0;
        }
        for (int64_t s = 0; s < a.nslices; ++s) {
#pragma unroll
            for (int j = 0; j < 3; ++j) nt.ins(a.pz[(s * 3 + j) * n + p], a.pzi[(s * 3 + j) * n + p]);
            cn += a.pc[(s * 2) * n + p];
            cz += a.pc[(s * 2 + 1) * n + p];
            rn += a.prn[s * n + p];
            pr += a.ppr[s * n + p];
#pragma unroll
            for (int l = 0; l < L; ++l) {
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    xt[l].ins(a.pxz[((s * L + l) * 3 + j) * n + p], a.pxi[((s * L + l) * 3 + j) * n + p]);
                xn[l] += a.pxc[((s * L + l) * 2) * n + p];
                xzr[l] += a.pxc[((s * L + l) * 2 + 1) * n + p];
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) a.seed[j * n + p] = nt.i[j] == INT32_MAX ? -1 : nt.i[j];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            if (a.rowp[l * n + p] < 0) continue;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                a.xz[(l * 3 + j) * n + p] = xt[l].z[j];
                a.seed[((1 + l) * 3 + j) * n + p] = xt[l].i[j] == INT32_MAX ? -1 : xt[l].i[j];
            }
            a.xc[(l * 2) * n + p] = xn[l];
            a.xc[(l * 2 + 1) * n + p] = xzr[l];
        }
        // eq. 10 on the 2nd and 3rd smallest Z of the degree row (n >= 4)
        const int64_t lamv = a.lam_in[p];
        const int64_t st = gdp_step(nt.z[1] + nt.z[2]);
        const int64_t nxt = lamv + st;
        if (copy_best) a.lam_best[p] = a.lam_out[p];
        a.lam_out[p] = nxt;
        a.lamp[p] = nxt;
        const int64_t lab = a.g.orig[p];
        v[0] = (unsigned long long)lamv;
        v[2] = (unsigned long long)rn;
        v[3] = (unsigned long long)pr;
        v[4] = (nt.z[1] > 0 || nt.z[2] < 0) ? 1 : 0;
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
        // the row's three smallest crossing (Z, edge), the edge (member,
        // column) packed member-major: values decide the step, edges only
        // seed the next scan's bound
        int64_t tz[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
        long long te[3] = {-1, -1, -1};
        auto ins = [&](int64_t z, long long ed) {
            if (!(z < tz[2] || (z == tz[2] && (unsigned long long)ed < (unsigned long long)te[2]))) return;
            tz[2] = z; te[2] = ed;
#pragma unroll
            for (int j = 2; j > 0; --j) {
                if (tz[j] < tz[j - 1] || (tz[j] == tz[j - 1] && (unsigned long long)te[j] < (unsigned long long)te[j - 1])) {
                    const int64_t x = tz[j]; tz[j] = tz[j - 1]; tz[j - 1] = x;
                    const long long y = te[j]; te[j] = te[j - 1]; te[j - 1] = y;
                }
            }
        };
        long long neg = 0, zero = 0;
        for (int32_t e = e0 + lane; e < e1; e += 64) {
            const int64_t m = a.rmem[e];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int32_t u = a.seed[((1 + l) * 3 + j) * n + m];
                ins(a.xz[(l * 3 + j) * n + m], u < 0 ? -1LL : (long long)(((unsigned long long)m << 32) | (uint32_t)u));
            }
            neg += a.xc[(l * 2) * n + m];
            zero += a.xc[(l * 2 + 1) * n + m];
        }
        // the wave's three smallest: merge with the partner lane's list at
        // each distance (the values are a multiset: the order does not matter)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            long long uz[3], ue[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                uz[j] = __shfl_xor((long long)tz[j], o, 64);
                ue[j] = __shfl_xor(te[j], o, 64);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) ins(uz[j], ue[j]);
        }
        if (lane < 3) {
            const long long ed = lane == 0 ? te[0] : (lane == 1 ? te[1] : te[2]);
            a.rseed[q * 3 + lane] = ed < 0 ? make_int2(-1, -1) : make_int2((int32_t)(ed >> 32), (int32_t)(ed & 0xffffffff));
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
    unsigned long long tt = 0;
    for (int64_t b = threadIdx.x; b < a.ntpart; b += kSB) tt += a.tpart[b];
    tt = wave_sum(tt);
    __shared__ unsigned long long redt[kSB / 64];
    if (lane == 0) redt[w] = tt;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 1; q < kSB / 64; ++q) tt += redt[q];
    c->pairs_tested += tt;
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

__global__ __launch_bounds__(kSB) void k_sec_tiles(const int64_t *lamp, int64_t n, float *tile_h)
{
    __shared__ float redf[kSB / 64];
    const int64_t p = (int64_t)blockIdx.x * kSB + threadIdx.x;
    // the same float the scan's column record holds
    const float h = p < n ? (float)(0.5 * (double)lamp[p]) : -INFINITY;
    float hs = h;
#pragma unroll
    for (int o = kSubCols / 2; o > 0; o >>= 1) hs = fmaxf(hs, __shfl_xor(hs, o, 64));
    if ((threadIdx.x & (kSubCols - 1)) == 0) tile_h[blockIdx.x * kBoxStride + 1 + threadIdx.x / kSubCols] = hs;
    const float hm = block_max(h, redf);
    if (threadIdx.x == 0) tile_h[blockIdx.x * kBoxStride] = hm;
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

hipError_t launch_sec_tiles(const int64_t *lamp, int64_t n, float *tile_h, hipStream_t st)
{
    hipLaunchKernelGGL(k_sec_tiles, dim3(blocks_of(n, kSB)), dim3(kSB), 0, st, lamp, n, tile_h);
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
