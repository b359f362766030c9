// HIP kernels of libf2m for gfx950 (MI355X): the complete-graph GDP scan,
// the per-node update with its device-side stop test, trivial-x extraction
// and the certificate.
//
// Notation (arXiv 2011.08170): c_e is the edge length, lambda_v the node
// multiplier, v^e = c_e - lambda_u - lambda_v the adjusted length (eq. 9).
// Fixed point: Lam = 2*lambda (int64), Z_uv = 2c_uv - Lam_u - Lam_v.
//
// The scan.  For every ordered pair (v, u) the GDP needs Z_vu only when it
// can change node v's statistics: the four smallest (Z, u) of the row and
// the counts of Z < 0, Z == 0 and the sum of the negative Z.  With theta_v
// an upper bound on the row's 4th smallest Z (seeded from the previous
// iteration's top-4 columns, tightened as the lane's own list fills) and
// theta_v >= 0, a pair matters only if Z <= theta_v, i.e.
//     2c <= R := theta_v + Lam_v + Lam_u.
// Since c = nint(sqrt D) >= sqrt(D) - 1/2, that needs sqrt(D) < (R+1)/2 = h,
// i.e.  E = D - h^2 < 0.  With h = hv + hu (hv per row, hu = Lam_u/2 per
// column) and centred coordinates,
//     E = K_v + q_u + (-2x_v) x_u + (-2y_v) y_u + (-2hv) hu,
//     K_v = x_v^2 + y_v^2 - hv^2,   q_u = x_u^2 + y_u^2 - hu^2,
// three FMAs per pair in float.  Every rounding in that chain is bounded by
// 2^-24 of M_v = 2(x_v^2 + y_v^2 + hv^2 + max_u(x_u^2 + y_u^2) + max_u hu^2),
// so a pair is skipped only when the float value exceeds K_v by more than
// 2^-18 M_v; everything else is re-evaluated exactly in int64 (exact D,
// nint(sqrt D) from sqrtf corrected by integer tests).  The filter is
// conservative: it never drops a pair with Z <= theta_v.
#include "f2m_internal.h"
#include "f2m_filter.h"
#include "f2m_device.h"

#include <float.h>
#include <limits.h>

#include <hipcub/hipcub.hpp>

namespace f2m {

constexpr int kBlock = 256;   // threads per workgroup (4 waves of 64)
constexpr int kTile = kTileCols;   // columns staged in LDS per tile
constexpr int kGroup = 8;     // columns per filter test
constexpr int kCollectBuf = 128;   // pairs a wave stages in LDS while collecting
constexpr int kSeedWin = 16;       // positions each side of a node whose distances seed its bounds
static_assert(kBlock == kTile, "one update block covers one column tile");
static_assert(kSubCols % kGroup == 0, "filter groups do not straddle sub-tiles");
constexpr int32_t kNoIdx = INT32_MAX;

// ---------------------------------------------------------------------------
// exact arithmetic helpers
// ---------------------------------------------------------------------------

// Z_vu from centred float coordinates (exact integers, |.| <= 2^19).
__device__ __forceinline__ int64_t exact_z(float xv, float yv, int64_t lamv, float xu, float yu,
                                           int64_t lamu)
{
    // the differences are exact (integers below 2^20); fma(fx, fx, fy * fy)
    // rounds twice, within 2^-23 relative of D
    const float fx = xv - xu, fy = yv - yu;
    const int32_t dx = (int32_t)fx, dy = (int32_t)fy;
    const int64_t D = (int64_t)dx * dx + (int64_t)dy * dy;
    return 2 * nint_sqrt_f(D, fmaf(fx, fx, fy * fy)) - lamv - lamu;
}

__device__ __forceinline__ bool key_less(int64_t za, int32_t ua, int64_t zb, int32_t ub)
{
    return za < zb || (za == zb && ua < ub);
}

// ---------------------------------------------------------------------------
// per-row scan state
// ---------------------------------------------------------------------------

struct Top4 {
    int64_t z[kTop];
    int32_t id[kTop];

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int j = 0; j < kTop; ++j) { z[j] = INT64_MAX; id[j] = kNoIdx; }
    }
    // keeps the four smallest keys in increasing (Z, u) order
    __device__ __forceinline__ void insert(int64_t zz, int32_t u)
    {
        if (!key_less(zz, u, z[3], id[3])) return;
        z[3] = zz; id[3] = u;
#pragma unroll
        for (int j = 3; j > 0; --j) {
            if (key_less(z[j], id[j], z[j - 1], id[j - 1])) {
                const int64_t tz = z[j]; z[j] = z[j - 1]; z[j - 1] = tz;
                const int32_t ti = id[j]; id[j] = id[j - 1]; id[j - 1] = ti;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// block reductions
// ---------------------------------------------------------------------------

// max over each aligned group of kSubCols lanes of a wave
static_assert(kSubCols <= 64 && 64 % kSubCols == 0, "sub-tiles split a wave evenly");
__device__ __forceinline__ float sub_max(float x)
{
#pragma unroll
    for (int o = kSubCols / 2; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
    return x;
}

// Sums (or maxes) one value per thread over the block; the result is
// returned to every thread.  `buf` holds kBlock/64 entries.
template <typename T, bool kMax>
__device__ __forceinline__ T block_reduce(T x, T *buf)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    x = kMax ? wave_max(x) : wave_sum(x);
    __syncthreads();
    if (lane == 0) buf[w] = x;
    __syncthreads();
    T r = buf[0];
    for (int i = 1; i < kBlock / 64; ++i) r = kMax ? (buf[i] > r ? buf[i] : r) : r + buf[i];
    return r;
}

// ---------------------------------------------------------------------------
// row scan: rows x column slices over the sorted order
// ---------------------------------------------------------------------------

// Upper bound of the 4th smallest Z of row p from four seed columns
// (positions): any four distinct columns bound the 4th order statistic.
// Returns false when fewer than four usable seeds exist.
__device__ __forceinline__ bool seeded_bound(const ScanArgs &a, int64_t p, float xv, float yv, int64_t lamv,
                                             int64_t *out)
{
    const int64_t n = a.g.n;
    int64_t mx = INT64_MIN;
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < kTop; ++j) {
        const int32_t u = a.seed[j * n + p];
        if (u >= 0 && u < n && u != p) {
            const float4 cu = a.lv.col[u];
            const int64_t z = exact_z(xv, yv, lamv, cu.x, cu.y, a.lv.lam[u]);
            mx = z > mx ? z : mx;
            ++cnt;
        }
    }
    *out = mx;
    return cnt == kTop;
}

// MODE kModeGdp: per row the four smallest (Z, label), #Z<0, #Z==0 and the
// sum of the negative Z over the slice's columns, written as partials.
// MODE kModeCert: the sum over the slice of min(0, Z) (theta = 0), added to
// acc[0].  MODE kModeCollect: every pair with Z <= theta_row, as Morton
// positions (lo, hi).
template <int R, int MODE, bool CULL>
__device__ __forceinline__ void rowscan_body(const ScanArgs &a, const int64_t rblk, const int64_t sl)
{
    if (a.check_done && a.lv.ctrl->done) return;
    __shared__ float4 sc[kTile];
    __shared__ long long slam[kTile];   // the tile's Lam (exact)
    __shared__ int32_t so[kTile];     // the tile's labels
    __shared__ float redf[kBlock / 64];
    __shared__ unsigned long long redu[kBlock / 64];
    const int t = threadIdx.x;
    const int64_t n = a.g.n;
    // the slice's columns: a contiguous range, or (interleaved culled scan)
    // every S-th surviving tile of all columns, starting with the sid-th
    const bool il = CULL && a.interleave > 0;
    const int64_t S = il ? a.interleave : 1, sid = il ? sl : 0;
    const int64_t c0 = il ? 0 : sl * a.slice_len;
    const int64_t c1 = il ? n : min(n, c0 + a.slice_len);
    const float colmax = col_bound(a.g.xy2max, a.lv.ctrl->maxabs_lam);

    Row rw[R];
    Top4 top[R];
    int32_t neg[R], zero[R];
    int64_t rn[R];
    float hvmax = -INFINITY;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t p = rblk * (kBlock * R) + r * kBlock + t;
        rw[r].v = p;
        top[r].clear();
        neg[r] = 0; zero[r] = 0; rn[r] = 0;
        if (p < n) {
            const float4 cv = a.lv.col[p];
            rw[r].xv = cv.x; rw[r].yv = cv.y;
            rw[r].lamv = a.lv.lam[p];
            int64_t th;
            if (MODE == kModeCert) {
                th = 0;
            } else {
                int64_t mx;
                const bool ok = a.seed && seeded_bound(a, p, cv.x, cv.y, rw[r].lamv, &mx);
                if (MODE == kModeGdp) th = ok ? (mx > 0 ? mx : 0) : kThetaNone;
                else th = ok ? (mx > 0 ? mx : 0) + a.slack : a.theta;
            }
            rw[r].theta = th;
            set_filter(rw[r], colmax);
            hvmax = fmaxf(hvmax, -0.5f * rw[r].c);
        } else {
            rw[r].xv = rw[r].yv = 0.0f;
            rw[r].lamv = 0; rw[r].theta = 0;
            rw[r].a = rw[r].b = rw[r].c = 0.0f;
            rw[r].thr = -INFINITY;   // never passes
        }
    }

    // culling data: the largest row half-radius and the box of the block's
    // rows, and the same for the rows of this wave
    float4 rbox = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
    float4 wbox = rbox;
    float hvw = -INFINITY;
    const int wave = t >> 6;
    if (CULL) {
        hvw = wave_max(hvmax);
        hvmax = block_reduce<float, true>(hvmax, redf);
        const int64_t ntiles = (n + kTile - 1) / kTile;
        for (int r = 0; r < R; ++r) {
            const int64_t ti = rblk * R + r;
            if (ti < ntiles) {
                const float4 b = a.g.box[ti * kBoxStride];
                rbox.x = fminf(rbox.x, b.x); rbox.y = fmaxf(rbox.y, b.y);
                rbox.z = fminf(rbox.z, b.z); rbox.w = fmaxf(rbox.w, b.w);
                // the wave's 64 rows of this row tile are whole sub-tiles
                for (int s = wave * (64 / kSubCols); s < (wave + 1) * (64 / kSubCols); ++s) {
                    const float4 sb = a.g.box[ti * kBoxStride + 1 + s];
                    wbox.x = fminf(wbox.x, sb.x); wbox.y = fmaxf(wbox.y, sb.y);
                    wbox.z = fminf(wbox.z, sb.z); wbox.w = fmaxf(wbox.w, sb.w);
                }
            }
        }
    }

    const int lane = t & 63;
    // collection: per-wave staging of the pairs found (see scan_cols)
    __shared__ int2 cbuf[kBlock / 64][kCollectBuf];
    __shared__ int cfill_s[kBlock / 64];
    volatile int *cfill = cfill_s;
    if (MODE == kModeCollect && lane == 0) cfill[wave] = 0;
    // ordered (row, column) pairs of this wave's rows and the columns
    // [col0, col1), the diagonal excluded; wave-uniform
    unsigned long long tested = 0;
    auto count_tested = [&](int64_t col0, int64_t col1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t w0 = rblk * (kBlock * R) + r * kBlock + wave * 64;
            const int64_t w1 = min(n, w0 + 64);
            if (w1 > w0)
                tested += (unsigned long long)((w1 - w0) * (col1 - col0) -
                                               max((int64_t)0, min(w1, col1) - max(w0, col0)));
        }
    };
    // every row of this lane against the LDS columns [g0, g1) of the tile
    // that starts at position `tile`
    // the exact evaluation of column c of the LDS tile (position tile + c)
    // for row r, after the float filter passed it
    auto eval_col = [&](int r, int64_t tile, int c) {
        const int64_t u = tile + c;
        if (u >= c1 || u == rw[r].v) return;
        const float4 cd = sc[c];
        if (!(filter_value(rw[r], cd) <= rw[r].thr)) return;   // theta may have dropped
        const int64_t z = exact_z(rw[r].xv, rw[r].yv, rw[r].lamv, cd.x, cd.y, slam[c]);
        if (MODE == kModeCert) {
            if (z < 0) rn[r] += z;
            return;
        }
        if (MODE == kModeCollect) {
            // the wave's pairs gather in its LDS buffer (the lanes with a
            // pair take consecutive places after the wave's fill count); the
            // buffer goes out at the end with one atomic, a full buffer's
            // excess goes out at once
            const bool emit = z <= rw[r].theta;
            const unsigned long long em = __ballot(emit);
            if (em) {
                const int base = cfill[wave];
                if (emit) {
                    const int32_t pv = (int32_t)rw[r].v, pu = (int32_t)u;
                    const int2 pr = make_int2(min(pv, pu), max(pv, pu));
                    const int slot = base + __popcll(em & ((1ULL << lane) - 1ULL));
                    if (slot < kCollectBuf) {
                        cbuf[wave][slot] = pr;
                    } else {
                        const unsigned long long gs = atomicAdd(a.count, 1ULL);
                        if ((int64_t)gs < a.cap) a.out[gs] = pr;
                    }
                }
                if (lane == __ffsll((long long)em) - 1) cfill[wave] = base + __popcll(em);
            }
            return;
        }
        if (z > rw[r].theta) return;
        if (z < 0) { ++neg[r]; rn[r] += z; }
        else if (z == 0) ++zero[r];
        top[r].insert(z, so[c]);
        if (top[r].id[3] != kNoIdx) {
            const int64_t nt = top[r].z[3] > 0 ? top[r].z[3] : 0;
            if (nt < rw[r].theta) { rw[r].theta = nt; set_filter(rw[r], colmax); }
        }
    };
    // the float filter over the group of kGroup columns at g: per row a bit
    // mask of the columns that pass (0 when none can)
    auto filter_group = [&](int g, unsigned (&pm)[R]) {
        float m[R];
#pragma unroll
        for (int r = 0; r < R; ++r) m[r] = INFINITY;
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            const float4 cd = sc[g + q];
#pragma unroll
            for (int r = 0; r < R; ++r) m[r] = fminf(m[r], filter_value(rw[r], cd));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pm[r] = 0;
            if (m[r] <= rw[r].thr) {
#pragma unroll
                for (int q = 0; q < kGroup; ++q)
                    pm[r] |= (filter_value(rw[r], sc[g + q]) <= rw[r].thr) ? (1u << q) : 0u;
            }
        }
    };
    // every row of this lane against the LDS columns [g0, g1), evaluated
    // group by group: each lane walks its own passing columns, so lanes
    // passing at different columns are evaluated together
    auto scan_cols = [&](int64_t tile, int g0, int g1) {
        for (int g = g0; g < g1; g += kGroup) {
            unsigned pm[R];
            filter_group(g, pm);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                while (pm[r]) {
                    const int q = __ffs(pm[r]) - 1;
                    pm[r] &= pm[r] - 1;
                    eval_col(r, tile, g + q);
                }
            }
        }
    };
    auto load_tile = [&](int64_t tile) {
        __syncthreads();
        const int64_t cc = tile + t;
        sc[t] = (cc < c1) ? a.lv.col[cc] : make_float4(0.0f, 0.0f, 0.0f, INFINITY);
        slam[t] = (cc < c1) ? a.lv.lam[cc] : 0;
        so[t] = (cc < c1) ? a.g.orig[cc] : 0;
        __syncthreads();
    };
    // the next tile's column of this thread, fetched while the current tile
    // is scanned
    float4 nx_c = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
    long long nx_l = 0;
    int32_t nx_o = 0;
    auto fetch_tile = [&](int64_t tile) {
        const int64_t cc = tile + t;
        const bool in = cc < c1;
        nx_c = in ? a.lv.col[cc] : make_float4(0.0f, 0.0f, 0.0f, INFINITY);
        nx_l = in ? a.lv.lam[cc] : 0;
        nx_o = in ? a.g.orig[cc] : 0;
    };
    auto store_tile = [&]() {
        __syncthreads();
        sc[t] = nx_c;
        slam[t] = nx_l;
        so[t] = nx_o;
        __syncthreads();
    };

    bool any = !CULL;   // block-uniform: some column tile was scanned
    if (!CULL) {
        for (int64_t tile = c0; tile < c1; tile += kTile) {
            load_tile(tile);
            const int ntile = (int)min((int64_t)kTile, c1 - tile);
            count_tested(tile, tile + ntile);
            scan_cols(tile, 0, ntile);
        }
    } else {
        // The slice's tiles are tested in parallel (one per thread) against
        // the block's rows; the survivors are compacted, in order, into an
        // LDS list.  Each wave then tests the eight sub-tiles of a loaded
        // tile in parallel (one per lane) against its own rows and scans
        // the survivors.
        __shared__ int32_t tlist[kBlock];
        __shared__ int32_t wcnt[kBlock / 64];
        const int64_t t0 = c0 / kTile, t1 = (c1 + kTile - 1) / kTile;
        int64_t jbase = 0;   // survivors in the chunks before
        for (int64_t base = t0; base < t1; base += kBlock) {
            const int64_t ti = base + t;
            const bool ok = ti < t1 && may_pass(a.g.box[ti * kBoxStride], rbox, hvmax,
                                                a.lv.tile_hmax[ti * kBoxStride]);
            const unsigned long long mk = __ballot(ok);
            __syncthreads();   // the previous chunk's list is no longer read
            if (lane == 0) wcnt[wave] = __popcll(mk);
            __syncthreads();
            int off = 0, total = 0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) {
                off += (w < wave) ? wcnt[w] : 0;
                total += wcnt[w];
            }
            if (ok) tlist[off + __popcll(mk & ((1ULL << lane) - 1ULL))] = (int32_t)(ti - t0);
            __syncthreads();
            // this slice's survivors: global index = sid (mod S)
            const int j0 = (int)((((sid - jbase) % S) + S) % S);
            jbase += total;
            any = any || j0 < total;
            if (j0 < total) fetch_tile((t0 + tlist[j0]) * kTile);
            for (int j = j0; j < total; j += (int)S) {
                const int64_t tj = t0 + tlist[j];
                const int64_t tile = tj * kTile;
                store_tile();
                if (j + S < total) fetch_tile((t0 + tlist[j + S]) * kTile);
                const int ntile = (int)min((int64_t)kTile, c1 - tile);
                const bool sp = lane < kSubs && lane * kSubCols < ntile &&
                                may_pass(a.g.box[tj * kBoxStride + 1 + lane], wbox, hvw,
                                         a.lv.tile_hmax[tj * kBoxStride + 1 + lane]);
                const unsigned long long sm0 = __ballot(sp);
                for (unsigned long long sm = sm0; sm;) {
                    const int sb = __ffsll((long long)sm) - 1;
                    sm &= sm - 1;
                    const int g0 = sb * kSubCols;
                    const int g1 = min(g0 + kSubCols, ntile);
                    count_tested(tile + g0, tile + g1);
                    scan_cols(tile, g0, g1);
                }
            }
        }
    }

    if (a.tested && lane == 0 && tested) atomicAdd(a.tested, tested);
    if (MODE == kModeCollect) {
        __syncthreads();   // every lane's buffer writes are done
        const int fill = min(cfill[wave], kCollectBuf);
        unsigned long long base = 0;
        if (lane == 0 && fill > 0) base = atomicAdd(a.count, (unsigned long long)fill);
        base = __shfl(base, 0, 64);
        for (int i = lane; i < fill; i += 64)
            if ((int64_t)(base + i) < a.cap) a.out[base + i] = cbuf[wave][i];
    }
    if (MODE == kModeGdp && a.pflag && t == 0) a.pflag[sl * a.nrb + rblk] = any ? 1 : 0;
    if (MODE == kModeGdp && (any || !a.pflag)) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t p = rw[r].v;
            if (p >= n) continue;
#pragma unroll
            for (int j = 0; j < kTop; ++j) {
                a.pz[(sl * kTop + j) * n + p] = top[r].z[j];
                a.pi[(sl * kTop + j) * n + p] = top[r].id[j];
            }
            a.pneg[sl * n + p] = neg[r];
            a.pzero[sl * n + p] = zero[r];
            a.prowneg[sl * n + p] = rn[r];
        }
    }
    if (MODE == kModeCert) {
        int64_t s = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) s += rn[r];
        const unsigned long long tot = block_reduce<unsigned long long, false>((unsigned long long)s, redu);
        if (threadIdx.x == 0 && tot != 0) atomicAdd(&a.acc[0], tot);
    }
}

// Culled scan, one row per lane, every wave on its own.  A wave holds 64
// Morton-consecutive rows (a small box); it tests the column tiles against
// that box (64 tiles at a time, one per lane), then the 32-column sub-tiles
// of eight surviving tiles at a time (one per lane), and keeps the
// survivors dealt to this slice (every S-th, round-robin) in a short list.  The list's
// sub-tiles are staged two at a time in the wave's own LDS (the next pair is
// fetched into registers meanwhile) and scanned by every lane against its
// row: the float filter marks columns in a 64-bit mask, the marked ones get
// the exact evaluation.  No wave waits for another until the end, where the
// block agrees on whether any of its waves scanned a column (pflag).
//
// QUAD: the four waves of a block hold the same 64 rows (block rblk of 64
// rows) and are four of the parts the survivors are dealt to (part
// 4 sl + wave of 4 S); at the end they merge their top-4 lists and counts in
// LDS and the block writes one partial per row for its slice.  Without
// QUAD each wave holds its own 64 of the block's 256 rows (part sl of S).
template <int MODE, bool QUAD>
__device__ __forceinline__ void rowscan_wave_body(const ScanArgs &a, const int64_t rblk, const int64_t sl)
{
    static_assert(kSubCols == 32 && kSubs == 8, "two sub-tiles per wave-wide stage, eight per tile test");
    if (a.check_done && a.lv.ctrl->done) return;
    constexpr int kList = 128;
    __shared__ int32_t wl[kBlock / 64][kList];       // the wave's sub-tile list
    __shared__ int32_t tl[kBlock / 64][64];          // the wave's pending surviving tiles
    __shared__ float4 wc[kBlock / 64][64];           // staged columns
    __shared__ long long wlam[kBlock / 64][64];
    __shared__ int32_t wlab[kBlock / 64][64];
    __shared__ int32_t wpos[kBlock / 64][64];        // position, -1: none
    __shared__ unsigned long long redu[kBlock / 64];
    __shared__ int bany;
    __shared__ int2 cbuf[kBlock / 64][MODE == kModeCollect ? kCollectBuf : 1];
    __shared__ int cfill_s[kBlock / 64];
    volatile int *cfill = cfill_s;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t n = a.g.n;
    const int64_t S0 = a.interleave > 0 ? a.interleave : 1, sl0 = a.interleave > 0 ? sl : 0;
    const int64_t S = QUAD ? 4 * S0 : S0, sid = QUAD ? 4 * sl0 + wave : sl0;
    // candidate lists (see ScanArgs::lst): an iteration that may use them
    // is left to the update, which evaluates them per row; a full scan may
    // store them during the walk (build, margin 2 LD)
    const bool lists = QUAD && MODE == kModeGdp && a.lst != nullptr;
    if (lists && a.lv.ctrl->list_ok != 0) return;
    const int64_t LD = lists ? a.lv.ctrl->list_D : 0;
    const bool build = LD > 0;
    const float colmax = col_bound(a.g.xy2max, a.lv.ctrl->maxabs_lam);
    if (t == 0) bany = 0;
    if (lane == 0) cfill[wave] = 0;

    Row rw;
    Top4 top;
    int32_t neg = 0, zero = 0;
    int64_t rn = 0;
    top.clear();
    const int64_t p = QUAD ? rblk * 64 + lane : rblk * kBlock + t;
    rw.v = p;
    if (p < n) {
        const float4 cv = a.lv.col[p];
        rw.xv = cv.x; rw.yv = cv.y;
        rw.lamv = a.lv.lam[p];
        int64_t th;
        if (MODE == kModeCert) {
            th = 0;
        } else {
            int64_t mx;
            const bool ok = a.seed && seeded_bound(a, p, cv.x, cv.y, rw.lamv, &mx);
            if (MODE == kModeGdp) th = ok ? (mx > 0 ? mx : 0) : kThetaNone;
            else th = ok ? (mx > 0 ? mx : 0) + a.slack : a.theta;
        }
        rw.theta = th;
        rw.slk = build ? 2 * LD : 0;
        set_filter(rw, colmax);
    } else {
        rw.xv = rw.yv = 0.0f;
        rw.lamv = 0; rw.theta = 0;
        rw.a = rw.b = rw.c = 0.0f;
        rw.thr = -INFINITY;   // never passes
    }
    int lc = 0;   // list entries found (build)
    // this lane's list: part `sid` of the S parts, entry i at
    // lst[(sid * kLW + i) * n + p] (consecutive lanes, consecutive addresses)
    // this wave's part of its rows' lists gathers in LDS during the walk;
    // the block writes them out compacted per row at the end
    __shared__ int32_t lbuf[QUAD && MODE == kModeGdp ? kBlock / 64 : 1][kLW][64];
    __syncthreads();   // bany and cfill are set

    // the wave's rows: positions [w0, w1), their box (two sub-tile boxes
    // of the row tile rt)
    const int64_t w0 = QUAD ? rblk * 64 : rblk * kBlock + wave * 64, w1 = min(n, w0 + 64);
    const int64_t rt = w0 / kTile;
    const int s0 = (int)((w0 % kTile) / kSubCols);
    float4 wbox = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
    if (w1 > w0) {
        for (int s = s0; s < s0 + 64 / kSubCols; ++s) {
            const float4 sb = a.g.box[rt * kBoxStride + 1 + s];
            wbox.x = fminf(wbox.x, sb.x); wbox.y = fmaxf(wbox.y, sb.y);
            wbox.z = fminf(wbox.z, sb.z); wbox.w = fmaxf(wbox.w, sb.w);
        }
    }
    const int64_t ntiles = (n + kTile - 1) / kTile;
    unsigned long long tested = 0;
    bool scanned = false;

    // exact evaluation of staged column c against this lane's row
    auto eval = [&](int c) {
        const int64_t u = wpos[wave][c];
        if (u < 0 || u == rw.v) return;
        const float4 cd = wc[wave][c];
        if (!(filter_value(rw, cd) <= rw.thr)) return;   // theta may have dropped
        const int64_t z = exact_z(rw.xv, rw.yv, rw.lamv, cd.x, cd.y, wlam[wave][c]);
        if (MODE == kModeCert) {
            if (z < 0) rn += z;
            return;
        }
        if (MODE == kModeCollect) {
            // the wave's pairs gather in its LDS buffer; a full buffer's
            // excess goes out at once
            bool emit = z <= rw.theta;
            if (emit && a.excl) {
                // skip the pairs already known: binary search of the key
                const uint64_t key = ((uint64_t)(uint32_t)min(rw.v, u) << 32) | (uint64_t)(uint32_t)max(rw.v, u);
                int64_t lo = 0, hi = a.nexcl;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (a.excl[mid] < key) lo = mid + 1;
                    else hi = mid;
                }
                emit = !(lo < a.nexcl && a.excl[lo] == key);
            }
            const unsigned long long em = __ballot(emit);
            if (em) {
                const int base = cfill[wave];
                if (emit) {
                    const int32_t pv = (int32_t)rw.v, pu = (int32_t)u;
                    const int2 pr = make_int2(min(pv, pu), max(pv, pu));
                    const int slot = base + __popcll(em & ((1ULL << lane) - 1ULL));
                    if (slot < kCollectBuf) {
                        cbuf[wave][slot] = pr;
                    } else {
                        const unsigned long long gs = atomicAdd(a.count, 1ULL);
                        if ((int64_t)gs < a.cap) a.out[gs] = pr;
                    }
                }
                if (lane == __ffsll((long long)em) - 1) cfill[wave] = base + __popcll(em);
            }
            return;
        }
        if (build && z <= rw.theta + rw.slk) {
            if (lc < kLW) lbuf[QUAD && MODE == kModeGdp ? wave : 0][lc][lane] = (int32_t)u;
            ++lc;
        }
        if (z > rw.theta) return;
        if (z < 0) { ++neg; rn += z; }
        else if (z == 0) ++zero;
        top.insert(z, wlab[wave][c]);
        if (top.id[3] != kNoIdx) {
            const int64_t nt = top.z[3] > 0 ? top.z[3] : 0;
            if (nt < rw.theta) { rw.theta = nt; set_filter(rw, colmax); }
        }
    };

    // the next pair of list entries' columns, one per lane (lanes 0-31
    // entry e, lanes 32-63 entry e + 1)
    float4 nx_c = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
    long long nx_l = 0;
    int32_t nx_o = 0, nx_u = -1;
    auto fetch = [&](int e, int cnt) {
        const int ee = e + (lane >> 5);
        nx_c = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
        nx_l = 0;
        nx_o = 0;
        nx_u = -1;
        if (ee < cnt) {
            const int32_t st = wl[wave][ee];
            const int64_t cc = (int64_t)(st / kSubs) * kTile + (int64_t)(st % kSubs) * kSubCols + (lane & 31);
            if (cc < n) {
                nx_c = a.lv.col[cc];
                nx_l = a.lv.lam[cc];
                nx_o = a.g.orig[cc];
                nx_u = (int32_t)cc;
            }
        }
    };

    if (w1 > w0) {
        // The culling radius comes from the rows' starting thresholds: every
        // slice must see the same survivors in the same order, or the
        // round-robin deal would lose or repeat sub-tiles.
        const float hvw = wave_max(p < n ? -0.5f * rw.c : -INFINITY);
        const unsigned long long below = (1ULL << lane) - 1ULL;
        int64_t tb = 0;               // next chunk of 64 tiles
        int tcnt = 0, tpos = 0;       // surviving tiles pending in tl: [tpos, tcnt)
        int64_t kk = 0;               // surviving sub-tiles so far (round-robin)
        for (;;) {
            int cnt = 0;
            while (cnt <= kList - 64) {
                if (tpos == tcnt) {
                    // the next surviving tiles, one chunk of 64 at a time
                    wave_sync();   // tl is no longer read
                    tpos = tcnt = 0;
                    while (tcnt == 0 && tb < ntiles) {
                        const int64_t ti = tb + lane;
                        const bool ok = ti < ntiles &&
                                        may_pass(a.g.box[ti * kBoxStride], wbox, hvw, a.lv.tile_hmax[ti * kBoxStride]);
                        const unsigned long long mk = __ballot(ok);
                        if (ok) tl[wave][__popcll(mk & below)] = (int32_t)ti;
                        tcnt = __popcll(mk);
                        tb += 64;
                    }
                    wave_sync();
                    if (tcnt == 0) break;
                }
                // up to eight pending tiles at once: lane 8i + s tests
                // sub-tile s of the i-th
                const int ti8 = lane >> 3, s8 = lane & 7;
                const int nt8 = min(8, tcnt - tpos);
                bool sp = false;
                int64_t tj = 0;
                if (ti8 < nt8) {
                    tj = tl[wave][tpos + ti8];
                    sp = (int64_t)s8 * kSubCols < n - tj * kTile &&
                         may_pass(a.g.box[tj * kBoxStride + 1 + s8], wbox, hvw,
                                  a.lv.tile_hmax[tj * kBoxStride + 1 + s8]);
                }
                const unsigned long long sm = __ballot(sp);
                const int64_t my = kk + __popcll(sm & below);
                const bool take = sp && (my % S) == sid;
                const unsigned long long tk = __ballot(take);
                if (take) wl[wave][cnt + __popcll(tk & below)] = (int32_t)(tj * kSubs + s8);
                cnt += __popcll(tk);
                kk += __popcll(sm);
                tpos += nt8;
            }
            if (cnt == 0) break;
            scanned = true;
            wave_sync();   // the list is written
            fetch(0, cnt);
            for (int e = 0; e < cnt; e += 2) {
                wave_sync();   // the previous pair's reads are done
                wc[wave][lane] = nx_c;
                wlam[wave][lane] = nx_l;
                wlab[wave][lane] = nx_o;
                wpos[wave][lane] = nx_u;
                wave_sync();
                const int ncol = (e + 1 < cnt) ? 64 : 32;
                // ordered pairs of the wave's rows against the staged columns
                for (int h = 0; h < ncol / 32; ++h) {
                    const int32_t st = wl[wave][e + h];
                    const int64_t cs = (int64_t)(st / kSubs) * kTile + (int64_t)(st % kSubs) * kSubCols;
                    const int64_t ce = min(n, cs + kSubCols);
                    tested += (unsigned long long)((w1 - w0) * (ce - cs) - max((int64_t)0, min(w1, ce) - max(w0, cs)));
                }
                if (e + 2 < cnt) fetch(e + 2, cnt);
                // float filter, kGroup columns at a time, into a pass mask
                unsigned long long pm = 0;
                // (each column's filter value is computed once; the group's
                // bits are gathered in 32 bits and placed with one shift)
                for (int g = 0; g < ncol; g += kGroup) {
                    float f[kGroup];
                    float m = INFINITY;
#pragma unroll
                    for (int q = 0; q < kGroup; ++q) {
                        f[q] = filter_value(rw, wc[wave][g + q]);
                        m = fminf(m, f[q]);
                    }
                    if (m <= rw.thr) {
                        unsigned int gm = 0;
#pragma unroll
                        for (int q = 0; q < kGroup; ++q) gm |= f[q] <= rw.thr ? (1u << q) : 0u;
                        pm |= (unsigned long long)gm << g;
                    }
                }
                while (pm) {
                    const int c = __ffsll((long long)pm) - 1;
                    pm &= pm - 1;
                    eval(c);
                }
            }
        }
    }

    // the count of pairs tested: one store per workgroup when k_update sums
    // them, else one atomic per wave
    const bool tstore = QUAD && MODE == kModeGdp && a.tpart != nullptr;
    if (!tstore && a.tested && lane == 0 && tested) atomicAdd(a.tested, tested);
    if (MODE == kModeCollect) {
        // the workgroup's buffers go out behind one atomic
        __shared__ unsigned long long cbase;
        __syncthreads();   // every wave's buffer is complete
        if (t == 0) {
            unsigned long long tot = 0;
            for (int w = 0; w < kBlock / 64; ++w) tot += (unsigned long long)min(cfill[w], kCollectBuf);
            cbase = tot ? atomicAdd(a.count, tot) : 0ULL;
        }
        __syncthreads();
        unsigned long long base = cbase;
        for (int w = 0; w < wave; ++w) base += (unsigned long long)min(cfill[w], kCollectBuf);
        const int fill = min(cfill[wave], kCollectBuf);
        for (int i = lane; i < fill; i += 64)
            if ((int64_t)(base + i) < a.cap) a.out[base + i] = cbuf[wave][i];
    }
    if (build) {
        // The block's 64 rows: every row's entries from the four parts go out
        // as one contiguous run, the rows one after another in the group's
        // segment of kListCap entries (see ScanArgs::lst).
        __shared__ int32_t lc_s[QUAD && MODE == kModeGdp ? kBlock / 64 : 1][64];
        __shared__ int32_t off_s[64];
        const int wv = QUAD && MODE == kModeGdp ? wave : 0;
        lc_s[wv][lane] = lc;
        __syncthreads();
        if (wave == 0) {
            int tot = 0;
            bool ovf = false;
            for (int w = 0; w < kBlock / 64; ++w) {
                const int c = lc_s[w][lane];
                ovf = ovf || c > kLW;
                tot += min(c, kLW);
            }
            const int mine = (ovf || p >= n) ? 0 : tot;
            int incl = mine;   // inclusive scan over the wave's lanes
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            off_s[lane] = ovf ? -1 : incl - mine;
            if (p < n) {
                a.lcnt[sl * n + p] = ovf ? -1 : tot;
                a.loff[sl * n + p] = incl - mine;
            }
            if (ovf && p < n) const_cast<Ctrl *>(a.lv.ctrl)->list_over = 1;   // the next update rebuilds
        }
        __syncthreads();
        if (off_s[lane] >= 0 && p < n) {
            int start = off_s[lane];
            for (int w = 0; w < wave; ++w) start += min(lc_s[w][lane], kLW);
            int32_t *seg = a.lst + (sl * (int64_t)gridDim.x + rblk) * kListCap;
            const int c = min(lc, kLW);
            for (int i = 0; i < c; ++i) seg[start + i] = lbuf[wv][i][lane];
        }
    }
    if (MODE == kModeGdp && QUAD) {
        // waves 1-3 hand their rows' lists and counts to wave 0
        __shared__ long long mz[QUAD && MODE == kModeGdp ? 3 : 1][kTop][64];
        __shared__ int32_t mi[QUAD && MODE == kModeGdp ? 3 : 1][kTop][64];
        __shared__ int32_t mneg[QUAD && MODE == kModeGdp ? 3 : 1][64], mzero[QUAD && MODE == kModeGdp ? 3 : 1][64];
        __shared__ long long mrn[QUAD && MODE == kModeGdp ? 3 : 1][64];
        if (wave > 0) {
#pragma unroll
            for (int j = 0; j < kTop; ++j) {
                mz[wave - 1][j][lane] = top.z[j];
                mi[wave - 1][j][lane] = top.id[j];
            }
            mneg[wave - 1][lane] = neg;
            mzero[wave - 1][lane] = zero;
            mrn[wave - 1][lane] = rn;
        }
        if (lane == 0) redu[wave] = tested;
        __syncthreads();
        if (tstore && t == 0) {
            unsigned long long tt = 0;
            for (int w = 0; w < kBlock / 64; ++w) tt += redu[w];
            a.tpart[sl * (int64_t)gridDim.x + rblk] = tt;
        }
        if (wave == 0 && p < n) {
            for (int w = 0; w < 3; ++w) {
#pragma unroll
                for (int j = 0; j < kTop; ++j) top.insert(mz[w][j][lane], mi[w][j][lane]);
                neg += mneg[w][lane];
                zero += mzero[w][lane];
                rn += mrn[w][lane];
            }
#pragma unroll
            for (int j = 0; j < kTop; ++j) {
                a.pz[(sl * kTop + j) * n + p] = top.z[j];
                a.pi[(sl * kTop + j) * n + p] = top.id[j];
            }
            a.pneg[sl * n + p] = neg;
            a.pzero[sl * n + p] = zero;
            a.prowneg[sl * n + p] = rn;
        }
    }
    if (MODE == kModeGdp && !QUAD) {
        if (scanned && lane == 0) bany = 1;
        __syncthreads();
        const bool any = bany != 0;
        if (a.pflag && t == 0) a.pflag[sl * a.nrb + rblk] = any ? 1 : 0;
        if ((any || !a.pflag) && p < n) {
#pragma unroll
            for (int j = 0; j < kTop; ++j) {
                a.pz[(sl * kTop + j) * n + p] = top.z[j];
                a.pi[(sl * kTop + j) * n + p] = top.id[j];
            }
            a.pneg[sl * n + p] = neg;
            a.pzero[sl * n + p] = zero;
            a.prowneg[sl * n + p] = rn;
        }
    }
    if (MODE == kModeCert) {
        const unsigned long long tot = block_reduce<unsigned long long, false>((unsigned long long)rn, redu);
        if (threadIdx.x == 0 && tot != 0) atomicAdd(&a.acc[0], tot);
    }
}

template <int R, int MODE, bool CULL>
__global__ __launch_bounds__(kBlock) void k_rowscan(ScanArgs a)
{
    rowscan_body<R, MODE, CULL>(a, blockIdx.x, blockIdx.y);
}

// the culled scan with one row per lane, four waves per 64 rows (see
// rowscan_wave_body)
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_rowscan_w(ScanArgs a)
{
    rowscan_wave_body<MODE, true>(a, blockIdx.x, blockIdx.y);
}

// batched GDP scan: one block per (instance, row block, slice)
template <int R, bool CULL>
__global__ __launch_bounds__(kBlock) void k_rowscan_batch(const ScanArgs *args, const BatchScanItem *items)
{
    const BatchScanItem w = items[blockIdx.x];
    ScanArgs a = args[w.inst];
    if (a.lv.ctrl->k_next & 1) a.lv.lam = a.lam_odd;
    if constexpr (CULL && R == 1) rowscan_wave_body<kModeGdp, false>(a, w.row_block, w.slice);
    else rowscan_body<R, kModeGdp, CULL>(a, w.row_block, w.slice);
}

// ---------------------------------------------------------------------------
// per-node step, iteration record and stop test (shared by the complete-graph
// update and the candidate-graph step)
// ---------------------------------------------------------------------------

struct RowOut {
    unsigned long long sumlam = 0, rowneg = 0, unsat = 0, bad = 0, nonzero = 0, hsh = 0, sumblam = 0;
    long long maxstep = 0, maxabs = 0;
    float hmax = -INFINITY;
};

// A row's own data, loaded at the start of a launch (at a clamped position,
// so the loads are unconditional and travel together with the others).
struct RowIn {
    int64_t v;       // label
    int bv;          // right-hand side of the degree row
    float2 xy;       // centred coordinates (when the column records are kept)
    int64_t lprev;   // lam_out on entry: Lam_{k-1}
};

__device__ __forceinline__ RowIn row_in(const Geo &g, const float4 *col, const int64_t *lam_out, int64_t pc)
{
    RowIn r;
    r.v = g.orig[pc];
    r.bv = g.b ? (int)g.b[pc] : 2;
    r.xy = col ? reinterpret_cast<const float2 *>(col)[2 * pc] : make_float2(0.0f, 0.0f);
    r.lprev = lam_out[pc];
    return r;
}

// Step of the row at position p from its merged statistics: eq. 10 on the
// 2nd and 3rd smallest Z; writes Lam_{k+1} and the per-node outputs.
// The four smallest go to z4p / i4p by position ([j][n], coalesced) when
// those are given, and to z4 / i4 by label (4v + j) when those are.
__device__ __forceinline__ void step_row(const Geo &g, int64_t p, const RowIn &ri, const Top4 &top, int64_t cn,
                                         int64_t cz, int64_t rn, int64_t lamv, bool copy_best, int64_t *lam_out,
                                         int64_t *lam_best, int64_t *z4, int32_t *i4, int32_t *seed,
                                         int32_t *neg, int32_t *zero, int64_t *step, float4 *col, RowOut &o,
                                         int64_t *z4p = nullptr, int32_t *i4p = nullptr)
{
    const int64_t n = g.n;
    const int64_t v = ri.v;
    // eq. 10 for a row with right-hand side b (Sec. 3): the b-th and
    // (b+1)-th smallest Z (F2M: b = 2, the 2nd and 3rd); the row needs b + 1
    // edges (n >= 4 on the complete graph)
    const int bv = ri.bv;
    // the three candidates are formed from values and then selected (a
    // selected index into the list would put it in scratch memory)
    const int64_t z0 = top.z[0], z1 = top.z[1], z2 = top.z[2], z3 = top.z[3];
    const bool h1 = top.id[1] != kNoIdx, h2 = top.id[2] != kNoIdx, h3 = top.id[3] != kNoIdx;
    const bool has = bv == 1 ? h1 : (bv == 2 ? h2 : h3);
    const int64_t st1 = h1 ? gdp_step(z0 + z1) : 0, st2 = h2 ? gdp_step(z1 + z2) : 0, st3 = h3 ? gdp_step(z2 + z3) : 0;
    const int64_t st = has ? (bv == 1 ? st1 : (bv == 2 ? st2 : st3)) : 0;
    const bool un1 = z0 > 0 || z1 < 0, un2 = z1 > 0 || z2 < 0, un3 = z2 > 0 || z3 < 0;
    const bool unsat = bv == 1 ? un1 : (bv == 2 ? un2 : un3);
    const int64_t nxt = lamv + st;
    if (copy_best) lam_best[p] = ri.lprev;
    lam_out[p] = nxt;
    if (col) {
        // only the (h, q) half changes: the (x, y) half of every record stays
        // untouched, so threads of the same launch may read it (list step)
        const float4 cv = col_record(ri.xy.x, ri.xy.y, nxt);
        reinterpret_cast<float2 *>(col)[2 * p + 1] = make_float2(cv.z, cv.w);
        o.hmax = cv.z;
    }
    // the seeds' position gathers are issued together (from a clamped label)
    int32_t sp[kTop];
#pragma unroll
    for (int j = 0; j < kTop; ++j) sp[j] = seed ? g.pos[top.id[j] != kNoIdx ? top.id[j] : 0] : 0;
#pragma unroll
    for (int j = 0; j < kTop; ++j) {
        const bool ok = top.id[j] != kNoIdx;
        if (z4p) {
            z4p[j * n + p] = top.z[j];
            i4p[j * n + p] = ok ? top.id[j] : -1;
        }
        if (z4) {
            z4[kTop * v + j] = top.z[j];
            i4[kTop * v + j] = ok ? top.id[j] : -1;
        }
        if (seed) seed[j * n + p] = ok ? sp[j] : -1;
    }
    const int64_t deg2 = 2 * cn + cz;
    if (neg) neg[v] = (int32_t)cn;
    if (zero) zero[v] = (int32_t)cz;
    if (step) step[v] = st;
    o.sumlam = (unsigned long long)lamv;
    o.sumblam = (unsigned long long)(bv * lamv);
    o.rowneg = (unsigned long long)rn;
    o.unsat = unsat ? 1 : 0;
    o.bad = deg2 != 2 * bv ? 1 : 0;
    o.nonzero = st != 0 ? 1 : 0;
    o.maxstep = st < 0 ? -st : st;
    o.maxabs = nxt < 0 ? -nxt : nxt;
    o.hsh = mix64((uint64_t)lamv ^ (0x9E3779B97F4A7C15ULL * (uint64_t)(v + 1)));
}

// Block reductions of the rows' records into the block's slot (plain stores:
// the control kernel that sums the slots runs after this launch).  Called by
// every thread of the block.  `tested` (summed over the block's threads) is
// the count of scanned pairs added to pairs_tested.
constexpr int kRecV = 10;   // record entries: 8 of the Ctrl order, the pairs tested, sum b Lam

__device__ __forceinline__ void block_record(RowOut o, float *tile_hmax, int64_t blk, unsigned long long *slots,
                                             unsigned long long tested)
{
    constexpr int kV = kRecV;
    __shared__ unsigned long long red8[kBlock / 64][kV];
    __shared__ float redf[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (tile_hmax) {
        // a block of kBlock positions is one column tile
        const float hs = sub_max(o.hmax);
        if ((threadIdx.x & (kSubCols - 1)) == 0) tile_hmax[blk * kBoxStride + 1 + threadIdx.x / kSubCols] = hs;
        const float hm = block_reduce<float, true>(o.hmax, redf);
        if (threadIdx.x == 0) tile_hmax[blk * kBoxStride] = hm;
    }
    // entries: sum Lam, sum rowneg, #unsat, #bad, max step, #nonzero, hash,
    // max |Lam_{k+1}|, pairs tested, sum b Lam; entries 4 and 7 are maxima,
    // the rest sums
    unsigned long long v[kV] = {o.sumlam, o.rowneg, o.unsat, o.bad, (unsigned long long)o.maxstep, o.nonzero,
                                o.hsh, (unsigned long long)o.maxabs, tested, o.sumblam};
#pragma unroll
    for (int i = 0; i < kV; ++i) v[i] = (i == 4 || i == 7) ? wave_max(v[i]) : wave_sum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kV; ++i) red8[w][i] = v[i];
    }
    __syncthreads();
    if (w == 0 && lane < kV) {
        unsigned long long mine = red8[0][lane];
        for (int q = 1; q < kBlock / 64; ++q) {
            const unsigned long long x = red8[q][lane];
            mine = (lane == 4 || lane == 7) ? (x > mine ? x : mine) : mine + x;
        }
        slots[blk * kSlotW + lane] = mine;
    }
}

// The iteration's control, by one block after the launch that filled the
// nblk slots: sums them, writes the iteration record, takes the stop
// decision and the candidate lists' decision (see ScanArgs::lst).  `kinds`
// (or null) receives the scan kind of iteration k; `progress` (or null) the
// host's progress word.
__device__ __forceinline__ void control_body(int64_t n, int64_t k, Ctrl *ctrl, int64_t *trace, int64_t nblk,
                                             const unsigned long long *slots, bool lists, int32_t *kinds,
                                             long long *progress)
{
    constexpr int kV = kRecV;
    __shared__ unsigned long long red8[kBlock / 64][kV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long acc[kV];
#pragma unroll
    for (int i = 0; i < kV; ++i) acc[i] = 0;
    for (int64_t b = threadIdx.x; b < nblk; b += kBlock) {
#pragma unroll
        for (int i = 0; i < kV; ++i) {
            const unsigned long long x = slots[b * kSlotW + i];
            acc[i] = (i == 4 || i == 7) ? (x > acc[i] ? x : acc[i]) : acc[i] + x;
        }
    }
#pragma unroll
    for (int i = 0; i < kV; ++i) acc[i] = (i == 4 || i == 7) ? wave_max(acc[i]) : wave_sum(acc[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < kV; ++i) red8[w][i] = acc[i];
    }
    __syncthreads();
    if (w != 0) return;
    unsigned long long got = 0;
    if (lane < kV) {
        got = red8[0][lane];
        for (int q = 1; q < kBlock / 64; ++q) {
            const unsigned long long x = red8[q][lane];
            got = (lane == 4 || lane == 7) ? (x > got ? x : got) : got + x;
        }
    }
    const long long sl = (long long)__shfl(got, 0, 64);
    const long long rnsum = (long long)__shfl(got, 1, 64);
    const long long un = (long long)__shfl(got, 2, 64);
    const long long bd = (long long)__shfl(got, 3, 64);
    const long long ms = (long long)__shfl(got, 4, 64);
    const long long nz = (long long)__shfl(got, 5, 64);
    const unsigned long long hh = __shfl(got, 6, 64);
    const long long mx = (long long)__shfl(got, 7, 64);
    const unsigned long long tt = __shfl(got, 8, 64);
    const long long sbl = (long long)__shfl(got, 9, 64);
    // the control block is read into LDS with one load per lane, decided on
    // there by lane 0 and written back with one store per lane (a chain of
    // dependent global accesses costs more than the decision itself)
    constexpr int kCW = (int)(sizeof(Ctrl) / sizeof(long long));
    static_assert(sizeof(Ctrl) % sizeof(long long) == 0 && kCW <= 64, "Ctrl fits one wave's words");
    __shared__ long long cw[kCW];
    long long *const gw = reinterpret_cast<long long *>(ctrl);
    if (lane < kCW) cw[lane] = gw[lane];
    wave_sync();
    if (lane == 0) {
        Ctrl *const c = reinterpret_cast<Ctrl *>(cw);
        c->pairs_tested += tt;
        // 2 L = sum_v b_v Lam_v + sum_e min(0, Z_e); each unordered pair sits
        // in two rows
        const long long dual2 = sbl + rnsum / 2;
        const long long kr = k - c->k_first;   // record index of iteration k
        if (trace && kr < c->trace_cap) {
            long long *rec = (long long *)trace + kTraceW * kr;
            rec[0] = k; rec[1] = dual2; rec[2] = un; rec[3] = bd;
            rec[4] = ms; rec[5] = nz; rec[6] = (long long)hh; rec[7] = sl;
        }
        if (c->best_k < 0 || dual2 > c->best_dual2) { c->best_dual2 = dual2; c->best_k = k; }
        long long stop = 0;
        if (bd == 0) stop = 1;                                                      // trivial
        else if (c->handoff_div > 0 && un * c->handoff_div <= n) stop = 5;    // handoff
        else if (nz == 0) stop = 2;                                                 // fixed
        else if (k >= 2 && (kr >= 2 || c->hvalid) && hh == c->h2) stop = 3;  // cycle
        else if (k >= c->max_iters) stop = 4;                                    // cap
        else if (mx >= kLamLimit) { stop = 4; c->overflow = 1; }
        int32_t kind = kScanFull;
        if (lists) {
            // Z moves by at most twice the max step per iteration: lists
            // built with margin 2D stay exact while the steps since the
            // build sum to at most D / 2
            if (kr == 0) c->list_ms0 = ms;
            const bool used = c->list_ok != 0;
            const bool built = !used && c->list_D > 0;
            kind = used ? kScanList : (built ? kScanBuild : kScanFull);
            c->list_uses += used ? 1 : 0;
            c->list_builds += built ? 1 : 0;
            const long long d = used ? c->list_d + ms : ms;
            const bool ok = (used || (built && !c->list_over)) && 2 * d <= c->list_D;
            c->list_ok = ok ? 1 : 0;
            c->list_d = ok ? d : 0;
            if (!ok) {
                // a build whose lists overflowed caps the later margins
                if (built && c->list_over) c->list_Dmax = c->list_D / 2;
                long long D = kListMult * ms;
                if (c->list_Dmax > 0 && D > c->list_Dmax) D = c->list_Dmax;
                const bool go = ms * 16 <= c->list_ms0 && D >= 2 * ms;
                c->list_D = go ? D : 0;
                c->list_over = 0;
            }
        }
        if (kinds && kr < c->trace_cap) kinds[kr] = kind;
        c->pairs_kind[kind] += tt;
        c->k_last = k;
        c->dual2_last = dual2;
        c->ms_last = ms;
        if (stop) {
            c->stop = stop;
            c->kstar = (stop == 3 || stop == 4) ? c->best_k : k;
            c->done = 1;
        } else {
            c->h2 = c->h1;
            c->h1 = hh;
            c->k_next = k + 1;
        }
        c->maxabs_lam = mx;
    }
    wave_sync();
    if (lane < kCW) gw[lane] = cw[lane];
    // the host waits on this word instead of synchronising the stream; it
    // reads nothing else before it synchronises, so no ordering is needed
    if (progress && lane == 0) {
        const Ctrl *const c = reinterpret_cast<const Ctrl *>(cw);
        __hip_atomic_store(progress, 2 * k + (c->done ? 1 : 0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// complete graph: merge the slices' partials, step, reduce, stop test
__device__ __forceinline__ void update_body(const UpdateArgs &a, const int64_t k, const int64_t blk,
                                            const int64_t nblk)
{
    Ctrl *ctrl = a.ctrl;
    // a list iteration: the scan has left this iteration's rows to the
    // update, which evaluates each row's candidate lists itself
    const bool use = a.lists && a.lst && ctrl->list_ok != 0;
    unsigned long long tt = 0;
    if (!use && a.tpart) {
        // the scan's pairs tested in this block's rows (groups of 64), one
        // count per thread (block_record sums them)
        const int64_t groups = (a.g.n + 63) / 64;
        for (int64_t i = threadIdx.x; i < a.nslices * (kBlock / 64); i += kBlock) {
            const int64_t s = i / (kBlock / 64), g = blk * (kBlock / 64) + i % (kBlock / 64);
            if (g < groups) tt += a.tpart[s * groups + g];
        }
    }
    const int64_t n = a.g.n;
    const int64_t p = blk * kBlock + threadIdx.x;
    const bool inb = p < n;
    // every load of a row is issued at a clamped position, so that the loads
    // are unconditional and travel together (a load under a branch waits
    // for the branch's own)
    const int64_t pc = inb ? p : 0;
    // Lam_{k-1} sits in lam_out until it is overwritten
    const bool copy_best = k > 0 && ctrl->best_k == k - 1;
    const RowIn ri = row_in(a.g, a.col, a.lam_out, pc);
    const int64_t lamv = inb ? a.lam_in[pc] : 0;
    RowOut o;
    Top4 top;
    top.clear();
    int64_t cn = 0, cz = 0, rn = 0;
    if (use) {
        // Every column that can matter is in the row's list (see
        // ScanArgs::lst).  A wave's 64 rows (one scan group) have their lists
        // in one segment per slice, row after row.  The wave takes each
        // segment in chunks: every lane marks its own row's run in the chunk,
        // then the lanes evaluate the chunk's entries lane, lane + 64, ...
        // against their rows (the gathers and the exact evaluations spread
        // over the whole wave, the next chunk's entries loaded meanwhile).
        // The counts take only entries with Z <= 0 and go to per-row LDS
        // counters; an entry joins its row's short candidate buffer only if
        // its Z is at most the row's bound (below), and each lane then
        // inserts its row's buffer into its four smallest.
        //
        // The bound: Z_k(u, v) = Z_{k-1}(u, v) - d_u - d_v with d = Lam_k -
        // Lam_{k-1} and |d_v| <= the last max step ms, so the four columns
        // that were smallest in row u at k-1 are all at most B = z4_{k-1}[3]
        // - d_u + ms at k; a column above B has four smaller ones and is not
        // among the four smallest (lists are exact, so this holds over the
        // list too).  A row whose buffer overflows in a chunk walks that
        // chunk's run instead.
        constexpr int kLChunk = 512;
        constexpr int kPB = 16;
        constexpr int kJ = kLChunk / 64;
        __shared__ long long sz[kBlock / 64][kLChunk];
        __shared__ int32_t slab[kBlock / 64][kLChunk];
        __shared__ unsigned char srow[kBlock / 64][kLChunk];
        __shared__ float2 rxy[kBlock / 64][64];
        __shared__ long long rlam[kBlock / 64][64];
        __shared__ long long rbnd[kBlock / 64][64];
        __shared__ unsigned long long rneg[kBlock / 64][64];
        __shared__ unsigned int rcnt[kBlock / 64][64];   // (#neg << 16) + #zero of this chunk
        __shared__ unsigned int rbc[kBlock / 64][64];    // candidates of this chunk
        __shared__ unsigned short rbuf[kBlock / 64][64][kPB];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int64_t grp = blk * (kBlock / 64) + wave, groups = (n + 63) / 64;
        // (without z4p the bound is off; the pointers are chosen first so
        // that the loads are unconditional)
        const bool hz = a.z4p != nullptr;
        const int64_t *zq = hz ? a.z4p + 3 * n : a.lam_in;
        const int32_t *iq = hz ? a.i4p + 3 * n : a.g.orig;
        const int32_t i43 = iq[pc];
        const int64_t z43 = zq[pc];
        const int rcn0 = a.lcnt[pc], rof0 = a.loff[pc];
        const long long bnd = (inb && hz && i43 >= 0) ? z43 - (lamv - ri.lprev) + ctrl->ms_last : INT64_MAX;
        rxy[wave][lane] = ri.xy;
        rlam[wave][lane] = lamv;
        rbnd[wave][lane] = bnd;
        rneg[wave][lane] = 0;
        rcnt[wave][lane] = 0;
        rbc[wave][lane] = 0;
        const float2 *col2 = reinterpret_cast<const float2 *>(a.col);
        for (int64_t sl = 0; sl < a.nslices && grp < groups; ++sl) {
            const int rcn = sl == 0 ? rcn0 : a.lcnt[sl * n + pc], rof = sl == 0 ? rof0 : a.loff[sl * n + pc];
            const int cnt = inb ? min(max(rcn, 0), kLW * (kBlock / 64)) : 0;
            const int off = inb ? rof : 0;
            tt += (unsigned long long)cnt;
            const int total = (int)wave_max((long long)(off + cnt));
            if (total == 0) continue;
            const int32_t *seg = a.lst + (sl * groups + grp) * kListCap;
            // entries past the end are read at the last one (and not used)
            int32_t nu[kJ];
#pragma unroll
            for (int j = 0; j < kJ; ++j) nu[j] = seg[min(j * 64 + lane, total - 1)];
            for (int c0 = 0; c0 < total; c0 += kLChunk) {
                wave_sync();   // the previous chunk's reads are done
                const int lo = max(off, c0), hi = min(off + cnt, c0 + kLChunk);
                for (int e = lo; e < hi; ++e) srow[wave][e - c0] = (unsigned char)lane;
                float2 cxy[kJ];
                int64_t clam[kJ];
                int32_t clab[kJ];
#pragma unroll
                for (int j = 0; j < kJ; ++j) {
                    const int64_t u = nu[j];
                    cxy[j] = col2[2 * u];
                    clam[j] = a.lam_in[u];
                    clab[j] = a.g.orig[u];
                    nu[j] = seg[min(c0 + kLChunk + j * 64 + lane, total - 1)];
                }
                wave_sync();
#pragma unroll
                for (int j = 0; j < kJ; ++j) {
                    const int e = c0 + j * 64 + lane;
                    if (e < total) {
                        const int r = srow[wave][e - c0] & 63;
                        const float2 rv = rxy[wave][r];
                        const int64_t z = exact_z(rv.x, rv.y, rlam[wave][r], cxy[j].x, cxy[j].y, clam[j]);
                        sz[wave][e - c0] = z;
                        slab[wave][e - c0] = clab[j];
                        if (z <= 0) {
                            atomicAdd(&rcnt[wave][r], z < 0 ? 0x10000u : 1u);
                            if (z < 0) atomicAdd(&rneg[wave][r], (unsigned long long)z);
                        }
                        if (z <= rbnd[wave][r]) {
                            const unsigned q = atomicAdd(&rbc[wave][r], 1u);
                            if (q < (unsigned)kPB) rbuf[wave][r][q] = (unsigned short)(e - c0);
                        }
                    }
                }
                wave_sync();
                const unsigned cc = rcnt[wave][lane], m = rbc[wave][lane];
                cn += cc >> 16;
                cz += cc & 0xffffu;
                rn += (long long)rneg[wave][lane];
                rcnt[wave][lane] = 0;
                rneg[wave][lane] = 0;
                rbc[wave][lane] = 0;
                if (m > (unsigned)kPB) {
                    for (int e = lo; e < hi; ++e) top.insert(sz[wave][e - c0], slab[wave][e - c0]);
                } else {
                    for (unsigned q = 0; q < m; ++q) {
                        const int i = rbuf[wave][lane][q];
                        top.insert(sz[wave][i], slab[wave][i]);
                    }
                }
            }
        }
    } else if (a.nslices == 1 && !a.pflag) {
        // one partial per row, already in (Z, u) order
#pragma unroll
        for (int j = 0; j < kTop; ++j) {
            top.z[j] = a.pz[j * n + pc];
            top.id[j] = a.pi[j * n + pc];
        }
        cn = a.pneg[pc];
        cz = a.pzero[pc];
        rn = a.prowneg[pc];
    } else if (inb) {
        // slices in groups of four: the group's loads are issued together,
        // then merged (the merge order does not matter: (Z, u) is a total
        // order and the counts are sums)
        constexpr int kG = 4;
        for (int64_t s0 = 0; s0 < a.nslices; s0 += kG) {
            int64_t gz[kG][kTop];
            int32_t gi[kG][kTop];
#pragma unroll
            for (int q = 0; q < kG; ++q) {
                const int64_t sl = s0 + q;
                const bool ok = sl < a.nslices && (!a.pflag || a.pflag[sl * a.nrb + blk / a.scan_rows] != 0);
#pragma unroll
                for (int j = 0; j < kTop; ++j) {
                    gz[q][j] = ok ? a.pz[(sl * kTop + j) * n + p] : INT64_MAX;
                    gi[q][j] = ok ? a.pi[(sl * kTop + j) * n + p] : kNoIdx;
                }
                if (ok) {
                    cn += a.pneg[sl * n + p];
                    cz += a.pzero[sl * n + p];
                    rn += a.prowneg[sl * n + p];
                }
            }
#pragma unroll
            for (int q = 0; q < kG; ++q)
#pragma unroll
                for (int j = 0; j < kTop; ++j) top.insert(gz[q][j], gi[q][j]);
        }
    }
    if (inb)
        step_row(a.g, p, ri, top, cn, cz, rn, lamv, copy_best, a.lam_out, a.lam_best, a.z4, a.i4, a.seed,
                 a.neg, a.zero, a.step, a.col, o, a.z4p, a.i4p);
    block_record(o, a.tile_hmax, blk, a.slots, tt);
}

__global__ __launch_bounds__(kBlock) void k_update(UpdateArgs a)
{
    if (a.ctrl->done) return;
    update_body(a, a.k, blockIdx.x, gridDim.x);
}

// batched update: the instance's iteration index lives in its Ctrl; the
// lam buffers swap with its parity (the argument struct holds k even)
__global__ __launch_bounds__(kBlock) void k_update_batch(const UpdateArgs *args, const BatchTileItem *items)
{
    const BatchTileItem w = items[blockIdx.x];
    UpdateArgs a = args[w.inst];
    if (a.ctrl->done) return;
    const int64_t k = a.ctrl->k_next;
    if (k & 1) {
        const int64_t *t = a.lam_in;
        a.lam_in = a.lam_out;
        a.lam_out = const_cast<int64_t *>(t);
    }
    update_body(a, k, w.block, a.ctrl->nblocks);
}

// one block: the control of iteration k after the update (or candidate-graph
// step) launch of nblk blocks
__global__ __launch_bounds__(kBlock) void k_control(ControlArgs a)
{
    if (a.ctrl->done) return;
    control_body(a.n, a.k, a.ctrl, a.trace, a.nblk, a.slots, a.lists != 0, a.kinds, a.progress);
}

// batched: one block per instance, after k_update_batch
__global__ __launch_bounds__(kBlock) void k_control_batch(const UpdateArgs *args)
{
    const UpdateArgs &a = args[blockIdx.x];
    if (!a.ctrl || a.ctrl->done) return;
    control_body(a.g.n, a.ctrl->k_next, a.ctrl, a.trace, a.ctrl->nblocks, a.slots, false, nullptr, nullptr);
}

__global__ void k_ctrl_nblocks(Ctrl *ctrls, const int64_t *nb, int64_t ninst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ninst) ctrls[i].nblocks = nb[i];
}

__global__ void k_count_active(const Ctrl *ctrls, int64_t ninst, int32_t *out)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int c = 0;
    for (int64_t i = threadIdx.x; i < ninst; i += blockDim.x) c += ctrls[i].done ? 0 : 1;
    atomicAdd(&cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) out[0] = cnt;
}

// candidate graph: one fused pass per iteration over the CSR rows.  A wave
// owns 64 consecutive rows, whose entries are contiguous in the CSR.  It
// reads them in chunks of kGChunk entries, every lane loading entries
// lane, lane + 64, ... (coalesced column and cost loads, and all the
// neighbours' Lam and label gathers of the chunk in flight at once) into the
// wave's LDS; then each lane walks its own row's entries of the chunk there.
constexpr int kGChunk = 1024;

__global__ __launch_bounds__(kBlock) void k_graph_step(GraphStepArgs a)
{
    Ctrl *ctrl = a.ctrl;
    if (ctrl->done) return;
    constexpr int kPB = 16;
    constexpr int kQ = kGChunk / 64;
    __shared__ long long sz[kBlock / 64][kGChunk];
    __shared__ int32_t slab[kBlock / 64][kGChunk];
    __shared__ unsigned char srow[kBlock / 64][kGChunk];
    __shared__ long long rlam[kBlock / 64][64];
    __shared__ long long rbnd[kBlock / 64][64];
    __shared__ unsigned long long rneg[kBlock / 64][64];
    __shared__ unsigned int rcnt[kBlock / 64][64];   // (#neg << 16) + #zero of this chunk
    __shared__ unsigned int rbc[kBlock / 64][64];    // candidates of this chunk
    __shared__ unsigned short rbuf[kBlock / 64][64][kPB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t n = a.g.n;
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t w0 = (int64_t)blockIdx.x * kBlock + wave * 64;
    const bool copy_best = a.k > 0 && ctrl->best_k == a.k - 1;
    RowOut o;
    Top4 top;
    top.clear();
    int64_t cn = 0, cz = 0, rn = 0;
    // the row's loads at a clamped position (unconditional, issued together)
    const bool inb = p < n;
    const int64_t pc = inb ? p : 0;
    const RowIn ri = row_in(a.g, nullptr, a.lam_out, pc);
    const int64_t lamv = inb ? a.lam_in[pc] : 0;
    const int32_t rb0 = a.csr.rowptr[pc], re0 = a.csr.rowptr[pc + 1];
    const int32_t rb = inb ? rb0 : 0, re = inb ? re0 : 0;
    // The entries of the wave's 64 rows are contiguous: every lane takes
    // entries lane, lane + 64, ... of a chunk and computes their Z against
    // their rows; the counts take the entries with Z <= 0 in per-row LDS
    // counters, and an entry joins its row's short candidate buffer only if
    // its Z is at most the row's bound B = z4_{k-1}[3] - d_u + ms (the four
    // columns smallest at k-1 are all at most B at k, as in the complete
    // graph's list iterations; off on the run's first iteration, where
    // z4p and lam_out hold nothing of this run).  A row whose buffer
    // overflows in a chunk walks that chunk's run instead.
    const bool hz = a.z4p != nullptr && a.k > ctrl->k_first;
    const int64_t *zq = a.z4p ? a.z4p + 3 * n : a.lam_in;
    const int32_t *iq = a.z4p ? a.i4p + 3 * n : a.g.orig;
    const int32_t i43 = iq[pc];
    const int64_t z43 = zq[pc];
    rlam[wave][lane] = lamv;
    rbnd[wave][lane] = (inb && hz && i43 >= 0) ? z43 - (lamv - ri.lprev) + ctrl->ms_last : INT64_MAX;
    rneg[wave][lane] = 0;
    rcnt[wave][lane] = 0;
    rbc[wave][lane] = 0;
    if (w0 < n) {
        const int32_t e0 = a.csr.rowptr[w0], e1 = a.csr.rowptr[min(n, w0 + 64)];
        for (int32_t c0 = e0; c0 < e1; c0 += kGChunk) {
            const int32_t cnt = min(kGChunk, e1 - c0);
            wave_sync();   // the previous chunk's reads are done
            const int32_t lo = max(rb, c0), hi = min(re, c0 + cnt);
            for (int32_t e = lo; e < hi; ++e) srow[wave][e - c0] = (unsigned char)lane;
            // loads past the chunk's end read its last entry (not used): the
            // column and cost loads go out together, then all the gathers
            int32_t cu[kQ], cc[kQ], cb[kQ];
            int64_t cl[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int32_t i = c0 + min(q * 64 + lane, cnt - 1);
                cu[q] = a.csr.col[i];
                cc[q] = a.csr.cost[i];
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                cl[q] = a.lam_in[cu[q]];
                cb[q] = a.g.orig[cu[q]];
            }
            wave_sync();
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int i = q * 64 + lane;
                if (i < cnt) {
                    const int r = srow[wave][i] & 63;
                    const int64_t z = 2 * (int64_t)cc[q] - rlam[wave][r] - cl[q];   // eq. 9, doubled
                    sz[wave][i] = z;
                    slab[wave][i] = cb[q];
                    if (z <= 0) {
                        atomicAdd(&rcnt[wave][r], z < 0 ? 0x10000u : 1u);
                        if (z < 0) atomicAdd(&rneg[wave][r], (unsigned long long)z);
                    }
                    if (z <= rbnd[wave][r]) {
                        const unsigned t = atomicAdd(&rbc[wave][r], 1u);
                        if (t < (unsigned)kPB) rbuf[wave][r][t] = (unsigned short)i;
                    }
                }
            }
            wave_sync();
            const unsigned ccount = rcnt[wave][lane], m = rbc[wave][lane];
            cn += ccount >> 16;
            cz += ccount & 0xffffu;
            rn += (long long)rneg[wave][lane];
            rcnt[wave][lane] = 0;
            rneg[wave][lane] = 0;
            rbc[wave][lane] = 0;
            if (m > (unsigned)kPB) {
                for (int32_t e = lo; e < hi; ++e) top.insert(sz[wave][e - c0], slab[wave][e - c0]);
            } else {
                for (unsigned t = 0; t < m; ++t) {
                    const int i = rbuf[wave][lane][t];
                    top.insert(sz[wave][i], slab[wave][i]);
                }
            }
        }
    }
    if (inb)
        step_row(a.g, p, ri, top, cn, cz, rn, lamv, copy_best, a.lam_out, a.lam_best, a.z4, a.i4, nullptr,
                 a.neg, a.zero, a.step, nullptr, o, a.z4p, a.i4p);
    block_record(o, nullptr, blockIdx.x, a.slots, 0);
}

// ---------------------------------------------------------------------------
// candidate graph: k nearest neighbours and the CSR
// ---------------------------------------------------------------------------

// K smallest (D, label) per row over every column.  A workgroup owns one
// tile of 256 Morton-consecutive rows: it first scans its own tile, which
// gives every row a K-th smallest D to beat; tiles whose box lies farther
// from the rows' box than the largest such bound are skipped (tested in
// parallel and compacted), and each wave skips the 32-column sub-tiles
// beyond its own rows' bound.  The float distance test keeps every pair with
// D <= the current K-th smallest exactly (see thrf); insertion is exact in
// int64 with ties broken by label.
// With S > 1 column slices (blockIdx.y), every slice scans the block's own
// tile (so all take the same culling decisions) and every S-th of the
// surviving tiles; each writes its K smallest to pp / pd [slice][n][K]
// (positions, D; -1 none) for k_knn_merge.  With S == 1 the block writes
// nbr / nbr_d itself.
template <int K>
__global__ __launch_bounds__(kBlock) void k_knn(Geo g, const float4 *col, int32_t *nbr, int64_t *nbr_d, int64_t S,
                                                int32_t *pp, int64_t *pd)
{
    __shared__ float2 sc[kTile];
    __shared__ int32_t sl[kTile];
    __shared__ int32_t tlist[kBlock];
    __shared__ int32_t wcnt[kBlock / 64];
    __shared__ float redf[kBlock / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t n = g.n;
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int64_t own = blockIdx.x;
    const int64_t p = own * kTile + t;
    const bool valid = p < n;
    float xv = 0.0f, yv = 0.0f;
    int64_t bd[K];
    int32_t bl[K], bp[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { bd[j] = INT64_MAX; bl[j] = kNoIdx; bp[j] = -1; }
    if (valid) { const float4 cv = col[p]; xv = cv.x; yv = cv.y; }
    // float bound of the current K-th smallest D (exact integers below 2^42;
    // the widening covers the rounding of the float distance).  It starts
    // at the K-th smallest D among the positions within kSeedWin of p in
    // Morton order (those cross tile boundaries, so a row in a stray
    // fragment of its tile still gets a near bound); the list itself is
    // filled by the tile scans only.
    float thrf = INFINITY;
    if (valid) {
        int64_t wd[K];
#pragma unroll
        for (int j = 0; j < K; ++j) wd[j] = INT64_MAX;
        const int64_t lo = p - kSeedWin < 0 ? 0 : p - kSeedWin;
        const int64_t hi = p + kSeedWin >= n ? n - 1 : p + kSeedWin;
        for (int64_t u = lo; u <= hi; ++u) {
            if (u == p) continue;
            const float4 cu = col[u];
            const int32_t ix = (int32_t)(xv - cu.x), iy = (int32_t)(yv - cu.y);
            int64_t d = (int64_t)ix * ix + (int64_t)iy * iy;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                if (d < wd[j]) { const int64_t td = wd[j]; wd[j] = d; d = td; }
            }
        }
        if (wd[K - 1] != INT64_MAX) thrf = (float)wd[K - 1] * (1.0f + 0x1p-20f) + 1.0f;
    }

    // all columns [tile, tile + ntile) of the LDS tile against this row
    auto scan = [&](int64_t tile, int j0, int j1) {
        for (int j = j0; j < j1; ++j) {
            const float2 cu = sc[j];
            const float ddx = xv - cu.x, ddy = yv - cu.y;
            if (!(fmaf(ddx, ddx, ddy * ddy) <= thrf)) continue;
            const int64_t u = tile + j;
            if (u == p || u >= n) continue;
            const int32_t ix = (int32_t)ddx, iy = (int32_t)ddy;
            const int64_t D = (int64_t)ix * ix + (int64_t)iy * iy;
            const int32_t lu = sl[j];
            if (!(D < bd[K - 1] || (D == bd[K - 1] && lu < bl[K - 1]))) continue;
            bd[K - 1] = D; bl[K - 1] = lu; bp[K - 1] = (int32_t)u;
#pragma unroll
            for (int q = K - 1; q > 0; --q) {
                if (bd[q] < bd[q - 1] || (bd[q] == bd[q - 1] && bl[q] < bl[q - 1])) {
                    const int64_t td = bd[q]; bd[q] = bd[q - 1]; bd[q - 1] = td;
                    const int32_t tl = bl[q]; bl[q] = bl[q - 1]; bl[q - 1] = tl;
                    const int32_t tp = bp[q]; bp[q] = bp[q - 1]; bp[q - 1] = tp;
                }
            }
            if (bp[K - 1] >= 0) thrf = fminf(thrf, (float)bd[K - 1] * (1.0f + 0x1p-20f) + 1.0f);
        }
    };
    auto load = [&](int64_t tile) {
        __syncthreads();
        const int64_t cc = tile + t;
        if (cc < n) { const float4 c4 = col[cc]; sc[t] = make_float2(c4.x, c4.y); sl[t] = g.orig[cc]; }
        else { sc[t] = make_float2(INFINITY, INFINITY); sl[t] = kNoIdx; }
        __syncthreads();
    };

    // 1. the block's own tile (its rows' spatial neighbourhood in Morton
    //    order) gives every row a first K-th distance
    load(own * kTile);
    scan(own * kTile, 0, (int)min((int64_t)kTile, n - own * kTile));

    // 2. bounds of the block and of each wave: the largest K-th distance of
    //    their rows (a squared radius), and their boxes
    const float thr_w = wave_max(valid ? thrf : -INFINITY);
    const float thr_b = block_reduce<float, true>(valid ? thrf : -INFINITY, redf);
    const float4 rbox = g.box[own * kBoxStride];
    float4 wbox = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
    for (int s = wave * (64 / kSubCols); s < (wave + 1) * (64 / kSubCols); ++s) {
        const float4 sb = g.box[own * kBoxStride + 1 + s];
        wbox.x = fminf(wbox.x, sb.x); wbox.y = fmaxf(wbox.y, sb.y);
        wbox.z = fminf(wbox.z, sb.z); wbox.w = fmaxf(wbox.w, sb.w);
    }
    // squared distance between boxes (exact integer corners) against a
    // squared radius, with a relative margin for the float rounding
    auto near_box = [](float4 b, float4 r, float thr2) {
        const float dx = fmaxf(0.0f, fmaxf(b.x - r.y, r.x - b.y));
        const float dy = fmaxf(0.0f, fmaxf(b.z - r.w, r.z - b.w));
        return fmaf(dx, dx, dy * dy) <= thr2 * (1.0f + 0x1p-16f);
    };

    // 3. the other tiles: tested in parallel against the block, compacted
    //    in order (this slice takes every S-th); each wave then tests the
    //    sub-tiles against its own rows
    const int64_t slc = blockIdx.y;
    int64_t seen = 0;   // surviving tiles before this chunk of tests
    for (int64_t base = 0; base < ntiles; base += kBlock) {
        const int64_t ti = base + t;
        const bool ok = ti < ntiles && ti != own && near_box(g.box[ti * kBoxStride], rbox, thr_b);
        const unsigned long long mk = __ballot(ok);
        __syncthreads();
        if (lane == 0) wcnt[wave] = __popcll(mk);
        __syncthreads();
        int off = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            off += (w < wave) ? wcnt[w] : 0;
            total += wcnt[w];
        }
        if (ok) tlist[off + __popcll(mk & ((1ULL << lane) - 1ULL))] = (int32_t)ti;
        __syncthreads();
        for (int j = 0; j < total; ++j) {
            if ((seen + j) % S != slc) continue;
            const int64_t tj = tlist[j];
            load(tj * kTile);
            const int ntile = (int)min((int64_t)kTile, n - tj * kTile);
            const bool sp = lane < kSubs && lane * kSubCols < ntile &&
                            near_box(g.box[tj * kBoxStride + 1 + lane], wbox, thr_w);
            unsigned long long sm = __ballot(sp);
            while (sm) {
                const int sb = __ffsll((long long)sm) - 1;
                sm &= sm - 1;
                scan(tj * kTile, sb * kSubCols, min(sb * kSubCols + kSubCols, ntile));
            }
        }
        seen += total;
    }
    if (valid) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (S > 1) {
                pp[(slc * n + p) * K + j] = bp[j];
                pd[(slc * n + p) * K + j] = bd[j];
            } else {
                nbr[p * K + j] = bp[j];
                if (nbr_d) nbr_d[p * K + j] = bd[j];
            }
        }
    }
}

// The K smallest (D, label) of a row over the slices' lists of k_knn; the
// own tile's columns are in every slice's list and are taken once.
template <int K>
__global__ __launch_bounds__(kBlock) void k_knn_merge(Geo g, int64_t S, const int32_t *pp, const int64_t *pd,
                                                      int32_t *nbr, int64_t *nbr_d)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t n = g.n;
    if (p >= n) return;
    int64_t bd[K];
    int32_t bl[K], bp[K];
#pragma unroll
    for (int j = 0; j < K; ++j) { bd[j] = INT64_MAX; bl[j] = kNoIdx; bp[j] = -1; }
    for (int64_t s = 0; s < S; ++s) {
        for (int j = 0; j < K; ++j) {
            const int32_t u = pp[(s * n + p) * K + j];
            if (u < 0) continue;
            bool dup = false;
#pragma unroll
            for (int q = 0; q < K; ++q) dup = dup || bp[q] == u;
            if (dup) continue;
            const int64_t D = pd[(s * n + p) * K + j];
            const int32_t lu = g.orig[u];
            if (!(D < bd[K - 1] || (D == bd[K - 1] && lu < bl[K - 1]))) continue;
            bd[K - 1] = D; bl[K - 1] = lu; bp[K - 1] = u;
#pragma unroll
            for (int q = K - 1; q > 0; --q) {
                if (bd[q] < bd[q - 1] || (bd[q] == bd[q - 1] && bl[q] < bl[q - 1])) {
                    const int64_t td = bd[q]; bd[q] = bd[q - 1]; bd[q - 1] = td;
                    const int32_t tl = bl[q]; bl[q] = bl[q - 1]; bl[q - 1] = tl;
                    const int32_t tp = bp[q]; bp[q] = bp[q - 1]; bp[q - 1] = tp;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        nbr[p * K + j] = bp[j];
        if (nbr_d) nbr_d[p * K + j] = bd[j];
    }
}

// undirected edge {p, q} -> (min << bb) | max, bb bits per end (ends below
// 2^bb, and min < max, so no key has all 2 bb bits set like the filler)
__global__ __launch_bounds__(kBlock) void k_pair_keys(const int32_t *nbr, int64_t nk, int K, int bb, uint64_t *keys)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nk) return;
    const int32_t qq = nbr[i];
    if (qq < 0) { keys[i] = ~0ULL; return; }   // unfilled slot: sorts last, never used
    const uint64_t p = (uint64_t)(i / K), q = (uint64_t)qq;
    keys[i] = p < q ? (p << bb) | q : (q << bb) | p;
}

// counts distinct undirected edges per endpoint (keys sorted)
__global__ __launch_bounds__(kBlock) void k_edge_count(const uint64_t *keys, int64_t nk, int bb, int32_t *deg)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nk || keys[i] == ~0ULL || (i > 0 && keys[i] == keys[i - 1])) return;
    atomicAdd(&deg[keys[i] >> bb], 1);
    atomicAdd(&deg[keys[i] & ((1ULL << bb) - 1)], 1);
}

__global__ __launch_bounds__(kBlock) void k_edge_fill(const uint64_t *keys, int64_t nk, int bb, const int32_t *rowptr,
                                                      int32_t *cursor, int32_t *col)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nk || keys[i] == ~0ULL || (i > 0 && keys[i] == keys[i - 1])) return;
    const int32_t a = (int32_t)(keys[i] >> bb), b = (int32_t)(keys[i] & ((1ULL << bb) - 1));
    col[rowptr[a] + atomicAdd(&cursor[a], 1)] = b;
    col[rowptr[b] + atomicAdd(&cursor[b], 1)] = a;
}

// sorts each row's columns (insertion sort: rows are short) and fills the
// exact costs
__global__ __launch_bounds__(kBlock) void k_row_finish(const int32_t *xy, const int32_t *orig, int64_t n,
                                                       const int32_t *rowptr, int32_t *col, int32_t *cost)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int32_t e0 = rowptr[p], e1 = rowptr[p + 1];
    for (int32_t e = e0 + 1; e < e1; ++e) {
        const int32_t x = col[e];
        int32_t f = e - 1;
        while (f >= e0 && col[f] > x) { col[f + 1] = col[f]; --f; }
        col[f + 1] = x;
    }
    const int64_t v = orig[p];
    for (int32_t e = e0; e < e1; ++e) {
        const int64_t u = orig[col[e]];
        const int64_t dx = (int64_t)xy[2 * v] - xy[2 * u], dy = (int64_t)xy[2 * v + 1] - xy[2 * u + 1];
        cost[e] = (int32_t)nint_sqrt(dx * dx + dy * dy);
    }
}

// sum over CSR entries of min(0, Z)
__global__ __launch_bounds__(kBlock) void k_graph_dual(Geo g, Csr csr, const int64_t *lam, unsigned long long *acc)
{
    __shared__ unsigned long long red[kBlock / 64];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t s = 0;
    if (p < g.n) {
        const int64_t lv = lam[p];
        for (int32_t e = csr.rowptr[p]; e < csr.rowptr[p + 1]; ++e) {
            const int64_t z = 2 * (int64_t)csr.cost[e] - lv - lam[csr.col[e]];
            if (z < 0) s += z;
        }
    }
    const unsigned long long tot = block_reduce<unsigned long long, false>((unsigned long long)s, red);
    if (threadIdx.x == 0 && tot) atomicAdd(&acc[0], tot);
}

__global__ __launch_bounds__(kBlock) void k_graph_collect(Geo g, Csr csr, const int64_t *lam, int64_t slack,
                                                          unsigned long long *count, int2 *out, int64_t cap)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = p < g.n;
    int64_t lv = 0, th = -1;
    int32_t e0 = 0, e1 = 0;
    if (valid) {
        lv = lam[p];
        e0 = csr.rowptr[p];
        e1 = csr.rowptr[p + 1];
        if (slack >= 0) {
            int64_t b[kTop] = {INT64_MAX, INT64_MAX, INT64_MAX, INT64_MAX};
            for (int32_t e = e0; e < e1; ++e) {
                int64_t z = 2 * (int64_t)csr.cost[e] - lv - lam[csr.col[e]];
#pragma unroll
                for (int j = 0; j < kTop; ++j) if (z < b[j]) { const int64_t tt = b[j]; b[j] = z; z = tt; }
            }
            th = b[3] == INT64_MAX ? INT64_MAX / 4 : (b[3] > 0 ? b[3] : 0) + slack;
        }
    }
    // the row's pairs counted, then written behind one atomic per wave
    int cnt = 0;
    for (int32_t e = e0; e < e1; ++e)
        if (2 * (int64_t)csr.cost[e] - lv - lam[csr.col[e]] <= th) ++cnt;
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    const int total = __shfl(incl, 63, 64);
    unsigned long long base = 0;
    if (lane == 0 && total > 0) base = atomicAdd(count, (unsigned long long)total);
    base = __shfl(base, 0, 64) + (unsigned long long)(incl - cnt);
    const int32_t pp = (int32_t)p;
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t u = csr.col[e];
        if (2 * (int64_t)csr.cost[e] - lv - lam[u] > th) continue;
        if ((int64_t)base < cap) out[base] = make_int2(min(pp, u), max(pp, u));
        ++base;
    }
}

__global__ __launch_bounds__(kBlock) void k_graph_membership(Geo g, Csr csr, int64_t m, const int32_t *eu,
                                                             const int32_t *ev, unsigned long long *acc)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    const int64_t u = eu[e], v = ev[e];
    if (u < 0 || v < 0 || u >= g.n || v >= g.n) return;   // counted by the edge check
    const int32_t pu = g.pos[u], pv = g.pos[v];
    int32_t lo = csr.rowptr[pu], hi = csr.rowptr[pu + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (csr.col[mid] < pv) lo = mid + 1; else hi = mid;
    }
    if (lo >= csr.rowptr[pu + 1] || csr.col[lo] != pv) atomicAdd(&acc[2], 1ULL);
}

// Pair (a, b) -> key (a << bb) | b, with bb bits per end (every end is
// below 2^bb): the sort then runs over 2 bb bits only.
__global__ __launch_bounds__(kBlock) void k_pair_to_key(const int2 *pairs, int64_t count, int bb, uint64_t *keys)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) keys[i] = ((uint64_t)(uint32_t)pairs[i].x << bb) | (uint64_t)(uint32_t)pairs[i].y;
}

// the distinct compact keys (i < *count) back to (a << 32) | b, in place
__global__ __launch_bounds__(kBlock) void k_key_widen(uint64_t *keys, const int64_t *count, int64_t cap, int bb)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= cap || i >= *count) return;
    const uint64_t k = keys[i];
    keys[i] = ((k >> bb) << 32) | (k & ((1ULL << bb) - 1));
}

// bytes [0, n16 * 16) as 16-byte words, then the tail byte by byte (both
// pointers 16-byte aligned); the destination may be mapped host memory
__global__ __launch_bounds__(kBlock) void k_copy_bytes(const uint8_t *src, uint8_t *dst, int64_t bytes)
{
    const int64_t n16 = bytes / 16;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
    uint4 *d4 = reinterpret_cast<uint4 *>(dst);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride) d4[i] = s4[i];
    if (blockIdx.x == 0 && threadIdx.x < bytes - 16 * n16) dst[16 * n16 + threadIdx.x] = src[16 * n16 + threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *p, int64_t count, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < count) p[i] = v;
}

__device__ __forceinline__ int64_t floor_half_d(int64_t x) { return x >= 0 ? x / 2 : -((-x + 1) / 2); }

// Per distinct pair key i (a << 32 | b, count on the device): the exact
// cost, and with lam the bits "arc a'->b'' (bit 0) / b'->a'' (bit 1) has
// negative reduced cost c - alpha_tail - beta_head" for alpha = floor(Lam/2),
// beta = Lam - alpha.
__global__ __launch_bounds__(kBlock) void k_key_info(const uint64_t *keys, const int64_t *count, int64_t cap,
                                                     const int32_t *xy, const int64_t *lam, int32_t *cost,
                                                     uint8_t *neg)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= cap || i >= *count) return;
    const int64_t a = (int64_t)(keys[i] >> 32), b = (int64_t)(keys[i] & 0xffffffffULL);
    const int64_t dx = (int64_t)xy[2 * a] - xy[2 * b], dy = (int64_t)xy[2 * a + 1] - xy[2 * b + 1];
    const int64_t c = nint_sqrt(dx * dx + dy * dy);
    cost[i] = (int32_t)c;
    if (lam) {
        const int64_t aa = floor_half_d(lam[a]), ab = floor_half_d(lam[b]);
        const int64_t ba = lam[a] - aa, bb = lam[b] - ab;
        neg[i] = (uint8_t)((c - aa - bb < 0 ? 1 : 0) | (c - ab - ba < 0 ? 2 : 0));
    }
}

// free slots after every node's incidence list (new pairs of pricing rounds
// are placed there without a rebuild)
constexpr int kIncSpare = 2;

// The finish's incidence lists by counting: each distinct pair i < *count
// adds one to both ends' counts (deg[v + 1]) ...
__global__ __launch_bounds__(kBlock) void k_inc_count(const uint64_t *keys, const int64_t *count, int64_t cap,
                                                      int32_t *deg)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= cap || i >= *count) return;
    const uint64_t k = keys[i];
    atomicAdd(&deg[(k >> 32) + 1], 1);
    atomicAdd(&deg[(k & 0xffffffffULL) + 1], 1);
}

// ... is placed at the next free slot of both ends' lists (in arrival
// order) ...
__global__ __launch_bounds__(kBlock) void k_inc_place(const uint64_t *keys, const int64_t *count, int64_t cap,
                                                      const int32_t *start, int32_t *cursor, int32_t *inc)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= cap || i >= *count) return;
    const uint64_t k = keys[i];
    const int64_t a = (int64_t)(k >> 32), b = (int64_t)(k & 0xffffffffULL);
    inc[start[a] + atomicAdd(&cursor[a], 1)] = (int32_t)i;
    inc[start[b] + atomicAdd(&cursor[b], 1)] = (int32_t)i;
}

// ... and every node's list is put in increasing edge order (insertion sort:
// lists are short).
__global__ __launch_bounds__(kBlock) void k_inc_order(const int32_t *start, const int32_t *len, int64_t n, int32_t *inc)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    const int32_t s0 = start[v], s1 = s0 + len[v];
    for (int32_t e = s0 + 1; e < s1; ++e) {
        const int32_t x = inc[e];
        int32_t f = e - 1;
        while (f >= s0 && inc[f] > x) { inc[f + 1] = inc[f]; --f; }
        inc[f + 1] = x;
    }
}

__global__ __launch_bounds__(kBlock) void k_label_degrees(Geo g, Csr csr, int32_t *deg)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= g.n) return;
    const int32_t p = g.pos[v];
    deg[v] = csr.rowptr[p + 1] - csr.rowptr[p];
}

__global__ __launch_bounds__(kBlock) void k_label_rows(Geo g, Csr csr, const int32_t *rowptr_l, int32_t *col_l)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= g.n) return;
    const int32_t p = g.pos[v];
    const int32_t o = rowptr_l[v];
    const int32_t e0 = csr.rowptr[p], e1 = csr.rowptr[p + 1];
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t x = g.orig[csr.col[e]];
        int32_t f = o + (e - e0) - 1;
        while (f >= o && col_l[f] > x) { col_l[f + 1] = col_l[f]; --f; }
        col_l[f + 1] = x;
    }
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------

__global__ void k_minmax_init(int32_t *out4)
{
    if (threadIdx.x == 0) { out4[0] = INT_MAX; out4[1] = INT_MIN; out4[2] = INT_MAX; out4[3] = INT_MIN; }
}

__global__ __launch_bounds__(kBlock) void k_minmax(const int32_t *xy, int64_t n, int32_t *out4)
{
    int32_t mnx = INT_MAX, mxx = INT_MIN, mny = INT_MAX, mxy = INT_MIN;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int32_t x = xy[2 * i], y = xy[2 * i + 1];
        mnx = min(mnx, x); mxx = max(mxx, x); mny = min(mny, y); mxy = max(mxy, y);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mnx = min(mnx, __shfl_xor(mnx, o, 64)); mxx = max(mxx, __shfl_xor(mxx, o, 64));
        mny = min(mny, __shfl_xor(mny, o, 64)); mxy = max(mxy, __shfl_xor(mxy, o, 64));
    }
    // one set of four atomics per block (atomics on one cache line serialise)
    __shared__ int32_t red[kBlock / 64][4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = mnx; red[w][1] = mxx; red[w][2] = mny; red[w][3] = mxy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kBlock / 64; ++q) {
            mnx = min(mnx, red[q][0]); mxx = max(mxx, red[q][1]);
            mny = min(mny, red[q][2]); mxy = max(mxy, red[q][3]);
        }
        atomicMin(&out4[0], mnx); atomicMax(&out4[1], mxx);
        atomicMin(&out4[2], mny); atomicMax(&out4[3], mxy);
    }
}

// spread the low 16 bits of x to the even bit positions
__device__ __forceinline__ uint32_t spread16(uint32_t x)
{
    x &= 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// Morton key of the top 16 bits of each (span < 2^20) coordinate offset
__global__ __launch_bounds__(kBlock) void k_morton(const int32_t *xy, int64_t n, int32_t minx, int32_t miny,
                                                   uint32_t *keys, int32_t *ids)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t x = (uint32_t)(xy[2 * i] - minx) >> 4, y = (uint32_t)(xy[2 * i + 1] - miny) >> 4;
    keys[i] = spread16(x) | (spread16(y) << 1);
    ids[i] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_inverse(const int32_t *orig, int64_t n, int32_t *pos)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < n) pos[orig[p]] = (int32_t)p;
}

// centred float coordinates in sorted order; one block is one tile
__global__ __launch_bounds__(kBlock) void k_prep(const int32_t *xy, const int32_t *orig, int64_t n, int32_t cx,
                                                 int32_t cy, float4 *col, float4 *box, unsigned int *xy2max_bits)
{
    __shared__ float redf[kBlock / 64];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    float r2 = 0.0f, x = 0.0f, y = 0.0f;
    const bool ok = p < n;
    if (ok) {
        const int64_t v = orig[p];
        x = (float)(xy[2 * v] - cx);
        y = (float)(xy[2 * v + 1] - cy);
        col[p] = make_float4(x, y, 0.0f, x * x + y * y);
        // round the bound up by a relative 2^-22 so it is >= the exact value
        r2 = xy2_bound(x, y);
    }
    // sub-tile boxes (an empty sub-tile gets an empty box: min +inf, max -inf)
    const float smnx = -sub_max(ok ? -x : -INFINITY), smxx = sub_max(ok ? x : -INFINITY);
    const float smny = -sub_max(ok ? -y : -INFINITY), smxy = sub_max(ok ? y : -INFINITY);
    if ((threadIdx.x & (kSubCols - 1)) == 0)
        box[blockIdx.x * kBoxStride + 1 + threadIdx.x / kSubCols] = make_float4(smnx, smxx, smny, smxy);
    const float mnx = -block_reduce<float, true>(ok ? -x : -INFINITY, redf);
    const float mxx = block_reduce<float, true>(ok ? x : -INFINITY, redf);
    const float mny = -block_reduce<float, true>(ok ? -y : -INFINITY, redf);
    const float mxy = block_reduce<float, true>(ok ? y : -INFINITY, redf);
    r2 = block_reduce<float, true>(r2, redf);
    if (threadIdx.x == 0) {
        box[blockIdx.x * kBoxStride] = make_float4(mnx, mxx, mny, mxy);
        atomicMax(xy2max_bits, __float_as_uint(r2));
    }
}

__global__ __launch_bounds__(kBlock) void k_set_lam(const int64_t *lam_label, const int32_t *orig, int64_t n,
                                                    int64_t *lam_sorted, float4 *col, float *tile_hmax, Ctrl *ctrl)
{
    __shared__ float redf[kBlock / 64];
    __shared__ unsigned long long redu[kBlock / 64];
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long ab = 0;
    float h = -INFINITY;
    if (p < n) {
        const int64_t l = orig ? lam_label[orig[p]] : lam_label[p];
        lam_sorted[p] = l;
        const float4 cv = col_record(col[p].x, col[p].y, l);
        h = cv.z;
        col[p] = cv;
        ab = (unsigned long long)(l < 0 ? -l : l);
    }
    const float hs = sub_max(h);
    if ((threadIdx.x & (kSubCols - 1)) == 0) tile_hmax[blockIdx.x * kBoxStride + 1 + threadIdx.x / kSubCols] = hs;
    h = block_reduce<float, true>(h, redf);
    ab = block_reduce<unsigned long long, true>(ab, redu);
    if (threadIdx.x == 0) {
        tile_hmax[blockIdx.x * kBoxStride] = h;
        atomicMax((unsigned long long *)&ctrl->maxabs_lam, ab);
    }
}

__global__ __launch_bounds__(kBlock) void k_unpermute(const int64_t *lam_sorted, const int32_t *orig, int64_t n,
                                                      int64_t *lam_label)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < n) lam_label[orig[p]] = lam_sorted[p];
}

// coordinates in Morton order
__global__ __launch_bounds__(kBlock) void k_gather_xy(const int32_t *xy, const int32_t *orig, int64_t n,
                                                      int32_t *xy_pos)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < n) {
        const int64_t l = orig[p];
        xy_pos[2 * p] = xy[2 * l];
        xy_pos[2 * p + 1] = xy[2 * l + 1];
    }
}

// edges given by positions -> labels, lo < hi, in place
__global__ __launch_bounds__(kBlock) void k_edges_to_labels(const int32_t *orig, int64_t m, int32_t *eu, int32_t *ev)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < m) {
        const int32_t a = orig[eu[e]], b = orig[ev[e]];
        eu[e] = min(a, b);
        ev[e] = max(a, b);
    }
}

// the first thresholds' seeds from a previous run's four smallest per node
// (labels, by label) as positions
__global__ __launch_bounds__(kBlock) void k_seed_from_top(const int32_t *i4, const int32_t *orig, const int32_t *pos,
                                                          int64_t n, int32_t *seed)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int64_t v = orig[p];
#pragma unroll
    for (int j = 0; j < kTop; ++j) {
        const int32_t u = i4[kTop * v + j];
        seed[j * n + p] = (u >= 0 && u < n) ? pos[u] : -1;
    }
}

// The first scan's threshold seeds: the four nearest (by exact D, then
// position) among the positions within kSeedWin of p in the sorted order
// (Morton order keeps most nearest neighbours close); any four columns
// bound the 4th smallest Z, close ones tightly.
__global__ __launch_bounds__(kBlock) void k_seed_neighbours(int64_t n, const float4 *col, int32_t *seed)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    if (n < 5) {
        for (int j = 0; j < kTop; ++j) seed[j * n + p] = -1;
        return;
    }
    const float4 cv = col[p];
    int64_t bd[kTop];
    int32_t bq[kTop];
#pragma unroll
    for (int j = 0; j < kTop; ++j) { bd[j] = INT64_MAX; bq[j] = -1; }
    const int64_t lo = p - kSeedWin < 0 ? 0 : p - kSeedWin;
    const int64_t hi = p + kSeedWin >= n ? n - 1 : p + kSeedWin;
    for (int64_t q = lo; q <= hi; ++q) {
        if (q == p) continue;
        const float4 cu = col[q];
        const int32_t dx = (int32_t)(cv.x - cu.x), dy = (int32_t)(cv.y - cu.y);
        int64_t d = (int64_t)dx * dx + (int64_t)dy * dy;
        int32_t qq = (int32_t)q;
        if (d >= bd[kTop - 1]) continue;
#pragma unroll
        for (int j = 0; j < kTop; ++j) {
            if (d < bd[j]) {
                const int64_t td = bd[j]; bd[j] = d; d = td;
                const int32_t tq = bq[j]; bq[j] = qq; qq = tq;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kTop; ++j) seed[j * n + p] = bq[j];
}

__global__ void k_ctrl_init(Ctrl *ctrl, int64_t max_iters, int64_t trace_cap, int64_t handoff_div, CtrlStart cs)
{
    if (threadIdx.x != 0) return;
    Ctrl c;
    unsigned char *p = (unsigned char *)&c;
    for (size_t i = 0; i < sizeof(Ctrl); ++i) p[i] = 0;
    c.best_k = -1;
    c.best_dual2 = LLONG_MIN;
    c.kstar = -1;
    c.k_last = -1;
    c.max_iters = max_iters;
    c.trace_cap = trace_cap;
    c.handoff_div = handoff_div;
    c.k_first = cs.k0;
    c.k_next = cs.k0;
    c.hvalid = cs.hvalid;
    c.h1 = cs.h1;
    c.h2 = cs.h2;
    *ctrl = c;
}

// ---------------------------------------------------------------------------
// trivial x (eq. 7) and compaction
// ---------------------------------------------------------------------------

// slot (v, j): edge {v, u} of v's j-th smallest entry when Z <= 0 and v < u
// (each such edge is in the top-4 of both endpoints once every trivial
// degree is 2, so the lower endpoint emits it exactly once)
__global__ __launch_bounds__(kBlock) void k_extract_trivial(const int64_t *z4, const int32_t *i4, int64_t n,
                                                            int32_t *su, int32_t *sv, uint8_t *sx)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= kTop * n) return;
    const int64_t v = s / kTop;
    const int64_t z = z4[s];
    const int32_t u = i4[s];
    if (u > v && u < n && z <= 0) { su[s] = (int32_t)v; sv[s] = u; sx[s] = z < 0 ? 2 : 1; }
    else { su[s] = -1; sv[s] = -1; sx[s] = 0; }
}

__device__ __forceinline__ int block_excl_scan(int flag, int *wbuf, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long bal = __ballot(flag);
    const int below = __popcll(bal & ((1ULL << lane) - 1ULL));
    if (lane == 0) wbuf[w] = __popcll(bal);
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < kBlock / 64; ++i) { if (i < w) off += wbuf[i]; tot += wbuf[i]; }
    *total = tot;
    return off + below;
}

__global__ __launch_bounds__(kBlock) void k_compact_count(const int32_t *su, int64_t ns, int32_t *bcount)
{
    __shared__ int wbuf[kBlock / 64];
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int flag = (s < ns && su[s] >= 0) ? 1 : 0;
    int tot;
    block_excl_scan(flag, wbuf, &tot);
    if (threadIdx.x == 0) bcount[blockIdx.x] = tot;
}

// exclusive scan of nb block counts in one block; total to *count
__global__ __launch_bounds__(1024) void k_compact_scan(int32_t *bcount, int64_t nb, int64_t *count)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = t * per, b1 = min(nb, b0 + per);
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += bcount[b];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int i = 0; i < 1024; ++i) { const int64_t x = part[i]; part[i] = acc; acc += x; }
        *count = acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t b = b0; b < b1; ++b) { const int32_t x = bcount[b]; bcount[b] = (int32_t)acc; acc += x; }
}

__global__ __launch_bounds__(kBlock) void k_compact_scatter(const int32_t *su, const int32_t *sv, const uint8_t *sx,
                                                            int64_t ns, const int32_t *boff, int32_t *eu,
                                                            int32_t *ev, uint8_t *ex)
{
    __shared__ int wbuf[kBlock / 64];
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int flag = (s < ns && su[s] >= 0) ? 1 : 0;
    int tot;
    const int pos = block_excl_scan(flag, wbuf, &tot);
    if (flag) {
        const int64_t o = (int64_t)boff[blockIdx.x] + pos;
        eu[o] = su[s]; ev[o] = sv[s]; ex[o] = sx[s];
    }
}

// ---------------------------------------------------------------------------
// certificate: primal side
// ---------------------------------------------------------------------------

// acc: [0] sum min(0,Z) ordered, [1] primal2, [2] #violations, [3] sum Lam
__global__ __launch_bounds__(kBlock) void k_cert_edges(const int32_t *xy, int64_t n, int64_t m, const int32_t *eu,
                                                       const int32_t *ev, const uint8_t *ex2, int32_t *deg,
                                                       int32_t *cnt, int32_t *nb, unsigned long long *acc)
{
    __shared__ unsigned long long red[kBlock / 64];
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long cost2 = 0, viol = 0;
    if (e < m) {
        const int64_t u = eu[e], v = ev[e];
        const int x2 = ex2[e];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v || (x2 != 1 && x2 != 2)) {
            viol = 1;
        } else {
            const int64_t dx = (int64_t)xy[2 * u] - xy[2 * v];
            const int64_t dy = (int64_t)xy[2 * u + 1] - xy[2 * v + 1];
            cost2 = (unsigned long long)(nint_sqrt(dx * dx + dy * dy) * x2);
            atomicAdd(&deg[u], x2);
            atomicAdd(&deg[v], x2);
            const int su = atomicAdd(&cnt[u], 1);
            if (su < kCertNb) nb[kCertNb * u + su] = (int32_t)v;
            const int sv = atomicAdd(&cnt[v], 1);
            if (sv < kCertNb) nb[kCertNb * v + sv] = (int32_t)u;
        }
    }
    // one atomic per block for the cost (atomics on one address serialise)
    cost2 = block_reduce<unsigned long long, false>(cost2, red);
    viol = block_reduce<unsigned long long, false>(viol, red);
    if (threadIdx.x == 0) {
        if (cost2) atomicAdd(&acc[1], cost2);
        if (viol) atomicAdd(&acc[2], viol);
    }
}

// b (by label) or null: every doubled degree must be 2 b_v (4 for F2M);
// acc[3] += sum_v b_v Lam_v
__global__ __launch_bounds__(kBlock) void k_cert_nodes(const int64_t *lam, int64_t n, const int32_t *deg,
                                                       const int32_t *cnt, const int32_t *nb,
                                                       unsigned long long *acc, const int8_t *b)
{
    __shared__ unsigned long long red[kBlock / 64];
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long bad = 0, sl = 0;
    if (v < n) {
        const int bv = b ? (int)b[v] : 2;
        sl = (unsigned long long)(bv * lam[v]);
        const int c = cnt[v];
        if (deg[v] != 2 * bv || c > kCertNb) bad = 1;
        else {
            for (int i = 0; i < c; ++i)
                for (int j = i + 1; j < c; ++j)
                    if (nb[kCertNb * v + i] == nb[kCertNb * v + j]) bad = 1;
        }
    }
    bad = block_reduce<unsigned long long, false>(bad, red);
    sl = block_reduce<unsigned long long, false>(sl, red);
    if (threadIdx.x == 0) {
        if (bad) atomicAdd(&acc[2], bad);
        atomicAdd(&acc[3], sl);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_minmax(const int32_t *xy, int64_t n, int32_t *out4, hipStream_t st)
{
    hipLaunchKernelGGL(k_minmax_init, dim3(1), dim3(64), 0, st, out4);
    // a few blocks that loop: few atomics, and the pass is bandwidth-trivial
    unsigned nb = blocks_for(n, kBlock * 8);
    if (nb > 256) nb = 256;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_minmax, dim3(nb), dim3(kBlock), 0, st, xy, n, out4);
    return hipGetLastError();
}

size_t sort_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                             (const int32_t *)nullptr, (int32_t *)nullptr, (int)n, 0, 32);
    return bytes;
}

hipError_t launch_sort(const int32_t *xy, int64_t n, int32_t minx, int32_t miny, uint32_t *keys, uint32_t *keys_alt,
                       int32_t *ids, int32_t *orig, int32_t *pos, void *temp, size_t temp_bytes, hipStream_t st)
{
    hipLaunchKernelGGL(k_morton, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, xy, n, minx, miny, keys, ids);
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_alt, ids, orig, (int)n, 0, 32, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_inverse, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, orig, n, pos);
    return hipGetLastError();
}

hipError_t launch_prep(const int32_t *xy, const int32_t *orig, int64_t n, int32_t cx, int32_t cy, float4 *col,
                       float4 *box, float *xy2max_dev, hipStream_t st)
{
    hipError_t e = hipMemsetAsync(xy2max_dev, 0, sizeof(float), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prep, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, xy, orig, n, cx, cy, col, box,
                       (unsigned int *)xy2max_dev);
    return hipGetLastError();
}

hipError_t launch_set_lam(const int64_t *lam_label, const int32_t *orig, int64_t n, int64_t *lam_sorted, float4 *col,
                          float *tile_hmax, Ctrl *ctrl, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_lam, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, lam_label, orig, n, lam_sorted,
                       col, tile_hmax, ctrl);
    return hipGetLastError();
}

hipError_t launch_unpermute(const int64_t *lam_sorted, const int32_t *orig, int64_t n, int64_t *lam_label,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_unpermute, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, lam_sorted, orig, n, lam_label);
    return hipGetLastError();
}

hipError_t launch_copy_bytes(const void *src, void *dst, int64_t bytes, hipStream_t st)
{
    if (bytes <= 0) return hipSuccess;
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0) return hipErrorInvalidValue;
    const int64_t n16 = bytes / 16;
    const int64_t want = (n16 + kBlock - 1) / kBlock;
    const unsigned blocks = (unsigned)(want < 1 ? 1 : (want > 1024 ? 1024 : want));
    hipLaunchKernelGGL(k_copy_bytes, dim3(blocks), dim3(kBlock), 0, st, static_cast<const uint8_t *>(src),
                       static_cast<uint8_t *>(dst), bytes);
    return hipGetLastError();
}

hipError_t launch_gather_xy(const int32_t *xy, const int32_t *orig, int64_t n, int32_t *xy_pos, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_xy, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, xy, orig, n, xy_pos);
    return hipGetLastError();
}

hipError_t launch_edges_to_labels(const int32_t *orig, int64_t m, int32_t *eu, int32_t *ev, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edges_to_labels, dim3(blocks_for(m, kBlock)), dim3(kBlock), 0, st, orig, m, eu, ev);
    return hipGetLastError();
}

hipError_t launch_seed_from_top(const int32_t *i4, const int32_t *orig, const int32_t *pos, int64_t n, int32_t *seed,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_seed_from_top, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, i4, orig, pos, n, seed);
    return hipGetLastError();
}

hipError_t launch_seed_neighbours(int64_t n, const float4 *col, int32_t *seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_seed_neighbours, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, n, col, seed);
    return hipGetLastError();
}

hipError_t launch_ctrl_init(Ctrl *ctrl, int64_t max_iters, int64_t trace_cap, int64_t handoff_div,
                            const CtrlStart &cs, hipStream_t st)
{
    hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, st, ctrl, max_iters, trace_cap, handoff_div, cs);
    return hipGetLastError();
}

template <int MODE, bool CULL>
static hipError_t launch_scan_mode(const ScanArgs &a, int64_t nslices, int R, hipStream_t st)
{
    const unsigned gy = (unsigned)nslices;
    switch (R) {
    case 1:
        if constexpr (CULL) hipLaunchKernelGGL((k_rowscan_w<MODE>), dim3(blocks_for(a.g.n, 64), gy), dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_rowscan<1, MODE, CULL>), dim3(blocks_for(a.g.n, kBlock), gy), dim3(kBlock), 0, st, a);
        break;
    case 2: hipLaunchKernelGGL((k_rowscan<2, MODE, CULL>), dim3(blocks_for(a.g.n, 2 * kBlock), gy), dim3(kBlock), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_rowscan<4, MODE, CULL>), dim3(blocks_for(a.g.n, 4 * kBlock), gy), dim3(kBlock), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_scan_mode(const ScanArgs &a, int64_t nslices, int R, hipStream_t st)
{
    return a.cull ? launch_scan_mode<MODE, true>(a, nslices, R, st) : launch_scan_mode<MODE, false>(a, nslices, R, st);
}

// the culled scan deals each row block's surviving tiles round-robin to the
// slices (the survivors gather near the block's own Morton position, so
// contiguous slices would leave most slice blocks idle)
static ScanArgs with_interleave(const ScanArgs &a, int64_t nslices)
{
    ScanArgs b = a;
    b.interleave = a.cull ? nslices : 0;
    return b;
}

hipError_t launch_scan(const ScanArgs &a, int mode, int64_t nslices, int rows_per_thread, hipStream_t st)
{
    if (a.slice_len % kTile != 0) return hipErrorInvalidValue;
    switch (mode) {
    case kModeGdp: return launch_scan_mode<kModeGdp>(with_interleave(a, nslices), nslices, rows_per_thread, st);
    case kModeCert: return launch_scan_mode<kModeCert>(with_interleave(a, nslices), nslices, rows_per_thread, st);
    case kModeCollect:
        return launch_scan_mode<kModeCollect>(with_interleave(a, nslices), nslices, rows_per_thread, st);
    }
    return hipErrorInvalidValue;
}

__global__ __launch_bounds__(kBlock) void k_top_to_labels(const int64_t *z4p, const int32_t *i4p,
                                                          const int32_t *orig, int64_t n, int64_t *z4, int32_t *i4)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int64_t v = orig[p];
#pragma unroll
    for (int j = 0; j < kTop; ++j) {
        z4[kTop * v + j] = z4p[j * n + p];
        i4[kTop * v + j] = i4p[j * n + p];
    }
}

__global__ __launch_bounds__(kBlock) void k_b_to_positions(const int8_t *b_label, const int32_t *orig, int64_t n,
                                                           int8_t *b_pos)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < n) b_pos[p] = b_label[orig[p]];
}

hipError_t launch_b_to_positions(const int8_t *b_label, const int32_t *orig, int64_t n, int8_t *b_pos, hipStream_t st)
{
    hipLaunchKernelGGL(k_b_to_positions, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, b_label, orig, n, b_pos);
    return hipGetLastError();
}

hipError_t launch_top_to_labels(const int64_t *z4p, const int32_t *i4p, const int32_t *orig, int64_t n, int64_t *z4,
                                int32_t *i4, hipStream_t st)
{
    hipLaunchKernelGGL(k_top_to_labels, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, z4p, i4p, orig, n, z4, i4);
    return hipGetLastError();
}

hipError_t launch_control(const ControlArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_control, dim3(1), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_control_batch(const UpdateArgs *args_dev, int64_t ninst, hipStream_t st)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_control_batch, dim3((unsigned)ninst), dim3(kBlock), 0, st, args_dev);
    return hipGetLastError();
}

hipError_t launch_update(const UpdateArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_update, dim3(blocks_for(a.g.n, kBlock)), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_scan_batch(const ScanArgs *args_dev, const BatchScanItem *items, int64_t nitems, int rows,
                             bool cull, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    const dim3 grid((unsigned)nitems);
    if (cull) {
        switch (rows) {
        case 1: hipLaunchKernelGGL((k_rowscan_batch<1, true>), grid, dim3(kBlock), 0, st, args_dev, items); break;
        case 2: hipLaunchKernelGGL((k_rowscan_batch<2, true>), grid, dim3(kBlock), 0, st, args_dev, items); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (rows) {
        case 1: hipLaunchKernelGGL((k_rowscan_batch<1, false>), grid, dim3(kBlock), 0, st, args_dev, items); break;
        case 2: hipLaunchKernelGGL((k_rowscan_batch<2, false>), grid, dim3(kBlock), 0, st, args_dev, items); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_update_batch(const UpdateArgs *args_dev, const BatchTileItem *items, int64_t nitems,
                               hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_batch, dim3((unsigned)nitems), dim3(kBlock), 0, st, args_dev, items);
    return hipGetLastError();
}

hipError_t launch_ctrl_nblocks(Ctrl *ctrls, const int64_t *nblocks, int64_t ninst, hipStream_t st)
{
    hipLaunchKernelGGL(k_ctrl_nblocks, dim3(blocks_for(ninst, kBlock)), dim3(kBlock), 0, st, ctrls, nblocks, ninst);
    return hipGetLastError();
}

hipError_t launch_count_active(const Ctrl *ctrls, int64_t ninst, int32_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, st, ctrls, ninst, out);
    return hipGetLastError();
}

hipError_t launch_graph_step(const GraphStepArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_graph_step, dim3(blocks_for(a.g.n, kBlock)), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

int64_t knn_slices(int64_t n)
{
    // enough workgroups for six waves per SIMD of the 256 CUs
    const int64_t tiles = (n + kTile - 1) / kTile;
    const int64_t s = (1536 + tiles - 1) / tiles;
    return s < 1 ? 1 : (s > 8 ? 8 : s);
}

hipError_t launch_knn(const Geo &g, const float4 *col, int K, int32_t *nbr, int64_t *nbr_d, int32_t *pp,
                      int64_t *pd, hipStream_t st)
{
    if (g.n < K + 1) return hipErrorInvalidValue;
    const int64_t S = knn_slices(g.n);
    const dim3 grid(blocks_for(g.n, kBlock), (unsigned)S);
    switch (K) {
    case 10:
        hipLaunchKernelGGL(k_knn<10>, grid, dim3(kBlock), 0, st, g, col, nbr, nbr_d, S, pp, pd);
        if (S > 1) hipLaunchKernelGGL(k_knn_merge<10>, dim3(blocks_for(g.n, kBlock)), dim3(kBlock), 0, st, g, S, pp, pd, nbr, nbr_d);
        break;
    case 16:
        hipLaunchKernelGGL(k_knn<16>, grid, dim3(kBlock), 0, st, g, col, nbr, nbr_d, S, pp, pd);
        if (S > 1) hipLaunchKernelGGL(k_knn_merge<16>, dim3(blocks_for(g.n, kBlock)), dim3(kBlock), 0, st, g, S, pp, pd, nbr, nbr_d);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Radix sorts of packed keys (the candidate graph's edges, the finish's
// pairs): always the one-sweep algorithm (the library's default sorts inputs
// up to 2^20 keys by block sorts and a dozen or more merge passes, each a
// launch), over the keys' used bits only.
using OnesweepSort = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                                rocprim::default_config, 0>;

static hipError_t sort_keys(void *temp, size_t &bytes, const uint64_t *in, uint64_t *out, int64_t count, int bits,
                            hipStream_t st)
{
    return rocprim::radix_sort_keys<OnesweepSort>(temp, bytes, in, out, (size_t)count, 0u, (unsigned)bits, st);
}

// bits of the largest value below `bound` (at least 1)
static int bits_below(int64_t bound)
{
    int b = 1;
    while (b < 62 && (int64_t(1) << b) < bound) ++b;
    return b;
}

size_t csr_temp_bytes(int64_t n, int K)
{
    size_t a = 0, b = 0;
    (void)sort_keys(nullptr, a, nullptr, nullptr, n * K, 64, nullptr);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, b, (const int32_t *)nullptr, (int32_t *)nullptr, (int)(n + 1));
    return a > b ? a : b;
}

hipError_t launch_build_csr(const Geo &g, const int32_t *xy, int64_t n, int K, const int32_t *nbr, uint64_t *keys,
                            uint64_t *keys_alt, int32_t *deg, int32_t *rowptr, int32_t *col, int32_t *cost,
                            int64_t *nnz_dev, void *temp, size_t temp_bytes, int64_t cap, hipStream_t st)
{
    const int64_t nk = n * K;
    const int bb = bits_below(n);
    hipLaunchKernelGGL(k_pair_keys, dim3(blocks_for(nk, kBlock)), dim3(kBlock), 0, st, nbr, nk, K, bb, keys);
    size_t tb = temp_bytes;
    hipError_t e = sort_keys(temp, tb, keys, keys_alt, nk, 2 * bb, st);
    if (e != hipSuccess) return e;
    if ((e = hipMemsetAsync(deg, 0, (n + 1) * sizeof(int32_t), st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_count, dim3(blocks_for(nk, kBlock)), dim3(kBlock), 0, st, keys_alt, nk, bb, deg);
    tb = temp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(temp, tb, deg, rowptr, (int)(n + 1), st);
    if (e != hipSuccess) return e;
    if ((e = hipMemcpyAsync(nnz_dev, rowptr + n, sizeof(int32_t), hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
    (void)cap;   // 2*n*K >= nnz always
    if ((e = hipMemsetAsync(deg, 0, (n + 1) * sizeof(int32_t), st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_fill, dim3(blocks_for(nk, kBlock)), dim3(kBlock), 0, st, keys_alt, nk, bb, rowptr, deg,
                       col);
    hipLaunchKernelGGL(k_row_finish, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, xy, g.orig, n, rowptr, col,
                       cost);
    return hipGetLastError();
}

size_t pair_sort_temp_bytes(int64_t count)
{
    size_t a = 0, b = 0;
    (void)sort_keys(nullptr, a, nullptr, nullptr, count, 64, nullptr);
    (void)hipcub::DeviceSelect::Unique(nullptr, b, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                       (int64_t *)nullptr, (int)count);
    return a > b ? a : b;
}

hipError_t launch_sort_unique_pairs(const int2 *pairs, int64_t count, int64_t n, uint64_t *keys,
                                    uint64_t *keys_sorted, uint64_t *keys_out, int64_t *count_dev, void *temp,
                                    size_t temp_bytes, const int32_t *xy, int32_t *costs, hipStream_t st)
{
    if (count <= 0) return hipMemsetAsync(count_dev, 0, sizeof(int64_t), st);
    // ends are positions below n
    const int bb = bits_below(n);
    hipLaunchKernelGGL(k_pair_to_key, dim3(blocks_for(count, kBlock)), dim3(kBlock), 0, st, pairs, count, bb, keys);
    size_t tb = temp_bytes;
    hipError_t e = sort_keys(temp, tb, keys, keys_sorted, count, 2 * bb, st);
    if (e != hipSuccess) return e;
    tb = temp_bytes;
    e = hipcub::DeviceSelect::Unique(temp, tb, keys_sorted, keys_out, count_dev, (int)count, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_key_widen, dim3(blocks_for(count, kBlock)), dim3(kBlock), 0, st, keys_out, count_dev, count,
                       bb);
    if (costs) {
        hipLaunchKernelGGL(k_key_info, dim3(blocks_for(count, kBlock)), dim3(kBlock), 0, st, keys_out, count_dev,
                           count, xy, (const int64_t *)nullptr, costs, (uint8_t *)nullptr);
        e = hipGetLastError();
    }
    return e;
}

// flags[i] = 1 for the distinct keys (i < count) not in the sorted set ex
__global__ __launch_bounds__(kBlock) void k_flag_new(const uint64_t *keys, const int64_t *count, int64_t cap,
                                                     const uint64_t *ex, int64_t nex, uint8_t *flags)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= cap) return;
    uint8_t f = 0;
    if (i < *count) {
        const uint64_t k = keys[i];
        int64_t lo = 0, hi = nex;   // first ex[j] >= k
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ex[mid] < k) lo = mid + 1;
            else hi = mid;
        }
        f = (lo < nex && ex[lo] == k) ? 0 : 1;
    }
    flags[i] = f;
}

size_t exclude_temp_bytes(int64_t count)
{
    size_t b = 0;
    (void)hipcub::DeviceSelect::Flagged(nullptr, b, (const uint64_t *)nullptr, (const uint8_t *)nullptr,
                                        (uint64_t *)nullptr, (int64_t *)nullptr, (int)count);
    return b;
}

hipError_t launch_exclude_keys(const uint64_t *keys, const int64_t *count_dev, int64_t cap, const uint64_t *ex,
                               int64_t nex, const int32_t *xy, uint8_t *flags, uint64_t *out, int64_t *out_count,
                               int32_t *costs, void *temp, size_t temp_bytes, hipStream_t st)
{
    if (cap <= 0) return hipMemsetAsync(out_count, 0, sizeof(int64_t), st);
    hipLaunchKernelGGL(k_flag_new, dim3(blocks_for(cap, kBlock)), dim3(kBlock), 0, st, keys, count_dev, cap, ex, nex,
                       flags);
    size_t tb = temp_bytes;
    hipError_t e = hipcub::DeviceSelect::Flagged(temp, tb, keys, flags, out, out_count, (int)cap, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_key_info, dim3(blocks_for(cap, kBlock)), dim3(kBlock), 0, st, out, out_count, cap, xy,
                       (const int64_t *)nullptr, costs, (uint8_t *)nullptr);
    return hipGetLastError();
}

size_t pair_bulk_temp_bytes(int64_t count, int64_t n)
{
    (void)count;
    size_t b = 0;
    (void)hipcub::DeviceScan::InclusiveSum(nullptr, b, (const int32_t *)nullptr, (int32_t *)nullptr, (int)(n + 1));
    return b;
}

hipError_t launch_pair_bulk(const uint64_t *keys, const int64_t *count_dev, int64_t cap, const int32_t *xy,
                            const int64_t *lam, int64_t n, int32_t *costs, uint8_t *neg, int32_t *deg, int32_t *start,
                            int32_t *inc, void *temp, size_t temp_bytes, hipStream_t st)
{
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_key_info, dim3(blocks_for(cap, kBlock)), dim3(kBlock), 0, st, keys, count_dev, cap, xy, lam,
                       costs, neg);
    // deg[0] = 0, deg[v + 1] = kIncSpare + incidences of v: its inclusive sum
    // is every list's start including the free slots
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, st, deg, (int64_t)1, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, deg + 1, n, kIncSpare);
    hipLaunchKernelGGL(k_inc_count, dim3(blocks_for(cap, kBlock)), dim3(kBlock), 0, st, keys, count_dev, cap, deg);
    size_t tb = temp_bytes;
    hipError_t e = hipcub::DeviceScan::InclusiveSum(temp, tb, deg, start, (int)(n + 1), st);
    if (e != hipSuccess) return e;
    // deg[0 .. n) becomes each list's fill cursor, then its length
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, deg, n, 0);
    hipLaunchKernelGGL(k_inc_place, dim3(blocks_for(cap, kBlock)), dim3(kBlock), 0, st, keys, count_dev, cap, start,
                       deg, inc);
    hipLaunchKernelGGL(k_inc_order, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, start, deg, n, inc);
    return hipGetLastError();
}

hipError_t launch_graph_dual(const Geo &g, const Csr &csr, const int64_t *lam_sorted, unsigned long long *acc,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_graph_dual, dim3(blocks_for(g.n, kBlock)), dim3(kBlock), 0, st, g, csr, lam_sorted, acc);
    return hipGetLastError();
}

hipError_t launch_graph_collect(const Geo &g, const Csr &csr, const int64_t *lam_sorted, int64_t slack,
                                unsigned long long *count, int2 *out, int64_t cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_graph_collect, dim3(blocks_for(g.n, kBlock)), dim3(kBlock), 0, st, g, csr, lam_sorted,
                       slack, count, out, cap);
    return hipGetLastError();
}

hipError_t launch_graph_membership(const Geo &g, const Csr &csr, int64_t m, const int32_t *eu, const int32_t *ev,
                                   unsigned long long *acc, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_graph_membership, dim3(blocks_for(m, kBlock)), dim3(kBlock), 0, st, g, csr, m, eu, ev, acc);
    return hipGetLastError();
}

hipError_t launch_csr_to_labels(const Geo &g, const Csr &csr, int32_t *rowptr_l, int32_t *col_l, int32_t *deg_tmp,
                                hipStream_t st)
{
    // rows by label: degrees, exclusive sum (host-sized scan in one block), fill
    hipLaunchKernelGGL(k_label_degrees, dim3(blocks_for(g.n, kBlock)), dim3(kBlock), 0, st, g, csr, deg_tmp);
    size_t tb = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, tb, deg_tmp, rowptr_l, (int)(g.n + 1), st);
    if (e != hipSuccess) return e;
    void *temp = nullptr;
    if ((e = hipMallocAsync(&temp, tb, st)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(deg_tmp + g.n, 0, sizeof(int32_t), st)) != hipSuccess) return e;
    e = hipcub::DeviceScan::ExclusiveSum(temp, tb, deg_tmp, rowptr_l, (int)(g.n + 1), st);
    (void)hipFreeAsync(temp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_label_rows, dim3(blocks_for(g.n, kBlock)), dim3(kBlock), 0, st, g, csr, rowptr_l, col_l);
    return hipGetLastError();
}

hipError_t launch_extract_trivial(const int64_t *z4, const int32_t *i4, int64_t n, int32_t *su, int32_t *sv,
                                  uint8_t *sx, hipStream_t st)
{
    hipLaunchKernelGGL(k_extract_trivial, dim3(blocks_for(kTop * n, kBlock)), dim3(kBlock), 0, st, z4, i4, n, su,
                       sv, sx);
    return hipGetLastError();
}

int64_t compact_block_tmp_len(int64_t nslots) { return (nslots + kBlock - 1) / kBlock; }

hipError_t launch_compact(const int32_t *su, const int32_t *sv, const uint8_t *sx, int64_t ns, int32_t *eu,
                          int32_t *ev, uint8_t *ex, int64_t *count_dev, int32_t *btmp, hipStream_t st)
{
    const unsigned nb = blocks_for(ns, kBlock);
    if (nb == 0) return hipMemsetAsync(count_dev, 0, sizeof(int64_t), st);
    hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(kBlock), 0, st, su, ns, btmp);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, st, btmp, (int64_t)nb, count_dev);
    hipLaunchKernelGGL(k_compact_scatter, dim3(nb), dim3(kBlock), 0, st, su, sv, sx, ns, btmp, eu, ev, ex);
    return hipGetLastError();
}

hipError_t launch_cert_edges(const int32_t *xy, int64_t n, int64_t m, const int32_t *eu, const int32_t *ev,
                             const uint8_t *ex2, int32_t *deg, int32_t *cnt, int32_t *nb, unsigned long long *acc,
                             hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cert_edges, dim3(blocks_for(m, kBlock)), dim3(kBlock), 0, st, xy, n, m, eu, ev, ex2, deg,
                       cnt, nb, acc);
    return hipGetLastError();
}

hipError_t launch_cert_nodes(const int64_t *lam, int64_t n, const int32_t *deg, const int32_t *cnt,
                             const int32_t *nb, unsigned long long *acc, const int8_t *b, hipStream_t st)
{
    hipLaunchKernelGGL(k_cert_nodes, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, st, lam, n, deg, cnt, nb, acc, b);
    return hipGetLastError();
}

}  // namespace f2m
