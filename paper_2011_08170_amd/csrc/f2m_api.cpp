// Host runtime of libf2m: contexts, device workspaces, the GDP loop with its
// device-side stop test, the finish and the certificate, behind the C ABI
// declared in include/f2m.h.
#include "f2m.h"
#include "f2m_finish.h"
#include "f2m_internal.h"
#include "f2m_mlp.h"
#include "f2m_sec.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <new>
#include <string>
#include <thread>
#include <sched.h>
#include <initializer_list>
#include <vector>

using namespace f2m;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct HostBuf {   // pinned host memory
    void *p = nullptr;
    void *dp = nullptr;   // the same memory as the device addresses it
    size_t bytes = 0;
};

}  // namespace

struct f2m_ctx {
    int device = 0;
    std::string device_name;   // hipDeviceProp_t::name, the tuner cache's device key
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<DevBuf *> bufs;
    // geometry of the current instance (sorted order)
    DevBuf xy, minmax, keys, keys_alt, ids, orig, pos, box, xy2max, sort_temp;
    // GDP loop state
    DevBuf col, lam[2], lam_best, lam_label, tile_hmax, pz, pi, pneg, pzero, prowneg, pflag, z4, i4, z4p, i4p, seed,
        ctrl, trace, lst, lcnt, loff, tpart, slots, kinds;
    // trivial x
    DevBuf slot_u, slot_v, slot_x, eu, ev, ex, btmp, count;
    // certificate / pair collection state
    DevBuf c_col, c_lam, c_tile_hmax, c_ctrl, c_deg, c_cnt, c_nb, c_acc, c_lam_label, c_eu, c_ev, c_ex;
    DevBuf p_pairs, p_count, p_keys, p_keys2, p_keys3, p_temp, p_ucount, p_costs, p_neg, p_deg, p_start, p_inc, p_ucount2,
        p_cand;
    // the exact finish's node order (Morton positions): coordinates, Lam
    DevBuf f_xyp, f_lam;
    // node degrees b (b-matching rows) by label and by position
    DevBuf deg_label, deg_pos;
    // candidate graph
    DevBuf knn_nbr, knn_pp, knn_pd, csr_keys, csr_keys2, csr_deg, csr_rowptr, csr_col, csr_cost, csr_temp, csr_nnz;
    // GDP with subtour rows
    DevBuf s_ctrl, s_rowp, s_cnt, s_rptr, s_cur, s_rmem, s_lam0, s_lam1, s_lamb, s_lamp, s_mu0, s_mu1, s_mub, s_pz,
        s_pc, s_prn, s_ppr, s_pxz, s_pxc, s_xz, s_xc, s_slots, s_trace, s_parent, s_pzi, s_pxi, s_seed, s_tileh,
        s_tpart, s_rseed;
    // warm-start network
    DevBuf m_nbr, m_nbrd, m_sorted, m_temp, m_scale, m_feat, m_w1b, m_w2b, m_z1, m_h1b, m_z2, m_h2, m_y, m_dy, m_g2b,
        m_g2f, m_pre1, m_g1b, m_g1f, m_sq, m_part, m_lam0;
    // batched solve pools
    DevBuf b_xy, b_orig, b_pos, b_col, b_box, b_x2m, b_lam0, b_lam1, b_best, b_lamlabel, b_thm, b_pz, b_pi, b_pneg,
        b_pzero, b_prn, b_z4, b_i4, b_seed, b_ctrl, b_trace, b_sargs, b_uargs, b_sitems, b_uitems, b_nblk, b_active,
        b_slots;
    Ctrl *ctrl_host = nullptr;   // pinned
    int64_t *scratch_host = nullptr;   // pinned, 16 entries
    // the finish's host side: pinned staging of the GPU's pair data, and its
    // workspace and result, kept from one solve to the next
    HostBuf h_keys, h_costs, h_neg, h_start, h_inc, h_xyp, h_lamp, h_up, h_down, h_progress;
    // recorded after the copy kernels that read h_up; the next upload waits
    // on it before it rewrites (or reallocates) the staging
    hipEvent_t up_done = nullptr;
    bool up_pending = false;
    // this device's copy of the no-alloc workspace (f2m_gdp_step_noalloc),
    // or null with noalloc_err set when the lookup failed
    void *noalloc = nullptr;
    hipError_t noalloc_err = hipSuccess;
    f2m::FinishWork *fwork = nullptr;
    f2m::FinishResult fres;
    // contexts (own stream and workspaces) of the batch's finishing threads
    std::vector<f2m_ctx *> workers;
    bool is_worker = false;   // one of those: its finish runs on one thread
    // opts of calls given none (f2m_create's defaults)
    f2m_opts defaults;
    // device bytes held by the DevBufs, and the cap of the current call (0: none)
    size_t dev_total = 0;
    size_t dev_cap = 0;

    f2m_ctx()
    {
        DevBuf *all[] = {&xy, &minmax, &keys, &keys_alt, &ids, &orig, &pos, &box, &xy2max, &sort_temp,
                         &col, &lam[0], &lam[1], &lam_best, &lam_label, &tile_hmax, &pz, &pi, &pneg, &pzero,
                         &prowneg, &pflag, &z4, &i4, &z4p, &i4p, &seed, &ctrl, &trace, &lst, &lcnt, &loff, &tpart, &slots, &kinds, &slot_u, &slot_v, &slot_x, &eu, &ev, &ex,
                         &btmp, &count, &c_col, &c_lam, &c_tile_hmax, &c_ctrl, &c_deg, &c_cnt, &c_nb, &c_acc,
                         &c_lam_label, &c_eu, &c_ev, &c_ex, &p_pairs, &p_count, &p_keys, &p_keys2, &p_keys3, &p_temp, &p_ucount, &p_costs, &p_neg, &p_deg, &p_start, &p_inc, &p_ucount2, &p_cand, &f_xyp, &f_lam, &deg_label, &deg_pos, &knn_nbr, &knn_pp, &knn_pd, &csr_keys,
                         &csr_keys2, &csr_deg, &csr_rowptr, &csr_col, &csr_cost, &csr_temp, &csr_nnz,
                         &b_xy, &b_orig, &b_pos, &b_col, &b_box, &b_x2m, &b_lam0, &b_lam1, &b_best, &b_lamlabel,
                         &b_thm, &b_pz, &b_pi, &b_pneg, &b_pzero, &b_prn, &b_z4, &b_i4, &b_seed, &b_ctrl, &b_trace,
                         &b_sargs, &b_uargs, &b_sitems, &b_uitems, &b_nblk, &b_active, &b_slots, &m_nbr, &m_nbrd, &m_sorted,
                         &m_temp, &m_scale, &m_feat, &m_w1b, &m_w2b, &m_z1, &m_h1b, &m_z2, &m_h2, &m_y, &m_dy, &m_g2b,
                         &m_g2f, &m_pre1, &m_g1b, &m_g1f, &m_sq, &m_part, &m_lam0, &s_ctrl, &s_rowp, &s_cnt,
                         &s_rptr, &s_cur, &s_rmem, &s_lam0, &s_lam1, &s_lamb, &s_lamp, &s_mu0, &s_mu1, &s_mub, &s_pz,
                         &s_pc, &s_prn, &s_ppr, &s_pxz, &s_pxc, &s_xz, &s_xc, &s_slots, &s_trace, &s_parent, &s_pzi,
                         &s_pxi, &s_seed, &s_tileh, &s_tpart, &s_rseed};
        bufs.assign(std::begin(all), std::end(all));
    }
};

namespace {

struct Fail {
    f2m_status st;
};

void fail(f2m_ctx *ctx, f2m_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    throw Fail{st};
}

void ck(f2m_ctx *ctx, hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        fail(ctx, e == hipErrorOutOfMemory ? F2M_ERR_NOMEM : F2M_ERR_DEVICE,
             std::string(what) + ": " + hipGetErrorString(e));
    }
}

// coherent: the device's writes reach host memory without waiting for the
// kernel to end (used for words the host polls)
template <typename T>
T *grow_host(f2m_ctx *ctx, HostBuf &b, size_t count, bool coherent = false)
{
    const size_t need = std::max<size_t>(count * sizeof(T), 256);
    if (b.bytes < need) {
        if (b.p) (void)hipHostFree(b.p);
        b.p = b.dp = nullptr;
        b.bytes = 0;
        ck(ctx, hipHostMalloc(&b.p, need, (coherent ? hipHostMallocCoherent : hipHostMallocDefault) | hipHostMallocMapped),
           "hipHostMalloc");
        b.bytes = need;
        ck(ctx, hipHostGetDevicePointer(&b.dp, b.p, 0), "hipHostGetDevicePointer");
    }
    return static_cast<T *>(b.p);
}

template <typename T>
T *grow(f2m_ctx *ctx, DevBuf &b, size_t count)
{
    const size_t need = std::max<size_t>(count * sizeof(T), 256);
    if (b.bytes < need) {
        if (ctx->dev_cap && ctx->dev_total - b.bytes + need > ctx->dev_cap)
            fail(ctx, F2M_ERR_NOMEM, "device workspace would pass max_device_bytes");
        if (b.p) (void)hipFree(b.p);
        ctx->dev_total -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
        ck(ctx, hipMalloc(&b.p, need), "hipMalloc");
        b.bytes = need;
        ctx->dev_total += need;
    }
    return static_cast<T *>(b.p);
}

// Start state of a GDP run from the resume options (k0, the two previous
// hashes); checked against max_iters and the warm mode.
CtrlStart resume_start(f2m_ctx *ctx, const f2m_opts &o)
{
    CtrlStart cs;
    if (o.k0 < 0 || o.k0 > o.max_iters) fail(ctx, F2M_ERR_ARG, "k0 must lie in [0, max_iters]");
    if (o.k0 > 0 && o.warm != F2M_WARM_USER) fail(ctx, F2M_ERR_ARG, "k0 > 0 resumes from lambda2_init (warm = USER)");
    if (o.resume_hash_valid && o.k0 < 2) fail(ctx, F2M_ERR_ARG, "resume hashes need k0 >= 2");
    cs.k0 = o.k0;
    cs.hvalid = o.resume_hash_valid ? 1 : 0;
    cs.h1 = o.resume_hash[0];
    cs.h2 = o.resume_hash[1];
    return cs;
}

// The call's options: the caller's, else the context's defaults; sets the
// call's device memory cap.
f2m_opts call_opts(f2m_ctx *ctx, const f2m_opts *opts)
{
    f2m_opts o = ctx->defaults;
    if (opts) {
        if (opts->struct_size != sizeof(f2m_opts)) fail(ctx, F2M_ERR_ARG, "opts.struct_size mismatch");
        o = *opts;
    }
    ctx->dev_cap = (size_t)o.max_device_bytes;
    return o;
}

// Host arrays to the device through the pinned staging h_up: copied there,
// then read by a kernel through its device mapping (parts[i] = {host
// source, device destination, bytes}).  The next call waits until those
// copy kernels have finished before it touches the staging.
struct UpPart {
    const void *src;
    void *dst;
    size_t bytes;
};
void upload(f2m_ctx *ctx, std::initializer_list<UpPart> parts, hipStream_t st);
// Device arrays to host memory the same way back (parts[i] = {device source,
// host destination, bytes}): kernels write them into the pinned staging
// h_down through its device mapping; after a stream synchronisation they
// are copied out.
void download(f2m_ctx *ctx, std::initializer_list<UpPart> parts, hipStream_t st);

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int64_t ntiles_of(int64_t n) { return (n + kTileCols - 1) / kTileCols; }
// threads per block of the update and candidate-graph step launches (one row
// per thread, one column tile per block)
constexpr int64_t kBlockThreads = kTileCols;

// Host threads for the batch's per-instance finishes: one per two hardware
// threads, at most 8 (the work per instance is a few host syncs and a small
// flow; more threads only contend).
int finish_threads()
{
    const unsigned hw = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(8u, hw / 2));
}

// Threads of a single solve's exact finish: every CPU this process may run
// on, at most 16 (measured at n = 100k: the flow takes 2.2 ms on 8 threads,
// 1.8 ms on 16).
int solve_finish_threads()
{
    cpu_set_t set;
    CPU_ZERO(&set);
    int cpus = 0;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) cpus = CPU_COUNT(&set);
    if (cpus <= 0) cpus = (int)std::thread::hardware_concurrency();
    return std::max(1, std::min(16, cpus));
}

// Scan launch shape: rows per lane and column slices (slice length a
// multiple of the tile width).  Results never depend on it.
struct ScanShape {
    int rows;          // rows per thread
    int64_t slices;
    int64_t slice_len;
};

ScanShape scan_shape_auto(int64_t n, bool cull);

ScanShape scan_shape(int64_t n, bool cull, int rows_override = 0, int64_t slices_override = 0)
{
    ScanShape s = scan_shape_auto(n, cull);
    const int64_t nt = ntiles_of(n);
    if (rows_override == 1 || rows_override == 2 || rows_override == 4) s.rows = rows_override;
    if (slices_override > 0) {
        const int64_t sl = std::min<int64_t>(slices_override, nt);
        s.slice_len = ((nt + sl - 1) / sl) * kTileCols;
        s.slices = (n + s.slice_len - 1) / s.slice_len;
    }
    return s;
}

ScanShape scan_shape_auto(int64_t n, bool cull)
{
    ScanShape s;
    const int64_t nt = ntiles_of(n);
    if (cull) {
        // one row per lane; the four waves of a block share 64 rows and the
        // surviving sub-tiles are dealt among them (4 parts: measured best at
        // n = 20k, 100k and 200k; 2 leave the SIMDs too few waves, 8 repeat
        // the tile walk too often), so one slice
        s.rows = 1;
        const int64_t sl = 1;
        s.slice_len = ((nt + sl - 1) / sl) * kTileCols;
    } else {
        s.rows = n >= 65536 ? 4 : (n >= 8192 ? 2 : 1);
        const int64_t row_blocks = (n + 256 * s.rows - 1) / (256 * s.rows);
        const int64_t target = 2048;
        int64_t sl = (target + row_blocks - 1) / row_blocks;
        sl = std::max<int64_t>(1, std::min(sl, nt));
        s.slice_len = ((nt + sl - 1) / sl) * kTileCols;
    }
    s.slices = (n + s.slice_len - 1) / s.slice_len;
    return s;
}

// Tuner cache (written by paper_2011_08170_amd/tune.py): a text file, one
// entry per line, tab-separated fields
//   device name, mode, size bucket, rows per lane, slices, chunk
// mode "culled" or "full" (f2m_solve's scan), "batch-culled" or
// "batch-full" (f2m_solve_batch: slices per instance, iterations per
// replayed graph); 0 in a field keeps the built-in choice.  Lines that start
// with '#' and lines that do not parse are skipped; a missing file is no
// error (the built-in shape is used).  The size bucket of n is the integer
// nearest to 2 log2 n, computed exactly as floor(bitlength(n^4) / 2).
int size_bucket(int64_t n)
{
    const unsigned __int128 x = (unsigned __int128)n * (unsigned __int128)n * (unsigned __int128)n * (unsigned __int128)n;
    int bits = 0;
    for (unsigned __int128 y = x; y; y >>= 1) ++bits;
    return bits / 2;
}

struct Tuned {
    bool found = false;
    int rows = 0;
    int64_t slices = 0;
    int32_t chunk = 0;
};

Tuned tuner_lookup(const f2m_ctx *ctx, const char *path, const char *mode, int64_t n)
{
    Tuned t;
    if (!path || !*path) return t;
    FILE *f = std::fopen(path, "r");
    if (!f) return t;
    const int b = size_bucket(n);
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#') continue;
        std::vector<std::string> fld;
        std::string cur;
        for (const char *c = line; *c && *c != '\n' && *c != '\r'; ++c) {
            if (*c == '\t') {
                fld.push_back(cur);
                cur.clear();
            } else {
                cur.push_back(*c);
            }
        }
        fld.push_back(cur);
        if (fld.size() < 6 || fld[0] != ctx->device_name || fld[1] != mode) continue;
        char *end = nullptr;
        const long bb = std::strtol(fld[2].c_str(), &end, 10);
        if (*end || bb != b) continue;
        const long r = std::strtol(fld[3].c_str(), &end, 10);
        if (*end || (r != 0 && r != 1 && r != 2 && r != 4)) continue;
        const long long sl = std::strtoll(fld[4].c_str(), &end, 10);
        if (*end || sl < 0) continue;
        const long ch = std::strtol(fld[5].c_str(), &end, 10);
        if (*end || ch < 0 || ch > 4096) continue;
        t.found = true;   // the last matching line wins
        t.rows = (int)r;
        t.slices = sl;
        t.chunk = (int32_t)ch;
    }
    std::fclose(f);
    return t;
}

hipStream_t pick_stream(f2m_ctx *ctx, const f2m_opts *o)
{
    return (o && o->hip_stream) ? static_cast<hipStream_t>(o->hip_stream) : ctx->stream;
}

int64_t cost_host(const int32_t *xy, int64_t u, int64_t v)
{
    const int64_t dx = (int64_t)xy[2 * u] - xy[2 * v], dy = (int64_t)xy[2 * u + 1] - xy[2 * v + 1];
    return nint_sqrt_host(dx * dx + dy * dy);
}

char *host_alloc(f2m_ctx *ctx, size_t bytes)
{
    char *p = static_cast<char *>(std::malloc(bytes ? bytes : 1));
    if (!p) fail(ctx, F2M_ERR_NOMEM, "host allocation failed");
    return p;
}

// Geometry of the instance on the device: span check, centre, Morton
// order, tile boxes.  The GDP column records are prepared in ctx->col.
struct GeoHost {
    Geo g;
    const int32_t *xy;   // device coordinates (labels)
    int32_t cx, cy;
    float4 *col;         // GDP column records
};

struct GeoBufs {
    int32_t *orig, *pos;
    float4 *col, *box;
    float *xy2max;
};

// Device buffers of the Morton sort (keys, their sorted copy, ids and the
// radix sort's temporary storage of tb bytes).
struct SortBufs {
    uint32_t *keys, *keys2;
    int32_t *ids;
    void *temp;
    size_t tb;
};

// Morton order, centred column records and tile boxes for one instance
// whose extents are known; enqueued on st without synchronising.
void enqueue_geo_into(f2m_ctx *ctx, const int32_t *xy_dev, int64_t n, int32_t minx, int32_t miny, int32_t cx,
                      int32_t cy, const GeoBufs &b, const SortBufs &s, hipStream_t st)
{
    ck(ctx, launch_sort(xy_dev, n, minx, miny, s.keys, s.keys2, s.ids, b.orig, b.pos, s.temp, s.tb, st), "sort");
    ck(ctx, launch_prep(xy_dev, b.orig, n, cx, cy, b.col, b.box, b.xy2max, st), "prep");
}

SortBufs grow_sort(f2m_ctx *ctx, int64_t n)
{
    const size_t tb = sort_temp_bytes(n);
    return SortBufs{grow<uint32_t>(ctx, ctx->keys, n), grow<uint32_t>(ctx, ctx->keys_alt, n),
                    grow<int32_t>(ctx, ctx->ids, n), grow<char>(ctx, ctx->sort_temp, tb), tb};
}

void enqueue_geo(f2m_ctx *ctx, const int32_t *xy_dev, int64_t n, int32_t minx, int32_t miny, int32_t cx, int32_t cy,
                 const GeoBufs &b, hipStream_t st)
{
    enqueue_geo_into(ctx, xy_dev, n, minx, miny, cx, cy, b, grow_sort(ctx, n), st);
}

// Span check, centre, Morton order and column records into the given
// buffers (m4: 4 int32 on the device); synchronises st twice.
GeoHost setup_geo_into(f2m_ctx *ctx, const int32_t *xy_dev, int64_t n, hipStream_t st, int32_t *m4,
                       const GeoBufs &b, const SortBufs &sb)
{
    GeoHost gh;
    ck(ctx, launch_minmax(xy_dev, n, m4, st), "minmax");
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, m4, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    int32_t h[4];
    std::memcpy(h, ctx->scratch_host, sizeof(h));
    if ((int64_t)h[1] - h[0] >= (1 << 20) || (int64_t)h[3] - h[2] >= (1 << 20))
        fail(ctx, F2M_ERR_RANGE, "coordinate span must be below 2^20 on each axis");
    gh.cx = (int32_t)(((int64_t)h[0] + h[1]) >> 1);
    gh.cy = (int32_t)(((int64_t)h[2] + h[3]) >> 1);
    gh.xy = xy_dev;
    enqueue_geo_into(ctx, xy_dev, n, h[0], h[2], gh.cx, gh.cy, b, sb, st);
    float x2host = 0.0f;
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, b.xy2max, sizeof(float), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    std::memcpy(&x2host, ctx->scratch_host, sizeof(float));
    gh.g = Geo{n, b.orig, b.pos, b.box, x2host};
    gh.col = b.col;
    return gh;
}

GeoHost setup_geo(f2m_ctx *ctx, const int32_t *xy_dev, int64_t n, hipStream_t st)
{
    int32_t *m4 = grow<int32_t>(ctx, ctx->minmax, 4);
    GeoBufs b{grow<int32_t>(ctx, ctx->orig, n), grow<int32_t>(ctx, ctx->pos, n), grow<float4>(ctx, ctx->col, n),
              grow<float4>(ctx, ctx->box, ntiles_of(n) * kBoxStride), grow<float>(ctx, ctx->xy2max, 1)};
    return setup_geo_into(ctx, xy_dev, n, st, m4, b, grow_sort(ctx, n));
}

// A Lam placed on the certificate / collection state: sorted Lam, column
// records and tile maxima; lam_label_dev is in label order.
LamView place_lam(f2m_ctx *ctx, const GeoHost &gh, const int64_t *lam_label_dev, hipStream_t st,
                  bool by_position = false)
{
    const int64_t n = gh.g.n;
    float4 *col = grow<float4>(ctx, ctx->c_col, n);
    int64_t *ls = grow<int64_t>(ctx, ctx->c_lam, n);
    float *th = grow<float>(ctx, ctx->c_tile_hmax, ntiles_of(n) * kBoxStride);
    Ctrl *cc = grow<Ctrl>(ctx, ctx->c_ctrl, 1);
    float *x2m = grow<float>(ctx, ctx->xy2max, 1);
    ck(ctx, launch_prep(gh.xy, gh.g.orig, n, gh.cx, gh.cy, col, const_cast<float4 *>(gh.g.box), x2m, st), "prep");
    ck(ctx, launch_ctrl_init(cc, 0, 0, 0, CtrlStart{}, st), "ctrl");
    ck(ctx, launch_set_lam(lam_label_dev, by_position ? nullptr : gh.g.orig, n, ls, col, th, cc, st), "set_lam");
    return LamView{col, ls, th, cc};
}

// Certificate of (lam, edges); lam and the edges are device arrays by label.
void certify_dev(f2m_ctx *ctx, const GeoHost &gh, const int64_t *lam_label, int64_t m, const int32_t *eu,
                 const int32_t *ev, const uint8_t *ex, hipStream_t st, int64_t out[4], const int8_t *b_label = nullptr)
{
    const int64_t n = gh.g.n;
    LamView lv = place_lam(ctx, gh, lam_label, st);
    int32_t *deg = grow<int32_t>(ctx, ctx->c_deg, n);
    int32_t *cnt = grow<int32_t>(ctx, ctx->c_cnt, n);
    int32_t *nb = grow<int32_t>(ctx, ctx->c_nb, kCertNb * n);
    unsigned long long *acc = grow<unsigned long long>(ctx, ctx->c_acc, 4);
    ck(ctx, hipMemsetAsync(deg, 0, n * sizeof(int32_t), st), "memset");
    ck(ctx, hipMemsetAsync(cnt, 0, n * sizeof(int32_t), st), "memset");
    ck(ctx, hipMemsetAsync(acc, 0, 4 * sizeof(unsigned long long), st), "memset");
    const ScanShape sh = scan_shape(n, true);
    ScanArgs sa{};
    sa.g = gh.g;
    sa.lv = lv;
    sa.slice_len = sh.slice_len;
    sa.cull = 1;
    sa.acc = acc;
    ck(ctx, launch_scan(sa, kModeCert, sh.slices, sh.rows, st), "cert_scan");
    ck(ctx, launch_cert_edges(gh.xy, n, m, eu, ev, ex, deg, cnt, nb, acc, st), "cert_edges");
    ck(ctx, launch_cert_nodes(lam_label, n, deg, cnt, nb, acc, b_label, st), "cert_nodes");
    unsigned long long h[4];
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, acc, sizeof(h), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    std::memcpy(h, ctx->scratch_host, sizeof(h));
    const int64_t rowneg = (int64_t)h[0], primal2 = (int64_t)h[1], viol = (int64_t)h[2], sl = (int64_t)h[3];
    out[0] = primal2;
    out[1] = sl + rowneg / 2;   // sl = sum_v b_v Lam_v
    out[2] = viol == 0 ? 1 : 0;
    out[3] = (viol == 0 && out[0] == out[1]) ? 1 : 0;
}

void upload(f2m_ctx *ctx, std::initializer_list<UpPart> parts, hipStream_t st)
{
    size_t total = 0;
    for (const UpPart &q : parts) total += (q.bytes + 255) / 256 * 256;
    if (ctx->up_pending) {
        // the previous upload's kernels may still read the staging
        ck(ctx, hipEventSynchronize(ctx->up_done), "upload wait");
        ctx->up_pending = false;
    }
    char *h = grow_host<char>(ctx, ctx->h_up, total);
    char *hd = static_cast<char *>(ctx->h_up.dp);
    size_t at = 0;
    for (const UpPart &q : parts) {
        if (q.bytes) {
            std::memcpy(h + at, q.src, q.bytes);
            ck(ctx, launch_copy_bytes(hd + at, q.dst, (int64_t)q.bytes, st), "upload");
        }
        at += (q.bytes + 255) / 256 * 256;
    }
    ck(ctx, hipEventRecord(ctx->up_done, st), "upload record");
    ctx->up_pending = true;
}

void download(f2m_ctx *ctx, std::initializer_list<UpPart> parts, hipStream_t st)
{
    size_t total = 0;
    for (const UpPart &q : parts) total += (q.bytes + 255) / 256 * 256;
    char *h = grow_host<char>(ctx, ctx->h_down, total);
    char *hd = static_cast<char *>(ctx->h_down.dp);
    size_t at = 0;
    for (const UpPart &q : parts) {
        if (q.bytes) ck(ctx, launch_copy_bytes(q.src, hd + at, (int64_t)q.bytes, st), "download");
        at += (q.bytes + 255) / 256 * 256;
    }
    ck(ctx, hipStreamSynchronize(st), "sync");
    at = 0;
    for (const UpPart &q : parts) {
        if (q.bytes) std::memcpy(q.dst, h + at, q.bytes);
        at += (q.bytes + 255) / 256 * 256;
    }
}

// Sorts and de-duplicates `found` collected pairs on the device and copies
// the distinct ones (increasing) and their exact costs to the host; with
// lam_bulk (device, labels) also the finish's bulk data (see PairSource).
// With exclude (a sorted device key set) only the keys outside it are
// returned; with keep the returned keys are also kept on the device
// (ctx->p_cand) and *kept is their number.
void fetch_unique_pairs(f2m_ctx *ctx, const int2 *pairs, int64_t found, const int32_t *xy_dev, int64_t n,
                        const int64_t *lam_bulk, PairSource &src, PairList &out, hipStream_t st,
                        const uint64_t *exclude = nullptr, int64_t nexclude = 0, int64_t *kept = nullptr)
{
    out.clear();
    src.costs = nullptr;
    src.keys = nullptr;
    src.nkeys = 0;
    src.neg = nullptr;
    src.inc_start = nullptr;
    src.inc = nullptr;
    if (found <= 0) return;
    uint64_t *k1 = grow<uint64_t>(ctx, ctx->p_keys, 2 * found);
    uint64_t *k2 = grow<uint64_t>(ctx, ctx->p_keys2, 2 * found);
    uint64_t *k3 = grow<uint64_t>(ctx, ctx->p_keys3, found);
    int32_t *cd = grow<int32_t>(ctx, ctx->p_costs, found);
    int64_t *uc = grow<int64_t>(ctx, ctx->p_ucount, 1);
    size_t tb = pair_sort_temp_bytes(found);
    if (lam_bulk) tb = std::max(tb, pair_bulk_temp_bytes(found, n));
    if (exclude) tb = std::max(tb, exclude_temp_bytes(found));
    void *temp = grow<char>(ctx, ctx->p_temp, tb);
    const bool excl = exclude && nexclude > 0;
    ck(ctx, launch_sort_unique_pairs(pairs, found, n, k1, k2, k3, uc, temp, tb, xy_dev,
                                     (lam_bulk || excl) ? nullptr : cd, st),
       "sort_unique");
    if (excl) {
        // only the pairs outside the kept set, compacted into k1
        int64_t *uc2 = grow<int64_t>(ctx, ctx->p_ucount2, 1);
        uint8_t *fl = grow<uint8_t>(ctx, ctx->p_neg, found);
        ck(ctx, launch_exclude_keys(k3, uc, found, exclude, nexclude, xy_dev, fl, k1, uc2, cd, temp, tb, st),
           "exclude");
        k3 = k1;
        uc = uc2;
    }
    uint8_t *ng = nullptr;
    int32_t *deg = nullptr, *stt = nullptr, *inc = nullptr;
    if (lam_bulk) {
        ng = grow<uint8_t>(ctx, ctx->p_neg, found);
        deg = grow<int32_t>(ctx, ctx->p_deg, n + 1);
        stt = grow<int32_t>(ctx, ctx->p_start, n + 1);
        inc = grow<int32_t>(ctx, ctx->p_inc, 2 * found + 2 * n);
        ck(ctx, launch_pair_bulk(k3, uc, found, xy_dev, lam_bulk, n, cd, ng, deg, stt, inc, temp, tb, st),
           "pair_bulk");
    }
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, uc, sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    const int64_t u = ctx->scratch_host[0];
    if (kept) {
        uint64_t *keep = grow<uint64_t>(ctx, ctx->p_cand, std::max<int64_t>(u, 1));
        if (u) ck(ctx, hipMemcpyAsync(keep, k3, u * sizeof(uint64_t), hipMemcpyDeviceToDevice, st), "copy");
        *kept = u;
    }
    if (u == 0) return;
    // into pinned staging, written by kernels through its device mapping;
    // the pair source's views point there
    uint64_t *hk = grow_host<uint64_t>(ctx, ctx->h_keys, u);
    int32_t *hc = grow_host<int32_t>(ctx, ctx->h_costs, u);
    ck(ctx, launch_copy_bytes(k3, ctx->h_keys.dp, u * sizeof(uint64_t), st), "copy");
    ck(ctx, launch_copy_bytes(cd, ctx->h_costs.dp, u * sizeof(int32_t), st), "copy");
    uint8_t *hn = nullptr;
    int32_t *hs = nullptr, *hi = nullptr;
    if (lam_bulk) {
        hn = grow_host<uint8_t>(ctx, ctx->h_neg, u);
        hs = grow_host<int32_t>(ctx, ctx->h_start, n + 1);
        hi = grow_host<int32_t>(ctx, ctx->h_inc, 2 * u + 2 * n);
        ck(ctx, launch_copy_bytes(ng, ctx->h_neg.dp, u, st), "copy");
        ck(ctx, launch_copy_bytes(stt, ctx->h_start.dp, (n + 1) * sizeof(int32_t), st), "copy");
        ck(ctx, launch_copy_bytes(inc, ctx->h_inc.dp, (2 * u + 2 * n) * sizeof(int32_t), st), "copy");
    }
    ck(ctx, hipStreamSynchronize(st), "sync");
    if (lam_bulk) {
        // the bulk pairs go to the finish as their sorted keys
        src.keys = hk;
        src.nkeys = u;
    } else {
        out.resize(u);
        for (int64_t i = 0; i < u; ++i) out[i] = {(int32_t)(hk[i] >> 32), (int32_t)(hk[i] & 0xffffffffULL)};
    }
    src.costs = hc;
    src.neg = hn;
    src.inc_start = hs;
    src.inc = hi;
}

// Candidate pairs for the exact finish from GPU scans of the complete
// graph.  The finish runs on Morton positions (nodes near in the plane are
// near in memory): Lam comes in and pairs go out in that order, and xyp
// holds the coordinates by position.
// pricing results up to this many pairs are sorted on the host
constexpr int64_t kHostSortMax = 1 << 16;

class GpuPairs : public PairSource {
public:
    GpuPairs(f2m_ctx *ctx, const GeoHost &gh, const int32_t *xyp, const int32_t *seed_dev, hipStream_t st)
        : ctx_(ctx), gh_(gh), xyp_(xyp), seed_(seed_dev), st_(st)
    {
    }
    bool near(const int64_t *lam, int64_t slack, PairList &out, std::string &err) override
    {
        return run(lam, seed_, 0, slack, out, err);
    }
    bool negative(const int64_t *lam, PairList &out, std::string &err) override
    {
        return run(lam, nullptr, price_slack - 1, 0, out, err);   // Z <= theta
    }

private:
    bool run(const int64_t *lam_host, const int32_t *seed, int64_t theta, int64_t slack, PairList &out,
             std::string &err)
    {
        try {
            f2m_ctx *ctx = ctx_;
            const int64_t n = gh_.g.n;
            int64_t *lam = grow<int64_t>(ctx, ctx->f_lam, n);
            unsigned long long *cnt = grow<unsigned long long>(ctx, ctx->p_count, 1);
            upload(ctx, {{lam_host, lam, n * sizeof(int64_t)}}, st_);
            LamView lv = place_lam(ctx, gh_, lam, st_, true);
            const ScanShape sh = scan_shape(n, true);
            int64_t cap = std::max<int64_t>(cap_, 8 * n);
            for (;;) {
                int2 *pairs = grow<int2>(ctx, ctx->p_pairs, cap);
                ck(ctx, hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st_), "memset");
                ScanArgs sa{};
                sa.g = gh_.g;
                sa.lv = lv;
                sa.slice_len = sh.slice_len;
                sa.cull = 1;
                sa.seed = seed;
                sa.theta = theta;
                sa.slack = slack;
                sa.count = cnt;
                sa.out = pairs;
                sa.cap = cap;
                // pricing: the scan itself drops the candidates already
                // known, so only new pairs (and their duplicates) come out
                const bool excl = !seed && ncand_ > 0;
                if (excl) {
                    sa.excl = static_cast<const uint64_t *>(ctx->p_cand.p);
                    sa.nexcl = ncand_;
                }
                ck(ctx, launch_scan(sa, kModeCollect, sh.slices, sh.rows, st_), "collect");
                ck(ctx, hipMemcpyAsync(ctx->scratch_host, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, st_), "copy");
                ck(ctx, hipStreamSynchronize(st_), "sync");
                const int64_t found = ctx->scratch_host[0];
                if (found > cap) { cap = found + found / 4; continue; }
                if (excl && found <= kHostSortMax) {
                    // few pairs: sorted and de-duplicated on the host (the
                    // finish computes their costs)
                    out.clear();
                    costs = nullptr;
                    keys = nullptr;
                    nkeys = 0;
                    neg = nullptr;
                    inc_start = nullptr;
                    inc = nullptr;
                    if (found > 0) {
                        const int2 *hp = static_cast<const int2 *>(static_cast<void *>(
                            grow_host<uint64_t>(ctx, ctx->h_keys, found)));
                        ck(ctx, launch_copy_bytes(pairs, ctx->h_keys.dp, found * sizeof(int2), st_), "copy");
                        ck(ctx, hipStreamSynchronize(st_), "sync");
                        out.resize(found);
                        for (int64_t i = 0; i < found; ++i) out[i] = {hp[i].x, hp[i].y};
                        std::sort(out.begin(), out.end());
                        out.erase(std::unique(out.begin(), out.end()), out.end());
                    }
                    cap_ = cap;
                    return true;
                }
                if (want_bulk && seed) {
                    fetch_unique_pairs(ctx, pairs, found, xyp_, n, lam, *this, out, st_, nullptr, 0, &ncand_);
                } else {
                    // (with excl the scan has already dropped the known pairs)
                    fetch_unique_pairs(ctx, pairs, found, xyp_, n, nullptr, *this, out, st_);
                }
                cap_ = cap;
                return true;
            }
        } catch (const Fail &) {
            err = ctx_->err;
            return false;
        }
    }

    f2m_ctx *ctx_;
    GeoHost gh_;
    const int32_t *xyp_;
    const int32_t *seed_;
    hipStream_t st_;
    int64_t cap_ = 0;
    int64_t ncand_ = 0;   // candidate keys kept on the device (ctx->p_cand)
};

// The candidate graph (k nearest neighbours, union-symmetrised) as CSR
// over positions.
Csr build_graph(f2m_ctx *ctx, const GeoHost &gh, int K, hipStream_t st)
{
    const int64_t n = gh.g.n;
    if (K != 10 && K != 16) fail(ctx, F2M_ERR_ARG, "knn_k must be 10 or 16");
    if (n < K + 1) fail(ctx, F2M_ERR_ARG, "the candidate graph needs n > knn_k");
    const int64_t nk = n * K;
    int32_t *nbr = grow<int32_t>(ctx, ctx->knn_nbr, nk);
    uint64_t *keys = grow<uint64_t>(ctx, ctx->csr_keys, nk);
    uint64_t *keys2 = grow<uint64_t>(ctx, ctx->csr_keys2, nk);
    int32_t *deg = grow<int32_t>(ctx, ctx->csr_deg, n + 1);
    int32_t *rowptr = grow<int32_t>(ctx, ctx->csr_rowptr, n + 1);
    int32_t *col = grow<int32_t>(ctx, ctx->csr_col, 2 * nk);
    int32_t *cost = grow<int32_t>(ctx, ctx->csr_cost, 2 * nk);
    int64_t *nnz_dev = grow<int64_t>(ctx, ctx->csr_nnz, 1);
    const size_t tb = csr_temp_bytes(n, K);
    void *temp = grow<char>(ctx, ctx->csr_temp, tb);
    ck(ctx, hipMemsetAsync(nnz_dev, 0, sizeof(int64_t), st), "memset");
    const int64_t kps = knn_slices(n) * n * K;
    ck(ctx, launch_knn(gh.g, gh.col, K, nbr, nullptr, grow<int32_t>(ctx, ctx->knn_pp, kps),
                       grow<int64_t>(ctx, ctx->knn_pd, kps), st), "knn");
    ck(ctx, launch_build_csr(gh.g, gh.xy, n, K, nbr, keys, keys2, deg, rowptr, col, cost, nnz_dev, temp, tb, 2 * nk,
                             st), "csr");
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, nnz_dev, sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    return Csr{rowptr, col, cost, ctx->scratch_host[0]};
}

// Certificate of (lam, edges) restricted to the candidate graph.
void certify_graph_dev(f2m_ctx *ctx, const GeoHost &gh, const Csr &csr, const int64_t *lam_label, int64_t m,
                       const int32_t *eu, const int32_t *ev, const uint8_t *ex, hipStream_t st, int64_t out[4],
                       const int8_t *b_label = nullptr)
{
    const int64_t n = gh.g.n;
    LamView lv = place_lam(ctx, gh, lam_label, st);
    int32_t *deg = grow<int32_t>(ctx, ctx->c_deg, n);
    int32_t *cnt = grow<int32_t>(ctx, ctx->c_cnt, n);
    int32_t *nb = grow<int32_t>(ctx, ctx->c_nb, kCertNb * n);
    unsigned long long *acc = grow<unsigned long long>(ctx, ctx->c_acc, 4);
    ck(ctx, hipMemsetAsync(deg, 0, n * sizeof(int32_t), st), "memset");
    ck(ctx, hipMemsetAsync(cnt, 0, n * sizeof(int32_t), st), "memset");
    ck(ctx, hipMemsetAsync(acc, 0, 4 * sizeof(unsigned long long), st), "memset");
    ck(ctx, launch_graph_dual(gh.g, csr, lv.lam, acc, st), "graph_dual");
    ck(ctx, launch_cert_edges(gh.xy, n, m, eu, ev, ex, deg, cnt, nb, acc, st), "cert_edges");
    ck(ctx, launch_graph_membership(gh.g, csr, m, eu, ev, acc, st), "membership");
    ck(ctx, launch_cert_nodes(lam_label, n, deg, cnt, nb, acc, b_label, st), "cert_nodes");
    unsigned long long h[4];
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, acc, sizeof(h), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    std::memcpy(h, ctx->scratch_host, sizeof(h));
    const int64_t rowneg = (int64_t)h[0], primal2 = (int64_t)h[1], viol = (int64_t)h[2], sl = (int64_t)h[3];
    out[0] = primal2;
    out[1] = sl + rowneg / 2;   // sl = sum_v b_v Lam_v
    out[2] = viol == 0 ? 1 : 0;
    out[3] = (viol == 0 && out[0] == out[1]) ? 1 : 0;
}

// Candidate pairs for the exact finish on the candidate graph.
class GpuGraphPairs : public PairSource {
public:
    GpuGraphPairs(f2m_ctx *ctx, const GeoHost &gh, const int32_t *xyp, const Csr &csr, hipStream_t st)
        : ctx_(ctx), gh_(gh), xyp_(xyp), csr_(csr), st_(st)
    {
    }
    bool near(const int64_t *lam, int64_t slack, PairList &out, std::string &err) override
    {
        return run(lam, slack < 0 ? 0 : slack, out, err);
    }
    // Z < 0 only (price_slack is not used on the candidate graph)
    bool negative(const int64_t *lam, PairList &out, std::string &err) override { return run(lam, -1, out, err); }

private:
    bool run(const int64_t *lam_host, int64_t slack, PairList &out, std::string &err)
    {
        try {
            f2m_ctx *ctx = ctx_;
            const int64_t n = gh_.g.n;
            int64_t *lam = grow<int64_t>(ctx, ctx->f_lam, n);
            unsigned long long *cnt = grow<unsigned long long>(ctx, ctx->p_count, 1);
            upload(ctx, {{lam_host, lam, n * sizeof(int64_t)}}, st_);
            LamView lv = place_lam(ctx, gh_, lam, st_, true);
            const int64_t cap = csr_.nnz + 1;
            int2 *pairs = grow<int2>(ctx, ctx->p_pairs, cap);
            ck(ctx, hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st_), "memset");
            ck(ctx, launch_graph_collect(gh_.g, csr_, lv.lam, slack, cnt, pairs, cap, st_), "graph_collect");
            ck(ctx, hipMemcpyAsync(ctx->scratch_host, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, st_), "copy");
            ck(ctx, hipStreamSynchronize(st_), "sync");
            const int64_t found = std::min<int64_t>(ctx->scratch_host[0], cap);
            if (want_bulk) {
                fetch_unique_pairs(ctx, pairs, found, xyp_, n, lam, *this, out, st_, nullptr, 0, &ncand_);
            } else {
                // pricing: known candidates stay on the device, only new pairs come back
                const bool excl = slack < 0 && ncand_ > 0;
                fetch_unique_pairs(ctx, pairs, found, xyp_, n, nullptr, *this, out, st_,
                                   excl ? static_cast<const uint64_t *>(ctx->p_cand.p) : nullptr,
                                   excl ? ncand_ : 0);
            }
            return true;
        } catch (const Fail &) {
            err = ctx_->err;
            return false;
        }
    }

    f2m_ctx *ctx_;
    GeoHost gh_;
    const int32_t *xyp_;
    Csr csr_;
    hipStream_t st_;
    int64_t ncand_ = 0;   // candidate keys kept on the device (ctx->p_cand)
};

struct LoopOut {
    Ctrl c;
    double scan_ms = 0.0;
    int64_t scan_launches = 0;
    ScanShape shape;
    int64_t *lam_star;     // device, sorted: Lam_kstar
    int64_t *lam_last;     // device, sorted: Lam_{k_last}
    double ms_kind[3] = {0.0, 0.0, 0.0};     // scan time by ScanKind (time_kernels)
    int64_t launches_kind[3] = {0, 0, 0};
    double update_ms = 0.0;                   // update launches (time_kernels)
    double update_ms_kind[3] = {0.0, 0.0, 0.0};
};

// The GDP loop on device buffers.  lam0_label_dev: device Lam_0 by label
// (null: zero).
LoopOut gdp_loop(f2m_ctx *ctx, const GeoHost &gh, const int64_t *lam0_label_dev, int64_t max_iters,
                 int64_t handoff_div, int32_t chunk_opt, bool want_trace, bool time_kernels, bool cull,
                 const Csr *csr, int rows_override, int64_t slices_override, hipStream_t st,
                 bool keep_seeds = false, const CtrlStart &cs = CtrlStart{})
{
    LoopOut o;
    const int64_t n = gh.g.n;
    // on the candidate graph the step is one fused kernel and needs no partials
    const ScanShape sh = csr ? ScanShape{1, 1, ((n + kTileCols - 1) / kTileCols) * kTileCols}
                             : scan_shape(n, cull, rows_override, slices_override);
    float4 *col = gh.col;
    int64_t *lam[2] = {grow<int64_t>(ctx, ctx->lam[0], n), grow<int64_t>(ctx, ctx->lam[1], n)};
    int64_t *best = grow<int64_t>(ctx, ctx->lam_best, n);
    int64_t *l0 = grow<int64_t>(ctx, ctx->lam_label, n);
    float *thm = grow<float>(ctx, ctx->tile_hmax, ntiles_of(n) * kBoxStride);
    int64_t *pz = grow<int64_t>(ctx, ctx->pz, sh.slices * kTop * n);
    int32_t *pi = grow<int32_t>(ctx, ctx->pi, sh.slices * kTop * n);
    int32_t *pneg = grow<int32_t>(ctx, ctx->pneg, sh.slices * n);
    int32_t *pzero = grow<int32_t>(ctx, ctx->pzero, sh.slices * n);
    int64_t *prn = grow<int64_t>(ctx, ctx->prowneg, sh.slices * n);
    const int64_t nrb = (n + (int64_t)kTileCols * sh.rows - 1) / ((int64_t)kTileCols * sh.rows);
    int32_t *pflag = grow<int32_t>(ctx, ctx->pflag, sh.slices * nrb);
    int64_t *z4 = grow<int64_t>(ctx, ctx->z4, kTop * n);
    int32_t *i4 = grow<int32_t>(ctx, ctx->i4, kTop * n);
    // the loop keeps the four smallest by position (coalesced stores); they
    // go to label order once, after the loop
    int64_t *z4p = grow<int64_t>(ctx, ctx->z4p, kTop * n);
    int32_t *i4p = grow<int32_t>(ctx, ctx->i4p, kTop * n);
    int32_t *seed = grow<int32_t>(ctx, ctx->seed, kTop * n);
    Ctrl *cd = grow<Ctrl>(ctx, ctx->ctrl, 1);
    const int64_t k0 = cs.k0;
    // records (and scan kinds) kept for iterations k0 .. k0 + trace_cap - 1
    const int64_t trace_cap = want_trace ? max_iters + 1 - k0 : std::min<int64_t>(max_iters + 1 - k0, 1 << 16);
    int64_t *trace = want_trace ? grow<int64_t>(ctx, ctx->trace, kTraceW * trace_cap) : nullptr;
    // the culled one-row-per-lane scan keeps candidate lists (kLW per row
    // and wave) and evaluates only them while they stay exact
    const bool lists = !csr && cull && sh.rows == 1;
    const int64_t groups = (n + 63) / 64;
    int32_t *lst = lists ? grow<int32_t>(ctx, ctx->lst, sh.slices * groups * kListCap) : nullptr;
    int32_t *lcnt = lists ? grow<int32_t>(ctx, ctx->lcnt, sh.slices * n) : nullptr;
    int32_t *loff = lists ? grow<int32_t>(ctx, ctx->loff, sh.slices * n) : nullptr;
    // its workgroups store their pairs tested for k_update to sum (one
    // atomic per update block instead of one per scan wave)
    unsigned long long *tpart = lists ? grow<unsigned long long>(ctx, ctx->tpart, sh.slices * ((n + 63) / 64)) : nullptr;
    unsigned long long *slots = grow<unsigned long long>(ctx, ctx->slots, (int64_t)kSlotW * ((n + kTileCols - 1) / kTileCols));
    int32_t *kinds = csr ? nullptr : grow<int32_t>(ctx, ctx->kinds, trace_cap);

    if (lam0_label_dev)
        ck(ctx, hipMemcpyAsync(l0, lam0_label_dev, n * sizeof(int64_t), hipMemcpyDeviceToDevice, st), "copy");
    else
        ck(ctx, hipMemsetAsync(l0, 0, n * sizeof(int64_t), st), "memset");
    ck(ctx, launch_ctrl_init(cd, max_iters, trace_cap, handoff_div, cs, st), "ctrl_init");
    ck(ctx, launch_set_lam(l0, gh.g.orig, n, lam[k0 & 1], col, thm, cd, st), "set_lam");
    if (!keep_seeds) ck(ctx, launch_seed_neighbours(n, col, seed, st), "seed");
    ck(ctx, hipMemcpyAsync(ctx->ctrl_host, cd, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    if (ctx->ctrl_host->maxabs_lam >= kLamLimit) fail(ctx, F2M_ERR_OVERFLOW, "|lambda2_init| must be below 2^38");

    // Iterations are queued `window` ahead of the last one the device has
    // finished, which the update's last block reports through a word of
    // pinned host memory; the host never waits for the stream to drain.
    // Iterations queued past the stop exit at once.  If the word is not
    // seen to move while the stream is idle, the control block itself is
    // read (the word only saves synchronisations).
    const int64_t window = chunk_opt > 0 ? chunk_opt : (n >= 50000 ? 2 : (n >= 5000 ? 4 : 8));
    volatile long long *pw = static_cast<volatile long long *>(grow_host<long long>(ctx, ctx->h_progress, 1, true));
    *pw = -1;
    long long *pw_dev = static_cast<long long *>(ctx->h_progress.dp);
    std::vector<hipEvent_t> evs;
    struct EvGuard {
        std::vector<hipEvent_t> &v;
        ~EvGuard() { for (auto e : v) (void)hipEventDestroy(e); }
    } guard{evs};
    int64_t k = k0, seen = k0 - 1;
    bool done = false;
    while (!done) {
        for (; k <= max_iters && k - seen <= window; ++k) {
            // three events per iteration: before the scan, between scan and
            // update, after the update (the candidate graph: around its step)
            if (time_kernels) {
                for (int q = 0; q < 3; ++q) {
                    evs.push_back(nullptr);
                    ck(ctx, hipEventCreate(&evs.back()), "hipEventCreate");
                }
            }
            hipEvent_t e0 = time_kernels ? evs[evs.size() - 3] : nullptr;
            hipEvent_t e1 = time_kernels ? evs[evs.size() - 2] : nullptr, e2 = time_kernels ? evs.back() : nullptr;
            if (csr) {
                GraphStepArgs ga{gh.g, *csr, k, lam[k & 1], lam[(k + 1) & 1], best, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, cd, trace, slots, pw_dev, z4p, i4p};
                if (e0) ck(ctx, hipEventRecord(e0, st), "hipEventRecord");
                ck(ctx, launch_graph_step(ga, st), "graph_step");
                if (e1) ck(ctx, hipEventRecord(e1, st), "hipEventRecord");
                const ControlArgs ca{cd, n, k, (n + kBlockThreads - 1) / kBlockThreads, slots, trace, nullptr, pw_dev, 0};
                ck(ctx, launch_control(ca, st), "control");
                if (e2) ck(ctx, hipEventRecord(e2, st), "hipEventRecord");
                continue;
            }
            ScanArgs sa{};
            sa.g = gh.g;
            sa.lv = LamView{col, lam[k & 1], thm, cd};
            sa.slice_len = sh.slice_len;
            sa.cull = cull ? 1 : 0;
            sa.check_done = 1;
            sa.tested = &cd->pairs_tested;
            sa.seed = seed;
            sa.pz = pz; sa.pi = pi; sa.pneg = pneg; sa.pzero = pzero; sa.prowneg = prn;
            // the culled one-row-per-lane scan writes every row's partial
            // (its blocks hold 64 rows, not the flags' row blocks)
            int32_t *pf = (cull && sh.rows == 1) ? nullptr : pflag;
            sa.pflag = pf;
            sa.nrb = nrb;
            sa.lst = lst;
            sa.lcnt = lcnt;
            sa.loff = loff;
            sa.tpart = tpart;
            if (e0) ck(ctx, hipEventRecord(e0, st), "hipEventRecord");
            ck(ctx, launch_scan(sa, kModeGdp, sh.slices, sh.rows, st), "scan");
            if (e1) ck(ctx, hipEventRecord(e1, st), "hipEventRecord");
            UpdateArgs ua{gh.g, sh.slices, k, pz, pi, pneg, pzero, prn, lam[k & 1], lam[(k + 1) & 1], best, col,
                          thm, nullptr, nullptr, seed, nullptr, nullptr, nullptr, cd, trace, pf, nrb, sh.rows,
                          lists ? 1 : 0, tpart, slots, kinds, pw_dev, z4p, i4p, lst, lcnt, loff};
            ck(ctx, launch_update(ua, st), "update");
            const ControlArgs ca{cd, n, k, (n + kBlockThreads - 1) / kBlockThreads, slots, trace, kinds, pw_dev,
                                 lists ? 1 : 0};
            ck(ctx, launch_control(ca, st), "control");
            if (e2) ck(ctx, hipEventRecord(e2, st), "hipEventRecord");
        }
        // wait for the device to finish another iteration
        for (long spin = 0;; ++spin) {
            const long long w = *pw;
            if (w >= 0 && (w >> 1) > seen) {
                seen = w >> 1;
                done = (w & 1) != 0;
                break;
            }
            if ((spin & 4095) == 4095 && hipStreamQuery(st) == hipSuccess) {
                // everything queued has run: read the control block
                ck(ctx, hipMemcpyAsync(ctx->ctrl_host, cd, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "copy");
                ck(ctx, hipStreamSynchronize(st), "sync");
                seen = std::max<int64_t>(seen, ctx->ctrl_host->k_last);
                done = ctx->ctrl_host->done != 0;
                if (!done && k > max_iters) fail(ctx, F2M_ERR_DEVICE, "GDP loop passed the cap without stopping");
                break;
            }
        }
    }
    ck(ctx, launch_top_to_labels(z4p, i4p, gh.g.orig, n, z4, i4, st), "top_to_labels");
    ck(ctx, hipMemcpyAsync(ctx->ctrl_host, cd, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    if (time_kernels) {
        // the iterations that ran (later ones exited at once), by the kind
        // of scan each was (complete graph)
        const int64_t ran = ctx->ctrl_host->k_last + 1 - k0;
        std::vector<int32_t> kk(std::max<int64_t>(ran, 1), kScanFull);
        const int64_t nk = kinds ? std::max<int64_t>(0, std::min<int64_t>(ran, trace_cap)) : 0;
        if (nk > 0) ck(ctx, hipMemcpy(kk.data(), kinds, nk * sizeof(int32_t), hipMemcpyDeviceToHost), "copy");
        for (int64_t j = 0; j < ran && 3 * j + 2 < (int64_t)evs.size(); ++j) {
            float ms = 0.0f, mu = 0.0f;
            ck(ctx, hipEventElapsedTime(&ms, evs[3 * j], evs[3 * j + 1]), "hipEventElapsedTime");
            ck(ctx, hipEventElapsedTime(&mu, evs[3 * j + 1], evs[3 * j + 2]), "hipEventElapsedTime");
            o.scan_ms += ms;
            ++o.scan_launches;
            const int kind = (kk[j] >= 0 && kk[j] < 3) ? kk[j] : kScanFull;
            o.ms_kind[kind] += ms;
            ++o.launches_kind[kind];
            o.update_ms += mu;
            o.update_ms_kind[kind] += mu;
        }
    }
    o.shape = sh;
    o.c = *ctx->ctrl_host;
    if (o.c.overflow) fail(ctx, F2M_ERR_OVERFLOW, "|lambda2| reached 2^38");
    int64_t *last = lam[o.c.k_last & 1];
    o.lam_star = (o.c.kstar == o.c.k_last) ? last : best;
    o.lam_last = last;
    return o;
}

f2m_status solve_n3(f2m_ctx *ctx, const int32_t *xy, f2m_result *out)
{
    // the triangle is the only degree-2 solution; lambda from c_uv = lambda_u + lambda_v
    const int64_t c01 = cost_host(xy, 0, 1), c02 = cost_host(xy, 0, 2), c12 = cost_host(xy, 1, 2);
    out->n = 3;
    out->lambda2 = reinterpret_cast<int64_t *>(host_alloc(ctx, 3 * sizeof(int64_t)));
    out->lambda2_gdp = reinterpret_cast<int64_t *>(host_alloc(ctx, 3 * sizeof(int64_t)));
    out->lambda2[0] = c01 + c02 - c12;
    out->lambda2[1] = c01 + c12 - c02;
    out->lambda2[2] = c02 + c12 - c01;
    std::memcpy(out->lambda2_gdp, out->lambda2, 3 * sizeof(int64_t));
    out->n_edges = 3;
    out->edge_u = reinterpret_cast<int32_t *>(host_alloc(ctx, 3 * sizeof(int32_t)));
    out->edge_v = reinterpret_cast<int32_t *>(host_alloc(ctx, 3 * sizeof(int32_t)));
    out->edge_x2 = reinterpret_cast<uint8_t *>(host_alloc(ctx, 3));
    const int32_t us[3] = {0, 0, 1}, vs[3] = {1, 2, 2};
    for (int e = 0; e < 3; ++e) { out->edge_u[e] = us[e]; out->edge_v[e] = vs[e]; out->edge_x2[e] = 2; }
    out->primal2 = 2 * (c01 + c02 + c12);
    out->dual2 = out->dual2_gdp = out->primal2;   // every Z is 0
    out->certified = 1;
    out->stop = F2M_STOP_TRIVIAL;
    return F2M_OK;
}

// Features of every node (by label) and the scale, on device.
void features_dev(f2m_ctx *ctx, const GeoHost &gh, uint16_t *feat, float *scale_dev, hipStream_t st)
{
    const int64_t n = gh.g.n;
    if (n < kMlpIn + 1) fail(ctx, F2M_ERR_ARG, "features need n >= 17");
    int32_t *nbr = grow<int32_t>(ctx, ctx->m_nbr, n * kMlpIn);
    int64_t *nbrd = grow<int64_t>(ctx, ctx->m_nbrd, n * kMlpIn);
    uint64_t *sorted = grow<uint64_t>(ctx, ctx->m_sorted, n * kMlpIn);
    const size_t tb = median_temp_bytes(n * kMlpIn);
    void *temp = grow<char>(ctx, ctx->m_temp, tb);
    const int64_t kps = knn_slices(n) * n * kMlpIn;
    ck(ctx, launch_knn(gh.g, gh.col, kMlpIn, nbr, nbrd, grow<int32_t>(ctx, ctx->knn_pp, kps),
                       grow<int64_t>(ctx, ctx->knn_pd, kps), st), "knn16");
    ck(ctx, launch_features(nbrd, gh.g.orig, n, sorted, temp, tb, scale_dev, feat, st), "features");
}

// Network forward over n rows; keeps h1 (bf16) and h2 (fp32) in the
// workspace for a following backward pass.
void mlp_forward_dev(f2m_ctx *ctx, const float *theta, const uint16_t *feat, int64_t n, float *y, hipStream_t st)
{
    uint16_t *w1b = grow<uint16_t>(ctx, ctx->m_w1b, kMlpH * kMlpIn);
    uint16_t *w2b = grow<uint16_t>(ctx, ctx->m_w2b, kMlpH * kMlpH);
    float *z1 = grow<float>(ctx, ctx->m_z1, n * kMlpH);
    uint16_t *h1b = grow<uint16_t>(ctx, ctx->m_h1b, n * kMlpH);
    float *z2 = grow<float>(ctx, ctx->m_z2, n * kMlpH);
    float *h2 = grow<float>(ctx, ctx->m_h2, n * kMlpH);
    ck(ctx, launch_to_bf16(theta + kMlpW1, kMlpH * kMlpIn, w1b, st), "bf16");
    ck(ctx, launch_to_bf16(theta + kMlpW2, kMlpH * kMlpH, w2b, st), "bf16");
    // z1 = x W1^T, h1 = relu(z1 + b1)
    ck(ctx, launch_gemm_bf16(GemmArgs{feat, w1b, z1, n, kMlpH, kMlpIn, kMlpIn, kMlpIn, 1, 1, kMlpIn}, st), "gemm1");
    ck(ctx, launch_bias_relu(z1, theta + kMlpB1, n, kMlpH, h1b, nullptr, st), "relu1");
    // z2 = h1 W2^T, y = relu(z2 + b2) . w3 + b3
    ck(ctx, launch_gemm_bf16(GemmArgs{h1b, w2b, z2, n, kMlpH, kMlpH, kMlpH, kMlpH, 1, 1, kMlpH}, st), "gemm2");
    ck(ctx, launch_out(z2, theta, n, y, h2, st), "out");
}

// MSE gradient over n rows (forward included); loss to the host.
void mlp_grad_dev(f2m_ctx *ctx, const float *theta, const uint16_t *feat, const float *target, int64_t n, float *grad,
                  double *loss, hipStream_t st)
{
    float *y = grow<float>(ctx, ctx->m_y, n);
    mlp_forward_dev(ctx, theta, feat, n, y, st);
    const uint16_t *w2b = static_cast<const uint16_t *>(ctx->m_w2b.p);
    const uint16_t *h1b = static_cast<const uint16_t *>(ctx->m_h1b.p);
    const float *h2 = static_cast<const float *>(ctx->m_h2.p);
    float *dy = grow<float>(ctx, ctx->m_dy, n);
    uint16_t *g2b = grow<uint16_t>(ctx, ctx->m_g2b, n * kMlpH);
    float *g2f = grow<float>(ctx, ctx->m_g2f, n * kMlpH);
    float *pre1 = grow<float>(ctx, ctx->m_pre1, n * kMlpH);
    uint16_t *g1b = grow<uint16_t>(ctx, ctx->m_g1b, n * kMlpH);
    float *g1f = grow<float>(ctx, ctx->m_g1f, n * kMlpH);
    float *sq = grow<float>(ctx, ctx->m_sq, n);
    const int64_t kchunk = 4096;
    const int64_t chunks = (n + kchunk - 1) / kchunk;
    const int64_t nparts = std::max<int64_t>(1, std::min<int64_t>(256, (n + 255) / 256));
    float *part = grow<float>(ctx, ctx->m_part, std::max<int64_t>(chunks * kMlpH * kMlpH, nparts * kMlpH));
    ck(ctx, launch_out_grad(y, target, h2, theta, n, 1.0f / (float)n, dy, g2b, g2f, sq, st), "out_grad");
    ck(ctx, launch_col_sums(h2, dy, n, kMlpH, part, grad + kMlpW3, nparts, st), "dw3");
    ck(ctx, launch_col_sums(dy, nullptr, n, 1, part, grad + kMlpB3, nparts, st), "db3");
    ck(ctx, launch_col_sums(g2f, nullptr, n, kMlpH, part, grad + kMlpB2, nparts, st), "db2");
    // dW2[j][i] = sum_v g2[v][j] h1[v][i]
    ck(ctx, launch_gemm_bf16(GemmArgs{g2b, h1b, part, kMlpH, kMlpH, n, kchunk, 1, kMlpH, kMlpH, 1}, st), "dW2");
    ck(ctx, launch_sum_chunks(part, chunks, kMlpH * kMlpH, grad + kMlpW2, st), "dW2 sum");
    // g1 = (g2 W2) * [h1 > 0]
    ck(ctx, launch_gemm_bf16(GemmArgs{g2b, w2b, pre1, n, kMlpH, kMlpH, kMlpH, kMlpH, 1, kMlpH, 1}, st), "g1");
    ck(ctx, launch_mask_bf16(pre1, h1b, n * kMlpH, g1b, g1f, st), "mask1");
    ck(ctx, launch_col_sums(g1f, nullptr, n, kMlpH, part, grad + kMlpB1, nparts, st), "db1");
    // dW1[j][f] = sum_v g1[v][j] x[v][f]
    ck(ctx, launch_gemm_bf16(GemmArgs{g1b, feat, part, kMlpH, kMlpIn, n, kchunk, 1, kMlpH, kMlpIn, 1}, st), "dW1");
    ck(ctx, launch_sum_chunks(part, chunks, kMlpH * kMlpIn, grad + kMlpW1, st), "dW1 sum");
    float *ls = y;   // y is no longer needed: reuse for the loss sum
    ck(ctx, launch_col_sums(sq, nullptr, n, 1, part, ls, nparts, st), "loss");
    float lh = 0.0f;
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, ls, sizeof(float), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    std::memcpy(&lh, ctx->scratch_host, sizeof(float));
    *loss = (double)lh / (double)n;
}

// Lam_0 by label from the network (features, forward, rounding).
const int64_t *mlp_lam0_dev(f2m_ctx *ctx, const GeoHost &gh, const float *theta, hipStream_t st)
{
    const int64_t n = gh.g.n;
    uint16_t *feat = grow<uint16_t>(ctx, ctx->m_feat, n * kMlpIn);
    float *scale = grow<float>(ctx, ctx->m_scale, 1);
    float *y = grow<float>(ctx, ctx->m_y, n);
    int64_t *lam0 = grow<int64_t>(ctx, ctx->m_lam0, n);
    features_dev(ctx, gh, feat, scale, st);
    mlp_forward_dev(ctx, theta, feat, n, y, st);
    ck(ctx, launch_lam_from_pred(y, scale, n, kLamLimit / 2, lam0, st), "lam0");
    return lam0;
}

// Everything after the GDP loop for one instance: Lam* by label, the
// trivial x or the exact finish, the certificate(s) and the host copies.
struct InstanceState {
    GeoHost gh;
    Ctrl c;
    const int64_t *lam_star;   // device, sorted
    const int64_t *z4;         // device, by label
    const int32_t *i4;
    const int32_t *seed;       // device, positions
    const int64_t *trace;      // device or null
    const Csr *csr;            // candidate graph or null
    const int32_t *kinds;      // device scan kinds (with trace) or null
    const int64_t *lam_last;   // device, sorted: Lam_{k_last}
    const int8_t *b_label = nullptr;   // device node degrees by label, or null (F2M)
};

void complete_result(f2m_ctx *ctx, const InstanceState &is, const f2m_opts &o, hipStream_t st,
                     f2m_result &res)
{
    const int64_t n = is.gh.g.n;
    const GeoHost &gh = is.gh;
    const Ctrl &c = is.c;
    res.n = n;
    res.iterations = c.k_last + 1 - c.k_first;
    res.kstar = c.kstar;
    res.stop = (int32_t)c.stop;
    int64_t *lstar = grow<int64_t>(ctx, ctx->lam_label, n);
    ck(ctx, launch_unpermute(is.lam_star, gh.g.orig, n, lstar, st), "unpermute");
    res.lambda2_gdp = reinterpret_cast<int64_t *>(host_alloc(ctx, n * sizeof(int64_t)));
    res.lambda2_last = reinterpret_cast<int64_t *>(host_alloc(ctx, n * sizeof(int64_t)));
    int64_t *llast = grow<int64_t>(ctx, ctx->f_lam, n);
    ck(ctx, launch_unpermute(is.lam_last, gh.g.orig, n, llast, st), "unpermute");
    if (is.trace) {
        res.trace_len = std::min<int64_t>(res.iterations, c.trace_cap);
        res.trace = reinterpret_cast<int64_t *>(host_alloc(ctx, res.trace_len * kTraceW * sizeof(int64_t)));
    }
    if (is.kinds) res.scan_kind = reinterpret_cast<int32_t *>(host_alloc(ctx, std::max<int64_t>(res.trace_len, 1) * sizeof(int32_t)));
    download(ctx, {{lstar, res.lambda2_gdp, n * sizeof(int64_t)}, {llast, res.lambda2_last, n * sizeof(int64_t)},
                   {is.trace, res.trace, is.trace ? res.trace_len * kTraceW * sizeof(int64_t) : 0},
                   {is.kinds, res.scan_kind, is.kinds ? res.trace_len * sizeof(int32_t) : 0}}, st);
    res.scan_list_uses = c.list_uses;
    res.scan_list_builds = c.list_builds;
    res.dual2_gdp = (c.kstar == c.k_last) ? c.dual2_last : c.best_dual2;

    int32_t *eu = nullptr, *ev = nullptr;
    uint8_t *ex = nullptr;
    int64_t m = 0;
    const int64_t *lam_final_dev = lstar;
    const double t3 = now_s();
    bool have_x = false;
    // with degrees b a node may have up to 2 b = 6 edges of Z <= 0, more
    // than its four smallest hold: the finish then produces x
    if (c.stop == F2M_STOP_TRIVIAL && !gh.g.b) {
        const int64_t ns = kTop * n;
        int32_t *su = grow<int32_t>(ctx, ctx->slot_u, ns);
        int32_t *sv = grow<int32_t>(ctx, ctx->slot_v, ns);
        uint8_t *sx = grow<uint8_t>(ctx, ctx->slot_x, ns);
        eu = grow<int32_t>(ctx, ctx->eu, ns);
        ev = grow<int32_t>(ctx, ctx->ev, ns);
        ex = grow<uint8_t>(ctx, ctx->ex, ns);
        int32_t *bt = grow<int32_t>(ctx, ctx->btmp, compact_block_tmp_len(ns));
        int64_t *cnt = grow<int64_t>(ctx, ctx->count, 1);
        ck(ctx, launch_extract_trivial(is.z4, is.i4, n, su, sv, sx, st), "extract");
        ck(ctx, launch_compact(su, sv, sx, ns, eu, ev, ex, cnt, bt, st), "compact");
        ck(ctx, hipMemcpyAsync(ctx->scratch_host, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
        ck(ctx, hipStreamSynchronize(st), "sync");
        m = ctx->scratch_host[0];
        have_x = true;
    } else if (o.finish == F2M_FINISH_EXACT) {
        // the finish runs on Morton positions: coordinates and Lam* in that
        // order go in, its Lam and edges come back to labels on the device
        int32_t *xyp = grow<int32_t>(ctx, ctx->f_xyp, 2 * n);
        ck(ctx, launch_gather_xy(gh.xy, gh.g.orig, n, xyp, st), "gather_xy");
        int32_t *xyp_host = grow_host<int32_t>(ctx, ctx->h_xyp, 2 * n);
        int64_t *lamp_host = grow_host<int64_t>(ctx, ctx->h_lamp, n);
        ck(ctx, launch_copy_bytes(xyp, ctx->h_xyp.dp, 2 * n * sizeof(int32_t), st), "copy");
        ck(ctx, launch_copy_bytes(is.lam_star, ctx->h_lamp.dp, n * sizeof(int64_t), st), "copy");
        ck(ctx, hipStreamSynchronize(st), "sync");
        if (!ctx->fwork) ctx->fwork = finish_work_create(ctx->is_worker ? 1 : solve_finish_threads());
        FinishResult &fr = ctx->fres;
        std::vector<int32_t> bpos;   // node degrees by position (b-matching), else empty
        if (gh.g.b) {
            std::vector<int8_t> b8(n);
            download(ctx, {{gh.g.b, b8.data(), (size_t)n}}, st);
            bpos.assign(b8.begin(), b8.end());
        }
        const int32_t *bp = bpos.empty() ? nullptr : bpos.data();
        if (is.csr) {
            GpuGraphPairs src(ctx, gh, xyp, *is.csr, st);
            finish_exact(xyp_host, n, lamp_host, src, &fr, ctx->fwork, bp);
        } else {
            GpuPairs src(ctx, gh, xyp, is.seed, st);
            finish_exact(xyp_host, n, lamp_host, src, &fr, ctx->fwork, bp);
        }
        res.finish_paths = fr.paths;
        res.finish_rounds = fr.rounds;
        res.finish_phases = fr.phases;
        res.finish_candidates = fr.candidates;
        res.finish_seconds[0] = fr.t_collect;
        res.finish_seconds[1] = fr.t_build;
        res.finish_seconds[2] = fr.t_flow;
        if (!fr.ok) fail(ctx, F2M_ERR_DEVICE, "exact finish failed: " + fr.msg);
        m = (int64_t)fr.eu.size();
        eu = grow<int32_t>(ctx, ctx->c_eu, std::max<int64_t>(m, 1));
        ev = grow<int32_t>(ctx, ctx->c_ev, std::max<int64_t>(m, 1));
        ex = grow<uint8_t>(ctx, ctx->c_ex, std::max<int64_t>(m, 1));
        // the GDP multipliers stay available in lstar; the certificate's
        // duals go to their own buffer
        int64_t *lf = grow<int64_t>(ctx, ctx->lam_best, n);
        int64_t *lp = grow<int64_t>(ctx, ctx->f_lam, n);
        upload(ctx, {{fr.lam.data(), lp, n * sizeof(int64_t)}, {fr.eu.data(), eu, m * sizeof(int32_t)},
                     {fr.ev.data(), ev, m * sizeof(int32_t)}, {fr.ex2.data(), ex, m * sizeof(uint8_t)}}, st);
        ck(ctx, launch_unpermute(lp, gh.g.orig, n, lf, st), "unpermute");
        if (m) ck(ctx, launch_edges_to_labels(gh.g.orig, m, eu, ev, st), "edges_to_labels");
        lam_final_dev = lf;
        have_x = true;
    }
    const double t4 = now_s();
    int64_t cert[4] = {0, 0, 0, 0}, cert_full[4] = {0, 0, 0, 0};
    if (have_x) {
        if (is.csr) {
            certify_graph_dev(ctx, gh, *is.csr, lam_final_dev, m, eu, ev, ex, st, cert, is.b_label);
            certify_dev(ctx, gh, lam_final_dev, m, eu, ev, ex, st, cert_full, is.b_label);
        } else {
            certify_dev(ctx, gh, lam_final_dev, m, eu, ev, ex, st, cert, is.b_label);
            std::memcpy(cert_full, cert, sizeof(cert));
        }
    }
    const double t5 = now_s();
    res.n_edges = m;
    res.edge_u = reinterpret_cast<int32_t *>(host_alloc(ctx, std::max<int64_t>(m, 1) * sizeof(int32_t)));
    res.edge_v = reinterpret_cast<int32_t *>(host_alloc(ctx, std::max<int64_t>(m, 1) * sizeof(int32_t)));
    res.edge_x2 = reinterpret_cast<uint8_t *>(host_alloc(ctx, std::max<int64_t>(m, 1)));
    res.lambda2 = reinterpret_cast<int64_t *>(host_alloc(ctx, n * sizeof(int64_t)));
    download(ctx, {{eu, res.edge_u, m * sizeof(int32_t)}, {ev, res.edge_v, m * sizeof(int32_t)},
                   {ex, res.edge_x2, m * sizeof(uint8_t)}, {lam_final_dev, res.lambda2, n * sizeof(int64_t)}}, st);
    res.primal2 = cert[0];
    res.dual2 = have_x ? cert[1] : res.dual2_gdp;
    res.certified = (int32_t)cert[3];
    res.dual2_complete = have_x ? cert_full[1] : 0;
    res.certified_complete = (int32_t)cert_full[3];
    res.scan_pairs = (int64_t)c.pairs_tested;
    res.seconds[3] = t4 - t3;
    res.seconds[4] = t5 - t4;
}

// Every device buffer one GDP iteration uses (f2m_gdp_step).
struct StepBufs {
    int32_t *m4;
    GeoBufs geo;
    SortBufs sort;
    int64_t *ls, *lo, *best;
    float *thm;
    int64_t *pz;
    int32_t *pi, *pneg, *pzero;
    int64_t *prn;
    int64_t *z4;
    int32_t *i4, *seed;
    Ctrl *cd;
    int64_t *trace;
    unsigned long long *slots;
};

// One GDP iteration (culled scan, update) from lam_in (device, labels) into
// the given buffers; lam_out, neg, zero, step by label; rec to the host.
void gdp_step_run(f2m_ctx *ctx, const int32_t *xy, int64_t n, const int64_t *lam_in, int64_t *lam_out, int32_t *neg,
                  int32_t *zero, int64_t *step, int64_t rec[F2M_TRACE_W], const StepBufs &b)
{
    hipStream_t st = ctx->stream;
    const GeoHost gh = setup_geo_into(ctx, xy, n, st, b.m4, b.geo, b.sort);
    const ScanShape sh = scan_shape(n, true);
    float4 *col = gh.col;
    ck(ctx, launch_ctrl_init(b.cd, INT64_MAX, 1, 0, CtrlStart{}, st), "ctrl_init");
    ck(ctx, launch_set_lam(lam_in, gh.g.orig, n, b.ls, col, b.thm, b.cd, st), "set_lam");
    ck(ctx, launch_seed_neighbours(n, col, b.seed, st), "seed");
    ck(ctx, hipMemcpyAsync(ctx->ctrl_host, b.cd, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    if (ctx->ctrl_host->maxabs_lam >= kLamLimit) fail(ctx, F2M_ERR_OVERFLOW, "|lambda2| must be below 2^38");
    ScanArgs sa{};
    sa.g = gh.g;
    sa.lv = LamView{col, b.ls, b.thm, b.cd};
    sa.slice_len = sh.slice_len;
    sa.cull = 1;
    sa.check_done = 1;
    sa.seed = b.seed;
    sa.pz = b.pz; sa.pi = b.pi; sa.pneg = b.pneg; sa.pzero = b.pzero; sa.prowneg = b.prn;
    ck(ctx, launch_scan(sa, kModeGdp, sh.slices, sh.rows, st), "scan");
    UpdateArgs ua{gh.g, sh.slices, 0, b.pz, b.pi, b.pneg, b.pzero, b.prn, b.ls, b.lo, b.best, col, b.thm,
                  b.z4, b.i4, b.seed, neg, zero, step, b.cd, b.trace};
    ua.slots = b.slots;
    ck(ctx, launch_update(ua, st), "update");
    const ControlArgs ca{b.cd, n, 0, (n + kBlockThreads - 1) / kBlockThreads, b.slots, b.trace, nullptr, nullptr, 0};
    ck(ctx, launch_control(ca, st), "control");
    ck(ctx, launch_unpermute(b.lo, gh.g.orig, n, lam_out, st), "unpermute");
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, b.trace, kTraceW * sizeof(int64_t), hipMemcpyDeviceToHost, st),
       "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    std::memcpy(rec, ctx->scratch_host, kTraceW * sizeof(int64_t));
}

// Buffers of one GDP iteration carved out of a fixed workspace at base
// (256-byte aligned pieces); returns the bytes used.  With base == null only
// the size is computed.  z4 and i4 get workspace only when the caller gives
// none.
size_t carve_step(char *base, int64_t n, bool own_z4, bool own_i4, StepBufs *b)
{
    const ScanShape sh = scan_shape(n, true);
    const int64_t nt = ntiles_of(n);
    size_t at = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? static_cast<void *>(base + at) : nullptr;
        at += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return p;
    };
    StepBufs t{};
    t.m4 = static_cast<int32_t *>(take(4 * sizeof(int32_t)));
    t.geo.orig = static_cast<int32_t *>(take(n * sizeof(int32_t)));
    t.geo.pos = static_cast<int32_t *>(take(n * sizeof(int32_t)));
    t.geo.col = static_cast<float4 *>(take(n * sizeof(float4)));
    t.geo.box = static_cast<float4 *>(take(nt * kBoxStride * sizeof(float4)));
    t.geo.xy2max = static_cast<float *>(take(sizeof(float)));
    t.sort.tb = sort_temp_bytes(n);
    t.sort.keys = static_cast<uint32_t *>(take(n * sizeof(uint32_t)));
    t.sort.keys2 = static_cast<uint32_t *>(take(n * sizeof(uint32_t)));
    t.sort.ids = static_cast<int32_t *>(take(n * sizeof(int32_t)));
    t.sort.temp = take(t.sort.tb);
    t.ls = static_cast<int64_t *>(take(n * sizeof(int64_t)));
    t.lo = static_cast<int64_t *>(take(n * sizeof(int64_t)));
    t.best = static_cast<int64_t *>(take(n * sizeof(int64_t)));
    t.thm = static_cast<float *>(take(nt * kBoxStride * sizeof(float)));
    t.pz = static_cast<int64_t *>(take(sh.slices * kTop * n * sizeof(int64_t)));
    t.pi = static_cast<int32_t *>(take(sh.slices * kTop * n * sizeof(int32_t)));
    t.pneg = static_cast<int32_t *>(take(sh.slices * n * sizeof(int32_t)));
    t.pzero = static_cast<int32_t *>(take(sh.slices * n * sizeof(int32_t)));
    t.prn = static_cast<int64_t *>(take(sh.slices * n * sizeof(int64_t)));
    t.z4 = own_z4 ? static_cast<int64_t *>(take(kTop * n * sizeof(int64_t))) : nullptr;
    t.i4 = own_i4 ? static_cast<int32_t *>(take(kTop * n * sizeof(int32_t))) : nullptr;
    t.seed = static_cast<int32_t *>(take(kTop * n * sizeof(int32_t)));
    t.cd = static_cast<Ctrl *>(take(sizeof(Ctrl)));
    t.trace = static_cast<int64_t *>(take(kTraceW * sizeof(int64_t)));
    t.slots = static_cast<unsigned long long *>(take((size_t)kSlotW * nt * sizeof(unsigned long long)));
    if (b) *b = t;
    return at;
}


// ---------------------------------------------------------------------------
// GDP with subtour rows
// ---------------------------------------------------------------------------

void sec_check_rows(f2m_ctx *ctx, int64_t n, const f2m_sec_rows *rows)
{
    if (!rows) fail(ctx, F2M_ERR_ARG, "rows is null");
    if (rows->nlayers < 0 || rows->nlayers > F2M_SEC_MAX_LAYERS)
        fail(ctx, F2M_ERR_ARG, "rows.nlayers must lie in [0, F2M_SEC_MAX_LAYERS]");
    if (rows->nrows < 0 || rows->nrows > INT32_MAX) fail(ctx, F2M_ERR_ARG, "rows.nrows out of range");
    if (rows->nlayers == 0 && rows->nrows != 0) fail(ctx, F2M_ERR_ARG, "rows without layers");
    if (rows->nlayers > 0 && !rows->row_of) fail(ctx, F2M_ERR_ARG, "rows.row_of is null");
    if ((int64_t)kSecMaxLayers * n >= INT32_MAX) fail(ctx, F2M_ERR_ARG, "n too large for subtour rows");
}

// The device state of one call: geometry, rows as positions and member
// lists, Lam (by position), M, Lam' and the control block.
struct SecSetup {
    GeoHost gh;
    int nlayers = 0, L = 1;
    int64_t nrows = 0;
    int32_t *rowp = nullptr, *rptr = nullptr, *rmem = nullptr, *rlayer = nullptr;
    float *tile_h = nullptr;
    SecCtrl *ctrl = nullptr;
    int64_t *lam[2] = {nullptr, nullptr}, *mu[2] = {nullptr, nullptr}, *lamp = nullptr;
};

SecSetup sec_setup(f2m_ctx *ctx, const int32_t *xy, int64_t n, const f2m_sec_rows *rows, const int64_t *lam_label,
                   const int64_t *mu, int64_t max_iters, int64_t trace_cap, hipStream_t st)
{
    SecSetup s;
    s.gh = setup_geo(ctx, xy, n, st);
    s.nlayers = rows->nlayers;
    s.L = sec_layers_inst(s.nlayers);
    s.nrows = rows->nrows;
    const int64_t Q = s.nrows, L = s.L;
    s.ctrl = grow<SecCtrl>(ctx, ctx->s_ctrl, 1);
    s.rowp = grow<int32_t>(ctx, ctx->s_rowp, L * n);
    int32_t *cnt = grow<int32_t>(ctx, ctx->s_cnt, 3 * (Q + 1));
    int32_t *lo = cnt + (Q + 1), *hi = cnt + 2 * (Q + 1);
    s.rlayer = lo;
    s.lam[0] = grow<int64_t>(ctx, ctx->s_lam0, n);
    s.lam[1] = grow<int64_t>(ctx, ctx->s_lam1, n);
    s.lamp = grow<int64_t>(ctx, ctx->s_lamp, n);
    s.mu[0] = grow<int64_t>(ctx, ctx->s_mu0, Q + 1);
    s.mu[1] = grow<int64_t>(ctx, ctx->s_mu1, Q + 1);
    ck(ctx, launch_sec_ctrl_init(s.ctrl, max_iters, trace_cap, s.nlayers, st), "sec ctrl");
    ck(ctx, hipMemsetAsync(cnt, 0, (Q + 1) * sizeof(int32_t), st), "memset");
    ck(ctx, hipMemsetAsync(lo, 0x7f, (Q + 1) * sizeof(int32_t), st), "memset");
    ck(ctx, hipMemsetAsync(hi, 0xff, (Q + 1) * sizeof(int32_t), st), "memset");
    ck(ctx, launch_sec_rows_in(rows->row_of, s.gh.g.orig, n, s.nlayers, s.L, Q, s.rowp, cnt, lo, hi, s.ctrl, st),
       "sec rows");
    if (Q > 0) ck(ctx, hipMemcpyAsync(s.mu[0], mu, Q * sizeof(int64_t), hipMemcpyDeviceToDevice, st), "copy");
    ck(ctx, launch_sec_start(lam_label, s.gh.g.orig, n, s.mu[0], Q, s.lam[0], s.lamp, s.ctrl, st), "sec start");
    std::vector<int32_t> hc(3 * (Q + 1));
    SecCtrl hctrl;
    download(ctx, {{cnt, hc.data(), hc.size() * sizeof(int32_t)}, {s.ctrl, &hctrl, sizeof(SecCtrl)}}, st);
    if (hctrl.bad_input & 1) fail(ctx, F2M_ERR_ARG, "row_of holds a row id outside [-1, nrows)");
    if (hctrl.bad_input & 2) fail(ctx, F2M_ERR_ARG, "mu holds a negative multiplier");
    std::vector<int32_t> ptr(Q + 1);
    int64_t total = 0;
    for (int64_t q = 0; q < Q; ++q) {
        const int32_t c = hc[q];
        if (c < 2 || c > n - 2) fail(ctx, F2M_ERR_ARG, "every row needs 2 .. n - 2 nodes");
        if (hc[(Q + 1) + q] != hc[2 * (Q + 1) + q]) fail(ctx, F2M_ERR_ARG, "a row id occurs in two layers");
        ptr[q] = (int32_t)total;
        total += c;
    }
    ptr[Q] = (int32_t)total;
    s.rptr = grow<int32_t>(ctx, ctx->s_rptr, Q + 1);
    s.rmem = grow<int32_t>(ctx, ctx->s_rmem, total + 1);
    int32_t *cur = grow<int32_t>(ctx, ctx->s_cur, Q + 1);
    upload(ctx, {{ptr.data(), s.rptr, (Q + 1) * sizeof(int32_t)}}, st);
    ck(ctx, hipMemsetAsync(cur, 0, (Q + 1) * sizeof(int32_t), st), "memset");
    ck(ctx, launch_sec_rows_fill(s.rowp, n, s.L, s.rptr, cur, s.rmem, st), "sec fill");
    ck(ctx, launch_sec_add_mu(s.rptr, s.rmem, s.mu[0], Q, s.lamp, s.ctrl, st), "sec add");
    s.tile_h = grow<float>(ctx, ctx->s_tileh, ntiles_of(n) * kBoxStride);
    ck(ctx, launch_sec_tiles(s.lamp, n, s.tile_h, st), "sec tiles");
    return s;
}

// Column slices of the scan: enough blocks to fill the chip at small n
struct SecShape {
    int64_t slices, slice_len;
};

SecShape sec_shape(int64_t n)
{
    const int64_t tiles = (n + 255) / 256;
    int64_t S = std::min(std::max<int64_t>(1, (1024 + tiles - 1) / tiles), tiles);
    const int64_t len = ((n + S - 1) / S + 255) / 256 * 256;
    return SecShape{(n + len - 1) / len, len};
}

// Runs iterations 0 .. until the stop (at most max_iters + 1); returns the
// final control block.  trace_dev: [trace_cap][kSecTraceW] or null.
SecCtrl sec_loop(f2m_ctx *ctx, SecSetup &s, int64_t max_iters, int64_t *trace_dev, hipStream_t st)
{
    const int64_t n = s.gh.g.n, Q = s.nrows, L = s.L;
    const SecShape sh = sec_shape(n);
    const int64_t S = sh.slices;
    const int64_t nbn = (n + 255) / 256, nbr = (Q + 3) / 4;
    SecScanArgs sa{};
    sa.g = s.gh.g;
    sa.col = s.gh.col;
    sa.lamp = s.lamp;
    sa.rowp = s.rowp;
    sa.ctrl = s.ctrl;
    sa.slice_len = sh.slice_len;
    sa.tile_h = s.tile_h;
    sa.pz = grow<int64_t>(ctx, ctx->s_pz, S * 3 * n);
    sa.pzi = grow<int32_t>(ctx, ctx->s_pzi, S * 3 * n);
    sa.pxi = grow<int32_t>(ctx, ctx->s_pxi, S * L * 3 * n);
    sa.tpart = grow<unsigned long long>(ctx, ctx->s_tpart, S * nbn);
    int32_t *seed = grow<int32_t>(ctx, ctx->s_seed, (1 + L) * 3 * n);
    sa.pc = grow<int32_t>(ctx, ctx->s_pc, S * 2 * n);
    sa.prn = grow<int64_t>(ctx, ctx->s_prn, S * n);
    sa.ppr = grow<int64_t>(ctx, ctx->s_ppr, S * n);
    sa.pxz = grow<int64_t>(ctx, ctx->s_pxz, S * L * 3 * n);
    sa.pxc = grow<int32_t>(ctx, ctx->s_pxc, S * L * 2 * n);
    unsigned long long *slots = grow<unsigned long long>(ctx, ctx->s_slots, (nbn + nbr) * kSecSlotW);
    SecNodeArgs na{};
    na.g = s.gh.g;
    na.nslices = S;
    na.pz = sa.pz; na.pc = sa.pc; na.prn = sa.prn; na.ppr = sa.ppr; na.pxz = sa.pxz; na.pxc = sa.pxc;
    na.pzi = sa.pzi; na.pxi = sa.pxi;
    na.seed = seed;
    na.rowp = s.rowp;
    na.lam_best = grow<int64_t>(ctx, ctx->s_lamb, n);
    na.lamp = s.lamp;
    na.xz = grow<int64_t>(ctx, ctx->s_xz, L * 3 * n);
    na.xc = grow<int32_t>(ctx, ctx->s_xc, L * 2 * n);
    na.ctrl = s.ctrl;
    na.slots = slots;
    SecRowArgs ra{};
    ra.n = n;
    ra.nrows = Q;
    ra.rptr = s.rptr;
    ra.rmem = s.rmem;
    ra.rlayer = s.rlayer;
    ra.xz = na.xz;
    ra.xc = na.xc;
    ra.mu_best = grow<int64_t>(ctx, ctx->s_mub, Q + 1);
    ra.lamp = s.lamp;
    ra.seed = seed;
    ra.rseed = grow<int2>(ctx, ctx->s_rseed, 3 * (Q + 1));
    sa.rseed = ra.rseed;
    ra.ctrl = s.ctrl;
    ra.slots = slots + nbn * kSecSlotW;
    SecControlArgs ca{s.ctrl, n, 0, nbn + nbr, slots, trace_dev, sa.tpart, S * nbn};
    SecCtrl hc;
    constexpr int64_t kChunk = 16;
    for (int64_t k = 0; k <= max_iters;) {
        for (int64_t j = 0; j < kChunk && k <= max_iters; ++j, ++k) {
            sa.mu = s.mu[k & 1];
            // iteration 0 has no seeds: its scan starts without bounds
            sa.seed = k > 0 ? seed : nullptr;
            na.k = ra.k = ca.k = k;
            na.lam_in = s.lam[k & 1];
            na.lam_out = s.lam[(k + 1) & 1];
            ra.mu_in = s.mu[k & 1];
            ra.mu_out = s.mu[(k + 1) & 1];
            ck(ctx, launch_sec_scan(sa, (int)L, S, st), "sec scan");
            ck(ctx, launch_sec_node(na, (int)L, st), "sec node");
            ck(ctx, launch_sec_rows(ra, st), "sec rows");
            ck(ctx, launch_sec_tiles(s.lamp, n, s.tile_h, st), "sec tiles");
            ck(ctx, launch_sec_control(ca, st), "sec control");
        }
        download(ctx, {{s.ctrl, &hc, sizeof(SecCtrl)}}, st);
        if (hc.done) return hc;
    }
    download(ctx, {{s.ctrl, &hc, sizeof(SecCtrl)}}, st);
    if (!hc.done) fail(ctx, F2M_ERR_DEVICE, "subtour GDP loop ended without a stop");
    return hc;
}

// (Lam*, M*) of a finished loop to the caller's arrays (Lam by label)
void sec_outputs(f2m_ctx *ctx, const SecSetup &s, const SecCtrl &c, int64_t *lam_label, int64_t *mu, hipStream_t st)
{
    const int64_t n = s.gh.g.n, Q = s.nrows;
    const bool last = c.kstar == c.k_last;
    const int64_t *lam = last ? s.lam[c.k_last & 1] : (const int64_t *)ctx->s_lamb.p;
    const int64_t *mm = last ? s.mu[c.k_last & 1] : (const int64_t *)ctx->s_mub.p;
    ck(ctx, launch_unpermute(lam, s.gh.g.orig, n, lam_label, st), "unpermute");
    if (Q > 0) ck(ctx, hipMemcpyAsync(mu, mm, Q * sizeof(int64_t), hipMemcpyDeviceToDevice, st), "copy");
}

// One GDP call; trace to host (optional).  Returns the control block.
SecCtrl sec_gdp(f2m_ctx *ctx, const int32_t *xy, int64_t n, const f2m_sec_rows *rows, int64_t *lam, int64_t *mu,
                int64_t max_iters, int64_t *trace, int64_t trace_cap, bool write_back)
{
    hipStream_t st = ctx->stream;
    if (!trace) trace_cap = 0;
    SecSetup s = sec_setup(ctx, xy, n, rows, lam, mu, max_iters, trace_cap, st);
    int64_t *tdev = trace_cap > 0 ? grow<int64_t>(ctx, ctx->s_trace, trace_cap * kSecTraceW) : nullptr;
    const SecCtrl c = sec_loop(ctx, s, max_iters, tdev, st);
    if (write_back) sec_outputs(ctx, s, c, lam, mu, st);
    const int64_t nrec = std::min<int64_t>(c.k_last + 1, trace_cap);
    if (nrec > 0)
        ck(ctx, hipMemcpyAsync(trace, tdev, nrec * kSecTraceW * sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    return c;
}

// Separation at (Lam, M): components of the support of the trivial x, new
// rows for the violated cuts that are not rows yet (see f2m_sec_separate).
// new_row_host[v]: the new row of v or -1.
void sec_separate(f2m_ctx *ctx, const int32_t *xy, int64_t n, const f2m_sec_rows *rows, const int64_t *lam,
                  const int64_t *mu, std::vector<int32_t> &new_row_host, int64_t *new_rows, int64_t *components)
{
    hipStream_t st = ctx->stream;
    SecSetup s = sec_setup(ctx, xy, n, rows, lam, mu, 0, 0, st);
    int32_t *parent = grow<int32_t>(ctx, ctx->s_parent, n);
    ck(ctx, launch_sec_uf_init(parent, n, st), "uf init");
    SecScanArgs sa{};
    sa.g = s.gh.g;
    sa.col = s.gh.col;
    sa.lamp = s.lamp;
    sa.rowp = s.rowp;
    sa.mu = s.mu[0];
    sa.ctrl = s.ctrl;
    sa.slice_len = sec_shape(n).slice_len;
    sa.tile_h = s.tile_h;
    sa.support = 1;
    sa.parent = parent;
    ck(ctx, launch_sec_scan(sa, s.L, sec_shape(n).slices, st), "sec support");
    ck(ctx, launch_sec_uf_final(parent, n, st), "uf final");
    // components by their smallest label; the given rows' sets
    std::vector<int32_t> comp(n), rof;
    if (s.nlayers > 0) rof.resize((size_t)s.nlayers * n);
    download(ctx, {{parent, comp.data(), n * sizeof(int32_t)}}, st);
    if (s.nlayers > 0)
        ck(ctx, hipMemcpy(rof.data(), rows->row_of, rof.size() * sizeof(int32_t), hipMemcpyDeviceToHost), "copy");
    // a cut is a set and its complement: key it by the side without label 0
    // (size, and the sum of a hash of its labels); equal keys are compared
    // member by member
    auto lab_hash = [](int64_t v) {
        uint64_t z = (uint64_t)(v + 1) * 0x9E3779B97F4A7C15ULL;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        return z ^ (z >> 31);
    };
    uint64_t hall = 0;
    for (int64_t v = 0; v < n; ++v) hall += lab_hash(v);
    struct Cut {
        int64_t size = 0;
        uint64_t h = 0;
        bool has0 = false;
        std::vector<int32_t> mem;   // the given side, sorted
    };
    auto canon = [&](Cut &c) {
        if (c.has0) { c.size = n - c.size; c.h = hall - c.h; }
    };
    auto same_cut = [&](const Cut &a, const Cut &b) {
        if (a.size != b.size || a.h != b.h) return false;
        if (a.has0 == b.has0) return a.mem == b.mem;
        // complements: no common member and the sizes add up to n
        if ((int64_t)(a.mem.size() + b.mem.size()) != n) return false;
        size_t i = 0, j = 0;
        while (i < a.mem.size() && j < b.mem.size()) {
            if (a.mem[i] == b.mem[j]) return false;
            if (a.mem[i] < b.mem[j]) ++i; else ++j;
        }
        return true;
    };
    std::vector<Cut> have(s.nrows);
    for (int64_t l = 0; l < s.nlayers; ++l)
        for (int64_t v = 0; v < n; ++v) {
            const int32_t r = rof[l * n + v];
            if (r >= 0) {
                have[r].mem.push_back((int32_t)v);
                have[r].h += lab_hash(v);
                have[r].has0 = have[r].has0 || v == 0;
            }
        }
    for (Cut &c : have) { c.size = (int64_t)c.mem.size(); canon(c); }
    std::vector<int64_t> csize(n, 0);
    for (int64_t v = 0; v < n; ++v) ++csize[comp[v]];
    int64_t ncomp = 0;
    for (int64_t v = 0; v < n; ++v) ncomp += comp[v] == v ? 1 : 0;
    *components = ncomp;
    new_row_host.assign(n, -1);
    *new_rows = 0;
    if (ncomp <= 1) return;
    std::vector<Cut> fresh;
    std::vector<int32_t> root_row(n, -1);
    std::vector<std::vector<int32_t>> members(n);
    for (int64_t v = 0; v < n; ++v) members[comp[v]].push_back((int32_t)v);
    for (int64_t r = 0; r < n; ++r) {
        if (comp[r] != r) continue;
        const int64_t sz = csize[r];
        if (sz < 2 || sz > n - 2) continue;
        Cut c;
        c.mem = members[r];
        c.size = sz;
        c.h = 0;
        for (int32_t v : c.mem) c.h += lab_hash(v);
        c.has0 = r == 0;   // the root is the smallest label
        canon(c);
        bool dup = false;
        for (const Cut &h : have) dup = dup || same_cut(h, c);
        for (const Cut &h : fresh) dup = dup || same_cut(h, c);
        if (dup) continue;
        root_row[r] = (int32_t)(s.nrows + (int64_t)fresh.size());
        fresh.push_back(std::move(c));
    }
    for (int64_t v = 0; v < n; ++v) new_row_host[v] = root_row[comp[v]];
    *new_rows = (int64_t)fresh.size();
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void f2m_opts_default(f2m_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(f2m_opts);
    o->rule_version = 1;
    o->graph = F2M_GRAPH_COMPLETE;
    o->warm = F2M_WARM_COLD;
    o->max_iters = 100000;
    o->handoff_div = 50;
    o->knn_k = 10;
    o->finish = F2M_FINISH_EXACT;
}

f2m_status f2m_create(f2m_ctx **out, int device, const f2m_opts *defaults)
{
    if (!out) return F2M_ERR_ARG;
    *out = nullptr;
    if (defaults && defaults->struct_size != sizeof(f2m_opts)) return F2M_ERR_ARG;
    f2m_ctx *ctx = new (std::nothrow) f2m_ctx();
    if (!ctx) return F2M_ERR_NOMEM;
    ctx->device = device;
    if (defaults) ctx->defaults = *defaults;
    else f2m_opts_default(&ctx->defaults);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        delete ctx;
        return F2M_ERR_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->device_name = prop.name;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void **)&ctx->ctrl_host, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->scratch_host, 16 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->up_done, hipEventDisableTiming) != hipSuccess) {
        f2m_destroy(ctx);
        return F2M_ERR_DEVICE;
    }
    // the no-alloc workspace's device address, looked up once per device
    // with the device current (a failure only disables f2m_gdp_step_noalloc)
    ctx->noalloc_err = noalloc_scratch(device, &ctx->noalloc);
    *out = ctx;
    return F2M_OK;
}

void f2m_destroy(f2m_ctx *ctx)
{
    if (!ctx) return;
    for (f2m_ctx *w : ctx->workers) f2m_destroy(w);
    ctx->workers.clear();
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (DevBuf *b : ctx->bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->ctrl_host) (void)hipHostFree(ctx->ctrl_host);
    if (ctx->scratch_host) (void)hipHostFree(ctx->scratch_host);
    for (HostBuf *h : {&ctx->h_keys, &ctx->h_costs, &ctx->h_neg, &ctx->h_start, &ctx->h_inc, &ctx->h_xyp, &ctx->h_lamp,
                       &ctx->h_up, &ctx->h_down, &ctx->h_progress})
        if (h->p) (void)hipHostFree(h->p);
    if (ctx->fwork) finish_work_destroy(ctx->fwork);
    if (ctx->up_done) (void)hipEventDestroy(ctx->up_done);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

void f2m_result_free(f2m_result *r)
{
    if (!r) return;
    std::free(r->lambda2);
    std::free(r->lambda2_gdp);
    std::free(r->lambda2_last);
    std::free(r->edge_u);
    std::free(r->edge_v);
    std::free(r->edge_x2);
    std::free(r->trace);
    std::free(r->scan_kind);
    std::memset(r, 0, sizeof(*r));
}

const char *f2m_status_str(f2m_status s)
{
    switch (s) {
    case F2M_OK: return "ok";
    case F2M_NOT_CERTIFIED: return "not certified";
    case F2M_ERR_ARG: return "invalid argument";
    case F2M_ERR_RANGE: return "coordinate span out of range";
    case F2M_ERR_INFEASIBLE: return "infeasible (n < 3)";
    case F2M_ERR_NOMEM: return "out of memory";
    case F2M_ERR_DEVICE: return "device error";
    case F2M_ERR_CAPACITY: return "buffer too small";
    case F2M_ERR_OVERFLOW: return "multiplier overflow";
    }
    return "unknown status";
}

const char *f2m_last_error(const f2m_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

const char *f2m_device_name(const f2m_ctx *ctx) { return ctx ? ctx->device_name.c_str() : ""; }

f2m_status f2m_gdp_step(f2m_ctx *ctx, const int32_t *xy, int64_t n, const int64_t *lam_in, int64_t *lam_out,
                        int64_t *z4_out, int32_t *i4_out, int32_t *neg, int32_t *zero, int64_t *step,
                        int64_t rec[F2M_TRACE_W])
{
    if (!ctx) return F2M_ERR_ARG;
    ctx->dev_cap = (size_t)ctx->defaults.max_device_bytes;
    try {
        if (!xy || !lam_in || !lam_out || !rec || n < 4 || lam_in == lam_out)
            fail(ctx, F2M_ERR_ARG, "gdp_step needs n >= 4, coords, distinct lambda2_in/out and rec");
        if (n >= (int64_t)1 << 30) fail(ctx, F2M_ERR_ARG, "n must be below 2^30");
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        const ScanShape sh = scan_shape(n, true);
        StepBufs b;
        b.m4 = grow<int32_t>(ctx, ctx->minmax, 4);
        b.geo = GeoBufs{grow<int32_t>(ctx, ctx->orig, n), grow<int32_t>(ctx, ctx->pos, n),
                        grow<float4>(ctx, ctx->col, n), grow<float4>(ctx, ctx->box, ntiles_of(n) * kBoxStride),
                        grow<float>(ctx, ctx->xy2max, 1)};
        b.sort = grow_sort(ctx, n);
        b.ls = grow<int64_t>(ctx, ctx->lam[0], n);
        b.lo = grow<int64_t>(ctx, ctx->lam[1], n);
        b.best = grow<int64_t>(ctx, ctx->lam_best, n);
        b.thm = grow<float>(ctx, ctx->tile_hmax, ntiles_of(n) * kBoxStride);
        b.pz = grow<int64_t>(ctx, ctx->pz, sh.slices * kTop * n);
        b.pi = grow<int32_t>(ctx, ctx->pi, sh.slices * kTop * n);
        b.pneg = grow<int32_t>(ctx, ctx->pneg, sh.slices * n);
        b.pzero = grow<int32_t>(ctx, ctx->pzero, sh.slices * n);
        b.prn = grow<int64_t>(ctx, ctx->prowneg, sh.slices * n);
        b.z4 = z4_out ? z4_out : grow<int64_t>(ctx, ctx->z4, kTop * n);
        b.i4 = i4_out ? i4_out : grow<int32_t>(ctx, ctx->i4, kTop * n);
        b.seed = grow<int32_t>(ctx, ctx->seed, kTop * n);
        b.cd = grow<Ctrl>(ctx, ctx->ctrl, 1);
        b.trace = grow<int64_t>(ctx, ctx->trace, kTraceW);
        b.slots = grow<unsigned long long>(ctx, ctx->slots, (int64_t)kSlotW * ntiles_of(n));
        gdp_step_run(ctx, xy, n, lam_in, lam_out, neg, zero, step, rec, b);
        return F2M_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}

f2m_status f2m_gdp_step_noalloc(f2m_ctx *ctx, const int32_t *xy, int64_t n, const int64_t *lam_in,
                                int64_t *lam_out, int64_t *z4_out, int32_t *i4_out, int32_t *neg, int32_t *zero,
                                int64_t *step, int64_t rec[F2M_TRACE_W])
{
    if (!ctx) return F2M_ERR_ARG;
    try {
        if (!xy || !lam_in || !lam_out || !rec || n < 4 || lam_in == lam_out)
            fail(ctx, F2M_ERR_ARG, "gdp_step_noalloc needs n >= 4, coords, distinct lambda2_in/out and rec");
        if (n > F2M_NOALLOC_MAX_N)
            fail(ctx, F2M_ERR_CAPACITY, "gdp_step_noalloc: n = " + std::to_string(n) + " is above its maximum " +
                                            std::to_string((long long)F2M_NOALLOC_MAX_N));
        if (!ctx->noalloc)
            fail(ctx, F2M_ERR_DEVICE, std::string("gdp_step_noalloc: no device workspace: ") +
                                          hipGetErrorString(ctx->noalloc_err));
        const size_t need = carve_step(nullptr, n, !z4_out, !i4_out, nullptr);
        if (need > kNoAllocBytes)
            fail(ctx, F2M_ERR_CAPACITY, "gdp_step_noalloc: n = " + std::to_string(n) + " needs " +
                                            std::to_string(need) + " bytes of workspace, " +
                                            std::to_string(kNoAllocBytes) + " exist");
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        StepBufs b;
        carve_step(static_cast<char *>(ctx->noalloc), n, !z4_out, !i4_out, &b);
        if (z4_out) b.z4 = z4_out;
        if (i4_out) b.i4 = i4_out;
        gdp_step_run(ctx, xy, n, lam_in, lam_out, neg, zero, step, rec, b);
        return F2M_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}

#define F2M_GUARD_BEGIN \
    if (!ctx) return F2M_ERR_ARG; \
    ctx->dev_cap = (size_t)ctx->defaults.max_device_bytes; \
    try {
#define F2M_GUARD_END \
    } catch (const Fail &f) { \
        return f.st; \
    } catch (const std::bad_alloc &) { \
        ctx->err = "host allocation failed"; \
        return F2M_ERR_NOMEM; \
    }

f2m_status f2m_features(f2m_ctx *ctx, const int32_t *xy, int64_t n, uint16_t *feat, float *scale)
{
    F2M_GUARD_BEGIN
    if (!xy || !feat || !scale) fail(ctx, F2M_ERR_ARG, "features need coords, feat and scale");
    ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t st = ctx->stream;
    const GeoHost gh = setup_geo(ctx, xy, n, st);
    float *sd = grow<float>(ctx, ctx->m_scale, 1);
    features_dev(ctx, gh, feat, sd, st);
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, sd, sizeof(float), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    std::memcpy(scale, ctx->scratch_host, sizeof(float));
    return F2M_OK;
    F2M_GUARD_END
}

f2m_status f2m_mlp_forward(f2m_ctx *ctx, const float *theta, const uint16_t *feat, int64_t n, float *y)
{
    F2M_GUARD_BEGIN
    if (!theta || !feat || !y || n < 1) fail(ctx, F2M_ERR_ARG, "mlp_forward needs theta, feat, y and n >= 1");
    ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    mlp_forward_dev(ctx, theta, feat, n, y, ctx->stream);
    ck(ctx, hipStreamSynchronize(ctx->stream), "sync");
    return F2M_OK;
    F2M_GUARD_END
}

f2m_status f2m_mlp_grad(f2m_ctx *ctx, const float *theta, const uint16_t *feat, const float *target, int64_t n,
                        float *grad, double *loss)
{
    F2M_GUARD_BEGIN
    if (!theta || !feat || !target || !grad || !loss || n < 1) fail(ctx, F2M_ERR_ARG, "mlp_grad needs every array");
    ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    mlp_grad_dev(ctx, theta, feat, target, n, grad, loss, ctx->stream);
    return F2M_OK;
    F2M_GUARD_END
}

f2m_status f2m_mlp_adamw(f2m_ctx *ctx, float *theta, const float *grad, float *m, float *v, int64_t step, float lr,
                         float wd)
{
    F2M_GUARD_BEGIN
    if (!theta || !grad || !m || !v || step < 1) fail(ctx, F2M_ERR_ARG, "mlp_adamw needs every array and step >= 1");
    ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ck(ctx, launch_adamw(theta, grad, m, v, kMlpParams, lr, 0.9f, 0.999f, 1e-8f, wd, step, ctx->stream), "adamw");
    ck(ctx, hipStreamSynchronize(ctx->stream), "sync");
    return F2M_OK;
    F2M_GUARD_END
}

f2m_status f2m_knn_graph(f2m_ctx *ctx, const int32_t *xy, int64_t n, int32_t k, int32_t *rowptr, int32_t *col,
                         int64_t cap, int64_t *nnz)
{
    if (!ctx) return F2M_ERR_ARG;
    ctx->dev_cap = (size_t)ctx->defaults.max_device_bytes;
    try {
        if (!xy || !rowptr || !col || !nnz || cap < 0) fail(ctx, F2M_ERR_ARG, "knn_graph needs coords and outputs");
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        hipStream_t st = ctx->stream;
        const GeoHost gh = setup_geo(ctx, xy, n, st);
        const Csr csr = build_graph(ctx, gh, k, st);
        *nnz = csr.nnz;
        if (cap < csr.nnz) fail(ctx, F2M_ERR_CAPACITY, "col capacity below the entry count");
        int32_t *deg = grow<int32_t>(ctx, ctx->c_deg, n + 1);
        ck(ctx, launch_csr_to_labels(gh.g, csr, rowptr, col, deg, st), "csr_to_labels");
        ck(ctx, hipStreamSynchronize(st), "sync");
        return F2M_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}

f2m_status f2m_certify(f2m_ctx *ctx, const int32_t *xy, int64_t n, const int64_t *lam, int64_t m,
                       const int32_t *eu, const int32_t *ev, const uint8_t *ex2, int64_t out[4])
{
    if (!ctx) return F2M_ERR_ARG;
    ctx->dev_cap = (size_t)ctx->defaults.max_device_bytes;
    try {
        if (!xy || !lam || !out || n < 3 || m < 0 || (m > 0 && (!eu || !ev || !ex2)))
            fail(ctx, F2M_ERR_ARG, "certify needs n >= 3, coords, lambda2 and the edge arrays");
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        const GeoHost gh = setup_geo(ctx, xy, n, ctx->stream);
        certify_dev(ctx, gh, lam, m, eu, ev, ex2, ctx->stream, out);
        return F2M_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}

f2m_status f2m_solve(f2m_ctx *ctx, const int32_t *coords, int64_t n, const f2m_opts *opts, f2m_result *out)
{
    if (!ctx) return F2M_ERR_ARG;
    f2m_result res;
    std::memset(&res, 0, sizeof(res));
    try {
        f2m_opts o = call_opts(ctx, opts);
        if (!coords || !out) fail(ctx, F2M_ERR_ARG, "null coords or result");
        if (o.rule_version != 1) fail(ctx, F2M_ERR_ARG, "only rule_version 1 exists");
        if (o.graph != F2M_GRAPH_COMPLETE && o.graph != F2M_GRAPH_KNN) fail(ctx, F2M_ERR_ARG, "unknown graph kind");
        const bool on_graph = o.graph == F2M_GRAPH_KNN;
        if (o.max_iters < 0) fail(ctx, F2M_ERR_ARG, "max_iters < 0");
        if (o.handoff_div < 0) fail(ctx, F2M_ERR_ARG, "handoff_div < 0");
        if (o.scan_rows != 0 && o.scan_rows != 1 && o.scan_rows != 2 && o.scan_rows != 4)
            fail(ctx, F2M_ERR_ARG, "scan_rows must be 0, 1, 2 or 4");
        if (o.scan_slices < 0) fail(ctx, F2M_ERR_ARG, "scan_slices < 0");
        if (o.warm == F2M_WARM_USER && !o.lambda2_init) fail(ctx, F2M_ERR_ARG, "warm start without lambda2_init");
        if (o.tuner_cache && o.scan_rows == 0 && o.scan_slices == 0 && !on_graph) {
            const Tuned tu = tuner_lookup(ctx, o.tuner_cache, o.scan_mode == F2M_SCAN_FULL ? "full" : "culled", n);
            if (tu.found) {
                o.scan_rows = tu.rows;
                o.scan_slices = tu.slices;
                if (o.chunk == 0) o.chunk = tu.chunk;
            }
        }
        const CtrlStart cs = resume_start(ctx, o);
        if (o.warm != F2M_WARM_COLD && o.warm != F2M_WARM_USER && o.warm != F2M_WARM_MLP &&
            o.warm != F2M_WARM_GRAPH)
            fail(ctx, F2M_ERR_ARG, "unknown warm mode");
        if (o.warm == F2M_WARM_GRAPH && on_graph) fail(ctx, F2M_ERR_ARG, "the graph warm start is for the complete graph");
        if (o.warm == F2M_WARM_MLP && !o.mlp_theta) fail(ctx, F2M_ERR_ARG, "warm start without mlp_theta");
        if (n < 3) fail(ctx, F2M_ERR_INFEASIBLE, "F2M needs n >= 3");
        if (n >= (int64_t)1 << 30) fail(ctx, F2M_ERR_ARG, "n must be below 2^30");
        if (o.degree_b) {
            if (n < 4) fail(ctx, F2M_ERR_ARG, "degree_b needs n >= 4");
            if (o.warm == F2M_WARM_MLP || o.warm == F2M_WARM_GRAPH)
                fail(ctx, F2M_ERR_ARG, "degree_b takes a cold or a user warm start");
            for (int64_t v = 0; v < n; ++v)
                if (o.degree_b[v] < 1 || o.degree_b[v] > 3) fail(ctx, F2M_ERR_ARG, "degree_b entries must be 1, 2 or 3");
        }
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        hipStream_t st = pick_stream(ctx, &o);
        const double t0 = now_s();

        // coordinates on the device and on the host (the finish and n == 3 need them)
        std::vector<int32_t> xy_host(2 * n);
        const int32_t *xy_dev;
        if (o.coords_on_device) {
            xy_dev = coords;
            ck(ctx, hipMemcpyAsync(xy_host.data(), coords, 2 * n * sizeof(int32_t), hipMemcpyDeviceToHost, st),
               "copy");
            ck(ctx, hipStreamSynchronize(st), "sync");
        } else {
            std::memcpy(xy_host.data(), coords, 2 * n * sizeof(int32_t));
            int32_t *d = grow<int32_t>(ctx, ctx->xy, 2 * n);
            ck(ctx, hipMemcpyAsync(d, coords, 2 * n * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy");
            xy_dev = d;
        }
        if (n == 3) {
            int64_t mn[2] = {xy_host[0], xy_host[1]}, mx[2] = {xy_host[0], xy_host[1]};
            for (int i = 1; i < 3; ++i)
                for (int a = 0; a < 2; ++a) {
                    mn[a] = std::min<int64_t>(mn[a], xy_host[2 * i + a]);
                    mx[a] = std::max<int64_t>(mx[a], xy_host[2 * i + a]);
                }
            if (mx[0] - mn[0] >= (1 << 20) || mx[1] - mn[1] >= (1 << 20))
                fail(ctx, F2M_ERR_RANGE, "coordinate span must be below 2^20 on each axis");
            f2m_status s = solve_n3(ctx, xy_host.data(), &res);
            res.seconds[5] = now_s() - t0;
            *out = res;
            return s;
        }
        GeoHost gh = setup_geo(ctx, xy_dev, n, st);
        const int8_t *b_label_dev = nullptr;
        if (o.degree_b) {
            // the rows' right-hand sides b_v (Sec. 3) by label, then by position
            std::vector<int8_t> b8(o.degree_b, o.degree_b + n);
            int8_t *bl = grow<int8_t>(ctx, ctx->deg_label, n);
            int8_t *bp = grow<int8_t>(ctx, ctx->deg_pos, n);
            upload(ctx, {{b8.data(), bl, (size_t)n}}, st);
            ck(ctx, launch_b_to_positions(bl, gh.g.orig, n, bp, st), "b_to_positions");
            gh.g.b = bp;
            b_label_dev = bl;
        }
        const int64_t *lam0_dev = nullptr;
        if (o.warm == F2M_WARM_USER) {
            int64_t *d = grow<int64_t>(ctx, ctx->c_lam_label, n);
            ck(ctx, hipMemcpyAsync(d, o.lambda2_init, n * sizeof(int64_t), hipMemcpyHostToDevice, st), "copy");
            lam0_dev = d;
        }
        Csr csr{};
        if (on_graph) {
            csr = build_graph(ctx, gh, o.knn_k, st);
            res.graph_nnz = csr.nnz;
        }
        const double tw = now_s();
        bool keep_seeds = false;
        if (o.warm == F2M_WARM_MLP) {
            lam0_dev = mlp_lam0_dev(ctx, gh, o.mlp_theta, st);
            ck(ctx, hipStreamSynchronize(st), "sync");
        } else if (o.warm == F2M_WARM_GRAPH && n > o.knn_k) {
            // cold GDP on the candidate graph; its Lam* and final four
            // smallest start the complete-graph GDP
            const Csr wcsr = build_graph(ctx, gh, o.knn_k, st);
            res.graph_nnz = wcsr.nnz;
            const LoopOut wl = gdp_loop(ctx, gh, nullptr, o.max_iters, o.handoff_div, o.chunk, false, false, true,
                                        &wcsr, 0, 0, st);
            int64_t *l = grow<int64_t>(ctx, ctx->m_lam0, n);
            ck(ctx, launch_unpermute(wl.lam_star, gh.g.orig, n, l, st), "unpermute");
            ck(ctx, launch_seed_from_top(static_cast<const int32_t *>(ctx->i4.p), gh.g.orig, gh.g.pos, n,
                                         static_cast<int32_t *>(ctx->seed.p), st), "seed");
            res.warm_iterations = wl.c.k_last + 1;
            lam0_dev = l;
            keep_seeds = true;
        }
        const double t1 = now_s();
        res.seconds[1] = t1 - tw;
        LoopOut lo = gdp_loop(ctx, gh, lam0_dev, o.max_iters, o.handoff_div, o.chunk, o.record_trace != 0,
                              o.time_kernels != 0, o.scan_mode != F2M_SCAN_FULL, on_graph ? &csr : nullptr,
                              o.scan_rows, o.scan_slices, st, keep_seeds, cs);
        const double t2 = now_s();
        InstanceState is{gh, lo.c, lo.lam_star, static_cast<const int64_t *>(ctx->z4.p),
                         static_cast<const int32_t *>(ctx->i4.p), static_cast<const int32_t *>(ctx->seed.p),
                         o.record_trace ? static_cast<const int64_t *>(ctx->trace.p) : nullptr,
                         on_graph ? &csr : nullptr,
                         (o.record_trace && !on_graph) ? static_cast<const int32_t *>(ctx->kinds.p) : nullptr,
                         lo.lam_last, b_label_dev};
        complete_result(ctx, is, o, st, res);
        res.scan_ms = lo.scan_ms;
        res.update_ms = lo.update_ms;
        res.scan_launches = lo.scan_launches;
        for (int q = 0; q < 3; ++q) {
            res.scan_ms_kind[q] = lo.ms_kind[q];
            res.scan_launches_kind[q] = lo.launches_kind[q];
            res.update_ms_kind[q] = lo.update_ms_kind[q];
            res.scan_pairs_kind[q] = (int64_t)lo.c.pairs_kind[q];
        }
        res.scan_rows = lo.shape.rows;
        res.scan_slices = lo.shape.slices;
        res.seconds[0] = tw - t0;
        res.seconds[2] = t2 - t1;
        res.seconds[5] = now_s() - t0;
        *out = res;
        return res.certified ? F2M_OK : F2M_NOT_CERTIFIED;
    } catch (const Fail &f) {
        f2m_result_free(&res);
        return f.st;
    } catch (const std::bad_alloc &) {
        f2m_result_free(&res);
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}


f2m_status f2m_solve_batch(f2m_ctx *ctx, const int32_t *coords, const int64_t *offsets, int32_t n_inst,
                           const f2m_opts *opts, f2m_result *outs)
{
    if (!ctx) return F2M_ERR_ARG;
    std::vector<f2m_result> res;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct GraphGuard {
        hipGraph_t &g;
        hipGraphExec_t &e;
        ~GraphGuard()
        {
            if (e) (void)hipGraphExecDestroy(e);
            if (g) (void)hipGraphDestroy(g);
        }
    } gguard{graph, exec};
    try {
        f2m_opts o = call_opts(ctx, opts);
        if (!coords || !offsets || !outs || n_inst <= 0) fail(ctx, F2M_ERR_ARG, "null inputs or no instances");
        if (o.rule_version != 1) fail(ctx, F2M_ERR_ARG, "only rule_version 1 exists");
        if (o.graph != F2M_GRAPH_COMPLETE) fail(ctx, F2M_ERR_ARG, "batched solves run on the complete graph");
        if (o.coords_on_device) fail(ctx, F2M_ERR_ARG, "batched solves take host coordinates");
        if (o.max_iters < 0 || o.handoff_div < 0) fail(ctx, F2M_ERR_ARG, "bad max_iters or handoff_div");
        if (o.warm != F2M_WARM_COLD && !(o.warm == F2M_WARM_USER && o.lambda2_init))
            fail(ctx, F2M_ERR_ARG, "bad warm start");
        const CtrlStart cs = resume_start(ctx, o);
        if (offsets[0] != 0) fail(ctx, F2M_ERR_ARG, "offsets[0] must be 0");
        if (o.degree_b) fail(ctx, F2M_ERR_ARG, "the batched solve takes no degree_b");
        for (int32_t i = 0; i < n_inst; ++i) {
            if (offsets[i + 1] - offsets[i] < 3) fail(ctx, F2M_ERR_INFEASIBLE, "every instance needs n >= 3");
            if (offsets[i + 1] - offsets[i] >= (int64_t)1 << 30) fail(ctx, F2M_ERR_ARG, "instance too large");
        }
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        hipStream_t st = pick_stream(ctx, &o);
        const double t0 = now_s();
        res.assign(n_inst, f2m_result{});
        const int64_t total = offsets[n_inst];
        const bool cull = o.scan_mode != F2M_SCAN_FULL;
        if (o.tuner_cache && o.scan_slices == 0) {
            // batch entries are keyed by the batch's total node count
            const Tuned tu = tuner_lookup(ctx, o.tuner_cache, cull ? "batch-culled" : "batch-full", total);
            if (tu.found) {
                o.scan_slices = tu.slices;
                if (o.chunk == 0) o.chunk = tu.chunk;
            }
        }

        // layout: positions and tiles 256-aligned per instance
        std::vector<int64_t> P(n_inst + 1, 0), T(n_inst + 1, 0), PZ(n_inst + 1, 0), PS(n_inst + 1, 0);
        std::vector<ScanShape> shp(n_inst);
        std::vector<int32_t> cxs(n_inst), cys(n_inst), mnx(n_inst), mny(n_inst);
        std::vector<int> active;   // instances with n >= 4
        for (int32_t i = 0; i < n_inst; ++i) {
            const int64_t n = offsets[i + 1] - offsets[i];
            const int32_t *xy = coords + 2 * offsets[i];
            int64_t lo[2] = {xy[0], xy[1]}, hi[2] = {xy[0], xy[1]};
            for (int64_t v = 1; v < n; ++v)
                for (int a = 0; a < 2; ++a) {
                    lo[a] = std::min<int64_t>(lo[a], xy[2 * v + a]);
                    hi[a] = std::max<int64_t>(hi[a], xy[2 * v + a]);
                }
            if (hi[0] - lo[0] >= (1 << 20) || hi[1] - lo[1] >= (1 << 20))
                fail(ctx, F2M_ERR_RANGE, "coordinate span must be below 2^20 on each axis");
            mnx[i] = (int32_t)lo[0]; mny[i] = (int32_t)lo[1];
            cxs[i] = (int32_t)((lo[0] + hi[0]) >> 1); cys[i] = (int32_t)((lo[1] + hi[1]) >> 1);
            const int64_t nt = ntiles_of(n);
            // one row per lane for the whole launch; the batch itself fills
            // the GPU, so culled scans take one slice and full scans a few
            shp[i].rows = 1;
            const int64_t sl = o.scan_slices > 0 ? std::min<int64_t>(nt, o.scan_slices)
                                                 : (cull ? 1 : std::min<int64_t>(nt, 4));
            shp[i].slice_len = ((nt + sl - 1) / sl) * kTileCols;
            shp[i].slices = (n + shp[i].slice_len - 1) / shp[i].slice_len;
            P[i + 1] = P[i] + nt * kTileCols;
            T[i + 1] = T[i] + nt * kBoxStride;   // box and tile-maximum slots
            PZ[i + 1] = PZ[i] + shp[i].slices * n;
            if (n >= 4) active.push_back(i);
        }
        const int64_t trace_cap = o.record_trace ? std::min<int64_t>(o.max_iters + 1 - cs.k0, 8192) : 0;

        // pools
        int32_t *xy = grow<int32_t>(ctx, ctx->b_xy, 2 * total);
        int32_t *orig = grow<int32_t>(ctx, ctx->b_orig, P[n_inst]);
        int32_t *pos = grow<int32_t>(ctx, ctx->b_pos, total);
        float4 *col = grow<float4>(ctx, ctx->b_col, P[n_inst]);
        float4 *box = grow<float4>(ctx, ctx->b_box, T[n_inst]);
        float *x2m = grow<float>(ctx, ctx->b_x2m, n_inst);
        int64_t *lam0 = grow<int64_t>(ctx, ctx->b_lam0, P[n_inst]);
        int64_t *lam1 = grow<int64_t>(ctx, ctx->b_lam1, P[n_inst]);
        int64_t *best = grow<int64_t>(ctx, ctx->b_best, P[n_inst]);
        int64_t *lamlabel = grow<int64_t>(ctx, ctx->b_lamlabel, total);
        float *thm = grow<float>(ctx, ctx->b_thm, T[n_inst]);
        int64_t *pz = grow<int64_t>(ctx, ctx->b_pz, kTop * PZ[n_inst]);
        int32_t *pi = grow<int32_t>(ctx, ctx->b_pi, kTop * PZ[n_inst]);
        int32_t *pneg = grow<int32_t>(ctx, ctx->b_pneg, PZ[n_inst]);
        int32_t *pzero = grow<int32_t>(ctx, ctx->b_pzero, PZ[n_inst]);
        int64_t *prn = grow<int64_t>(ctx, ctx->b_prn, PZ[n_inst]);
        int64_t *z4 = grow<int64_t>(ctx, ctx->b_z4, kTop * total);
        int32_t *i4 = grow<int32_t>(ctx, ctx->b_i4, kTop * total);
        int32_t *seed = grow<int32_t>(ctx, ctx->b_seed, kTop * total);
        Ctrl *ctrl = grow<Ctrl>(ctx, ctx->b_ctrl, n_inst);
        int64_t *trace = trace_cap ? grow<int64_t>(ctx, ctx->b_trace, (int64_t)n_inst * trace_cap * kTraceW) : nullptr;
        int64_t *nblk = grow<int64_t>(ctx, ctx->b_nblk, n_inst);
        int32_t *act = grow<int32_t>(ctx, ctx->b_active, 1);
        unsigned long long *bslots = grow<unsigned long long>(ctx, ctx->b_slots, (int64_t)kSlotW * (T[n_inst] / kBoxStride));

        ck(ctx, hipMemcpyAsync(xy, coords, 2 * total * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy");
        if (o.warm == F2M_WARM_USER)
            ck(ctx, hipMemcpyAsync(lamlabel, o.lambda2_init, total * sizeof(int64_t), hipMemcpyHostToDevice, st), "copy");
        else
            ck(ctx, hipMemsetAsync(lamlabel, 0, total * sizeof(int64_t), st), "memset");
        std::vector<int64_t> nb_host(n_inst, 0);
        for (int32_t i : active) {
            const int64_t n = offsets[i + 1] - offsets[i], X = offsets[i];
            GeoBufs b{orig + P[i], pos + X, col + P[i], box + T[i], x2m + i};
            enqueue_geo(ctx, xy + 2 * X, n, mnx[i], mny[i], cxs[i], cys[i], b, st);
            ck(ctx, launch_ctrl_init(ctrl + i, o.max_iters, trace_cap, o.handoff_div, cs, st), "ctrl_init");
            ck(ctx, launch_set_lam(lamlabel + X, orig + P[i], n, ((cs.k0 & 1) ? lam1 : lam0) + P[i], col + P[i],
                                   thm + T[i], ctrl + i, st),
               "set_lam");
            ck(ctx, launch_seed_neighbours(n, col + P[i], seed + kTop * X, st), "seed");
            nb_host[i] = ntiles_of(n);
        }
        ck(ctx, hipMemcpyAsync(nblk, nb_host.data(), n_inst * sizeof(int64_t), hipMemcpyHostToDevice, st), "copy");
        ck(ctx, launch_ctrl_nblocks(ctrl, nblk, n_inst, st), "nblocks");
        std::vector<float> x2h(n_inst);
        std::vector<Ctrl> ch(n_inst);
        ck(ctx, hipMemcpyAsync(x2h.data(), x2m, n_inst * sizeof(float), hipMemcpyDeviceToHost, st), "copy");
        ck(ctx, hipMemcpyAsync(ch.data(), ctrl, n_inst * sizeof(Ctrl), hipMemcpyDeviceToHost, st), "copy");
        ck(ctx, hipStreamSynchronize(st), "sync");
        for (int32_t i : active)
            if (ch[i].maxabs_lam >= kLamLimit) fail(ctx, F2M_ERR_OVERFLOW, "|lambda2_init| must be below 2^38");

        // per-instance argument tables and work items
        std::vector<ScanArgs> sa(n_inst);
        std::vector<UpdateArgs> ua(n_inst);
        std::vector<BatchScanItem> sitems;
        std::vector<BatchTileItem> uitems;
        // longest processing time first: larger instances' blocks launch first
        std::vector<int> order(active);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
        });
        for (int32_t i : order) {
            const int64_t n = offsets[i + 1] - offsets[i], X = offsets[i];
            const Geo g{n, orig + P[i], pos + X, box + T[i], x2h[i]};
            ScanArgs &a = sa[i];
            a = ScanArgs{};
            a.g = g;
            a.lv = LamView{col + P[i], lam0 + P[i], thm + T[i], ctrl + i};
            a.lam_odd = lam1 + P[i];
            a.slice_len = shp[i].slice_len;
            a.cull = cull ? 1 : 0;
            a.interleave = cull ? shp[i].slices : 0;
            a.check_done = 1;
            a.tested = &ctrl[i].pairs_tested;
            a.seed = seed + kTop * X;
            a.pz = pz + kTop * PZ[i]; a.pi = pi + kTop * PZ[i];
            a.pneg = pneg + PZ[i]; a.pzero = pzero + PZ[i]; a.prowneg = prn + PZ[i];
            ua[i] = UpdateArgs{g, shp[i].slices, 0, a.pz, a.pi, a.pneg, a.pzero, a.prowneg, lam0 + P[i], lam1 + P[i],
                               best + P[i], col + P[i], thm + T[i], z4 + kTop * X, i4 + kTop * X, seed + kTop * X,
                               nullptr, nullptr, nullptr, ctrl + i,
                               trace ? trace + (int64_t)i * trace_cap * kTraceW : nullptr};
            ua[i].slots = bslots + (int64_t)kSlotW * (T[i] / kBoxStride);
            const int64_t rb = ntiles_of(n);
            for (int64_t r = 0; r < rb; ++r)
                for (int64_t sl = 0; sl < shp[i].slices; ++sl)
                    sitems.push_back(BatchScanItem{i, (int32_t)r, (int32_t)sl, 0});
            for (int64_t b = 0; b < rb; ++b) uitems.push_back(BatchTileItem{i, (int32_t)b});
        }
        ScanArgs *sa_d = grow<ScanArgs>(ctx, ctx->b_sargs, n_inst);
        UpdateArgs *ua_d = grow<UpdateArgs>(ctx, ctx->b_uargs, n_inst);
        BatchScanItem *si_d = grow<BatchScanItem>(ctx, ctx->b_sitems, std::max<size_t>(sitems.size(), 1));
        BatchTileItem *ui_d = grow<BatchTileItem>(ctx, ctx->b_uitems, std::max<size_t>(uitems.size(), 1));
        ck(ctx, hipMemcpyAsync(sa_d, sa.data(), n_inst * sizeof(ScanArgs), hipMemcpyHostToDevice, st), "copy");
        ck(ctx, hipMemcpyAsync(ua_d, ua.data(), n_inst * sizeof(UpdateArgs), hipMemcpyHostToDevice, st), "copy");
        if (!sitems.empty()) {
            ck(ctx, hipMemcpyAsync(si_d, sitems.data(), sitems.size() * sizeof(BatchScanItem), hipMemcpyHostToDevice, st),
               "copy");
            ck(ctx, hipMemcpyAsync(ui_d, uitems.data(), uitems.size() * sizeof(BatchTileItem), hipMemcpyHostToDevice, st),
               "copy");
        }
        ck(ctx, hipStreamSynchronize(st), "sync");
        const double t1 = now_s();

        // the loop: a chunk of iterations captured once as a graph and
        // replayed until every instance has stopped
        if (!active.empty()) {
            const int chunk = o.chunk > 0 ? 2 * ((o.chunk + 1) / 2) : 8;
            ck(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            for (int j = 0; j < chunk; ++j) {
                hipError_t e1 = launch_scan_batch(sa_d, si_d, (int64_t)sitems.size(), 1, cull, st);
                hipError_t e2 = launch_update_batch(ua_d, ui_d, (int64_t)uitems.size(), st);
                hipError_t e3 = e2 == hipSuccess ? launch_control_batch(ua_d, n_inst, st) : e2;
                if (e1 != hipSuccess || e3 != hipSuccess) {
                    hipGraph_t g2 = nullptr;
                    (void)hipStreamEndCapture(st, &g2);
                    if (g2) (void)hipGraphDestroy(g2);
                    ck(ctx, e1 != hipSuccess ? e1 : e3, "batched launch");
                }
            }
            ck(ctx, hipStreamEndCapture(st, &graph), "hipStreamEndCapture");
            ck(ctx, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
            const int64_t max_replays = (o.max_iters - cs.k0) / chunk + 2;
            int64_t replays = 0;
            for (;;) {
                ck(ctx, hipGraphLaunch(exec, st), "hipGraphLaunch");
                ++replays;
                ck(ctx, launch_count_active(ctrl, n_inst, act, st), "count_active");
                ck(ctx, hipMemcpyAsync(ctx->scratch_host, act, sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
                ck(ctx, hipStreamSynchronize(st), "sync");
                int32_t left;
                std::memcpy(&left, ctx->scratch_host, sizeof(int32_t));
                // instances of n = 3 never start: count only the others
                int32_t idle = 0;
                for (int32_t i = 0; i < n_inst; ++i) idle += (offsets[i + 1] - offsets[i] < 4) ? 1 : 0;
                if (left - idle <= 0) break;
                if (replays > max_replays) fail(ctx, F2M_ERR_DEVICE, "batched GDP loop passed the cap");
            }
        }
        const double t2 = now_s();
        ck(ctx, hipMemcpyAsync(ch.data(), ctrl, n_inst * sizeof(Ctrl), hipMemcpyDeviceToHost, st), "copy");
        ck(ctx, hipStreamSynchronize(st), "sync");

        // per-instance finish and certificate: independent instances, so
        // host threads take them largest first, each with its own context
        // (stream, workspaces); every kernel they launch reads the pools
        // the loop above has finished writing (st is synchronised)
        std::vector<int32_t> todo;
        for (int32_t i = 0; i < n_inst; ++i) {
            const int64_t n = offsets[i + 1] - offsets[i];
            if (n == 3) (void)solve_n3(ctx, coords + 2 * offsets[i], &res[i]);
            else if (n >= 4) todo.push_back(i);
        }
        for (int32_t i : todo)
            if (ch[i].overflow) fail(ctx, F2M_ERR_OVERFLOW, "|lambda2| reached 2^38");
        std::stable_sort(todo.begin(), todo.end(), [&](int32_t a, int32_t b) {
            return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
        });
        const int nw = (int)std::min<size_t>(todo.size(), (size_t)finish_threads());
        while ((int)ctx->workers.size() < nw) {
            f2m_ctx *w = nullptr;
            const f2m_status cs = f2m_create(&w, ctx->device, &ctx->defaults);
            if (cs != F2M_OK) fail(ctx, cs, "cannot create a finishing context");
            w->is_worker = true;
            ctx->workers.push_back(w);
        }
        std::vector<f2m_status> ist(n_inst, F2M_OK);
        std::vector<std::string> imsg(n_inst);
        std::atomic<size_t> next{0};
        auto work = [&](f2m_ctx *wc) {
            (void)hipSetDevice(wc->device);
            for (size_t j; (j = next.fetch_add(1)) < todo.size();) {
                const int32_t i = todo[j];
                const int64_t n = offsets[i + 1] - offsets[i], X = offsets[i];
                const double ti = now_s();
                try {
                    GeoHost gh;
                    gh.g = Geo{n, orig + P[i], pos + X, box + T[i], x2h[i]};
                    gh.xy = xy + 2 * X;
                    gh.cx = cxs[i];
                    gh.cy = cys[i];
                    gh.col = col + P[i];
                    const Ctrl &c = ch[i];
                    const int64_t *last = (c.k_last & 1) ? lam1 + P[i] : lam0 + P[i];
                    const int64_t *lstar = (c.kstar == c.k_last) ? last : best + P[i];
                    InstanceState is{gh, c, lstar, z4 + kTop * X, i4 + kTop * X, seed + kTop * X,
                                     trace ? trace + (int64_t)i * trace_cap * kTraceW : nullptr, nullptr, nullptr,
                                     last};
                    complete_result(wc, is, o, wc->stream, res[i]);
                } catch (const Fail &f) {
                    ist[i] = f.st;
                    imsg[i] = wc->err;
                } catch (const std::bad_alloc &) {
                    ist[i] = F2M_ERR_NOMEM;
                    imsg[i] = "host allocation failed";
                }
                res[i].scan_rows = 1;
                res[i].scan_slices = shp[i].slices;
                res[i].seconds[2] = t2 - t1;
                res[i].seconds[5] = now_s() - ti;
            }
        };
        {
            std::vector<std::thread> pool;
            for (int w = 1; w < nw; ++w) {
                try {
                    pool.emplace_back(work, ctx->workers[w]);
                } catch (const std::exception &) {
                    break;   // fewer threads: the shared queue still covers every instance
                }
            }
            if (nw > 0) work(ctx->workers[0]);
            for (auto &th : pool) th.join();
        }
        for (int32_t i = 0; i < n_inst; ++i)
            if (ist[i] != F2M_OK) fail(ctx, ist[i], "instance " + std::to_string(i) + ": " + imsg[i]);
        for (int32_t i = 0; i < n_inst; ++i) {
            res[i].seconds[0] = t1 - t0;
            outs[i] = res[i];
        }
        bool all = true;
        for (int32_t i = 0; i < n_inst; ++i) all = all && res[i].certified;
        return all ? F2M_OK : F2M_NOT_CERTIFIED;
    } catch (const Fail &f) {
        for (auto &r : res) f2m_result_free(&r);
        return f.st;
    } catch (const std::bad_alloc &) {
        for (auto &r : res) f2m_result_free(&r);
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}


f2m_status f2m_sec_gdp(f2m_ctx *ctx, const int32_t *xy, int64_t n, const f2m_sec_rows *rows, int64_t *lam,
                       int64_t *mu, int64_t max_iters, int64_t *trace, int64_t trace_cap, f2m_sec_result *out)
{
    if (!ctx) return F2M_ERR_ARG;
    ctx->dev_cap = (size_t)ctx->defaults.max_device_bytes;
    try {
        if (!xy || !lam || !out || n < 4) fail(ctx, F2M_ERR_ARG, "sec_gdp needs n >= 4, coords, lambda2 and out");
        if (max_iters < 0 || trace_cap < 0) fail(ctx, F2M_ERR_ARG, "max_iters and trace_cap must be >= 0");
        sec_check_rows(ctx, n, rows);
        if (rows->nrows > 0 && !mu) fail(ctx, F2M_ERR_ARG, "mu is null");
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        const double t0 = now_s();
        const SecCtrl c = sec_gdp(ctx, xy, n, rows, lam, mu, max_iters, trace, trace_cap, true);
        f2m_sec_result r;
        std::memset(&r, 0, sizeof(r));
        r.iterations = c.k_last + 1;
        r.kstar = c.kstar;
        r.stop = (int32_t)c.stop;
        r.overflow = (int32_t)c.overflow;
        r.dual2 = (c.kstar == c.k_last) ? c.dual2_last : c.best_dual2;
        r.primal2_last = c.primal2_last;
        r.bad_last = c.node_bad_last + c.row_infeas_last + c.row_loose_last;
        r.seconds = now_s() - t0;
        r.pairs_tested = (int64_t)c.pairs_tested;
        *out = r;
        return c.overflow ? F2M_ERR_OVERFLOW : F2M_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}

f2m_status f2m_sec_certify(f2m_ctx *ctx, const int32_t *xy, int64_t n, const f2m_sec_rows *rows,
                           const int64_t *lam, const int64_t *mu, int64_t out[5])
{
    if (!ctx) return F2M_ERR_ARG;
    ctx->dev_cap = (size_t)ctx->defaults.max_device_bytes;
    try {
        if (!xy || !lam || !out || n < 4) fail(ctx, F2M_ERR_ARG, "sec_certify needs n >= 4, coords, lambda2 and out");
        sec_check_rows(ctx, n, rows);
        if (rows->nrows > 0 && !mu) fail(ctx, F2M_ERR_ARG, "mu is null");
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        // iteration 0 of a loop capped at 0: the statistics of (Lam, M)
        const SecCtrl c = sec_gdp(ctx, xy, n, rows, const_cast<int64_t *>(lam), const_cast<int64_t *>(mu), 0,
                                  nullptr, 0, false);
        const bool feasible = c.node_bad_last == 0 && c.row_infeas_last == 0;
        const bool tight = c.row_loose_last == 0;
        out[0] = c.primal2_last;
        out[1] = c.dual2_last;
        out[2] = feasible ? 1 : 0;
        out[3] = tight ? 1 : 0;
        out[4] = (feasible && tight && c.primal2_last == c.dual2_last) ? 1 : 0;
        return F2M_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}

f2m_status f2m_sec_separate(f2m_ctx *ctx, const int32_t *xy, int64_t n, const f2m_sec_rows *rows,
                            const int64_t *lam, const int64_t *mu, int32_t *new_row_of, int64_t *new_rows,
                            int64_t *components)
{
    if (!ctx) return F2M_ERR_ARG;
    ctx->dev_cap = (size_t)ctx->defaults.max_device_bytes;
    try {
        if (!xy || !lam || !new_row_of || !new_rows || !components || n < 4)
            fail(ctx, F2M_ERR_ARG, "sec_separate needs n >= 4 and every output");
        sec_check_rows(ctx, n, rows);
        if (rows->nrows > 0 && !mu) fail(ctx, F2M_ERR_ARG, "mu is null");
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        std::vector<int32_t> nr;
        int64_t nnew = 0, ncomp = 0;
        sec_separate(ctx, xy, n, rows, lam, mu, nr, &nnew, &ncomp);
        // new_row_of need not be 16-byte aligned: a plain copy
        ck(ctx, hipMemcpyAsync(new_row_of, nr.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream),
           "copy");
        ck(ctx, hipStreamSynchronize(ctx->stream), "sync");
        *new_rows = nnew;
        *components = ncomp;
        return F2M_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}

f2m_status f2m_sec_solve(f2m_ctx *ctx, const int32_t *xy, int64_t n, int64_t *lam, int32_t *row_of,
                         int32_t nlayers0, int64_t nrows0, int64_t *mu, int64_t mu_cap, int32_t max_rounds,
                         int64_t max_iters, f2m_sec_solve_result *res)
{
    if (!ctx) return F2M_ERR_ARG;
    ctx->dev_cap = (size_t)ctx->defaults.max_device_bytes;
    try {
        if (!xy || !lam || !row_of || !res || n < 4) fail(ctx, F2M_ERR_ARG, "sec_solve needs n >= 4 and its arrays");
        if (max_rounds < 0 || max_iters < 0 || mu_cap < nrows0 || (mu_cap > 0 && !mu))
            fail(ctx, F2M_ERR_ARG, "bad max_rounds, max_iters or mu capacity");
        f2m_sec_rows rows{nlayers0, 0, nrows0, row_of};
        sec_check_rows(ctx, n, &rows);
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        const double t0 = now_s();
        f2m_sec_solve_result r;
        std::memset(&r, 0, sizeof(r));
        // the start's bound (its rows and M)
        {
            const SecCtrl c = sec_gdp(ctx, xy, n, &rows, lam, mu, 0, nullptr, 0, false);
            r.dual2_start = c.dual2_last;
            r.best_dual2 = c.dual2_last;
        }
        f2m_status st = F2M_OK;
        for (int32_t round = 0; round < max_rounds && rows.nlayers < F2M_SEC_MAX_LAYERS; ++round) {
            std::vector<int32_t> nr;
            int64_t nnew = 0, ncomp = 0;
            sec_separate(ctx, xy, n, &rows, lam, mu, nr, &nnew, &ncomp);
            r.components = (int32_t)std::min<int64_t>(ncomp, INT32_MAX);
            if (nnew == 0 || rows.nrows + nnew > mu_cap) break;
            ck(ctx, hipMemcpyAsync(row_of + (int64_t)rows.nlayers * n, nr.data(), n * sizeof(int32_t),
                                   hipMemcpyHostToDevice, ctx->stream), "copy");
            ck(ctx, hipStreamSynchronize(ctx->stream), "sync");
            ck(ctx, hipMemsetAsync(mu + rows.nrows, 0, nnew * sizeof(int64_t), ctx->stream), "memset");
            rows.nlayers += 1;
            rows.nrows += nnew;
            const SecCtrl c = sec_gdp(ctx, xy, n, &rows, lam, mu, max_iters, nullptr, 0, true);
            r.rows_added[round] = nnew;
            r.iterations[round] = c.k_last + 1;
            r.stop[round] = (int32_t)c.stop;
            r.dual2[round] = (c.kstar == c.k_last) ? c.dual2_last : c.best_dual2;
            r.best_dual2 = std::max(r.best_dual2, r.dual2[round]);
            r.rounds = round + 1;
            if (c.overflow) { st = F2M_ERR_OVERFLOW; break; }
        }
        r.nlayers = rows.nlayers;
        r.nrows = rows.nrows;
        {
            const SecCtrl c = sec_gdp(ctx, xy, n, &rows, lam, mu, 0, nullptr, 0, false);
            const bool ok = c.node_bad_last == 0 && c.row_infeas_last == 0 && c.row_loose_last == 0;
            r.certified = (ok && c.primal2_last == c.dual2_last) ? 1 : 0;
        }
        r.seconds = now_s() - t0;
        *res = r;
        return st;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}

}  // extern "C"
