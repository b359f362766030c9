// Host runtime of libf2m: contexts, device workspaces, the GDP loop with its
// device-side stop test, the finish and the certificate, behind the C ABI
// declared in include/f2m.h.
#include "f2m.h"
#include "f2m_finish.h"
#include "f2m_internal.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace f2m;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct f2m_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<DevBuf *> bufs;
    // geometry of the current instance (sorted order)
    DevBuf xy, minmax, keys, keys_alt, ids, orig, pos, box, xy2max, sort_temp;
    // GDP loop state
    DevBuf col, lam[2], lam_best, lam_label, tile_hmax, pz, pi, pneg, pzero, prowneg, z4, i4, seed, ctrl, trace;
    // trivial x
    DevBuf slot_u, slot_v, slot_x, eu, ev, ex, btmp, count;
    // certificate / pair collection state
    DevBuf c_col, c_lam, c_tile_hmax, c_ctrl, c_deg, c_cnt, c_nb, c_acc, c_lam_label, c_eu, c_ev, c_ex;
    DevBuf p_pairs, p_count;
    // candidate graph
    DevBuf knn_nbr, csr_keys, csr_keys2, csr_deg, csr_rowptr, csr_col, csr_cost, csr_temp, csr_nnz;
    Ctrl *ctrl_host = nullptr;   // pinned
    int64_t *scratch_host = nullptr;   // pinned, 16 entries

    f2m_ctx()
    {
        DevBuf *all[] = {&xy, &minmax, &keys, &keys_alt, &ids, &orig, &pos, &box, &xy2max, &sort_temp,
                         &col, &lam[0], &lam[1], &lam_best, &lam_label, &tile_hmax, &pz, &pi, &pneg, &pzero,
                         &prowneg, &z4, &i4, &seed, &ctrl, &trace, &slot_u, &slot_v, &slot_x, &eu, &ev, &ex,
                         &btmp, &count, &c_col, &c_lam, &c_tile_hmax, &c_ctrl, &c_deg, &c_cnt, &c_nb, &c_acc,
                         &c_lam_label, &c_eu, &c_ev, &c_ex, &p_pairs, &p_count, &knn_nbr, &csr_keys,
                         &csr_keys2, &csr_deg, &csr_rowptr, &csr_col, &csr_cost, &csr_temp, &csr_nnz};
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

template <typename T>
T *grow(f2m_ctx *ctx, DevBuf &b, size_t count)
{
    const size_t need = std::max<size_t>(count * sizeof(T), 256);
    if (b.bytes < need) {
        if (b.p) (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        ck(ctx, hipMalloc(&b.p, need), "hipMalloc");
        b.bytes = need;
    }
    return static_cast<T *>(b.p);
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int64_t ntiles_of(int64_t n) { return (n + kTileCols - 1) / kTileCols; }

// Scan launch shape: rows per lane and column slices (slice length a
// multiple of the tile width).  Results never depend on it.
struct ScanShape {
    int rows;          // rows per thread
    int64_t slices;
    int64_t slice_len;
};

ScanShape scan_shape(int64_t n, bool cull)
{
    ScanShape s;
    const int64_t nt = ntiles_of(n);
    if (cull) {
        s.rows = 1;
        const int64_t sl = std::max<int64_t>(1, std::min<int64_t>(nt, 8));
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
};

GeoHost setup_geo(f2m_ctx *ctx, const int32_t *xy_dev, int64_t n, hipStream_t st)
{
    GeoHost gh;
    int32_t *m4 = grow<int32_t>(ctx, ctx->minmax, 4);
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
    const size_t tb = sort_temp_bytes(n);
    uint32_t *keys = grow<uint32_t>(ctx, ctx->keys, n);
    uint32_t *keys2 = grow<uint32_t>(ctx, ctx->keys_alt, n);
    int32_t *ids = grow<int32_t>(ctx, ctx->ids, n);
    int32_t *orig = grow<int32_t>(ctx, ctx->orig, n);
    int32_t *pos = grow<int32_t>(ctx, ctx->pos, n);
    void *temp = grow<char>(ctx, ctx->sort_temp, tb);
    ck(ctx, launch_sort(xy_dev, n, h[0], h[2], keys, keys2, ids, orig, pos, temp, tb, st), "sort");
    float4 *col = grow<float4>(ctx, ctx->col, n);
    float4 *box = grow<float4>(ctx, ctx->box, ntiles_of(n));
    float *x2m = grow<float>(ctx, ctx->xy2max, 1);
    ck(ctx, launch_prep(xy_dev, orig, n, gh.cx, gh.cy, col, box, x2m, st), "prep");
    float x2host = 0.0f;
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, x2m, sizeof(float), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    std::memcpy(&x2host, ctx->scratch_host, sizeof(float));
    gh.g = Geo{n, orig, pos, box, x2host};
    return gh;
}

// A Lam placed on the certificate / collection state: sorted Lam, column
// records and tile maxima; lam_label_dev is in label order.
LamView place_lam(f2m_ctx *ctx, const GeoHost &gh, const int64_t *lam_label_dev, hipStream_t st)
{
    const int64_t n = gh.g.n;
    float4 *col = grow<float4>(ctx, ctx->c_col, n);
    int64_t *ls = grow<int64_t>(ctx, ctx->c_lam, n);
    float *th = grow<float>(ctx, ctx->c_tile_hmax, ntiles_of(n));
    Ctrl *cc = grow<Ctrl>(ctx, ctx->c_ctrl, 1);
    float *x2m = grow<float>(ctx, ctx->xy2max, 1);
    ck(ctx, launch_prep(gh.xy, gh.g.orig, n, gh.cx, gh.cy, col, (float4 *)ctx->box.p, x2m, st), "prep");
    ck(ctx, launch_ctrl_init(cc, 0, 0, 0, st), "ctrl");
    ck(ctx, launch_set_lam(lam_label_dev, gh.g.orig, n, ls, col, th, cc, st), "set_lam");
    return LamView{col, ls, th, cc};
}

// Certificate of (lam, edges); lam and the edges are device arrays by label.
void certify_dev(f2m_ctx *ctx, const GeoHost &gh, const int64_t *lam_label, int64_t m, const int32_t *eu,
                 const int32_t *ev, const uint8_t *ex, hipStream_t st, int64_t out[4])
{
    const int64_t n = gh.g.n;
    LamView lv = place_lam(ctx, gh, lam_label, st);
    int32_t *deg = grow<int32_t>(ctx, ctx->c_deg, n);
    int32_t *cnt = grow<int32_t>(ctx, ctx->c_cnt, n);
    int32_t *nb = grow<int32_t>(ctx, ctx->c_nb, kTop * n);
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
    ck(ctx, launch_cert_nodes(lam_label, n, deg, cnt, nb, acc, st), "cert_nodes");
    unsigned long long h[4];
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, acc, sizeof(h), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    std::memcpy(h, ctx->scratch_host, sizeof(h));
    const int64_t rowneg = (int64_t)h[0], primal2 = (int64_t)h[1], viol = (int64_t)h[2], sl = (int64_t)h[3];
    out[0] = primal2;
    out[1] = 2 * sl + rowneg / 2;
    out[2] = viol == 0 ? 1 : 0;
    out[3] = (viol == 0 && out[0] == out[1]) ? 1 : 0;
}

// Candidate pairs for the exact finish from GPU scans of the complete graph.
class GpuPairs : public PairSource {
public:
    GpuPairs(f2m_ctx *ctx, const GeoHost &gh, const int32_t *seed_dev, hipStream_t st)
        : ctx_(ctx), gh_(gh), seed_(seed_dev), st_(st)
    {
    }
    bool near(const int64_t *lam, int64_t slack, PairList &out, std::string &err) override
    {
        return run(lam, seed_, 0, slack, out, err);
    }
    bool negative(const int64_t *lam, PairList &out, std::string &err) override
    {
        return run(lam, nullptr, -1, 0, out, err);
    }

private:
    bool run(const int64_t *lam_host, const int32_t *seed, int64_t theta, int64_t slack, PairList &out,
             std::string &err)
    {
        try {
            f2m_ctx *ctx = ctx_;
            const int64_t n = gh_.g.n;
            int64_t *lam = grow<int64_t>(ctx, ctx->c_lam_label, n);
            unsigned long long *cnt = grow<unsigned long long>(ctx, ctx->p_count, 1);
            ck(ctx, hipMemcpyAsync(lam, lam_host, n * sizeof(int64_t), hipMemcpyHostToDevice, st_), "copy");
            LamView lv = place_lam(ctx, gh_, lam, st_);
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
                ck(ctx, launch_scan(sa, kModeCollect, sh.slices, sh.rows, st_), "collect");
                ck(ctx, hipMemcpyAsync(ctx->scratch_host, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, st_), "copy");
                ck(ctx, hipStreamSynchronize(st_), "sync");
                const int64_t found = ctx->scratch_host[0];
                if (found > cap) { cap = found + found / 4; continue; }
                std::vector<int2> h(found);
                if (found)
                    ck(ctx, hipMemcpyAsync(h.data(), pairs, found * sizeof(int2), hipMemcpyDeviceToHost, st_), "copy");
                ck(ctx, hipStreamSynchronize(st_), "sync");
                out.clear();
                out.reserve(found);
                for (const int2 &p : h) out.emplace_back(p.x, p.y);
                std::sort(out.begin(), out.end());
                out.erase(std::unique(out.begin(), out.end()), out.end());
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
    const int32_t *seed_;
    hipStream_t st_;
    int64_t cap_ = 0;
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
    ck(ctx, launch_knn(gh.g, static_cast<const float4 *>(ctx->col.p), K, nbr, nullptr, st), "knn");
    ck(ctx, launch_build_csr(gh.g, gh.xy, n, K, nbr, keys, keys2, deg, rowptr, col, cost, nnz_dev, temp, tb, 2 * nk,
                             st), "csr");
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, nnz_dev, sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    return Csr{rowptr, col, cost, ctx->scratch_host[0]};
}

// Certificate of (lam, edges) restricted to the candidate graph.
void certify_graph_dev(f2m_ctx *ctx, const GeoHost &gh, const Csr &csr, const int64_t *lam_label, int64_t m,
                       const int32_t *eu, const int32_t *ev, const uint8_t *ex, hipStream_t st, int64_t out[4])
{
    const int64_t n = gh.g.n;
    LamView lv = place_lam(ctx, gh, lam_label, st);
    int32_t *deg = grow<int32_t>(ctx, ctx->c_deg, n);
    int32_t *cnt = grow<int32_t>(ctx, ctx->c_cnt, n);
    int32_t *nb = grow<int32_t>(ctx, ctx->c_nb, kTop * n);
    unsigned long long *acc = grow<unsigned long long>(ctx, ctx->c_acc, 4);
    ck(ctx, hipMemsetAsync(deg, 0, n * sizeof(int32_t), st), "memset");
    ck(ctx, hipMemsetAsync(cnt, 0, n * sizeof(int32_t), st), "memset");
    ck(ctx, hipMemsetAsync(acc, 0, 4 * sizeof(unsigned long long), st), "memset");
    ck(ctx, launch_graph_dual(gh.g, csr, lv.lam, acc, st), "graph_dual");
    ck(ctx, launch_cert_edges(gh.xy, n, m, eu, ev, ex, deg, cnt, nb, acc, st), "cert_edges");
    ck(ctx, launch_graph_membership(gh.g, csr, m, eu, ev, acc, st), "membership");
    ck(ctx, launch_cert_nodes(lam_label, n, deg, cnt, nb, acc, st), "cert_nodes");
    unsigned long long h[4];
    ck(ctx, hipMemcpyAsync(ctx->scratch_host, acc, sizeof(h), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    std::memcpy(h, ctx->scratch_host, sizeof(h));
    const int64_t rowneg = (int64_t)h[0], primal2 = (int64_t)h[1], viol = (int64_t)h[2], sl = (int64_t)h[3];
    out[0] = primal2;
    out[1] = 2 * sl + rowneg / 2;
    out[2] = viol == 0 ? 1 : 0;
    out[3] = (viol == 0 && out[0] == out[1]) ? 1 : 0;
}

// Candidate pairs for the exact finish on the candidate graph.
class GpuGraphPairs : public PairSource {
public:
    GpuGraphPairs(f2m_ctx *ctx, const GeoHost &gh, const Csr &csr, hipStream_t st)
        : ctx_(ctx), gh_(gh), csr_(csr), st_(st)
    {
    }
    bool near(const int64_t *lam, int64_t slack, PairList &out, std::string &err) override
    {
        return run(lam, slack < 0 ? 0 : slack, out, err);
    }
    bool negative(const int64_t *lam, PairList &out, std::string &err) override { return run(lam, -1, out, err); }

private:
    bool run(const int64_t *lam_host, int64_t slack, PairList &out, std::string &err)
    {
        try {
            f2m_ctx *ctx = ctx_;
            const int64_t n = gh_.g.n;
            int64_t *lam = grow<int64_t>(ctx, ctx->c_lam_label, n);
            unsigned long long *cnt = grow<unsigned long long>(ctx, ctx->p_count, 1);
            ck(ctx, hipMemcpyAsync(lam, lam_host, n * sizeof(int64_t), hipMemcpyHostToDevice, st_), "copy");
            LamView lv = place_lam(ctx, gh_, lam, st_);
            const int64_t cap = csr_.nnz + 1;
            int2 *pairs = grow<int2>(ctx, ctx->p_pairs, cap);
            ck(ctx, hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st_), "memset");
            ck(ctx, launch_graph_collect(gh_.g, csr_, lv.lam, slack, cnt, pairs, cap, st_), "graph_collect");
            ck(ctx, hipMemcpyAsync(ctx->scratch_host, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, st_), "copy");
            ck(ctx, hipStreamSynchronize(st_), "sync");
            const int64_t found = std::min<int64_t>(ctx->scratch_host[0], cap);
            std::vector<int2> h(found);
            if (found)
                ck(ctx, hipMemcpyAsync(h.data(), pairs, found * sizeof(int2), hipMemcpyDeviceToHost, st_), "copy");
            ck(ctx, hipStreamSynchronize(st_), "sync");
            out.clear();
            out.reserve(found);
            for (const int2 &p : h) out.emplace_back(p.x, p.y);
            std::sort(out.begin(), out.end());
            out.erase(std::unique(out.begin(), out.end()), out.end());
            return true;
        } catch (const Fail &) {
            err = ctx_->err;
            return false;
        }
    }

    f2m_ctx *ctx_;
    GeoHost gh_;
    Csr csr_;
    hipStream_t st_;
};

struct LoopOut {
    Ctrl c;
    double scan_ms = 0.0;
    int64_t scan_launches = 0;
    ScanShape shape;
    int64_t *lam_star;     // device, sorted: Lam_kstar
};

// The GDP loop on device buffers.  lam0_label_dev: device Lam_0 by label
// (null: zero).
LoopOut gdp_loop(f2m_ctx *ctx, const GeoHost &gh, const int64_t *lam0_label_dev, int64_t max_iters,
                 int64_t handoff_div, int32_t chunk_opt, bool want_trace, bool time_kernels, bool cull,
                 const Csr *csr, hipStream_t st)
{
    LoopOut o;
    const int64_t n = gh.g.n;
    // on the candidate graph the step is one fused kernel and needs no partials
    const ScanShape sh = csr ? ScanShape{1, 1, ((n + kTileCols - 1) / kTileCols) * kTileCols} : scan_shape(n, cull);
    float4 *col = static_cast<float4 *>(ctx->col.p);
    int64_t *lam[2] = {grow<int64_t>(ctx, ctx->lam[0], n), grow<int64_t>(ctx, ctx->lam[1], n)};
    int64_t *best = grow<int64_t>(ctx, ctx->lam_best, n);
    int64_t *l0 = grow<int64_t>(ctx, ctx->lam_label, n);
    float *thm = grow<float>(ctx, ctx->tile_hmax, ntiles_of(n));
    int64_t *pz = grow<int64_t>(ctx, ctx->pz, sh.slices * kTop * n);
    int32_t *pi = grow<int32_t>(ctx, ctx->pi, sh.slices * kTop * n);
    int32_t *pneg = grow<int32_t>(ctx, ctx->pneg, sh.slices * n);
    int32_t *pzero = grow<int32_t>(ctx, ctx->pzero, sh.slices * n);
    int64_t *prn = grow<int64_t>(ctx, ctx->prowneg, sh.slices * n);
    int64_t *z4 = grow<int64_t>(ctx, ctx->z4, kTop * n);
    int32_t *i4 = grow<int32_t>(ctx, ctx->i4, kTop * n);
    int32_t *seed = grow<int32_t>(ctx, ctx->seed, kTop * n);
    Ctrl *cd = grow<Ctrl>(ctx, ctx->ctrl, 1);
    const int64_t trace_cap = want_trace ? max_iters + 1 : 0;
    int64_t *trace = want_trace ? grow<int64_t>(ctx, ctx->trace, kTraceW * trace_cap) : nullptr;

    if (lam0_label_dev)
        ck(ctx, hipMemcpyAsync(l0, lam0_label_dev, n * sizeof(int64_t), hipMemcpyDeviceToDevice, st), "copy");
    else
        ck(ctx, hipMemsetAsync(l0, 0, n * sizeof(int64_t), st), "memset");
    ck(ctx, launch_ctrl_init(cd, max_iters, trace_cap, handoff_div, st), "ctrl_init");
    ck(ctx, launch_set_lam(l0, gh.g.orig, n, lam[0], col, thm, cd, st), "set_lam");
    ck(ctx, launch_seed_neighbours(n, seed, st), "seed");
    ck(ctx, hipMemcpyAsync(ctx->ctrl_host, cd, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "copy");
    ck(ctx, hipStreamSynchronize(st), "sync");
    if (ctx->ctrl_host->maxabs_lam >= kLamLimit) fail(ctx, F2M_ERR_OVERFLOW, "|lambda2_init| must be below 2^38");

    const int chunk = chunk_opt > 0 ? chunk_opt : (n >= 50000 ? 4 : (n >= 5000 ? 16 : 64));
    std::vector<hipEvent_t> evs;
    if (time_kernels) {
        evs.resize(2 * chunk);
        for (auto &e : evs) ck(ctx, hipEventCreate(&e), "hipEventCreate");
    }
    struct EvGuard {
        std::vector<hipEvent_t> &v;
        ~EvGuard() { for (auto e : v) (void)hipEventDestroy(e); }
    } guard{evs};
    int64_t k = 0;
    for (;;) {
        int issued = 0;
        for (int j = 0; j < chunk && k <= max_iters; ++j, ++k, ++issued) {
            if (csr) {
                GraphStepArgs ga{gh.g, *csr, k, lam[k & 1], lam[(k + 1) & 1], best, z4, i4, nullptr, nullptr,
                                 nullptr, cd, trace};
                if (time_kernels) ck(ctx, hipEventRecord(evs[2 * j], st), "hipEventRecord");
                ck(ctx, launch_graph_step(ga, st), "graph_step");
                if (time_kernels) ck(ctx, hipEventRecord(evs[2 * j + 1], st), "hipEventRecord");
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
            if (time_kernels) ck(ctx, hipEventRecord(evs[2 * j], st), "hipEventRecord");
            ck(ctx, launch_scan(sa, kModeGdp, sh.slices, sh.rows, st), "scan");
            if (time_kernels) ck(ctx, hipEventRecord(evs[2 * j + 1], st), "hipEventRecord");
            UpdateArgs ua{gh.g, sh.slices, k, pz, pi, pneg, pzero, prn, lam[k & 1], lam[(k + 1) & 1], best, col,
                          thm, z4, i4, seed, nullptr, nullptr, nullptr, cd, trace};
            ck(ctx, launch_update(ua, st), "update");
        }
        ck(ctx, hipMemcpyAsync(ctx->ctrl_host, cd, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "copy");
        ck(ctx, hipStreamSynchronize(st), "sync");
        if (time_kernels) {
            // iterations after the stop exit at once; count the ones that ran
            const int64_t k0 = k - issued;
            const int64_t ran = std::min<int64_t>(issued, ctx->ctrl_host->k_last + 1 - k0);
            for (int64_t j = 0; j < ran; ++j) {
                float ms = 0.0f;
                ck(ctx, hipEventElapsedTime(&ms, evs[2 * j], evs[2 * j + 1]), "hipEventElapsedTime");
                o.scan_ms += ms;
                ++o.scan_launches;
            }
        }
        if (ctx->ctrl_host->done) break;
        if (k > max_iters) fail(ctx, F2M_ERR_DEVICE, "GDP loop passed the cap without stopping");
    }
    o.shape = sh;
    o.c = *ctx->ctrl_host;
    if (o.c.overflow) fail(ctx, F2M_ERR_OVERFLOW, "|lambda2| reached 2^38");
    int64_t *last = lam[o.c.k_last & 1];
    o.lam_star = (o.c.kstar == o.c.k_last) ? last : best;
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
    o->handoff_div = 300;
    o->knn_k = 10;
    o->finish = F2M_FINISH_EXACT;
}

f2m_status f2m_create(f2m_ctx **out, int device)
{
    if (!out) return F2M_ERR_ARG;
    *out = nullptr;
    f2m_ctx *ctx = new (std::nothrow) f2m_ctx();
    if (!ctx) return F2M_ERR_NOMEM;
    ctx->device = device;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        delete ctx;
        return F2M_ERR_DEVICE;
    }
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void **)&ctx->ctrl_host, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->scratch_host, 16 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
        f2m_destroy(ctx);
        return F2M_ERR_DEVICE;
    }
    *out = ctx;
    return F2M_OK;
}

void f2m_destroy(f2m_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (DevBuf *b : ctx->bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->ctrl_host) (void)hipHostFree(ctx->ctrl_host);
    if (ctx->scratch_host) (void)hipHostFree(ctx->scratch_host);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

void f2m_result_free(f2m_result *r)
{
    if (!r) return;
    std::free(r->lambda2);
    std::free(r->lambda2_gdp);
    std::free(r->edge_u);
    std::free(r->edge_v);
    std::free(r->edge_x2);
    std::free(r->trace);
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

f2m_status f2m_gdp_step(f2m_ctx *ctx, const int32_t *xy, int64_t n, const int64_t *lam_in, int64_t *lam_out,
                        int64_t *z4_out, int32_t *i4_out, int32_t *neg, int32_t *zero, int64_t *step,
                        int64_t rec[F2M_TRACE_W])
{
    if (!ctx) return F2M_ERR_ARG;
    try {
        if (!xy || !lam_in || !lam_out || !rec || n < 4 || lam_in == lam_out)
            fail(ctx, F2M_ERR_ARG, "gdp_step needs n >= 4, coords, distinct lambda2_in/out and rec");
        ck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        hipStream_t st = ctx->stream;
        const GeoHost gh = setup_geo(ctx, xy, n, st);
        const bool cull = true;
        const ScanShape sh = scan_shape(n, cull);
        float4 *col = static_cast<float4 *>(ctx->col.p);
        int64_t *ls = grow<int64_t>(ctx, ctx->lam[0], n);
        int64_t *lo = grow<int64_t>(ctx, ctx->lam[1], n);
        int64_t *best = grow<int64_t>(ctx, ctx->lam_best, n);
        float *thm = grow<float>(ctx, ctx->tile_hmax, ntiles_of(n));
        int64_t *pz = grow<int64_t>(ctx, ctx->pz, sh.slices * kTop * n);
        int32_t *pi = grow<int32_t>(ctx, ctx->pi, sh.slices * kTop * n);
        int32_t *pneg = grow<int32_t>(ctx, ctx->pneg, sh.slices * n);
        int32_t *pzero = grow<int32_t>(ctx, ctx->pzero, sh.slices * n);
        int64_t *prn = grow<int64_t>(ctx, ctx->prowneg, sh.slices * n);
        int64_t *z4 = z4_out ? z4_out : grow<int64_t>(ctx, ctx->z4, kTop * n);
        int32_t *i4 = i4_out ? i4_out : grow<int32_t>(ctx, ctx->i4, kTop * n);
        int32_t *seed = grow<int32_t>(ctx, ctx->seed, kTop * n);
        Ctrl *cd = grow<Ctrl>(ctx, ctx->ctrl, 1);
        int64_t *trace = grow<int64_t>(ctx, ctx->trace, kTraceW);
        ck(ctx, launch_ctrl_init(cd, INT64_MAX, 1, 0, st), "ctrl_init");
        ck(ctx, launch_set_lam(lam_in, gh.g.orig, n, ls, col, thm, cd, st), "set_lam");
        ck(ctx, launch_seed_neighbours(n, seed, st), "seed");
        ck(ctx, hipMemcpyAsync(ctx->ctrl_host, cd, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "copy");
        ck(ctx, hipStreamSynchronize(st), "sync");
        if (ctx->ctrl_host->maxabs_lam >= kLamLimit) fail(ctx, F2M_ERR_OVERFLOW, "|lambda2| must be below 2^38");
        ScanArgs sa{};
        sa.g = gh.g;
        sa.lv = LamView{col, ls, thm, cd};
        sa.slice_len = sh.slice_len;
        sa.cull = cull ? 1 : 0;
        sa.check_done = 1;
        sa.seed = seed;
        sa.pz = pz; sa.pi = pi; sa.pneg = pneg; sa.pzero = pzero; sa.prowneg = prn;
        ck(ctx, launch_scan(sa, kModeGdp, sh.slices, sh.rows, st), "scan");
        UpdateArgs ua{gh.g, sh.slices, 0, pz, pi, pneg, pzero, prn, ls, lo, best, col, thm,
                      z4, i4, seed, neg, zero, step, cd, trace};
        ck(ctx, launch_update(ua, st), "update");
        ck(ctx, launch_unpermute(lo, gh.g.orig, n, lam_out, st), "unpermute");
        ck(ctx, hipMemcpyAsync(ctx->scratch_host, trace, kTraceW * sizeof(int64_t), hipMemcpyDeviceToHost, st),
           "copy");
        ck(ctx, hipStreamSynchronize(st), "sync");
        std::memcpy(rec, ctx->scratch_host, kTraceW * sizeof(int64_t));
        return F2M_OK;
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return F2M_ERR_NOMEM;
    }
}

f2m_status f2m_knn_graph(f2m_ctx *ctx, const int32_t *xy, int64_t n, int32_t k, int32_t *rowptr, int32_t *col,
                         int64_t cap, int64_t *nnz)
{
    if (!ctx) return F2M_ERR_ARG;
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
        f2m_opts o;
        f2m_opts_default(&o);
        if (opts) {
            if (opts->struct_size != sizeof(f2m_opts)) fail(ctx, F2M_ERR_ARG, "opts.struct_size mismatch");
            o = *opts;
        }
        if (!coords || !out) fail(ctx, F2M_ERR_ARG, "null coords or result");
        if (o.rule_version != 1) fail(ctx, F2M_ERR_ARG, "only rule_version 1 exists");
        if (o.graph != F2M_GRAPH_COMPLETE && o.graph != F2M_GRAPH_KNN) fail(ctx, F2M_ERR_ARG, "unknown graph kind");
        const bool on_graph = o.graph == F2M_GRAPH_KNN;
        if (o.max_iters < 0) fail(ctx, F2M_ERR_ARG, "max_iters < 0");
        if (o.handoff_div < 0) fail(ctx, F2M_ERR_ARG, "handoff_div < 0");
        if (o.warm == F2M_WARM_USER && !o.lambda2_init) fail(ctx, F2M_ERR_ARG, "warm start without lambda2_init");
        if (o.warm != F2M_WARM_COLD && o.warm != F2M_WARM_USER) fail(ctx, F2M_ERR_ARG, "unknown warm mode");
        if (n < 3) fail(ctx, F2M_ERR_INFEASIBLE, "F2M needs n >= 3");
        if (n >= (int64_t)1 << 30) fail(ctx, F2M_ERR_ARG, "n must be below 2^30");
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
        const GeoHost gh = setup_geo(ctx, xy_dev, n, st);
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
        const double t1 = now_s();
        LoopOut lo = gdp_loop(ctx, gh, lam0_dev, o.max_iters, o.handoff_div, o.chunk, o.record_trace != 0,
                              o.time_kernels != 0, o.scan_mode != F2M_SCAN_FULL, on_graph ? &csr : nullptr, st);
        const double t2 = now_s();
        res.n = n;
        res.iterations = lo.c.k_last + 1;
        res.kstar = lo.c.kstar;
        res.stop = (int32_t)lo.c.stop;
        int64_t *lstar = grow<int64_t>(ctx, ctx->lam_label, n);
        ck(ctx, launch_unpermute(lo.lam_star, gh.g.orig, n, lstar, st), "unpermute");
        res.lambda2_gdp = reinterpret_cast<int64_t *>(host_alloc(ctx, n * sizeof(int64_t)));
        ck(ctx, hipMemcpyAsync(res.lambda2_gdp, lstar, n * sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
        if (o.record_trace) {
            res.trace_len = res.iterations;
            res.trace = reinterpret_cast<int64_t *>(host_alloc(ctx, res.trace_len * kTraceW * sizeof(int64_t)));
            ck(ctx, hipMemcpyAsync(res.trace, ctx->trace.p, res.trace_len * kTraceW * sizeof(int64_t),
                                   hipMemcpyDeviceToHost, st), "copy");
        }
        ck(ctx, hipStreamSynchronize(st), "sync");
        res.dual2_gdp = (lo.c.kstar == lo.c.k_last) ? lo.c.dual2_last : lo.c.best_dual2;

        int32_t *eu = nullptr, *ev = nullptr;
        uint8_t *ex = nullptr;
        int64_t m = 0;
        const int64_t *lam_final_dev = lstar;
        const double t3 = now_s();
        bool have_x = false;
        if (lo.c.stop == F2M_STOP_TRIVIAL) {
            const int64_t ns = kTop * n;
            int32_t *su = grow<int32_t>(ctx, ctx->slot_u, ns);
            int32_t *sv = grow<int32_t>(ctx, ctx->slot_v, ns);
            uint8_t *sx = grow<uint8_t>(ctx, ctx->slot_x, ns);
            eu = grow<int32_t>(ctx, ctx->eu, ns);
            ev = grow<int32_t>(ctx, ctx->ev, ns);
            ex = grow<uint8_t>(ctx, ctx->ex, ns);
            int32_t *bt = grow<int32_t>(ctx, ctx->btmp, compact_block_tmp_len(ns));
            int64_t *cnt = grow<int64_t>(ctx, ctx->count, 1);
            ck(ctx, launch_extract_trivial((const int64_t *)ctx->z4.p, (const int32_t *)ctx->i4.p, n, su, sv, sx, st),
               "extract");
            ck(ctx, launch_compact(su, sv, sx, ns, eu, ev, ex, cnt, bt, st), "compact");
            ck(ctx, hipMemcpyAsync(ctx->scratch_host, cnt, sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
            ck(ctx, hipStreamSynchronize(st), "sync");
            m = ctx->scratch_host[0];
            have_x = true;
        } else if (o.finish == F2M_FINISH_EXACT) {
            FinishResult fr;
            if (on_graph) {
                GpuGraphPairs src(ctx, gh, csr, st);
                finish_exact(xy_host.data(), n, res.lambda2_gdp, src, &fr);
            } else {
                GpuPairs src(ctx, gh, (const int32_t *)ctx->seed.p, st);
                finish_exact(xy_host.data(), n, res.lambda2_gdp, src, &fr);
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
            int64_t *ld = grow<int64_t>(ctx, ctx->c_lam_label, n);
            eu = grow<int32_t>(ctx, ctx->c_eu, std::max<int64_t>(m, 1));
            ev = grow<int32_t>(ctx, ctx->c_ev, std::max<int64_t>(m, 1));
            ex = grow<uint8_t>(ctx, ctx->c_ex, std::max<int64_t>(m, 1));
            // the GDP multipliers stay available in lstar; the certificate's
            // duals go to their own buffer
            int64_t *lf = grow<int64_t>(ctx, ctx->lam_best, n);
            ck(ctx, hipMemcpyAsync(lf, fr.lam.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, st), "copy");
            (void)ld;
            if (m) {
                ck(ctx, hipMemcpyAsync(eu, fr.eu.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy");
                ck(ctx, hipMemcpyAsync(ev, fr.ev.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy");
                ck(ctx, hipMemcpyAsync(ex, fr.ex2.data(), m * sizeof(uint8_t), hipMemcpyHostToDevice, st), "copy");
            }
            lam_final_dev = lf;
            have_x = true;
        }
        const double t4 = now_s();
        int64_t cert[4] = {0, 0, 0, 0}, cert_full[4] = {0, 0, 0, 0};
        if (have_x) {
            if (on_graph) {
                certify_graph_dev(ctx, gh, csr, lam_final_dev, m, eu, ev, ex, st, cert);
                certify_dev(ctx, gh, lam_final_dev, m, eu, ev, ex, st, cert_full);
            } else {
                certify_dev(ctx, gh, lam_final_dev, m, eu, ev, ex, st, cert);
                std::memcpy(cert_full, cert, sizeof(cert));
            }
        }
        const double t5 = now_s();
        res.n_edges = m;
        res.edge_u = reinterpret_cast<int32_t *>(host_alloc(ctx, std::max<int64_t>(m, 1) * sizeof(int32_t)));
        res.edge_v = reinterpret_cast<int32_t *>(host_alloc(ctx, std::max<int64_t>(m, 1) * sizeof(int32_t)));
        res.edge_x2 = reinterpret_cast<uint8_t *>(host_alloc(ctx, std::max<int64_t>(m, 1)));
        res.lambda2 = reinterpret_cast<int64_t *>(host_alloc(ctx, n * sizeof(int64_t)));
        if (m) {
            ck(ctx, hipMemcpyAsync(res.edge_u, eu, m * sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
            ck(ctx, hipMemcpyAsync(res.edge_v, ev, m * sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
            ck(ctx, hipMemcpyAsync(res.edge_x2, ex, m * sizeof(uint8_t), hipMemcpyDeviceToHost, st), "copy");
        }
        ck(ctx, hipMemcpyAsync(res.lambda2, lam_final_dev, n * sizeof(int64_t), hipMemcpyDeviceToHost, st), "copy");
        ck(ctx, hipStreamSynchronize(st), "sync");
        res.primal2 = cert[0];
        res.dual2 = have_x ? cert[1] : res.dual2_gdp;
        res.certified = (int32_t)cert[3];
        res.dual2_complete = have_x ? cert_full[1] : 0;
        res.certified_complete = (int32_t)cert_full[3];
        res.scan_pairs = (int64_t)lo.c.pairs_tested;
        res.scan_ms = lo.scan_ms;
        res.scan_launches = lo.scan_launches;
        res.scan_rows = lo.shape.rows;
        res.scan_slices = lo.shape.slices;
        res.seconds[0] = t1 - t0;
        res.seconds[2] = t2 - t1;
        res.seconds[3] = t4 - t3;
        res.seconds[4] = t5 - t4;
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

}  // extern "C"
