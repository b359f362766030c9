// Test harness: runs libf2m's exact finish (f2m_finish.cpp) on the CPU with a
// brute-force pair source, so the finish can be checked without a GPU.
#include "f2m_finish.h"

#include <cstring>
#include <vector>

using namespace f2m;

namespace {

struct BrutePairs : PairSource {
    const int32_t *xy;
    int64_t n;
    bool bulk = false;   // also supply costs and the bulk data, as the library's GPU source does
    bool as_keys = false;   // the bulk pairs as sorted keys, the pair list left empty
    std::vector<int32_t> c_, start_, inc_;
    std::vector<uint64_t> keys_v;
    std::vector<uint8_t> neg_;
    int64_t cost(int64_t u, int64_t v) const
    {
        const int64_t dx = (int64_t)xy[2 * u] - xy[2 * v], dy = (int64_t)xy[2 * u + 1] - xy[2 * v + 1];
        return nint_sqrt_host(dx * dx + dy * dy);
    }
    int64_t z(const int64_t *lam, int64_t u, int64_t v) const { return 2 * cost(u, v) - lam[u] - lam[v]; }
    static int64_t floor_half(int64_t x) { return x >= 0 ? x / 2 : -((-x + 1) / 2); }
    void extras(const int64_t *lam, const PairList &out)
    {
        costs = nullptr;
        keys = nullptr;
        nkeys = 0;
        neg = nullptr;
        inc_start = nullptr;
        inc = nullptr;
        if (!bulk) return;
        c_.clear();
        for (const auto &p : out) c_.push_back((int32_t)cost(p.first, p.second));
        costs = c_.data();
        if (!want_bulk) return;
        // arc u'->v'' has reduced cost c - alpha_u - beta_v
        neg_.clear();
        for (size_t i = 0; i < out.size(); ++i) {
            const int64_t u = out[i].first, v = out[i].second;
            const int64_t au = floor_half(lam[u]), av = floor_half(lam[v]);
            const int64_t bu = lam[u] - au, bv = lam[v] - av;
            neg_.push_back((uint8_t)((c_[i] - au - bv < 0 ? 1 : 0) | (c_[i] - av - bu < 0 ? 2 : 0)));
        }
        std::vector<int32_t> deg(n, 0);
        for (const auto &p : out) { ++deg[p.first]; ++deg[p.second]; }
        start_.assign(n + 1, 0);
        for (int64_t v = 0; v < n; ++v) start_[v + 1] = start_[v] + deg[v] + 2;
        inc_.assign(start_[n], 0);
        std::vector<int32_t> at(start_.begin(), start_.end() - 1);
        for (size_t i = 0; i < out.size(); ++i) {
            inc_[at[out[i].first]++] = (int32_t)i;
            inc_[at[out[i].second]++] = (int32_t)i;
        }
        neg = neg_.data();
        inc_start = start_.data();
        inc = inc_.data();
        if (as_keys) {
            keys_v.clear();
            for (const auto &p : out) keys_v.push_back(((uint64_t)(uint32_t)p.first << 32) | (uint32_t)p.second);
            keys = keys_v.data();
            nkeys = (int64_t)keys_v.size();
        }
    }
    bool near(const int64_t *lam, int64_t slack, PairList &out, std::string &) override
    {
        std::vector<int64_t> th(n);
        for (int64_t v = 0; v < n; ++v) {
            int64_t b[4] = {INT64_MAX, INT64_MAX, INT64_MAX, INT64_MAX};
            for (int64_t u = 0; u < n; ++u) {
                if (u == v) continue;
                int64_t x = z(lam, u, v);
                for (int j = 0; j < 4; ++j) if (x < b[j]) { int64_t t = b[j]; b[j] = x; x = t; }
            }
            th[v] = (b[3] > 0 ? b[3] : 0) + slack;
        }
        out.clear();
        for (int64_t u = 0; u < n; ++u)
            for (int64_t v = u + 1; v < n; ++v) {
                const int64_t x = z(lam, u, v);
                if (x <= th[u] || x <= th[v]) out.emplace_back((int32_t)u, (int32_t)v);
            }
        extras(lam, out);
        if (keys) out.clear();   // the pairs went as keys
        return true;
    }
    bool negative(const int64_t *lam, PairList &out, std::string &) override
    {
        out.clear();
        for (int64_t u = 0; u < n; ++u)
            for (int64_t v = u + 1; v < n; ++v)
                if (z(lam, u, v) < price_slack) out.emplace_back((int32_t)u, (int32_t)v);
        extras(lam, out);
        return true;
    }
};

FinishWork *g_work = nullptr;   // kept across calls (reuse = 1)
FinishWork *g_par = nullptr;    // four threads, chunked tail from one excess node (reuse = 2)
FinishWork *g_one = nullptr;    // the same on one thread (reuse = 3)

}  // namespace

// Returns the edge count (or -1 on failure); stats: paths, rounds, phases, candidates.
// b: node degrees (b-matching), or null for 2.
// bulk: the source also supplies costs and the bulk data; reuse 1: one
// workspace serves every call; reuse 2: the same with the flow's chunked
// single-source tail from the first excess node, on four threads; reuse 3:
// that on one thread.
extern "C" int64_t finish_cpu(int64_t n, const int32_t *xy, const int64_t *lam0, int64_t *lam_out, int64_t cap,
                              int32_t *eu, int32_t *ev, uint8_t *ex2, int64_t *stats, int32_t bulk, int32_t reuse,
                              const int32_t *b)
{
    BrutePairs src;
    src.xy = xy;
    src.n = n;
    src.bulk = bulk != 0;
    src.as_keys = bulk == 2;
    FinishResult r;
    if (reuse == 1 && !g_work) g_work = finish_work_create();
    if (reuse == 2 && !g_par) g_par = finish_work_create(4, 1);
    if (reuse == 3 && !g_one) g_one = finish_work_create(1, 1);
    FinishWork *w = reuse == 1 ? g_work : (reuse == 2 ? g_par : (reuse == 3 ? g_one : nullptr));
    finish_exact(xy, n, lam0, src, &r, w, b);
    if (!r.ok || (int64_t)r.eu.size() > cap) return -1;
    std::memcpy(lam_out, r.lam.data(), n * sizeof(int64_t));
    for (size_t i = 0; i < r.eu.size(); ++i) { eu[i] = r.eu[i]; ev[i] = r.ev[i]; ex2[i] = r.ex2[i]; }
    stats[0] = r.paths; stats[1] = r.rounds; stats[2] = r.phases; stats[3] = r.candidates;
    return (int64_t)r.eu.size();
}
