// Test harness: runs libf2m's exact finish (f2m_finish.cpp) on the CPU with a
// brute-force pair source, so the finish can be checked without a GPU.
#include "f2m_finish.h"

#include <cstring>

using namespace f2m;

namespace {

struct BrutePairs : PairSource {
    const int32_t *xy;
    int64_t n;
    int64_t z(const int64_t *lam, int64_t u, int64_t v) const
    {
        const int64_t dx = (int64_t)xy[2 * u] - xy[2 * v], dy = (int64_t)xy[2 * u + 1] - xy[2 * v + 1];
        return 2 * nint_sqrt_host(dx * dx + dy * dy) - lam[u] - lam[v];
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
        return true;
    }
    bool negative(const int64_t *lam, PairList &out, std::string &) override
    {
        out.clear();
        for (int64_t u = 0; u < n; ++u)
            for (int64_t v = u + 1; v < n; ++v)
                if (z(lam, u, v) < 0) out.emplace_back((int32_t)u, (int32_t)v);
        return true;
    }
};

}  // namespace

// Returns the edge count (or -1 on failure); stats: paths, rounds, phases, candidates.
extern "C" int64_t finish_cpu(int64_t n, const int32_t *xy, const int64_t *lam0, int64_t *lam_out, int64_t cap,
                              int32_t *eu, int32_t *ev, uint8_t *ex2, int64_t *stats)
{
    BrutePairs src;
    src.xy = xy;
    src.n = n;
    FinishResult r;
    finish_exact(xy, n, lam0, src, &r);
    if (!r.ok || (int64_t)r.eu.size() > cap) return -1;
    std::memcpy(lam_out, r.lam.data(), n * sizeof(int64_t));
    for (size_t i = 0; i < r.eu.size(); ++i) { eu[i] = r.eu[i]; ev[i] = r.ev[i]; ex2[i] = r.ex2[i]; }
    stats[0] = r.paths; stats[1] = r.rounds; stats[2] = r.phases; stats[3] = r.candidates;
    return (int64_t)r.eu.size();
}
