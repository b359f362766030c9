// Exact finish: primal-dual min-cost flow on the bipartite double cover of
// a candidate graph, warm-started from the GDP multipliers, with pricing on
// the complete graph.  See f2m_finish.h.
#include "f2m_finish.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <queue>
#include <chrono>
#include <iterator>

namespace f2m {

int64_t nint_sqrt_host(int64_t D)
{
    int64_t k = (int64_t)std::llround(std::sqrt((double)D));
    const int64_t d4 = 4 * D;
    while ((2 * k + 1) * (2 * k + 1) <= d4) ++k;
    while (k > 0 && (2 * k - 1) * (2 * k - 1) > d4) --k;
    return k;
}

namespace {

constexpr int64_t kInf = std::numeric_limits<int64_t>::max() / 4;

int64_t floor_half(int64_t x) { return x >= 0 ? x / 2 : -((-x + 1) / 2); }

// Node ids: left copy v' -> v, right copy u'' -> n + u.
// Arc 2i is a_i' -> b_i'', arc 2i+1 is b_i' -> a_i'' for candidate edge i.
class DoubleCover {
public:
    DoubleCover(const int32_t *xy, int64_t n, const int64_t *lam) : xy_(xy), n_(n), alpha_(n), beta_(n), ex_(2 * n, 0)
    {
        for (int64_t v = 0; v < n; ++v) {
            alpha_[v] = floor_half(lam[v]);
            beta_[v] = lam[v] - alpha_[v];
            ex_[v] = 2;        // left copies supply 2
            ex_[n + v] = -2;   // right copies demand 2
            src_.push_back(v);
        }
        build_adjacency();
    }

    int64_t edges() const { return (int64_t)ea_.size(); }

    // Adds new candidate edges (a sorted list of distinct pairs); arcs of
    // negative reduced cost start saturated.
    void add(const PairList &pl)
    {
        std::vector<uint64_t> fresh;
        fresh.reserve(pl.size());
        size_t j = 0;
        for (const auto &p : pl) {
            const int32_t a = std::min(p.first, p.second), b = std::max(p.first, p.second);
            if (a == b || a < 0 || b >= n_) continue;
            const uint64_t key = (uint64_t)a * (uint64_t)n_ + (uint64_t)b;
            while (j < keys_.size() && keys_[j] < key) ++j;
            if (j < keys_.size() && keys_[j] == key) continue;
            if (!fresh.empty() && fresh.back() >= key) {
                if (fresh.back() == key) continue;
                // unsorted input: fall back to a sorted copy
                std::vector<std::pair<int32_t, int32_t>> cp(pl.begin(), pl.end());
                std::sort(cp.begin(), cp.end());
                cp.erase(std::unique(cp.begin(), cp.end()), cp.end());
                add(cp);
                return;
            }
            fresh.push_back(key);
        }
        ea_.reserve(ea_.size() + fresh.size());
        eb_.reserve(eb_.size() + fresh.size());
        ec_.reserve(ec_.size() + fresh.size());
        y_.reserve(y_.size() + 2 * fresh.size());
        for (uint64_t key : fresh) {
            const int32_t a = (int32_t)(key / (uint64_t)n_), b = (int32_t)(key - (uint64_t)a * (uint64_t)n_);
            const int64_t dx = (int64_t)xy_[2 * a] - xy_[2 * b], dy = (int64_t)xy_[2 * a + 1] - xy_[2 * b + 1];
            const int64_t c = nint_sqrt_host(dx * dx + dy * dy);
            ea_.push_back(a);
            eb_.push_back(b);
            ec_.push_back(c);
            for (int d = 0; d < 2; ++d) {
                const int64_t k = 2 * ((int64_t)ea_.size() - 1) + d;
                const bool neg = red(k) < 0;
                y_.push_back(neg ? 1 : 0);
                if (neg) {
                    --ex_[tail(k)];
                    const int64_t h = n_ + head(k);
                    if (++ex_[h] == 1) src_.push_back(h);
                }
            }
        }
        if (fresh.empty()) return;
        std::vector<uint64_t> merged;
        merged.reserve(keys_.size() + fresh.size());
        std::merge(keys_.begin(), keys_.end(), fresh.begin(), fresh.end(), std::back_inserter(merged));
        keys_.swap(merged);
        build_adjacency();
    }

    // Min-cost flow on the current candidates; false when some excess
    // cannot reach a deficit (the candidate graph is too small).
    //
    // Primal-dual: while many excess nodes remain, one Dijkstra from all of
    // them sets the distance D of the nearest deficit, the potentials move
    // by min(dist, D) and every excess node augments along zero-reduced-cost
    // paths.  Once a phase augments few paths, the remaining excess nodes
    // are served one at a time (successive shortest paths): a Dijkstra from
    // the node alone stops at its nearest deficit and the path of the
    // search tree is augmented.  Both keep every residual reduced cost
    // nonnegative, so the end result is a minimum-cost flow.
    bool solve(int64_t &paths, int64_t &phases)
    {
        dist_.assign(2 * n_, kInf);
        par_.assign(2 * n_, -1);
        std::vector<int32_t> seen(2 * n_, 0);
        int32_t stamp = 0;
        bool single = false;
        for (;;) {
            // the excess nodes (the list only shrinks while solving)
            size_t w = 0;
            for (size_t i = 0; i < src_.size(); ++i)
                if (ex_[src_[i]] > 0) src_[w++] = src_[i];
            src_.resize(w);
            std::sort(src_.begin(), src_.end());
            src_.erase(std::unique(src_.begin(), src_.end()), src_.end());
            if (src_.empty()) return true;
            if (single) {
                for (int64_t s : src_) {
                    while (ex_[s] > 0) {
                        int64_t t;
                        if (!shortest(&s, 1, t)) return false;
                        ++phases;
                        for (int64_t x = t; x != s;) {   // flip the tree path back to s
                            const int64_t k = par_[x];
                            y_[k] ^= 1;
                            x = (x < n_) ? n_ + head(k) : tail(k);
                        }
                        --ex_[s];
                        ++ex_[t];
                        ++paths;
                    }
                }
                continue;
            }
            int64_t t;
            if (!shortest(src_.data(), src_.size(), t)) return false;
            ++phases;
            // unit augmentations along zero-reduced-cost paths
            ++stamp;
            int64_t found = 0;
            for (int64_t s : src_) {
                while (ex_[s] > 0 && seen[s] != stamp) {
                    if (!augment_from(s, stamp, seen)) break;
                    ++paths;
                    ++found;
                }
            }
            single = found < std::max<int64_t>(8, (int64_t)src_.size() / 16);
        }
    }

    void lam(std::vector<int64_t> &out) const
    {
        out.resize(n_);
        for (int64_t v = 0; v < n_; ++v) out[v] = alpha_[v] + A_ + beta_[v] + B_;
    }

    void x(std::vector<int32_t> &eu, std::vector<int32_t> &ev, std::vector<uint8_t> &ex2) const
    {
        std::vector<int64_t> order;
        for (int64_t i = 0; i < (int64_t)ea_.size(); ++i)
            if (y_[2 * i] + y_[2 * i + 1] > 0) order.push_back(i);
        std::sort(order.begin(), order.end(), [&](int64_t p, int64_t q) {
            return ea_[p] != ea_[q] ? ea_[p] < ea_[q] : eb_[p] < eb_[q];
        });
        eu.clear(); ev.clear(); ex2.clear();
        for (int64_t i : order) {
            eu.push_back(ea_[i]);
            ev.push_back(eb_[i]);
            ex2.push_back((uint8_t)(y_[2 * i] + y_[2 * i + 1]));
        }
    }

private:
    int64_t tail(int64_t k) const { return (k & 1) ? eb_[k >> 1] : ea_[k >> 1]; }
    int64_t head(int64_t k) const { return (k & 1) ? ea_[k >> 1] : eb_[k >> 1]; }
    // alpha, beta are stored relative to the global offsets A_, B_
    int64_t red(int64_t k) const { return ec_[k >> 1] - alpha_[tail(k)] - beta_[head(k)] - A_ - B_; }

    void build_adjacency()
    {
        // arc 2i leaves a_i' and enters b_i''; arc 2i+1 leaves b_i' and
        // enters a_i'': both copies of a node see the same arc count
        const int64_t e = (int64_t)ea_.size();
        lstart_.assign(n_ + 1, 0);
        for (int64_t i = 0; i < e; ++i) { ++lstart_[ea_[i] + 1]; ++lstart_[eb_[i] + 1]; }
        for (int64_t v = 0; v < n_; ++v) lstart_[v + 1] += lstart_[v];
        rstart_ = lstart_;
        larc_.resize(2 * e);
        rarc_.resize(2 * e);
        std::vector<int64_t> lp(lstart_.begin(), lstart_.end() - 1), rp(lp);
        for (int64_t i = 0; i < e; ++i) {
            const int64_t a = ea_[i], b = eb_[i];
            larc_[lp[a]++] = 2 * i;
            larc_[lp[b]++] = 2 * i + 1;
            rarc_[rp[b]++] = 2 * i;
            rarc_[rp[a]++] = 2 * i + 1;
        }
    }

    // Dijkstra on reduced costs from the given excess nodes up to the first
    // deficit t (at distance D); then p(x) moves by min(dist(x), D) for
    // every node (through the global offsets for the nodes not reached).
    // par_ holds the search tree's arcs.  False when no deficit is reachable.
    bool shortest(const int64_t *srcs, size_t ns, int64_t &t)
    {
        std::vector<int64_t> &dist = dist_;
        using Item = std::pair<int64_t, int64_t>;
        std::priority_queue<Item, std::vector<Item>, std::greater<Item>> pq;
        for (int64_t x : touched_) dist[x] = kInf;
        touched_.clear();
        for (size_t i = 0; i < ns; ++i) {
            const int64_t x = srcs[i];
            dist[x] = 0;
            par_[x] = -1;
            touched_.push_back(x);
            pq.push({0, x});
        }
        int64_t D = -1;
        while (!pq.empty()) {
            const auto [d, x] = pq.top();
            pq.pop();
            if (d != dist[x]) continue;
            if (ex_[x] < 0) { D = d; t = x; break; }
            relax_from(x, d, dist, touched_, pq);
        }
        if (D < 0) return false;
        for (int64_t x : touched_) {
            const int64_t d = dist[x];
            if (d >= D) continue;
            if (x < n_) alpha_[x] += D - d;
            else beta_[x - n_] -= D - d;
        }
        A_ -= D;
        B_ += D;
        return true;
    }

    template <typename PQ>
    void relax_from(int64_t x, int64_t d, std::vector<int64_t> &dist, std::vector<int64_t> &touched, PQ &pq)
    {
        if (x < n_) {   // left copy: arcs with y = 0, forward
            for (int64_t p = lstart_[x]; p < lstart_[x + 1]; ++p) {
                const int64_t k = larc_[p];
                if (y_[k]) continue;
                const int64_t to = n_ + head(k);
                const int64_t nd = d + red(k);
                if (nd < dist[to]) { if (dist[to] == kInf) touched.push_back(to); dist[to] = nd; par_[to] = k; pq.push({nd, to}); }
            }
        } else {        // right copy: arcs with y = 1, backward
            const int64_t u = x - n_;
            for (int64_t p = rstart_[u]; p < rstart_[u + 1]; ++p) {
                const int64_t k = rarc_[p];
                if (!y_[k]) continue;
                const int64_t to = tail(k);
                const int64_t nd = d - red(k);
                if (nd < dist[to]) { if (dist[to] == kInf) touched.push_back(to); dist[to] = nd; par_[to] = k; pq.push({nd, to}); }
            }
        }
    }

    // Depth-first search from s over zero-reduced-cost residual arcs to a
    // node with a deficit; flips the arcs of the path found.
    bool augment_from(int64_t s, int32_t stamp, std::vector<int32_t> &seen)
    {
        struct Frame { int64_t x, p, via; };
        std::vector<Frame> st;
        seen[s] = stamp;
        st.push_back({s, s < n_ ? lstart_[s] : rstart_[s - n_], -1});
        while (!st.empty()) {
            Frame &f = st.back();
            const int64_t x = f.x;
            if (x != s && ex_[x] < 0) {
                // flip the path
                for (size_t i = 1; i < st.size(); ++i) y_[st[i].via] ^= 1;
                --ex_[s];
                ++ex_[x];
                return true;
            }
            bool pushed = false;
            if (x < n_) {
                for (; f.p < lstart_[x + 1]; ++f.p) {
                    const int64_t k = larc_[f.p];
                    if (y_[k] || red(k) != 0) continue;
                    const int64_t to = n_ + head(k);
                    if (seen[to] == stamp) continue;
                    seen[to] = stamp;
                    ++f.p;
                    st.push_back({to, rstart_[head(k)], k});
                    pushed = true;
                    break;
                }
            } else {
                const int64_t u = x - n_;
                for (; f.p < rstart_[u + 1]; ++f.p) {
                    const int64_t k = rarc_[f.p];
                    if (!y_[k] || red(k) != 0) continue;
                    const int64_t to = tail(k);
                    if (seen[to] == stamp) continue;
                    seen[to] = stamp;
                    ++f.p;
                    st.push_back({to, lstart_[to], k});
                    pushed = true;
                    break;
                }
            }
            if (!pushed) st.pop_back();
        }
        return false;
    }

    const int32_t *xy_;
    int64_t n_;
    std::vector<int64_t> alpha_, beta_;
    int64_t A_ = 0, B_ = 0;          // global offsets of alpha and beta
    std::vector<int64_t> ex_;
    std::vector<int64_t> src_;       // nodes with excess (may hold stale entries)
    std::vector<int64_t> dist_, par_, touched_;
    std::vector<uint64_t> keys_;     // sorted keys a*n+b of the candidate edges
    std::vector<int32_t> ea_, eb_;
    std::vector<int64_t> ec_;
    std::vector<uint8_t> y_;
    std::vector<int64_t> lstart_, rstart_, larc_, rarc_;
};

}  // namespace

static double secs()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void finish_exact(const int32_t *xy, int64_t n, const int64_t *lam0, PairSource &src, FinishResult *out)
{
    FinishResult &r = *out;
    r = FinishResult();
    double t = secs();
    DoubleCover g(xy, n, lam0);
    std::string err;
    PairList pl;
    int64_t slack = 16;
    if (!src.near(lam0, slack, pl, err)) { r.msg = err; return; }
    r.t_collect += secs() - t;
    t = secs();
    g.add(pl);
    r.t_build += secs() - t;
    std::vector<int64_t> lam;
    for (int round = 0; round < 64; ++round) {
        ++r.rounds;
        t = secs();
        const bool ok = g.solve(r.paths, r.phases);
        r.t_flow += secs() - t;
        if (!ok) {
            // too few candidates for a degree-2 flow: widen around the current duals
            slack *= 4;
            g.lam(lam);
            pl.clear();
            t = secs();
            if (!src.near(lam.data(), slack, pl, err)) { r.msg = err; return; }
            r.t_collect += secs() - t;
            t = secs();
            g.add(pl);
            r.t_build += secs() - t;
            continue;
        }
        g.lam(lam);
        pl.clear();
        t = secs();
        if (!src.negative(lam.data(), pl, err)) { r.msg = err; return; }
        r.t_collect += secs() - t;
        const int64_t before = g.edges();
        t = secs();
        g.add(pl);
        r.t_build += secs() - t;
        if (g.edges() == before) {
            r.ok = true;
            r.lam = lam;
            g.x(r.eu, r.ev, r.ex2);
            r.candidates = g.edges();
            return;
        }
    }
    r.msg = "pricing did not converge in 64 rounds";
}

}  // namespace f2m
