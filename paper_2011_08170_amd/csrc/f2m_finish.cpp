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
#include <memory>

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

// candidate edge key: (a, b), a < b, in lexicographic order
uint64_t pair_key(int64_t a, int64_t b) { return ((uint64_t)a << 32) | (uint64_t)b; }

// Node ids: left copy v' -> v, right copy u'' -> n + u.
// Arc 2i is a_i' -> b_i'', arc 2i+1 is b_i' -> a_i'' for candidate edge i.
// One object serves one instance after another (reset): its buffers keep
// their capacity.
class DoubleCover {
public:
    void reset(const int32_t *xy, int64_t n, const int64_t *lam)
    {
        xy_ = xy;
        n_ = n;
        alpha_.resize(n);
        beta_.resize(n);
        ex_.resize(2 * n);
        src_.clear();
        for (int64_t v = 0; v < n; ++v) {
            alpha_[v] = floor_half(lam[v]);
            beta_[v] = lam[v] - alpha_[v];
            ex_[v] = 2;        // left copies supply 2
            ex_[n + v] = -2;   // right copies demand 2
            src_.push_back(v);
        }
        A_ = B_ = 0;
        keys_.clear();
        ea_.clear();
        eb_.clear();
        ec_.clear();
        y_.clear();
        start_.assign(n, 0);
        end_.assign(n, 0);
        cap_.assign(n, 0);
        inc_.clear();
        built_ = 0;
        // search state: dist is infinite outside the last search's touched set
        if ((int64_t)dist_.size() != 2 * n) {
            dist_.assign(2 * n, kInf);
        } else {
            for (int64_t x : touched_) dist_[x] = kInf;
        }
        touched_.clear();
        par_.resize(2 * n);
        if ((int64_t)seen_.size() != 2 * n) {
            seen_.assign(2 * n, 0);
            stamp_ = 0;
        }
    }

    int64_t edges() const { return (int64_t)ea_.size(); }

    // The first candidates in bulk: the pair source's costs, the initial
    // flow (negative-reduced-cost bits under the starting potentials) and
    // the incidence lists.  False (nothing changed) when the cover already
    // has edges or the data is missing or does not fit; then add() does the
    // work.
    bool add_bulk(const PairList &pl, const PairSource &src)
    {
        const int64_t m = (int64_t)pl.size();
        if (!ea_.empty() || m == 0 || !src.costs || !src.neg || !src.inc_start || !src.inc) return false;
        const int32_t *is = src.inc_start;
        if (is[0] != 0 || (int64_t)is[n_] != 2 * m + kSpare * n_) return false;
        for (int64_t v = 0; v < n_; ++v)
            if (is[v + 1] - is[v] < kSpare) return false;
        keys_.resize(m);
        for (int64_t i = 0; i < m; ++i) {
            const int64_t a = pl[i].first, b = pl[i].second;
            if (a < 0 || a >= b || b >= n_) return false;
            keys_[i] = pair_key(a, b);
            if (i > 0 && keys_[i - 1] >= keys_[i]) return false;
        }
        ea_.resize(m);
        eb_.resize(m);
        ec_.resize(m);
        y_.resize(2 * m);
        for (int64_t i = 0; i < m; ++i) {
            const int32_t a = pl[i].first, b = pl[i].second;
            ea_[i] = a;
            eb_[i] = b;
            ec_[i] = src.costs[i];
            const uint8_t f = src.neg[i];
            y_[2 * i] = f & 1;
            y_[2 * i + 1] = (f >> 1) & 1;
            if (f & 1) {
                --ex_[a];
                if (++ex_[n_ + b] == 1) src_.push_back(n_ + b);
            }
            if (f & 2) {
                --ex_[b];
                if (++ex_[n_ + a] == 1) src_.push_back(n_ + a);
            }
        }
        for (int64_t v = 0; v < n_; ++v) {
            start_[v] = is[v];
            end_[v] = is[v + 1] - kSpare;
            cap_[v] = is[v + 1];
        }
        inc_.assign(src.inc, src.inc + is[n_]);
        built_ = m;
        return true;
    }

    // Adds new candidate edges (pairs with costs, or null: computed here);
    // pairs already present are skipped.  Arcs of negative reduced cost
    // start saturated.
    void add(const PairList &pl, const int32_t *costs)
    {
        fresh_.clear();
        fresh_c_.clear();
        size_t j = 0;
        uint64_t prev = 0;
        bool have_prev = false;
        for (size_t q = 0; q < pl.size(); ++q) {
            const int32_t a = std::min(pl[q].first, pl[q].second), b = std::max(pl[q].first, pl[q].second);
            if (a == b || a < 0 || b >= n_) continue;
            const uint64_t key = pair_key(a, b);
            if (have_prev && key <= prev) {
                if (key == prev) continue;
                // unsorted input: go again over a sorted copy (costs recomputed)
                PairList cp;
                cp.reserve(pl.size());
                for (const auto &p : pl) cp.emplace_back(std::min(p.first, p.second), std::max(p.first, p.second));
                std::sort(cp.begin(), cp.end());
                cp.erase(std::unique(cp.begin(), cp.end()), cp.end());
                fresh_.clear();
                fresh_c_.clear();
                add(cp, nullptr);
                return;
            }
            prev = key;
            have_prev = true;
            j = (size_t)(std::lower_bound(keys_.begin() + j, keys_.end(), key) - keys_.begin());
            if (j < keys_.size() && keys_[j] == key) continue;
            fresh_.push_back(key);
            fresh_c_.push_back(costs ? costs[q] : -1);
        }
        if (fresh_.empty()) return;
        for (size_t q = 0; q < fresh_.size(); ++q) {
            const int32_t a = (int32_t)(fresh_[q] >> 32), b = (int32_t)(fresh_[q] & 0xffffffffULL);
            int64_t c = fresh_c_[q];
            if (!costs) {
                const int64_t dx = (int64_t)xy_[2 * a] - xy_[2 * b], dy = (int64_t)xy_[2 * a + 1] - xy_[2 * b + 1];
                c = nint_sqrt_host(dx * dx + dy * dy);
            }
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
        merged_.resize(keys_.size() + fresh_.size());
        std::merge(keys_.begin(), keys_.end(), fresh_.begin(), fresh_.end(), merged_.begin());
        keys_.swap(merged_);
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
        bool single = false, first = true;
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
            // the starting potentials are feasible, so the first pass
            // augments along the zero-reduced-cost paths they already have;
            // later passes follow a Dijkstra that moves the potentials
            if (!first) {
                int64_t t;
                if (!shortest(src_.data(), src_.size(), t)) return false;
                ++phases;
            }
            first = false;
            // unit augmentations along zero-reduced-cost paths
            const int32_t stamp = ++stamp_;
            int64_t found = 0;
            for (int64_t s : src_) {
                while (ex_[s] > 0 && seen_[s] != stamp) {
                    if (!augment_from(s, stamp)) break;
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

    // the edges with flow, in candidate order
    void x(std::vector<int32_t> &eu, std::vector<int32_t> &ev, std::vector<uint8_t> &ex2) const
    {
        eu.clear();
        ev.clear();
        ex2.clear();
        for (int64_t i = 0; i < (int64_t)ea_.size(); ++i) {
            const int f = y_[2 * i] + y_[2 * i + 1];
            if (f == 0) continue;
            eu.push_back(ea_[i]);
            ev.push_back(eb_[i]);
            ex2.push_back((uint8_t)f);
        }
    }

private:
    int64_t tail(int64_t k) const { return (k & 1) ? eb_[k >> 1] : ea_[k >> 1]; }
    int64_t head(int64_t k) const { return (k & 1) ? ea_[k >> 1] : eb_[k >> 1]; }
    // alpha, beta are stored relative to the global offsets A_, B_
    int64_t red(int64_t k) const { return ec_[k >> 1] - alpha_[tail(k)] - beta_[head(k)] - A_ - B_; }

    // Incident edges per node, in increasing edge index: both copies of a
    // node use the same list (edge e leaves a_e' and b_e' and enters b_e''
    // and a_e'').  Node v's list is inc_[start_[v], end_[v]) with free slots
    // up to cap_[v].  Edges [built_, size) are new since the last call: they
    // go into the free slots (new edges have the largest indexes, so every
    // list stays sorted); a full list first moves to the end of inc_ with
    // room to grow.  Without bulk lists the first call builds them all by a
    // counting sort, kSpare free slots each.
    static constexpr int64_t kSpare = 2;
    void build_adjacency()
    {
        const int64_t e = (int64_t)ea_.size();
        if (built_ == 0 && inc_.empty()) {
            int64_t at = 0;
            for (int64_t v = 0; v < n_; ++v) end_[v] = 0;
            for (int64_t i = 0; i < e; ++i) { ++end_[ea_[i]]; ++end_[eb_[i]]; }
            for (int64_t v = 0; v < n_; ++v) {
                start_[v] = at;
                at += end_[v] + kSpare;
                cap_[v] = at;
                end_[v] = start_[v];
            }
            inc_.resize(at);
            for (int64_t i = 0; i < e; ++i) {
                inc_[end_[ea_[i]]++] = (int32_t)i;
                inc_[end_[eb_[i]]++] = (int32_t)i;
            }
        } else {
            for (int64_t i = built_; i < e; ++i) {
                place(ea_[i], (int32_t)i);
                place(eb_[i], (int32_t)i);
            }
        }
        built_ = e;
    }

    void place(int64_t v, int32_t i)
    {
        if (end_[v] == cap_[v]) {
            const int64_t len = end_[v] - start_[v], ncap = 2 * len + kSpare + 2;
            const int64_t at = (int64_t)inc_.size();
            inc_.resize(at + ncap);
            std::copy(inc_.begin() + start_[v], inc_.begin() + end_[v], inc_.begin() + at);
            start_[v] = at;
            end_[v] = at + len;
            cap_[v] = at + ncap;
        }
        inc_[end_[v]++] = i;
    }

    // Dijkstra on reduced costs from the given excess nodes up to the first
    // deficit t (at distance D); then p(x) moves by min(dist(x), D) for
    // every node (through the global offsets for the nodes not reached).
    // par_ holds the search tree's arcs.  False when no deficit is reachable.
    bool shortest(const int64_t *srcs, size_t ns, int64_t &t)
    {
        std::vector<int64_t> &dist = dist_;
        for (int64_t x : touched_) dist[x] = kInf;
        touched_.clear();
        // nodes at the current distance wait in a plain list (zero-cost
        // arcs are common here); larger distances go through the heap
        std::vector<int64_t> &cur = cur_;
        cur.clear();
        heap_.clear();
        int64_t dcur = 0;
        for (size_t i = 0; i < ns; ++i) {
            const int64_t x = srcs[i];
            dist[x] = 0;
            par_[x] = -1;
            touched_.push_back(x);
            cur.push_back(x);
        }
        int64_t D = -1;
        for (;;) {
            int64_t x;
            if (!cur.empty()) {
                x = cur.back();
                cur.pop_back();
                if (dist[x] != dcur) continue;
            } else {
                if (heap_.empty()) break;
                std::pop_heap(heap_.begin(), heap_.end(), std::greater<Item>());
                const Item it = heap_.back();
                heap_.pop_back();
                if (it.first != dist[it.second]) continue;
                dcur = it.first;
                x = it.second;
            }
            if (ex_[x] < 0) { D = dcur; t = x; break; }
            relax_from(x, dcur);
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

    void push(int64_t to, int64_t nd, int64_t dcur, int64_t k)
    {
        if (nd >= dist_[to]) return;
        if (dist_[to] == kInf) touched_.push_back(to);
        dist_[to] = nd;
        par_[to] = k;
        if (nd == dcur) {
            cur_.push_back(to);
        } else {
            heap_.push_back({nd, to});
            std::push_heap(heap_.begin(), heap_.end(), std::greater<Item>());
        }
    }

    // the arc of incident edge ie that leaves v' (left) or enters v''
    int64_t out_arc(int64_t ie, int64_t v) const { return 2 * ie + (ea_[ie] != v); }
    int64_t in_arc(int64_t ie, int64_t v) const { return 2 * ie + (eb_[ie] != v); }
    int64_t other(int64_t ie, int64_t v) const { return (int64_t)ea_[ie] + eb_[ie] - v; }

    void relax_from(int64_t x, int64_t d)
    {
        if (x < n_) {   // left copy: arcs with y = 0, forward
            for (int64_t p = start_[x]; p < end_[x]; ++p) {
                const int64_t ie = inc_[p], k = out_arc(ie, x);
                if (y_[k]) continue;
                push(n_ + other(ie, x), d + red(k), d, k);
            }
        } else {        // right copy: arcs with y = 1, backward
            const int64_t u = x - n_;
            for (int64_t p = start_[u]; p < end_[u]; ++p) {
                const int64_t ie = inc_[p], k = in_arc(ie, u);
                if (!y_[k]) continue;
                push(other(ie, u), d - red(k), d, k);
            }
        }
    }

    // Depth-first search from s over zero-reduced-cost residual arcs to a
    // node with a deficit; flips the arcs of the path found.
    bool augment_from(int64_t s, int32_t stamp)
    {
        std::vector<int32_t> &seen = seen_;
        std::vector<Frame> &st = frames_;
        st.clear();
        seen[s] = stamp;
        st.push_back({s, start_[s < n_ ? s : s - n_], -1});
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
                for (; f.p < end_[x]; ++f.p) {
                    const int64_t ie = inc_[f.p], k = out_arc(ie, x);
                    if (y_[k] || red(k) != 0) continue;
                    const int64_t w = other(ie, x), to = n_ + w;
                    if (seen[to] == stamp) continue;
                    seen[to] = stamp;
                    ++f.p;
                    st.push_back({to, start_[w], k});
                    pushed = true;
                    break;
                }
            } else {
                const int64_t u = x - n_;
                for (; f.p < end_[u]; ++f.p) {
                    const int64_t ie = inc_[f.p], k = in_arc(ie, u);
                    if (!y_[k] || red(k) != 0) continue;
                    const int64_t to = other(ie, u);
                    if (seen[to] == stamp) continue;
                    seen[to] = stamp;
                    ++f.p;
                    st.push_back({to, start_[to], k});
                    pushed = true;
                    break;
                }
            }
            if (!pushed) st.pop_back();
        }
        return false;
    }

    const int32_t *xy_ = nullptr;
    int64_t n_ = 0;
    std::vector<int64_t> alpha_, beta_;
    int64_t A_ = 0, B_ = 0;          // global offsets of alpha and beta
    std::vector<int64_t> ex_;
    std::vector<int64_t> src_;       // nodes with excess (may hold stale entries)
    using Item = std::pair<int64_t, int64_t>;
    std::vector<int64_t> dist_, par_, touched_, cur_;
    std::vector<Item> heap_;
    std::vector<uint64_t> keys_;     // sorted keys (pair_key) of the candidate edges
    std::vector<uint64_t> fresh_, merged_;
    std::vector<int32_t> fresh_c_;
    std::vector<int32_t> ea_, eb_;
    std::vector<int64_t> ec_;
    std::vector<uint8_t> y_;
    std::vector<int64_t> start_, end_, cap_;   // incident-edge lists (see build_adjacency)
    std::vector<int32_t> inc_;
    int64_t built_ = 0;              // edges covered by the lists
    std::vector<int32_t> seen_;      // augmentation pass stamps
    int32_t stamp_ = 0;
    struct Frame { int64_t x, p, via; };
    std::vector<Frame> frames_;
};

}  // namespace

static double secs()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct FinishWork {
    DoubleCover g;
    PairList pl;
    std::vector<int64_t> lam;
};

FinishWork *finish_work_create() { return new FinishWork(); }

void finish_work_destroy(FinishWork *work) { delete work; }

void finish_exact(const int32_t *xy, int64_t n, const int64_t *lam0, PairSource &src, FinishResult *out,
                  FinishWork *work)
{
    std::unique_ptr<FinishWork> own;
    if (!work) {
        own.reset(new FinishWork());
        work = own.get();
    }
    FinishResult &r = *out;
    r.ok = false;
    r.msg.clear();
    r.lam.clear();
    r.eu.clear();
    r.ev.clear();
    r.ex2.clear();
    r.paths = r.rounds = r.phases = r.candidates = 0;
    r.t_collect = r.t_build = r.t_flow = 0.0;
    double t = secs();
    DoubleCover &g = work->g;
    g.reset(xy, n, lam0);
    PairList &pl = work->pl;
    std::vector<int64_t> &lam = work->lam;
    std::string err;
    pl.clear();
    int64_t slack = 16;
    src.want_bulk = true;
    const bool got = src.near(lam0, slack, pl, err);
    src.want_bulk = false;
    if (!got) { r.msg = err; return; }
    r.t_collect += secs() - t;
    t = secs();
    if (!g.add_bulk(pl, src)) g.add(pl, src.costs);
    r.t_build += secs() - t;
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
            g.add(pl, src.costs);
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
        g.add(pl, src.costs);
        r.t_build += secs() - t;
        if (g.edges() == before) {
            r.ok = true;
            r.lam.assign(lam.begin(), lam.end());
            g.x(r.eu, r.ev, r.ex2);
            r.candidates = g.edges();
            return;
        }
    }
    r.msg = "pricing did not converge in 64 rounds";
}

}  // namespace f2m
