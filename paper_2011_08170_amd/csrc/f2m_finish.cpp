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
#include <atomic>
#include <condition_variable>
#include <exception>
#include <functional>
#include <mutex>
#include <memory>
#include <thread>

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


// A fixed set of threads that run one function at a time, fn(worker) for
// workers 1 .. T-1 while the caller runs fn(0); they stay for the owner's
// lifetime, so a solve starts no thread.
class Pool {
public:
    ~Pool()
    {
        {
            std::lock_guard<std::mutex> lk(m_);
            quit_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }

    void run(int T, const std::function<void(int)> &fn)
    {
        if (T <= 1) {
            fn(0);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(m_);
            // a new thread starts from the generation before this run's
            while ((int)th_.size() < T - 1) {
                const int id = (int)th_.size() + 1;
                th_.emplace_back([this, id, g = gen_] { loop(id, g); });
            }
            fn_ = &fn;
            want_ = T - 1;
            done_ = 0;
            err_ = nullptr;
            ++gen_;
        }
        cv_.notify_all();
        // the workers use fn (and what it refers to) until they report done:
        // wait for them whatever fn(0) does, then rethrow the first error
        std::exception_ptr mine;
        try {
            fn(0);
        } catch (...) {
            mine = std::current_exception();
        }
        std::unique_lock<std::mutex> lk(m_);
        cv_done_.wait(lk, [&] { return done_ == want_; });
        fn_ = nullptr;
        if (!mine) mine = err_;
        err_ = nullptr;
        lk.unlock();
        if (mine) std::rethrow_exception(mine);
    }

private:
    void loop(int id, uint64_t seen)
    {
        std::unique_lock<std::mutex> lk(m_);
        for (;;) {
            cv_.wait(lk, [&] { return quit_ || gen_ != seen; });
            if (quit_) return;
            seen = gen_;
            if (id > want_) continue;   // not needed this time
            const std::function<void(int)> *f = fn_;
            lk.unlock();
            std::exception_ptr e;
            try {
                (*f)(id);
            } catch (...) {
                e = std::current_exception();
            }
            lk.lock();
            if (e && !err_) err_ = e;
            if (++done_ == want_) cv_done_.notify_one();
        }
    }

    std::mutex m_;
    std::condition_variable cv_, cv_done_;
    std::vector<std::thread> th_;
    const std::function<void(int)> *fn_ = nullptr;
    int want_ = 0, done_ = 0;
    std::exception_ptr err_;   // first error a worker threw in this run
    uint64_t gen_ = 0;
    bool quit_ = false;
};

// Node ids: left copy v' -> v, right copy u'' -> n + u.
// Arc 2i is a_i' -> b_i'', arc 2i+1 is b_i' -> a_i'' for candidate edge i.
// The data a search touches per arc sit together: one record per edge
// (ends, cost, the flow of its two arcs) and one per node copy (potential,
// excess, search state).  One object serves one instance after another
// (reset): its buffers keep their capacity.
class DoubleCover {
public:
    // b: every node's degree (right-hand side of its row), or null for 2
    void reset(const int32_t *xy, int64_t n, const int64_t *lam, const int32_t *b)
    {
        xy_ = xy;
        n_ = n;
        b_ = b;
        // search state: dist is infinite outside the last search's touched
        // set, so every copy's dist is reset (one pass over the records that
        // are written anyway, on the pool's threads)
        if ((int64_t)cp_.size() != 2 * n) cp_.assign(2 * n, Copy{});
        touched_.clear();
        src_.resize(n);
        start_.resize(n);
        end_.resize(n);
        cap_.resize(n);
        parallel_for(n, [&](int64_t lo, int64_t hi) {
            for (int64_t v = lo; v < hi; ++v) {
                const int64_t al = floor_half(lam[v]);
                Copy &l = cp_[v], &r = cp_[n + v];
                l.pot = al;            // alpha_v
                l.ex = deg(v);         // left copies supply b_v
                l.dist = kInf;
                r.pot = lam[v] - al;   // beta_v
                r.ex = -deg(v);        // right copies demand b_v
                r.dist = kInf;
                src_[v] = v;
                start_[v] = end_[v] = cap_[v] = 0;
            }
        });
        A_ = B_ = 0;
        keys_.clear();
        extra_.clear();
        e_.clear();
        inc_.clear();
        built_ = 0;
    }

    int64_t edges() const { return (int64_t)e_.size(); }
    int32_t deg(int64_t v) const { return b_ ? b_[v] : 2; }

    // The first candidates in bulk: the pair source's keys and costs, the
    // initial flow (negative-reduced-cost bits under the starting
    // potentials) and the incidence lists.  False (nothing changed) when
    // the cover already has edges or the data is missing or does not fit;
    // then add() does the work.
    bool add_bulk(const PairList &pl, const PairSource &src)
    {
        // the pairs come as keys or as the list
        const uint64_t *sk = src.keys;
        const int64_t m = sk ? src.nkeys : (int64_t)pl.size();
        if (!e_.empty() || m == 0 || !src.costs || !src.neg || !src.inc_start || !src.inc) return false;
        const int32_t *is = src.inc_start;
        if (is[0] != 0 || (int64_t)is[n_] != 2 * m + kSpare * n_) return false;
        std::atomic<bool> ok{true};
        // the pairs: in range, strictly increasing; edge records
        keys_.resize(m);
        e_.resize(m);
        parallel_for(m, [&](int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) {
                const int32_t a = sk ? (int32_t)(sk[i] >> 32) : pl[i].first;
                const int32_t b = sk ? (int32_t)(sk[i] & 0xffffffffULL) : pl[i].second;
                const uint64_t pk = i == 0 ? 0 : (sk ? sk[i - 1] : pair_key(pl[i - 1].first, pl[i - 1].second));
                if (a < 0 || a >= b || b >= n_ || (i > 0 && pk >= pair_key(a, b))) {
                    ok = false;
                    return;
                }
                keys_[i] = pair_key(a, b);
                const uint8_t f = src.neg[i];
                Edge &ed = e_[i];
                ed.a = a;
                ed.b = b;
                ed.c = src.costs[i];
                ed.y[0] = f & 1;
                ed.y[1] = (f >> 1) & 1;
            }
        });
        // per node: its list (copied, with its free slots), and the excess
        // of both copies from the arcs its list's edges saturate
        if (ok) {
            parallel_for(n_, [&](int64_t lo, int64_t hi) {
                for (int64_t v = lo; v < hi; ++v) {
                    const int64_t s0 = is[v], s1 = is[v + 1] - kSpare;
                    if (s1 < s0) { ok = false; return; }
                    int32_t out = 0, in = 0;
                    for (int64_t p = s0; p < s1; ++p) {
                        const int32_t ie = src.inc[p];
                        if (ie < 0 || ie >= m || (e_[ie].a != v && e_[ie].b != v)) { ok = false; return; }
                        const Edge &ed = e_[ie];
                        out += ed.y[ed.a != v];   // the arc that leaves v'
                        in += ed.y[ed.b != v];    // the arc that enters v''
                    }
                    cp_[v].ex = deg(v) - out;
                    cp_[n_ + v].ex = -deg(v) + in;
                    start_[v] = s0;
                    end_[v] = s1;
                    cap_[v] = is[v + 1];
                }
            });
        }
        if (!ok) {
            keys_.clear();
            e_.clear();
            for (int64_t v = 0; v < n_; ++v) {
                cp_[v].ex = deg(v);
                cp_[n_ + v].ex = -deg(v);
                start_[v] = end_[v] = cap_[v] = 0;
            }
            return false;
        }
        // the lists (copied in ranges) and the nodes with excess (gathered
        // in ranges, then joined in node order)
        inc_.resize(is[n_]);
        parallel_for(is[n_], [&](int64_t lo, int64_t hi) { std::copy(src.inc + lo, src.inc + hi, inc_.begin() + lo); });
        const int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads_, n_ / 4096));
        std::vector<std::vector<int64_t>> part(T);
        auto gather = [&](int w) {
            for (int64_t v = n_ * w / T; v < n_ * (w + 1) / T; ++v)
                if (cp_[n_ + v].ex > 0) part[w].push_back(n_ + v);
        };
        if (T == 1) gather(0);
        else pool_.run(T, gather);
        for (const auto &q : part) src_.insert(src_.end(), q.begin(), q.end());
        built_ = m;
        return true;
    }

    // f(lo, hi) over [0, count) split in contiguous ranges, one per thread
    template <class F>
    void parallel_for(int64_t count, F f)
    {
        const int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads_, count / 4096));
        if (T == 1) {
            f(0, count);
            return;
        }
        pool_.run(T, [&](int w) { f(count * w / T, count * (w + 1) / T); });
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
            if (std::binary_search(extra_.begin(), extra_.end(), key)) continue;
            fresh_.push_back(key);
            fresh_c_.push_back(costs ? costs[q] : -1);
        }
        if (fresh_.empty()) return;
        for (size_t q = 0; q < fresh_.size(); ++q) {
            Edge ed;
            ed.a = (int32_t)(fresh_[q] >> 32);
            ed.b = (int32_t)(fresh_[q] & 0xffffffffULL);
            if (costs) {
                ed.c = fresh_c_[q];
            } else {
                const int64_t dx = (int64_t)xy_[2 * ed.a] - xy_[2 * ed.b];
                const int64_t dy = (int64_t)xy_[2 * ed.a + 1] - xy_[2 * ed.b + 1];
                ed.c = (int32_t)nint_sqrt_host(dx * dx + dy * dy);
            }
            for (int d = 0; d < 2; ++d) {
                const int64_t t = d ? ed.b : ed.a, h = d ? ed.a : ed.b;
                const bool neg = ed.c - cp_[t].pot - cp_[n_ + h].pot - A_ - B_ < 0;
                ed.y[d] = neg ? 1 : 0;
                if (neg) {
                    --cp_[t].ex;
                    if (++cp_[n_ + h].ex == 1) src_.push_back(n_ + h);
                }
            }
            e_.push_back(ed);
        }
        merged_.resize(extra_.size() + fresh_.size());
        std::merge(extra_.begin(), extra_.end(), fresh_.begin(), fresh_.end(), merged_.begin());
        extra_.swap(merged_);
        if (extra_.size() * 8 > keys_.size()) {
            merged_.resize(keys_.size() + extra_.size());
            std::merge(keys_.begin(), keys_.end(), extra_.begin(), extra_.end(), merged_.begin());
            keys_.swap(merged_);
            extra_.clear();
        }
        build_adjacency();
    }

    bool has_key(uint64_t key) const
    {
        return std::binary_search(keys_.begin(), keys_.end(), key) ||
               std::binary_search(extra_.begin(), extra_.end(), key);
    }

    // Whether some pair of pl that is not a candidate yet has Z < 0 under
    // lam (costs: the pairs' costs, or null: computed here)
    bool fresh_negative(const PairList &pl, const int32_t *costs, const std::vector<int64_t> &lam) const
    {
        for (size_t q = 0; q < pl.size(); ++q) {
            const int32_t a = std::min(pl[q].first, pl[q].second), b = std::max(pl[q].first, pl[q].second);
            if (a == b || a < 0 || b >= n_) continue;
            if (has_key(pair_key(a, b))) continue;
            int64_t c;
            if (costs) {
                c = costs[q];
            } else {
                const int64_t dx = (int64_t)xy_[2 * a] - xy_[2 * b], dy = (int64_t)xy_[2 * a + 1] - xy_[2 * b + 1];
                c = nint_sqrt_host(dx * dx + dy * dy);
            }
            if (2 * c - lam[a] - lam[b] < 0) return true;
        }
        return false;
    }

    // Min-cost flow on the current candidates; false when some excess
    // cannot reach a deficit (the candidate graph is too small).
    //
    // Primal-dual from feasible potentials (every residual reduced cost
    // nonnegative).  The first pass augments unit paths along the
    // zero-reduced-cost arcs the starting potentials already have.  The
    // excess nodes left then lie at many different distances from their
    // deficits (one Dijkstra from all of them would serve only the nearest
    // few: measured at n = 100k, such a phase found 11 paths for 3000
    // excess nodes), so they are served one at a time (successive shortest
    // paths): a Dijkstra from the node alone stops at its nearest deficit,
    // the potentials move by min(dist, D) and the path of the search tree
    // is augmented.  Both keep every residual reduced cost nonnegative, so
    // the end result is a minimum-cost flow.  With many excess nodes both
    // run by chunks first (in parallel); the first pass then leaves the rest
    // to the tail, the tail to its sequential part.
    bool solve(int64_t &paths, int64_t &phases)
    {
        bool first = true;
        for (;;) {
            // the excess nodes (the list only shrinks while solving)
            size_t w = 0;
            for (size_t i = 0; i < src_.size(); ++i)
                if (cp_[src_[i]].ex > 0) src_[w++] = src_[i];
            src_.resize(w);
            std::sort(src_.begin(), src_.end());
            src_.erase(std::unique(src_.begin(), src_.end()), src_.end());
            if (src_.empty()) return true;
            if (first) {
                first = false;
                // by chunks when there are many excess nodes: the ones left
                // then go straight to the tail (which finds their
                // zero-distance paths too, and runs by chunks as well)
                if ((int64_t)src_.size() >= parallel_min_) {
                    zero_chunks(paths);
                    continue;
                }
                const int32_t stamp = ++stamp_;
                for (int64_t s : src_) {
                    while (cp_[s].ex > 0 && cp_[s].seen != stamp) {
                        if (!augment_from(s, stamp)) break;
                        ++paths;
                    }
                }
                continue;
            }
            if ((int64_t)src_.size() >= parallel_min_) {
                single_chunks(paths, phases);
                if (src_.empty()) return true;
            }
            for (int64_t s : src_) {
                while (cp_[s].ex > 0) {
                    int64_t t;
                    if (!shortest(&s, 1, t)) return false;
                    ++phases;
                    for (int64_t x = t; x != s;) {   // flip the tree path back to s
                        const int64_t k = cp_[x].par;
                        Edge &ed = e_[k >> 1];
                        ed.y[k & 1] ^= 1;
                        x = (x < n_) ? n_ + head(ed, k & 1) : tail(ed, k & 1);
                    }
                    --cp_[s].ex;
                    ++cp_[t].ex;
                    ++paths;
                }
            }
        }
    }

    void set_threads(int t, int64_t parallel_min)
    {
        threads_ = std::max(1, t);
        parallel_min_ = std::max<int64_t>(1, parallel_min);
    }

    void lam(std::vector<int64_t> &out)
    {
        out.resize(n_);
        int64_t *o = out.data();
        parallel_for(n_, [&](int64_t lo, int64_t hi) {
            for (int64_t v = lo; v < hi; ++v) o[v] = cp_[v].pot + A_ + cp_[n_ + v].pot + B_;
        });
    }

    // the edges with flow, in candidate order
    void x(RawVec<int32_t> &eu, RawVec<int32_t> &ev, RawVec<uint8_t> &ex2)
    {
        // in ranges of edges on the pool's threads: each range counts its
        // edges with flow, then writes them from its offset (only those: the
        // slot after a range's last one is the next range's first)
        const int64_t m = (int64_t)e_.size();
        const int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads_, m / 8192));
        std::vector<int64_t> at(T + 1, 0);
        auto range = [&](int w, bool write) {
            const int64_t lo = m * w / T, hi = m * (w + 1) / T;
            int64_t k = write ? at[w] : 0;
            for (int64_t i = lo; i < hi; ++i) {
                const Edge &ed = e_[i];
                const int f = ed.y[0] + ed.y[1];
                if (f == 0) continue;
                if (write) {
                    eu[k] = ed.a;
                    ev[k] = ed.b;
                    ex2[k] = (uint8_t)f;
                }
                ++k;
            }
            if (!write) at[w + 1] = k;
        };
        if (T == 1) range(0, false);
        else pool_.run(T, [&](int w) { range(w, false); });
        for (int w = 0; w < T; ++w) at[w + 1] += at[w];
        eu.resize(at[T]);
        ev.resize(at[T]);
        ex2.resize(at[T]);
        if (T == 1) range(0, true);
        else pool_.run(T, [&](int w) { range(w, true); });
    }

private:
    using Item = std::pair<int64_t, int64_t>;   // (distance, node copy)
    struct Frame { int64_t x, p, via; };        // depth-first search stack entry
    struct Edge {
        int32_t a, b;      // a < b
        int32_t c;         // cost
        uint8_t y[2];      // flow of arc a'->b'' (0) and b'->a'' (1)
        uint8_t pad[2];
    };
    struct Copy {
        int64_t pot;       // alpha (left copy) or beta (right copy), before the global offsets
        int64_t dist = kInf;
        int64_t par = -1;  // arc of the search tree into this copy
        int32_t ex = 0;    // excess
        int32_t seen = 0;  // augmentation pass stamp
    };
    static_assert(sizeof(Edge) == 16 && sizeof(Copy) == 32, "records share cache lines evenly");

    static int64_t tail(const Edge &ed, int d) { return d ? ed.b : ed.a; }
    static int64_t head(const Edge &ed, int d) { return d ? ed.a : ed.b; }
    // reduced cost of arc d of edge ed: c - alpha_tail - beta_head (with
    // the global offsets A_ of alpha and B_ of beta)
    int64_t red(const Edge &ed, int d) const
    {
        return ed.c - cp_[tail(ed, d)].pot - cp_[n_ + head(ed, d)].pot - A_ - B_;
    }

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
        const int64_t e = (int64_t)e_.size();
        if (built_ == 0 && inc_.empty()) {
            int64_t at = 0;
            for (int64_t v = 0; v < n_; ++v) end_[v] = 0;
            for (int64_t i = 0; i < e; ++i) { ++end_[e_[i].a]; ++end_[e_[i].b]; }
            for (int64_t v = 0; v < n_; ++v) {
                start_[v] = at;
                at += end_[v] + kSpare;
                cap_[v] = at;
                end_[v] = start_[v];
            }
            inc_.resize(at);
            for (int64_t i = 0; i < e; ++i) {
                inc_[end_[e_[i].a]++] = (int32_t)i;
                inc_[end_[e_[i].b]++] = (int32_t)i;
            }
        } else {
            for (int64_t i = built_; i < e; ++i) {
                place(e_[i].a, (int32_t)i);
                place(e_[i].b, (int32_t)i);
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
    // The tree arcs are in Copy::par.  False when no deficit is reachable.
    bool shortest(const int64_t *srcs, size_t ns, int64_t &t)
    {
        for (int64_t x : touched_) cp_[x].dist = kInf;
        touched_.clear();
        // nodes at the current distance wait in a plain list (zero-cost
        // arcs are common here); larger distances go through the heap
        cur_.clear();
        heap_.clear();
        int64_t dcur = 0;
        for (size_t i = 0; i < ns; ++i) {
            const int64_t x = srcs[i];
            cp_[x].dist = 0;
            cp_[x].par = -1;
            touched_.push_back(x);
            cur_.push_back(x);
        }
        int64_t D = -1;
        for (;;) {
            int64_t x;
            if (!cur_.empty()) {
                x = cur_.back();
                cur_.pop_back();
                if (cp_[x].dist != dcur) continue;
            } else {
                if (heap_.empty()) break;
                std::pop_heap(heap_.begin(), heap_.end(), std::greater<Item>());
                const Item it = heap_.back();
                heap_.pop_back();
                if (it.first != cp_[it.second].dist) continue;
                dcur = it.first;
                x = it.second;
            }
            if (cp_[x].ex < 0) { D = dcur; t = x; break; }
            relax_from(x, dcur);
        }
        if (D < 0) return false;
        for (int64_t x : touched_) {
            Copy &c = cp_[x];
            if (c.dist >= D) continue;
            if (x < n_) c.pot += D - c.dist;
            else c.pot -= D - c.dist;
        }
        A_ -= D;
        B_ += D;
        return true;
    }

    // The single-source tail by chunks, in parallel.  Nodes are split into
    // contiguous chunks (the callers number them in a spatial order, so a
    // chunk is a region); a thread serves the excess nodes of its chunks,
    // and a search
    // that would reach a node outside its chunk is undone and left to the
    // sequential tail.  A chunk's searches read and write only its own
    // nodes and the edges inside it, and skip the global offsets (which
    // change no reduced cost and no Lam), so chunks never share state and
    // every chunk's result is the same whatever the threads' timing.  Leaves
    // the deferred excess nodes in src_ (sorted).
    struct Worker {
        std::vector<int64_t> touched, cur, deferred;
        std::vector<Item> heap;
        std::vector<Frame> frames;
        int64_t paths = 0, phases = 0;
    };
    // at most 64 chunks of W nodes, at least 256 each (never a function of
    // the thread count, so every count gives the same result)
    int64_t chunk_width() const
    {
        const int64_t K = std::max<int64_t>(1, std::min<int64_t>(64, n_ / 256));
        return (n_ + K - 1) / K;
    }

    void single_chunks(int64_t &paths, int64_t &phases)
    {
        // the last sequential search's distances are still set
        for (int64_t x : touched_) cp_[x].dist = kInf;
        touched_.clear();
        // a second round with the boundaries moved by W / 2 serves most of
        // the searches that crossed one;
        const int64_t W = chunk_width();
        auto serve = [&](Worker &wk, int64_t lo, int64_t hi, int64_t s) {
            while (cp_[s].ex > 0) {
                int64_t t;
                if (!shortest_in(wk, s, lo, hi, t)) {
                    wk.deferred.push_back(s);
                    return;
                }
                ++wk.phases;
                for (int64_t x = t; x != s;) {
                    const int64_t k = cp_[x].par;
                    Edge &ed = e_[k >> 1];
                    ed.y[k & 1] ^= 1;
                    x = (x < n_) ? n_ + head(ed, k & 1) : tail(ed, k & 1);
                }
                --cp_[s].ex;
                ++cp_[t].ex;
                ++wk.paths;
            }
        };
        // rounds with 4 W and 16 W wide chunks take most of the long searches
        for (int round = 0; round < 4; ++round) {
            if (src_.empty() || (round == 1 && W < 2) || (round == 2 && 4 * W >= n_) || (round == 3 && 16 * W >= n_))
                break;
            if (round < 2) chunk_round(W, round == 0 ? 0 : W / 2, serve);
            else chunk_round(round == 2 ? 4 * W : 16 * W, 0, serve);
            src_.clear();
            for (Worker &wk : workers_) {
                paths += wk.paths;
                phases += wk.phases;
                src_.insert(src_.end(), wk.deferred.begin(), wk.deferred.end());
            }
            std::sort(src_.begin(), src_.end());
        }
    }

    // The first augmentations of the zero-reduced-cost pass, chunk by chunk
    // (a search never leaves its chunk; a second round with the boundaries
    // moved by half a chunk); returns the paths found.  src_ is kept:
    // solve() goes on with a pass over the whole graph.
    int64_t zero_chunks(int64_t &paths)
    {
        const int64_t W = chunk_width();
        int64_t found = 0;
        for (int round = 0; round < 2; ++round) {
            if (round == 1 && W < 2) break;
            const int32_t stamp = ++stamp_;
            auto serve = [&](Worker &wk, int64_t lo, int64_t hi, int64_t s) {
                while (cp_[s].ex > 0 && cp_[s].seen != stamp) {
                    if (!augment_in(wk, s, stamp, lo, hi)) return;
                    ++wk.paths;
                }
            };
            chunk_round(W, round == 0 ? 0 : W / 2, serve);
            for (Worker &wk : workers_) found += wk.paths;
        }
        paths += found;
        return found;
    }

    // One parallel round over the chunks c = [max(0, (c - 1) W + o),
    // min(n, c W + o)): serve(worker, lo, hi, s) for every excess node of
    // src_ in chunk c, in increasing order; the workers' counters and
    // deferred lists start empty.
    template <class Serve>
    void chunk_round(int64_t W, int64_t o, Serve &serve)
    {
        auto chunk_of = [&](int64_t x) { return ((x < n_ ? x : x - n_) + W - o) / W; };
        const int64_t K = chunk_of(n_ - 1) + 1;
        std::vector<int64_t> first(K + 1, 0);
        for (int64_t x : src_) ++first[chunk_of(x) + 1];
        for (int64_t c = 0; c < K; ++c) first[c + 1] += first[c];
        std::vector<int64_t> bysrc(src_.size());
        {
            std::vector<int64_t> at(first.begin(), first.end() - 1);
            for (int64_t x : src_) bysrc[at[chunk_of(x)]++] = x;
        }
        const int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads_, K));
        workers_.resize(T);
        std::atomic<int64_t> next{0};
        auto run = [&](int w) {
            Worker &wk = workers_[w];
            wk.paths = wk.phases = 0;
            wk.deferred.clear();
            for (int64_t c; (c = next.fetch_add(1)) < K;) {
                const int64_t lo = std::max<int64_t>(0, (c - 1) * W + o), hi = std::min<int64_t>(n_, c * W + o);
                for (int64_t i = first[c]; i < first[c + 1]; ++i) serve(wk, lo, hi, bysrc[i]);
            }
            for (int64_t x : wk.touched) cp_[x].dist = kInf;
            wk.touched.clear();
        };
        pool_.run(T, run);
    }

    // shortest() from one node, restricted to the nodes [lo, hi) (both
    // copies): false (nothing changed) when the search would leave them or
    // finds no deficit inside.  No global offsets (see single_chunks).
    bool shortest_in(Worker &wk, int64_t s, int64_t lo, int64_t hi, int64_t &t)
    {
        for (int64_t x : wk.touched) cp_[x].dist = kInf;
        wk.touched.clear();
        wk.cur.clear();
        wk.heap.clear();
        int64_t dcur = 0;
        cp_[s].dist = 0;
        cp_[s].par = -1;
        wk.touched.push_back(s);
        wk.cur.push_back(s);
        auto inside = [&](int64_t x) { const int64_t v = x < n_ ? x : x - n_; return v >= lo && v < hi; };
        auto push = [&](int64_t to, int64_t nd, int64_t k) {
            Copy &c = cp_[to];
            if (nd >= c.dist) return;
            if (c.dist == kInf) wk.touched.push_back(to);
            c.dist = nd;
            c.par = k;
            if (nd == dcur) {
                wk.cur.push_back(to);
            } else {
                wk.heap.push_back({nd, to});
                std::push_heap(wk.heap.begin(), wk.heap.end(), std::greater<Item>());
            }
        };
        int64_t D = -1;
        for (;;) {
            int64_t x;
            if (!wk.cur.empty()) {
                x = wk.cur.back();
                wk.cur.pop_back();
                if (cp_[x].dist != dcur) continue;
            } else {
                if (wk.heap.empty()) break;
                std::pop_heap(wk.heap.begin(), wk.heap.end(), std::greater<Item>());
                const Item it = wk.heap.back();
                wk.heap.pop_back();
                if (it.first != cp_[it.second].dist) continue;
                dcur = it.first;
                x = it.second;
            }
            if (cp_[x].ex < 0) { D = dcur; t = x; break; }
            // relax x's residual arcs; any head outside the chunk ends the search
            const int64_t base = cp_[x].pot + A_ + B_;
            if (x < n_) {
                for (int64_t p = start_[x]; p < end_[x]; ++p) {
                    const int64_t ie = inc_[p];
                    const Edge &ed = e_[ie];
                    const int dd = ed.a != x;
                    if (ed.y[dd]) continue;
                    const int64_t w = dd ? ed.a : ed.b;
                    if (!inside(w)) return false;
                    push(n_ + w, dcur + ed.c - base - cp_[n_ + w].pot, 2 * ie + dd);
                }
            } else {
                const int64_t u = x - n_;
                for (int64_t p = start_[u]; p < end_[u]; ++p) {
                    const int64_t ie = inc_[p];
                    const Edge &ed = e_[ie];
                    const int dd = ed.b != u;
                    if (!ed.y[dd]) continue;
                    const int64_t w = dd ? ed.b : ed.a;
                    if (!inside(w)) return false;
                    push(w, dcur - (ed.c - cp_[w].pot - base), 2 * ie + dd);
                }
            }
        }
        if (D < 0) return false;
        for (int64_t x : wk.touched) {
            Copy &c = cp_[x];
            if (c.dist >= D) continue;
            if (x < n_) c.pot += D - c.dist;
            else c.pot -= D - c.dist;
        }
        return true;
    }

    void push(int64_t to, int64_t nd, int64_t dcur, int64_t k)
    {
        Copy &c = cp_[to];
        if (nd >= c.dist) return;
        if (c.dist == kInf) touched_.push_back(to);
        c.dist = nd;
        c.par = k;
        if (nd == dcur) {
            cur_.push_back(to);
        } else {
            heap_.push_back({nd, to});
            std::push_heap(heap_.begin(), heap_.end(), std::greater<Item>());
        }
    }

    void relax_from(int64_t x, int64_t d)
    {
        if (x < n_) {   // left copy: arcs with y = 0, forward
            const int64_t base = cp_[x].pot + A_ + B_;
            for (int64_t p = start_[x]; p < end_[x]; ++p) {
                const int64_t ie = inc_[p];
                const Edge &ed = e_[ie];
                const int dd = ed.a != x;            // the arc that leaves x'
                if (ed.y[dd]) continue;
                const int64_t w = dd ? ed.a : ed.b;  // its head w''
                push(n_ + w, d + ed.c - base - cp_[n_ + w].pot, d, 2 * ie + dd);
            }
        } else {        // right copy: arcs with y = 1, backward
            const int64_t u = x - n_;
            const int64_t base = cp_[x].pot + A_ + B_;
            for (int64_t p = start_[u]; p < end_[u]; ++p) {
                const int64_t ie = inc_[p];
                const Edge &ed = e_[ie];
                const int dd = ed.b != u;            // the arc that enters u''
                if (!ed.y[dd]) continue;
                const int64_t w = dd ? ed.b : ed.a;  // its tail w'
                push(w, d - (ed.c - cp_[w].pot - base), d, 2 * ie + dd);
            }
        }
    }

    // Depth-first search from s over zero-reduced-cost residual arcs to a
    // node with a deficit; flips the arcs of the path found.
    bool augment_from(int64_t s, int32_t stamp) { return augment(frames_, s, stamp, 0, n_); }

    // The same inside the nodes [lo, hi) (both copies), with the worker's
    // own stack.
    bool augment_in(Worker &wk, int64_t s, int32_t stamp, int64_t lo, int64_t hi)
    {
        return augment(wk.frames, s, stamp, lo, hi);
    }

    bool augment(std::vector<Frame> &st, int64_t s, int32_t stamp, int64_t lo, int64_t hi)
    {
        st.clear();
        cp_[s].seen = stamp;
        st.push_back({s, start_[s < n_ ? s : s - n_], -1});
        while (!st.empty()) {
            Frame &f = st.back();
            const int64_t x = f.x;
            if (x != s && cp_[x].ex < 0) {
                // flip the path
                for (size_t i = 1; i < st.size(); ++i) {
                    const int64_t k = st[i].via;
                    e_[k >> 1].y[k & 1] ^= 1;
                }
                --cp_[s].ex;
                ++cp_[x].ex;
                return true;
            }
            bool pushed = false;
            if (x < n_) {
                const int64_t base = cp_[x].pot + A_ + B_;
                for (; f.p < end_[x]; ++f.p) {
                    const int64_t ie = inc_[f.p];
                    const Edge &ed = e_[ie];
                    const int dd = ed.a != x;
                    if (ed.y[dd]) continue;
                    const int64_t w = dd ? ed.a : ed.b, to = n_ + w;
                    if (w < lo || w >= hi) continue;
                    if (ed.c - base - cp_[to].pot != 0) continue;
                    if (cp_[to].seen == stamp) continue;
                    cp_[to].seen = stamp;
                    ++f.p;
                    st.push_back({to, start_[w], 2 * ie + dd});
                    pushed = true;
                    break;
                }
            } else {
                const int64_t u = x - n_;
                const int64_t base = cp_[x].pot + A_ + B_;
                for (; f.p < end_[u]; ++f.p) {
                    const int64_t ie = inc_[f.p];
                    const Edge &ed = e_[ie];
                    const int dd = ed.b != u;
                    if (!ed.y[dd]) continue;
                    const int64_t to = dd ? ed.b : ed.a;
                    if (to < lo || to >= hi) continue;
                    if (ed.c - cp_[to].pot - base != 0) continue;
                    if (cp_[to].seen == stamp) continue;
                    cp_[to].seen = stamp;
                    ++f.p;
                    st.push_back({to, start_[to], 2 * ie + dd});
                    pushed = true;
                    break;
                }
            }
            if (!pushed) st.pop_back();
        }
        return false;
    }

    const int32_t *xy_ = nullptr;
    const int32_t *b_ = nullptr;     // degrees, or null for 2
    int64_t n_ = 0;
    int64_t A_ = 0, B_ = 0;          // global offsets of alpha and beta
    std::vector<Copy> cp_;           // node copies: left v, right n + v
    std::vector<int64_t> src_;       // nodes with excess (may hold stale entries)
    std::vector<int64_t> touched_, cur_;
    std::vector<Item> heap_;
    RawVec<uint64_t> keys_;          // sorted keys (pair_key) of the candidate edges
    // keys added after keys_ was last merged, sorted: a few pricing rounds
    // add tens of pairs each, so they wait here instead of rewriting keys_
    RawVec<uint64_t> extra_;
    std::vector<uint64_t> fresh_;
    RawVec<uint64_t> merged_;
    std::vector<int32_t> fresh_c_;
    RawVec<Edge> e_;
    std::vector<int64_t> start_, end_, cap_;   // incident-edge lists (see build_adjacency)
    RawVec<int32_t> inc_;
    int64_t built_ = 0;              // edges covered by the lists
    int32_t stamp_ = 0;              // augmentation pass stamps (Copy::seen)
    std::vector<Frame> frames_;
    int threads_ = 1;
    int64_t parallel_min_ = 256;     // excess nodes for the chunked tail
    Pool pool_;
    std::vector<Worker> workers_;
};

}  // namespace

static double secs()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// pricing also returns the pairs with 0 <= Z < kPriceSlack
constexpr int64_t kPriceSlack = 16;

struct FinishWork {
    DoubleCover g;
    PairList pl;
    std::vector<int64_t> lam;
};

FinishWork *finish_work_create(int threads, int64_t parallel_min)
{
    FinishWork *w = new FinishWork();
    w->g.set_threads(threads, parallel_min);
    return w;
}

void finish_work_destroy(FinishWork *work) { delete work; }

void finish_exact(const int32_t *xy, int64_t n, const int64_t *lam0, PairSource &src, FinishResult *out,
                  FinishWork *work, const int32_t *b)
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
    PairList &pl = work->pl;
    std::vector<int64_t> &lam = work->lam;
    std::string err;
    pl.clear();
    int64_t slack = 16;
    // the double cover is reset on another thread while the first
    // collection runs (the pair source mostly waits for the GPU); the two
    // touch disjoint state
    std::exception_ptr reset_err;
    std::thread resetter([&] {
        try {
            g.reset(xy, n, lam0, b);
        } catch (...) {
            reset_err = std::current_exception();
        }
    });
    src.want_bulk = true;
    bool got = false;
    try {
        got = src.near(lam0, slack, pl, err);
    } catch (...) {
        resetter.join();
        throw;
    }
    resetter.join();
    src.want_bulk = false;
    if (reset_err) std::rethrow_exception(reset_err);
    if (!got) { r.msg = err; return; }
    r.t_collect += secs() - t;
    t = secs();
    if (!g.add_bulk(pl, src)) {
        if (pl.empty() && src.keys)
            for (int64_t i = 0; i < src.nkeys; ++i)
                pl.emplace_back((int32_t)(src.keys[i] >> 32), (int32_t)(src.keys[i] & 0xffffffffULL));
        g.add(pl, src.costs);
    }
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
        // pricing: the pairs with Z < kPriceSlack; optimal when none of
        // them with Z < 0 is new, else all the new ones join (the near-tight
        // ones often save the next round)
        src.price_slack = kPriceSlack;
        const bool priced = src.negative(lam.data(), pl, err);
        src.price_slack = 0;
        if (!priced) { r.msg = err; return; }
        r.t_collect += secs() - t;
        if (!g.fresh_negative(pl, src.costs, lam)) {
            r.ok = true;
            r.lam.assign(lam.begin(), lam.end());
            g.x(r.eu, r.ev, r.ex2);
            r.candidates = g.edges();
            return;
        }
        t = secs();
        g.add(pl, src.costs);
        r.t_build += secs() - t;
    }
    r.msg = "pricing did not converge in 64 rounds";
}

}  // namespace f2m
