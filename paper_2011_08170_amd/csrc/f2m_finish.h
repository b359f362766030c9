// Exact finish of the GDP (host C++): from the GDP multipliers to a
// certified F2M optimum.
//
// The GDP's fixed points are stationary for every single multiplier but
// need not be optimal (degenerate cases, Sec. 3 of arXiv 2011.08170).  The
// finish solves F2M exactly as a min-cost flow on the bipartite double
// cover (left copy v', right copy v'', arc v'->u'' of cost c_uv and
// capacity 1, every copy of degree 2 -- or b_v, see finish_exact; its
// optimum is twice the F2M optimum
// and x_e = (y_u'v'' + y_v'u'')/2), by a primal-dual method: Dijkstra on
// reduced costs from every node with excess, a potential update, then unit
// augmentations along zero-reduced-cost paths.  It starts from the GDP's
// Lam: alpha_v = floor(Lam_v / 2), beta_v = Lam_v - alpha_v, and the flow
// y = 1 exactly on the arcs of negative reduced cost.  The arc set is a
// candidate set of near-tight pairs; pricing asks the caller for every pair
// of the complete graph whose Z is negative under the finished
// Lam = alpha + beta and repeats until there is none, which makes the
// result optimal on the complete graph (dual2 == primal2).
#pragma once
#include <stdint.h>

#include <memory>
#include <string>
#include <utility>
#include <vector>

namespace f2m {

// exact nint(sqrt(D)) on the host
int64_t nint_sqrt_host(int64_t D);

using PairList = std::vector<std::pair<int32_t, int32_t>>;   // (u, v), u < v

// Candidate pairs for the finish, supplied by the caller (the library
// uses GPU scans).
struct PairSource {
    virtual ~PairSource() = default;
    // Data returned beside the pairs of the last call, as views into the
    // source's own memory, valid until its next call; null when the source
    // does not compute them.  costs: the exact costs c of the pairs, in the
    // same order (else the finish computes them itself).
    const int32_t *costs = nullptr;
    // Bulk data the finish asks for (want_bulk) on its first call, for the
    // pairs returned in the same order: neg bit 0 / bit 1 = the arc u'->v''
    // / v'->u'' has negative reduced cost c - alpha_tail - beta_head under
    // alpha = floor(lam/2), beta = lam - alpha of the lam passed, and every
    // node's incident pair indices in increasing order, each node's list
    // followed by two free slots (node v: inc[inc_start[v] ..
    // inc_start[v + 1] - 2), inc_start of n + 1 entries, inc of 2 * pairs +
    // 2 * n entries).
    bool want_bulk = false;
    // Bulk data, optional: the pairs as sorted keys (u << 32 | v, u < v) in
    // place of the pair list, which the source may then leave empty
    const uint64_t *keys = nullptr;
    int64_t nkeys = 0;
    const uint8_t *neg = nullptr;
    const int32_t *inc_start = nullptr;
    const int32_t *inc = nullptr;
    // pairs {u, v} with Z_uv(lam) <= max(0, 4th smallest Z at u or v) + slack
    virtual bool near(const int64_t *lam, int64_t slack, PairList &out, std::string &err) = 0;
    // pairs {u, v} with Z_uv(lam) < price_slack (the finish sets it: a few
    // near-tight pairs priced together with the negative ones)
    int64_t price_slack = 0;
    virtual bool negative(const int64_t *lam, PairList &out, std::string &err) = 0;
};

// An allocator whose resize leaves new elements uninitialised (default-
// initialised): the finish's large arrays and its results are written in
// full right after they grow, so zeroing them first is wasted time.
template <class T>
struct NoInit : std::allocator<T> {
    template <class U>
    struct rebind { using other = NoInit<U>; };
    NoInit() = default;
    template <class U>
    NoInit(const NoInit<U> &) {}
    template <class U>
    void construct(U *p) { ::new (static_cast<void *>(p)) U; }
    template <class U, class... A>
    void construct(U *p, A &&...a) { ::new (static_cast<void *>(p)) U(std::forward<A>(a)...); }
};
template <class T>
using RawVec = std::vector<T, NoInit<T>>;

struct FinishResult {
    bool ok = false;
    std::string msg;
    RawVec<int64_t> lam;            // Lam = alpha + beta
    RawVec<int32_t> eu, ev;         // edges of x, eu < ev (no particular order)
    RawVec<uint8_t> ex2;            // 2x in {1, 2}
    int64_t paths = 0;              // unit augmentations
    int64_t rounds = 0;             // pricing rounds
    int64_t phases = 0;             // Dijkstra phases
    int64_t candidates = 0;         // candidate pairs at the end
    double t_collect = 0.0;         // seconds in the pair source
    double t_build = 0.0;           // seconds adding candidates
    double t_flow = 0.0;            // seconds in the flow phases
};

// Host memory of the finish, kept from one call to the next so that its
// buffers are reused (no fresh pages per solve); one per finishing thread.
// Once parallel_min excess nodes are left for the flow's single-source
// tail, it runs over ranges of nodes, on `threads` threads; the result
// depends neither on the thread count nor on the threads' timing.
struct FinishWork;
FinishWork *finish_work_create(int threads = 1, int64_t parallel_min = 256);
void finish_work_destroy(FinishWork *work);

// work may be null (a temporary one is used).  out's vectors keep their
// capacity when it is reused.  b: the degree of every node (the right-hand
// side b_v of its row, 1 to 3: the b-matching of Sec. 3), or null for 2
// (F2M); both copies of node v then carry b_v units.
void finish_exact(const int32_t *xy, int64_t n, const int64_t *lam0, PairSource &src, FinishResult *out,
                  FinishWork *work = nullptr, const int32_t *b = nullptr);

}  // namespace f2m
