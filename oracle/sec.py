"""F2M with subtour-elimination rows: the GDP of Sec. 3 on inequality rows.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The relaxation (Sec. 4 plus the extension named in Sec. 5): for a family of
node sets S_q (2 <= |S_q| <= n - 2),

    min c.x   s.t.  x(delta(v)) = 2 for every node v,
                    x(delta(S_q)) >= 2 for every q,      0 <= x <= 1,

delta(S) being the edges with exactly one end in S.  Sec. 2 adds the active
inequality rows to the objective with multipliers lambda_q >= 0 (eq. 4-5);
Sec. 3 gives every row with binary coefficients and an integral right-hand
side b the gradient from positions b and b + 1 of its sorted adjusted
lengths.  A subtour row has b = 2 over the edges of delta(S_q), so it moves
exactly like a node row, then is projected back onto lambda_q >= 0.

Integer form (doubled, as in the rest of the oracle): Lam_v = 2 lambda_v,
M_q = 2 lambda_q >= 0, and for an edge e = {u, v}

    Z_e = 2 c_e - Lam_u - Lam_v - sum_{q : e in delta(S_q)} M_q      (eq. 9)

With s the sum of a row's 2nd and 3rd smallest Z, moving that row's
multiplier alone by s/2 would put zero midway between them (Sec. 3).  All
rows step from the same iterate (Jacobi), so each move is divided by the
number of rows that share an edge: a degree row's edge lies in two degree
rows, so it moves by sign(s) floor((|s| + 2) / 4) (the rule of the F2M
oracle); an edge crossing a subtour row lies in the two degree rows and,
within its layer, in the subtour rows of both of its ends, so a subtour row
moves by sign(s) floor((|s| + 4) / 8), and its new value is
max(0, M_q + step).  (Moved like a degree row, by s/4, the subtour rows
make the iterates diverge on families from two separation rounds.)  The
Lagrangian (doubled):

    2 L = 2 sum_v Lam_v + 2 sum_q M_q + sum_e min(0, Z_e)

is a lower bound on twice the optimum for every Lam and every M >= 0 (weak
duality); it equals it when the trivial x of (Lam, M) -- x_e = 1, 1/2, 0 for
Z_e < 0, = 0, > 0 (eq. 7) -- is feasible and every row with M_q > 0 is
tight (complementary slackness).

Plain dense numpy over the complete graph: meant for n up to a few hundred.
"""
from __future__ import annotations

import math

import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def cost_matrix(xy):
    """c[u, v] = nint(sqrt(D_uv)) (TSPLIB EUC_2D), the k with
    (2k - 1)^2 <= 4 D < (2k + 1)^2, by the integer square root."""
    xy = np.asarray(xy, dtype=np.int64)
    n = len(xy)
    c = np.zeros((n, n), np.int64)
    for u in range(n):
        for v in range(u + 1, n):
            dx = int(xy[u, 0]) - int(xy[v, 0])
            dy = int(xy[u, 1]) - int(xy[v, 1])
            k = (math.isqrt(4 * (dx * dx + dy * dy)) + 1) // 2
            c[u, v] = c[v, u] = k
    return c


def crossing(n, cuts):
    """X[q] = boolean n x n matrix of the edges in delta(S_q)."""
    out = []
    for S in cuts:
        ins = np.zeros(n, bool)
        ins[np.asarray(S, dtype=np.int64)] = True
        out.append(ins[:, None] != ins[None, :])
    return out


def canonical_cut(n, S):
    """The side of the cut that does not hold node 0, sorted (delta(S) and
    delta(V - S) are one row)."""
    S = sorted(set(int(v) for v in S))
    if 0 in S:
        S = sorted(set(range(n)) - set(S))
    return tuple(S)


def z_matrix(c, lam, mu, X):
    """Z (eq. 9, doubled) for every ordered pair; the diagonal is unused."""
    lam = np.asarray(lam, dtype=np.int64)
    Z = 2 * c - lam[:, None] - lam[None, :]
    for q, Xq in enumerate(X):
        Z = Z - np.where(Xq, np.int64(mu[q]), np.int64(0))
    return Z


def step(s: int) -> int:
    """sign(s) floor((|s| + 2) / 4): a degree row's damped midpoint move."""
    a = (abs(int(s)) + 2) // 4
    return a if s > 0 else (-a if s < 0 else 0)


def row_step(s: int) -> int:
    """sign(s) floor((|s| + 4) / 8): a subtour row's damped midpoint move."""
    a = (abs(int(s)) + 4) // 8
    return a if s > 0 else (-a if s < 0 else 0)


def mix64(z: int) -> int:
    """SplitMix64 output finaliser (Steele, Lea, Flood 2014)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def state_hash(lam, mu) -> int:
    """Order-free fingerprint of (Lam, M): node v at index v, row q at
    index n + q."""
    vals = [int(x) for x in lam] + [int(x) for x in mu]
    h = 0
    for i, x in enumerate(vals):
        h = (h + mix64((x & M64) ^ ((GOLDEN * (i + 1)) & M64))) & M64
    return h


def _row_stats(vals):
    """(2nd, 3rd smallest, #neg, #zero, sum of negatives) of a row's Z."""
    v = np.sort(np.asarray(vals, dtype=np.int64))
    z2 = int(v[1]) if len(v) > 1 else None
    z3 = int(v[2]) if len(v) > 2 else None
    return z2, z3, int((v < 0).sum()), int((v == 0).sum()), int(v[v < 0].sum())


def gdp_iter(xy, lam, cuts, mu, c=None, X=None):
    """One Jacobi iteration at (Lam, M).  Returns a dict with the record
    (dual2, unsat, bad, max_step, nonzero, hash), the node steps, the new
    M (projected) and the per-row statistics."""
    n = len(xy)
    c = cost_matrix(xy) if c is None else c
    X = crossing(n, cuts) if X is None else X
    lam = np.asarray(lam, dtype=np.int64)
    mu = np.asarray(mu, dtype=np.int64)
    Z = z_matrix(c, lam, mu, X)
    iu = np.triu_indices(n, 1)
    dual2 = 2 * int(lam.sum()) + 2 * int(mu.sum()) + int(np.minimum(Z[iu], 0).sum())
    nstep = np.zeros(n, np.int64)
    unsat = bad = 0
    for v in range(n):
        z2, z3, neg, zero, _ = _row_stats(np.delete(Z[v], v))
        nstep[v] = step(z2 + z3)
        unsat += 1 if (z2 > 0 or z3 < 0) else 0
        bad += 1 if 2 * neg + zero != 4 else 0
    new_mu = mu.copy()
    cut_deg2 = []
    for q, Xq in enumerate(X):
        vals = Z[iu][Xq[iu]]
        z2, z3, neg, zero, _ = _row_stats(vals)
        d2 = 2 * neg + zero                      # doubled crossing degree of the trivial x
        cut_deg2.append(d2)
        new_mu[q] = max(0, int(mu[q]) + row_step(z2 + z3))
        # an inequality row: violated if fewer than two crossing edges can
        # be taken (Z_(2) > 0), or, while its multiplier is positive, if more
        # than two must be (Z_(3) < 0)
        unsat += 1 if (z2 > 0 or (mu[q] > 0 and z3 < 0)) else 0
        bad += 1 if (d2 < 4 or (mu[q] > 0 and d2 != 4)) else 0
    dmu = new_mu - mu
    steps = np.concatenate([nstep, dmu])
    rec = dict(dual2=dual2, unsat=unsat, bad=bad, max_step=int(np.abs(steps).max()) if len(steps) else 0,
               nonzero=int((steps != 0).sum()), hash=state_hash(lam, mu), sum_lam=int(lam.sum()),
               sum_mu=int(mu.sum()))
    return dict(rec=rec, step=nstep, mu_next=new_mu, cut_deg2=cut_deg2, Z=Z)


def gdp_solve(xy, cuts, lam0=None, mu0=None, max_iters=100000):
    """The GDP loop with subtour rows.  Stops, tested in this order: every
    row trivially satisfied ("trivial"), every step zero ("fixed"), the
    state equal to the one two iterations back by hash ("cycle"), the cap
    ("cap").  (Lam*, M*) is the current iterate for trivial and fixed, the
    largest-dual iterate (earliest on ties) for cycle and cap."""
    n = len(xy)
    c = cost_matrix(xy)
    X = crossing(n, cuts)
    lam = np.zeros(n, np.int64) if lam0 is None else np.array(lam0, dtype=np.int64)
    mu = np.zeros(len(cuts), np.int64) if mu0 is None else np.array(mu0, dtype=np.int64)
    trace = []
    best = None
    hist = []
    k = 0
    while True:
        it = gdp_iter(xy, lam, cuts, mu, c, X)
        r = it["rec"]
        trace.append(r)
        if best is None or r["dual2"] > best[0]:
            best = (r["dual2"], k, lam.copy(), mu.copy())
        if r["bad"] == 0:
            stop = "trivial"
        elif r["nonzero"] == 0:
            stop = "fixed"
        elif k >= 2 and r["hash"] == hist[-2]:
            stop = "cycle"
        elif k >= max_iters:
            stop = "cap"
        else:
            stop = None
        if stop:
            if stop in ("cycle", "cap"):
                _, kstar, lam_s, mu_s = best
            else:
                kstar, lam_s, mu_s = k, lam, mu
            return dict(stop=stop, iters=k + 1, kstar=kstar, lam=lam_s, mu=mu_s, trace=trace)
        hist.append(r["hash"])
        lam = lam + it["step"]
        mu = it["mu_next"]
        k += 1


def trivial_x(xy, lam, cuts, mu):
    """Edges with Z <= 0 (eq. 7): (u, v, x2) with x2 = 2 for Z < 0, 1 for
    Z = 0, u < v."""
    n = len(xy)
    Z = z_matrix(cost_matrix(xy), lam, mu, crossing(n, cuts))
    out = []
    for u in range(n):
        for v in range(u + 1, n):
            if Z[u, v] <= 0:
                out.append((u, v, 2 if Z[u, v] < 0 else 1))
    return out


def certify(xy, lam, cuts, mu, edges):
    """primal2 = 2 c.x, dual2 = 2 L(Lam, M); feasible: degrees 2, every
    subtour row >= 2, x in {1/2, 1}; certified: feasible, every row with
    M_q > 0 tight and primal2 == dual2."""
    n = len(xy)
    c = cost_matrix(xy)
    X = crossing(n, cuts)
    mu = np.asarray(mu, dtype=np.int64)
    lam = np.asarray(lam, dtype=np.int64)
    deg2 = np.zeros(n, np.int64)
    cut2 = np.zeros(len(cuts), np.int64)
    primal2 = 0
    ok = all(mq >= 0 for mq in mu)
    seen = set()
    for (u, v, x2) in edges:
        if u == v or (min(u, v), max(u, v)) in seen or x2 not in (1, 2):
            ok = False
            continue
        seen.add((min(u, v), max(u, v)))
        primal2 += int(c[u, v]) * x2
        deg2[u] += x2
        deg2[v] += x2
        for q, Xq in enumerate(X):
            if Xq[u, v]:
                cut2[q] += x2
    feasible = ok and bool(np.all(deg2 == 4)) and bool(np.all(cut2 >= 4))
    tight = bool(np.all((mu == 0) | (cut2 == 4)))
    Z = z_matrix(c, lam, mu, X)
    iu = np.triu_indices(n, 1)
    dual2 = 2 * int(lam.sum()) + 2 * int(mu.sum()) + int(np.minimum(Z[iu], 0).sum())
    return dict(primal2=primal2, dual2=dual2, feasible=feasible,
                certified=feasible and tight and primal2 == dual2)


def components(n, edges):
    """Connected components of the support graph of x (node lists, each
    sorted, in order of their smallest node)."""
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for (u, v, _) in edges:
        a, b = find(u), find(v)
        if a != b:
            parent[max(a, b)] = min(a, b)
    comp = {}
    for v in range(n):
        comp.setdefault(find(v), []).append(v)
    return sorted(comp.values(), key=lambda s: s[0])


def separate(n, edges, cuts=()):
    """Subtour rows violated by x: every component S of its support that is
    not the whole graph has x(delta(S)) = 0 < 2.  Returns the new canonical
    cuts (the ones not already in `cuts`)."""
    have = {canonical_cut(n, S) for S in cuts}
    out = []
    comps = components(n, edges)
    if len(comps) <= 1:
        return out
    for S in comps:
        key = canonical_cut(n, S)
        if 2 <= len(key) <= n - 2 and key not in have:
            have.add(key)
            out.append(list(key))
    return out
