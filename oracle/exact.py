"""Pure-Python exact checkers for the F2M optimum (Sec. 4) and for its
generalisation to per-node degrees b_v (fractional b-matching: rows with
binary coefficients and integral right-hand sides, Sec. 3, condition 8).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* brute_force_opt2: enumerates every x in {0, 1/2, 1}^E with all degrees
  equal to 2 (backtracking with degree pruning), valid because some optimal
  vertex of F2M is half-integral (Sec. 4, Edmonds).  Practical for n <= 7.
* simplex_opt2: exact-rational bounded-variable primal simplex (Bland's rule)
  on   min c.x  s.t.  sum_{e in delta(v)} x_e = 2,  0 <= x <= 1,
  with a phase 1 on artificial variables.  Practical for n <= ~40.

Both return 2 * optimum as an int (the optimum is a multiple of 1/2) and use
math.isqrt for the EUC_2D length, independently of the C oracle.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def euc2d(xy, u, v) -> int:
    """nint(sqrt(D)): the k with (2k-1)^2 <= 4D < (2k+1)^2."""
    dx = int(xy[u][0]) - int(xy[v][0])
    dy = int(xy[u][1]) - int(xy[v][1])
    D = dx * dx + dy * dy
    r = math.isqrt(4 * D)          # floor(2 sqrt D)
    return (r + 1) // 2


def edges_of(n):
    return [(u, v) for u in range(n) for v in range(u + 1, n)]


def graph_edges(graph, n):
    """Edge list (u < v) of a CSR graph (rowptr, col); all pairs if None."""
    if graph is None:
        return edges_of(n)
    rowptr, col = graph
    return [(u, int(v)) for u in range(n) for v in col[rowptr[u]:rowptr[u + 1]] if u < v]


def _rhs(b, n):
    return [2] * n if b is None else [int(x) for x in b]


def brute_force_opt2(xy, graph=None, b=None):
    """2 * min c.x over x in {0,1/2,1}^E with every degree b_v (2 when b is
    None); None if none.  Some optimal vertex is half-integral (the double
    cover argument holds for any b), so the enumeration is exact."""
    n = len(xy)
    need = [2 * x for x in _rhs(b, n)]   # doubled degrees
    E = graph_edges(graph, n)
    c = [euc2d(xy, u, v) for (u, v) in E]
    deg = [0] * n              # doubled degrees so far
    left = [0] * n             # undecided incident edges per node
    for (u, v) in E:
        left[u] += 1
        left[v] += 1
    best = [None]
    # order edges so each node's edges close early: already lexicographic

    def rec(i, acc):
        if best[0] is not None and acc >= best[0]:
            return
        if i == len(E):
            if all(d == t for d, t in zip(deg, need)):
                best[0] = acc
            return
        u, v = E[i]
        left[u] -= 1; left[v] -= 1
        for x2 in (0, 1, 2):
            du, dv = deg[u] + x2, deg[v] + x2
            if du > need[u] or dv > need[v]:
                continue
            if du + 2 * left[u] < need[u] or dv + 2 * left[v] < need[v]:
                continue
            deg[u], deg[v] = du, dv
            rec(i + 1, acc + x2 * c[i])
            deg[u] -= x2; deg[v] -= x2
        left[u] += 1; left[v] += 1

    rec(0, 0)
    return best[0]


def simplex_opt2(xy, max_pivots=200000, b=None):
    """Exact optimum * 2 by a bounded-variable simplex over Fractions.

    Standard form: rows A x = b (one per node, b_v = 2 unless given),
    0 <= x <= 1.  Phase 1
    adds one artificial per row (x_a >= 0, no upper bound) and minimises
    their sum; phase 2 minimises c.x.  Nonbasic variables sit at 0 or at
    their upper bound; entering/leaving by Bland's rule (smallest index)."""
    n = len(xy)
    E = edges_of(n)
    m = len(E)
    cost = [Fraction(euc2d(xy, u, v)) for (u, v) in E]
    nv = m + n                     # structural + artificial
    INF = None
    ub = [Fraction(1)] * m + [INF] * n
    # dense tableau rows: B^-1 A, and B^-1 b, kept explicitly
    A = [[Fraction(0)] * nv for _ in range(n)]
    for j, (u, v) in enumerate(E):
        A[u][j] = Fraction(1)
        A[v][j] = Fraction(1)
    for i in range(n):
        A[i][m + i] = Fraction(1)
    basis = [m + i for i in range(n)]
    at_upper = [False] * nv
    xB = [Fraction(r) for r in _rhs(b, n)]   # values of basic variables

    def run(obj, allowed):
        pivots = 0
        while True:
            # reduced costs d_j = obj_j - obj_B . column_j
            cb = [obj[b] for b in basis]
            entering, direction = None, 0
            inbasis = set(basis)
            for j in range(allowed):
                if j in inbasis:
                    continue
                d = obj[j] - sum(cb[i] * A[i][j] for i in range(n) if A[i][j] != 0)
                if not at_upper[j] and d < 0:
                    entering, direction = j, +1
                    break
                if at_upper[j] and d > 0:
                    entering, direction = j, -1
                    break
            if entering is None:
                return
            j = entering
            # ratio test: moving x_j by t*direction changes x_B by -t*direction*col
            tmax = ub[j] if ub[j] is not None else None
            leave, leave_to_upper = None, False
            for i in range(n):
                a = A[i][j] * direction
                if a > 0:            # x_B[i] decreases to 0
                    t = xB[i] / a
                    cand = (t, basis[i], i, False)
                elif a < 0 and ub[basis[i]] is not None:   # increases to its bound
                    t = (ub[basis[i]] - xB[i]) / (-a)
                    cand = (t, basis[i], i, True)
                else:
                    continue
                if tmax is None or cand[0] < tmax or (cand[0] == tmax and leave is not None and cand[1] < leave[1]):
                    tmax = cand[0]
                    leave = cand
            if tmax is None:
                raise RuntimeError("unbounded")
            t = tmax
            for i in range(n):
                xB[i] -= t * direction * A[i][j]
            if leave is None:          # bound flip of the entering variable
                at_upper[j] = not at_upper[j]
            else:
                _, _, r, to_upper = leave
                old = basis[r]
                newval = t if direction > 0 else ub[j] - t
                piv = A[r][j]
                A[r] = [a / piv for a in A[r]]
                for i in range(n):
                    if i != r and A[i][j] != 0:
                        f = A[i][j]
                        A[i] = [a - f * b for a, b in zip(A[i], A[r])]
                basis[r] = j
                xB[r] = newval
                at_upper[j] = False
                at_upper[old] = to_upper
            pivots += 1
            if pivots > max_pivots:
                raise RuntimeError("pivot limit")

    run([Fraction(0)] * m + [Fraction(1)] * n, nv)
    art = sum(xB[i] for i in range(n) if basis[i] >= m) + \
        sum(ub[j] for j in range(m, nv) if at_upper[j] and ub[j] is not None)
    if art != 0:
        return None
    # phase 2: artificials never enter again; a degenerate basic artificial
    # (value 0) gets upper bound 0 so that it leaves rather than grows
    for i in range(n):
        ub[m + i] = Fraction(0)
    run(cost + [Fraction(0)] * n, m)
    x = [Fraction(0)] * m
    for j in range(m):
        if at_upper[j]:
            x[j] = Fraction(1)
    for i, b in enumerate(basis):
        if b < m:
            x[b] = xB[i]
    val = sum(ci * xi for ci, xi in zip(cost, x))
    assert (2 * val).denominator == 1
    return int(2 * val)


def highs_opt2(xy, graph=None, b=None):
    """2 * optimum from scipy's HiGHS LP solver (a library cross-check;
    the optimum is a half-integer, recovered by rounding 2*fun)."""
    from scipy.optimize import linprog
    from scipy.sparse import coo_matrix
    n = len(xy)
    E = graph_edges(graph, n)
    c = np.array([euc2d(xy, u, v) for (u, v) in E], dtype=float)
    m = len(E)
    rows = np.array([u for u, v in E] + [v for u, v in E])
    cols = np.concatenate([np.arange(m), np.arange(m)])
    A = coo_matrix((np.ones(2 * m), (rows, cols)), shape=(n, m)).tocsr()
    r = linprog(c, A_eq=A, b_eq=np.array(_rhs(b, n), dtype=float), bounds=(0, 1), method="highs")
    if r.status == 2:
        return None
    assert r.status == 0
    return int(round(2 * r.fun))


def lp_min_exact(cost, rows, rhs, ub, max_pivots=500000):
    """min cost.x  s.t.  rows[i] . x = rhs[i] (rhs >= 0),  0 <= x_j <= ub[j]
    (ub[j] None: no upper bound), by the same exact-rational bounded-variable
    simplex as simplex_opt2 (phase 1 on one artificial per row, Bland's
    rule).  rows[i] is a dict {j: coefficient}.  Returns the optimum as a
    Fraction, or None when infeasible."""
    nr = len(rows)
    m = len(cost)
    nv = m + nr
    ubs = [None if u is None else Fraction(u) for u in ub] + [None] * nr
    A = [[Fraction(0)] * nv for _ in range(nr)]
    for i, row in enumerate(rows):
        for j, a in row.items():
            A[i][j] = Fraction(a)
        A[i][m + i] = Fraction(1)
    basis = [m + i for i in range(nr)]
    at_upper = [False] * nv
    xB = [Fraction(r) for r in rhs]

    def run(obj, allowed):
        pivots = 0
        while True:
            cb = [obj[b] for b in basis]
            entering, direction = None, 0
            inbasis = set(basis)
            for j in range(allowed):
                if j in inbasis:
                    continue
                d = obj[j] - sum(cb[i] * A[i][j] for i in range(nr) if A[i][j] != 0)
                if not at_upper[j] and d < 0:
                    entering, direction = j, +1
                    break
                if at_upper[j] and d > 0:
                    entering, direction = j, -1
                    break
            if entering is None:
                return
            j = entering
            tmax = ubs[j]
            leave = None
            for i in range(nr):
                a = A[i][j] * direction
                if a > 0:
                    cand = (xB[i] / a, basis[i], i, False)
                elif a < 0 and ubs[basis[i]] is not None:
                    cand = ((ubs[basis[i]] - xB[i]) / (-a), basis[i], i, True)
                else:
                    continue
                if tmax is None or cand[0] < tmax or (cand[0] == tmax and leave is not None and cand[1] < leave[1]):
                    tmax = cand[0]
                    leave = cand
            if tmax is None:
                raise RuntimeError("unbounded")
            t = tmax
            for i in range(nr):
                xB[i] -= t * direction * A[i][j]
            if leave is None:
                at_upper[j] = not at_upper[j]
            else:
                _, _, r, to_upper = leave
                old = basis[r]
                newval = t if direction > 0 else ubs[j] - t
                piv = A[r][j]
                A[r] = [a / piv for a in A[r]]
                for i in range(nr):
                    if i != r and A[i][j] != 0:
                        f = A[i][j]
                        A[i] = [a - f * b for a, b in zip(A[i], A[r])]
                basis[r] = j
                xB[r] = newval
                at_upper[j] = False
                at_upper[old] = to_upper
            pivots += 1
            if pivots > max_pivots:
                raise RuntimeError("pivot limit")

    run([Fraction(0)] * m + [Fraction(1)] * nr, nv)
    art = sum(xB[i] for i in range(nr) if basis[i] >= m)
    if art != 0:
        return None
    for i in range(nr):
        ubs[m + i] = Fraction(0)
    run([Fraction(c) for c in cost] + [Fraction(0)] * nr, m)
    x = [Fraction(0)] * m
    for j in range(m):
        if at_upper[j]:
            x[j] = ubs[j]
    for i, b in enumerate(basis):
        if b < m:
            x[b] = xB[i]
    return sum(Fraction(c) * xi for c, xi in zip(cost, x))


def subtour_rows(n, cuts):
    """The edges (u < v) of delta(S) for every cut S."""
    out = []
    for S in cuts:
        ins = set(int(v) for v in S)
        out.append([j for j, (u, v) in enumerate(edges_of(n)) if (u in ins) != (v in ins)])
    return out


def simplex_sec_opt2(xy, cuts):
    """2 * the optimum of F2M with the subtour rows x(delta(S)) >= 2 of
    `cuts`, exactly (a Fraction: with subtour rows the optimum need not be
    a multiple of 1/2).  Each inequality row gets a surplus variable:
    x(delta(S)) - s = 2, s >= 0."""
    n = len(xy)
    E = edges_of(n)
    m = len(E)
    cost = [euc2d(xy, u, v) for (u, v) in E]
    rows, rhs = [], []
    for v in range(n):
        rows.append({j: 1 for j, (a, b) in enumerate(E) if a == v or b == v})
        rhs.append(2)
    for q, cross in enumerate(subtour_rows(n, cuts)):
        row = {j: 1 for j in cross}
        row[m + q] = -1
        rows.append(row)
        rhs.append(2)
    val = lp_min_exact(cost + [0] * len(cuts), rows, rhs, [1] * m + [None] * len(cuts))
    return None if val is None else 2 * val


def highs_sec_opt2(xy, cuts):
    """The same optimum (times 2, float) from scipy's HiGHS."""
    from scipy.optimize import linprog
    n = len(xy)
    E = edges_of(n)
    m = len(E)
    c = np.array([euc2d(xy, u, v) for (u, v) in E], dtype=float)
    Aeq = np.zeros((n, m))
    for j, (u, v) in enumerate(E):
        Aeq[u, j] = Aeq[v, j] = 1.0
    Aub = np.zeros((len(cuts), m))
    for q, cross in enumerate(subtour_rows(n, cuts)):
        Aub[q, cross] = -1.0
    r = linprog(c, A_eq=Aeq, b_eq=np.full(n, 2.0), A_ub=Aub if len(cuts) else None,
                b_ub=np.full(len(cuts), -2.0) if len(cuts) else None, bounds=(0, 1), method="highs")
    if r.status == 2:
        return None
    assert r.status == 0
    return 2 * r.fun
