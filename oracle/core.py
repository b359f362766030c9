"""ctypes wrapper over the plain C oracle (f2m_oracle.c).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions: coordinates are int32 arrays of shape (n, 2); Lam = 2*lambda
is int64; Z_uv = 2 c_uv - Lam_u - Lam_v (eq. 9 doubled); the step is
sign(s) * floor((|s| + 2) / 4) with s = Z_(2) + Z_(3) (eq. 10 read as a
damped midpoint move).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

STOP_TRIVIAL, STOP_FIXED, STOP_CYCLE, STOP_CAP, STOP_HANDOFF = 1, 2, 3, 4, 5
STOP_NAMES = {1: "trivial", 2: "fixed", 3: "cycle", 4: "cap", 5: "handoff"}
TRACE_W = 8
TRACE_FIELDS = ("k", "dual2", "unsat", "bad", "max_step", "nonzero", "hash", "sum_lam")

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        i64, i32, p = C.c_int64, C.c_int32, C.c_void_p
        L.or_isqrt.restype = i64; L.or_isqrt.argtypes = [i64]
        L.or_nint_sqrt.restype = i64; L.or_nint_sqrt.argtypes = [i64]
        L.or_cost.restype = i64; L.or_cost.argtypes = [p, i64, i64]
        L.or_step.restype = i64; L.or_step.argtypes = [i64]
        L.or_hash.restype = C.c_uint64; L.or_hash.argtypes = [i64, p]
        L.or_check_coords.restype = C.c_int; L.or_check_coords.argtypes = [p, i64]
        L.or_gdp_rows.restype = None
        L.or_gdp_rows.argtypes = [i64, p, p, p, p, p, i64, p, p, p, p, p, p, p]
        L.or_gdp_iter.restype = C.c_int
        L.or_gdp_iter.argtypes = [i64, p, p, p, p, p, p, p, p, p, p, p]
        L.or_gdp_solve.restype = C.c_int
        L.or_gdp_solve.argtypes = [i64, p, p, p, p, p, i64, i64, p, p, p, p, p, p, p, p]
        L.or_certify.restype = C.c_int
        L.or_certify.argtypes = [i64, p, p, p, p, p, i64, p, p, p, p]
        L.or_knn.restype = C.c_int
        L.or_knn.argtypes = [i64, p, i64, p]
        L.or_knn_rows.restype = C.c_int
        L.or_knn_rows.argtypes = [i64, p, i64, i64, p, p]
        L.or_trivial_x.restype = i64
        L.or_trivial_x.argtypes = [i64, p, p, i64, p, p, p]
        L.or_exact_opt2.restype = C.c_int
        L.or_exact_opt2.argtypes = [i64, p, p, p, p, p, p, p]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _graph(graph):
    """(rowptr int64, col int32) or (None, None) for the complete graph."""
    if graph is None:
        return None, None
    rowptr, col = graph
    return np.ascontiguousarray(rowptr, dtype=np.int64), np.ascontiguousarray(col, dtype=np.int32)


def _coords(xy):
    xy = np.ascontiguousarray(xy, dtype=np.int32)
    assert xy.ndim == 2 and xy.shape[1] == 2
    return xy


def num_threads() -> int:
    return int(lib().or_num_threads())


def isqrt(x: int) -> int:
    return int(lib().or_isqrt(int(x)))


def nint_sqrt(D: int) -> int:
    return int(lib().or_nint_sqrt(int(D)))


def cost(xy, u: int, v: int) -> int:
    xy = _coords(xy)
    return int(lib().or_cost(_ptr(xy), int(u), int(v)))


def step(s: int) -> int:
    return int(lib().or_step(int(s)))


def lam_hash(lam) -> int:
    lam = np.ascontiguousarray(lam, dtype=np.int64)
    return int(lib().or_hash(lam.size, _ptr(lam)))


def check_coords(xy) -> int:
    xy = _coords(xy)
    return int(lib().or_check_coords(_ptr(xy), xy.shape[0]))


def _degrees(b, n):
    """Per-node right-hand sides b_v as int32 (None: F2M, every b_v = 2)."""
    if b is None:
        return None
    b = np.ascontiguousarray(b, dtype=np.int32)
    assert b.shape == (n,)
    return b


def gdp_rows(xy, lam, rows, graph=None, b=None):
    """Per-row GDP quantities at Lam for the listed rows (on `graph`, a
    (rowptr, col) CSR candidate graph, or the complete graph; b: per-node
    degrees, None for F2M).
    Returns dict: z4 (r,4) int64, i4 (r,4) int32, neg, zero (int32),
    rowneg, step (int64)."""
    xy = _coords(xy)
    n = xy.shape[0]
    lam = np.ascontiguousarray(lam, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    r = rows.size
    out = dict(z4=np.empty((r, 4), np.int64), i4=np.empty((r, 4), np.int32),
               neg=np.empty(r, np.int32), zero=np.empty(r, np.int32),
               rowneg=np.empty(r, np.int64), step=np.empty(r, np.int64))
    rp, cl = _graph(graph)
    bb = _degrees(b, n)
    lib().or_gdp_rows(n, _ptr(xy), _ptr(rp), _ptr(cl), _ptr(lam), _ptr(bb), r, _ptr(rows), _ptr(out["z4"]),
                      _ptr(out["i4"]),
                      _ptr(out["neg"]), _ptr(out["zero"]), _ptr(out["rowneg"]), _ptr(out["step"]))
    return out


def gdp_iter(xy, lam, graph=None, b=None):
    """One full GDP evaluation at Lam: per-node arrays plus the record
    (dict keyed by TRACE_FIELDS; 'k' is 0)."""
    xy = _coords(xy)
    n = xy.shape[0]
    lam = np.ascontiguousarray(lam, dtype=np.int64)
    z4 = np.empty((n, 4), np.int64); i4 = np.empty((n, 4), np.int32)
    neg = np.empty(n, np.int32); zero = np.empty(n, np.int32); st = np.empty(n, np.int64)
    rec = np.zeros(TRACE_W, np.int64)
    rp, cl = _graph(graph)
    bb = _degrees(b, n)
    rc = lib().or_gdp_iter(n, _ptr(xy), _ptr(rp), _ptr(cl), _ptr(lam), _ptr(bb), _ptr(z4), _ptr(i4), _ptr(neg),
                           _ptr(zero), _ptr(st), _ptr(rec))
    if rc:
        raise RuntimeError("or_gdp_iter failed: %d" % rc)
    r = dict(zip(TRACE_FIELDS, (int(x) for x in rec)))
    r["hash"] &= (1 << 64) - 1
    return dict(z4=z4, i4=i4, neg=neg, zero=zero, step=st, rec=r)


def gdp_solve(xy, lam0=None, max_iters=100000, handoff_div=0, graph=None, b=None):
    """GDP rule loop (handoff_div > 0: stop once #unsatisfied*div <= n).
    Returns dict: lam (Lam*), stop (name), iters,
    kstar, trace (iters x TRACE_W int64), z4/i4/neg/zero at the last
    evaluated iterate."""
    xy = _coords(xy)
    n = xy.shape[0]
    lam = np.zeros(n, np.int64) if lam0 is None else np.array(lam0, dtype=np.int64, copy=True)
    trace = np.zeros((max_iters + 1, TRACE_W), np.int64)
    iters = C.c_int64(0); stop = C.c_int32(0); kstar = C.c_int64(0)
    z4 = np.empty((n, 4), np.int64); i4 = np.empty((n, 4), np.int32)
    neg = np.empty(n, np.int32); zero = np.empty(n, np.int32)
    rp, cl = _graph(graph)
    bb = _degrees(b, n)
    rc = lib().or_gdp_solve(n, _ptr(xy), _ptr(rp), _ptr(cl), _ptr(bb), _ptr(lam), int(max_iters), int(handoff_div),
                            _ptr(trace), C.byref(iters),
                            C.byref(stop), C.byref(kstar), _ptr(z4), _ptr(i4), _ptr(neg), _ptr(zero))
    if rc:
        raise RuntimeError("or_gdp_solve failed: %d" % rc)
    k = iters.value
    return dict(lam=lam, stop=STOP_NAMES[stop.value], iters=k, kstar=kstar.value,
                trace=trace[:k].copy(), z4=z4, i4=i4, neg=neg, zero=zero)


def certify(xy, lam, eu, ev, ex2, graph=None, b=None):
    """Returns dict(primal2, dual2, feasible, certified) on `graph` (the
    complete graph by default)."""
    xy = _coords(xy)
    n = xy.shape[0]
    lam = np.ascontiguousarray(lam, dtype=np.int64)
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    ex2 = np.ascontiguousarray(ex2, dtype=np.uint8)
    out = np.zeros(4, np.int64)
    rp, cl = _graph(graph)
    bb = _degrees(b, n)
    rc = lib().or_certify(n, _ptr(xy), _ptr(rp), _ptr(cl), _ptr(bb), _ptr(lam), eu.size, _ptr(eu), _ptr(ev),
                          _ptr(ex2), _ptr(out))
    if rc:
        raise RuntimeError("or_certify failed: %d" % rc)
    return dict(primal2=int(out[0]), dual2=int(out[1]), feasible=bool(out[2]), certified=bool(out[3]))


def trivial_x(xy, lam, cap=None):
    """Edge list of the trivial solution of Lam (eq. 7): (eu, ev, ex2)."""
    xy = _coords(xy)
    n = xy.shape[0]
    lam = np.ascontiguousarray(lam, dtype=np.int64)
    cap = 4 * n if cap is None else cap
    eu = np.empty(cap, np.int32); ev = np.empty(cap, np.int32); ex2 = np.empty(cap, np.uint8)
    m = lib().or_trivial_x(n, _ptr(xy), _ptr(lam), cap, _ptr(eu), _ptr(ev), _ptr(ex2))
    if m < 0:
        raise RuntimeError("trivial x has more than %d edges" % cap)
    return eu[:m].copy(), ev[:m].copy(), ex2[:m].copy()


def exact_opt2(xy, want_x=False, graph=None, b=None):
    """2 * F2M optimum by min-cost flow on the double cover.  With want_x,
    returns (opt2, x2, lam): the optimal x as a dense (n, n) uint8 matrix of
    x2 = 2x and an optimal Lam = 2*lambda from the flow's potentials."""
    xy = _coords(xy)
    n = xy.shape[0]
    out = C.c_int64(0)
    x2 = np.zeros((n, n), np.uint8) if want_x else None
    lam = np.zeros(n, np.int64) if want_x else None
    rp, cl = _graph(graph)
    bb = _degrees(b, n)
    rc = lib().or_exact_opt2(n, _ptr(xy), _ptr(rp), _ptr(cl), _ptr(bb), C.byref(out), _ptr(x2), _ptr(lam))
    if rc == -3:
        return (None, None, None) if want_x else None
    if rc:
        raise RuntimeError("or_exact_opt2 failed: %d" % rc)
    return (out.value, x2, lam) if want_x else out.value


def dense_to_edges(x2):
    """(n, n) symmetric x2 matrix -> edge list (u < v, x2 > 0)."""
    u, v = np.nonzero(np.triu(x2, 1))
    return u.astype(np.int32), v.astype(np.int32), x2[u, v].astype(np.uint8)


def knn(xy, k):
    """The k nearest neighbours of every node by (D, index): (n, k) int32."""
    xy = _coords(xy)
    n = xy.shape[0]
    idx = np.empty((n, k), np.int32)
    rc = lib().or_knn(n, _ptr(xy), int(k), _ptr(idx))
    if rc:
        raise RuntimeError("or_knn failed: %d" % rc)
    return idx


def knn_rows(xy, k, rows):
    """The k nearest neighbours of the listed rows: (len(rows), k) int32."""
    xy = _coords(xy)
    n = xy.shape[0]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    idx = np.empty((rows.size, k), np.int32)
    rc = lib().or_knn_rows(n, _ptr(xy), int(k), rows.size, _ptr(rows), _ptr(idx))
    if rc:
        raise RuntimeError("or_knn_rows failed: %d" % rc)
    return idx


def knn_graph(xy, k):
    """Union-symmetrised k-nearest-neighbour graph as CSR (rowptr int64,
    col int32), each row's columns increasing."""
    idx = knn(xy, k)
    n = idx.shape[0]
    a = np.repeat(np.arange(n), k)
    b = idx.ravel().astype(np.int64)
    u = np.concatenate([a, b])
    v = np.concatenate([b, a])
    key = np.unique(u * n + v)
    rows, cols = key // n, key % n
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    return np.cumsum(rowptr), cols.astype(np.int32)
