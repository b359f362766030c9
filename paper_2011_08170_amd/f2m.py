"""ctypes binding of libf2m (include/f2m.h): argument marshalling only.

Every computation runs in libf2m.so (HIP kernels for gfx950 plus its host
runtime).  There is no fallback: if the library is missing or no GPU is
present, the calls raise.  Device arrays are passed as torch CUDA tensors
(torch provides device memory only) or raw device pointers.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libf2m.so")

OK, NOT_CERTIFIED = 0, 1
STATUS = {0: "ok", 1: "not certified", -1: "invalid argument", -2: "coordinate span out of range",
          -3: "infeasible (n < 3)", -4: "out of memory", -5: "device error", -6: "buffer too small",
          -7: "multiplier overflow"}
STOP_NAMES = {0: "none", 1: "trivial", 2: "fixed", 3: "cycle", 4: "cap", 5: "handoff"}
FINISH = {"none": 0, "exact": 1}
SCAN = {"culled": 0, "full": 1}
SCAN_KIND_FULL, SCAN_KIND_BUILD, SCAN_KIND_LIST = 0, 1, 2
TRACE_W = 8
TRACE_FIELDS = ("k", "dual2", "unsat", "bad", "max_step", "nonzero", "hash", "sum_lam")
SYMBOLS = ("f2m_opts_default", "f2m_create", "f2m_destroy", "f2m_solve", "f2m_gdp_step", "f2m_certify",
           "f2m_knn_graph", "f2m_solve_batch", "f2m_features", "f2m_mlp_forward", "f2m_mlp_grad", "f2m_mlp_adamw",
           "f2m_result_free", "f2m_status_str", "f2m_last_error", "f2m_device_name",
           "f2m_gdp_step_noalloc", "f2m_sec_gdp", "f2m_sec_certify", "f2m_sec_separate", "f2m_sec_solve")
SEC_MAX_LAYERS = 8   # F2M_SEC_MAX_LAYERS
SEC_TRACE_W = 9
SEC_TRACE_FIELDS = TRACE_FIELDS + ("sum_mu",)
MLP_PARAMS = 18817
NOALLOC_MAX_N = 131072   # F2M_NOALLOC_MAX_N
WARM = {"cold": 0, "user": 1, "mlp": 2, "graph": 3}
GRAPH = {"complete": 0, "knn": 1}
HANDOFF_DIV = 50   # the library default: hand off once #unsatisfied * 50 <= n


class F2MError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))
        self.status = status


class Opts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("rule_version", C.c_uint32), ("graph", C.c_int32),
                ("knn_k", C.c_int32), ("warm", C.c_int32), ("lambda2_init", C.c_void_p), ("mlp_theta", C.c_void_p),
                ("max_iters", C.c_int64),
                ("handoff_div", C.c_int64),
                ("finish", C.c_int32), ("coords_on_device", C.c_int32), ("record_trace", C.c_int32),
                ("chunk", C.c_int32), ("time_kernels", C.c_int32), ("scan_mode", C.c_int32),
                ("scan_rows", C.c_int32), ("scan_slices", C.c_int32), ("hip_stream", C.c_void_p),
                ("k0", C.c_int64), ("resume_hash", C.c_uint64 * 2), ("resume_hash_valid", C.c_int32),
                ("pad_opts", C.c_int32), ("max_device_bytes", C.c_uint64), ("tuner_cache", C.c_char_p),
                ("degree_b", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("n", C.c_int64), ("iterations", C.c_int64), ("kstar", C.c_int64), ("stop", C.c_int32),
                ("certified", C.c_int32), ("lambda2", C.POINTER(C.c_int64)),
                ("lambda2_gdp", C.POINTER(C.c_int64)), ("n_edges", C.c_int64),
                ("edge_u", C.POINTER(C.c_int32)), ("edge_v", C.POINTER(C.c_int32)),
                ("edge_x2", C.POINTER(C.c_uint8)), ("primal2", C.c_int64), ("dual2", C.c_int64),
                ("dual2_gdp", C.c_int64), ("finish_paths", C.c_int64), ("finish_rounds", C.c_int64),
                ("trace_len", C.c_int64), ("trace", C.POINTER(C.c_int64)), ("seconds", C.c_double * 6),
                ("scan_ms", C.c_double), ("scan_launches", C.c_int64), ("scan_rows", C.c_int32),
                ("pad0", C.c_int32), ("scan_slices", C.c_int64), ("scan_pairs", C.c_int64),
                ("finish_phases", C.c_int64), ("finish_candidates", C.c_int64), ("finish_seconds", C.c_double * 3),
                ("dual2_complete", C.c_int64), ("certified_complete", C.c_int32), ("pad1", C.c_int32),
                ("graph_nnz", C.c_int64), ("warm_iterations", C.c_int64),
                ("scan_kind", C.POINTER(C.c_int32)), ("scan_list_uses", C.c_int64),
                ("scan_list_builds", C.c_int64), ("lambda2_last", C.POINTER(C.c_int64)),
                ("scan_ms_kind", C.c_double * 3), ("scan_launches_kind", C.c_int64 * 3),
                ("scan_pairs_kind", C.c_int64 * 3), ("update_ms", C.c_double), ("update_ms_kind", C.c_double * 3)]


_lib = None


class SecRows(C.Structure):
    _fields_ = [("nlayers", C.c_int32), ("reserved", C.c_int32), ("nrows", C.c_int64), ("row_of", C.c_void_p)]


class SecResult(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("kstar", C.c_int64), ("stop", C.c_int32), ("overflow", C.c_int32),
                ("dual2", C.c_int64), ("primal2_last", C.c_int64), ("bad_last", C.c_int64),
                ("seconds", C.c_double), ("pairs_tested", C.c_int64)]


class SecSolveResult(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("nlayers", C.c_int32), ("nrows", C.c_int64),
                ("rows_added", C.c_int64 * SEC_MAX_LAYERS), ("iterations", C.c_int64 * SEC_MAX_LAYERS),
                ("stop", C.c_int32 * SEC_MAX_LAYERS), ("dual2", C.c_int64 * SEC_MAX_LAYERS),
                ("dual2_start", C.c_int64), ("best_dual2", C.c_int64), ("certified", C.c_int32),
                ("components", C.c_int32), ("seconds", C.c_double)]


def lib():
    """Loads libf2m.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libf2m.so is not built: run `python -m paper_2011_08170_amd.build`")
        # Device memory comes from torch; load torch's HIP runtime first so
        # that libf2m binds to the same one (both carry the SONAME
        # libamdhip64.so.7) instead of bringing a second runtime into the
        # process, which would hide the GPUs from torch.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        p, i64 = C.c_void_p, C.c_int64
        L.f2m_opts_default.restype = None
        L.f2m_opts_default.argtypes = [C.POINTER(Opts)]
        L.f2m_create.restype = C.c_int
        L.f2m_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(Opts)]
        L.f2m_destroy.restype = None
        L.f2m_destroy.argtypes = [p]
        L.f2m_solve.restype = C.c_int
        L.f2m_solve.argtypes = [p, p, i64, C.POINTER(Opts), C.POINTER(Result)]
        L.f2m_gdp_step.restype = C.c_int
        L.f2m_gdp_step.argtypes = [p, p, i64, p, p, p, p, p, p, p, p]
        L.f2m_gdp_step_noalloc.restype = C.c_int
        L.f2m_gdp_step_noalloc.argtypes = [p, p, i64, p, p, p, p, p, p, p, p]
        L.f2m_certify.restype = C.c_int
        L.f2m_certify.argtypes = [p, p, i64, p, i64, p, p, p, p]
        L.f2m_features.restype = C.c_int
        L.f2m_features.argtypes = [p, p, i64, p, C.POINTER(C.c_float)]
        L.f2m_mlp_forward.restype = C.c_int
        L.f2m_mlp_forward.argtypes = [p, p, p, i64, p]
        L.f2m_mlp_grad.restype = C.c_int
        L.f2m_mlp_grad.argtypes = [p, p, p, p, i64, p, C.POINTER(C.c_double)]
        L.f2m_mlp_adamw.restype = C.c_int
        L.f2m_mlp_adamw.argtypes = [p, p, p, p, p, i64, C.c_float, C.c_float]
        L.f2m_solve_batch.restype = C.c_int
        L.f2m_solve_batch.argtypes = [p, p, p, C.c_int32, C.POINTER(Opts), p]
        L.f2m_knn_graph.restype = C.c_int
        L.f2m_knn_graph.argtypes = [p, p, i64, C.c_int32, p, p, i64, p]
        L.f2m_sec_gdp.restype = C.c_int
        L.f2m_sec_gdp.argtypes = [p, p, i64, C.POINTER(SecRows), p, p, i64, p, i64, C.POINTER(SecResult)]
        L.f2m_sec_certify.restype = C.c_int
        L.f2m_sec_certify.argtypes = [p, p, i64, C.POINTER(SecRows), p, p, p]
        L.f2m_sec_separate.restype = C.c_int
        L.f2m_sec_separate.argtypes = [p, p, i64, C.POINTER(SecRows), p, p, p, p, p]
        L.f2m_sec_solve.restype = C.c_int
        L.f2m_sec_solve.argtypes = [p, p, i64, p, p, C.c_int32, i64, p, i64, C.c_int32, i64,
                                    C.POINTER(SecSolveResult)]
        L.f2m_result_free.restype = None
        L.f2m_result_free.argtypes = [C.POINTER(Result)]
        L.f2m_status_str.restype = C.c_char_p
        L.f2m_status_str.argtypes = [C.c_int]
        L.f2m_last_error.restype = C.c_char_p
        L.f2m_last_error.argtypes = [p]
        L.f2m_device_name.restype = C.c_char_p
        L.f2m_device_name.argtypes = [p]
        _lib = L
    return _lib


def _dptr(t):
    """Device pointer of a torch tensor (or an int), None for None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class _Owner:
    """Keeps an f2m_result's host arrays alive while numpy views of them
    exist; the library frees them when the last view goes."""

    def __init__(self, res):
        self.res = res

    def __del__(self):
        try:
            lib().f2m_result_free(C.byref(self.res))
        except Exception:
            pass


def _view(owner, ptr, ctype, count):
    """numpy view of `count` entries of a library-owned array (no copy), or
    a copy when there is no owner (the caller frees the result)."""
    if not ptr or count <= 0:
        return np.zeros(0, np.dtype(ctype))
    buf = (ctype * count).from_address(C.cast(ptr, C.c_void_p).value)
    if owner is None:
        return np.frombuffer(buf, dtype=np.dtype(ctype)).copy()
    buf._owner = owner
    return np.frombuffer(buf, dtype=np.dtype(ctype))


def _result_dict(res, n, st, own=True):
    """The result as a dict; with own, its arrays are views that keep the
    result's memory until the last of them goes (else copies)."""
    m = res.n_edges
    owner = _Owner(res) if own else None
    out = dict(
        status=STATUS[st], certified=bool(res.certified), stop=STOP_NAMES.get(res.stop, "?"),
        iterations=res.iterations, kstar=res.kstar, primal2=res.primal2, dual2=res.dual2,
        dual2_gdp=res.dual2_gdp, finish_paths=res.finish_paths, finish_rounds=res.finish_rounds,
        lambda2=_view(owner, res.lambda2, C.c_int64, n),
        lambda2_gdp=_view(owner, res.lambda2_gdp, C.c_int64, n),
        lambda2_last=_view(owner, res.lambda2_last, C.c_int64, n) if res.lambda2_last else None,
        edge_u=_view(owner, res.edge_u, C.c_int32, m),
        edge_v=_view(owner, res.edge_v, C.c_int32, m),
        edge_x2=_view(owner, res.edge_x2, C.c_uint8, m),
        seconds=dict(zip(("setup", "warm", "gdp", "finish", "certify", "total"), list(res.seconds))),
        scan_ms=res.scan_ms, scan_launches=res.scan_launches, scan_rows=res.scan_rows,
        scan_slices=res.scan_slices, scan_pairs=res.scan_pairs,
        finish_phases=res.finish_phases, finish_candidates=res.finish_candidates,
        finish_seconds=dict(zip(("collect", "build", "flow"), list(res.finish_seconds))),
        dual2_complete=res.dual2_complete, certified_complete=bool(res.certified_complete),
        graph_nnz=res.graph_nnz, warm_iterations=res.warm_iterations,
        scan_list_uses=res.scan_list_uses, scan_list_builds=res.scan_list_builds,
        scan_by_kind={name: dict(ms=res.scan_ms_kind[q], launches=res.scan_launches_kind[q],
                                 pairs=res.scan_pairs_kind[q], update_ms=res.update_ms_kind[q])
                      for q, name in enumerate(("full", "build", "list"))},
        update_ms=res.update_ms,
    )
    if res.trace_len:
        out["trace"] = np.ctypeslib.as_array(res.trace, (res.trace_len * TRACE_W,)).reshape(
            res.trace_len, TRACE_W).copy()
        if res.scan_kind:
            out["scan_kind"] = np.ctypeslib.as_array(res.scan_kind, (res.trace_len,)).copy()
    return out


class Context:
    """One libf2m context (device + stream)."""

    def __init__(self, device: int = 0, max_device_bytes: int = 0):
        self._h = C.c_void_p()
        self._max_dev = int(max_device_bytes)
        d = Opts()
        lib().f2m_opts_default(C.byref(d))
        d.max_device_bytes = int(max_device_bytes)
        st = lib().f2m_create(C.byref(self._h), int(device), C.byref(d))
        if st != OK:
            raise F2MError(st, "f2m_create(device=%d) failed" % device)

    def device_name(self) -> str:
        """The device's name as the tuner cache keys it."""
        return lib().f2m_device_name(self._h).decode()

    def close(self):
        if self._h:
            lib().f2m_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st < 0:
            raise F2MError(st, lib().f2m_last_error(self._h).decode())
        return st

    def solve(self, coords, *, max_iters=100000, handoff_div=HANDOFF_DIV, finish="exact", lambda2_init=None,
              trace=False, chunk=0, stream=None, time_kernels=False, scan="culled", graph="complete", knn_k=10,
              shape=None, mlp_theta=None, warm=None, k0=0, resume_hash=None, max_device_bytes=None,
              tuner_cache=None, degree_b=None):
        """Solves F2M on the complete graph.  `coords` is an int32 (n, 2)
        array on the host or a contiguous int32 device tensor."""
        o = Opts()
        lib().f2m_opts_default(C.byref(o))
        o.max_iters = int(max_iters)
        o.handoff_div = int(handoff_div)
        o.finish = FINISH[finish]
        o.record_trace = 1 if trace else 0
        o.chunk = int(chunk)
        o.time_kernels = 1 if time_kernels else 0
        o.scan_mode = SCAN[scan]
        o.graph = GRAPH[graph]
        o.knn_k = int(knn_k)
        if shape is not None:
            o.scan_rows, o.scan_slices = int(shape[0]), int(shape[1])
        o.k0 = int(k0)
        if resume_hash is not None:
            o.resume_hash[0] = int(resume_hash[0]) & ((1 << 64) - 1)
            o.resume_hash[1] = int(resume_hash[1]) & ((1 << 64) - 1)
            o.resume_hash_valid = 1
        o.max_device_bytes = self._max_dev if max_device_bytes is None else int(max_device_bytes)
        keep = []
        if tuner_cache is not None:
            tc = os.fsencode(tuner_cache)
            keep.append(tc)
            o.tuner_cache = tc
        if degree_b is not None:
            bd = _np(degree_b, np.int32)
            keep.append(bd)
            o.degree_b = bd.ctypes.data
        if lambda2_init is not None:
            l0 = _np(lambda2_init, np.int64)
            keep.append(l0)
            o.warm = 1
            o.lambda2_init = l0.ctypes.data
        if stream is not None:
            o.hip_stream = stream
        if mlp_theta is not None:
            o.warm = WARM["mlp"]
            o.mlp_theta = _dptr(mlp_theta)
        if warm is not None:
            o.warm = WARM[warm]
        if hasattr(coords, "is_cuda") and coords.is_cuda:
            o.coords_on_device = 1
            n = coords.shape[0]
            ptr = _dptr(coords)
        else:
            xy = _np(coords, np.int32)
            keep.append(xy)
            n = xy.shape[0]
            ptr = xy.ctypes.data
        res = Result()
        st = self._check(lib().f2m_solve(self._h, ptr, n, C.byref(o), C.byref(res)))
        # the arrays are views of the result's host memory, freed with the last of them
        return _result_dict(res, n, st)

    def solve_batch(self, coords, offsets, *, max_iters=100000, handoff_div=HANDOFF_DIV, finish="exact", trace=False,
                    chunk=0, scan="culled", lambda2_init=None, slices=0, tuner_cache=None):
        """Solves many instances in one batched loop.  coords: int32 (sum n, 2)
        on the host; offsets: int64 (n_inst + 1).  Returns (status, [dict])."""
        o = Opts()
        lib().f2m_opts_default(C.byref(o))
        o.max_iters = int(max_iters)
        o.handoff_div = int(handoff_div)
        o.finish = FINISH[finish]
        o.record_trace = 1 if trace else 0
        o.chunk = int(chunk)
        o.scan_mode = SCAN[scan]
        o.scan_slices = int(slices)
        xy = _np(coords, np.int32)
        off = _np(offsets, np.int64)
        keep = [xy, off]
        if tuner_cache is not None:
            tc = os.fsencode(tuner_cache)
            keep.append(tc)
            o.tuner_cache = tc
        if lambda2_init is not None:
            l0 = _np(lambda2_init, np.int64)
            keep.append(l0)
            o.warm = 1
            o.lambda2_init = l0.ctypes.data
        k = off.size - 1
        arr = (Result * k)()
        st = self._check(lib().f2m_solve_batch(self._h, xy.ctypes.data, off.ctypes.data, k, C.byref(o),
                                               C.cast(arr, C.c_void_p)))
        out = []
        try:
            for i in range(k):
                out.append(_result_dict(arr[i], int(off[i + 1] - off[i]), 0 if arr[i].certified else 1, own=False))
        finally:
            for i in range(k):
                lib().f2m_result_free(C.byref(arr[i]))
        return STATUS[st], out

    def gdp_step(self, coords, lam_in, lam_out, z4=None, i4=None, neg=None, zero=None, step=None):
        """One GDP iteration on device tensors; returns the record dict."""
        return self._step(lib().f2m_gdp_step, coords, lam_in, lam_out, z4, i4, neg, zero, step)

    def gdp_step_noalloc(self, coords, lam_in, lam_out, z4=None, i4=None, neg=None, zero=None, step=None):
        """gdp_step on the library's fixed device workspace (no allocation;
        n <= NOALLOC_MAX_N; calls on one device must not overlap)."""
        return self._step(lib().f2m_gdp_step_noalloc, coords, lam_in, lam_out, z4, i4, neg, zero, step)

    def _step(self, fn, coords, lam_in, lam_out, z4, i4, neg, zero, step):
        n = coords.shape[0]
        rec = np.zeros(TRACE_W, np.int64)
        self._check(fn(self._h, _dptr(coords), n, _dptr(lam_in), _dptr(lam_out), _dptr(z4),
                       _dptr(i4), _dptr(neg), _dptr(zero), _dptr(step), rec.ctypes.data_as(C.c_void_p)))
        r = dict(zip(TRACE_FIELDS, (int(x) for x in rec)))
        r["hash"] &= (1 << 64) - 1
        return r

    def features(self, coords, feat):
        """Warm-start features into feat (uint16 bf16 [n, 16] device tensor,
        viewed as int16 in torch); returns the scale."""
        sc = C.c_float(0.0)
        self._check(lib().f2m_features(self._h, _dptr(coords), coords.shape[0], _dptr(feat), C.byref(sc)))
        return sc.value

    def mlp_forward(self, theta, feat, y):
        self._check(lib().f2m_mlp_forward(self._h, _dptr(theta), _dptr(feat), y.shape[0], _dptr(y)))

    def mlp_grad(self, theta, feat, target, grad):
        loss = C.c_double(0.0)
        self._check(lib().f2m_mlp_grad(self._h, _dptr(theta), _dptr(feat), _dptr(target), target.shape[0],
                                       _dptr(grad), C.byref(loss)))
        return loss.value

    def mlp_adamw(self, theta, grad, m, v, step, lr, wd=0.0):
        self._check(lib().f2m_mlp_adamw(self._h, _dptr(theta), _dptr(grad), _dptr(m), _dptr(v), int(step),
                                        float(lr), float(wd)))

    def certify(self, coords, lam, eu, ev, ex2):
        """Certificate on device tensors: dict(primal2, dual2, feasible, certified)."""
        n = coords.shape[0]
        m = eu.shape[0]
        out = np.zeros(4, np.int64)
        self._check(lib().f2m_certify(self._h, _dptr(coords), n, _dptr(lam), m, _dptr(eu) if m else None,
                                      _dptr(ev) if m else None, _dptr(ex2) if m else None,
                                      out.ctypes.data_as(C.c_void_p)))
        return dict(primal2=int(out[0]), dual2=int(out[1]), feasible=bool(out[2]), certified=bool(out[3]))


    # ---- subtour-elimination rows ----
    @staticmethod
    def _rows(row_of, nrows):
        """f2m_sec_rows from an int32 device tensor [L, n] (or None)."""
        if row_of is None or row_of.shape[0] == 0:
            return SecRows(0, 0, 0, None)
        return SecRows(int(row_of.shape[0]), 0, int(nrows), _dptr(row_of))

    def sec_gdp(self, coords, row_of, nrows, lam, mu, max_iters=100000, trace=True):
        """GDP with subtour rows on device tensors: lam (int64 [n], Lam_0 in,
        Lam* out), mu (int64 [nrows], M_0 in, M* out), row_of (int32 [L, n]
        or None).  Returns the result dict with the trace records."""
        n = coords.shape[0]
        rows = self._rows(row_of, nrows)
        cap = max_iters + 1 if trace else 0
        tr = np.zeros((max(cap, 1), SEC_TRACE_W), np.int64)
        res = SecResult()
        st = lib().f2m_sec_gdp(self._h, _dptr(coords), n, C.byref(rows), _dptr(lam),
                               _dptr(mu) if nrows else None, int(max_iters),
                               tr.ctypes.data_as(C.c_void_p) if cap else None, cap, C.byref(res))
        if st not in (0, -7):
            self._check(st)
        out = dict(iterations=res.iterations, kstar=res.kstar, stop=STOP_NAMES.get(res.stop, str(res.stop)),
                   overflow=bool(res.overflow), dual2=res.dual2, primal2_last=res.primal2_last,
                   bad_last=res.bad_last, seconds=res.seconds, pairs_tested=res.pairs_tested)
        if cap:
            recs = []
            for row in tr[:min(res.iterations, cap)]:
                r = dict(zip(SEC_TRACE_FIELDS, (int(x) for x in row)))
                r["hash"] &= (1 << 64) - 1
                recs.append(r)
            out["trace"] = recs
        return out

    def sec_certify(self, coords, row_of, nrows, lam, mu):
        """Certificate of the trivial x of (Lam, M): dict(primal2, dual2,
        feasible, tight, certified)."""
        rows = self._rows(row_of, nrows)
        out = np.zeros(5, np.int64)
        self._check(lib().f2m_sec_certify(self._h, _dptr(coords), coords.shape[0], C.byref(rows), _dptr(lam),
                                          _dptr(mu) if nrows else None, out.ctypes.data_as(C.c_void_p)))
        return dict(primal2=int(out[0]), dual2=int(out[1]), feasible=bool(out[2]), tight=bool(out[3]),
                    certified=bool(out[4]))

    def sec_separate(self, coords, row_of, nrows, lam, mu, new_row_of):
        """New rows of the violated cuts at (Lam, M) into new_row_of (int32
        [n] device tensor); returns (new rows, components)."""
        rows = self._rows(row_of, nrows)
        nn, nc = C.c_int64(0), C.c_int64(0)
        self._check(lib().f2m_sec_separate(self._h, _dptr(coords), coords.shape[0], C.byref(rows), _dptr(lam),
                                           _dptr(mu) if nrows else None, _dptr(new_row_of), C.byref(nn),
                                           C.byref(nc)))
        return nn.value, nc.value

    def sec_solve(self, coords, lam, row_of, mu, nlayers0=0, nrows0=0, max_rounds=SEC_MAX_LAYERS,
                  max_iters=100000):
        """Rounds of separation and GDP (f2m_sec_solve) on device tensors:
        lam int64 [n] in/out, row_of int32 [SEC_MAX_LAYERS, n], mu int64
        [cap]; returns the result dict."""
        res = SecSolveResult()
        st = lib().f2m_sec_solve(self._h, _dptr(coords), coords.shape[0], _dptr(lam), _dptr(row_of),
                                 int(nlayers0), int(nrows0), _dptr(mu), int(mu.shape[0]), int(max_rounds),
                                 int(max_iters), C.byref(res))
        if st not in (0, -7):
            self._check(st)
        r = res.rounds
        return dict(rounds=r, nlayers=res.nlayers, nrows=res.nrows, rows_added=list(res.rows_added[:r]),
                    iterations=list(res.iterations[:r]), stop=[STOP_NAMES.get(x, str(x)) for x in res.stop[:r]],
                    dual2=list(res.dual2[:r]), dual2_start=res.dual2_start, best_dual2=res.best_dual2,
                    certified=bool(res.certified), components=res.components, seconds=res.seconds,
                    overflow=st == -7)


def knn_graph(ctx, coords, k=10):
    """CSR (rowptr, col) of the candidate graph over labels, from a device
    coordinate tensor; returns numpy arrays."""
    import torch
    n = coords.shape[0]
    rowptr = torch.empty(n + 1, dtype=torch.int32, device=coords.device)
    cap = 2 * k * n
    col = torch.empty(cap, dtype=torch.int32, device=coords.device)
    nnz = C.c_int64(0)
    ctx._check(lib().f2m_knn_graph(ctx._h, _dptr(coords), n, int(k), _dptr(rowptr), _dptr(col), cap,
                                   C.byref(nnz)))
    return rowptr.cpu().numpy().astype(np.int64), col[:nnz.value].cpu().numpy()
