"""Builds and loads the CPU harness around libf2m's host finish."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2011_08170_amd", "csrc")


def build(outdir):
    so = os.path.join(str(outdir), "finish_harness.so")
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", CSRC, "-o", so,
           os.path.join(HERE, "finish_harness.cpp"), os.path.join(CSRC, "f2m_finish.cpp")]
    subprocess.run(cmd, check=True)
    L = C.CDLL(so)
    L.finish_cpu.restype = C.c_int64
    L.finish_cpu.argtypes = [C.c_int64] + [C.c_void_p] * 2 + [C.c_void_p, C.c_int64] + [C.c_void_p] * 4 + \
        [C.c_int32, C.c_int32, C.c_void_p]
    return L


def finish(L, xy, lam0, bulk=False, reuse=0, b=None):
    xy = np.ascontiguousarray(xy, np.int32)
    n = xy.shape[0]
    lam0 = np.ascontiguousarray(lam0, np.int64)
    lam = np.zeros(n, np.int64)
    cap = 6 * n
    eu = np.zeros(cap, np.int32); ev = np.zeros(cap, np.int32); ex = np.zeros(cap, np.uint8)
    st = np.zeros(4, np.int64)
    bb = None if b is None else np.ascontiguousarray(b, np.int32)
    m = L.finish_cpu(n, xy.ctypes.data, lam0.ctypes.data, lam.ctypes.data, cap, eu.ctypes.data,
                     ev.ctypes.data, ex.ctypes.data, st.ctypes.data, int(bulk), int(reuse),
                     None if bb is None else bb.ctypes.data)
    assert m >= 0, "finish failed"
    return lam, eu[:m], ev[:m], ex[:m], dict(zip(("paths", "rounds", "phases", "candidates"), st.tolist()))
