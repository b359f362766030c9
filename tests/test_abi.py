"""The C-ABI library loads and exports every function include/f2m.h
declares (no GPU needed: nothing here launches work)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "f2m.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(f2m_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("f2m_create", "f2m_solve", "f2m_gdp_step", "f2m_certify", "f2m_destroy",
                 "f2m_result_free", "f2m_last_error", "f2m_status_str", "f2m_opts_default"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2011_08170_amd import f2m
    L = f2m.lib()
    for name in declared():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", f2m.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (f2m_\w+)", out))
    assert set(declared()) <= exported
    assert set(f2m.SYMBOLS) <= exported


def test_header_compiles_as_c():
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c",
                        os.path.join(ROOT, "include", "f2m.h")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_struct_layout_matches_binding():
    # the ctypes structures must match the C structs byte for byte
    from paper_2011_08170_amd import f2m
    probe = r'''
#include "f2m.h"
#include <stdio.h>
#include <stddef.h>
int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(f2m_opts), sizeof(f2m_result),
 offsetof(f2m_opts, hip_stream), offsetof(f2m_result, seconds), offsetof(f2m_result, graph_nnz),
 offsetof(f2m_result, warm_iterations), offsetof(f2m_result, scan_kind),
 offsetof(f2m_result, scan_list_builds), offsetof(f2m_opts, tuner_cache),
 offsetof(f2m_result, lambda2_last), offsetof(f2m_result, scan_pairs_kind),
 offsetof(f2m_result, update_ms_kind), offsetof(f2m_opts, degree_b));return 0;}
'''
    import tempfile
    d = tempfile.mkdtemp()
    c = os.path.join(d, "p.c")
    open(c, "w").write(probe)
    exe = os.path.join(d, "p")
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
    vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(f2m.Opts), ctypes.sizeof(f2m.Result), f2m.Opts.hip_stream.offset,
                    f2m.Result.seconds.offset, f2m.Result.graph_nnz.offset, f2m.Result.warm_iterations.offset,
                    f2m.Result.scan_kind.offset, f2m.Result.scan_list_builds.offset, f2m.Opts.tuner_cache.offset,
                    f2m.Result.lambda2_last.offset, f2m.Result.scan_pairs_kind.offset,
                    f2m.Result.update_ms_kind.offset, f2m.Opts.degree_b.offset]


def test_sec_struct_layout_matches_binding():
    from paper_2011_08170_amd import f2m
    probe = r'''
#include "f2m.h"
#include <stdio.h>
#include <stddef.h>
int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %d %d\n", sizeof(f2m_sec_rows), offsetof(f2m_sec_rows, row_of),
 sizeof(f2m_sec_result), offsetof(f2m_sec_result, dual2), offsetof(f2m_sec_result, pairs_tested),
 sizeof(f2m_sec_solve_result), offsetof(f2m_sec_solve_result, stop), offsetof(f2m_sec_solve_result, dual2),
 offsetof(f2m_sec_solve_result, certified), offsetof(f2m_sec_solve_result, seconds),
 F2M_SEC_MAX_LAYERS, F2M_SEC_TRACE_W);return 0;}
'''
    import tempfile
    d = tempfile.mkdtemp()
    c = os.path.join(d, "p.c")
    open(c, "w").write(probe)
    exe = os.path.join(d, "p")
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
    vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(f2m.SecRows), f2m.SecRows.row_of.offset, ctypes.sizeof(f2m.SecResult),
                    f2m.SecResult.dual2.offset, f2m.SecResult.pairs_tested.offset, ctypes.sizeof(f2m.SecSolveResult),
                    f2m.SecSolveResult.stop.offset, f2m.SecSolveResult.dual2.offset,
                    f2m.SecSolveResult.certified.offset, f2m.SecSolveResult.seconds.offset,
                    f2m.SEC_MAX_LAYERS, f2m.SEC_TRACE_W]


def test_no_gpu_fails_loudly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2011_08170_amd import f2m
    with pytest.raises(f2m.F2MError):
        f2m.Context(0)
