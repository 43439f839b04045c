"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and its host-side validator returns the documented
status codes."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import gen
import paper_2306_10025_amd as pr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "patchrelax.h")
INCLUDE = HEADER

pytestmark = pytest.mark.skipif(not os.path.exists(pr.LIB_PATH),
                                reason="libpatchrelax.so not built (run __graft_entry__.build())")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:void|int|const char\*)\s+(pr_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["pr_setup", "pr_apply", "pr_solve", "pr_destroy", "pr_get_assignment",
                     "pr_get_patch_tile", "pr_validate_host", "pr_batch_inverse",
                     "pr_batch_criterion"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(pr.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) == set(pr._SIGS)


def test_param_defaults_and_struct_layout():
    p = pr.pr_params_default()
    assert p.algo == 0 and p.criterion == 0 and p.eps == 1e-8 and p.kmeans_max_iter == 100
    assert p.seed == 5 and p.tie_rel == 1e-9 and p.omega == 1.0 and p.sweeps == 1
    assert p.gmres_restart == 30 and p.max_iters == 10000 and p.partition_bc == 1
    assert p.mlp == 0 and p.mlp_topk == 4 and p.mlp_train_frac == 0.1 and p.mlp_hidden == 64
    assert p.mlp_precision == pr.PREC["fp16"]


def test_struct_layouts_match_the_c_compiler(tmp_path):
    # the binding's ctypes structs against gcc's layout of the header
    structs = [pr.pr_params, pr.pr_stats, pr.pr_solve_info, pr.pr_csr, pr.pr_patches]
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{INCLUDE}"', 'int main(void) {']
    for S in structs:
        lines.append(f'printf("{S.__name__} %zu\\n", sizeof({S.__name__}));')
        for f, _ in S._fields_:
            lines.append(f'printf("{S.__name__}.{f} %zu\\n", offsetof({S.__name__}, {f}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for S in structs:
        assert int(got[S.__name__]) == ctypes.sizeof(S), S.__name__
        for f, _ in S._fields_:
            assert int(got[f"{S.__name__}.{f}"]) == getattr(S, f).offset, (S.__name__, f)


def test_status_strings():
    assert pr.pr_status_string(0) == "ok"
    assert "uncovered" in pr.pr_status_string(pr.PR_ERR_UNCOVERED_DOF) or \
        "no patch" in pr.pr_status_string(pr.PR_ERR_UNCOVERED_DOF)
    assert pr.pr_status_string(12345) == "unknown status"


def _q1():
    P = gen.q1_poisson_2d(4)
    return P.A.indptr, P.A.indices, P.A.data, P.ptr, P.dofs, P.n


def test_validate_host_accepts_good_input():
    assert pr.pr_validate_host(*_q1()) == pr.PR_OK


def test_validate_host_error_codes():
    indptr, indices, data, ptr, dofs, n = _q1()
    d = dofs.copy()
    d[3] = n + 5
    assert pr.pr_validate_host(indptr, indices, data, ptr, d, n) == pr.PR_ERR_DOF_OUT_OF_RANGE
    d = dofs.copy()
    d[1] = d[0]
    assert pr.pr_validate_host(indptr, indices, data, ptr, d, n) == pr.PR_ERR_DUP_DOF_IN_PATCH
    # drop the last patch: the corner dof it alone covers becomes uncovered
    assert pr.pr_validate_host(indptr, indices, data, ptr[:-1], dofs[:ptr[-2]], n) == \
        pr.PR_ERR_UNCOVERED_DOF
    bad = indices.copy()
    row = int(np.argmax(np.diff(indptr)))          # a row with several entries
    bad[indptr[row]], bad[indptr[row] + 1] = bad[indptr[row] + 1], bad[indptr[row]]
    assert pr.pr_validate_host(indptr, bad, data, ptr, dofs, n) == pr.PR_ERR_BAD_CSR
    p2 = ptr.copy()
    p2[2] = p2[1]
    assert pr.pr_validate_host(indptr, indices, data, p2, dofs, n) == pr.PR_ERR_BAD_PATCH_PTR
    nan = data.copy()
    nan[7] = np.nan
    assert pr.pr_validate_host(indptr, indices, nan, ptr, dofs, n) == pr.PR_ERR_NONFINITE
    # patches above 32 dofs take the wide kernels, up to 512 dofs
    A = gen.q1_poisson_2d(6)    # 49 dofs
    ptr2 = np.array([0, 33, 49], dtype=np.int64)
    dofs2 = np.arange(49, dtype=np.int32)
    assert pr.pr_validate_host(A.A.indptr, A.A.indices, A.A.data, ptr2, dofs2, A.n) == pr.PR_OK
    B = gen.q1_poisson_2d(22)   # 529 dofs
    ptr3 = np.array([0, 513, 529], dtype=np.int64)
    dofs3 = np.arange(529, dtype=np.int32)
    assert pr.pr_validate_host(B.A.indptr, B.A.indices, B.A.data, ptr3, dofs3, B.n) == \
        pr.PR_ERR_UNSUPPORTED
    ptr4 = np.array([0, 512, 529], dtype=np.int64)
    assert pr.pr_validate_host(B.A.indptr, B.A.indices, B.A.data, ptr4, dofs3, B.n) == pr.PR_OK


def test_setup_rejects_host_pointers_without_gpu_work():
    # host memory passed where device memory is required -> HOST_POINTER,
    # decided before any kernel launch
    indptr, indices, data, ptr, dofs, n = _q1()
    indptr = np.ascontiguousarray(indptr, np.int64)
    indices = np.ascontiguousarray(indices, np.int32)
    data = np.ascontiguousarray(data)
    ptr = np.ascontiguousarray(ptr, np.int64)
    dofs = np.ascontiguousarray(dofs, np.int32)
    A = pr.pr_csr(n, len(indices), indptr.ctypes.data_as(ctypes.c_void_p),
                  indices.ctypes.data_as(ctypes.c_void_p), data.ctypes.data_as(ctypes.c_void_p))
    P = pr.pr_patches(len(ptr) - 1, ptr.ctypes.data_as(ctypes.c_void_p),
                      dofs.ctypes.data_as(ctypes.c_void_p))
    prm = pr.pr_params_default()
    h = ctypes.c_void_p()
    rc = pr.lib().pr_setup(ctypes.byref(A), ctypes.byref(P), ctypes.byref(prm), ctypes.byref(h))
    assert rc in (pr.PR_ERR_HOST_POINTER, pr.PR_ERR_HIP)
    assert not h.value


def test_setup_rejects_bad_params():
    prm = pr.make_params(sweeps=0)
    A = pr.pr_csr(4, 0, None, None, None)
    P = pr.pr_patches(1, None, None)
    h = ctypes.c_void_p()
    rc = pr.lib().pr_setup(ctypes.byref(A), ctypes.byref(P), ctypes.byref(prm), ctypes.byref(h))
    assert rc == pr.PR_ERR_INVALID_ARG


def test_memory_cache_calls_need_no_gpu():
    # a device never used reports an empty cache; bad arguments are rejected
    info = pr.pr_memory_cache_info(7)
    assert info == dict(idle_bytes=0, idle_blocks=0, reuses=0, mallocs=0)
    L = pr.lib()
    assert L.pr_memory_cache_info(0, None) == pr.PR_ERR_INVALID_ARG
    assert L.pr_memory_cache_info(-2, (ctypes.c_int64 * 4)()) == pr.PR_ERR_INVALID_ARG
    assert L.pr_set_memory_cache_limit(-2) == pr.PR_ERR_INVALID_ARG
