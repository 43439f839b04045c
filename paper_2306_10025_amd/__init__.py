"""Python binding of libpatchrelax.so (compressed patch-based relaxation on
MI355X / gfx950).

Argument marshalling only: every step of setup, apply and solve runs in the
library's HIP kernels.  PyTorch supplies device memory (tensor data pointers)
and the HIP stream.  The functions keep the C names (``pr_setup``,
``pr_apply``, ``pr_solve``, ...); ``PatchRelax`` is a small owner object on
top of them.  The library must be built first (``__graft_entry__.build()``);
nothing here falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, byref, c_char_p, c_double, c_int, c_int32, c_int64,
                    c_uint32, c_uint64, c_void_p)

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpatchrelax.so")

# status codes (include/patchrelax.h)
PR_OK = 0
PR_NOT_CONVERGED = 1
PR_ERR_INVALID_ARG = -1
PR_ERR_HOST_POINTER = -2
PR_ERR_DOF_OUT_OF_RANGE = -3
PR_ERR_DUP_DOF_IN_PATCH = -4
PR_ERR_UNCOVERED_DOF = -5
PR_ERR_SINGULAR_PATCH = -6
PR_ERR_NONFINITE = -7
PR_ERR_OOM = -8
PR_ERR_HIP = -9
PR_ERR_UNSUPPORTED = -10
PR_ERR_BAD_CSR = -11
PR_ERR_BAD_PATCH_PTR = -12

ALGO = dict(full=0, tolerance=1, kmeans_spectral=2, kmeans_entrywise=3, varmin=4, bootstrap=5)
CRIT = dict(spectral=0, l1=1, fro=2)
PREC = dict(fp64=0, fp32=1, bf16=2, fp16=3, bf16x3=4)
FORM = dict(auto=0, general=1, tiles=2)


class pr_csr(Structure):
    _fields_ = [("n", c_int64), ("nnz", c_int64), ("row_ptr", c_void_p), ("col", c_void_p),
                ("val", c_void_p)]


class pr_patches(Structure):
    _fields_ = [("n_p", c_int64), ("ptr", c_void_p), ("dofs", c_void_p)]


class pr_interp(Structure):
    _fields_ = [("n_fine", c_int64), ("n_coarse", c_int64), ("nnz", c_int64), ("row_ptr", c_void_p),
                ("col", c_void_p), ("val", c_void_p)]


class pr_params(Structure):
    _fields_ = [("algo", c_int32), ("criterion", c_int32), ("eps", c_double),
                ("m_target", c_int64), ("partition_bc", c_int32), ("kmeans_max_iter", c_int32),
                ("seed", c_uint64), ("tie_rel", c_double), ("apply_precision", c_int32),
                ("omega", c_double), ("sweeps", c_int32), ("gmres_restart", c_int32),
                ("max_iters", c_int64), ("deterministic", c_int32), ("timing", c_int32),
                ("stream", c_void_p), ("mlp", c_int32), ("mlp_topk", c_int32),
                ("mlp_train_frac", c_double), ("mlp_epochs", c_int32), ("mlp_hidden", c_int32),
                ("mlp_seed", c_uint64), ("mlp_lr", c_double), ("mlp_batch", c_int32),
                ("mlp_precision", c_int32), ("graph", c_int32), ("autotune", c_int32),
                ("apply_form", c_int32), ("alg1_prune", c_int32), ("alg1_match", c_int32),
                ("flexible", c_int32), ("orth", c_int32)]


class pr_solve_info(Structure):
    _fields_ = [("iters", c_int64), ("cycles", c_int64), ("relres", c_double),
                ("relres_est", c_double), ("status", c_int32), ("reorth", c_int32),
                ("seconds", c_double), ("apply_ms", c_double), ("spmv_ms", c_double),
                ("orth_ms", c_double), ("n_apply", c_int64), ("n_spmv", c_int64),
                ("n_orth", c_int64), ("coarse_ms", c_double), ("n_coarse", c_int64)]


class pr_stats(Structure):
    _fields_ = [("n", c_int64), ("nnz", c_int64), ("n_p", c_int64), ("m_p", c_int64),
                ("max_ps", c_int32), ("min_ps", c_int32), ("n_groups", c_int32), ("algo", c_int32),
                ("crit_evals", c_int64), ("crit_pruned", c_int64), ("crit_exact", c_int64),
                ("alg1_rounds", c_int64), ("kmeans_iters", c_int64), ("empty_events", c_int64),
                ("n_items", c_int64), ("bytes_tiles", c_int64), ("bytes_db", c_int64),
                ("bytes_db_lowp", c_int64), ("bytes_index", c_int64),
                ("t_validate", c_double), ("t_extract", c_double), ("t_database", c_double),
                ("t_factor", c_double), ("t_group", c_double), ("t_total", c_double),
                ("apply_precision", c_int32), ("apply_tile_p", c_int32),
                ("mlp_train", c_int64), ("mlp_classes", c_int64), ("mlp_accepted", c_int64),
                ("mlp_scanned", c_int64), ("mlp_fallback", c_int64), ("mlp_loss", c_double),
                ("mlp_train_acc", c_double), ("t_mlp_train", c_double),
                ("tune_threads", c_int32), ("tune_slot", c_int32), ("tune_cap", c_int64),
                ("t_autotune", c_double), ("tune_tiles_per_wave", c_int64),
                ("tune_xcd_remap", c_int64), ("crit_refined", c_int64), ("sell_slots", c_int64),
                ("sell_diag_slices", c_int64), ("sell_diag_offsets", c_int64), ("sell_col_entries", c_int64),
                ("alg1_batch_inverted", c_int64), ("closest_evals", c_int64),
                ("closest_moved", c_int64), ("n_coarse", c_int64), ("coarse_nnz", c_int64),
                ("coarse_bandwidth", c_int64), ("coarse_block", c_int64), ("coarse_blocks", c_int64),
                ("t_coarse", c_double), ("reuse_kept", c_int64), ("reuse_rescanned", c_int64),
                ("reuse_appended", c_int64), ("sell_csr_slices", c_int64), ("sell_csr_entries", c_int64)]


_SIGS = {
    "pr_params_default": (None, [POINTER(pr_params)]),
    "pr_setup": (c_int, [POINTER(pr_csr), POINTER(pr_patches), POINTER(pr_params), POINTER(c_void_p)]),
    "pr_apply": (c_int, [c_void_p, c_void_p, c_void_p]),
    "pr_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_double]),
    "pr_get_solve_info": (c_int, [c_void_p, POINTER(pr_solve_info)]),
    "pr_export_database": (c_int, [c_void_p, c_void_p, POINTER(c_int64)]),
    "pr_setup_reuse": (c_int, [POINTER(pr_csr), POINTER(pr_patches), POINTER(pr_params), c_void_p, c_int64,
                               POINTER(c_void_p)]),
    "pr_set_coarse": (c_int, [c_void_p, POINTER(pr_interp)]),
    "pr_get_coarse_matrix": (c_int, [c_void_p, POINTER(c_int64), POINTER(c_int64), c_void_p, c_void_p,
                                     c_void_p]),
    "pr_get_stats": (c_int, [c_void_p, POINTER(pr_stats)]),
    "pr_get_assignment": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_int64)]),
    "pr_get_patch_tile": (c_int, [c_void_p, c_int64, c_void_p]),
    "pr_get_weights": (c_int, [c_void_p, c_void_p]),
    "pr_get_boundary_keys": (c_int, [c_void_p, c_void_p]),
    "pr_get_rep_inverse": (c_int, [c_void_p, c_int64, c_void_p]),
    "pr_get_entry_matrix": (c_int, [c_void_p, c_int64, c_void_p]),
    "pr_set_stream": (c_int, [c_void_p, c_void_p]),
    "pr_validate_host": (c_int, [POINTER(pr_csr), POINTER(pr_patches)]),
    "pr_destroy": (None, [c_void_p]),
    "pr_set_memory_cache_limit": (c_int, [c_int64]),
    "pr_release_cached_memory": (c_int, []),
    "pr_memory_cache_info": (c_int, [c_int32, POINTER(c_int64)]),
    "pr_status_string": (c_char_p, [c_int]),
    "pr_last_error": (c_char_p, [c_void_p]),
    "pr_batch_inverse": (c_int, [c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pr_batch_criterion": (c_int, [c_int32, c_int64, c_int32, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p]),
    "pr_set_systems": (c_int, [c_void_p, c_void_p, c_int64]),
    "pr_get_system_info": (c_int, [c_void_p, c_void_p, c_void_p]),
    "pr_get_mlp_candidates": (c_int, [c_void_p, c_void_p, c_void_p]),
    "pr_get_mlp_features": (c_int, [c_void_p, c_void_p, POINTER(c_int32)]),
    "pr_mlp_loss_grad": (c_int, [c_int32, c_int64, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double), c_void_p]),
    "pr_mlp_predict": (c_int, [c_int32, c_int64, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "pr_mlp_predict_noalloc": (c_int, [c_int32, c_int64, c_int32, c_int32, c_int32, c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                       c_void_p]),
}

_lib = None


def lib():
    """Load libpatchrelax.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class PatchRelaxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{code} ({pr_status_string(code)}): {msg}")
        self.code = code


def pr_status_string(code: int) -> str:
    return lib().pr_status_string(code).decode()


def pr_last_error(h=None) -> str:
    s = lib().pr_last_error(h)
    return s.decode() if s else ""


def _check(code, h=None, allow=(PR_OK,)):
    if code not in allow:
        raise PatchRelaxError(code, pr_last_error(h))
    return code


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def pr_params_default() -> pr_params:
    p = pr_params()
    lib().pr_params_default(byref(p))
    return p


def make_params(algo="full", criterion="spectral", eps=1e-8, m_target=0, partition_bc=True,
                kmeans_max_iter=100, seed=5, tie_rel=1e-9, precision="fp64", omega=1.0, sweeps=1,
                restart=30, max_iters=10000, deterministic=False, timing=False,
                stream=None, mlp=False, mlp_topk=4, mlp_train_frac=0.1, mlp_epochs=60,
                mlp_hidden=64, mlp_seed=6, mlp_lr=3e-3, mlp_batch=256,
                mlp_precision="fp16", graph=False, autotune=False, apply_form="auto",
                alg1_prune=True, alg1_match="first", flexible=False, orth="delayed") -> pr_params:
    p = pr_params_default()
    p.flexible = int(flexible)
    p.orth = {"delayed": 0, "selective": 1}[orth] if isinstance(orth, str) else int(orth)
    p.alg1_prune = int(alg1_prune)
    p.alg1_match = {"first": 0, "closest": 1}[alg1_match] if isinstance(alg1_match, str) else int(alg1_match)
    p.graph = int(graph)
    p.autotune = int(autotune)
    p.apply_form = FORM[apply_form] if isinstance(apply_form, str) else int(apply_form)
    p.mlp = int(mlp)
    p.mlp_topk = mlp_topk
    p.mlp_train_frac = mlp_train_frac
    p.mlp_epochs = mlp_epochs
    p.mlp_hidden = mlp_hidden
    p.mlp_seed = mlp_seed
    p.mlp_lr = mlp_lr
    p.mlp_batch = mlp_batch
    p.mlp_precision = PREC[mlp_precision] if isinstance(mlp_precision, str) else int(mlp_precision)
    p.algo = ALGO[algo] if isinstance(algo, str) else int(algo)
    p.criterion = CRIT[criterion] if isinstance(criterion, str) else int(criterion)
    p.eps = eps
    p.m_target = m_target
    p.partition_bc = int(partition_bc)
    p.kmeans_max_iter = kmeans_max_iter
    p.seed = seed
    p.tie_rel = tie_rel
    p.apply_precision = PREC[precision] if isinstance(precision, str) else int(precision)
    p.omega = omega
    p.sweeps = sweeps
    p.gmres_restart = restart
    p.max_iters = max_iters
    p.deterministic = int(deterministic)
    p.timing = int(timing)
    p.stream = stream
    return p


def pr_setup(row_ptr, col, val, ptr, dofs, n, params: pr_params):
    """Device tensors in, handle out (raises PatchRelaxError on failure)."""
    A = pr_csr(n, int(col.numel()), _ptr(row_ptr), _ptr(col), _ptr(val))
    P = pr_patches(int(ptr.numel()) - 1, _ptr(ptr), _ptr(dofs))
    h = c_void_p()
    _check(lib().pr_setup(byref(A), byref(P), byref(params), byref(h)))
    return h


def pr_export_database(h):
    """The handle's database (phi and entry patch ids) as bytes."""
    n = c_int64()
    _check(lib().pr_export_database(h, None, byref(n)), h)
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().pr_export_database(h, buf, byref(n)), h)
    return buf.raw[:n.value]


def pr_setup_reuse(row_ptr, col, val, ptr, dofs, n, params: pr_params, blob: bytes):
    """pr_setup seeded with an exported database (the previous system's)."""
    A = pr_csr(n, int(col.numel()), _ptr(row_ptr), _ptr(col), _ptr(val))
    P = pr_patches(int(ptr.numel()) - 1, _ptr(ptr), _ptr(dofs))
    h = c_void_p()
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(lib().pr_setup_reuse(byref(A), byref(P), byref(params), buf, len(blob), byref(h)))
    return h


def pr_apply(h, r, z):
    return _check(lib().pr_apply(h, _ptr(r), _ptr(z)), h)


def pr_solve(h, b, x, tol):
    return _check(lib().pr_solve(h, _ptr(b), _ptr(x), tol), h, allow=(PR_OK, PR_NOT_CONVERGED))


def pr_get_solve_info(h) -> dict:
    i = pr_solve_info()
    _check(lib().pr_get_solve_info(h, byref(i)), h)
    return {k: getattr(i, k) for k, _ in pr_solve_info._fields_ if k != "reserved0"}


def pr_get_stats(h) -> dict:
    s = pr_stats()
    _check(lib().pr_get_stats(h, byref(s)), h)
    return {k: getattr(s, k) for k, _ in pr_stats._fields_}


def pr_get_assignment(h, n_p):
    m = c_int64()
    _check(lib().pr_get_assignment(h, None, None, byref(m)), h)
    phi = np.zeros(n_p, dtype=np.int32)
    reps = np.zeros(max(m.value, 1), dtype=np.int32)
    _check(lib().pr_get_assignment(h, phi.ctypes.data_as(c_void_p), reps.ctypes.data_as(c_void_p),
                                   byref(m)), h)
    return phi, reps[:m.value]


def pr_get_patch_tile(h, k, p):
    t = np.zeros(p * p, dtype=np.float64)
    _check(lib().pr_get_patch_tile(h, k, t.ctypes.data_as(c_void_p)), h)
    return t.reshape(p, p)


def pr_get_weights(h, n):
    W = np.zeros(n, dtype=np.float64)
    _check(lib().pr_get_weights(h, W.ctypes.data_as(c_void_p)), h)
    return W


def pr_get_boundary_keys(h, n_p):
    k = np.zeros(n_p, dtype=np.uint32)
    _check(lib().pr_get_boundary_keys(h, k.ctypes.data_as(c_void_p)), h)
    return k


def pr_get_rep_inverse(h, j, p):
    X = np.zeros(p * p, dtype=np.float64)
    _check(lib().pr_get_rep_inverse(h, j, X.ctypes.data_as(c_void_p)), h)
    return X.reshape(p, p)


def pr_get_entry_matrix(h, j, p):
    B = np.zeros(p * p, dtype=np.float64)
    _check(lib().pr_get_entry_matrix(h, j, B.ctypes.data_as(c_void_p)), h)
    return B.reshape(p, p)


def pr_set_systems(h, system_ptr):
    sp = np.ascontiguousarray(system_ptr, dtype=np.int64)
    return _check(lib().pr_set_systems(h, sp.ctypes.data_as(c_void_p), len(sp) - 1), h)


def pr_get_system_info(h, n_sys):
    it = np.zeros(n_sys, dtype=np.int64)
    rel = np.zeros(n_sys, dtype=np.float64)
    _check(lib().pr_get_system_info(h, it.ctypes.data_as(c_void_p), rel.ctypes.data_as(c_void_p)), h)
    return it, rel


def pr_get_mlp_candidates(h, n_p, n_train, k):
    train = np.zeros(max(n_train, 1), dtype=np.int32)
    cand = np.zeros(n_p * k, dtype=np.int32)
    _check(lib().pr_get_mlp_candidates(h, train.ctypes.data_as(c_void_p), cand.ctypes.data_as(c_void_p)), h)
    return train[:n_train], cand.reshape(n_p, k)


def pr_get_mlp_features(h, n_p):
    F = c_int32()
    _check(lib().pr_get_mlp_features(h, None, byref(F)), h)
    X = np.zeros(n_p * F.value, dtype=np.float32)
    _check(lib().pr_get_mlp_features(h, X.ctypes.data_as(c_void_p), byref(F)), h)
    return X.reshape(n_p, F.value)


def pr_mlp_loss_grad(precision, X, y, params, grads, F, H, C, row_key=None, class_key=None):
    """Mean cross-entropy and its gradient (device tensors; returns the loss)."""
    prec = PREC[precision] if isinstance(precision, str) else int(precision)
    loss = c_double()
    _check(lib().pr_mlp_loss_grad(prec, int(y.numel()), F, H, C, _ptr(X), _ptr(y), _ptr(row_key),
                                  _ptr(class_key), _ptr(params), _ptr(grads), byref(loss), _stream()))
    return loss.value


def pr_mlp_predict(precision, X, params, F, H, C, k, logits=None, topk=None, row_key=None,
                   class_key=None):
    prec = PREC[precision] if isinstance(precision, str) else int(precision)
    rows = int(X.numel()) // F
    return _check(lib().pr_mlp_predict(prec, rows, F, H, C, _ptr(X), _ptr(row_key), _ptr(class_key),
                                       _ptr(params), k, _ptr(logits), _ptr(topk), _stream()))


def pr_mlp_predict_noalloc(precision, X, params, F, H, C, k, logits=None, topk=None, row_key=None,
                           class_key=None):
    """pr_mlp_predict on the library's fixed workspace (asynchronous on the current stream)."""
    prec = PREC[precision] if isinstance(precision, str) else int(precision)
    rows = int(X.numel()) // F
    return _check(lib().pr_mlp_predict_noalloc(prec, rows, F, H, C, _ptr(X), _ptr(row_key),
                                               _ptr(class_key), _ptr(params), k, _ptr(logits),
                                               _ptr(topk), _stream()))


MLP_NOALLOC_SCRATCH_BYTES = 32 << 20


def pr_set_coarse(h, row_ptr, col, val, n_fine, n_coarse):
    """Two-level combination (Eq.(2)) from the interpolation P0 given as device
    CSR tensors (n_fine rows, n_coarse columns)."""
    P = pr_interp(n_fine, n_coarse, int(col.numel()), _ptr(row_ptr), _ptr(col), _ptr(val))
    return _check(lib().pr_set_coarse(h, byref(P)), h)


def pr_get_coarse_matrix(h):
    """A0 = R0 A P0 as a SciPy CSR matrix (host copy)."""
    import scipy.sparse as sp
    n0, nnz = c_int64(), c_int64()
    _check(lib().pr_get_coarse_matrix(h, byref(n0), byref(nnz), None, None, None), h)
    rp = np.zeros(n0.value + 1, dtype=np.int64)
    ci = np.zeros(max(nnz.value, 1), dtype=np.int32)
    v = np.zeros(max(nnz.value, 1), dtype=np.float64)
    _check(lib().pr_get_coarse_matrix(h, byref(n0), byref(nnz), rp.ctypes.data_as(c_void_p),
                                      ci.ctypes.data_as(c_void_p), v.ctypes.data_as(c_void_p)), h)
    return sp.csr_matrix((v[:nnz.value], ci[:nnz.value], rp), shape=(n0.value, n0.value))


def pr_destroy(h):
    if h:
        lib().pr_destroy(h)


def pr_set_memory_cache_limit(nbytes):
    return _check(lib().pr_set_memory_cache_limit(int(nbytes)))


def pr_set_stream(h, stream):
    """Moves the handle to `stream` (a torch stream or a raw hipStream_t);
    work already queued on the old stream finishes first."""
    raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    return _check(lib().pr_set_stream(h, c_void_p(raw)), h)


def pr_release_cached_memory():
    return _check(lib().pr_release_cached_memory())


def pr_memory_cache_info(device=0):
    """{idle_bytes, idle_blocks, reuses, mallocs} of the device memory cache
    (device -1: pinned host blocks)."""
    out = (c_int64 * 4)()
    _check(lib().pr_memory_cache_info(int(device), out))
    return dict(idle_bytes=out[0], idle_blocks=out[1], reuses=out[2], mallocs=out[3])


def pr_batch_inverse(p, A, X, info):
    count = A.numel() // (p * p)
    return _check(lib().pr_batch_inverse(p, count, _ptr(A), _ptr(X), _ptr(info), _stream()))


def pr_batch_criterion(p, criterion, A, B, X, d):
    count = A.numel() // (p * p)
    crit = CRIT[criterion] if isinstance(criterion, str) else int(criterion)
    return _check(lib().pr_batch_criterion(p, count, crit, _ptr(A), _ptr(B), _ptr(X), _ptr(d),
                                           _stream()))


def pr_validate_host(indptr, indices, data, ptr, dofs, n):
    """Host-only validation of numpy arrays; returns the status code."""
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    data = np.ascontiguousarray(data, dtype=np.float64)
    ptr = np.ascontiguousarray(ptr, dtype=np.int64)
    dofs = np.ascontiguousarray(dofs, dtype=np.int32)
    A = pr_csr(n, len(indices), indptr.ctypes.data_as(c_void_p), indices.ctypes.data_as(c_void_p),
               data.ctypes.data_as(c_void_p))
    P = pr_patches(len(ptr) - 1, ptr.ctypes.data_as(c_void_p), dofs.ctypes.data_as(c_void_p))
    return lib().pr_validate_host(byref(A), byref(P))


class PatchRelax:
    """Owner of a setup handle and the device copies of its inputs.

    ``A`` is a SciPy CSR matrix (int32 indices), ``ptr``/``dofs`` the patch
    lists; they are copied to the current device and handed to ``pr_setup``.
    """

    def __init__(self, A, ptr, dofs, device="cuda", **params):
        import torch
        self.n = A.shape[0]
        self.n_p = len(ptr) - 1
        self.sizes = np.diff(np.asarray(ptr))
        self.dev = torch.device(device)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(self.dev)
        self.row_ptr = t(A.indptr.astype(np.int64), torch.int64)
        self.col = t(A.indices.astype(np.int32), torch.int32)
        self.val = t(A.data.astype(np.float64), torch.float64)
        self.ptr = t(np.asarray(ptr, dtype=np.int64), torch.int64)
        self.dofs = t(np.asarray(dofs, dtype=np.int32), torch.int32)
        params.setdefault("stream", _stream())
        reuse = params.pop("reuse", None)
        self.params = make_params(**params)
        if reuse is None:
            self.h = pr_setup(self.row_ptr, self.col, self.val, self.ptr, self.dofs, self.n, self.params)
        else:
            self.h = pr_setup_reuse(self.row_ptr, self.col, self.val, self.ptr, self.dofs, self.n, self.params,
                                    reuse)

    def apply(self, r, z):
        return pr_apply(self.h, r, z)

    def set_stream(self, stream):
        return pr_set_stream(self.h, stream)

    def solve(self, b, x, tol=1e-8):
        return pr_solve(self.h, b, x, tol)

    def solve_info(self):
        return pr_get_solve_info(self.h)

    def stats(self):
        return pr_get_stats(self.h)

    def assignment(self):
        return pr_get_assignment(self.h, self.n_p)

    def tile(self, k):
        return pr_get_patch_tile(self.h, k, int(self.sizes[k]))

    def weights(self):
        return pr_get_weights(self.h, self.n)

    def keys(self):
        return pr_get_boundary_keys(self.h, self.n_p)

    def rep_inverse(self, j, p):
        return pr_get_rep_inverse(self.h, j, p)

    def entry_matrix(self, j, p):
        return pr_get_entry_matrix(self.h, j, p)

    def export_database(self):
        return pr_export_database(self.h)

    def set_coarse(self, P0):
        """Two-level combination with the interpolation P0 (SciPy CSR, n rows)."""
        import torch
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(self.dev)
        self.p0 = (t(P0.indptr.astype(np.int64), torch.int64), t(P0.indices.astype(np.int32), torch.int32),
                   t(P0.data.astype(np.float64), torch.float64))
        return pr_set_coarse(self.h, *self.p0, P0.shape[0], P0.shape[1])

    def coarse_matrix(self):
        return pr_get_coarse_matrix(self.h)

    def set_systems(self, system_ptr):
        self.n_sys = len(system_ptr) - 1
        return pr_set_systems(self.h, system_ptr)

    def system_info(self):
        return pr_get_system_info(self.h, self.n_sys)

    def mlp_features(self):
        return pr_get_mlp_features(self.h, self.n_p)

    def mlp_candidates(self):
        st = self.stats()
        return pr_get_mlp_candidates(self.h, self.n_p, int(st["mlp_train"]), self.params.mlp_topk)

    def close(self):
        if self.h:
            pr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
