"""Patch objects of Section 2 and the preconditioners of Eq.(1) and Eq.(3).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class OracleError(RuntimeError):
    """An input the method cannot handle (uncovered dof, singular patch...)."""


def cover_weights(n, ptr, dofs):
    """Cover counts and the weight matrix W (Section 2).

    W is the inverse of sum_l V_l^T V_l: a diagonal whose entry i is one over
    the number of patches that contain global dof i.  A dof in no patch makes W
    undefined and is an error.
    Returns (count int64[n], W float64[n]).
    """
    dofs = np.asarray(dofs)
    cnt = np.bincount(dofs.astype(np.int64), minlength=n)
    if cnt.shape[0] != n:
        raise OracleError("dof index out of range")
    if (cnt == 0).any():
        raise OracleError(f"uncovered dof {int(np.flatnonzero(cnt == 0)[0])}")
    return cnt, 1.0 / cnt.astype(np.float64)


def patch_tiles(A, ptr, dofs, ks=None):
    """Dense patch matrices A_k = V_k A V_k^T (Section 2).

    V_k picks the patch's global dofs in list order, so A_k[a, b] is the global
    entry at (dofs_k[a], dofs_k[b]); it is read with SciPy fancy indexing.
    Returns a list of dense float64 arrays (patch sizes may differ).
    """
    ks = range(len(ptr) - 1) if ks is None else ks
    out = []
    for k in ks:
        d = dofs[ptr[k]:ptr[k + 1]]
        out.append(A[d][:, d].toarray())
    return out


def patch_tiles_csr(A, ptr, dofs):
    """The same tiles A_k = V_k A V_k^T read straight from the CSR arrays:
    entry (a, b) of patch k is the stored value at row dofs_k[a], column
    dofs_k[b], found by binary search of the key row * n + column in the
    sorted list of stored keys, or 0.0 where nothing is stored.  Patches of
    one size are read together.  Returns a list of dense float64 arrays."""
    A = A.tocsr()
    A.sort_indices()
    n = A.shape[0]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.indptr))
    keys = rows * n + A.indices.astype(np.int64)
    sizes = np.diff(ptr)
    out = [None] * (len(ptr) - 1)
    for p in np.unique(sizes):
        ks = np.flatnonzero(sizes == p)
        D = np.stack([dofs[ptr[k]:ptr[k + 1]] for k in ks]).astype(np.int64)
        want = (D[:, :, None] * n + D[:, None, :]).ravel()
        pos = np.searchsorted(keys, want)
        pos = np.minimum(pos, len(keys) - 1)
        hit = keys[pos] == want
        vals = np.where(hit, A.data[pos], 0.0).reshape(len(ks), p, p)
        for t, k in enumerate(ks):
            out[k] = vals[t]
    return out


def batch_inverse(tiles):
    """Inverses of equal-size patch matrices by LAPACK's LU with partial
    pivoting (numpy.linalg.inv on the stacked tiles): the operator of
    factor_inverse, computed for many tiles at once."""
    return list(np.linalg.inv(np.stack(tiles)))


def boundary_mask(tile) -> int:
    """Boundary-condition key of a patch (Section 3.2, boundary partitioning).

    A boundary condition shows in a patch as a row with exactly one nonzero
    entry.  Bit a of the key is set iff row a of the tile has exactly one
    entry different from 0.0.
    """
    key = 0
    for a in range(tile.shape[0]):
        if np.count_nonzero(tile[a] != 0.0) == 1:
            key |= 1 << a
    return key


def factor_inverse(B):
    """Inverse of a database matrix through an LU factorisation with partial
    pivoting (the GETRF/GETRS pair used in the numerical results, Experiment 3).

    The paper keeps LU factors; the explicit inverse represents the same
    operator.  An exactly zero pivot is an error.
    """
    lu, piv = sla.lu_factor(B, check_finite=True)
    if np.any(np.diag(lu) == 0.0):
        raise OracleError("singular patch")
    return sla.lu_solve((lu, piv), np.eye(B.shape[0]))


def apply_patch(ptr, dofs, W, X, phi, r, omega=1.0):
    """z = omega * W * sum_k V_k^T X_{phi(k)} V_k r   (Eq.(3); Eq.(1) when
    phi is the identity and X_k = A_k^{-1}).

    ``X`` is a list of dense inverses (the database), ``phi`` maps patches to
    database entries.  Restrict r to each patch, multiply by the database
    inverse, inject back and add; then average with W (Section 2).
    """
    r = np.asarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    sizes = np.diff(ptr)
    if len(sizes) and (sizes == sizes[0]).all() and all(x.shape[0] == sizes[0] for x in X):
        # all patches of one size: the same sum written with batched products
        ps = int(sizes[0])
        D = np.asarray(dofs[:ptr[-1]]).reshape(-1, ps)
        Y = np.einsum('kab,kb->ka', np.stack(X)[np.asarray(phi)], r[D])
        np.add.at(z, D.ravel(), Y.ravel())
    else:
        for k in range(len(ptr) - 1):
            d = dofs[ptr[k]:ptr[k + 1]]
            np.add.at(z, d, X[phi[k]] @ r[d])
    return omega * W * z


def apply_operator_dense(n, ptr, dofs, X, phi, omega=1.0):
    """Dense n x n matrix of Eq.(3) built from explicit boolean V_k matrices
    (brute force for tiny inputs): omega * W * sum_k V_k^T X_phi(k) V_k with
    W = (sum_k V_k^T V_k)^{-1}."""
    S = np.zeros((n, n))
    C = np.zeros((n, n))
    for k in range(len(ptr) - 1):
        d = dofs[ptr[k]:ptr[k + 1]]
        V = np.zeros((len(d), n))
        V[np.arange(len(d)), d] = 1.0
        S += V.T @ X[phi[k]] @ V
        C += V.T @ V
    return omega * np.linalg.inv(C) @ S


def objective(tiles, Xdb, phi, beta):
    """L(B, phi) = beta |B| + sum_k ||I - A_k B_phi(k)^{-1}||_2^2   (Eq.(4)).

    ``Xdb`` holds the database inverses B_j^{-1}."""
    tot = beta * len(Xdb)
    for k, Ak in enumerate(tiles):
        E = np.eye(Ak.shape[0]) - Ak @ Xdb[phi[k]]
        tot += np.linalg.norm(E, 2) ** 2
    return tot


def storage_bytes(n_p, p_s, m_p, n, value_bytes=8, index_bytes=8):
    """Storage accounting of Experiment 3: dense factors of the database,
    one lookup index per patch, versus all factors, versus a Jacobi diagonal."""
    return dict(database=m_p * p_s * p_s * value_bytes,
                indices=n_p * index_bytes,
                full=n_p * p_s * p_s * value_bytes,
                jacobi=n * value_bytes)
