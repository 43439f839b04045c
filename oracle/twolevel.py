"""Two-level combination preconditioner of Eq.(2):

    M_combo^{-1} = M^{-1} + P0 M_amg^{-1} R0,

with M^{-1} the (possibly compressed) patch preconditioner, P0 the
interpolation from a first-order discretisation on the same mesh to the
high-order one, R0 = P0^T and, as in the first two numerical experiments, a
direct solve with R0 A P0 in place of the AMG cycle.  P0 is linear
interpolation that treats the spatial locations of the high-order dofs as a
fine mesh.

Readings (also in the design notes):
* the coarse unknowns are the interior vertices of the mesh; boundary
  vertices carry the Dirichlet data, which the fine system keeps as identity
  rows, so their hat functions are left out;
* P0 entry (i, v) is the value at node i of the multilinear hat function of
  vertex v on the uniform grid of unit-cube cells;
* R0 A P0 is formed as a sparse triple product; an entry below 1e-13 of its
  row's largest magnitude is the rounding residue of a coupling that vanishes
  in exact arithmetic (hat functions with disjoint supports) and is dropped;
* the damping and the smoothing steps act on the patch term only; the coarse
  term is added once per preconditioner application.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .krylov import make_preconditioner


def linear_interpolation(coords, nc, keep_boundary=False):
    """P0 (n x n0, sparse): row i holds the hat functions of the grid
    vertices evaluated at node coords[i]; the grid has nc cells per direction
    on [0, 1]^d and vertex (v_1..v_d) sits at v / nc.  The hat function of
    vertex v is prod_d max(0, 1 - |nc x_d - v_d|).  Columns are the interior
    vertices (x fastest), or every vertex with ``keep_boundary``."""
    coords = np.asarray(coords, dtype=np.float64)
    n, dim = coords.shape
    lo = 0 if keep_boundary else 1
    hi = nc if keep_boundary else nc - 1
    per = hi - lo + 1
    rows, cols, vals = [], [], []
    t = coords * nc
    base = np.floor(t).astype(np.int64)
    for corner in range(1 << dim):
        v = base + np.array([(corner >> d) & 1 for d in range(dim)])
        w = np.prod(np.maximum(0.0, 1.0 - np.abs(t - v)), axis=1)
        ok = (w > 0.0) & np.all((v >= lo) & (v <= hi), axis=1)
        col = np.zeros(n, dtype=np.int64)
        for d in reversed(range(dim)):
            col = col * per + (v[:, d] - lo)
        rows.append(np.flatnonzero(ok))
        cols.append(col[ok])
        vals.append(w[ok])
    P0 = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n, per ** dim)).tocsr()
    P0.sum_duplicates()
    return P0


def coarse_operator(A, P0, drop=1e-13):
    """R0 A P0 with R0 = P0^T (sparse products), without the entries below
    ``drop`` times the largest magnitude of their row."""
    A0 = (P0.T @ (A @ P0)).tocsr()
    A0.sum_duplicates()
    rmax = np.zeros(A0.shape[0])
    for v in range(A0.shape[0]):
        seg = A0.data[A0.indptr[v]:A0.indptr[v + 1]]
        if len(seg):
            rmax[v] = np.abs(seg).max()
    row = np.repeat(np.arange(A0.shape[0]), np.diff(A0.indptr))
    A0.data[np.abs(A0.data) <= drop * rmax[row]] = 0.0
    A0.eliminate_zeros()
    A0.sort_indices()
    return A0


def combo_preconditioner(A, ptr, dofs, W, X, phi, P0, A0=None, omega=1.0, sweeps=1):
    """r -> (sweeps damped patch steps from 0 applied to r) + P0 A0^{-1} P0^T r,
    with A0 = R0 A P0 solved directly (sparse LU)."""
    if A0 is None:
        A0 = coarse_operator(A, P0)
    lu = spla.splu(sp.csc_matrix(A0))
    patch = make_preconditioner(A, ptr, dofs, W, X, phi, omega, sweeps)

    def prec(r):
        return patch(r) + P0 @ lu.solve(P0.T @ r)
    return prec
