"""Outer Krylov solve: right-preconditioned restarted GMRES with the patch
preconditioner (numerical results: GMRES from a zero initial guess, stopped
when the residual has dropped by the tolerance; the damped smoothing step
x <- x + omega M^{-1} r used as the preconditioner in Experiment 3).

Readings: right preconditioning, so the stopping test is on the true residual
||b - A x||_2 <= tol ||b||_2 (x_0 = 0); modified Gram-Schmidt Arnoldi with
Givens rotations (Saad, Iterative Methods for Sparse Linear Systems, GMRES with
right preconditioning); the true residual is recomputed at each restart and
at exit.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .patch import apply_patch


def make_preconditioner(A, ptr, dofs, W, X, phi, omega=1.0, sweeps=1):
    """r -> e after ``sweeps`` damped patch-smoothing steps from e = 0:
    e <- e + omega M~^{-1} (r - A e)."""
    def prec(r):
        e = np.zeros_like(r)
        for s in range(sweeps):
            res = r if s == 0 else r - A @ e
            e = e + apply_patch(ptr, dofs, W, X, phi, res, omega)
        return e
    return prec


def gmres(matvec, precond, b, tol=1e-8, restart=30, max_iters=10000, flexible=False):
    """Right-preconditioned GMRES(restart) from x0 = 0.

    ``flexible``: keep z_j = precond(v_j) and update x by Z y (flexible GMRES,
    Saad, SIAM J. Sci. Comput. 14 (1993)) instead of precond(V y); the two
    coincide for a linear preconditioner, and the flexible form stays exact
    for one that is not (a reduced-precision apply rounds its input).
    Returns (x, info) with info = dict(iters, relres, converged, cycles)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, dict(iters=0, relres=0.0, converged=True, cycles=0)
    r = b.copy()
    iters = 0
    cycles = 0
    while True:
        beta = float(np.linalg.norm(r))
        if beta <= tol * bnorm:
            break
        if iters >= max_iters:
            break
        cycles += 1
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n)) if flexible else None
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        m = 0
        for j in range(restart):
            zj = precond(V[j])
            if flexible:
                Z[j] = zj
            w = matvec(zj)
            iters += 1
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                           # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            m = j + 1
            if abs(g[j + 1]) <= tol * bnorm or iters >= max_iters:
                break
        y = sla.solve_triangular(H[:m, :m], g[:m])
        x = x + (Z[:m].T @ y if flexible else precond(V[:m].T @ y))
        r = b - matvec(x)
    relres = float(np.linalg.norm(b - matvec(x))) / bnorm
    return x, dict(iters=iters, relres=relres, converged=relres <= tol, cycles=cycles)
