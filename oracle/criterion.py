"""Patch-similarity criteria (Section 3: Eq.(4), Eq.(5) and the remark on
entrywise norms).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np


def crit_spectral_x(A, X):
    """||I - A X||_2 with X = B^{-1} given (Eq.(5), Algorithm 1's test).

    Computed exactly with the LAPACK SVD behind ``numpy.linalg.norm(., 2)``
    (the remark after Eq.(4) allows a small SVD).  The paper's derivation first
    yields I - B^{-1} A_i; Eq.(4), Eq.(5) and Algorithm 1 use I - A B^{-1},
    which is taken literally here (for symmetric A, B both have the same norm).
    """
    E = np.eye(A.shape[0]) - A @ X
    return float(np.linalg.norm(E, 2))


def crit_spectral(A, B):
    """d(A, B) = ||I - A B^{-1}||_2   (Eq.(5))."""
    return crit_spectral_x(A, np.linalg.inv(B))


def crit_l1(A, B):
    """Entrywise l1 difference sum_ab |A_ab - B_ab| (remark after Eq.(4);
    the criterion used in Experiment 3 and in entrywise k-means)."""
    return float(np.abs(A - B).sum())


def crit_fro(A, B):
    """Entrywise Frobenius difference ||A - B||_F (remark after Eq.(4))."""
    return float(np.sqrt(((A - B) ** 2).sum()))


def criterion(name, A, B, X=None):
    """Dispatch by name: 'spectral' uses X = B^{-1} when given."""
    if name == "spectral":
        return crit_spectral_x(A, X) if X is not None else crit_spectral(A, B)
    if name == "l1":
        return crit_l1(A, B)
    if name == "fro":
        return crit_fro(A, B)
    raise ValueError(name)
