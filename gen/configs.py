"""The five benchmark workloads, at full or reduced size.

Index 0: Q1 diffusion 32x32.  1: Taylor-Hood Stokes 64x64.  2: Nedelec hex 64^3
with four Voronoi materials.  3: 256 uneven Stokes systems.  4: Q2 hex 32^3 with
a lognormal coefficient.  ``scale`` < 1 shrinks the mesh for fast checks.
"""
from __future__ import annotations

from . import fem

CONFIG_NAMES = ["q1_poisson_2d", "stokes_th_2d", "nedelec_hex", "stokes_batch", "q2_hex_lognormal"]


def make_config(i: int, size: int | None = None, n_sys: int | None = None):
    if i == 0:
        return fem.q1_poisson_2d(size or 32)
    if i == 1:
        return fem.taylor_hood_stokes_2d(size or 64)
    if i == 2:
        return fem.nedelec_hex(size or 64)
    if i == 3:
        if size is None and n_sys is None:
            return fem.uneven_stokes_batch()
        nmax = size or 128
        return fem.uneven_stokes_batch(n_sys=n_sys or 256, nmin=min(16, nmax), nmax=nmax)
    if i == 4:
        return fem.q2_hex_diffusion(size or 32)
    raise ValueError(i)
