"""Seeded finite-element problem generators (test and benchmark inputs).

These routines assemble the global sparse matrices and cell patch lists that the
patch-relaxation method consumes.  They hold none of the method's arithmetic:
the method starts from an assembled CSR matrix and a list of patches (Section 2,
definition of V_k), and everything here happens before that point.

Conventions shared by every generator
-------------------------------------
* Matrices are ``scipy.sparse.csr_matrix`` in canonical form (sorted, unique
  column indices per row, int32 indices) with explicit zeros removed.
* Dirichlet conditions are imposed by symmetric elimination that keeps an
  identity row and column (diagonal 1.0); the paper identifies such a condition
  inside a patch as a row with a single nonzero (Section 3.2, boundary
  partitioning).  ``eliminate_dirichlet=True`` removes the dofs instead.
* A patch is the ordered list of the global dofs of one mesh cell, in
  reference-element (tensor, x fastest) order; list order is the local order
  (Section 2, V_k).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Problem:
    name: str
    A: sp.csr_matrix
    ptr: np.ndarray          # int64[n_p + 1]
    dofs: np.ndarray         # int32[ptr[-1]]
    meta: dict

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def n_p(self) -> int:
        return len(self.ptr) - 1

    def patch(self, k: int) -> np.ndarray:
        return self.dofs[self.ptr[k]:self.ptr[k + 1]]


# ---------------------------------------------------------------------------
# 1D building blocks
# ---------------------------------------------------------------------------

def gauss_legendre(nq: int):
    """Gauss points/weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_1d(order: int, x: np.ndarray):
    """Values and derivatives of the equispaced 1D Lagrange basis on [0,1]."""
    nodes = np.linspace(0.0, 1.0, order + 1)
    nb = order + 1
    val = np.ones((nb, len(x)))
    der = np.zeros((nb, len(x)))
    for i in range(nb):
        for j in range(nb):
            if j == i:
                continue
            val[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
        for m in range(nb):
            if m == i:
                continue
            term = np.ones(len(x)) / (nodes[i] - nodes[m])
            for j in range(nb):
                if j == i or j == m:
                    continue
                term *= (x - nodes[j]) / (nodes[i] - nodes[j])
            der[i] += term
    return val, der


def _finish(rows, cols, vals, n, bnd_mask=None, eliminate=False):
    """COO -> canonical CSR, then impose Dirichlet rows on ``bnd_mask``."""
    rows = np.asarray(rows, dtype=np.int64).ravel()
    cols = np.asarray(cols, dtype=np.int64).ravel()
    vals = np.asarray(vals, dtype=np.float64).ravel()
    keep_map = None
    if bnd_mask is not None and bnd_mask.any():
        keep = ~(bnd_mask[rows] | bnd_mask[cols])
        rows, cols, vals = rows[keep], cols[keep], vals[keep]
        if eliminate:
            keep_map = -np.ones(n, dtype=np.int64)
            interior = np.flatnonzero(~bnd_mask)
            keep_map[interior] = np.arange(len(interior))
            rows, cols = keep_map[rows], keep_map[cols]
            n = len(interior)
        else:
            bd = np.flatnonzero(bnd_mask)
            rows = np.concatenate([rows, bd])
            cols = np.concatenate([cols, bd])
            vals = np.concatenate([vals, np.ones(len(bd))])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int64)
    return A, keep_map


def _cells_to_coo(cell_dofs: np.ndarray, Ke: np.ndarray):
    """Element matrices Ke[c, a, b] on dofs cell_dofs[c, a] -> COO triplets."""
    nc, nl = cell_dofs.shape
    rows = np.repeat(cell_dofs[:, :, None], nl, axis=2)
    cols = np.repeat(cell_dofs[:, None, :], nl, axis=1)
    if Ke.ndim == 2:
        vals = np.broadcast_to(Ke, (nc, nl, nl))
    else:
        vals = Ke
    return rows.ravel(), cols.ravel(), np.ascontiguousarray(vals).ravel()


def _patches_from_cells(cell_dofs):
    nc, nl = cell_dofs.shape
    ptr = np.arange(nc + 1, dtype=np.int64) * nl
    return ptr, np.ascontiguousarray(cell_dofs, dtype=np.int32).ravel()


def _patches_from_lists(lists):
    lens = np.array([len(l) for l in lists], dtype=np.int64)
    ptr = np.zeros(len(lists) + 1, dtype=np.int64)
    np.cumsum(lens, out=ptr[1:])
    dofs = np.concatenate(lists).astype(np.int32) if lists else np.zeros(0, np.int32)
    return ptr, dofs


# ---------------------------------------------------------------------------
# Reference-element matrices
# ---------------------------------------------------------------------------

def _tensor_basis_2d(order, xq):
    v, d = lagrange_1d(order, xq)
    nb = order + 1
    nq = len(xq)
    # local index a = ix + nb*iy ; quad index q = qx + nq*qy
    phi = np.einsum('iq,jr->jirq', v, v).reshape(nb * nb, nq * nq)
    dx = np.einsum('iq,jr->jirq', d, v).reshape(nb * nb, nq * nq)
    dy = np.einsum('iq,jr->jirq', v, d).reshape(nb * nb, nq * nq)
    return phi, dx, dy


def ref_laplace_3d(order: int) -> np.ndarray:
    """Stiffness of the Q_order Lagrange element on the unit cube (x fastest)."""
    xq, wq = gauss_legendre(order + 1)
    v, d = lagrange_1d(order, xq)
    m1 = np.einsum('iq,jq,q->ij', v, v, wq)
    k1 = np.einsum('iq,jq,q->ij', d, d, wq)
    # index (ix, iy, iz) -> ix + nb*(iy + nb*iz): kron order z, y, x
    return (np.kron(np.kron(m1, m1), k1) + np.kron(np.kron(m1, k1), m1)
            + np.kron(np.kron(k1, m1), m1))


def ref_nedelec_hex():
    """Lowest-order hexahedral edge element on the unit cube.

    Edge functions are scaled to unit tangential moment and oriented along the
    positive coordinate axis.  Local edge order: 4 x-edges at (y, z) =
    (0,0),(1,0),(0,1),(1,1); 4 y-edges at (x, z) in the same pattern; 4 z-edges
    at (x, y).  Returns (mass, curlcurl), each 12x12, integrated with 3-point
    Gauss per direction.
    """
    xq, wq = gauss_legendre(3)
    X, Y, Z = np.meshgrid(xq, xq, xq, indexing='ij')
    Wt = np.einsum('i,j,k->ijk', wq, wq, wq)
    X, Y, Z, Wt = X.ravel(), Y.ravel(), Z.ravel(), Wt.ravel()
    l = [lambda t: 1.0 - t, lambda t: t]
    dl = [-1.0, 1.0]
    N = np.zeros((12, 3, len(X)))
    C = np.zeros((12, 3, len(X)))
    pat = [(0, 0), (1, 0), (0, 1), (1, 1)]
    for e, (a, b) in enumerate(pat):
        # x-edge: (l_a(y) l_b(z), 0, 0); curl = (0, d/dz, -d/dy)
        N[e, 0] = l[a](Y) * l[b](Z)
        C[e, 1] = l[a](Y) * dl[b]
        C[e, 2] = -dl[a] * l[b](Z)
        # y-edge: (0, l_a(x) l_b(z), 0); curl = (-d/dz, 0, d/dx)
        N[4 + e, 1] = l[a](X) * l[b](Z)
        C[4 + e, 0] = -l[a](X) * dl[b]
        C[4 + e, 2] = dl[a] * l[b](Z)
        # z-edge: (0, 0, l_a(x) l_b(y)); curl = (d/dy, -d/dx, 0)
        N[8 + e, 2] = l[a](X) * l[b](Y)
        C[8 + e, 0] = l[a](X) * dl[b]
        C[8 + e, 1] = -dl[a] * l[b](Y)
    M = np.einsum('icq,jcq,q->ij', N, N, Wt)
    S = np.einsum('icq,jcq,q->ij', C, C, Wt)
    return M, S


# ---------------------------------------------------------------------------
# Coarse interpolation input of the two-level combination (Eq.(2))
# ---------------------------------------------------------------------------

def tensor_interpolation(order: int, nc: int, dim: int) -> sp.csr_matrix:
    """P0 of the two-level combination: values at the interior vertices of an
    nc^dim grid of unit-cube cells -> values at the nodes of the order-`order`
    tensor Lagrange discretisation on the same cells (equispaced nodes,
    (order*nc + 1)^dim of them, x fastest), by multilinear interpolation in
    each cell.  Boundary vertices carry Dirichlet values and are left out, so
    the coarse unknowns are the (nc - 1)^dim interior vertices (x fastest).
    Built from integer node indices (node I of a line lies in cell
    min(I // order, nc - 1) at local coordinate (I - order * cell) / order).
    """
    nf = order * nc + 1
    I = np.arange(nf)
    cell = np.minimum(I // order, nc - 1)
    xi = (I - order * cell) / order
    # 1D: node I -> (vertex, weight) pairs; weight-0 pairs dropped
    v1 = [cell, cell + 1]
    w1 = [1.0 - xi, xi]
    nci = nc - 1                                 # interior vertices per line
    rows, cols, vals = [], [], []
    for corner in range(1 << dim):
        bits = [(corner >> d) & 1 for d in range(dim)]
        # node multi-index (x fastest) via broadcasting over all nodes
        grids = np.meshgrid(*([I] * dim), indexing='ij')          # grids[d][..] = index along axis d
        vtx = [v1[bits[d]][grids[d]] for d in range(dim)]
        wt = np.ones(grids[0].shape)
        for d in range(dim):
            wt = wt * w1[bits[d]][grids[d]]
        inner = np.ones(grids[0].shape, dtype=bool)
        for d in range(dim):
            inner &= (vtx[d] >= 1) & (vtx[d] <= nc - 1)
        keep = inner & (wt != 0.0)
        node = np.zeros(grids[0].shape, dtype=np.int64)
        coarse = np.zeros(grids[0].shape, dtype=np.int64)
        for d in reversed(range(dim)):
            node = node * nf + grids[d]
            coarse = coarse * nci + (vtx[d] - 1)
        rows.append(node[keep])
        cols.append(coarse[keep])
        vals.append(wt[keep])
    P0 = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(nf ** dim, nci ** dim)).tocsr()
    P0.sum_duplicates()
    P0.sort_indices()
    P0.indices = P0.indices.astype(np.int32)
    P0.indptr = P0.indptr.astype(np.int64)
    return P0


def tensor_node_coords(order: int, nc: int, dim: int) -> np.ndarray:
    """Coordinates (n x dim) of the equispaced tensor Lagrange nodes, x fastest."""
    nf = order * nc + 1
    x = np.arange(nf) / (order * nc)
    g = np.meshgrid(*([x] * dim), indexing='ij')
    return np.stack([gd.transpose(*reversed(range(dim))).ravel() for gd in g], axis=1)


# ---------------------------------------------------------------------------
# Config generators
# ---------------------------------------------------------------------------

def q1_poisson_2d(nc: int = 32, k: float = 1.0) -> Problem:
    """-div(k grad u) = f on the unit square, Q1 on nc x nc quads, Dirichlet."""
    nn = nc + 1
    xq, wq = gauss_legendre(2)
    phi, dx, dy = _tensor_basis_2d(1, xq)
    w2 = np.kron(wq, wq)
    Ke = k * (np.einsum('aq,bq,q->ab', dx, dx, w2) + np.einsum('aq,bq,q->ab', dy, dy, w2))
    ci, cj = np.meshgrid(np.arange(nc), np.arange(nc), indexing='xy')
    ci, cj = ci.ravel(), cj.ravel()
    loc = [(0, 0), (1, 0), (0, 1), (1, 1)]
    cell_dofs = np.stack([(ci + a) + nn * (cj + b) for a, b in loc], axis=1)
    I, J = np.meshgrid(np.arange(nn), np.arange(nn), indexing='xy')
    bnd = ((I == 0) | (I == nc) | (J == 0) | (J == nc)).ravel()
    r, c, v = _cells_to_coo(cell_dofs, Ke)
    A, _ = _finish(r, c, v, nn * nn, bnd)
    ptr, dofs = _patches_from_cells(cell_dofs)
    return Problem(f"q1_poisson_2d_{nc}", A, ptr, dofs,
                   dict(nc=nc, k=k, p_s=4, boundary=bnd))


def qp_diffusion_2d(nc: int = 60, order: int = 2, rho=None) -> Problem:
    """-div(rho grad u) = f on the unit square with Q_order Lagrange elements
    (equispaced nodes) on nc x nc quads, Dirichlet identity rows on the
    boundary nodes, one patch per cell ((order + 1)^2 dofs, tensor order).
    rho defaults to sin^2(pi x) sin^2(pi y) + 0.1, the smooth coefficient of
    the first numerical experiment, evaluated at (order + 2)^2 Gauss points
    per cell.  meta['b_exact'] = A u for the nodal values of
    u = sin(pi x) sin(pi y), so that the discrete solution is that
    interpolant; meta['P0'] is the coarse interpolation from the interior
    vertices of the same mesh."""
    if rho is None:
        rho = lambda x, y: np.sin(np.pi * x) ** 2 * np.sin(np.pi * y) ** 2 + 0.1
    nb = order + 1
    nf = order * nc + 1
    h = 1.0 / nc
    xq, wq = gauss_legendre(order + 2)
    phi, dx, dy = _tensor_basis_2d(order, xq)
    w2 = np.kron(wq, wq)
    ci, cj = np.meshgrid(np.arange(nc), np.arange(nc), indexing='xy')
    ci, cj = ci.ravel(), cj.ravel()
    # quadrature points per cell (index q = qx + nq*qy)
    qx = np.tile(xq, len(xq))
    qy = np.repeat(xq, len(xq))
    X = (ci[:, None] + qx[None, :]) * h
    Y = (cj[:, None] + qy[None, :]) * h
    R = rho(X, Y)                                        # [cells, nq^2]
    # reference gradients scale by 1/h, the Jacobian by h^2: the 2D stiffness is h-independent
    Ke = (np.einsum('aq,bq,cq->cab', dx, dx, R * w2) + np.einsum('aq,bq,cq->cab', dy, dy, R * w2))
    loc = [(a, b) for b in range(nb) for a in range(nb)]
    cell_dofs = np.stack([(order * ci + a) + nf * (order * cj + b) for a, b in loc], axis=1)
    I, J = np.meshgrid(np.arange(nf), np.arange(nf), indexing='xy')
    bnd = ((I == 0) | (I == nf - 1) | (J == 0) | (J == nf - 1)).ravel()
    r, c, v = _cells_to_coo(cell_dofs, Ke)
    A, _ = _finish(r, c, v, nf * nf, bnd)
    ptr, dofs = _patches_from_cells(cell_dofs)
    coords = tensor_node_coords(order, nc, 2)
    u = np.sin(np.pi * coords[:, 0]) * np.sin(np.pi * coords[:, 1])
    u[bnd] = 0.0
    return Problem(f"qp_diffusion_2d_p{order}_{nc}", A, ptr, dofs,
                   dict(nc=nc, order=order, p_s=nb * nb, boundary=bnd, coords=coords, u_exact=u,
                        b_exact=A @ u, P0=tensor_interpolation(order, nc, 2)))


def _quad_geometry(vx, vy, xq):
    """Bilinear map per cell: vertex coords vx, vy [nc, 4] in tensor order."""
    v1, d1 = lagrange_1d(1, xq)
    nq = len(xq)
    # bilinear shape functions at quad points (tensor, x fastest)
    phi = np.einsum('iq,jr->jirq', v1, v1).reshape(4, nq * nq)
    dxi = np.einsum('iq,jr->jirq', d1, v1).reshape(4, nq * nq)
    deta = np.einsum('iq,jr->jirq', v1, d1).reshape(4, nq * nq)
    x = vx @ phi
    y = vy @ phi
    J11, J12 = vx @ dxi, vx @ deta
    J21, J22 = vy @ dxi, vy @ deta
    det = J11 * J22 - J12 * J21
    return x, y, J11, J12, J21, J22, det


def _stokes_cells(nc, vx, vy, nu):
    """Taylor-Hood Q2-Q1 element matrices for cells with vertex coords vx, vy."""
    xq, wq = gauss_legendre(3)
    w2 = np.kron(wq, wq)
    _, J11, J12, J21, J22, det = _quad_geometry(vx, vy, xq)[1:]
    phi2, dx2, dy2 = _tensor_basis_2d(2, xq)
    phi1, _, _ = _tensor_basis_2d(1, xq)
    # physical gradients: grad = J^{-T} grad_ref
    inv = 1.0 / det
    gx = (J22[:, None, :] * dx2[None] - J21[:, None, :] * dy2[None]) * inv[:, None, :]
    gy = (-J12[:, None, :] * dx2[None] + J11[:, None, :] * dy2[None]) * inv[:, None, :]
    wdet = det * w2[None, :]
    K = nu * (np.einsum('caq,cbq,cq->cab', gx, gx, wdet) + np.einsum('caq,cbq,cq->cab', gy, gy, wdet))
    Bx = -np.einsum('iq,cjq,cq->cij', phi1, gx, wdet)
    By = -np.einsum('iq,cjq,cq->cij', phi1, gy, wdet)
    ncell = vx.shape[0]
    Ke = np.zeros((ncell, 22, 22))
    Ke[:, 0:9, 0:9] = K
    Ke[:, 9:18, 9:18] = K
    Ke[:, 18:22, 0:9] = Bx
    Ke[:, 18:22, 9:18] = By
    Ke[:, 0:9, 18:22] = Bx.transpose(0, 2, 1)
    Ke[:, 9:18, 18:22] = By.transpose(0, 2, 1)
    return Ke


def _stokes_mesh(nc, perturb=0.0, rng=None):
    h = 1.0 / nc
    I, J = np.meshgrid(np.arange(nc + 1), np.arange(nc + 1), indexing='xy')
    X = (I * h).astype(np.float64)
    Y = (J * h).astype(np.float64)
    if perturb > 0.0:
        inner = (I > 0) & (I < nc) & (J > 0) & (J < nc)
        dxy = rng.uniform(-perturb * h, perturb * h, size=(2,) + X.shape)
        X = X + np.where(inner, dxy[0], 0.0)
        Y = Y + np.where(inner, dxy[1], 0.0)
    ci, cj = np.meshgrid(np.arange(nc), np.arange(nc), indexing='xy')
    ci, cj = ci.ravel(), cj.ravel()
    loc = [(0, 0), (1, 0), (0, 1), (1, 1)]
    vx = np.stack([X[cj + b, ci + a] for a, b in loc], axis=1)
    vy = np.stack([Y[cj + b, ci + a] for a, b in loc], axis=1)
    return ci, cj, vx, vy


def taylor_hood_stokes_2d(nc: int = 64, nu: float = 1.0, perturb: float = 0.0,
                          perturb_seed: int = 3, eliminate_dirichlet: bool = False,
                          name: str | None = None) -> Problem:
    """Stokes, Taylor-Hood Q2-Q1 on nc x nc quads, Vanka cell patches.

    Dof order: x-velocity nodes, y-velocity nodes, pressure vertices.  Velocity
    is Dirichlet on the whole boundary; the pressure is pinned at vertex (0, 0)
    by an identity row.  A cell patch lists its 9 x-velocity, 9 y-velocity and
    4 pressure dofs (22); with ``eliminate_dirichlet`` boundary velocity dofs
    are removed, so boundary patches are smaller.
    """
    rng = np.random.default_rng(perturb_seed) if perturb > 0 else None
    ci, cj, vx, vy = _stokes_mesh(nc, perturb, rng)
    Ke = _stokes_cells(nc, vx, vy, nu)
    nv = 2 * nc + 1
    nvel = nv * nv
    npr = (nc + 1) ** 2
    n = 2 * nvel + npr
    loc2 = [(a, b) for b in range(3) for a in range(3)]
    loc1 = [(0, 0), (1, 0), (0, 1), (1, 1)]
    ux = np.stack([(2 * ci + a) + nv * (2 * cj + b) for a, b in loc2], axis=1)
    uy = ux + nvel
    pp = np.stack([2 * nvel + (ci + a) + (nc + 1) * (cj + b) for a, b in loc1], axis=1)
    cell_dofs = np.concatenate([ux, uy, pp], axis=1)
    I, J = np.meshgrid(np.arange(nv), np.arange(nv), indexing='xy')
    vb = ((I == 0) | (I == nv - 1) | (J == 0) | (J == nv - 1)).ravel()
    bnd = np.zeros(n, dtype=bool)
    bnd[:nvel] = vb
    bnd[nvel:2 * nvel] = vb
    pin = np.zeros(n, dtype=bool)
    pin[2 * nvel] = True
    r, c, v = _cells_to_coo(cell_dofs, Ke)
    if eliminate_dirichlet:
        # remove velocity boundary dofs, keep the pressure pin as identity row
        keep = ~(bnd[r] | bnd[c])
        r, c, v = r[keep], c[keep], v[keep]
        keep = ~(pin[r] | pin[c])
        r, c, v = r[keep], c[keep], v[keep]
        r = np.concatenate([r, [2 * nvel]])
        c = np.concatenate([c, [2 * nvel]])
        v = np.concatenate([v, [1.0]])
        A, kmap = _finish(r, c, v, n, bnd, eliminate=True)
        lists = []
        for cd in cell_dofs:
            m = kmap[cd]
            lists.append(m[m >= 0])
        ptr, dofs = _patches_from_lists(lists)
        n_new = A.shape[0]
        return Problem(name or f"stokes_th_{nc}_elim", A, ptr, dofs,
                       dict(nc=nc, nu=nu, perturb=perturb, p_s_max=22, n_full=n, n=n_new))
    A, _ = _finish(r, c, v, n, bnd | pin)
    ptr, dofs = _patches_from_cells(cell_dofs)
    return Problem(name or f"stokes_th_{nc}", A, ptr, dofs,
                   dict(nc=nc, nu=nu, perturb=perturb, p_s=22, boundary=bnd | pin))


def nedelec_regions(nc: int, seed: int = 1, coeffs=(1.0, 10.0, 100.0, 1000.0)):
    """Cell coefficient for 4 Voronoi regions of seeded uniform sites in [0,1]^3."""
    rng = np.random.default_rng(seed)
    sites = rng.random((4, 3))
    perm = rng.permutation(4)
    h = 1.0 / nc
    c = (np.arange(nc) + 0.5) * h
    X, Y, Z = np.meshgrid(c, c, c, indexing='ij')  # X[i, j, k]
    P = np.stack([X, Y, Z], axis=-1)
    d2 = ((P[..., None, :] - sites[None, None, None]) ** 2).sum(-1)
    reg = np.argmin(d2, axis=-1)
    vals = np.asarray(coeffs)[perm][reg]
    # cell order (i fastest): transpose to [k, j, i]
    return vals.transpose(2, 1, 0).ravel(), reg.transpose(2, 1, 0).ravel()


def nedelec_hex(nc: int = 64, alpha: float = 1e-3, seed: int = 1,
                coeffs=(1.0, 10.0, 100.0, 1000.0)) -> Problem:
    """curl(c curl u) + alpha u on the unit cube, lowest-order hex edge elements.

    c is piecewise constant on 4 seeded Voronoi regions; tangential Dirichlet on
    all boundary edges.  Patches: the 12 edges of each cell.
    """
    h = 1.0 / nc
    Mr, Sr = ref_nedelec_hex()
    coef, reg = nedelec_regions(nc, seed, coeffs)
    n1 = nc + 1
    Ex = nc * n1 * n1
    i, j, k = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing='ij')
    # cell order: i fastest
    i, j, k = i.transpose(2, 1, 0).ravel(), j.transpose(2, 1, 0).ravel(), k.transpose(2, 1, 0).ravel()
    xe = lambda ii, jj, kk: ii + nc * (jj + n1 * kk)
    ye = lambda ii, jj, kk: Ex + ii + n1 * (jj + nc * kk)
    ze = lambda ii, jj, kk: 2 * Ex + ii + n1 * (jj + n1 * kk)
    pat = [(0, 0), (1, 0), (0, 1), (1, 1)]
    cols = []
    for a, b in pat:
        cols.append(xe(i, j + a, k + b))
    for a, b in pat:
        cols.append(ye(i + a, j, k + b))
    for a, b in pat:
        cols.append(ze(i + a, j + b, k))
    cell_dofs = np.stack(cols, axis=1)
    Ke = coef[:, None, None] * (Sr / h)[None] + alpha * h * Mr[None]
    n = 3 * Ex
    # boundary edges: lying on a boundary face
    bnd = np.zeros(n, dtype=bool)
    I, J, K = np.meshgrid(np.arange(nc), np.arange(n1), np.arange(n1), indexing='ij')
    bnd[xe(I, J, K).ravel()] = ((J == 0) | (J == nc) | (K == 0) | (K == nc)).ravel()
    I, J, K = np.meshgrid(np.arange(n1), np.arange(nc), np.arange(n1), indexing='ij')
    bnd[ye(I, J, K).ravel()] = ((I == 0) | (I == nc) | (K == 0) | (K == nc)).ravel()
    I, J, K = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(nc), indexing='ij')
    bnd[ze(I, J, K).ravel()] = ((I == 0) | (I == nc) | (J == 0) | (J == nc)).ravel()
    r, c, v = _cells_to_coo(cell_dofs, Ke)
    A, _ = _finish(r, c, v, n, bnd)
    ptr, dofs = _patches_from_cells(cell_dofs)
    return Problem(f"nedelec_hex_{nc}", A, ptr, dofs,
                   dict(nc=nc, alpha=alpha, seed=seed, p_s=12, coef=coef, region=reg, boundary=bnd))


def lognormal_field(nc: int, sigma: float = 1.5, corr: float = 0.1, seed: int = 4):
    """log k = sigma * g, g a unit-variance Gaussian process with squared-
    exponential covariance at the cell centres, sampled exactly through the
    Kronecker product of three 1D Cholesky factors (jitter 1e-10)."""
    c = (np.arange(nc) + 0.5) / nc
    C = np.exp(-(c[:, None] - c[None, :]) ** 2 / (2.0 * corr * corr))
    L = np.linalg.cholesky(C + 1e-10 * np.eye(nc))
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((nc, nc, nc))  # indices (k, j, i)
    g = np.einsum('ka,jb,ic,abc->kji', L, L, L, xi)
    return np.exp(sigma * g).ravel()  # i fastest


def q2_hex_diffusion(nc: int = 32, sigma: float = 1.5, corr: float = 0.1, seed: int = 4,
                     kfield: np.ndarray | None = None) -> Problem:
    """-div(k grad u) = f on the unit cube, Q2 hexes, k lognormal per cell,
    identity Dirichlet rows on all boundary nodes; 27-dof cell patches."""
    h = 1.0 / nc
    if kfield is None:
        kfield = lognormal_field(nc, sigma, corr, seed) if sigma != 0.0 else np.ones(nc ** 3)
    Kr = ref_laplace_3d(2)
    nn = 2 * nc + 1
    i, j, k = np.meshgrid(np.arange(nc), np.arange(nc), np.arange(nc), indexing='ij')
    i, j, k = i.transpose(2, 1, 0).ravel(), j.transpose(2, 1, 0).ravel(), k.transpose(2, 1, 0).ravel()
    loc = [(a, b, c) for c in range(3) for b in range(3) for a in range(3)]
    cell_dofs = np.stack([(2 * i + a) + nn * ((2 * j + b) + nn * (2 * k + c)) for a, b, c in loc], axis=1)
    Ke = (kfield * h)[:, None, None] * Kr[None]
    I, J, K = np.meshgrid(np.arange(nn), np.arange(nn), np.arange(nn), indexing='ij')
    bnd3 = (I == 0) | (I == nn - 1) | (J == 0) | (J == nn - 1) | (K == 0) | (K == nn - 1)
    bnd = bnd3.transpose(2, 1, 0).ravel()
    r, c, v = _cells_to_coo(cell_dofs, Ke)
    A, _ = _finish(r, c, v, nn ** 3, bnd)
    ptr, dofs = _patches_from_cells(cell_dofs)
    return Problem(f"q2_hex_{nc}", A, ptr, dofs,
                   dict(nc=nc, sigma=sigma, corr=corr, seed=seed, p_s=27, k=kfield, boundary=bnd,
                        P0=tensor_interpolation(2, nc, 3)))


def _line_matrices(order: int, nc: int):
    """Assembled 1D Q_order mass and stiffness matrices on nc equal cells of
    [0, 1] (equispaced nodes, order * nc + 1 of them), CSR float64."""
    h = 1.0 / nc
    xq, wq = gauss_legendre(order + 1)
    v, d = lagrange_1d(order, xq)
    m1 = np.einsum('iq,jq,q->ij', v, v, wq) * h
    k1 = np.einsum('iq,jq,q->ij', d, d, wq) / h
    nl = order + 1
    cell_dofs = order * np.arange(nc)[:, None] + np.arange(nl)[None, :]
    nf = order * nc + 1
    out = []
    for Ke in (m1, k1):
        r, c, x = _cells_to_coo(cell_dofs, Ke)
        M = sp.coo_matrix((x, (r, c)), shape=(nf, nf)).tocsr()
        M.sum_duplicates()
        out.append(M)
    return out


def qp_hex_diffusion(nc: int = 20, order: int = 5, sigma: float = 0.0, corr: float = 0.1,
                     seed: int = 4, kfield: np.ndarray | None = None) -> Problem:
    """-div(k grad u) = f on the unit cube with tensor Q_order hexes on an nc^3
    grid, k constant per cell, identity Dirichlet rows on every boundary node;
    one patch per cell holding its (order + 1)^3 dofs (p_s = (p + 1)^d with
    q = 1, Section 2).  order 5, nc 20, k = 1 is the problem of Experiment 3
    (101^3 = 1,030,301 dofs, 8000 patches of 216 dofs).

    With k = 1 (sigma 0, no kfield) the matrix is the Kronecker sum of the 1D
    mass and stiffness matrices, which assembles the 20^3 problem without a
    per-cell triplet list; otherwise the cells are assembled in chunks."""
    nl = order + 1
    nn = order * nc + 1
    if kfield is None and sigma != 0.0:
        kfield = lognormal_field(nc, sigma, corr, seed)
    I, J, K = np.meshgrid(np.arange(nn), np.arange(nn), np.arange(nn), indexing='ij')
    bnd = ((I == 0) | (I == nn - 1) | (J == 0) | (J == nn - 1) | (K == 0) | (K == nn - 1)).transpose(2, 1, 0).ravel()
    del I, J, K
    ci = np.arange(nc)
    cz, cy, cx = np.meshgrid(ci, ci, ci, indexing='ij')          # cell id = cx + nc (cy + nc cz)
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    a = np.arange(nl)
    lz, ly, lx = np.meshgrid(a, a, a, indexing='ij')             # local id = lx + nl (ly + nl lz)
    lx, ly, lz = lx.ravel(), ly.ravel(), lz.ravel()
    cell_dofs = ((order * cx[:, None] + lx[None, :])
                 + nn * ((order * cy[:, None] + ly[None, :]) + nn * (order * cz[:, None] + lz[None, :])))
    cell_dofs = cell_dofs.astype(np.int64)
    n = nn ** 3
    if kfield is None:
        M1, K1 = _line_matrices(order, nc)
        A = (sp.kron(M1, sp.kron(M1, K1, format='csr'), format='csr')
             + sp.kron(M1, sp.kron(K1, M1, format='csr'), format='csr')
             + sp.kron(K1, sp.kron(M1, M1, format='csr'), format='csr')).tocsr()
    else:
        h = 1.0 / nc
        Kr = ref_laplace_3d(order)
        A = sp.csr_matrix((n, n))
        step = max(1, (1 << 22) // (nl ** 6))
        for c0 in range(0, nc ** 3, step):
            cd = cell_dofs[c0:c0 + step]
            Ke = (kfield[c0:c0 + step] * h)[:, None, None] * Kr[None]
            r, c, v = _cells_to_coo(cd, Ke)
            A = A + sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    # identity Dirichlet rows and columns (symmetric elimination)
    A = A.tocoo()
    keep = ~(bnd[A.row] | bnd[A.col])
    bd = np.flatnonzero(bnd)
    rows = np.concatenate([A.row[keep].astype(np.int64), bd])
    cols = np.concatenate([A.col[keep].astype(np.int64), bd])
    vals = np.concatenate([A.data[keep], np.ones(len(bd))])
    del A, keep
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    del rows, cols, vals
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int64)
    ptr, dofs = _patches_from_cells(cell_dofs)
    name = f"q{order}_hex_{nc}" + ("" if kfield is None else "_k")
    return Problem(name, A, ptr, dofs,
                   dict(nc=nc, order=order, sigma=sigma if kfield is not None else 0.0, p_s=nl ** 3,
                        k=kfield, boundary=bnd, P0=tensor_interpolation(order, nc, 3)))


def uneven_stokes_batch(n_sys: int = 256, nmin: int = 16, nmax: int = 128,
                        seed_n: int = 2, seed_perturb: int = 3, perturb: float = 0.1,
                        sizes=None) -> Problem:
    """Block-diagonal batch of independent Taylor-Hood Stokes systems.

    Mesh sizes n ~ U{nmin..nmax} (seeded); interior vertices displaced by
    U(-perturb h, perturb h) per coordinate; Dirichlet velocity dofs removed,
    so boundary patches hold fewer than 22 dofs.  ``meta['system_ptr']`` gives
    the dof offset of each system.
    """
    if sizes is None:
        sizes = np.random.default_rng(seed_n).integers(nmin, nmax + 1, size=n_sys)
    rng_p = np.random.default_rng(seed_perturb)
    mats, lists = [], []
    sys_ptr = [0]
    patch_sys = []
    off = 0
    for s, nc in enumerate(sizes):
        sub_seed = int(rng_p.integers(0, 2 ** 31))
        P = taylor_hood_stokes_2d(int(nc), perturb=perturb, perturb_seed=sub_seed,
                                  eliminate_dirichlet=True)
        mats.append(P.A)
        for kk in range(P.n_p):
            lists.append(P.patch(kk).astype(np.int64) + off)
        patch_sys.extend([s] * P.n_p)
        off += P.n
        sys_ptr.append(off)
    rows, cols, vals = [], [], []
    for s, M in enumerate(mats):
        rows.append(np.repeat(np.arange(M.shape[0], dtype=np.int64), np.diff(M.indptr)) + sys_ptr[s])
        cols.append(M.indices.astype(np.int64) + sys_ptr[s])
        vals.append(M.data)
    A, _ = _finish(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), off)
    ptr, dofs = _patches_from_lists(lists)
    return Problem(f"stokes_batch_{len(sizes)}", A, ptr, dofs,
                   dict(sizes=np.asarray(sizes), system_ptr=np.asarray(sys_ptr, dtype=np.int64),
                        patch_system=np.asarray(patch_sys, dtype=np.int32), p_s_max=22))


def rhs(n: int, seed: int = 0) -> np.ndarray:
    """b ~ N(0, 1) i.i.d. over all dofs."""
    return np.random.default_rng(seed).standard_normal(n)
