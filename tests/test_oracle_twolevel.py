"""Pins of the oracle's two-level combination preconditioner (Eq.(2)).

P0 against the generator's independent construction and against the
multilinear functions it must reproduce; R0 A P0 against the first-order
stiffness matrix assembled directly; the combined operator against a dense
brute force; and, as a soft pin, the all-patch iteration counts of the first
numerical experiment (Table 1)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "experiment1_table1.txt")


@pytest.mark.parametrize("order,nc,dim", [(2, 6, 2), (3, 5, 2), (4, 4, 2), (5, 3, 2), (2, 3, 3)])
def test_linear_interpolation_matches_the_generator(order, nc, dim):
    coords = gen.tensor_node_coords(order, nc, dim)
    P0 = O.linear_interpolation(coords, nc)
    G = gen.tensor_interpolation(order, nc, dim)
    assert P0.shape == G.shape == ((order * nc + 1) ** dim, (nc - 1) ** dim)
    assert abs(P0 - G).max() <= 1e-14
    assert P0.nnz == G.nnz


@pytest.mark.parametrize("order,nc,dim", [(2, 5, 2), (3, 4, 2), (2, 3, 3)])
def test_interpolation_reproduces_multilinear_functions(order, nc, dim):
    coords = gen.tensor_node_coords(order, nc, dim)
    P = O.linear_interpolation(coords, nc, keep_boundary=True)
    verts = gen.tensor_node_coords(1, nc, dim)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(1 << dim)

    def f(x):
        # sum over corners of c_m prod_{d in m} x_d: every multilinear monomial
        out = np.zeros(len(x))
        for m in range(1 << dim):
            t = np.full(len(x), c[m])
            for d in range(dim):
                if (m >> d) & 1:
                    t = t * x[:, d]
            out += t
        return out
    assert np.abs(P @ f(verts) - f(coords)).max() <= 1e-13
    assert np.abs(P @ np.ones(P.shape[1]) - 1.0).max() <= 1e-15


@pytest.mark.parametrize("order", [2, 3, 4])
def test_coarse_operator_is_the_first_order_stiffness(order):
    # with rho = 1, R0 A P0 is the bilinear (Q1) Laplacian on the same mesh,
    # since the hat functions are exact members of the high-order space
    nc = 6
    P = gen.qp_diffusion_2d(nc, order, rho=lambda x, y: np.ones_like(x))
    A0 = O.coarse_operator(P.A, P.meta["P0"])
    Q1 = gen.q1_poisson_2d(nc).A
    inner = np.flatnonzero(~gen.q1_poisson_2d(nc).meta["boundary"])
    Q1i = Q1[inner][:, inner]
    assert abs(A0 - Q1i).max() <= 1e-13 * abs(Q1i).max()
    assert abs(A0 - A0.T).max() == 0.0 or abs(A0 - A0.T).max() <= 1e-15 * abs(A0).max()


def test_coarse_operator_drops_rounding_residue_only():
    P = gen.qp_diffusion_2d(8, 3)
    full = (P.meta["P0"].T @ (P.A @ P.meta["P0"])).tocsr()
    A0 = O.coarse_operator(P.A, P.meta["P0"])
    # every kept entry of the 9-point bilinear stencil stays; what is dropped is tiny
    D = (full - A0).tocsr()
    assert abs(D).max() <= 1e-13 * abs(full).max()
    assert A0.nnz <= 9 * A0.shape[0]


def test_combo_preconditioner_dense_brute_force():
    P = gen.qp_diffusion_2d(4, 2)
    n = P.n
    cnt, W = O.cover_weights(n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    phi = np.arange(P.n_p)
    P0 = P.meta["P0"].toarray()
    Ad = P.A.toarray()
    M = O.apply_operator_dense(n, P.ptr, P.dofs, X, phi) + P0 @ np.linalg.inv(P0.T @ Ad @ P0) @ P0.T
    prec = O.combo_preconditioner(P.A, P.ptr, P.dofs, W, X, phi, P.meta["P0"])
    R = np.random.default_rng(2).standard_normal((5, n))
    for r in R:
        z = prec(r)
        assert np.abs(z - M @ r).max() <= 1e-12 * np.abs(M @ r).max()


def _experiment1_iterations(order):
    P = gen.qp_diffusion_2d(60, order)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    prec = O.combo_preconditioner(P.A, P.ptr, P.dofs, W, X, np.arange(P.n_p), P.meta["P0"])
    x, info = O.gmres(lambda v: P.A @ v, prec, P.meta["b_exact"], tol=1e-8, restart=20, max_iters=300)
    return info, np.abs(x - P.meta["u_exact"]).max()


@pytest.mark.slow
@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_experiment1_all_patch_iterations_soft_pin(order):
    # soft pin: the paper does not state its node placement or quadrature;
    # with equispaced nodes and Gauss quadrature the counts land within four
    # of Table 1's all-patch column, and the one-level method (no coarse
    # term) needs hundreds of iterations on the same systems
    table = dict(np.loadtxt(GOLDEN, dtype=int))
    info, err = _experiment1_iterations(order)
    assert info["converged"]
    assert abs(info["iters"] - table[order]) <= 4, (order, info["iters"], table[order])
    assert err <= 1e-8          # the discrete solution is the nodal interpolant of sin(pi x) sin(pi y)
