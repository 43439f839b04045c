"""Checks of the seeded input generators (sizes, symmetry, Dirichlet rows)."""
import numpy as np
import pytest

import gen


def test_q1_sizes():
    P = gen.q1_poisson_2d(32)
    assert P.n == 1089 and P.A.nnz == 8409 and P.n_p == 1024


def test_dof_count_formulas():
    # full-size counts without assembling the big ones
    assert 2 * (2 * 64 + 1) ** 2 + 65 ** 2 == 37507
    assert 3 * 64 * 65 * 65 == 811200
    assert 65 ** 3 == 274625
    P = gen.taylor_hood_stokes_2d(8)
    assert P.n == 2 * 17 ** 2 + 9 ** 2
    P = gen.nedelec_hex(4)
    assert P.n == 3 * 4 * 5 * 5
    P = gen.q2_hex_diffusion(3)
    assert P.n == 7 ** 3


@pytest.mark.parametrize("make", [lambda: gen.q1_poisson_2d(6), lambda: gen.taylor_hood_stokes_2d(4),
                                  lambda: gen.nedelec_hex(3), lambda: gen.q2_hex_diffusion(3),
                                  lambda: gen.uneven_stokes_batch(n_sys=3, nmin=2, nmax=5)])
def test_symmetric_canonical_csr(make):
    P = make()
    A = P.A
    assert A.has_sorted_indices
    assert A.indices.dtype == np.int32 and A.indptr.dtype == np.int64
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
    d = np.diff(P.ptr)
    assert P.dofs.min() >= 0 and P.dofs.max() < P.n
    for k in range(P.n_p):
        assert len(np.unique(P.patch(k))) == d[k]


def test_dirichlet_rows_have_one_nonzero():
    P = gen.nedelec_hex(3)
    bnd = P.meta['boundary']
    rows = np.diff(P.A.indptr)
    assert np.all(rows[bnd] == 1)
    assert np.all(P.A.diagonal()[bnd] == 1.0)


def test_q1_element_closed_form():
    # the Q1 stiffness on a square is (1/6)[[4,-1,-1,-2],...] (tensor order)
    P = gen.q1_poisson_2d(1)
    # one cell, all four nodes on the boundary: identity
    assert np.array_equal(P.A.toarray(), np.eye(4))
    P = gen.q1_poisson_2d(2)
    # centre node: 4 cells x 4/6
    assert abs(P.A[4, 4] - 16.0 / 6.0) < 1e-15


def test_nedelec_curl_of_gradient_vanishes():
    # the discrete gradient of any vertex function lies in the curl-curl kernel
    Mr, Sr = gen.fem.ref_nedelec_hex()
    # vertex values f at (x,y,z) in {0,1}^3; edge dof = f(end) - f(start)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((2, 2, 2))
    pat = [(0, 0), (1, 0), (0, 1), (1, 1)]
    g = [f[1, a, b] - f[0, a, b] for a, b in pat]
    g += [f[a, 1, b] - f[a, 0, b] for a, b in pat]
    g += [f[a, b, 1] - f[a, b, 0] for a, b in pat]
    g = np.array(g)
    assert np.abs(Sr @ g).max() < 1e-13
    assert np.all(np.linalg.eigvalsh(Mr) > 0)


def test_lognormal_field_statistics():
    k = gen.lognormal_field(32, sigma=1.5, corr=0.1, seed=4)
    lg = np.log(k) / 1.5
    assert abs(lg.mean()) < 0.5 and 0.3 < lg.std() < 1.7
    assert np.array_equal(k, gen.lognormal_field(32, sigma=1.5, corr=0.1, seed=4))


def test_batch_sizes_seeded():
    s = np.random.default_rng(2).integers(16, 129, size=256)
    assert s.min() >= 16 and s.max() <= 128
    P = gen.uneven_stokes_batch(n_sys=3, nmin=3, nmax=5)
    sp_ = P.meta['system_ptr']
    assert sp_[-1] == P.n
    sizes = np.diff(P.ptr)
    assert sizes.max() == 22 and sizes.min() < 22
