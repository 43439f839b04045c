"""Pins for patches above 32 dofs: the Q_p hexahedral generator behind the
paper's Experiment 3 (degree-5 elements, 216-dof cell patches) and the
oracle's database construction at those sizes."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


@pytest.mark.parametrize("order,nc", [(3, 2), (5, 2), (4, 3)])
def test_qp_hex_sizes_and_dirichlet_rows(order, nc):
    P = gen.qp_hex_diffusion(nc, order)
    assert P.n == (order * nc + 1) ** 3
    assert P.n_p == nc ** 3
    assert np.all(np.diff(P.ptr) == (order + 1) ** 3)
    A = P.A
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()
    bnd = P.meta["boundary"]
    rows = np.flatnonzero(bnd)
    D = A[rows]
    # a Dirichlet node keeps exactly its unit diagonal
    assert np.all(np.diff(D.indptr) == 1) and np.all(D.indices == rows) and np.all(D.data == 1.0)
    # the interior block is positive definite
    inner = np.flatnonzero(~bnd)
    if len(inner):
        assert np.linalg.eigvalsh(A[inner][:, inner].toarray()).min() > 0


def test_experiment3_problem_sizes_from_the_generator_rule():
    # Experiment 3 prints 8000 patches of 216 dofs and 1,030,301 unknowns for
    # the 20^3 mesh of degree-5 elements; the generator's rules at (20, 5):
    g = _golden("experiment3_storage.txt")
    order, nc = 5, 20
    assert nc ** 3 == g["n_patches"]
    assert (order + 1) ** 3 == g["patch_size"]
    assert (order * nc + 1) ** 3 == g["matrix_rows"]
    # and the rules hold for the assembled problem on a smaller mesh
    P = gen.qp_hex_diffusion(2, order)
    assert (P.n, P.n_p, int(P.ptr[1])) == ((order * 2 + 1) ** 3, 8, 216)


def test_kronecker_assembly_equals_cell_assembly():
    # constant coefficient: the Kronecker-sum path and the per-cell path
    # assemble the same matrix up to rounding
    for order, nc in [(5, 2), (3, 3)]:
        P = gen.qp_hex_diffusion(nc, order)
        Q = gen.qp_hex_diffusion(nc, order, kfield=np.ones(nc ** 3))
        assert P.A.shape == Q.A.shape
        assert abs(P.A - Q.A).max() < 1e-13 * abs(P.A).max()
        assert np.array_equal(P.ptr, Q.ptr) and np.array_equal(P.dofs, Q.dofs)


def test_experiment3_database_has_27_entries():
    # Experiment 3: the l1 criterion with eps = 1e-7 on the constant-
    # coefficient cube keeps 27 entries (8 corners, 12 edges, 6 faces, one
    # interior); a 4^3 mesh already holds every type and repeats some
    g = _golden("experiment3_storage.txt")
    P = gen.qp_hex_diffusion(4, 5)
    t = O.patch_tiles_csr(P.A, P.ptr, P.dofs)
    for crit in ("l1", "fro"):
        res = O.alg1_tolerance(t, 1e-7, crit)
        assert len(res["reps"]) == g["database_entries"]
        assert res["margin"] > 1e-3
    # every interior cell maps to the interior cell's entry
    nc = 4
    ids = np.arange(nc ** 3)
    ix, iy, iz = ids % nc, (ids // nc) % nc, ids // (nc * nc)
    inner = ids[(ix > 0) & (ix < nc - 1) & (iy > 0) & (iy < nc - 1) & (iz > 0) & (iz < nc - 1)]
    res = O.alg1_tolerance(t, 1e-7, "l1")
    assert len(set(res["phi"][inner])) == 1 and res["reps"][res["phi"][inner[0]]] == inner[0]


def test_spectral_database_on_64_dof_patches():
    P = gen.qp_hex_diffusion(4, 3)
    t = O.patch_tiles_csr(P.A, P.ptr, P.dofs)
    res = O.alg1_tolerance(t, 1e-8, "spectral")
    assert len(res["reps"]) == 27
    # a lognormal coefficient leaves more entries, each patch within eps of its own
    Q = gen.qp_hex_diffusion(4, 3, sigma=0.5)
    tq = O.patch_tiles_csr(Q.A, Q.ptr, Q.dofs)
    rq = O.alg1_tolerance(tq, 0.5, "spectral")
    assert 27 < len(rq["reps"]) < Q.n_p
    assert O.alg1_invariants_hold(lambda k: tq[k], rq["phi"], rq["reps"], 0.5, "spectral", range(Q.n_p))


def test_large_patch_tiles_and_inverses():
    P = gen.qp_hex_diffusion(3, 5, sigma=1.0)
    t_csr = O.patch_tiles_csr(P.A, P.ptr, P.dofs)
    t_fancy = O.patch_tiles(P.A, P.ptr, P.dofs, ks=[0, 13, 26])
    for a, k in enumerate([0, 13, 26]):
        assert np.array_equal(t_csr[k], t_fancy[a])
    X = O.factor_inverse(t_csr[13])
    assert np.abs(t_csr[13] @ X - np.eye(216)).max() < 1e-10
