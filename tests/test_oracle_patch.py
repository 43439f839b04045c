"""Pins of the oracle's patch objects, criterion, factorisation and apply
against closed forms, brute force and the properties the paper states."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle as O


def _golden(name):
    """key value pairs of a fixture under tests/golden (comments start with #)."""
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out[line[0]] = float(line[1])
    return out


def _c1(nc=32):
    return gen.q1_poisson_2d(nc)


# ---- W (Section 2) -------------------------------------------------------

def test_weights_closed_form_q1():
    P = _c1(32)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    nn = 33
    I, J = np.meshgrid(np.arange(nn), np.arange(nn), indexing='xy')
    I, J = I.ravel(), J.ravel()
    corner = ((I == 0) | (I == 32)) & ((J == 0) | (J == 32))
    edge = ((I == 0) | (I == 32) | (J == 0) | (J == 32)) & ~corner
    inner = ~(corner | edge)
    assert np.all(W[corner] == 1.0)
    assert np.all(W[edge] == 0.5)
    assert np.all(W[inner] == 0.25)


def test_weights_brute_force_dense_restrictions():
    P = gen.taylor_hood_stokes_2d(3)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    C = np.zeros((P.n, P.n))
    for k in range(P.n_p):
        d = P.patch(k)
        V = np.zeros((len(d), P.n))
        V[np.arange(len(d)), d] = 1.0
        C += V.T @ V
    assert np.array_equal(np.diag(np.linalg.inv(C)), W)


def test_uncovered_dof_is_an_error():
    with pytest.raises(O.OracleError):
        O.cover_weights(5, np.array([0, 2]), np.array([0, 1]))


# ---- tiles A_k = V_k A V_k^T (Section 2) ---------------------------------

def test_tile_q1_interior_closed_form():
    P = _c1(32)
    k = 5 + 32 * 7                     # an interior cell
    T = O.patch_tiles(P.A, P.ptr, P.dofs, [k])[0]
    expect = 3.0 * np.eye(4) - np.ones((4, 4)) / 3.0
    assert np.allclose(T, expect, rtol=0, atol=1e-14)  # quadrature rounding


@pytest.mark.parametrize("make", [lambda: gen.q1_poisson_2d(4), lambda: gen.nedelec_hex(2),
                                  lambda: gen.taylor_hood_stokes_2d(2),
                                  lambda: gen.uneven_stokes_batch(n_sys=3, nmin=2, nmax=4)])
def test_tiles_brute_force_boolean_products(make):
    P = make()
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    Ad = P.A.toarray()
    for k in range(P.n_p):
        d = P.patch(k)
        V = np.zeros((len(d), P.n))
        V[np.arange(len(d)), d] = 1.0
        assert np.array_equal(V @ Ad @ V.T, tiles[k])   # 0/1 products are exact


# ---- boundary keys (Section 3.2) -----------------------------------------

def test_boundary_groups_2d_and_3d():
    # the counts Section 3.2 prints: 9 groups on a square, 27 on a cube
    g = _golden("boundary_groups.txt")
    P = gen.taylor_hood_stokes_2d(8)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    assert len(O.partition_groups(t)) == g["square"]
    P = gen.q2_hex_diffusion(4, sigma=0.0)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    assert len(O.partition_groups(t)) == g["cube"]
    P = gen.nedelec_hex(4)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    assert len(O.partition_groups(t)) == g["cube"]


def test_boundary_key_q1_corner_degenerates():
    # Q1: in a corner cell the one interior node's row keeps only its diagonal,
    # so all four corner patches share key 0b1111 and C1 has 6 groups.
    P = _c1(32)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    assert O.boundary_mask(t[0]) == 0b1111
    assert O.boundary_mask(t[1]) == 0b0011
    assert O.boundary_mask(t[5 + 32 * 7]) == 0
    assert len(O.partition_groups(t)) == 6


def test_boundary_key_hand_example():
    T = np.array([[1.0, 0, 0], [2.0, 3.0, 0], [0, 0, -4.0]])
    assert O.boundary_mask(T) == 0b101


# ---- criterion (Eq.(5), remark after Eq.(4)) -----------------------------

def test_criterion_scaled_copy_closed_form():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((6, 6)) + 6 * np.eye(6)
    for c in [0.5, 1.0, 2.5, 10.0]:
        # I - cB B^{-1} = (1 - c) I
        assert abs(O.crit_spectral(c * B, B) - abs(1.0 - c)) <= 1e-13 * max(1, c)


def test_criterion_identical_is_zero():
    P = _c1(32)
    t = O.patch_tiles(P.A, P.ptr, P.dofs, [100, 200])
    assert O.crit_spectral(t[0], t[1]) < 1e-14


def test_criterion_diagonal_closed_form():
    a = np.array([1.0, 2.0, 3.0, 4.0])
    b = np.array([2.0, 2.0, 1.0, 5.0])
    expect = np.max(np.abs(1.0 - a / b))
    assert abs(O.crit_spectral(np.diag(a), np.diag(b)) - expect) < 1e-15


def test_criterion_operand_order_nonsymmetric():
    # B = I + N (N nilpotent), A = diag(1, 2): ||I - A B^-1|| = sqrt(2) while
    # ||I - B^-1 A|| = sqrt(5); the criterion is the former (Eq.(5))
    A = np.diag([1.0, 2.0])
    B = np.array([[1.0, 1.0], [0.0, 1.0]])
    assert abs(O.crit_spectral(A, B) - np.sqrt(2.0)) < 1e-15
    assert abs(O.crit_spectral(A, B) - np.sqrt(5.0)) > 0.5


def test_entrywise_criteria_closed_form():
    A = np.array([[1.0, -2.0], [3.0, 4.0]])
    B = np.array([[0.0, -2.0], [1.0, 7.0]])
    assert O.crit_l1(A, B) == 6.0
    assert O.crit_fro(A, B) == np.sqrt(14.0)


def test_frobenius_lower_bound_property():
    # d(A,B) >= ||B - A||_F / (sqrt(p_s) ||B||_2): the bound used to prune
    rng = np.random.default_rng(7)
    for _ in range(300):
        p = int(rng.integers(2, 28))
        M = rng.standard_normal((p, p))
        B = M @ M.T + p * np.eye(p)
        A = B + 0.3 * rng.standard_normal((p, p)) * rng.random()
        lb = np.linalg.norm(B - A, 'fro') / (np.sqrt(p) * np.linalg.norm(B, 2))
        assert O.crit_spectral(A, B) >= lb * (1 - 1e-12)


# ---- factorisation -------------------------------------------------------

def test_inverse_q1_interior_closed_form():
    T = 3.0 * np.eye(4) - np.ones((4, 4)) / 3.0
    X = O.factor_inverse(T)
    assert np.allclose(X, np.eye(4) / 3.0 + np.ones((4, 4)) / 15.0, rtol=0, atol=1e-15)


def test_inverse_saddle_point_needs_pivoting():
    P = gen.taylor_hood_stokes_2d(4)
    T = O.patch_tiles(P.A, P.ptr, P.dofs, [5])[0]
    assert np.all(T[18:, 18:] == 0.0)        # zero pressure block
    X = O.factor_inverse(T)
    assert np.abs(T @ X - np.eye(22)).max() < 1e-10


def test_singular_patch_is_an_error():
    T = np.eye(3)
    T[1] = 0.0
    with pytest.raises((O.OracleError, Exception)):
        O.factor_inverse(T)


# ---- apply (Eq.(1), Eq.(3)) ----------------------------------------------

def test_apply_matches_dense_brute_force_nonsymmetric():
    P = gen.taylor_hood_stokes_2d(2)
    rng = np.random.default_rng(3)
    m = 5
    X = [rng.standard_normal((22, 22)) for _ in range(m)]   # nonsymmetric on purpose
    phi = rng.integers(0, m, size=P.n_p)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    r = rng.standard_normal(P.n)
    M = O.apply_operator_dense(P.n, P.ptr, P.dofs, X, phi, omega=0.7)
    z = O.apply_patch(P.ptr, P.dofs, W, X, phi, r, omega=0.7)
    assert np.allclose(z, M @ r, rtol=1e-13, atol=1e-13)


def test_apply_uneven_sizes_matches_dense():
    P = gen.uneven_stokes_batch(n_sys=2, nmin=2, nmax=3)
    rng = np.random.default_rng(4)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    phi = np.arange(P.n_p)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    r = rng.standard_normal(P.n)
    M = O.apply_operator_dense(P.n, P.ptr, P.dofs, X, phi)
    assert np.allclose(O.apply_patch(P.ptr, P.dofs, W, X, phi, r), M @ r, rtol=1e-12, atol=1e-12)


def test_block_jacobi_disjoint_patches_give_exact_inverse():
    # block-diagonal A with disjoint patches on its blocks: W = I and the
    # patch preconditioner is A^{-1} (block Jacobi, Section 2)
    rng = np.random.default_rng(5)
    blocks = [rng.standard_normal((s, s)) + s * np.eye(s) for s in (3, 5, 4, 3)]
    A = sp.block_diag(blocks).tocsr()
    n = A.shape[0]
    perm = rng.permutation(n)                  # scramble the numbering
    Pm = sp.eye(n).tocsr()[perm]
    A = (Pm.T @ A @ Pm).tocsr()
    ptr = np.cumsum([0, 3, 5, 4, 3])
    # (P^T A P)[perm[i], perm[j]] = A[i, j]: block b sits on perm[block b]
    dofs = np.concatenate([perm[ptr[i]:ptr[i + 1]] for i in range(4)]).astype(np.int32)
    cnt, W = O.cover_weights(n, ptr, dofs)
    assert np.all(W == 1.0)
    tiles = O.patch_tiles(A, ptr, dofs)
    X = [O.factor_inverse(t) for t in tiles]
    r = rng.standard_normal(n)
    z = O.apply_patch(ptr, dofs, W, X, np.arange(4), r)
    assert np.allclose(A @ z, r, rtol=1e-12, atol=1e-12)
    prec = O.make_preconditioner(A, ptr, dofs, W, X, np.arange(4))
    x, info = O.gmres(lambda v: A @ v, prec, r, tol=1e-10)
    assert info['iters'] == 1 and info['converged']


def _disjoint_blocks(seed=5):
    rng = np.random.default_rng(seed)
    sizes = (3, 5, 4, 3)
    blocks = [rng.standard_normal((s, s)) + s * np.eye(s) for s in sizes]
    A = sp.block_diag(blocks).tocsr()
    ptr = np.cumsum((0,) + sizes)
    return A, ptr, np.arange(A.shape[0], dtype=np.int32), rng


@pytest.mark.parametrize("sweeps", [1, 2, 3])
@pytest.mark.parametrize("omega", [0.5, 0.8])
def test_damped_sweeps_closed_form_on_disjoint_patches(sweeps, omega):
    # disjoint patches covering a block-diagonal A: W = I and M^{-1} = A^{-1},
    # so each damped step e <- e + omega M^{-1} (r - A e) (Experiment 3's
    # smoothing step) shrinks A^{-1} r - e by the factor 1 - omega, and from
    # e = 0 the s-th step gives e = (1 - (1 - omega)^s) A^{-1} r
    A, ptr, dofs, rng = _disjoint_blocks()
    n = A.shape[0]
    cnt, W = O.cover_weights(n, ptr, dofs)
    X = [O.factor_inverse(t) for t in O.patch_tiles(A, ptr, dofs)]
    r = rng.standard_normal(n)
    e = O.make_preconditioner(A, ptr, dofs, W, X, np.arange(4), omega=omega, sweeps=sweeps)(r)
    want = (1.0 - (1.0 - omega) ** sweeps) * np.linalg.solve(A.toarray(), r)
    assert np.allclose(e, want, rtol=1e-12, atol=1e-13)


def test_damped_sweeps_match_the_dense_iteration_with_overlap():
    # overlapping Q2 patches: s damped steps from e = 0 equal
    # sum_{t<s} (I - omega M A)^t omega M r with M the dense Eq.(1) operator
    # built from explicit restriction matrices
    P = gen.q2_hex_diffusion(2)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in O.patch_tiles(P.A, P.ptr, P.dofs)]
    phi = np.arange(P.n_p)
    M = O.apply_operator_dense(P.n, P.ptr, P.dofs, X, phi)
    Ad = P.A.toarray()
    r = np.random.default_rng(3).standard_normal(P.n)
    omega = 0.6
    for sweeps in (2, 3):
        e = O.make_preconditioner(P.A, P.ptr, P.dofs, W, X, phi, omega=omega, sweeps=sweeps)(r)
        T = np.eye(P.n) - omega * M @ Ad
        want = np.zeros(P.n)
        term = omega * M @ r
        for _ in range(sweeps):
            want += term
            term = T @ term
        assert np.allclose(e, want, rtol=1e-11, atol=1e-12 * np.abs(want).max())


def test_compressed_with_every_patch_its_own_rep_equals_full():
    P = gen.nedelec_hex(3)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    r = np.random.default_rng(0).standard_normal(P.n)
    full = O.apply_patch(P.ptr, P.dofs, W, X, np.arange(P.n_p), r)
    # Algorithm 1 with eps = 0 never matches: every patch is its own entry
    res = O.alg1_tolerance(tiles, 0.0)
    assert len(res['reps']) == P.n_p
    comp = O.apply_patch(P.ptr, P.dofs, W, res['X'], res['phi'], r)
    assert np.array_equal(full, comp)


# ---- GMRES ---------------------------------------------------------------

def test_gmres_small_dense_system():
    rng = np.random.default_rng(2)
    n = 40
    A = rng.standard_normal((n, n)) + 8 * np.eye(n)
    xs = rng.standard_normal(n)
    b = A @ xs
    x, info = O.gmres(lambda v: A @ v, lambda v: v, b, tol=1e-12, restart=n)
    assert info['converged'] and info['iters'] <= n
    assert np.allclose(x, xs, rtol=1e-9, atol=1e-9)


def test_gmres_restarted_reaches_tolerance_on_q1():
    P = _c1(16)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    b = gen.rhs(P.n)
    prec = O.make_preconditioner(P.A, P.ptr, P.dofs, W, X, np.arange(P.n_p))
    x, info = O.gmres(lambda v: P.A @ v, prec, b, tol=1e-8, restart=30)
    assert info['converged']
    assert np.linalg.norm(b - P.A @ x) <= 1e-8 * np.linalg.norm(b)


def test_gmres_omega_invariance():
    P = _c1(16)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    b = gen.rhs(P.n)
    res = []
    for om in (1.0, 0.7):
        prec = O.make_preconditioner(P.A, P.ptr, P.dofs, W, X, np.arange(P.n_p), omega=om)
        res.append(O.gmres(lambda v: P.A @ v, prec, b, tol=1e-8, restart=30))
    assert res[0][1]['iters'] == res[1][1]['iters']
    assert np.allclose(res[0][0], res[1][0], rtol=1e-7, atol=1e-9)


# ---- storage accounting (Experiment 3) -----------------------------------

def test_storage_arithmetic_experiment3():
    g = _golden("experiment3_storage.txt")
    s = O.storage_bytes(n_p=int(g["n_patches"]), p_s=int(g["patch_size"]), m_p=int(g["database_entries"]),
                        n=int(g["matrix_rows"]), value_bytes=int(g["bytes_per_value"]))
    # the paper prints one decimal (two significant digits for 62.5)
    assert round(s['database'] / 2 ** 20, 1) == g["database_MiB"]
    assert s['indices'] / 2 ** 10 == g["indices_KiB"]
    assert round(s['full'] / 2 ** 30, 1) == g["full_GiB"]
    assert round(s['jacobi'] / 2 ** 20, 1) == g["jacobi_MiB"]
    # the matrix is the degree-5 Q-mesh of 20^3 cells: (5 * 20 + 1)^3 nodes
    assert (5 * 20 + 1) ** 3 == int(g["matrix_rows"])
    # and a patch is one cell's (5 + 1)^3 nodes
    assert (5 + 1) ** 3 == int(g["patch_size"])


# ---- reduced-precision emulation -----------------------------------------

def test_bf16_rounding_bit_patterns():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7 + 2 ** -8, -2.0 ** -130,
                  3.0e38], dtype=np.float32)
    y = O.round_bf16(x)
    # tie to even, round up, tie to even (upward), subnormal, large
    expect = np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6, -2.0 ** -130, 2.9980229e38],
                      dtype=np.float32)
    assert np.array_equal(y.view(np.uint32) & 0xFFFF, np.zeros(6, np.uint32))
    assert np.allclose(y, expect, rtol=2 ** -8)
    assert y[1] == 1.0 and y[2] == np.float32(1.0 + 2 ** -7) and y[3] == np.float32(1.0 + 2 ** -6)


def test_fp16_scale_exponent():
    assert O.fp16_scale_exp(np.float32(1.0)) == -13      # 1 * 2^13 in [2^13, 2^14)
    assert O.fp16_scale_exp(np.float32(1.5e-5)) == -30
    assert O.fp16_scale_exp(np.float32(0.0)) == 0
    for m in [3.7, 1e-3, 12345.0, 2.0 ** -20]:
        e = O.fp16_scale_exp(np.float32(m))
        assert 2 ** 13 <= m * 2.0 ** (-e) < 2 ** 14


def test_lowprec_apply_close_to_fp64():
    P = _c1(8)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    phi = np.arange(P.n_p)
    r = np.random.default_rng(0).standard_normal(P.n)
    z = O.apply_patch(P.ptr, P.dofs, W, X, phi, r)
    for prec, tol in [("fp32", 1e-6), ("bf16", 2e-2), ("fp16", 2e-3), ("bf16x3", 1e-4)]:
        zl = O.apply_lowprec(P.ptr, P.dofs, W, X, phi, r, precision=prec)
        assert np.linalg.norm(zl - z) / np.linalg.norm(z) < tol


def test_bf16_split_pins():
    from oracle.lowprec import split_bf16
    hi, lo = split_bf16(np.array([1.0 + 2.0 ** -10, 3.0, 1.0 / 3.0]))
    assert hi[0] == 1.0 and lo[0] == 2.0 ** -10
    assert hi[1] == 3.0 and lo[1] == 0.0
    # the split keeps about 16 significant bits
    assert abs(hi[2] + lo[2] - 1.0 / 3.0) <= 2.0 ** -17 / 3.0


@pytest.mark.parametrize("make", [lambda: gen.q2_hex_diffusion(4), lambda: gen.nedelec_hex(4),
                                  lambda: gen.uneven_stokes_batch(n_sys=3, nmin=2, nmax=4)])
def test_csr_tile_read_equals_fancy_indexing(make):
    P = make()
    a = O.patch_tiles(P.A, P.ptr, P.dofs)
    b = O.patch_tiles_csr(P.A, P.ptr, P.dofs)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_batch_inverse_equals_factor_inverse():
    P = gen.q2_hex_diffusion(4)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X1 = [O.factor_inverse(t) for t in tiles]
    X2 = O.batch_inverse(tiles)
    for t, x1, x2 in zip(tiles, X1, X2):
        k = np.linalg.cond(t)
        assert np.abs(x1 - x2).max() <= 64 * k * 2.2e-16 * np.abs(x1).max()


def test_flexible_gmres_equals_gmres_for_a_linear_preconditioner():
    P = gen.q2_hex_diffusion(4)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    res = O.alg1_tolerance(tiles, 0.5)
    prec = O.make_preconditioner(P.A, P.ptr, P.dofs, W, res["X"], res["phi"])
    b = gen.rhs(P.n)
    x0, i0 = O.gmres(lambda v: P.A @ v, prec, b, tol=1e-10, restart=10)
    x1, i1 = O.gmres(lambda v: P.A @ v, prec, b, tol=1e-10, restart=10, flexible=True)
    assert i0["iters"] == i1["iters"] and i0["cycles"] == i1["cycles"]
    assert np.linalg.norm(x0 - x1) <= 1e-8 * np.linalg.norm(x0)


def test_flexible_gmres_stays_exact_with_a_nonlinear_preconditioner():
    # a preconditioner that rounds its input to FP32 first is not linear:
    # the flexible form's last residual estimate equals the true residual
    P = gen.q2_hex_diffusion(4)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    base = O.make_preconditioner(P.A, P.ptr, P.dofs, W, X, np.arange(P.n_p))
    prec = lambda r: base(O.round_fp32(r))
    b = gen.rhs(P.n)
    x, info = O.gmres(lambda v: P.A @ v, prec, b, tol=1e-10, restart=40, flexible=True)
    assert info["converged"] and info["cycles"] == 1
