"""GPU parity of the two-level combination preconditioner (Eq.(2)) through
the C ABI.

Bars: the coarse matrix R0 A P0 has the oracle's pattern bit for bit and its
values within 1e-13 of the largest entry (summation order only); the combined
application within 1e-12 for the patch part plus the coarse solve's rounding,
kappa(A0) u relative to the coarse term (explicit inverse or block LU on the
GPU against a sparse LU in the oracle); GMRES iteration counts within one of
the oracle's, to the same tolerance.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2306_10025_amd as pr  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dt(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


CASES = {
    # n0 <= 4096: explicit inverse of A0
    "qp2_p2_8": lambda: gen.qp_diffusion_2d(8, 2),
    "qp2_p3_6": lambda: gen.qp_diffusion_2d(6, 3),
    "qp2_p4_5": lambda: gen.qp_diffusion_2d(5, 4),
    "q2hex_4": lambda: gen.q2_hex_diffusion(4),
    # n0 > 4096: block LU over the band
    "qp2_p2_70": lambda: gen.qp_diffusion_2d(70, 2),
    "q2hex_18": lambda: gen.q2_hex_diffusion(18),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    say("two-level case", request.param)
    return request.param, CASES[request.param]()


def test_coarse_matrix_matches_oracle(case):
    name, P = case
    P0 = P.meta["P0"]
    h = pr.PatchRelax(P.A, P.ptr, P.dofs)
    h.set_coarse(P0)
    st = h.stats()
    A0 = h.coarse_matrix()
    h.close()
    R = O.coarse_operator(P.A, P0)
    assert A0.shape == R.shape
    assert np.array_equal(A0.indptr, R.indptr) and np.array_equal(A0.indices, R.indices), name
    assert np.abs(A0.data - R.data).max() <= 1e-13 * np.abs(R.data).max()
    bw = max(int(np.abs(np.repeat(np.arange(R.shape[0]), np.diff(R.indptr)) - R.indices).max()), 1)
    assert st["n_coarse"] == R.shape[0] and st["coarse_nnz"] == R.nnz and st["coarse_bandwidth"] == bw
    dense = R.shape[0] <= 4096
    assert (st["coarse_block"] == 0) == dense
    say(f"  n0 {R.shape[0]} nnz {R.nnz} bandwidth {bw} block {st['coarse_block']} x {st['coarse_blocks']} "
        f"setup {st['t_coarse']:.4f}s")


def test_coarse_matrix_of_a_wide_interpolation():
    # each fine dof interpolates from ten random coarse dofs, so rows of A P0
    # reach more than 32 coarse columns: the setup takes the triple product
    # per coarse row instead of the two sparse products
    P = gen.q2_hex_diffusion(4)
    rng = np.random.default_rng(9)
    n0, per = 60, 10
    cols = np.concatenate([rng.choice(n0, size=per, replace=False) for _ in range(P.n)])
    vals = rng.uniform(0.1, 1.0, P.n * per)
    P0 = sp.csr_matrix((vals, cols, np.arange(0, P.n * per + 1, per)), shape=(P.n, n0))
    P0.sort_indices()
    assert np.diff((P.A @ P0).tocsr().indptr).max() > 32
    h = pr.PatchRelax(P.A, P.ptr, P.dofs)
    h.set_coarse(P0)
    A0 = h.coarse_matrix()
    h.close()
    R = O.coarse_operator(P.A, P0)
    assert np.array_equal(A0.indptr, R.indptr) and np.array_equal(A0.indices, R.indices)
    assert np.abs(A0.data - R.data).max() <= 1e-13 * np.abs(R.data).max()


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_combined_apply_matches_oracle(case, precision):
    name, P = case
    P0 = P.meta["P0"]
    algo = "full" if precision == "fp64" else "tolerance"
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo=algo, eps=1e-8, precision=precision, deterministic=True)
    h.set_coarse(P0)
    phi, reps = h.assignment()
    _, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    Xdb = [O.factor_inverse(tiles[x]) for x in reps]
    A0 = O.coarse_operator(P.A, P0)
    import scipy.sparse.linalg as spla
    lu = spla.splu(sp.csc_matrix(A0))
    r = np.random.default_rng(5).standard_normal(P.n)
    z = torch.full((P.n,), np.nan, dtype=torch.float64, device=DEV)
    h.apply(dt(r, torch.float64), z)
    torch.cuda.synchronize()
    zg = z.cpu().numpy()
    coarse = P0 @ lu.solve(P0.T @ r)
    # coarse-solve rounding: kappa_1(A0) u, with ||A0^{-1}||_1 estimated
    # through the oracle's LU (Higham's 1-norm estimator)
    inv = spla.LinearOperator(A0.shape, matvec=lu.solve, rmatvec=lambda y: lu.solve(y, trans="T"),
                              dtype=np.float64)
    kappa = spla.onenormest(A0) * spla.onenormest(inv)
    ctol = 64 * kappa * 2.2e-16 * np.abs(coarse).max()
    if precision == "fp64":
        patch = O.apply_patch(P.ptr, P.dofs, W, Xdb, phi, r)
        kp = max(np.linalg.cond(t) for t in tiles[:64])
        ptol = max(1e-12, 8 * 32 * kp * 2.2e-16) * np.abs(patch).max()
    else:
        patch, bound = O.apply_lowprec(P.ptr, P.dofs, W, Xdb, phi, r, 1.0, precision, return_bound=True)
        ptol = (int(np.diff(P.ptr).max()) + 8) * 2.0 ** -24 * bound.max()
    err = np.abs(zg - (patch + coarse)).max()
    say(f"  {name} {precision}: err {err:.2e} (patch tol {ptol:.2e}, coarse tol {ctol:.2e})")
    assert err <= ptol + ctol, (name, precision, err)
    h.close()


def _oracle_iters(P, eps, restart=30, tol=1e-8, b=None):
    _, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    if eps is None:
        X, phi = [O.factor_inverse(t) for t in tiles], np.arange(P.n_p)
    else:
        res = O.alg1_tolerance(tiles, eps)
        X, phi = res["X"], res["phi"]
    prec = O.combo_preconditioner(P.A, P.ptr, P.dofs, W, X, phi, P.meta["P0"])
    b = gen.rhs(P.n) if b is None else b
    x, info = O.gmres(lambda v: P.A @ v, prec, b, tol=tol, restart=restart, max_iters=1000)
    return info, x


SOLVE_CASES = {
    "qp2_p3_20_full": (lambda: gen.qp_diffusion_2d(20, 3), None),
    "q2hex_8_full": (lambda: gen.q2_hex_diffusion(8), None),
    "q2hex_8_alg1": (lambda: gen.q2_hex_diffusion(8), 0.5),
    "q2hex_18_full_band": (lambda: gen.q2_hex_diffusion(18), None),
}


@pytest.mark.parametrize("case", list(SOLVE_CASES))
def test_twolevel_solve_iterations(case):
    make, eps = SOLVE_CASES[case]
    P = make()
    say("two-level solve", case)
    b = gen.rhs(P.n)
    info_o, x_o = _oracle_iters(P, eps, b=b)
    kw = dict(algo="full") if eps is None else dict(algo="tolerance", eps=eps)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, deterministic=True, **kw)
    h.set_coarse(P.meta["P0"])
    bt = dt(b, torch.float64)
    x = torch.zeros_like(bt)
    rc = h.solve(bt, x, 1e-8)
    info = h.solve_info()
    h.close()
    xg = x.cpu().numpy()
    rel = np.linalg.norm(b - P.A @ xg) / np.linalg.norm(b)
    say(f"  iters gpu {info['iters']} oracle {info_o['iters']}, relres {rel:.2e}")
    assert rc == pr.PR_OK and rel <= 1e-8
    assert abs(info["iters"] - info_o["iters"]) <= 1
    assert np.linalg.norm(xg - x_o) <= 1e-5 * np.linalg.norm(x_o)


@pytest.mark.parametrize("order", [2, 3, 4])
def test_experiment1_on_the_gpu(order):
    # the first numerical experiment's all-patch runs (60 x 60, GMRES(20),
    # the two-level combination) give the oracle's iteration counts
    P = gen.qp_diffusion_2d(60, order)
    b = P.meta["b_exact"]
    info_o, _ = _oracle_iters(P, None, restart=20, b=b)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="full", restart=20, deterministic=True)
    h.set_coarse(P.meta["P0"])
    bt = dt(b, torch.float64)
    x = torch.zeros_like(bt)
    rc = h.solve(bt, x, 1e-8)
    info = h.solve_info()
    h.close()
    err = np.abs(x.cpu().numpy() - P.meta["u_exact"]).max()
    say(f"  p={order}: gpu {info['iters']} oracle {info_o['iters']} max error {err:.2e}")
    assert rc == pr.PR_OK
    assert abs(info["iters"] - info_o["iters"]) <= 1
    assert err <= 1e-7


def test_twolevel_graph_replay_matches_eager():
    P = gen.q2_hex_diffusion(6)
    b = dt(gen.rhs(P.n), torch.float64)
    out = []
    for graph in (False, True):
        h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=0.5, precision="bf16x3",
                          deterministic=True, graph=graph)
        h.set_coarse(P.meta["P0"])
        for rep in range(3 if graph else 1):
            x = torch.zeros_like(b)
            h.solve(b, x, 1e-8)
            torch.cuda.synchronize()
            out.append((h.solve_info()["iters"], x.cpu().numpy().copy()))
        h.close()
    it0, x0 = out[0]
    for it, xx in out[1:]:
        assert it == it0 and np.array_equal(xx, x0)


def test_coarse_errors():
    P = gen.qp_diffusion_2d(6, 2)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs)
    bad = P.meta["P0"].copy()
    bad.indices = bad.indices.copy()
    bad.indices[0] = bad.shape[1] + 3          # a column outside [0, n0)
    with pytest.raises(pr.PatchRelaxError) as e:
        h.set_coarse(bad)
    assert e.value.code == pr.PR_ERR_INVALID_ARG
    h.set_coarse(P.meta["P0"])
    with pytest.raises(pr.PatchRelaxError) as e:
        h.set_coarse(P.meta["P0"])            # once per handle
    assert e.value.code == pr.PR_ERR_INVALID_ARG
    h.close()


@pytest.mark.parametrize("precision,eps,two", [("fp64", None, True), ("bf16x3", 0.5, True),
                                                ("bf16x3", 0.5, False), ("bf16", 0.5, True)])
def test_flexible_gmres_matches_oracle(precision, eps, two):
    # flexible GMRES keeps z_j = M v_j; the oracle runs the same outer method
    # with its emulation of the reduced-precision apply (same roundings, FP32
    # sums in another order), so the iteration counts agree within one
    P = gen.q2_hex_diffusion(8)
    b = gen.rhs(P.n)
    _, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    if eps is None:
        X, phi = [O.factor_inverse(t) for t in tiles], np.arange(P.n_p)
        kw = dict(algo="full")
    else:
        res = O.alg1_tolerance(tiles, eps)
        X, phi = res["X"], res["phi"]
        kw = dict(algo="tolerance", eps=eps)
    P0 = P.meta["P0"]
    import scipy.sparse.linalg as spla
    lu = spla.splu(sp.csc_matrix(O.coarse_operator(P.A, P0))) if two else None

    def prec(r):
        z = (O.apply_patch(P.ptr, P.dofs, W, X, phi, r) if precision == "fp64"
             else O.apply_lowprec(P.ptr, P.dofs, W, X, phi, r, 1.0, precision))
        return z + P0 @ lu.solve(P0.T @ r) if two else z
    _, info_o = O.gmres(lambda v: P.A @ v, prec, b, tol=1e-8, restart=30, max_iters=2000, flexible=True)
    out = {}
    for flexible in (False, True):
        h = pr.PatchRelax(P.A, P.ptr, P.dofs, precision=precision, deterministic=True, flexible=flexible,
                          max_iters=2000, **kw)
        if two:
            h.set_coarse(P0)
        bt = dt(b, torch.float64)
        x = torch.zeros_like(bt)
        rc = h.solve(bt, x, 1e-8)
        out[flexible] = (rc, h.solve_info())
        h.close()
    rc, info = out[True]
    say(f"  {precision} eps {eps} two-level {two}: flexible {info['iters']} (oracle {info_o['iters']}), "
        f"standard {out[False][1]['iters']}")
    assert rc == pr.PR_OK and info["relres"] <= 1e-8
    assert abs(info["iters"] - info_o["iters"]) <= 1
    assert info["iters"] <= out[False][1]["iters"] + 1
