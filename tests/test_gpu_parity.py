"""GPU parity: every step of the HIP path against the CPU oracle, through the
C ABI, on seeded inputs.

Bars: bit-exact for W, tiles, boundary keys, database choice and patch map;
FP64 inverses within a condition-number bound; the FP64 apply within 1e-12
(relative to the largest entry); reduced-precision applies within the FP32
accumulation bound around the oracle's emulation of the same rounding; GMRES
iteration counts within one of the oracle's.
"""
import sys

import numpy as np
import pytest

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


SMALL = {
    "q1_32": lambda: gen.q1_poisson_2d(32),
    "stokes_8": lambda: gen.taylor_hood_stokes_2d(8),
    "nedelec_6": lambda: gen.nedelec_hex(6),
    "q2hex_4": lambda: gen.q2_hex_diffusion(4),
    "batch_5": lambda: gen.uneven_stokes_batch(n_sys=5, nmin=2, nmax=6),
}


@pytest.fixture(scope="module", params=list(SMALL))
def problem(request):
    say("problem", request.param)
    return request.param, SMALL[request.param]()


# ---- Section 2 objects -----------------------------------------------------

def test_weights_tiles_keys_bit_exact(problem):
    name, P = problem
    h = pr.PatchRelax(P.A, P.ptr, P.dofs)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    assert np.array_equal(h.weights(), W)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    keys = h.keys()
    for k in range(P.n_p):
        assert np.array_equal(h.tile(k), tiles[k]), (name, k)
        assert keys[k] == O.boundary_mask(tiles[k]), (name, k)
    st = h.stats()
    assert st["n_groups"] == len(set(O.boundary_mask(t) for t in tiles))
    h.close()


# ---- batched inverse -------------------------------------------------------

@pytest.mark.parametrize("p", [1, 3, 4, 12, 16, 22, 27, 32])
def test_batch_inverse_matches_oracle(p):
    rng = np.random.default_rng(p)
    count = 37
    A = rng.standard_normal((count, p, p)) + p * np.eye(p)
    A[0] = np.eye(p)[::-1] * 2.0 + 0.1 * rng.standard_normal((p, p))     # needs pivoting
    At = dt(A, torch.float64)
    X = torch.empty_like(At)
    info = torch.full((count,), -1, dtype=torch.int32, device=DEV)
    pr.pr_batch_inverse(p, At, X, info)
    torch.cuda.synchronize()
    Xg = X.cpu().numpy()
    assert np.all(info.cpu().numpy() == 0)
    for i in range(count):
        Xo = O.factor_inverse(A[i])
        kappa = np.linalg.cond(A[i])
        err = np.abs(Xg[i] - Xo).max() / np.abs(Xo).max()
        assert err <= 8 * p * kappa * 2.2e-16, (p, i, err, kappa)


def test_batch_inverse_reports_zero_pivot():
    p = 5
    A = np.stack([np.eye(p), np.eye(p)])
    A[1, 2, :] = 0.0                        # row 2 zero: column 3 has no pivot left
    A[1, :, 2] = 0.0
    At = dt(A, torch.float64)
    X = torch.empty_like(At)
    info = torch.zeros(2, dtype=torch.int32, device=DEV)
    pr.pr_batch_inverse(p, At, X, info)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 3]


def test_stokes_tile_inverses():
    P = gen.taylor_hood_stokes_2d(4)
    tiles = np.stack(O.patch_tiles(P.A, P.ptr, P.dofs))
    At = dt(tiles, torch.float64)
    X = torch.empty_like(At)
    info = torch.zeros(P.n_p, dtype=torch.int32, device=DEV)
    pr.pr_batch_inverse(22, At, X, info)
    torch.cuda.synchronize()
    Xg = X.cpu().numpy()
    assert np.all(info.cpu().numpy() == 0)
    for k in range(P.n_p):
        Xo = O.factor_inverse(tiles[k])
        kappa = np.linalg.cond(tiles[k])
        assert np.abs(Xg[k] - Xo).max() / np.abs(Xo).max() <= 8 * 22 * kappa * 2.2e-16


# ---- criterion -------------------------------------------------------------

@pytest.mark.parametrize("p", [2, 4, 12, 22, 27, 32])
def test_batch_criterion_matches_oracle(p):
    rng = np.random.default_rng(100 + p)
    count = 24
    B = rng.standard_normal((count, p, p)) + p * np.eye(p)
    A = B * (1.0 + rng.uniform(-0.3, 0.3, size=(count, 1, 1))) + \
        rng.standard_normal((count, p, p)) * rng.uniform(0, 0.5, size=(count, 1, 1))
    A[0] = B[0]                                          # identical pair
    A[1] = 2.5 * B[1]                                    # d = 1.5 exactly
    X = np.stack([O.factor_inverse(b) for b in B])
    d = torch.zeros(count, dtype=torch.float64, device=DEV)
    pr.pr_batch_criterion(p, "spectral", dt(A, torch.float64), None, dt(X, torch.float64), d)
    torch.cuda.synchronize()
    dg = d.cpu().numpy()
    for i in range(count):
        do = O.crit_spectral_x(A[i], X[i])
        assert abs(dg[i] - do) <= 1e-12 * max(do, 1.0) + 1e-14, (p, i, dg[i], do)
    assert abs(dg[1] - 1.5) < 1e-12
    for crit, fn in [("l1", O.crit_l1), ("fro", O.crit_fro)]:
        pr.pr_batch_criterion(p, crit, dt(A, torch.float64), dt(B, torch.float64), None, d)
        torch.cuda.synchronize()
        dg = d.cpu().numpy()
        for i in range(count):
            do = fn(A[i], B[i])
            assert abs(dg[i] - do) <= 1e-13 * max(do, 1e-300) + 1e-300


# ---- Algorithm 1 -----------------------------------------------------------

ALG1_CASES = {
    "q1_32_spec": (lambda: gen.q1_poisson_2d(32), "spectral", 1e-8),
    "stokes_8_spec": (lambda: gen.taylor_hood_stokes_2d(8), "spectral", 1e-8),
    "nedelec_6_spec": (lambda: gen.nedelec_hex(6), "spectral", 1e-8),
    "nedelec_6_l1": (lambda: gen.nedelec_hex(6), "l1", 1e-7),
    "q2hex_const_4_fro": (lambda: gen.q2_hex_diffusion(4, sigma=0.0), "fro", 1e-7),
    "q2hex_4_spec_loose": (lambda: gen.q2_hex_diffusion(4), "spectral", 0.5),
    "batch_5_spec": (lambda: gen.uneven_stokes_batch(n_sys=5, nmin=2, nmax=6), "spectral", 1e-8),
    # one component of 216 distinct patches: the unresolved patches are
    # inverted in one batch after the first 14 rounds, then rounds open
    # several entries
    "q2hex_6_spec_long": (lambda: gen.q2_hex_diffusion(6), "spectral", 0.5),
}


@pytest.mark.parametrize("case", list(ALG1_CASES))
def test_alg1_assignment_bit_exact(case):
    make, crit, eps = ALG1_CASES[case]
    say("alg1", case)
    P = make()
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    if len(set(t.shape[0] for t in tiles)) > 1:
        # Algorithm 1 runs on each patch size on its own (Section 2 remark)
        phi_o = np.zeros(P.n_p, dtype=np.int64)
        reps_o = []
        sizes = np.diff(P.ptr)
        for s in sorted(set(sizes)):
            ids = np.flatnonzero(sizes == s)
            r = O.alg1_tolerance([tiles[i] for i in ids], eps, crit)
            reps_o += [(ids[x], s) for x in r['reps']]
            phi_o[ids] = -1 - ids[r['reps']][r['phi']]
        reps_sorted = sorted(x[0] for x in reps_o)
        pos = {r: j for j, r in enumerate(reps_sorted)}
        phi_o = np.array([pos[-1 - v] for v in phi_o])
        reps_o = np.array(reps_sorted)
    else:
        res = O.alg1_tolerance(tiles, eps, crit)
        phi_o, reps_o = res['phi'], res['reps']
        if crit == "spectral" and eps < 1e-3:
            assert res['margin'] > 1e-6      # no decision within rounding of eps
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", criterion=crit, eps=eps)
    phi, reps = h.assignment()
    assert np.array_equal(reps, reps_o), (case, len(reps), len(reps_o))
    assert np.array_equal(phi, phi_o), case
    st = h.stats()
    assert st["m_p"] == len(reps_o)
    h.close()


def test_alg1_batched_inverses_match_the_oracle():
    # after the batched inversion every round copies its entry's inverse from
    # the batch: each entry's inverse must be that of its own tile
    P = gen.q2_hex_diffusion(6)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=0.5)
    st = h.stats()
    say("long alg1", st["alg1_rounds"], st["m_p"], st["alg1_batch_inverted"])
    assert st["alg1_rounds"] > 14 and st["alg1_batch_inverted"] == 1
    phi, reps = h.assignment()
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    for j, k in enumerate(reps):
        B = tiles[k]
        p = B.shape[0]
        assert np.array_equal(pr.pr_get_entry_matrix(h.h, j, p), B)
        Xg = pr.pr_get_rep_inverse(h.h, j, p)
        Xo = O.factor_inverse(B)
        tol = 8 * p * np.linalg.cond(B) * 2.2e-16
        assert np.abs(Xg - Xo).max() <= tol * np.abs(Xo).max(), j
    assert st["alg1_rounds"] < st["m_p"]
    # a short run does not take the batch
    Q = gen.nedelec_hex(6)
    h2 = pr.PatchRelax(Q.A, Q.ptr, Q.dofs, algo="tolerance", eps=1e-8)
    assert h2.stats()["alg1_batch_inverted"] == 0
    h.close()
    h2.close()


@pytest.mark.parametrize("case", list(ALG1_CASES))
def test_alg1_evaluation_count_is_the_sequential_count(case):
    # the oracle counts the comparisons of the sequential construction; without
    # the certified bound the GPU's rounds (several entries per round after the
    # batched inversion in the long case) must make exactly those evaluations,
    # and with it the evaluations made plus the pairs skipped must add up to
    # the same count
    make, crit, eps = ALG1_CASES[case]
    say("alg1 count", case)
    P = make()
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    ref = O.alg1_tolerance(tiles, eps, crit)
    h0 = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", criterion=crit, eps=eps,
                       alg1_prune=False)
    st0 = h0.stats()
    assert st0["crit_evals"] == ref["evals"], (case, st0["crit_evals"], ref["evals"])
    assert st0["crit_pruned"] == 0
    phi0, reps0 = h0.assignment()
    h0.close()
    h1 = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", criterion=crit, eps=eps)
    st1 = h1.stats()
    phi1, reps1 = h1.assignment()
    h1.close()
    assert np.array_equal(phi0, phi1) and np.array_equal(reps0, reps1)
    assert st1["crit_evals"] + st1["crit_pruned"] == ref["evals"]
    assert st1["crit_evals"] <= ref["evals"]
    if case == "nedelec_6_spec":
        assert st1["crit_evals"] < ref["evals"]      # the bound skips most pairs here


CLOSEST_CASES = {
    "q2hex_5_spec": (lambda: gen.q2_hex_diffusion(5), "spectral", 0.99),
    "q2hex_5_l1": (lambda: gen.q2_hex_diffusion(5), "l1", 50.0),
    "q2hex_5_fro": (lambda: gen.q2_hex_diffusion(5), "fro", 5.0),
    "q2hex_6_spec": (lambda: gen.q2_hex_diffusion(6), "spectral", 0.5),
    "nedelec_6_spec": (lambda: gen.nedelec_hex(6), "spectral", 1e-8),
    "batch_5_spec": (lambda: gen.uneven_stokes_batch(n_sys=5, nmin=2, nmax=6), "spectral", 0.3),
}


@pytest.mark.parametrize("case", list(CLOSEST_CASES))
def test_alg1_closest_matches_oracle(case):
    # closest matching (remarks after Algorithm 1): the database is Algorithm
    # 1's, bit for bit; the map equals the oracle's, and where a distance tie
    # could fall either way the GPU's choice must lie in the oracle's band
    make, crit, eps = CLOSEST_CASES[case]
    say("alg1 closest", case)
    P = make()
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    ref = O.alg1_closest(tiles, eps, crit)
    first = O.alg1_tolerance(tiles, eps, crit)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", criterion=crit, eps=eps, alg1_match="closest")
    phi, reps = h.assignment()
    st = h.stats()
    h.close()
    assert np.array_equal(reps, ref["reps"]), (case, len(reps), len(ref["reps"]))
    moved = int((ref["phi"] != first["phi"]).sum())
    assert st["closest_moved"] == int((phi != first["phi"]).sum())
    say(f"  entries {len(reps)}, moved {moved} (gpu {st['closest_moved']}), evals {st['closest_evals']}")
    bad = np.flatnonzero(phi != ref["phi"])
    for i in bad:
        t = tiles[i]
        scale = {"spectral": 1.0, "l1": np.abs(t).sum(), "fro": np.linalg.norm(t)}[crit]
        X = O.factor_inverse(tiles[reps[phi[i]]])
        d = O.criterion(crit, t, tiles[reps[phi[i]]], X)
        assert d < eps and d <= ref["dmin"][i] * (1 + 1e-8) + 1e-8 * scale, (case, i, d, ref["dmin"][i])
    assert len(bad) <= max(1, len(tiles) // 1000), (case, len(bad))
    if case.startswith("q2hex_5"):
        assert moved > 0          # the variant changes the map on these inputs


# ---- apply ------------------------------------------------------------------

def _rhs(n, seed=0):
    return gen.rhs(n, seed)


def test_apply_fp64_full_matches_oracle(problem):
    name, P = problem
    omega = 0.7
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, omega=omega)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    kappa = max(np.linalg.cond(t) for t in tiles)
    for seed in (0, 1):
        r = _rhs(P.n, seed)
        z_o = O.apply_patch(P.ptr, P.dofs, W, X, np.arange(P.n_p), r, omega)
        rt = dt(r, torch.float64)
        z = torch.full_like(rt, np.nan)
        h.apply(rt, z)
        torch.cuda.synchronize()
        zg = z.cpu().numpy()
        ps = int(np.diff(P.ptr).max())
        tol = max(1e-12, 8 * ps * kappa * 2.2e-16)
        err = np.abs(zg - z_o).max() / np.abs(z_o).max()
        say(name, "fp64 apply err", err, "kappa", kappa)
        assert err <= tol, (name, err, tol)
    h.close()


def test_apply_compressed_fp64_matches_oracle(problem):
    name, P = problem
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=1e-8)
    phi, reps = h.assignment()
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    # oracle database: its own inverses of the entries' patches
    Xdb = [O.factor_inverse(tiles[r]) for r in reps]
    r = _rhs(P.n, 3)
    z_o = O.apply_patch(P.ptr, P.dofs, W, Xdb, phi, r)
    rt = dt(r, torch.float64)
    z = torch.zeros_like(rt)
    h.apply(rt, z)
    torch.cuda.synchronize()
    kappa = max(np.linalg.cond(tiles[r]) for r in reps)
    err = np.abs(z.cpu().numpy() - z_o).max() / np.abs(z_o).max()
    assert err <= max(1e-12, 8 * 32 * kappa * 2.2e-16), (name, err)
    h.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16", "bf16x3"])
def test_apply_lowprec_matches_emulation(problem, precision):
    name, P = problem
    omega = 0.9
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=1e-8, precision=precision,
                      omega=omega)
    phi, reps = h.assignment()
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    Xdb = [O.factor_inverse(tiles[r]) for r in reps]
    r = _rhs(P.n, 5) * np.exp(np.random.default_rng(9).uniform(-3, 3, P.n))  # mixed magnitudes
    z_e, bound = O.apply_lowprec(P.ptr, P.dofs, W, Xdb, phi, r, omega, precision, return_bound=True)
    rt = dt(r, torch.float64)
    z = torch.zeros_like(rt)
    h.apply(rt, z)
    torch.cuda.synchronize()
    zg = z.cpu().numpy()
    ps = int(np.diff(P.ptr).max())
    tol = (ps + 4) * 2.0 ** -24 * bound + 1e-300
    bad = np.abs(zg - z_e) > tol
    say(name, precision, "max |dz|/bound", np.max(np.abs(zg - z_e) / np.maximum(bound, 1e-300)))
    assert not bad.any(), (name, precision, int(bad.sum()))
    # and the reduced-precision operator is close to the FP64 one
    z64 = O.apply_patch(P.ptr, P.dofs, W, Xdb, phi, r, omega)
    rel = np.linalg.norm(zg - z64) / np.linalg.norm(z64)
    assert rel < {"fp32": 1e-5, "bf16": 3e-2, "fp16": 3e-3, "bf16x3": 2e-4}[precision]
    h.close()


# ---- GMRES -------------------------------------------------------------------

SOLVE_CASES = {
    "q1_32_full": (lambda: gen.q1_poisson_2d(32), dict(algo="full", omega=0.7)),
    "q1_32_alg1": (lambda: gen.q1_poisson_2d(32), dict(algo="tolerance")),
    "q2hex_4_full": (lambda: gen.q2_hex_diffusion(4), dict(algo="full")),
    "q2hex_6_sweeps2": (lambda: gen.q2_hex_diffusion(6), dict(algo="full", sweeps=2, omega=0.8)),
}


@pytest.mark.parametrize("case", list(SOLVE_CASES))
def test_gmres_matches_oracle(case):
    make, kw = SOLVE_CASES[case]
    say("solve", case)
    P = make()
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, **kw)
    phi, reps = h.assignment()
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    Xdb = [O.factor_inverse(tiles[r]) for r in reps]
    b = _rhs(P.n)
    prec = O.make_preconditioner(P.A, P.ptr, P.dofs, W, Xdb, phi, omega=kw.get("omega", 1.0),
                                 sweeps=kw.get("sweeps", 1))
    x_o, info_o = O.gmres(lambda v: P.A @ v, prec, b, tol=1e-8, restart=30)
    bt = dt(b, torch.float64)
    x = torch.zeros_like(bt)
    rc = h.solve(bt, x, 1e-8)
    info = h.solve_info()
    xg = x.cpu().numpy()
    relres = np.linalg.norm(b - P.A @ xg) / np.linalg.norm(b)
    say(case, "iters gpu", info["iters"], "oracle", info_o["iters"], "relres", relres, "reorth", info["reorth"])
    assert 0 <= info["reorth"] <= info["iters"]
    assert rc == pr.PR_OK
    assert relres <= 1e-8
    assert abs(info["iters"] - info_o["iters"]) <= 1
    assert abs(info["relres"] - relres) <= 1e-10
    assert np.linalg.norm(xg - x_o) / np.linalg.norm(x_o) < 1e-5
    h.close()


def test_gmres_long_restart_matches_oracle():
    """Restart 40: steps beyond 31 basis vectors take both projections."""
    P = gen.q2_hex_diffusion(5)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="full", restart=40)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    phi, reps = h.assignment()
    Xdb = [O.factor_inverse(tiles[r]) for r in reps]
    b = _rhs(P.n)
    prec = O.make_preconditioner(P.A, P.ptr, P.dofs, W, Xdb, phi)
    x_o, info_o = O.gmres(lambda v: P.A @ v, prec, b, tol=1e-8, restart=40)
    bt = dt(b, torch.float64)
    x = torch.zeros_like(bt)
    assert h.solve(bt, x, 1e-8) == pr.PR_OK
    info = h.solve_info()
    xg = x.cpu().numpy()
    say("restart 40: iters gpu", info["iters"], "oracle", info_o["iters"], "reorth", info["reorth"])
    assert abs(info["iters"] - info_o["iters"]) <= 1
    assert np.linalg.norm(b - P.A @ xg) / np.linalg.norm(b) <= 1e-8
    assert info["reorth"] >= max(0, info["iters"] - 31)
    h.close()


@pytest.mark.parametrize("stride", [1, 7])
def test_solve_timing_counts_the_steps_that_ran(stride):
    """Per-class event timing counts every launch that did work (stride 1) or
    the launches of every stride-th Arnoldi step; the steps a converged cycle
    skips are never counted.  Timing does not change the iterates."""
    P = gen.q1_poisson_2d(32)
    b = dt(_rhs(P.n), torch.float64)
    h0 = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", deterministic=True)
    ht = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", deterministic=True, timing=stride)
    x0 = torch.zeros_like(b)
    xt = torch.zeros_like(b)
    h0.solve(b, x0, 1e-8)
    ht.solve(b, xt, 1e-8)
    i0, it = h0.solve_info(), ht.solve_info()
    assert it["iters"] == i0["iters"] and torch.equal(x0, xt)
    iters, cycles = it["iters"], it["cycles"]
    say("timing stride", stride, "iters", iters, "cycles", cycles, "timed", it["n_apply"], it["n_spmv"], it["n_orth"])
    assert iters % 30 != 0                      # the last cycle stopped early
    if stride == 1:
        assert (it["n_apply"], it["n_spmv"], it["n_orth"]) == (iters + cycles, iters + cycles, iters)
    else:
        k = -(-iters // stride)                  # steps 0, 7, 14, ... below iters
        assert (it["n_apply"], it["n_spmv"], it["n_orth"]) == (k, k, k)
    assert it["apply_ms"] > 0 and it["spmv_ms"] > 0 and it["orth_ms"] > 0
    assert i0["n_apply"] == 0
    h0.close()
    ht.close()


def test_gmres_bf16_compressed_within_iteration_bound():
    P = gen.q1_poisson_2d(32)
    b = _rhs(P.n)
    bt = dt(b, torch.float64)
    its = {}
    for prec in ("fp64", "bf16", "fp16", "bf16x3"):
        h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", precision=prec)
        x = torch.zeros_like(bt)
        rc = h.solve(bt, x, 1e-8)
        assert rc == pr.PR_OK
        xg = x.cpu().numpy()
        assert np.linalg.norm(b - P.A @ xg) / np.linalg.norm(b) <= 1e-8
        its[prec] = h.solve_info()["iters"]
        h.close()
    say("iterations", its)
    # scaled FP16 and split BF16 meet the +10% bar; plain BF16 (8-bit
    # significand) is slower to converge and is only held to +30%
    assert its["fp16"] <= 1.10 * its["fp64"]
    assert its["bf16x3"] <= 1.10 * its["fp64"]
    assert its["bf16"] <= 1.30 * its["fp64"]


def test_omega_invariance_on_gpu():
    P = gen.q1_poisson_2d(16)
    b = _rhs(P.n)
    bt = dt(b, torch.float64)
    res = []
    for om in (1.0, 0.7):
        h = pr.PatchRelax(P.A, P.ptr, P.dofs, omega=om)
        x = torch.zeros_like(bt)
        h.solve(bt, x, 1e-8)
        res.append((h.solve_info()["iters"], x.cpu().numpy()))
        h.close()
    assert res[0][0] == res[1][0]
    assert np.allclose(res[0][1], res[1][1], rtol=1e-6, atol=1e-9)


# ---- failure handling (conditions forced from the host) ----------------------

def _setup_rc(A, ptr, dofs, **kw):
    try:
        h = pr.PatchRelax(A, ptr, dofs, **kw)
    except pr.PatchRelaxError as e:
        return e.code
    h.close()
    return pr.PR_OK


def test_error_codes_on_device():
    P = gen.q1_poisson_2d(6)
    d = P.dofs.copy()
    d[5] = P.n + 3
    assert _setup_rc(P.A, P.ptr, d) == pr.PR_ERR_DOF_OUT_OF_RANGE
    d = P.dofs.copy()
    d[1] = d[0]
    assert _setup_rc(P.A, P.ptr, d) == pr.PR_ERR_DUP_DOF_IN_PATCH
    assert _setup_rc(P.A, P.ptr[:-1], P.dofs[:P.ptr[-2]]) == pr.PR_ERR_UNCOVERED_DOF
    A = P.A.copy()
    A.data = A.data.copy()
    A.data[10] = np.inf
    assert _setup_rc(A, P.ptr, P.dofs) == pr.PR_ERR_NONFINITE
    A = P.A.copy().tolil()
    A[8, :] = 0.0                              # a zero row inside a patch
    A = A.tocsr()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int64)
    assert _setup_rc(A, P.ptr, P.dofs) == pr.PR_ERR_SINGULAR_PATCH
    assert _setup_rc(A, P.ptr, P.dofs, algo="tolerance") == pr.PR_ERR_SINGULAR_PATCH


def test_apply_rejects_host_pointer():
    P = gen.q1_poisson_2d(4)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs)
    r = torch.zeros(P.n, dtype=torch.float64)                # host tensor
    z = torch.zeros(P.n, dtype=torch.float64, device=DEV)
    with pytest.raises(pr.PatchRelaxError) as e:
        h.apply(r, z)
    assert e.value.code == pr.PR_ERR_HOST_POINTER
    h.close()


# ---- deterministic (two-stage) scatter ----------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16"])
def test_deterministic_apply_repeats_bitwise_and_matches(problem, precision):
    name, P = problem
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=1e-8, precision=precision,
                      deterministic=True, omega=0.8)
    phi, reps = h.assignment()
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    Xdb = [O.factor_inverse(tiles[r]) for r in reps]
    r = _rhs(P.n, 11)
    rt = dt(r, torch.float64)
    z1 = torch.full_like(rt, np.nan)
    z2 = torch.full_like(rt, np.nan)
    h.apply(rt, z1)
    h.apply(rt, z2)
    torch.cuda.synchronize()
    a, b = z1.cpu().numpy(), z2.cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), name
    if precision == "fp64":
        z_o = O.apply_patch(P.ptr, P.dofs, W, Xdb, phi, r, 0.8)
        kappa = max(np.linalg.cond(tiles[x]) for x in reps)
        assert np.abs(a - z_o).max() / np.abs(z_o).max() <= max(1e-12, 8 * 32 * kappa * 2.2e-16)
    else:
        z_e, bound = O.apply_lowprec(P.ptr, P.dofs, W, Xdb, phi, r, 0.8, precision, return_bound=True)
        ps = int(np.diff(P.ptr).max())
        # FP32 slot values: one more rounding per slot than the atomic path
        assert np.all(np.abs(a - z_e) <= (ps + 8) * 2.0 ** -24 * bound + 1e-300), name
    h.close()


def test_deterministic_solve_matches_atomic_iterations():
    P = gen.q1_poisson_2d(32)
    b = _rhs(P.n)
    bt = dt(b, torch.float64)
    its = []
    for det in (False, True):
        h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", precision="bf16x3",
                          deterministic=det)
        x = torch.zeros_like(bt)
        assert h.solve(bt, x, 1e-8) == pr.PR_OK
        its.append(h.solve_info()["iters"])
        h.close()
    assert abs(its[0] - its[1]) <= 1


# ---- apply forms: fixed tiles + padded slot table vs work items + CSR lists ----

def _dup_patches(P, times):
    """The same problem with every patch listed `times` times (dofs then lie in
    up to 4 * times patches: the padded slot table no longer applies)."""
    lists = [P.patch(k) for k in range(P.n_p)] * times
    ptr = np.zeros(len(lists) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(d) for d in lists])
    return gen.Problem(P.name + "_dup", P.A, ptr, np.concatenate(lists).astype(np.int32), dict(P.meta))


FORM_CASES = {
    "q1_32": lambda: gen.q1_poisson_2d(32),            # p 4, whole tiles
    "nedelec_6": lambda: gen.nedelec_hex(6),           # p 12, ragged last tile
    "stokes_7": lambda: gen.taylor_hood_stokes_2d(7),  # p 22 (32-member tiles), ragged
    "q2hex_5": lambda: gen.q2_hex_diffusion(5),        # p 27, ragged, 8 slots per vertex dof
    "q1_8_dup3": lambda: _dup_patches(gen.q1_poisson_2d(8), 3),  # 12 slots per dof: CSR lists
    "batch_5": lambda: gen.uneven_stokes_batch(n_sys=5, nmin=2, nmax=6),  # uneven: items
}


@pytest.mark.parametrize("case", list(FORM_CASES))
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16", "fp16", "bf16x3"])
def test_apply_forms_are_bit_identical(case, precision):
    P = FORM_CASES[case]()
    kw = dict(algo="tolerance", eps=1e-8, precision=precision, deterministic=True, omega=0.9)
    ha = pr.PatchRelax(P.A, P.ptr, P.dofs, **kw)
    hg = pr.PatchRelax(P.A, P.ptr, P.dofs, apply_form="general", **kw)
    ht = pr.PatchRelax(P.A, P.ptr, P.dofs, apply_form="tiles", **kw)
    r = _rhs(P.n, 4) * np.exp(np.random.default_rng(3).uniform(-3, 3, P.n))
    rt = dt(r, torch.float64)
    za = torch.full_like(rt, np.nan)
    zg = torch.full_like(rt, np.nan)
    zt = torch.full_like(rt, np.nan)
    ha.apply(rt, za)
    hg.apply(rt, zg)
    ht.apply(rt, zt)
    torch.cuda.synchronize()
    a, g = za.cpu().numpy(), zg.cpu().numpy()
    assert np.array_equal(a.view(np.uint64), g.view(np.uint64)), (case, precision)
    assert np.array_equal(zt.cpu().numpy().view(np.uint64), g.view(np.uint64)), (case, precision)
    # the forced form runs fixed tiles wherever every patch has one size of at most 32 dofs
    ps_all = np.diff(P.ptr)
    uniform_small = ps_all.min() == ps_all.max() and ps_all.max() <= 32 and precision in ("bf16", "fp16", "bf16x3")
    assert ht.stats()["apply_tile_p"] == (int(ps_all.max()) if uniform_small else 0), case
    assert hg.stats()["apply_tile_p"] == 0
    # the automatic form: 16-patch tiles of long groups only (at most 1.25 items per tile)
    sa = ha.stats()
    n_tiles = (P.n_p + 15) // 16
    auto_tiles = uniform_small and ps_all.max() <= 16 and 4 * sa["n_items"] <= 5 * n_tiles
    assert sa["apply_tile_p"] == (int(ps_all.max()) if auto_tiles else 0), case
    # and both are the operator of the oracle
    phi, reps = ha.assignment()
    _, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    Xdb = [O.factor_inverse(tiles[x]) for x in reps]
    ps = int(np.diff(P.ptr).max())
    if precision == "fp64":
        z_o = O.apply_patch(P.ptr, P.dofs, W, Xdb, phi, r, 0.9)
        kappa = max(np.linalg.cond(tiles[x]) for x in reps)
        assert np.abs(a - z_o).max() / np.abs(z_o).max() <= max(1e-12, 8 * 32 * kappa * 2.2e-16)
    else:
        z_e, bound = O.apply_lowprec(P.ptr, P.dofs, W, Xdb, phi, r, 0.9, precision, return_bound=True)
        assert np.all(np.abs(a - z_e) <= (ps + 8) * 2.0 ** -24 * bound + 1e-300), (case, precision)
    # atomic scatter through the tile kernel: the same operator up to summation order
    hat = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=1e-8, precision=precision, omega=0.9)
    zt = torch.zeros_like(rt)
    hat.apply(rt, zt)
    torch.cuda.synchronize()
    t = zt.cpu().numpy()
    assert np.abs(t - a).max() <= 1e-10 * np.abs(a).max(), (case, precision)
    ha.close()
    hg.close()
    hat.close()


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_apply_graph_replays_match_eager(precision):
    # a HIP graph of back-to-back applications on distinct inputs (the warm
    # protocol of the benchmark) replayed several times, with eager work and
    # synchronisations in between: every replay gives the eager bits
    P = gen.nedelec_hex(6)
    algo = "full" if precision == "fp64" else "tolerance"
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo=algo, eps=1e-8, precision=precision, deterministic=True)
    side = torch.cuda.Stream()
    pr.pr_set_stream(h.h, side)
    rng = np.random.default_rng(9)
    R = dt(rng.standard_normal((4, P.n)), torch.float64)
    Z = torch.full_like(R, np.nan)
    E = torch.full_like(R, np.nan)
    with torch.cuda.stream(side):
        for k in range(4):
            h.apply(R[k], E[k])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for k in range(4):
            h.apply(R[k], Z[k])
    for rep in range(3):
        Z.fill_(np.nan)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Z, E), (precision, rep)
        with torch.cuda.stream(side):       # eager work between replays
            h.apply(R[0], E[0])
        torch.cuda.synchronize()
    del g
    h.close()


def test_memory_cache_reuse_gives_the_same_results():
    # the blocks a destroyed handle leaves in the device memory cache hold
    # another system's values; a setup on them must give the bits of a setup
    # on freshly mapped memory
    P = gen.nedelec_hex(6)
    kw = dict(algo="tolerance", eps=1e-8, precision="bf16x3", deterministic=True)

    def run(A):
        h = pr.PatchRelax(A, P.ptr, P.dofs, **kw)
        bt = dt(_rhs(P.n), torch.float64)
        x = torch.zeros_like(bt)
        h.solve(bt, x, 1e-8)
        r = dt(np.random.default_rng(3).standard_normal(P.n), torch.float64)
        z = torch.empty_like(r)
        h.apply(r, z)
        torch.cuda.synchronize()
        out = (x.cpu().numpy(), z.cpu().numpy(), h.assignment()[0].copy(), h.stats()["n_groups"],
               h.solve_info()["iters"])
        h.close()
        return out

    try:
        pr.pr_set_memory_cache_limit(0)
        assert pr.pr_memory_cache_info(0)["idle_bytes"] == 0
        ref = run(P.A)
        assert pr.pr_memory_cache_info(0)["idle_bytes"] == 0
        pr.pr_set_memory_cache_limit(1 << 32)
        run(P.A * 2.0 + 1e-3 * P.A.multiply(P.A > 0))       # other values, same sizes
        before = pr.pr_memory_cache_info(0)
        assert before["idle_blocks"] > 10
        out = run(P.A)
        after = pr.pr_memory_cache_info(0)
        say("cache", before, after)
        assert after["reuses"] - before["reuses"] >= before["idle_blocks"] // 2
        for a, b in zip(ref, out):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        pr.pr_release_cached_memory()
        assert pr.pr_memory_cache_info(0)["idle_bytes"] == 0
    finally:
        pr.pr_set_memory_cache_limit(-1)


def _sell_forms(A):
    """Per 64-row slice: 1 (diagonal form) when 8 * distinct offsets <=
    12 * longest row and there are at most 192 of them, else 0; host replay of
    the plan's rule for the test."""
    A = A.tocsr()
    n = A.shape[0]
    lens = np.diff(A.indptr)
    rows = np.repeat(np.arange(n), lens)
    off = A.indices.astype(np.int64) - rows
    forms = []
    for s in range((n + 63) // 64):
        a, b = A.indptr[s * 64], A.indptr[min(n, s * 64 + 64)]
        mlen = lens[s * 64:s * 64 + 64].max()
        nd = len(np.unique(off[a:b]))
        forms.append(int(mlen > 0 and 2 * nd <= 3 * mlen and nd <= 192))
    return np.array(forms)


def _mixed_length_matrix(seed=11):
    """Strictly diagonally dominant matrix: first banded rows with the five
    offsets -2 .. 2 (diagonal-form slices with an odd offset count, pairs
    with and without adjacent offsets), then rows whose 64-row slices mix
    very short and very long rows (read from the CSR copy), with rows of one
    entry, a ragged last slice and a long last row that ends at the last
    stored entry."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    n_band, n_csr = 64 * 2 + 7, 64 * 3 + 21
    n = n_band + n_csr
    rows, cols = [], []
    for i in range(n_band):
        for d in (-2, -1, 1, 2):
            if 0 <= i + d < n_band:
                rows.append(i)
                cols.append(i + d)
    for i in range(n_band, n):
        if i == n - 1:
            k = 170
        elif i % 9 == 0:
            k = 0                                # only the diagonal
        else:
            k = 150 if i % 2 else 2
        c = n_band + rng.choice(n_csr, size=k, replace=False)
        c = c[c != i]
        rows += [i] * len(c)
        cols += c.tolist()
    vals = rng.uniform(-1.0, 1.0, len(rows))
    off = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    d = np.asarray(abs(off).sum(axis=1)).ravel() + 1.0
    A = (off + sp.diags(d)).tocsr()
    A.sort_indices()
    ptr = np.arange(0, n + 1, 4, dtype=np.int64)
    if ptr[-1] != n:
        ptr = np.append(ptr, n)
    return A, ptr, np.arange(n, dtype=np.int32)


def test_spmv_paired_forms_match_the_residual():
    # the CSR-row form reads entries in pairs (short rows, one-entry rows and
    # the last stored entry exercise the clamp and the padding) and the
    # diagonal form reads pairs of diagonals (an odd offset count is padded);
    # the solve's reported residual comes from the device product b - A x
    A, ptr, dofs = _mixed_length_matrix()
    n = A.shape[0]
    h = pr.PatchRelax(A, ptr, dofs, algo="full", deterministic=True)
    st = h.stats()
    h.close()
    say("csr slices", st["sell_csr_slices"], "diag slices", st["sell_diag_slices"])
    assert st["sell_csr_slices"] >= 2 and st["sell_diag_slices"] >= 2
    b = _rhs(n, 5)
    bt = dt(b, torch.float64)
    for cap in (3, 200):
        h = pr.PatchRelax(A, ptr, dofs, algo="full", deterministic=True, max_iters=cap)
        x = torch.zeros_like(bt)
        h.solve(bt, x, 1e-12)
        info = h.solve_info()
        h.close()
        rel = np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b)
        say("cap", cap, "iters", info["iters"], "relres lib", info["relres"], "host", rel)
        assert abs(info["relres"] - rel) <= 1e-12


def test_spmv_hybrid_slices_match_the_residual():
    # one matrix with both slice forms: a Q1 block (diagonal form) stacked with
    # a Taylor-Hood block (column form); the solve's reported residual comes
    # from the device product b - A x and must match the host's
    import scipy.sparse as sp
    P1, P2 = gen.q1_poisson_2d(40), gen.taylor_hood_stokes_2d(8)
    A = sp.csr_matrix((np.concatenate([P1.A.data, P2.A.data]),
                       np.concatenate([P1.A.indices, P2.A.indices + P1.n]).astype(np.int32),
                       np.concatenate([P1.A.indptr, P1.A.nnz + P2.A.indptr[1:]]).astype(np.int64)),
                      shape=(P1.n + P2.n, P1.n + P2.n))
    ptr = np.concatenate([P1.ptr, P1.ptr[-1] + np.asarray(P2.ptr[1:])]).astype(np.int64)
    dofs = np.concatenate([P1.dofs, P2.dofs + P1.n]).astype(np.int32)
    n = A.shape[0]
    forms = _sell_forms(A)
    assert 0 < forms.sum() < len(forms)
    h = pr.PatchRelax(A, ptr, dofs, algo="full", deterministic=True)
    st = h.stats()
    say("sell", st["sell_diag_slices"], "of", len(forms), "slots", st["sell_slots"])
    assert st["sell_diag_slices"] == forms.sum()
    lens = np.diff(A.indptr)
    col_entries = sum(int(lens[s * 64:s * 64 + 64].sum()) for s in range(len(forms)) if not forms[s])
    assert st["sell_col_entries"] == col_entries
    h.close()
    b = _rhs(n, 4)
    bt = dt(b, torch.float64)
    for cap in (7, 400):        # stopped early, and converged
        h = pr.PatchRelax(A, ptr, dofs, algo="full", deterministic=True, max_iters=cap)
        x = torch.zeros_like(bt)
        h.solve(bt, x, 1e-10)
        info = h.solve_info()
        h.close()
        rel = np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b)
        say("cap", cap, "iters", info["iters"], "relres lib", info["relres"], "host", rel)
        assert abs(info["relres"] - rel) <= 1e-10
