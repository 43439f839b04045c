"""GPU parity of patches above 32 dofs (the 64- and 216-dof cell patches of
degree-3 and degree-5 hexahedra, Experiment 3's regime) through the C ABI.

Bars: tiles, W and the boundary keys (the 32-bit XOR fold of the oracle's
single-nonzero row mask) bit for bit; Algorithm 1's phi and database bit
for bit, with evaluations plus pruned pairs equal to the oracle's sequential
comparison count, on cases whose oracle margin min |d - eps| / eps exceeds
1e-9; inverses within 64 p kappa u of LAPACK's; the FP64 apply within
1e-11 of the oracle relative to max |z| (inverses from different
eliminations); the FP32 apply within 1e-5; the deterministic apply bit
identical across calls; GMRES iterations within one of the oracle's.  The
oracle's database and patch map come from its own Algorithm 1 (the GPU's
are checked equal to them first).
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


def dt(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def fold32(mask: int) -> int:
    out = 0
    while mask:
        out ^= mask & 0xFFFFFFFF
        mask >>= 32
    return out


def mixed_sizes():
    """Degree-3 cells (64 dofs) plus 20-dof partial patches: one handle with
    two sizes, uneven tiles, and patches of both kinds of kernel size."""
    P = gen.qp_hex_diffusion(3, 3, sigma=0.8)
    lists = [P.patch(k) for k in range(P.n_p)] + [P.patch(k)[:20] for k in range(0, P.n_p, 2)]
    ptr = np.zeros(len(lists) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(l) for l in lists])
    return gen.Problem("mixed", P.A, ptr, np.concatenate(lists).astype(np.int32), P.meta)


PROBLEMS = {
    "q3_4_const": lambda: gen.qp_hex_diffusion(4, 3),
    "q3_4_logn": lambda: gen.qp_hex_diffusion(4, 3, sigma=0.5),
    "q5_3_logn": lambda: gen.qp_hex_diffusion(3, 5, sigma=1.0),
    "q5_4_const": lambda: gen.qp_hex_diffusion(4, 5),
    "mixed": mixed_sizes,
    "q6_2_logn": lambda: gen.qp_hex_diffusion(2, 6, sigma=1.0),     # 343 dofs
    "q7_2_const": lambda: gen.qp_hex_diffusion(2, 7),                # 512 dofs, the largest
}
_cache = {}


def problem(name):
    if name not in _cache:
        P = PROBLEMS[name]()
        _cache[name] = (P, O.patch_tiles_csr(P.A, P.ptr, P.dofs))
    return _cache[name]


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_extraction_weights_keys(name):
    P, tiles = problem(name)
    say("wide extraction", name, "max p", int(np.diff(P.ptr).max()))
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="full")
    for k in range(P.n_p):
        assert np.array_equal(h.tile(k), tiles[k]), k
    _, W = O.cover_weights(P.n, P.ptr, P.dofs)
    assert np.array_equal(h.weights(), W)
    keys = h.keys()
    ref = np.array([fold32(O.boundary_mask(t)) for t in tiles], dtype=np.uint32)
    assert np.array_equal(keys, ref)
    st = h.stats()
    assert st["max_ps"] == int(np.diff(P.ptr).max()) and st["n_groups"] == len(set(ref.tolist()))
    h.close()


@pytest.mark.parametrize("name", ["q3_4_logn", "q5_3_logn", "mixed", "q7_2_const"])
def test_full_inverses(name):
    P, tiles = problem(name)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="full")
    worst = 0.0
    for k in range(0, P.n_p, 3):
        p = tiles[k].shape[0]
        Xo = np.linalg.inv(tiles[k])
        Xg = h.rep_inverse(k, p)
        kappa = np.linalg.cond(tiles[k])
        err = np.abs(Xg - Xo).max() / np.abs(Xo).max()
        worst = max(worst, err / (kappa * 2.2e-16 * p))
        assert err <= 64 * p * kappa * 2.2e-16, (k, err, kappa)
    say(f"  {name}: worst inverse error / (p kappa u) = {worst:.3g}")
    h.close()


def test_batch_inverse_wide_and_zero_pivot():
    rng = np.random.default_rng(3)
    for p in (33, 100, 216):
        A = rng.standard_normal((5, p, p)) + p * np.eye(p)
        A[4] = A[3]
        A[4][:, 7] = 0.0                       # singular: a zero column
        X = torch.zeros((5, p, p), dtype=torch.float64, device=DEV)
        info = torch.zeros(5, dtype=torch.int32, device=DEV)
        pr.pr_batch_inverse(p, dt(A), X, info)
        torch.cuda.synchronize()
        inf = info.cpu().numpy()
        assert list(inf[:4]) == [0, 0, 0, 0] and inf[4] > 0
        for i in range(4):
            Xo = np.linalg.inv(A[i])
            assert np.abs(X[i].cpu().numpy() - Xo).max() <= 64 * p * np.linalg.cond(A[i]) * 2.2e-16 * np.abs(Xo).max()


def _eps_for(tiles, crit, frac):
    """eps as a fraction of the median norm, so that a share of pairs match"""
    if crit == "spectral":
        return frac
    f = (lambda t: np.abs(t).sum()) if crit == "l1" else (lambda t: np.sqrt((t * t).sum()))
    return frac * float(np.median([f(t) for t in tiles]))


ALG1_CASES = [
    ("q5_4_const", "l1", None, 1e-7),       # Experiment 3: 27 entries
    ("q5_4_const", "fro", None, 1e-7),
    ("q3_4_const", "spectral", None, 1e-8),
    ("q3_4_logn", "spectral", None, 0.5),
    ("q3_4_logn", "spectral", None, 0.3),
    ("q3_4_logn", "l1", 0.3, None),
    ("q3_4_logn", "fro", 0.3, None),
    ("q5_3_logn", "spectral", None, 0.9),
    ("mixed", "spectral", None, 0.5),
    ("mixed", "l1", 0.3, None),
    ("q7_2_const", "l1", None, 1e-7),
    ("q6_2_logn", "spectral", None, 0.9),
]


@pytest.mark.parametrize("name,crit,frac,eps", ALG1_CASES)
def test_alg1_matches_oracle(name, crit, frac, eps):
    P, tiles = problem(name)
    eps = eps if eps is not None else _eps_for(tiles, crit, frac)
    ref = O.alg1_tolerance(tiles, eps, crit)
    say(f"alg1 wide {name} {crit} eps {eps:.4g}: m_p {len(ref['reps'])}, evals {ref['evals']}, "
        f"margin {ref['margin']:.2e}")
    assert ref["margin"] > 1e-9
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", criterion=crit, eps=eps)
    phi, reps = h.assignment()
    st = h.stats()
    assert np.array_equal(reps, ref["reps"]) and np.array_equal(phi, ref["phi"])
    assert st["crit_evals"] + st["crit_pruned"] == ref["evals"]
    assert st["alg1_rounds"] == len(ref["reps"])
    if name == "q5_4_const":
        assert len(reps) == 27
    # the database holds the entries' inverses
    for j in range(0, len(reps), max(1, len(reps) // 5)):
        p = tiles[reps[j]].shape[0]
        Xo = np.linalg.inv(tiles[reps[j]])
        kappa = np.linalg.cond(tiles[reps[j]])
        assert np.abs(h.rep_inverse(j, p) - Xo).max() <= 64 * p * kappa * 2.2e-16 * np.abs(Xo).max()
    say(f"  evals {st['crit_evals']} pruned {st['crit_pruned']} refined {st['crit_refined']} "
        f"midpoint {st['crit_exact']}, database {st['t_database'] * 1e3:.1f} ms")
    h.close()


APPLY_CASES = [
    ("q5_3_logn", dict(algo="full")),                                   # one patch per block
    ("q5_4_const", dict(algo="tolerance", criterion="l1", eps=1e-7)),   # grouped, matrix cores
    ("q3_4_logn", dict(algo="tolerance", eps=0.5)),
    ("mixed", dict(algo="tolerance", eps=0.5)),
    ("mixed", dict(algo="full")),
    ("q7_2_const", dict(algo="tolerance", criterion="l1", eps=1e-7)),
    ("q6_2_logn", dict(algo="full")),
]


def _oracle_db(P, tiles, kw, h):
    """The oracle's inverses and patch map for the setup in kw; the GPU's
    patch map must be the same."""
    if kw.get("algo") == "full":
        X, phi, reps = [O.factor_inverse(t) for t in tiles], np.arange(P.n_p), np.arange(P.n_p)
    else:
        ref = O.alg1_tolerance(tiles, kw["eps"], kw.get("criterion", "spectral"))
        X, phi, reps = ref["X"], ref["phi"], ref["reps"]
    phig, repsg = h.assignment()
    assert np.array_equal(phig, phi) and np.array_equal(repsg, reps)
    return X, phi


def _oracle_apply(P, tiles, kw, h, r):
    _, W = O.cover_weights(P.n, P.ptr, P.dofs)
    X, phi = _oracle_db(P, tiles, kw, h)
    return O.apply_patch(P.ptr, P.dofs, W, X, phi, r)


@pytest.mark.parametrize("name,kw", APPLY_CASES)
@pytest.mark.parametrize("det", [False, True])
def test_apply_fp64_matches_oracle(name, kw, det):
    P, tiles = problem(name)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, precision="fp64", deterministic=det, **kw)
    r = gen.rhs(P.n, seed=7)
    z = torch.zeros(P.n, dtype=torch.float64, device=DEV)
    h.apply(dt(r), z)
    zg = z.cpu().numpy()
    zo = _oracle_apply(P, tiles, kw, h, r)
    err = np.abs(zg - zo).max() / np.abs(zo).max()
    say(f"  apply fp64 {name} {kw.get('algo')} det={det}: {err:.2e}")
    assert err < 1e-11
    if det:
        z2 = torch.full((P.n,), 3.0, dtype=torch.float64, device=DEV)
        h.apply(dt(r), z2)
        assert torch.equal(z, z2)
    h.close()


@pytest.mark.parametrize("name,kw", APPLY_CASES[:3])
def test_apply_fp32_within_bound(name, kw):
    P, tiles = problem(name)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, precision="fp32", deterministic=True, **kw)
    r = gen.rhs(P.n, seed=8)
    z = torch.zeros(P.n, dtype=torch.float64, device=DEV)
    h.apply(dt(r), z)
    zo = _oracle_apply(P, tiles, kw, h, r)
    err = np.abs(z.cpu().numpy() - zo).max() / np.abs(zo).max()
    say(f"  apply fp32 {name}: {err:.2e}")
    assert err < 1e-5
    h.close()


SOLVE_CASES = {
    "q5_3_logn_full": ("q5_3_logn", dict(algo="full")),
    "q5_4_const_l1": ("q5_4_const", dict(algo="tolerance", criterion="l1", eps=1e-7)),
    "q3_4_logn_spec": ("q3_4_logn", dict(algo="tolerance", eps=0.5)),
}


@pytest.mark.parametrize("case", list(SOLVE_CASES))
@pytest.mark.parametrize("twolevel", [False, True])
def test_solve_iterations_match_oracle(case, twolevel):
    name, kw = SOLVE_CASES[case]
    P, tiles = problem(name)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, precision="fp64", **kw)
    if twolevel:
        h.set_coarse(P.meta["P0"])
    b = gen.rhs(P.n)
    x = torch.zeros(P.n, dtype=torch.float64, device=DEV)
    h.solve(dt(b), x, 1e-8)
    info = h.solve_info()
    _, W = O.cover_weights(P.n, P.ptr, P.dofs)
    X, phi = _oracle_db(P, tiles, kw, h)
    if twolevel:
        prec = O.combo_preconditioner(P.A, P.ptr, P.dofs, W, X, phi, P.meta["P0"])
    else:
        prec = O.make_preconditioner(P.A, P.ptr, P.dofs, W, X, phi)
    xo, io = O.gmres(lambda v: P.A @ v, prec, b, tol=1e-8, restart=30, max_iters=3000)
    say(f"  solve {case} twolevel={twolevel}: {info['iters']} iterations (oracle {io['iters']}), "
        f"relres {info['relres']:.2e}")
    assert info["status"] == pr.PR_OK and info["relres"] < 1e-8
    assert abs(info["iters"] - io["iters"]) <= 1
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-6 * np.abs(xo).max()
    h.close()


def test_unsupported_options_for_wide_patches():
    P, _ = problem("q3_4_const")
    for kw in (dict(algo="kmeans_spectral", m_target=30), dict(algo="varmin", m_target=30),
               dict(algo="bootstrap", m_target=30), dict(algo="tolerance", mlp=True),
               dict(algo="tolerance", alg1_match="closest"), dict(algo="full", precision="bf16"),
               dict(algo="full", precision="bf16x3")):
        with pytest.raises(pr.PatchRelaxError) as e:
            pr.PatchRelax(P.A, P.ptr, P.dofs, **kw)
        assert e.value.code == pr.PR_ERR_UNSUPPORTED, kw
    # database reuse: the blob exports, a seeded setup is refused
    hq = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", criterion="l1", eps=1e-7)
    blob = hq.export_database()
    hq.close()
    with pytest.raises(pr.PatchRelaxError) as e:
        pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", criterion="l1", eps=1e-7, reuse=blob)
    assert e.value.code == pr.PR_ERR_UNSUPPORTED
    # batches of systems
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="full")
    with pytest.raises(pr.PatchRelaxError) as e:
        h.set_systems(np.array([0, P.n], dtype=np.int64))
    assert e.value.code == pr.PR_ERR_UNSUPPORTED
    h.close()
    # above 512 dofs
    B = gen.q1_poisson_2d(22)
    ptr = np.array([0, 513, B.n], dtype=np.int64)
    with pytest.raises(pr.PatchRelaxError) as e:
        pr.PatchRelax(B.A, ptr, np.arange(B.n, dtype=np.int32))
    assert e.value.code == pr.PR_ERR_UNSUPPORTED


def test_wide_validation_errors():
    P, _ = problem("q3_4_const")
    d = P.dofs.copy()
    d[P.ptr[5] + 3] = d[P.ptr[5]]                # duplicate inside a 64-dof patch
    with pytest.raises(pr.PatchRelaxError) as e:
        pr.PatchRelax(P.A, P.ptr, d)
    assert e.value.code == pr.PR_ERR_DUP_DOF_IN_PATCH and "patch 5" in str(e.value)
    d = P.dofs.copy()
    d[P.ptr[9] + 40] = P.n                       # out of range
    with pytest.raises(pr.PatchRelaxError) as e:
        pr.PatchRelax(P.A, P.ptr, d)
    assert e.value.code == pr.PR_ERR_DOF_OUT_OF_RANGE
