"""GPU parity of Algorithm 2 and its variants (Section 3.2) against the
oracle, through the C ABI.

Bar: the patch map, the initial draw, the representative patches and the
number of passes are bit-exact; entry matrices are bit-exact (means are
summed in ascending member id on both sides); the FP64 inverses of the
entries agree within a condition-number bound.  Distances are computed
differently on the two sides (Jacobi on the GPU, LAPACK's SVD in the oracle),
so each case also checks that no decision of the oracle lies within rounding
of the relative tie band's edge.
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


def say(*a):
    print(*a, file=sys.stderr, flush=True)


ORACLE_VARIANT = {"kmeans_spectral": "spectral", "kmeans_entrywise": "entrywise",
                  "varmin": "varmin", "bootstrap": "bootstrap"}

# name: (problem, algo, m_target, partition, extra)
KM_CASES = {
    "q2hex_4_spectral": (lambda: gen.q2_hex_diffusion(4), "kmeans_spectral", 40, True, {}),
    "q2hex_4_entrywise": (lambda: gen.q2_hex_diffusion(4), "kmeans_entrywise", 40, True, {}),
    "q2hex_4_varmin": (lambda: gen.q2_hex_diffusion(4), "varmin", 40, True, {}),
    "q2hex_4_spectral_nopart": (lambda: gen.q2_hex_diffusion(4), "kmeans_spectral", 9, False, {}),
    "stokes_8_spectral": (lambda: gen.taylor_hood_stokes_2d(8), "kmeans_spectral", 16, True, {}),
    "stokes_8_varmin_nopart": (lambda: gen.taylor_hood_stokes_2d(8), "varmin", 7, False, {}),
    "nedelec_6_spectral": (lambda: gen.nedelec_hex(6), "kmeans_spectral", 60, True, {}),
    "nedelec_6_entrywise_nopart": (lambda: gen.nedelec_hex(6), "kmeans_entrywise", 12, False, {}),
    "q1_32_varmin_ties": (lambda: gen.q1_poisson_2d(32), "varmin", 10, True, {}),
    "q1_32_spectral_seed": (lambda: gen.q1_poisson_2d(32), "kmeans_spectral", 20, True, {"seed": 77}),
    "q2hex_4_maxiter2": (lambda: gen.q2_hex_diffusion(4), "kmeans_spectral", 9, False,
                         {"kmeans_max_iter": 2}),
    "q2hex_4_bootstrap": (lambda: gen.q2_hex_diffusion(4), "bootstrap", 0, False, {"eps": 0.99}),
    # medoid updates cycle here: the pass limit ends the loop
    "q2hex_4_s03_bootstrap_cycle": (lambda: gen.q2_hex_diffusion(4, sigma=0.3), "bootstrap", 0, False,
                                    {"eps": 0.5}),
    "batch_5_spectral": (lambda: gen.uneven_stokes_batch(n_sys=5, nmin=2, nmax=6),
                         "kmeans_spectral", 12, True, {}),
}


def _oracle(tiles, algo, m, part, extra):
    kw = dict(seed=extra.get("seed", 5), max_iter=extra.get("kmeans_max_iter", 100),
              partition=part)
    if algo == "bootstrap":
        a1 = O.alg1_tolerance(tiles, extra["eps"], "spectral")
        return O.kmeans(tiles, len(a1["reps"]), variant="bootstrap", init_reps=a1["reps"], **kw)
    return O.kmeans(tiles, m, variant=ORACLE_VARIANT[algo], **kw)


def _tie_margin(tiles, res, crit):
    """Smallest relative distance of any d_j from the tie band's edge
    d_min (1 + tie) + tie s_i in the oracle's final assignment pass."""
    tie = 1e-9
    worst = np.inf
    for i, t in enumerate(tiles):
        cand = [j for j in range(len(res["B"])) if res["B"][j].shape == t.shape]
        d = np.array([O.criterion(crit, t, res["B"][j], res["X"][j]) for j in cand])
        s = 1.0 if crit == "spectral" else np.sum(np.abs(t))
        edge = d.min() * (1 + tie) + tie * s
        worst = min(worst, (np.abs(d - edge) / edge).min())
    return worst


@pytest.mark.parametrize("case", list(KM_CASES))
def test_kmeans_bit_exact(case):
    make, algo, m, part, extra = KM_CASES[case]
    say("kmeans", case)
    P = make()
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    res = _oracle(tiles, algo, m, part, extra)
    kw = dict(algo=algo, m_target=m, partition_bc=part, seed=extra.get("seed", 5),
              kmeans_max_iter=extra.get("kmeans_max_iter", 100))
    if algo == "bootstrap":
        kw.update(criterion="spectral", eps=extra["eps"])
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, **kw)
    phi, reps = h.assignment()
    st = h.stats()
    assert st["m_p"] == len(res["B"]), case
    assert np.array_equal(reps, res["rep_patch"]), case
    assert np.array_equal(phi, res["phi"]), case
    assert st["kmeans_iters"] == max(res["iters"]), (case, st["kmeans_iters"], res["iters"])
    assert st["empty_events"] == res["empty_events"], case
    for j, B in enumerate(res["B"]):
        p = B.shape[0]
        assert np.array_equal(h.entry_matrix(j, p), B), (case, j)
        X = h.rep_inverse(j, p)
        Xo = O.factor_inverse(B)
        kappa = np.linalg.cond(B)
        assert np.abs(X - Xo).max() <= 8 * p * kappa * 2.2e-16 * np.abs(Xo).max(), (case, j)
    crit = "l1" if algo == "kmeans_entrywise" else "spectral"
    margin = _tie_margin(tiles, res, crit)
    say(case, "m_p", st["m_p"], "passes", st["kmeans_iters"], "tie margin", margin)
    assert margin > 1e-11, case
    h.close()


def test_kmeans_apply_and_solve_with_clustered_database():
    P = gen.q2_hex_diffusion(4)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    res = O.kmeans(tiles, 40, variant="spectral")
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="kmeans_spectral", m_target=40)
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    Xdb = [O.factor_inverse(B) for B in res["B"]]
    r = gen.rhs(P.n, 4)
    z_o = O.apply_patch(P.ptr, P.dofs, W, Xdb, res["phi"], r)
    rt = torch.as_tensor(r).to("cuda:0")
    z = torch.zeros_like(rt)
    h.apply(rt, z)
    torch.cuda.synchronize()
    kappa = max(np.linalg.cond(B) for B in res["B"])
    err = np.abs(z.cpu().numpy() - z_o).max() / np.abs(z_o).max()
    assert err <= max(1e-12, 8 * 32 * kappa * 2.2e-16), err
    b = torch.as_tensor(gen.rhs(P.n, 5)).to("cuda:0")
    x = torch.zeros_like(b)
    rc = h.solve(b, x, 1e-8)
    M = O.make_preconditioner(P.A, P.ptr, P.dofs, W, Xdb, res["phi"])
    xo, info_o = O.gmres(lambda v: P.A @ v, M, gen.rhs(P.n, 5), tol=1e-8, restart=30)
    info = h.solve_info()
    say("kmeans solve iters", info["iters"], "oracle", info_o["iters"])
    assert rc == pr.PR_OK
    assert abs(info["iters"] - info_o["iters"]) <= 1
    h.close()


def test_kmeans_rejects_bad_m_target():
    P = gen.q2_hex_diffusion(4)      # 27 boundary groups, 64 patches
    for m in (5, 65):
        with pytest.raises(pr.PatchRelaxError) as e:
            pr.PatchRelax(P.A, P.ptr, P.dofs, algo="kmeans_spectral", m_target=m)
        assert e.value.code == -1


def test_kmeans_repeatable_on_device():
    P = gen.nedelec_hex(6)
    out = []
    for _ in range(2):
        h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="kmeans_spectral", m_target=60)
        out.append(h.assignment())
        h.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
