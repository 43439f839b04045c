"""GPU tests of the uneven-batch solve (one GMRES per independent system,
masked as systems converge) and of graph replay of restart cycles, through
the C ABI.

Bars: per-system iteration counts within one of the oracle's GMRES on each
system alone, per-system residuals at the tolerance; at a fixed iteration
cap, per-system residuals within 1e-6 (relative) of the oracle's; graph
replays bit-identical to the eager solve in deterministic mode, also after
eager work between replays.
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


def stack(problems):
    """Block-diagonal matrix and patch lists of several problems."""
    data, indices, indptr, off, nnz = [], [], [np.zeros(1, np.int64)], 0, 0
    for P in problems:
        data.append(P.A.data)
        indices.append(P.A.indices.astype(np.int64) + off)
        indptr.append(P.A.indptr[1:].astype(np.int64) + nnz)
        off += P.n
        nnz += P.A.nnz
    A = sp.csr_matrix((np.concatenate(data), np.concatenate(indices).astype(np.int32), np.concatenate(indptr)),
                      shape=(off, off))
    ptrs, dofs, sptr = [0], [], [0]
    for P in problems:
        dofs.append(P.dofs.astype(np.int64) + sptr[-1])
        ptrs += list(np.asarray(P.ptr[1:]) + ptrs[-1])
        sptr.append(sptr[-1] + P.n)
    return A, np.array(ptrs, dtype=np.int64), np.concatenate(dofs).astype(np.int32), np.array(sptr)


def oracle_solve(P, b, tol, max_iters=10000, restart=30):
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    X = [O.factor_inverse(t) for t in tiles]
    prec = O.make_preconditioner(P.A, P.ptr, P.dofs, W, X, np.arange(P.n_p))
    return O.gmres(lambda v: P.A @ v, prec, b, tol=tol, restart=restart, max_iters=max_iters)


def test_batch_per_system_iterations_match_oracle():
    probs = [gen.q1_poisson_2d(n) for n in (8, 24, 12, 32, 16)]
    A, ptr, dofs, sptr = stack(probs)
    rng = np.random.default_rng(3)
    bs = [gen.rhs(P.n, i) * 10.0 ** (i - 2) for i, P in enumerate(probs)]   # very different scales
    h = pr.PatchRelax(A, ptr, dofs, algo="full", deterministic=True)
    h.set_systems(sptr)
    b = torch.as_tensor(np.concatenate(bs)).to(DEV)
    x = torch.zeros_like(b)
    assert h.solve(b, x, 1e-8) == pr.PR_OK
    its, rel = h.system_info()
    xg = x.cpu().numpy()
    for s, P in enumerate(probs):
        xo, info = oracle_solve(P, bs[s], 1e-8)
        xs = xg[sptr[s]:sptr[s + 1]]
        r = np.linalg.norm(bs[s] - P.A @ xs) / np.linalg.norm(bs[s])
        say("system", s, "n", P.n, "iters gpu", its[s], "oracle", info["iters"], "relres", r)
        assert abs(its[s] - info["iters"]) <= 1, s
        assert r <= 1e-8 and abs(rel[s] - r) <= 1e-10, s
    # the same systems one by one on the GPU
    for s, P in enumerate(probs):
        h1 = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="full", deterministic=True)
        bb = torch.as_tensor(bs[s]).to(DEV)
        xx = torch.zeros_like(bb)
        h1.solve(bb, xx, 1e-8)
        assert abs(h1.solve_info()["iters"] - its[s]) <= 1
        h1.close()
    st = h.solve_info()
    assert st["iters"] == its.max()
    h.close()


def _subsystems(B):
    sptr = np.asarray(B.meta["system_ptr"])
    psys = np.asarray(B.meta["patch_system"])
    out = []
    for s in range(len(sptr) - 1):
        lo, hi = sptr[s], sptr[s + 1]
        ids = np.flatnonzero(psys == s)
        sub_ptr = np.concatenate([[0], np.cumsum(np.diff(B.ptr)[ids])]).astype(np.int64)
        sub_dofs = np.concatenate([B.dofs[B.ptr[k]:B.ptr[k + 1]] for k in ids]) - lo
        out.append(gen.fem.Problem(name="sys", A=B.A[lo:hi, lo:hi].tocsr(), ptr=sub_ptr,
                                   dofs=sub_dofs.astype(np.int32), meta={}))
    return sptr, out


def test_batch_stokes_capped_residuals_match_oracle():
    # Stokes with one-level cell patches stalls under GMRES(30): compare the
    # residual of every system after the same number of iterations (FP64 apply)
    B = gen.uneven_stokes_batch(n_sys=4, nmin=2, nmax=5)
    sptr, subs = _subsystems(B)
    h = pr.PatchRelax(B.A, B.ptr, B.dofs, algo="full", max_iters=20)
    h.set_systems(sptr)
    b_np = gen.rhs(B.n, 0)
    b = torch.as_tensor(b_np).to(DEV)
    x = torch.zeros_like(b)
    h.solve(b, x, 1e-12)
    its, rel = h.system_info()
    for s, Ps in enumerate(subs):
        lo, hi = sptr[s], sptr[s + 1]
        xo, info = oracle_solve(Ps, b_np[lo:hi], 1e-12, max_iters=20)
        say("stokes system", s, "n", Ps.n, "iters", its[s], info["iters"], "relres", rel[s], info["relres"])
        assert its[s] == info["iters"] == 20
        # relative agreement, down to the rounding floor of FP64 sums
        assert abs(rel[s] - info["relres"]) <= 1e-6 * info["relres"] + 1e-13
    h.close()


def test_batch_fp32_matches_single_system_solves():
    # the uneven batch in FP32 (the configuration of the 256-system workload,
    # at reduced size): each system of the batch equals its own solve
    B = gen.uneven_stokes_batch(n_sys=6, nmin=2, nmax=7)
    sptr, subs = _subsystems(B)
    h = pr.PatchRelax(B.A, B.ptr, B.dofs, algo="full", precision="fp32", deterministic=True, max_iters=30)
    h.set_systems(sptr)
    b_np = gen.rhs(B.n, 1)
    b = torch.as_tensor(b_np).to(DEV)
    x = torch.zeros_like(b)
    h.solve(b, x, 1e-10)
    its, rel = h.system_info()
    for s, Ps in enumerate(subs):
        lo, hi = sptr[s], sptr[s + 1]
        # the batch solver projects with the selective form, so the single
        # solves use it too (the default delayed form rounds differently)
        h1 = pr.PatchRelax(Ps.A, Ps.ptr, Ps.dofs, algo="full", precision="fp32", deterministic=True, max_iters=30,
                           orth="selective")
        bb = torch.as_tensor(b_np[lo:hi]).to(DEV)
        xx = torch.zeros_like(bb)
        h1.solve(bb, xx, 1e-10)
        i1 = h1.solve_info()
        say("fp32 system", s, "iters", its[s], i1["iters"], "relres", rel[s], i1["relres"])
        assert its[s] == i1["iters"]
        assert abs(rel[s] - i1["relres"]) <= 1e-6 * i1["relres"]
        h1.close()
    h.close()


def test_set_systems_rejects_coupling_and_bad_ranges():
    probs = [gen.q1_poisson_2d(n) for n in (4, 6)]
    A, ptr, dofs, sptr = stack(probs)
    h = pr.PatchRelax(A, ptr, dofs, algo="full")
    for bad in ([0, 5, A.shape[0]], [0, A.shape[0] - 1], [0, sptr[1], sptr[1], A.shape[0]]):
        with pytest.raises(pr.PatchRelaxError) as e:
            h.set_systems(bad)
        assert e.value.code == pr.PR_ERR_INVALID_ARG
    h.close()


GRAPH_CASES = {
    "q1_32_alg1": (lambda: gen.q1_poisson_2d(32), dict(algo="tolerance")),
    "q2hex_6_full": (lambda: gen.q2_hex_diffusion(6), dict(algo="full")),
    "stokes_8_bf16x3_capped": (lambda: gen.taylor_hood_stokes_2d(8),
                               dict(algo="tolerance", precision="bf16x3", max_iters=75)),
}


@pytest.mark.parametrize("case", list(GRAPH_CASES))
def test_graph_replay_matches_eager(case):
    make, kw = GRAPH_CASES[case]
    P = make()
    eager = pr.PatchRelax(P.A, P.ptr, P.dofs, deterministic=True, **kw)
    graph = pr.PatchRelax(P.A, P.ptr, P.dofs, deterministic=True, graph=True, **kw)
    for seed in (0, 1, 2):
        b = torch.as_tensor(gen.rhs(P.n, seed)).to(DEV)
        xe = torch.zeros_like(b)
        xg = torch.full_like(b, np.nan)
        eager.solve(b, xe, 1e-8)
        ie = eager.solve_info()
        # eager work on the default stream between replays
        junk = torch.randn(1 << 20, device=DEV, dtype=torch.float64).sum()
        graph.solve(b, xg, 1e-8)
        ig = graph.solve_info()
        torch.cuda.synchronize()
        say(case, "seed", seed, "iters", ie["iters"], ig["iters"], "relres", ie["relres"], ig["relres"], float(junk))
        assert ie["iters"] == ig["iters"] and ie["cycles"] == ig["cycles"]
        assert torch.equal(xe, xg)
    eager.close()
    graph.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_graph_replay_matches_eager(precision):
    """A captured restart cycle of the batch solve, replayed for three
    right-hand sides with eager work between, gives the eager solve's
    per-system iterations and the same bits; a second set of systems on the
    same handle recaptures."""
    B = gen.uneven_stokes_batch(n_sys=6, nmin=2, nmax=7)
    sptr, _ = _subsystems(B)
    kw = dict(algo="full", precision=precision, deterministic=True, max_iters=40)
    eager = pr.PatchRelax(B.A, B.ptr, B.dofs, **kw)
    graph = pr.PatchRelax(B.A, B.ptr, B.dofs, graph=True, **kw)
    for h in (eager, graph):
        h.set_systems(sptr)
    for seed in (0, 1, 2):
        b = torch.as_tensor(gen.rhs(B.n, seed)).to(DEV)
        xe = torch.zeros_like(b)
        xg = torch.full_like(b, np.nan)
        eager.solve(b, xe, 1e-10)
        ie = eager.system_info()
        junk = torch.randn(1 << 20, device=DEV, dtype=torch.float64).sum()
        graph.solve(b, xg, 1e-10)
        ig = graph.system_info()
        torch.cuda.synchronize()
        say(precision, "seed", seed, "iters", list(ie[0]), list(ig[0]), float(junk))
        assert np.array_equal(ie[0], ig[0])
        assert torch.equal(xe, xg)
    # fewer, larger systems: the handle drops the old capture
    coarse = np.array([sptr[0], sptr[3], sptr[-1]])
    for h in (eager, graph):
        h.set_systems(coarse)
    b = torch.as_tensor(gen.rhs(B.n, 5)).to(DEV)
    xe = torch.zeros_like(b)
    xg = torch.full_like(b, np.nan)
    eager.solve(b, xe, 1e-10)
    graph.solve(b, xg, 1e-10)
    torch.cuda.synchronize()
    assert np.array_equal(eager.system_info()[0], graph.system_info()[0])
    assert torch.equal(xe, xg)
    eager.close()
    graph.close()


@pytest.mark.parametrize("precision,shape", [("fp64", "uneven"), ("fp32", "uneven"), ("bf16x3", "uneven"),
                                             ("bf16x3", "uniform"), ("fp16", "uniform")])
def test_autotuned_apply_is_bit_identical(precision, shape):
    P = gen.uneven_stokes_batch(n_sys=6, nmin=2, nmax=7) if shape == "uneven" else gen.nedelec_hex(7)
    # the uniform shape forces fixed tiles, so the tiles-per-wave choice is tuned
    kw = dict(algo="tolerance", precision=precision, deterministic=True,
              apply_form="tiles" if shape == "uniform" else "auto")
    plain = pr.PatchRelax(P.A, P.ptr, P.dofs, **kw)
    tuned = pr.PatchRelax(P.A, P.ptr, P.dofs, autotune=True, **kw)
    st = tuned.stats()
    say(precision, shape, "tuned shape", st["tune_threads"], st["tune_cap"], st["tune_slot"],
        st["tune_tiles_per_wave"], "in %.4f s" % st["t_autotune"])
    assert st["tune_tiles_per_wave"] in ((1, 2) if shape == "uniform" and precision != "fp64" else (0,))
    assert st["tune_xcd_remap"] in (0, 1)
    assert st["tune_threads"] in (64, 128, 256) and st["tune_slot"] in (64, 128, 256)
    assert st["tune_cap"] in (0, 1024, 2048, 4096, 8192)
    r = torch.as_tensor(gen.rhs(P.n, 7)).to(DEV)
    z1 = torch.zeros_like(r)
    z2 = torch.full_like(r, np.nan)
    plain.apply(r, z1)
    tuned.apply(r, z2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    # a second setup of the same shape reuses the choice without timing
    again = pr.PatchRelax(P.A, P.ptr, P.dofs, autotune=True, **kw)
    st2 = again.stats()
    assert (st2["tune_threads"], st2["tune_cap"], st2["tune_slot"], st2["tune_tiles_per_wave"]) == \
        (st["tune_threads"], st["tune_cap"], st["tune_slot"], st["tune_tiles_per_wave"])
    assert st2["t_autotune"] < 0.25 * st["t_autotune"]
    z3 = torch.full_like(r, np.nan)
    again.apply(r, z3)
    torch.cuda.synchronize()
    assert torch.equal(z1, z3)
    plain.close()
    tuned.close()
    again.close()
