"""GPU parity of database reuse across a sequence of linear systems
(pr_export_database / pr_setup_reuse) through the C ABI.

Bars: the exported blob carries the handle's phi and entries; Algorithm 1
seeded with the previous database gives the oracle's patch map, entries and
kept / rescanned / appended counts bit for bit; warm-started k-means gives
the oracle's assignment bit for bit and converges in one pass from a fixed
point."""
import struct
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


def step_system(nc, t, delta=0.05, seed=11):
    """System t of a sequence: the lognormal coefficient drifts by a seeded
    factor exp(delta g_t) per step (as a time-dependent material would)."""
    P = gen.q2_hex_diffusion(nc)
    k = P.meta["k"].copy()
    rng = np.random.default_rng(seed)
    for _ in range(t):
        k = k * np.exp(delta * rng.standard_normal(len(k)))
    return gen.q2_hex_diffusion(nc, kfield=k) if t else P


def test_export_blob_layout():
    P = gen.q2_hex_diffusion(4)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=0.5)
    blob = h.export_database()
    phi, reps = h.assignment()
    h.close()
    assert blob[:8] == b"PRDB0001"
    n_p, m_p, algo, crit, eps = struct.unpack("<qqiid", blob[8:40])
    assert (n_p, m_p, algo, crit, eps) == (P.n_p, len(reps), 1, 0, 0.5)
    assert np.array_equal(np.frombuffer(blob[40:40 + 4 * n_p], dtype="<i4"), phi)
    assert np.array_equal(np.frombuffer(blob[40 + 4 * n_p:], dtype="<i4"), reps)


@pytest.mark.parametrize("nc,eps,t", [(6, 0.99, 0), (6, 0.99, 1), (6, 0.99, 3), (8, 0.99, 2)])
def test_alg1_reuse_matches_oracle(nc, eps, t):
    P0 = step_system(nc, 0)
    Pt = step_system(nc, t)
    say(f"reuse nc={nc} eps={eps} step {t}")
    h0 = pr.PatchRelax(P0.A, P0.ptr, P0.dofs, algo="tolerance", eps=eps)
    blob = h0.export_database()
    phi0, reps0 = h0.assignment()
    h0.close()
    h = pr.PatchRelax(Pt.A, Pt.ptr, Pt.dofs, algo="tolerance", eps=eps, reuse=blob)
    phi, reps = h.assignment()
    st = h.stats()
    h.close()
    tiles = O.patch_tiles(Pt.A, Pt.ptr, Pt.dofs)
    ref = O.alg1_reuse(tiles, eps, "spectral", phi0, reps0)
    assert np.array_equal(reps, ref["reps"]) and np.array_equal(phi, ref["phi"])
    assert (st["reuse_kept"], st["reuse_rescanned"], st["reuse_appended"]) == \
        (ref["kept"], ref["rescanned"], ref["appended"])
    assert len(reps0) < 0.6 * P0.n_p          # a database worth reusing
    if t == 0:
        assert np.array_equal(phi, phi0) and st["crit_evals"] == P0.n_p - len(reps0)
    else:
        assert ref["kept"] > 0 and ref["rescanned"] + ref["appended"] > 0
    say(f"  kept {ref['kept']} rescanned {ref['rescanned']} appended {ref['appended']}, "
        f"evals {st['crit_evals']} (fresh Algorithm 1: {O.alg1_tolerance(tiles, eps)['evals']} sequential)")


@pytest.mark.parametrize("algo,variant", [("kmeans_spectral", "spectral"), ("varmin", "varmin"),
                                          ("kmeans_entrywise", "entrywise")])
def test_kmeans_warm_start_matches_oracle(algo, variant):
    P0 = step_system(5, 0)
    P1 = step_system(5, 1)
    m = 40
    h0 = pr.PatchRelax(P0.A, P0.ptr, P0.dofs, algo=algo, m_target=m)
    blob = h0.export_database()
    phi0, _ = h0.assignment()
    h0.close()
    # same system: the previous assignment is a fixed point
    hs = pr.PatchRelax(P0.A, P0.ptr, P0.dofs, algo=algo, m_target=m, reuse=blob)
    phis, _ = hs.assignment()
    assert np.array_equal(phis, phi0) and hs.stats()["kmeans_iters"] == 1
    hs.close()
    # next system: the oracle's warm-started passes
    h1 = pr.PatchRelax(P1.A, P1.ptr, P1.dofs, algo=algo, m_target=m, reuse=blob)
    phi1, _ = h1.assignment()
    its = h1.stats()["kmeans_iters"]
    h1.close()
    ref = O.kmeans(O.patch_tiles(P1.A, P1.ptr, P1.dofs), m, variant=variant, init_phi=phi0)
    assert np.array_equal(phi1, ref["phi"])
    assert its == max(ref["iters"])
    say(f"  {variant}: warm passes {its}")


def test_reuse_rejects_mismatched_blobs():
    P = gen.q2_hex_diffusion(4)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=0.5)
    blob = h.export_database()
    h.close()
    Q = gen.q2_hex_diffusion(5)
    for kw, bad in ((dict(algo="tolerance", eps=0.5), blob[:20]),            # truncated
                    (dict(algo="tolerance", eps=0.5), b"XXXX" + blob[4:]),   # not a blob
                    (dict(algo="full"), blob)):                               # nothing to reuse
        with pytest.raises(pr.PatchRelaxError) as e:
            pr.PatchRelax(P.A, P.ptr, P.dofs, reuse=bad, **kw)
        assert e.value.code == pr.PR_ERR_INVALID_ARG
    with pytest.raises(pr.PatchRelaxError) as e:                              # other patches
        pr.PatchRelax(Q.A, Q.ptr, Q.dofs, algo="tolerance", eps=0.5, reuse=blob)
    assert e.value.code == pr.PR_ERR_INVALID_ARG
