"""Parity at the full size of the benchmark workload (Nedelec 64^3: 811,200
dofs, 262,144 patches), in the configuration bench.py times, on outputs the
oracle computes one by one: sampled tiles and weights (bit-exact), Algorithm
1's patch map and entries for all 262,144 patches against the oracle's
sequential loop (SHA-256 digests written once by
tests/golden/make_alg1_nedelec64.py) and its defining properties on sampled
patches, and the apply at sampled dofs (FP64 within 1e-12 of the oracle; the
split-BF16 apply within its accuracy of the FP64 one).
"""
import hashlib
import os
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
EPS = 1e-8


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def big():
    say("generating nedelec_hex(64)")
    P = gen.nedelec_hex(64)
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=EPS, precision="bf16x3",
                      deterministic=True)
    yield P, h
    h.close()


def _tile(P, k):
    d = P.patch(k)
    return P.A[d][:, d].toarray()


def test_fullsize_tiles_weights_keys(big):
    P, h = big
    rng = np.random.default_rng(0)
    ks = rng.choice(P.n_p, size=300, replace=False)
    keys = h.keys()
    for k in ks:
        t = _tile(P, k)
        assert np.array_equal(h.tile(k), t), k
        assert keys[k] == O.boundary_mask(t), k
    cnt = np.bincount(P.dofs, minlength=P.n)
    W = h.weights()
    idx = rng.choice(P.n, size=2000, replace=False)
    assert np.array_equal(W[idx], 1.0 / cnt[idx])


def _golden_alg1():
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "alg1_nedelec_hex_64.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split(None, 1)
                out[k] = v.strip()
    return out


def test_fullsize_algorithm1_equals_the_sequential_oracle(big):
    # every patch: phi and the entries bit for bit, and evaluations plus
    # pruned pairs equal to the comparisons of the oracle's sequential loop
    P, h = big
    g = _golden_alg1()
    phi, reps = h.assignment()
    st = h.stats()
    say("m_p", len(reps), "evals + pruned", st["crit_evals"] + st["crit_pruned"], "oracle", g["evals"])
    assert P.n_p == int(g["n_p"]) and len(reps) == int(g["m_p"])
    assert hashlib.sha256(np.asarray(phi, dtype="<i4").tobytes()).hexdigest() == g["phi_sha256"]
    assert hashlib.sha256(np.asarray(reps, dtype="<i4").tobytes()).hexdigest() == g["reps_sha256"]
    assert st["crit_evals"] + st["crit_pruned"] == int(g["evals"])


def test_fullsize_algorithm1_properties(big):
    P, h = big
    phi, reps = h.assignment()
    st = h.stats()
    say("m_p", st["m_p"], "evals", st["crit_evals"], "pruned", st["crit_pruned"])
    assert np.all(np.diff(reps) > 0)                 # entries in ascending patch id
    assert np.all(phi[reps] == np.arange(len(reps)))  # an entry's patch maps to itself
    rng = np.random.default_rng(1)
    X = {}

    def Xof(j):
        if j not in X:
            X[j] = O.factor_inverse(_tile(P, reps[j]))
        return X[j]
    # sampled patches: within eps of their entry, and no earlier entry matches
    for i in rng.choice(P.n_p, size=60, replace=False):
        A = _tile(P, i)
        j = int(phi[i])
        assert reps[j] <= i
        assert O.crit_spectral_x(A, Xof(j)) < EPS, i
        for jj in range(j):
            assert O.crit_spectral_x(A, Xof(jj)) >= EPS, (i, jj)
    # sampled entries: no earlier entry matches them
    for j in rng.choice(len(reps), size=20, replace=False):
        A = _tile(P, reps[j])
        for jj in range(j):
            assert O.crit_spectral_x(A, Xof(jj)) >= EPS, (j, jj)


def test_fullsize_apply_at_sampled_dofs(big):
    P, h = big
    phi, reps = h.assignment()
    r_np = gen.rhs(P.n, 11)
    r = torch.as_tensor(r_np).to(DEV)
    z_lp = torch.zeros_like(r)
    h.apply(r, z_lp)
    h64 = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=EPS, precision="fp64", deterministic=True)
    z64 = torch.zeros_like(r)
    h64.apply(r, z64)
    torch.cuda.synchronize()
    zl, zd = z_lp.cpu().numpy(), z64.cpu().numpy()
    # patches containing each dof
    order = np.argsort(P.dofs, kind="stable")
    patch_of = np.repeat(np.arange(P.n_p), np.diff(P.ptr))[order]
    start = np.searchsorted(P.dofs[order], np.arange(P.n + 1))
    cnt = np.diff(start)
    rng = np.random.default_rng(2)
    X, kappa = {}, {}
    errs = []
    for i in rng.choice(P.n, size=400, replace=False):
        zi = 0.0
        kmax = 1.0
        for k in patch_of[start[i]:start[i + 1]]:
            d = P.patch(k)
            j = int(phi[k])
            if j not in X:
                T = _tile(P, reps[j])
                X[j] = O.factor_inverse(T)
                kappa[j] = np.linalg.cond(T)
            kmax = max(kmax, kappa[j])
            a = int(np.flatnonzero(d == i)[0])
            zi += X[j][a] @ r_np[d]
        zi *= 1.0 / cnt[i]
        # the two sides invert the entries differently (Gauss-Jordan / LU):
        # they agree to a few units of kappa * u
        tol = max(1e-12, 8 * 12 * kmax * 2.2e-16) * np.abs(zd).max()
        errs.append(abs(zd[i] - zi) / np.abs(zd).max())
        assert abs(zd[i] - zi) <= tol, (i, zd[i], zi, kmax)
    say("fp64 apply at sampled dofs: largest error relative to max|z|", max(errs))
    rel = np.linalg.norm(zl - zd) / np.linalg.norm(zd)
    say("split-bf16 vs fp64 apply, relative 2-norm", rel)
    assert rel < 2e-4
    h64.close()
