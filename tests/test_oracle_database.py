"""Pins of the oracle's database construction (Algorithms 1 and 2)."""
import itertools
import os

import numpy as np
import pytest

import gen
import oracle as O


def test_alg1_q1_finds_nine_distinct_patches():
    P = gen.q1_poisson_2d(32)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    res = O.alg1_tolerance(t, 1e-8)
    assert len(res['reps']) == 9
    # append order equals ascending patch id
    assert np.all(np.diff(res['reps']) > 0)
    assert O.alg1_invariants_hold(lambda k: t[k], res['phi'], res['reps'], 1e-8, 'spectral',
                                  range(P.n_p))


@pytest.mark.parametrize("make", [lambda: gen.q2_hex_diffusion(4, sigma=0.0),
                                  lambda: gen.nedelec_hex(4, coeffs=(1, 1, 1, 1))])
def test_alg1_constant_coefficient_cube_gives_27(make):
    # constant coefficients on a cube: 8 corners, 12 edges, 6 faces, 1 interior
    P = make()
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    for crit, eps in [('spectral', 1e-8), ('l1', 1e-7)]:
        res = O.alg1_tolerance(t, eps, crit)
        assert len(res['reps']) == 27


def test_alg1_stokes_nine():
    P = gen.taylor_hood_stokes_2d(8)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    assert len(O.alg1_tolerance(t, 1e-8)['reps']) == 9


def test_alg1_first_match_semantics_hand_example():
    # d(B1,B0) = 0.2, d(A2,B0) = 0.1, d(A2,B1) = 1/12: at eps = 0.15 patch 2
    # matches both entries and takes the first, although B1 is closer
    B0 = np.diag([1.0, 1.0])
    B1 = np.diag([1.2, 1.0])
    A2 = np.diag([1.1, 1.0])
    res = O.alg1_tolerance([B0, B1, A2], eps=0.15)
    assert list(res['reps']) == [0, 1] and list(res['phi']) == [0, 1, 0]
    res = O.alg1_tolerance([B0, B1, A2], eps=0.09)
    # B1 does not match B0 (d = 0.2); A2 matches B1 (1/12 < 0.09) but not B0
    assert list(res['reps']) == [0, 1] and list(res['phi']) == [0, 1, 1]


def test_alg1_attains_brute_force_minimum_of_objective():
    # n_p = 7 patches in 3 identical classes; small beta: Eq.(4)'s minimum over
    # every database drawn from the patches (with the optimal phi) is attained
    rng = np.random.default_rng(11)
    classes = [rng.standard_normal((4, 4)) + 5 * np.eye(4) for _ in range(3)]
    labels = [0, 1, 0, 2, 1, 1, 0]
    tiles = [classes[c].copy() for c in labels]
    beta = 1e-3
    res = O.alg1_tolerance(tiles, 1e-8)
    L_alg1 = O.objective(tiles, res['X'], res['phi'], beta)
    Xall = [O.factor_inverse(t) for t in tiles]
    best = np.inf
    for m in range(1, len(tiles) + 1):
        for sub in itertools.combinations(range(len(tiles)), m):
            Xs = [Xall[s] for s in sub]
            d = np.array([[np.linalg.norm(np.eye(4) - A @ X, 2) ** 2 for X in Xs] for A in tiles])
            best = min(best, beta * m + d.min(axis=1).sum())
    assert abs(L_alg1 - best) < 1e-12
    assert len(res['reps']) == 3


def test_objective_is_permutation_invariant():
    rng = np.random.default_rng(1)
    tiles = [rng.standard_normal((3, 3)) + 4 * np.eye(3) for _ in range(6)]
    X = [O.factor_inverse(tiles[i]) for i in (0, 3)]
    phi = np.array([0, 0, 1, 1, 0, 1])
    a = O.objective(tiles, X, phi, 0.5)
    b = O.objective(tiles, X[::-1], 1 - phi, 0.5)
    assert abs(a - b) < 1e-12


def test_apportion_examples():
    assert O.apportion([900, 30, 30, 30, 10], 20) == [16, 1, 1, 1, 1]
    assert O.apportion([50, 50], 3) == [2, 1]
    assert O.apportion([10, 10, 10], 3) == [1, 1, 1]
    with pytest.raises(O.OracleError):
        O.apportion([5, 5, 5], 2)
    rng = np.random.default_rng(0)
    for _ in range(200):
        sizes = list(rng.integers(1, 500, size=int(rng.integers(1, 27))))
        m = int(rng.integers(len(sizes), sum(sizes) + 1))
        a = O.apportion(sizes, m)
        assert sum(a) == m and all(1 <= x <= s for x, s in zip(a, sizes))
        # roughly proportional: within one seat of the quota, except forced minimums
        for x, s in zip(a, sizes):
            q = m * s / sum(sizes)
            assert x <= np.ceil(q) + 1e-9 or x == 1


def test_splitmix64_is_invertible_state_walk():
    # the output mix is a bijection: undo it and recover seed + k * gamma
    def unmix(z):
        M = (1 << 64) - 1
        def unxs(v, s):
            x = v
            for _ in range(64 // s + 1):
                x = v ^ (x >> s)
            return x & M
        z = unxs(z, 31)
        z = (z * pow(0x94D049BB133111EB, -1, 1 << 64)) & M
        z = unxs(z, 27)
        z = (z * pow(0xBF58476D1CE4E5B9, -1, 1 << 64)) & M
        return unxs(z, 30)
    g = O.SplitMix64(12345)
    for k in range(1, 50):
        assert unmix(g.next()) == (12345 + k * 0x9E3779B97F4A7C15) % (1 << 64)


def test_splitmix64_published_streams():
    # the published first outputs for seeds 1234567 and 0 (tests/golden)
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")
    rows = [ln.split("#", 1)[0].split() for ln in open(path)]
    rows = [r for r in rows if r]
    assert len(rows) == 2
    for r in rows:
        vals = [int(v, 0) for v in r]
        g = O.SplitMix64(vals[0])
        assert [g.next() for _ in vals[1:]] == vals[1:]


def test_varmin_representative_identity():
    # member nearest the mean == argmin_m sum_k ||A_k - A_m||_F^2 (brute force)
    rng = np.random.default_rng(3)
    for _ in range(50):
        mats = [rng.standard_normal((3, 3)) for _ in range(int(rng.integers(2, 9)))]
        mean = np.mean(mats, axis=0)
        near = np.array([np.sum((A - mean) ** 2) for A in mats])
        pair = np.array([sum(np.sum((Ak - Am) ** 2) for Ak in mats) for Am in mats])
        # same minimiser; with two members both are exactly tied (rounding decides)
        band_near = set(np.flatnonzero(near <= near.min() * (1 + 1e-9)))
        band_pair = set(np.flatnonzero(pair <= pair.min() * (1 + 1e-9)))
        assert band_near == band_pair


@pytest.mark.parametrize("variant", ["spectral", "entrywise", "varmin"])
def test_kmeans_fixed_point_and_partition(variant):
    P = gen.q2_hex_diffusion(4, sigma=0.5, seed=4)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    res = O.kmeans(t, 30, variant=variant, seed=5)
    phi = res['phi']
    assert phi.min() >= 0
    assert len(res['B']) == 30
    keys = np.array([O.boundary_mask(x) for x in t])
    # every cluster holds one boundary key only
    for j in range(30):
        assert len(set(keys[phi == j])) <= 1
    # fixed point: at exit each patch sits in its tie band
    if all(res['converged']):
        for i in range(len(t)):
            grp = [j for j in range(30) if len(set(keys[phi == j]) | {keys[i]}) == 1 or j == phi[i]]
            same = [j for j in range(30) if np.any((phi == j)) and keys[phi == j][0] == keys[i]]
            d = [O.criterion('l1' if variant == 'entrywise' else 'spectral', t[i], res['B'][j],
                             res['X'][j]) for j in same]
            dmin = min(d)
            s = np.sum(np.abs(t[i])) if variant == 'entrywise' else 1.0
            assert O.criterion('l1' if variant == 'entrywise' else 'spectral', t[i],
                               res['B'][phi[i]], res['X'][phi[i]]) <= dmin * (1 + 1e-9) + 1e-9 * s


def test_bootstrap_from_identical_classes_converges_at_once():
    P = gen.q2_hex_diffusion(4, sigma=0.0)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    a1 = O.alg1_tolerance(t, 1e-8)
    res = O.kmeans(t, len(a1['reps']), variant='bootstrap', init_reps=a1['reps'])
    assert res['iters'] == [2] and all(res['converged'])
    assert np.array_equal(res['phi'], a1['phi'])


def test_kmeans_initial_draw_reproducible():
    P = gen.q1_poisson_2d(8)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    a = O.kmeans(t, 10, seed=9, max_iter=1)
    b = O.kmeans(t, 10, seed=9, max_iter=1)
    assert np.array_equal(a['rep_patch'], b['rep_patch'])
    c = O.kmeans(t, 10, seed=10, max_iter=1)
    assert not np.array_equal(a['rep_patch'], c['rep_patch'])


@pytest.mark.parametrize("variant,vals,centres", [
    # 1x1 patches: entrywise k-means is Lloyd's algorithm on the line
    ("entrywise", [1.0, 2.0, 3.0, 10.0, 11.0, 12.0], [2.0, 11.0]),
    # spectral distance |1 - a/b| of 1x1 patches: two clusters a decade apart
    ("spectral", [1.0, 1.1, 1.2, 100.0, 110.0, 120.0], [1.1, 110.0]),
])
def test_kmeans_two_separated_triples_from_every_draw(variant, vals, centres):
    # from any two distinct initial centres the passes end with the two triples
    # and their means as centres (worked by hand for every initial pair)
    tiles = [np.array([[v]]) for v in vals]
    seen = set()
    for seed in range(40):
        res = O.kmeans(tiles, 2, variant=variant, seed=seed, partition=False)
        seen.add(tuple(sorted(int(r) for r in res['rep_patch'] if r >= 0)))
        phi = res['phi']
        assert len(set(phi[:3])) == 1 and len(set(phi[3:])) == 1 and phi[0] != phi[3]
        got = sorted(float(b[0, 0]) for b in res['B'])
        assert np.allclose(got, centres, rtol=1e-14, atol=0)
        assert all(res['converged'])
    assert len(seen) <= 1      # centres became means, no patch representative left


def test_kmeans_groups_never_mix_sizes():
    rng = np.random.default_rng(2)
    tiles = [rng.standard_normal((p, p)) + 4 * np.eye(p) for p in (2, 3, 2, 3, 3, 2, 2)]
    g = O.partition_groups(tiles, partition=False)
    assert [k for k, _ in g] == [2, 3]
    assert [list(m) for _, m in g] == [[0, 2, 5, 6], [1, 3, 4]]
    res = O.kmeans(tiles, 3, variant="spectral", seed=1, partition=False)
    for j in range(3):
        sizes = {tiles[i].shape[0] for i in np.flatnonzero(res['phi'] == j)}
        assert len(sizes) <= 1


def test_alg1_mixed_sizes_runs_each_size_on_its_own():
    # interleaved sizes: the joint run equals the per-size runs, with entries
    # numbered in one ascending-id order
    P = gen.uneven_stokes_batch(n_sys=3, nmin=2, nmax=4)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    res = O.alg1_tolerance(t, 1e-8)
    sizes = np.array([x.shape[0] for x in t])
    assert len(set(sizes)) > 1
    rep_of = {}
    for s in sorted(set(sizes)):
        ids = np.flatnonzero(sizes == s)
        r = O.alg1_tolerance([t[i] for i in ids], 1e-8)
        for q, i in enumerate(ids):
            rep_of[int(i)] = int(ids[r["reps"][r["phi"][q]]])
    assert sorted(set(rep_of.values())) == list(res["reps"])
    assert all(int(res["reps"][res["phi"][i]]) == rep_of[i] for i in range(len(t)))


def _scalars(vals):
    return [np.array([[float(v)]]) for v in vals]


def test_alg1_closest_hand_example():
    # 1 x 1 patches: d(a, b) = |1 - a/b|.  eps = 0.3: 1.3 is 0.3 from 1.0 (not
    # below eps) and becomes an entry; 1.25 is 0.25 from entry 0 and 0.0385
    # from entry 1: first match takes entry 0, closest match entry 1
    tiles = _scalars([1.0, 1.3, 1.25])
    first = O.alg1_tolerance(tiles, 0.3)
    close = O.alg1_closest(tiles, 0.3)
    assert first["phi"].tolist() == [0, 1, 0]
    assert close["phi"].tolist() == [0, 1, 1]
    assert close["reps"].tolist() == [0, 1] == first["reps"].tolist()
    assert close["evals"] == 0 + 1 + 2
    assert abs(close["dmin"][2] - (1 - 1.25 / 1.3)) < 1e-15


def test_alg1_closest_only_sees_entries_created_before():
    # entry 1 (1.5) appears after patch 1 (1.2): patch 1 can only take entry 0
    tiles = _scalars([1.0, 1.2, 1.5, 1.45])
    close = O.alg1_closest(tiles, 0.3)
    assert close["reps"].tolist() == [0, 2]
    assert close["phi"].tolist() == [0, 0, 1, 1]


def test_alg1_closest_tie_band_takes_lowest_entry():
    # entries 1.0 and 1.25 (d = 0.25 >= eps = 0.2 between them); a patch at
    # 10/9 is equally far from both (d = 1/9); just above 10/9 entry 1 is
    # closer by 1.6e-10, inside the band 1e-9 (1 + d) -> lowest entry, 0
    a = 1.1111111112
    d0, d1 = a - 1.0, 1.0 - a / 1.25
    assert 0 < d0 - d1 < 1e-9
    close = O.alg1_closest(_scalars([1.0, 1.25, a]), 0.2)
    assert close["phi"].tolist() == [0, 1, 0]
    # outside the band the strictly closer entry wins
    close = O.alg1_closest(_scalars([1.0, 1.25, 1.112]), 0.2)
    assert close["phi"].tolist() == [0, 1, 1]


@pytest.mark.parametrize("crit,eps", [("spectral", 0.99), ("l1", 50.0), ("fro", 5.0)])
def test_alg1_closest_keeps_algorithm_1_database(crit, eps):
    # a patch becomes an entry iff no earlier entry lies within eps, whichever
    # would match: the database does not depend on the matching rule
    P = gen.q2_hex_diffusion(5)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    first = O.alg1_tolerance(tiles, eps, crit)
    close = O.alg1_closest(tiles, eps, crit)
    assert np.array_equal(first["reps"], close["reps"])
    assert len(first["reps"]) < len(tiles)
    # every patch lies within eps of its entry, and no other earlier entry is
    # closer by more than the tie band (brute force over every pair)
    X = {j: O.factor_inverse(tiles[r]) for j, r in enumerate(close["reps"])}
    for i, t in enumerate(tiles):
        if i in set(close["reps"].tolist()):
            continue
        dist = {j: O.criterion(crit, t, tiles[r], X[j]) for j, r in enumerate(close["reps"]) if r < i}
        dj = dist[int(close["phi"][i])]
        assert dj < eps
        assert dj <= min(dist.values()) * (1 + 1e-9) + 1e-9 * {"spectral": 1.0, "l1": np.abs(t).sum(),
                                                              "fro": np.linalg.norm(t)}[crit]
    assert (close["phi"] != first["phi"]).any()


def test_compressibility_ratio():
    assert O.compressibility(3600, 36) == 0.99
    assert O.compressibility(8000, 27) == pytest.approx(0.996625)


def test_alg1_reuse_on_an_unchanged_system_keeps_everything():
    P = gen.q2_hex_diffusion(4)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    prev = O.alg1_tolerance(tiles, 0.5)
    r = O.alg1_reuse(tiles, 0.5, "spectral", prev["phi"], prev["reps"])
    m = len(prev["reps"])
    assert np.array_equal(r["phi"], prev["phi"]) and np.array_equal(r["reps"], prev["reps"])
    assert r["kept"] == len(tiles) - m and r["rescanned"] == 0 and r["appended"] == 0
    assert r["evals"] == len(tiles) - m          # one comparison per patch that is not an entry


def test_alg1_reuse_hand_example():
    # previous system: entries 1.0 and 1.3 (d = 0.3 is not below eps), patch 2
    # (1.25) on entry 0; next systems move patch 2
    prev = O.alg1_tolerance(_scalars([1.0, 1.3, 1.25]), 0.3)
    assert prev["phi"].tolist() == [0, 1, 0]
    r = O.alg1_reuse(_scalars([1.0, 1.3, 1.6]), 0.3, "spectral", prev["phi"], prev["reps"])
    # d(1.6, 1.0) = 0.6 >= eps: rescan; d(1.6, 1.3) = 0.2308 < eps: entry 1
    assert r["phi"].tolist() == [0, 1, 1] and r["rescanned"] == 1 and r["appended"] == 0
    r = O.alg1_reuse(_scalars([1.0, 1.3, 2.0]), 0.3, "spectral", prev["phi"], prev["reps"])
    assert r["phi"].tolist() == [0, 1, 2] and r["reps"].tolist() == [0, 1, 2] and r["appended"] == 1
    # the previous entries stay entries even when they now match each other
    r = O.alg1_reuse(_scalars([1.0, 1.1, 1.05]), 0.3, "spectral", prev["phi"], prev["reps"])
    assert r["reps"].tolist() == [0, 1] and r["phi"].tolist() == [0, 1, 0]


def test_alg1_reuse_on_a_perturbed_system_keeps_the_tolerance():
    P = gen.q2_hex_diffusion(5)
    P2 = gen.q2_hex_diffusion(5, kfield=P.meta["k"] * np.exp(0.05 * np.random.default_rng(7).standard_normal(125)))
    t1 = O.patch_tiles(P.A, P.ptr, P.dofs)
    t2 = O.patch_tiles(P2.A, P2.ptr, P2.dofs)
    prev = O.alg1_tolerance(t1, 0.99)
    r = O.alg1_reuse(t2, 0.99, "spectral", prev["phi"], prev["reps"])
    assert r["kept"] > 0 and r["rescanned"] + r["appended"] > 0
    X = {j: O.factor_inverse(t2[e]) for j, e in enumerate(r["reps"])}
    for i, t in enumerate(t2):
        assert O.crit_spectral_x(t, X[int(r["phi"][i])]) < 0.99
    assert r["evals"] < O.alg1_tolerance(t2, 0.99)["evals"]


@pytest.mark.parametrize("variant", ["spectral", "varmin", "entrywise"])
def test_kmeans_warm_start_from_a_fixed_point_takes_one_pass(variant):
    P = gen.q2_hex_diffusion(5)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    cold = O.kmeans(tiles, 40, variant=variant)
    assert all(cold["converged"])
    warm = O.kmeans(tiles, 40, variant=variant, init_phi=cold["phi"])
    assert np.array_equal(warm["phi"], cold["phi"])
    assert max(warm["iters"]) == 1
    for a, b in zip(warm["B"], cold["B"]):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
