"""Pins of the oracle's learned predictor and of Algorithm 1 with predictions."""
import numpy as np
import pytest

import gen
import oracle as O

M = O.mlp


def _rand_problem(seed=0, B=7, F=10, H=6, C=5):
    rng = np.random.default_rng(seed)
    P = M.init_params(F, H, C, seed=seed + 1)
    for k in ("b1", "b2", "b3"):
        P[k] = 0.1 * rng.standard_normal(P[k].shape)
    X = rng.standard_normal((B, F))
    y = rng.integers(0, C, size=B)
    allowed = rng.random((B, C)) < 0.8
    allowed[np.arange(B), y] = True
    return P, X, y, allowed


@pytest.mark.parametrize("masked", [False, True])
def test_gradients_match_central_differences(masked):
    P, X, y, allowed = _rand_problem()
    al = allowed if masked else None
    loss, g = M.loss_and_grads(P, X, y, al)
    h = 1e-6
    for name in P:
        num = np.zeros_like(P[name])
        it = np.nditer(P[name], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name][idx] += h
            Pm[name][idx] -= h
            num[idx] = (M.loss_and_grads(Pp, X, y, al)[0] - M.loss_and_grads(Pm, X, y, al)[0]) / (2 * h)
        scale = max(np.abs(g[name]).max(), 1e-3)
        assert np.abs(num - g[name]).max() <= 1e-7 * scale + 1e-9, name


def test_loss_of_zero_network_is_log_class_count():
    P, X, y, allowed = _rand_problem()
    for k in P:
        P[k] = np.zeros_like(P[k])
    loss, g = M.loss_and_grads(P, X, y, allowed)
    assert abs(loss - np.mean(np.log(allowed.sum(axis=1)))) < 1e-14
    loss, _ = M.loss_and_grads(P, X, y)
    assert abs(loss - np.log(P["b3"].shape[0])) < 1e-14


def test_features_of_q1_tiles_closed_form():
    P = gen.q1_poisson_2d(8)
    t = O.patch_tiles(P.A, P.ptr, P.dofs)
    k = 3 + 8 * 4                      # an interior cell: tile 3I - J/3
    f = M.features([t[k]], 4)[0]
    assert np.allclose(f[:4], 1.0, rtol=0, atol=1e-15)
    assert np.allclose(f[4:8], 11.0 / 8.0, rtol=0, atol=1e-15)
    assert np.all(f[8:12] == 0.0)
    assert abs(f[12] - np.log(8.0 / 3.0)) < 1e-15
    # corner cell: three identity rows and the interior node's row, which keeps
    # only its diagonal 8/3: every row is single-entry, mean |diag| = 17/12
    f0 = M.features([t[0]], 5)[0]
    assert np.all(f0[10:14] == 1.0) and f0[14] == 0.0     # padded slot stays 0
    assert abs(f0[15] - np.log(17.0 / 12.0)) < 1e-15
    assert sorted(f0[:4] * 17.0 / 12.0) == pytest.approx([1, 1, 1, 8.0 / 3.0], abs=1e-15)


def test_adam_first_step_is_signed_learning_rate():
    P, X, y, allowed = _rand_problem(3)
    _, g = M.loss_and_grads(P, X, y)
    P0 = {k: v.copy() for k, v in P.items()}
    M.adam_step(P, g, {}, 1, lr=1e-3)
    for k in P:
        expect = P0[k] - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(P[k], expect, rtol=0, atol=1e-15)


def test_topk_orders_by_value_then_index():
    L = np.array([[0.5, 2.0, 2.0, -1.0, 3.0]])
    assert M.topk(L, 3).tolist() == [[4, 1, 2]]
    allowed = np.array([[True, False, True, True, False]])
    assert M.topk(L, 2, allowed).tolist() == [[2, 0]]


def _tiles(make):
    P = make()
    return O.patch_tiles(P.A, P.ptr, P.dofs)


def test_predictions_reduce_to_alg1_on_a_prefix():
    t = _tiles(lambda: gen.q2_hex_diffusion(5, sigma=0.0))    # 27 classes
    n = len(t)
    ref = O.alg1_tolerance(t, 1e-8)
    none = [[] for _ in range(n)]
    for cut in (0, 1, n // 3, n):
        r = O.alg1_with_predictions(t, 1e-8, "spectral", range(cut), none)
        assert np.array_equal(r["phi"], ref["phi"]) and np.array_equal(r["reps"], ref["reps"])
    # a perfect predictor (the true first match) keeps the result and accepts
    # every patch whose entry comes from the training prefix
    cut = n // 2
    n0 = int(np.sum(ref["reps"] < cut))
    cand = [[int(ref["phi"][i])] if ref["phi"][i] < n0 else [] for i in range(n)]
    r = O.alg1_with_predictions(t, 1e-8, "spectral", range(cut), cand)
    assert np.array_equal(r["phi"], ref["phi"])
    assert r["accepted"] == sum(1 for i in range(cut, n) if ref["phi"][i] < n0)
    assert r["evals"] < ref["evals"]


def test_predictions_keep_the_tolerance_invariant():
    t = _tiles(lambda: gen.q2_hex_diffusion(4))
    n = len(t)
    rng = np.random.default_rng(0)
    train = np.sort(rng.choice(n, size=10, replace=False))
    # an arbitrary (bad) predictor: the result must still honour eps
    cand = [list(rng.integers(0, 5, size=3)) for _ in range(n)]
    eps = 0.9
    r = O.alg1_with_predictions(t, eps, "spectral", train, cand)
    X = [O.factor_inverse(t[q]) for q in r["reps"]]
    for i in range(n):
        assert O.crit_spectral_x(t[i], X[r["phi"][i]]) < eps
    assert r["accepted"] + r["scanned"] + r["appended"] == n - len(train)
    # entries are the training entries followed by appended patches, ascending
    assert np.all(np.diff(r["reps"][r["n_train_entries"]:]) > 0)


def test_round_sig_is_ieee_half_rounding_in_range():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(20000) * 10.0 ** rng.uniform(-4, 4, 20000)
    x = x[(np.abs(x) >= 2.0 ** -14) & (np.abs(x) <= 60000)]
    assert np.array_equal(M.round_sig(x, 11), x.astype(np.float16).astype(np.float64))
    # ties go to even
    assert M.round_sig(1.0 + 2.0 ** -11, 11) == 1.0
    assert M.round_sig(1.0 + 3 * 2.0 ** -11, 11) == 1.0 + 2 * 2.0 ** -10
    # no range: far below FP16's smallest normal the significand still has 11 bits
    assert M.round_sig(3.0e-9, 11) == np.ldexp(np.round(np.frexp(3.0e-9)[0] * 2048) / 2048, np.frexp(3.0e-9)[1])


def test_operand_rounding_changes_only_the_products():
    P, X, y, allowed = _rand_problem(4)
    l0, g0 = M.loss_and_grads(P, X, y, allowed)
    l1, g1 = M.loss_and_grads(P, X, y, allowed, operand_bits=53)
    assert l0 == l1 and all(np.array_equal(g0[k], g1[k]) for k in g0)
    l2, g2 = M.loss_and_grads(P, X, y, allowed, operand_bits=11)
    assert abs(l2 - l0) < 1e-2 * abs(l0) and abs(l2 - l0) > 0
