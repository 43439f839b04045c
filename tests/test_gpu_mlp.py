"""GPU parity of the learned entry predictor and of Algorithm 1 with
predictions, through the C ABI.

Bars: features within FP32 rounding of the oracle's FP64 values; loss and
gradients within 1e-5 (FP32 kernels) or 2e-2 (FP16 MFMA operands) of the
oracle's FP64 analytic backward, relative to each parameter block's largest
entry; top-k bit-exact against the oracle's selection on the same logits;
the patch map and database of the setup bit-exact against the oracle's
sequential definition fed with the GPU's training set and candidate lists
(the network is a heuristic input, like a random draw; the exact criterion
decides every assignment).
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
M = O.mlp


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dt(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def pack(P):
    return np.concatenate([P[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unpack(v, F, H, C):
    out, o = {}, 0
    for k, shp in (("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, C)), ("b3", (C,))):
        n = int(np.prod(shp))
        out[k] = v[o:o + n].reshape(shp)
        o += n
    return out


def _net(seed, rows=300, F=82, H=64, C=37, keyed=True):
    rng = np.random.default_rng(seed)
    P = M.init_params(F, H, C, seed=seed)
    for k in ("b1", "b2", "b3"):
        P[k] = 0.1 * rng.standard_normal(P[k].shape)
    # keep the inputs exactly representable in FP32 so both sides see them
    P = {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}
    X = rng.standard_normal((rows, F)).astype(np.float32).astype(np.float64)
    ckey = rng.integers(0, 3, size=C).astype(np.int32) if keyed else None
    if keyed:
        ckey[:3] = [0, 1, 2]
        rkey = rng.integers(0, 3, size=rows).astype(np.int32)
        y = np.array([rng.choice(np.flatnonzero(ckey == r)) for r in rkey], dtype=np.int32)
        allowed = rkey[:, None] == ckey[None, :]
    else:
        rkey, allowed = None, None
        y = rng.integers(0, C, size=rows).astype(np.int32)
    return P, X, y, rkey, ckey, allowed


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp16", 2e-2)])
@pytest.mark.parametrize("keyed", [False, True])
def test_loss_and_gradients_match_oracle(precision, tol, keyed):
    F, H, C = 82, 64, 37
    P, X, y, rkey, ckey, allowed = _net(1, F=F, H=H, C=C, keyed=keyed)
    loss_o, g_o = M.loss_and_grads(P, X, y, allowed)
    params = dt(pack(P), torch.float32)
    grads = torch.full_like(params, np.nan)
    loss = pr.pr_mlp_loss_grad(precision, dt(X, torch.float32), dt(y, torch.int32), params, grads, F, H, C,
                               None if rkey is None else dt(rkey, torch.int32),
                               None if ckey is None else dt(ckey, torch.int32))
    g = unpack(grads.cpu().numpy().astype(np.float64), F, H, C)
    say(precision, "keyed", keyed, "loss", loss, "oracle", loss_o)
    assert abs(loss - loss_o) <= tol * abs(loss_o)
    if precision == "fp16":
        # FP16 operands move pre-activations by ~1e-3, enough to flip a few
        # ReLU masks against the exact network; the bar is therefore against
        # the oracle with FP16-rounded operands (11 significant bits), and
        # against the exact network only where no mask enters (W3, b3)
        loss_e, g_e = M.loss_and_grads(P, X, y, allowed, operand_bits=11)
        assert abs(loss - loss_e) <= 2e-4 * abs(loss_e)
        for k in g_e:
            err = np.abs(g[k] - g_e[k]).max() / np.abs(g_e[k]).max()
            say("  ", k, "rel err vs FP16-operand oracle %.2e" % err)
            assert err <= 2e-3, (precision, k, err)
        names = ("W3", "b3")
    else:
        names = tuple(g_o)
    for k in names:
        err = np.abs(g[k] - g_o[k]).max() / np.abs(g_o[k]).max()
        say("  ", k, "rel err %.2e" % err)
        assert err <= tol, (precision, k, err)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp16", 2e-2)])
def test_forward_and_topk(precision, tol):
    F, H, C, rows, k = 82, 64, 300, 1000, 8
    P, X, y, rkey, ckey, allowed = _net(2, rows=rows, F=F, H=H, C=C, keyed=True)
    logits = torch.empty((rows, C), dtype=torch.float32, device=DEV)
    topk = torch.empty((rows, k), dtype=torch.int32, device=DEV)
    pr.pr_mlp_predict(precision, dt(X, torch.float32), dt(pack(P), torch.float32), F, H, C, k, logits, topk,
                      dt(rkey, torch.int32), dt(ckey, torch.int32))
    L = logits.cpu().numpy().astype(np.float64)
    Lo = M.forward(P, X)["logits"]
    assert np.abs(L - Lo).max() <= tol * np.abs(Lo).max()
    # selection is integer work: exact on the same logits, -1 past the allowed classes
    sel = M.topk(L, k, allowed)
    nallowed = allowed.sum(axis=1)
    for r in range(rows):
        want = [int(c) if t < nallowed[r] else -1 for t, c in enumerate(sel[r])]
        assert topk[r].tolist() == want, r


SETUP_CASES = {
    # piecewise-constant materials: tile classes repeat exactly
    "nedelec_8_spec": (lambda: gen.nedelec_hex(8), dict(eps=1e-8), {}),
    # lognormal coefficient, loose tolerance: every tile differs
    "q2hex_6_loose": (lambda: gen.q2_hex_diffusion(6), dict(eps=0.99), dict(mlp_train_frac=0.3)),
    "q2hex_const_5_l1": (lambda: gen.q2_hex_diffusion(5, sigma=0.0), dict(eps=1e-7, criterion="l1"), {}),
    "stokes_batch_5": (lambda: gen.uneven_stokes_batch(n_sys=5, nmin=2, nmax=6), dict(eps=1e-8),
                       dict(mlp_train_frac=0.2)),
    "nedelec_8_fp32": (lambda: gen.nedelec_hex(8), dict(eps=1e-8), dict(mlp_precision="fp32", mlp_topk=1)),
}


@pytest.mark.parametrize("case", list(SETUP_CASES))
def test_setup_with_predictions_bit_exact(case):
    make, a1, mk = SETUP_CASES[case]
    say("mlp setup", case)
    P = make()
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    crit = a1.get("criterion", "spectral")
    h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", mlp=True, **a1, **mk)
    st = h.stats()
    train, cand = h.mlp_candidates()
    phi, reps = h.assignment()
    # features against the oracle's
    Fo = M.features(tiles, int(np.diff(P.ptr).max()))
    Fg = h.mlp_features()
    assert np.abs(Fg - Fo).max() <= 2e-6 * max(1.0, np.abs(Fo).max()), case
    res = O.alg1_with_predictions(tiles, a1["eps"], crit, train, [list(c) for c in cand])
    say(case, "n_p", P.n_p, "train", len(train), "classes", st["mlp_classes"], "accepted", st["mlp_accepted"],
        "scanned", st["mlp_scanned"], "fallback", st["mlp_fallback"], "m_p", st["m_p"],
        "train acc %.3f loss %.3f" % (st["mlp_train_acc"], st["mlp_loss"]))
    assert np.array_equal(reps, res["reps"]), case
    assert np.array_equal(phi, res["phi"]), case
    assert st["mlp_classes"] == res["n_train_entries"]
    # the library counts scan matches on training entries; the rest of the
    # scanned patches matched entries that Algorithm 1 appended
    assert st["mlp_accepted"] == res["accepted"] and st["mlp_scanned"] == res["scanned_train"]
    assert st["mlp_fallback"] == res["scanned"] - res["scanned_train"] + res["appended"]
    # the tolerance holds for every patch (exact criterion as the judge)
    X = {int(r): O.factor_inverse(tiles[r]) for r in reps}
    for i in range(0, P.n_p, max(1, P.n_p // 200)):
        r = int(reps[phi[i]])
        d = O.criterion(crit, tiles[i], tiles[r], X[r])
        assert d < a1["eps"], (case, i, d)
    h.close()


def test_trained_network_against_pruned_algorithm_1():
    """What the network costs and buys on a fresh system, against the
    library's own default Algorithm 1 (with the certified pruning), on
    repeated tile classes (the structure of the 64^3 edge-element workload):
    most patches are placed by their first prediction, the database and the
    solve are unchanged, but the pruned scan already needs fewer criterion
    evaluations than the predictions, and the training comes on top, so a
    network trained for one setup does not pay for itself.  Reusing a trained
    network on the next system of a sequence is where it can."""
    P = gen.nedelec_hex(12)
    plain = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=1e-8, max_iters=300)
    learned = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=1e-8, mlp=True, max_iters=300)
    sp, sl = plain.stats(), learned.stats()
    say("pruned Algorithm 1: evals", sp["crit_evals"], "setup s %.4f" % sp["t_total"],
        "| with predictions: evals", sl["crit_evals"], "setup s %.4f" % sl["t_total"],
        "training s %.4f" % sl["t_mlp_train"], "accepted", sl["mlp_accepted"], "of",
        P.n_p - sl["mlp_train"], "train acc %.3f" % sl["mlp_train_acc"])
    assert sl["mlp_accepted"] >= 0.5 * (P.n_p - sl["mlp_train"])
    assert sl["m_p"] == sp["m_p"]
    # measured: the predictor loses on both counts on a fresh system
    assert sp["crit_evals"] < sl["crit_evals"]
    assert sp["t_total"] < sl["t_total"]
    # GMRES(30) with one-level cell patches does not reach 1e-8 on this H(curl)
    # problem; equal iteration counts must give the same residual
    b = torch.as_tensor(gen.rhs(P.n, 0)).to(DEV)
    rel = []
    for h in (plain, learned):
        x = torch.zeros_like(b)
        h.solve(b, x, 1e-8)
        rel.append(h.solve_info()["relres"])
        h.close()
    say("relres after 300 iterations plain / learned", rel)
    assert abs(rel[1] - rel[0]) <= 1e-6 * rel[0]


def test_trained_network_solve_iterations_match():
    P = gen.q1_poisson_2d(64)
    its = []
    for mlp in (False, True):
        h = pr.PatchRelax(P.A, P.ptr, P.dofs, algo="tolerance", eps=1e-8, mlp=mlp)
        st = h.stats()
        b = torch.as_tensor(gen.rhs(P.n, 0)).to(DEV)
        x = torch.zeros_like(b)
        assert h.solve(b, x, 1e-8) == pr.PR_OK
        its.append(h.solve_info()["iters"])
        say("mlp", mlp, "m_p", st["m_p"], "evals", st["crit_evals"], "pruned", st["crit_pruned"],
            "accepted", st["mlp_accepted"], "iters", its[-1])
        h.close()
    assert abs(its[1] - its[0]) <= 1


def test_predictor_parameter_errors():
    P = gen.q1_poisson_2d(8)
    for kw in (dict(mlp_topk=9), dict(mlp_train_frac=0.0), dict(mlp_precision="bf16"), dict(algo="full")):
        args = dict(algo="tolerance", mlp=True)
        args.update(kw)
        with pytest.raises(pr.PatchRelaxError) as e:
            pr.PatchRelax(P.A, P.ptr, P.dofs, **args)
        assert e.value.code == pr.PR_ERR_INVALID_ARG
