"""Learned predictor of a patch's database entry, in plain FP64 NumPy.

The paper's closing remarks on clustering (end of Section 3.2, and Section 5)
point to neural networks as a way to cut the cost of building the database.
This module defines the predictor used for that: cheap invariants of a patch
matrix go through a small multilayer perceptron whose classes are the entries
of a database built on a training subset; the exact criterion still decides
every assignment (``database.alg1_with_predictions``).

Features of a p x p patch matrix A, padded to width pmax (F = 3 pmax + 1):
  m = mean_a |A_aa| (1 when it is 0),
  A_aa / m (pmax slots), sum_b |A_ab| / m (pmax slots),
  1 if row a has exactly one nonzero else 0 (pmax slots), log m.
Standardisation: per feature, (x - mean) / std over the training rows
(population std; a zero std counts as 1).

Network: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), l = h2 W3 + b3.  Loss:
the mean over rows of logsumexp(l_i) - l_i[y_i], the sum running over the
classes allowed for row i (entries of the row's patch size).  The backward
pass is the chain rule written out; Adam (Kingma and Ba, 2015) updates.

Test infrastructure only (see the package docstring).  Pinned by central
finite differences of the loss and by closed-form features of the Q1 tile.
"""
from __future__ import annotations

import numpy as np


def features(tiles, pmax=None):
    """Rows of patch invariants (module docstring), FP64."""
    if pmax is None:
        pmax = max(t.shape[0] for t in tiles)
    F = 3 * pmax + 1
    out = np.zeros((len(tiles), F))
    for k, A in enumerate(tiles):
        p = A.shape[0]
        d = np.diag(A)
        m = float(np.mean(np.abs(d)))
        if m == 0.0:
            m = 1.0
        out[k, :p] = d / m
        out[k, pmax:pmax + p] = np.sum(np.abs(A), axis=1) / m
        out[k, 2 * pmax:2 * pmax + p] = (np.count_nonzero(A, axis=1) == 1).astype(float)
        out[k, 3 * pmax] = np.log(m)
    return out


def standardize(X, rows):
    """Per-feature mean and std over ``rows`` (population std, 0 -> 1)."""
    mu = X[rows].mean(axis=0)
    sd = X[rows].std(axis=0)
    sd[sd == 0.0] = 1.0
    return mu, sd


def init_params(F, H, C, seed=0):
    """He-scaled normal weights, zero biases (any initialisation will do for
    the gradient pins; the library draws its own)."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((F, H)) * np.sqrt(2.0 / F), "b1": np.zeros(H),
        "W2": rng.standard_normal((H, H)) * np.sqrt(2.0 / H), "b2": np.zeros(H),
        "W3": rng.standard_normal((H, C)) * np.sqrt(2.0 / H), "b3": np.zeros(C),
    }


def round_sig(a, bits):
    """Round to ``bits`` significant bits, to nearest with ties to even, with
    no exponent limit: the significand rounding of a narrow float format
    without its range (FP16 has 11 bits)."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)
    return np.ldexp(np.round(m * 2.0 ** bits) / 2.0 ** bits, e)


def _mm(A, B, rnd):
    return rnd(A) @ rnd(B)


def forward(P, X, operand_bits=None):
    """Forward pass; with operand_bits every factor of every matrix product
    is first rounded to that many significant bits (reduced-precision
    operands, exact sums)."""
    rnd = (lambda a: a) if operand_bits is None else (lambda a: round_sig(a, operand_bits))
    z1 = _mm(X, P["W1"], rnd) + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = _mm(h1, P["W2"], rnd) + P["b2"]
    h2 = np.maximum(z2, 0.0)
    logits = _mm(h2, P["W3"], rnd) + P["b3"]
    return dict(X=X, h1=h1, h2=h2, logits=logits)


def loss_and_grads(P, X, y, allowed=None, operand_bits=None):
    """Mean cross-entropy over the rows and its gradient for every parameter.

    allowed: optional boolean [rows, classes]; classes outside it take no
    probability (their logits are dropped from the log-sum-exp).
    operand_bits: as in ``forward``, for every product of the backward pass too.
    """
    rnd = (lambda a: a) if operand_bits is None else (lambda a: round_sig(a, operand_bits))
    c = forward(P, X, operand_bits)
    L = c["logits"].copy()
    if allowed is not None:
        L[~allowed] = -np.inf
    mx = L.max(axis=1, keepdims=True)
    e = np.exp(L - mx)
    s = e.sum(axis=1, keepdims=True)
    B = X.shape[0]
    rows = np.arange(B)
    loss = float(np.mean(np.log(s[:, 0]) + mx[:, 0] - L[rows, y]))
    G3 = e / s
    G3[rows, y] -= 1.0
    G3 /= B
    g = {"W3": _mm(c["h2"].T, G3, rnd), "b3": G3.sum(axis=0)}
    G2 = _mm(G3, P["W3"].T, rnd) * (c["h2"] > 0.0)
    g["W2"] = _mm(c["h1"].T, G2, rnd)
    g["b2"] = G2.sum(axis=0)
    G1 = _mm(G2, P["W2"].T, rnd) * (c["h1"] > 0.0)
    g["W1"] = _mm(X.T, G1, rnd)
    g["b1"] = G1.sum(axis=0)
    return loss, g


def adam_step(P, g, state, t, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); ``state`` holds m and v per name."""
    for k in P:
        m = state.setdefault("m" + k, np.zeros_like(P[k]))
        v = state.setdefault("v" + k, np.zeros_like(P[k]))
        m[...] = b1 * m + (1.0 - b1) * g[k]
        v[...] = b2 * v + (1.0 - b2) * g[k] * g[k]
        mh = m / (1.0 - b1 ** t)
        vh = v / (1.0 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P


def topk(logits, k, allowed=None):
    """Indices of the k largest logits per row, largest first, lower index
    first on equal values."""
    L = logits.copy()
    if allowed is not None:
        L[~allowed] = -np.inf
    order = np.lexsort((np.broadcast_to(np.arange(L.shape[1]), L.shape), -L), axis=1)
    return order[:, :k]
