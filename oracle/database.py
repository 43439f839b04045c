"""Construction of the inverse database and the patch map phi (Section 3).

* ``alg1_tolerance``: Algorithm 1 (patch tolerance construction) from its
  definition: each patch, in ascending id, takes the earliest entry within
  the tolerance or becomes a new entry.
* ``kmeans``: Algorithm 2 (spectral clustering construction) and its variants
  listed in Section 3.2 (entrywise k-means, spectral k-means,
  variance-minimising clustering, bootstrapping), with the boundary
  partitioning and proportional apportionment of Section 3.2.

Readings taken where the paper is silent (each also listed in the design notes):
* indices are 0-based; database entries are numbered in append order;
* comparisons against the tolerance are strict (d < eps), as printed;
* Algorithm 2's initial ``randperm(n_p, m_p)`` draws m_p distinct patches as
  initial representatives; the draw is a partial Fisher-Yates shuffle driven by
  SplitMix64 so that any implementation can reproduce it bit for bit;
* argmin ties: a band around the minimum, d_j <= d_min (1 + tie) + tie s_i,
  with s_i = 1 for the spectral distance (a dimensionless quantity) and
  s_i = sum |A_i| for the entrywise l1 distance; the absolute term makes
  distances at rounding level (a patch equal to a centre up to rounding) tie
  instead of being ordered by rounding noise; the current assignment is kept
  if it lies in the band, else the lowest index in it;
* an empty cluster keeps its previous centre;
* the loop stops when no assignment changes or after max_iter passes; the
  final database is the one used in the last assignment pass;
* "the member which minimises the in-cluster variance" is the member whose
  matrix is nearest (Frobenius) to the entrywise cluster mean, which equals
  argmin_m sum_k ||A_k - A_m||_F^2; members whose squared distance lies
  within delta_min (1 + tie) + tie^2 ||mean||_F^2 count as tied and the
  lowest patch id wins (a two-member cluster is always an exact tie);
* apportionment: largest-remainder method in exact integer arithmetic, with
  at least one cluster per non-empty group and at most the group size.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .criterion import crit_spectral_x, crit_l1, crit_fro
from .patch import OracleError, factor_inverse, boundary_mask

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood 2014): state += golden gamma, then two
    xor-shift-multiply rounds and a final xor-shift; arithmetic mod 2^64."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)


def _dist(crit, Ai, Bj, Xj):
    if crit == "spectral":
        return crit_spectral_x(Ai, Xj)
    if crit == "l1":
        return crit_l1(Ai, Bj)
    if crit == "fro":
        return crit_fro(Ai, Bj)
    raise ValueError(crit)


def alg1_tolerance(tiles, eps, crit="spectral"):
    """Algorithm 1: greedy tolerance construction of the database and phi.

    Definition: patch i is mapped to the earliest database entry of its size
    (entries numbered in the order they were created) whose criterion value
    against it is below eps; a patch with no such entry creates the next
    entry, its own inverse, and is mapped to it.  Patches are taken in
    ascending id.  Entries of another patch size are no candidates (the
    criterion is defined for equal sizes; remark in Section 2), so with
    several sizes each size runs Algorithm 1 on its own while entries keep one
    numbering.  The criterion is evaluated entry by entry up to the first
    value below eps, so ``evals`` is the number of comparisons the greedy
    construction makes.
    Returns dict(phi, reps, X, evals, margin): reps are the patch ids whose
    inverses form the database and margin is min |d - eps| / eps over every
    value computed.
    """
    reps, X = [], []
    phi = np.zeros(len(tiles), dtype=np.int64)
    seen = []                                   # every criterion value computed

    def d(i, j):
        v = _dist(crit, tiles[i], tiles[reps[j]], X[j])
        seen.append(v)
        return v

    for i, Ai in enumerate(tiles):
        same_size = (j for j in range(len(reps)) if tiles[reps[j]].shape == Ai.shape)
        first = next((j for j in same_size if d(i, j) < eps), None)
        if first is None:
            reps.append(i)
            X.append(factor_inverse(Ai))
            first = len(reps) - 1
        phi[i] = first
    margin = np.inf
    if seen and eps > 0:
        margin = float(np.min(np.abs(np.asarray(seen) - eps)) / eps)
    return dict(phi=phi, reps=np.asarray(reps, dtype=np.int64), X=X, evals=len(seen),
                margin=margin)


def alg1_closest(tiles, eps, crit="spectral", tie=1e-9):
    """Algorithm 1 with closest matching (the variant proposed in the remarks
    after Algorithm 1): instead of stopping at the first database entry
    within the tolerance, patch i is compared with every entry of its size
    that exists when i is visited and is mapped to the closest one among
    those with d < eps; with none it is appended, as in Algorithm 1.

    Whether a patch is appended depends only on whether some earlier entry
    lies within eps, so the database is the one of ``alg1_tolerance``; only
    the map phi can differ.  Reading for equal distances: the entries j with
    d_j < eps and d_j <= d_min (1 + tie) + tie s_i tie (s_i = 1 for the
    spectral distance, sum |A_i| for l1 and ||A_i||_F for Frobenius), and
    the lowest entry index among them is taken, so that distances at
    rounding level do not order the entries by noise.
    Returns dict(phi, reps, X, evals, dmin): evals counts the comparisons
    made, dmin[i] is the distance of patch i to its entry (0 for entries).
    """
    reps, X = [], []
    phi = np.zeros(len(tiles), dtype=np.int64)
    dmin_of = np.zeros(len(tiles))
    evals = 0
    for i, Ai in enumerate(tiles):
        scale = {"spectral": 1.0, "l1": float(np.abs(Ai).sum()),
                 "fro": float(np.linalg.norm(Ai))}[crit]
        cand = [j for j in range(len(reps)) if tiles[reps[j]].shape == Ai.shape]
        dist = np.array([_dist(crit, Ai, tiles[reps[j]], X[j]) for j in cand])
        evals += len(cand)
        within = dist < eps
        if not within.any():
            reps.append(i)
            X.append(factor_inverse(Ai))
            phi[i] = len(reps) - 1
            continue
        dmin = float(dist[within].min())
        band = within & (dist <= dmin * (1.0 + tie) + tie * scale)
        phi[i] = cand[int(np.flatnonzero(band)[0])]
        dmin_of[i] = dmin
    return dict(phi=phi, reps=np.asarray(reps, dtype=np.int64), X=X, evals=evals, dmin=dmin_of)


def alg1_reuse(tiles, eps, crit, phi_prev, reps_prev):
    """Algorithm 1 seeded with the database of the previous system of a
    linear-problem sequence (the reuse of database assignments suggested
    after the third numerical experiment; Section 3.2 on problem sequences).

    The previous entries (patch ids reps_prev, in their order) are the first
    entries, now with the current matrices of those patches.  Every other
    patch i, in ascending id, keeps its previous entry phi_prev[i] when
    d < eps; otherwise it takes the first entry in append order with
    d < eps (the previous entries, then those appended so far), or is
    appended as a new entry.
    Returns dict(phi, reps, X, kept, rescanned, appended, evals)."""
    reps = [int(r) for r in reps_prev]
    X = [factor_inverse(tiles[r]) for r in reps]
    is_rep = set(reps)
    phi = np.zeros(len(tiles), dtype=np.int64)
    for j, r in enumerate(reps):
        phi[r] = j
    kept = rescanned = appended = evals = 0
    for i, Ai in enumerate(tiles):
        if i in is_rep:
            continue
        j0 = int(phi_prev[i])
        if tiles[reps[j0]].shape == Ai.shape:
            evals += 1
            if _dist(crit, Ai, tiles[reps[j0]], X[j0]) < eps:
                phi[i] = j0
                kept += 1
                continue
        hit = None
        for j in range(len(reps)):
            if tiles[reps[j]].shape != Ai.shape:
                continue
            evals += 1
            if _dist(crit, Ai, tiles[reps[j]], X[j]) < eps:
                hit = j
                break
        if hit is None:
            reps.append(i)
            X.append(factor_inverse(Ai))
            hit = len(reps) - 1
            appended += 1
        else:
            rescanned += 1
        phi[i] = hit
    return dict(phi=phi, reps=np.asarray(reps, dtype=np.int64), X=X, kept=kept, rescanned=rescanned,
                appended=appended, evals=evals)


def compressibility(n_p, m_p):
    """Compression ratio (n_p - m_p) / n_p of a database of m_p entries for
    n_p patches: the quantity of the compressibility curve in Experiment 4."""
    return (n_p - m_p) / n_p


def alg1_with_predictions(tiles, eps, crit, train, cand):
    """Algorithm 1 with a predictor of the matching entry (the learned
    shortcut suggested by the closing remarks of Section 3.2).

    1. Algorithm 1 runs on the training patches ``train`` alone (ascending
       id); its entries are the predictor's classes.
    2. Every other patch i, in ascending id, tries the entries ``cand[i]``
       (indices into the training database, most probable first) and takes the
       first with d < eps;
    3. failing that, it scans the current database in append order (the
       training entries, then the entries appended in this step) and takes
       the first with d < eps, or is appended as a new entry.
    Entries of another patch size are never compared.  With ``train`` a
    prefix of the patch ids and no predictions this is Algorithm 1 itself.
    Returns dict(phi, reps, n_train_entries, accepted, scanned,
    scanned_train, appended, evals): scanned counts the patches placed by the
    scan, scanned_train those among them placed on a training entry.
    """
    n = len(tiles)
    train = sorted(int(t) for t in train)
    sub = alg1_tolerance([tiles[i] for i in train], eps, crit)
    reps = [train[int(r)] for r in sub["reps"]]
    X = list(sub["X"])
    phi = -np.ones(n, dtype=np.int64)
    phi[train] = sub["phi"]
    n0 = len(reps)
    evals = int(sub["evals"])
    accepted = scanned = scanned_train = appended = 0
    in_train = np.zeros(n, dtype=bool)
    in_train[train] = True
    for i in range(n):
        if in_train[i]:
            continue
        Ai = tiles[i]
        hit = -1
        for j in cand[i]:
            j = int(j)
            if j < 0 or j >= n0 or tiles[reps[j]].shape != Ai.shape:
                continue
            evals += 1
            if _dist(crit, Ai, tiles[reps[j]], X[j]) < eps:
                hit = j
                break
        if hit >= 0:
            phi[i] = hit
            accepted += 1
            continue
        for j in range(len(reps)):
            if tiles[reps[j]].shape != Ai.shape:
                continue
            evals += 1
            if _dist(crit, Ai, tiles[reps[j]], X[j]) < eps:
                hit = j
                break
        if hit >= 0:
            scanned += 1
            scanned_train += 1 if hit < n0 else 0
        else:
            reps.append(i)
            X.append(factor_inverse(Ai))
            hit = len(reps) - 1
            appended += 1
        phi[i] = hit
    return dict(phi=phi, reps=np.asarray(reps, dtype=np.int64), n_train_entries=n0,
                accepted=accepted, scanned=scanned, scanned_train=scanned_train,
                appended=appended, evals=evals)


def alg1_invariants_hold(tiles_of, phi, reps, eps, crit, sample, X_of=None):
    """Check Algorithm 1's defining properties on sampled patches i:
    a database entry's patch matches no earlier entry; any other patch matches
    its entry (d < eps) and no earlier entry (d >= eps).  ``tiles_of(k)``
    returns the tile of patch k so that huge inputs need not be materialised.
    """
    X_of = X_of or (lambda k: factor_inverse(tiles_of(k)))
    rep_pos = {int(r): j for j, r in enumerate(reps)}
    for i in sample:
        Ai = tiles_of(int(i))
        j = int(phi[i])
        if int(i) in rep_pos:
            if rep_pos[int(i)] != j:
                return False
            earlier = range(j)
        else:
            if reps[j] >= i:
                return False
            if not _dist(crit, Ai, tiles_of(int(reps[j])), X_of(int(reps[j]))) < eps:
                return False
            earlier = range(j)
        for jj in earlier:
            r = int(reps[jj])
            if _dist(crit, Ai, tiles_of(r), X_of(r)) < eps:
                return False
    return True


def partition_groups(tiles, partition=True):
    """Boundary partitioning (Section 3.2): group patches whose boundary
    conditions sit in the same local rows; groups in ascending key order (the
    interior, key 0, first); members in ascending patch id.

    Patches of different sizes are never compared (a matrix of another size
    is no candidate, remark in Section 2), so groups are first split by size:
    the group key is (size, boundary mask), or the size alone without
    partitioning.  With one patch size this is the partition of Section 3.2."""
    sizes = np.array([t.shape[0] for t in tiles], dtype=np.int64)
    if partition:
        masks = np.array([boundary_mask(t) for t in tiles], dtype=np.int64)
    else:
        masks = np.zeros(len(tiles), dtype=np.int64)
    pairs = sorted(set(zip(sizes.tolist(), masks.tolist())))
    return [((int(s), int(m)) if partition else int(s),
             np.flatnonzero((sizes == s) & (masks == m))) for s, m in pairs]


def apportion(sizes, m_total):
    """Split m_total clusters over groups roughly in proportion to their
    sizes (Section 3.2).

    Largest-remainder method in exact integer arithmetic: group g first gets
    floor(m_total * n_g / N); the seats left go one each to the groups with
    the largest remainders (ties: lower group).  A group left with none then
    takes one from the group holding the most (ties: lower group), so every
    group has at least one cluster and never more than its size.
    """
    sizes = [int(s) for s in sizes]
    N = sum(sizes)
    G = len(sizes)
    if m_total < G:
        raise OracleError("fewer clusters than boundary groups")
    if m_total > N:
        raise OracleError("more clusters than patches")
    base = [(m_total * s) // N for s in sizes]
    rem = [(m_total * s) % N for s in sizes]
    left = m_total - sum(base)
    for g in sorted(range(G), key=lambda g: (-rem[g], g))[:left]:
        base[g] += 1
    while 0 in base:
        g0 = base.index(0)
        donor = max(range(G), key=lambda g: (base[g], -g))
        base[donor] -= 1
        base[g0] += 1
    return base


def _initial_reps(groups, m_per, rng):
    """Partial Fisher-Yates draw of m_g distinct members per group, groups in
    order, one SplitMix64 stream: j = i + (u mod (len - i))."""
    out = []
    for (key, members), m_g in zip(groups, m_per):
        a = list(int(x) for x in members)
        L = len(a)
        for i in range(m_g):
            u = rng.next()
            j = i + (u % (L - i))
            a[i], a[j] = a[j], a[i]
        out.append(a[:m_g])
    return out


def _centre(tiles, mem, upd, tie_rel):
    """Centre update of a cluster with members mem (ascending): the entrywise
    mean (Eq.(6)), or the member nearest it (lowest id in the tie band).
    Returns (matrix, patch id or -1)."""
    mean = np.mean(np.stack([tiles[k] for k in mem]), axis=0)
    if upd == "mean":
        return mean, -1
    dist = np.array([np.sum((tiles[k] - mean) ** 2) for k in mem])
    floor = tie_rel * tie_rel * float(np.sum(mean * mean))
    near = np.flatnonzero(dist <= dist.min() * (1.0 + tie_rel) + floor)
    m = int(mem[near[0]])
    return tiles[m].copy(), m


def kmeans(tiles, m_p, variant="spectral", seed=5, max_iter=100, partition=True,
           tie_rel=1e-9, init_reps=None, init_phi=None):
    """Algorithm 2 and the variants of Section 3.2.

    variant: 'spectral'  d = ||I - A B^{-1}||_2, centre = entrywise mean (Eq.(6));
             'entrywise' d = l1 difference to the mean matrix, centre = mean;
             'varmin'    d spectral, centre = member nearest the mean;
             'bootstrap' initial database from Algorithm 1 (``init_reps``),
                         no partitioning, variance-minimising updates.
    Returns dict(phi, B, X, rep_patch, iters, converged, empty_events, groups).
    ``rep_patch[j]`` is the patch whose matrix is centre j (-1 for a mean).
    ``init_phi``: warm start from the assignment of the previous system of a
    linear-problem sequence (Section 3.2 on problem sequences: initialise
    the database from the previous step): the centres start as the update
    of that assignment (mean or medoid of the current matrices), then the
    passes run as usual.  Every centre must keep a member and lie in the
    group of its members.
    """
    if variant == "bootstrap":
        if init_reps is None:
            raise ValueError("bootstrap needs Algorithm 1's representatives")
        groups = partition_groups(tiles, partition=False)
        starts = [[int(r) for r in init_reps if tiles[int(r)].shape[0] == key] for key, _ in groups]
        upd = "varmin"
        crit = "spectral"
    else:
        groups = partition_groups(tiles, partition)
        m_per = apportion([len(g[1]) for g in groups], m_p)
        starts = _initial_reps(groups, m_per, SplitMix64(seed))
        upd = "varmin" if variant == "varmin" else "mean"
        crit = "l1" if variant == "entrywise" else "spectral"

    n_p = len(tiles)
    phi = -np.ones(n_p, dtype=np.int64)
    B_all, X_all, rep_patch = [], [], []
    iters, conv, empty = [], [], 0
    for (key, members), start in zip(groups, starts):
        off = len(B_all)
        B = [tiles[s].copy() for s in start]
        X = [factor_inverse(b) for b in B] if crit == "spectral" else [None] * len(B)
        rp = list(start)
        loc = -np.ones(len(members), dtype=np.int64)
        if init_phi is not None:
            loc = np.asarray(init_phi)[members] - off
            if (loc < 0).any() or (loc >= len(B)).any():
                raise OracleError("previous assignment leaves its group")
            for j in range(len(B)):
                mem = members[loc == j]
                if len(mem) == 0:
                    raise OracleError("previous assignment leaves a centre without members")
                B[j], rp[j] = _centre(tiles, mem, upd, tie_rel)
                if crit == "spectral":
                    X[j] = factor_inverse(B[j])
        it = 0
        converged = False
        while it < max_iter:
            it += 1
            changed = False
            for t, i in enumerate(members):
                d = np.array([_dist(crit, tiles[i], B[j], X[j]) for j in range(len(B))])
                dmin = d.min()
                scale = 1.0 if crit == "spectral" else float(np.sum(np.abs(tiles[i])))
                band = np.flatnonzero(d <= dmin * (1.0 + tie_rel) + tie_rel * scale)
                if loc[t] in band:
                    continue
                loc[t] = band[0]
                changed = True
            if not changed:
                converged = True
                break
            if it == max_iter:
                break
            for j in range(len(B)):
                mem = members[loc == j]
                if len(mem) == 0:
                    empty += 1
                    continue
                B[j], rp[j] = _centre(tiles, mem, upd, tie_rel)
                if crit == "spectral":
                    X[j] = factor_inverse(B[j])
        phi[members] = loc + off
        B_all += B
        X_all += [factor_inverse(b) for b in B] if crit != "spectral" else X
        rep_patch += rp
        iters.append(it)
        conv.append(converged)
    return dict(phi=phi, B=B_all, X=X_all, rep_patch=np.asarray(rep_patch, dtype=np.int64),
                iters=iters, converged=conv, empty_events=empty,
                groups=[(k, m) for k, m in groups])
