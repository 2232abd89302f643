"""Selection rules written out plainly (test infrastructure only).

COMPAR's runtime picks, per call, one implementation variant of an interface
from the runtime context (Sec. 1 names input size, the resources' capability
and the system configuration; Sec. 2.2.2 has the runtime choose a codelet per
task).  OpenMP's declare-variant, which COMPAR extends (Sec. 2.1), first keeps
the variants whose context matches and then scores them.  Here the context is
(M, N, K, tolerance); a variant "matches" when its stated error bound is within
the caller's tolerance, and the score is its (measured or predicted) time.

Ties: equal times prefer the variant with the tighter stated bound, then the
lower registration id.  Nearest-neighbour distance ties prefer the earliest
recorded row.
"""
from __future__ import annotations

import math

import numpy as np


def admissible(bounds, tol):
    """Indices of variants whose stated error bound is <= tol."""
    return [i for i, b in enumerate(bounds) if b <= tol]


def argmin_tiebreak(times, cand, bounds):
    """Variant in cand with the lowest time; ties -> tighter bound, then lower id."""
    best = None
    for i in cand:
        key = (times[i], bounds[i], i)
        if best is None or key < best[0]:
            best = (key, i)
    return None if best is None else best[1]


def exhaustive_best(times, bounds, tol):
    """The selection oracle: best measured admissible variant."""
    return argmin_tiebreak(times, admissible(bounds, tol), bounds)


def shape_features(M, N, K):
    return (math.log2(M), math.log2(N), math.log2(K))


def nearest_row(train_shapes, M, N, K):
    """Index of the recorded shape nearest to (M, N, K) in (log2 M, log2 N, log2 K);
    Euclidean distance compared through its square; ties -> earliest row."""
    q = shape_features(M, N, K)
    best_i, best_d = None, None
    for i, (m, n, k) in enumerate(train_shapes):
        f = shape_features(int(m), int(n), int(k))
        d = (f[0] - q[0]) ** 2 + (f[1] - q[1]) ** 2 + (f[2] - q[2]) ** 2
        if best_d is None or d < best_d:
            best_i, best_d = i, d
    return best_i


def nn_select(train_shapes, train_times, bounds, M, N, K, tol):
    """History nearest-neighbour choice: the nearest recorded shape's best admissible variant."""
    r = nearest_row(train_shapes, M, N, K)
    return argmin_tiebreak(list(train_times[r]), admissible(bounds, tol), bounds)


def static_choice(train_times, bounds, tol):
    """Best single variant for a tolerance: the admissible variant with the lowest total
    recorded time over the recorded shapes (every row holds all variants' times);
    with no rows, the tightest bound, then the lowest id."""
    cand = admissible(bounds, tol)
    if len(train_times) == 0:
        return argmin_tiebreak([0.0] * len(bounds), cand, bounds)
    tot = [sum(row[v] for row in train_times) for v in range(len(bounds))]
    return argmin_tiebreak(tot, cand, bounds)


def regret(times, choices, tols, bounds):
    """Aggregate and per-shape regret of `choices` against the exhaustive best.

    Returns dict(aggregate = sum T[s, choice] / sum T[s, best] - 1,
                 mean, p95 of T[s, choice] / T[s, best] - 1).
    """
    T = np.asarray(times, dtype=np.float64)
    best = [exhaustive_best(list(T[s]), bounds, tols[s]) for s in range(T.shape[0])]
    sel = np.array([T[s, c] for s, c in enumerate(choices)])
    opt = np.array([T[s, b] for s, b in enumerate(best)])
    per = sel / opt - 1.0
    return dict(aggregate=float(sel.sum() / opt.sum() - 1.0), mean=float(per.mean()),
                p95=float(np.percentile(per, 95)), best=best)
