"""Edge-based gradient-descent path and spurious minima (Sections IV and V).

Path rule (Section IV, "Gradient-descent path generation", edge-based variant):
from the current vertex move to the neighbour that decreases the distance the
most, i.e. the neighbour with the smallest distance value.  Readings where the
paper is silent: ties go to the lowest vertex index; the walk stops as STUCK
when no neighbour is strictly lower (a local minimum), as REACHED at the
target, and as MAX_STEPS after ``max_steps`` moves.

Spurious minimum (Section V, "Low resolution discretizations"): a vertex other
than the target none of whose neighbours is strictly lower.
"""

import numpy as np

REACHED, STUCK, MAX_STEPS = 0, 1, 2


def steepest_descent_path(d, adj_ptr, adj_idx, source, target, max_steps):
    """Vertex list from ``source`` and its status, decided on the FP64 field d."""
    d = np.asarray(d, dtype=np.float64)
    v = int(source)
    path = [v]
    while True:
        if v == target:
            return path, REACHED
        if len(path) - 1 >= max_steps:
            return path, MAX_STEPS
        best = -1
        best_val = np.inf
        for u in adj_idx[adj_ptr[v]:adj_ptr[v + 1]]:
            u = int(u)
            du = d[u]
            if du < best_val or (du == best_val and (best < 0 or u < best)):
                best, best_val = u, du
        if best < 0 or not best_val < d[v]:
            return path, STUCK
        v = best
        path.append(v)


def steepest_descent_path_lazy(dist, adj_ptr, adj_idx, source, target, max_steps):
    """The same walk with distances evaluated on demand (Section V: on the CPU
    the distances are computed only for the vertices the path needs).

    ``dist(xs)`` returns the FP64 distances of the vertex list xs.  Each vertex
    is evaluated at most once.  Returns (path, status, number of evaluations).
    """
    cache = {}

    def d(xs):
        need = [x for x in xs if x not in cache]
        if need:
            for x, v in zip(need, dist(need)):
                cache[x] = float(v)
        return [cache[x] for x in xs]

    v = int(source)
    dv = d([v])[0]
    path = [v]
    while True:
        if v == target:
            return path, REACHED, len(cache)
        if len(path) - 1 >= max_steps:
            return path, MAX_STEPS, len(cache)
        nb = [int(u) for u in adj_idx[adj_ptr[v]:adj_ptr[v + 1]]]
        best = -1
        best_val = np.inf
        for u, du in zip(nb, d(nb)):
            if du < best_val or (du == best_val and (best < 0 or u < best)):
                best, best_val = u, du
        if best < 0 or not best_val < dv:
            return path, STUCK, len(cache)
        v, dv = best, best_val
        path.append(v)


def spurious_minima(d, adj_ptr, adj_idx, target):
    """Sorted list of vertices v != target with min over neighbours d(u) >= d(v)."""
    d = np.asarray(d, dtype=np.float64)
    out = []
    for v in range(len(d)):
        if v == target:
            continue
        nb = adj_idx[adj_ptr[v]:adj_ptr[v + 1]]
        if len(nb) == 0 or d[nb].min() >= d[v]:
            out.append(v)
    return out
