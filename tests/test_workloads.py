"""Seeded workload generators: determinism, sizes and the arrival process."""

import numpy as np

from workloads import build_config, grid_domain
from workloads.seeds import targets_sources
from workloads.serving import poisson_arrivals


def test_generators_are_seeded():
    a = build_config("disk4096")
    b = build_config("disk4096")
    assert np.array_equal(a.P, b.P) and np.array_equal(a.adj_idx, b.adj_idx)
    g1 = grid_domain(65, 2, seed_id=9)
    g2 = grid_domain(65, 2, seed_id=9)
    assert g1.rects == g2.rects and np.array_equal(g1.interior, g2.interior)
    t1, s1 = targets_sources(4, 1000, 50)
    t2, s2 = targets_sources(4, 1000, 50)
    assert np.array_equal(t1, t2) and np.array_equal(s1, s2) and np.all(t1 != s1)


def test_grid_geometry_invariants():
    g = grid_domain(97, 3, (0.1, 0.25), seed_id=5)
    G = g.G
    assert g.N + g.K + sum((r[2] - r[0] - 1) * (r[3] - r[1] - 1) for r in g.rects) == G * G
    deg = np.diff(g.adj_ptr)
    assert deg.max() <= 6 and deg.min() >= 1
    # the adjacency is symmetric
    e = set()
    for v in range(g.N):
        for u in g.adj_idx[g.adj_ptr[v]:g.adj_ptr[v + 1]]:
            e.add((v, int(u)))
    assert all((u, v) in e for v, u in e)


def test_c2_sizes():
    g = build_config("grid257")
    assert (g.N, g.K) == (60695, 1482)


def test_poisson_arrivals_rate_and_determinism():
    doms = [("a", 100), ("b", 50), ("c", 30)]
    a = poisson_arrivals(3, doms, 200.0, 60.0)
    b = poisson_arrivals(3, doms, 200.0, 60.0)
    assert a == b
    assert abs(len(a) / 60.0 - 200.0) < 200.0 * 0.05
    gaps = np.diff([x[0] for x in a])
    assert np.all(gaps > 0) and abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0
    assert all(s != t for _, _, s, t in a)
    counts = {n: sum(1 for x in a if x[1] == n) for n, _ in doms}
    assert min(counts.values()) > 0.28 * len(a)
