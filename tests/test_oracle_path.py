"""Pins for the oracle's edge-based path and spurious-minimum count."""

import numpy as np
import pytest

from conftest import read_golden
from oracle import disk as odisk
from oracle import divergence as dv
from oracle import path as op
from workloads import build_config
from workloads.disk import edges_to_csr
from workloads.seeds import targets_sources


def grid_graph(rows, cols):
    edges = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                edges.append((v, v + 1))
            if r + 1 < rows:
                edges.append((v, v + cols))
            if r + 1 < rows and c + 1 < cols:
                edges.append((v, v + cols + 1))
    return edges_to_csr(rows * cols, edges)


@pytest.fixture(scope="module")
def c1():
    return build_config("disk4096")


def test_hand_traced_paths_on_small_grid():
    lines = read_golden("path_grid4x4.txt")
    field = np.array([float(v) for v in lines[0][1:]])
    target = int(lines[1][1])
    ptr, idx = grid_graph(4, 4)
    for ln in lines[2:]:
        expect = [int(v) for v in ln[1:]]
        got, status = op.steepest_descent_path(field, ptr, idx, expect[0], target, 100)
        assert status == op.REACHED
        assert got == expect


def test_stuck_at_planted_minimum_and_step_cap():
    ptr, idx = grid_graph(3, 5)
    d = np.arange(15, dtype=float)[::-1].copy()   # decreasing towards vertex 14
    d[7] = -1.0                                    # a pit in the middle
    path, status = op.steepest_descent_path(d, ptr, idx, 0, 14, 100)
    assert status == op.STUCK and path[-1] == 7
    path, status = op.steepest_descent_path(np.arange(15.0)[::-1], ptr, idx, 0, 14, 2)
    assert status == op.MAX_STEPS and len(path) == 3
    path, status = op.steepest_descent_path(d, ptr, idx, 14, 14, 100)
    assert status == op.REACHED and path == [14]


def test_plateau_counts_as_stuck():
    ptr, idx = grid_graph(1, 4)
    d = np.array([3.0, 2.0, 2.0, 0.0])
    path, status = op.steepest_descent_path(d, ptr, idx, 0, 3, 10)
    assert status == op.STUCK and path == [0, 1]


@pytest.mark.parametrize("k", range(6))
def test_disk_kl_paths_follow_hyperbolic_geodesics(c1, k):
    # Appendix Section 2.2: gradient-descent paths of D and of every divergence
    # distance on the disk are hyperbolic geodesics.  The edge path must reach
    # the target, stay near that arc, and equal the argmin path of the exact
    # (monotone in rho) closed-form field.
    t, s = targets_sources(0, c1.N, 6)
    t, s = int(t[k]), int(s[k])
    kl = dv.kl_field(c1.P, t)
    path, status = op.steepest_descent_path(kl, c1.adj_ptr, c1.adj_idx, s, t, 4000)
    assert status == op.REACHED
    vals = kl[path]
    assert np.all(np.diff(vals) < 0)
    e = c1.adj_idx
    r = np.repeat(np.arange(c1.N), np.diff(c1.adj_ptr))
    mean_edge = np.abs(c1.z[r] - c1.z[e]).mean()
    assert odisk.geodesic_distance(c1.z[path], c1.z[s], c1.z[t]).max() < 4.0 * mean_edge
    rho_path, _ = op.steepest_descent_path(odisk.rho(c1.z, c1.z[t]), c1.adj_ptr, c1.adj_idx, s, t, 4000)
    assert path == rho_path


def test_spurious_minima_planted():
    ptr, idx = grid_graph(5, 5)
    d = np.zeros(25)
    for v in range(25):
        r, c = divmod(v, 5)
        d[v] = abs(r - 4) + abs(c - 4)    # decreasing towards the target 24
    assert op.spurious_minima(d, ptr, idx, 24) == []
    d[6] = -0.5      # a pit
    d[0] = d[1] = d[5] = 10.0
    d[2] = 10.0      # vertex 1 now has neighbours 0, 2, 5, 6 -> 6 is lower: not a minimum
    assert op.spurious_minima(d, ptr, idx, 24) == [6]


def test_no_spurious_minima_in_disk_fields(c1):
    # Section V: the paper never met a spurious minimum for KL; on the
    # continuous disk neither field has one (Theorem A5).
    t = int(targets_sources(0, c1.N, 1)[0][0])
    for field in (dv.kl_field(c1.P, t), dv.tv_field(c1.P, t)):
        assert op.spurious_minima(field, c1.adj_ptr, c1.adj_idx, t) == []


@pytest.mark.parametrize("kind", ["kl", "tv"])
def test_on_demand_walk_equals_full_field_walk(c1, kind):
    # Section V: the CPU evaluates distances only where the path needs them;
    # the walk must be the one the full field gives, at a small fraction of
    # the evaluations
    ts, ss = targets_sources(0, c1.N, 4)
    for s, t in zip(ss, ts):
        s, t = int(s), int(t)
        full = dv.FIELDS[kind](c1.P, t)
        ref, ref_st = op.steepest_descent_path(full, c1.adj_ptr, c1.adj_idx, s, t, 4000)
        got, st, n_eval = op.steepest_descent_path_lazy(
            lambda xs: dv.distances(c1.P, t, xs, kind), c1.adj_ptr, c1.adj_idx, s, t, 4000)
        assert got == ref and st == ref_st
        deg = int(np.diff(c1.adj_ptr).max())
        assert n_eval <= 1 + (len(got) - 1) * deg and n_eval < c1.N // 10
