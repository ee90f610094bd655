"""Pins for the oracle's triangle-based descent path (Section IV, second
method of "Gradient-descent path generation"; Fig. 2)."""

import numpy as np
import pytest

from conftest import frac, read_golden
from oracle import disk as odisk
from oracle import divergence as dv
from oracle import path as op
from oracle import triangle_path as tp
from workloads import build_config, grid_domain
from workloads.seeds import targets_sources


def grid_mesh(g):
    return tp.Mesh(*g.interior_mesh())


def test_hand_traced_square():
    rows = read_golden("triangle_path_square4.txt")
    xy = np.array([[float(r[2]), float(r[3])] for r in rows if r[0] == "vertex"])
    faces = np.array([[int(v) for v in r[1:]] for r in rows if r[0] == "face"])
    d = np.array([float(v) for v in [r for r in rows if r[0] == "value"][0][1:]])
    src = int([r for r in rows if r[0] == "source"][0][1])
    tgt = int([r for r in rows if r[0] == "target"][0][1])
    exp = [r for r in rows if r[0] == "point"]
    adj = {0: [1, 3, 4], 1: [0, 2, 4], 2: [1, 3, 4], 3: [0, 2, 4], 4: [0, 1, 2, 3]}
    ptr = np.cumsum([0] + [len(adj[v]) for v in range(5)])
    idx = np.concatenate([adj[v] for v in range(5)])
    pts, where, st = tp.triangle_path(tp.Mesh(faces, xy), d, ptr, idx, src, tgt, 100)
    assert st == tp.REACHED
    assert len(pts) == len(exp)
    for p, w, e in zip(pts, where, exp):
        assert p == pytest.approx([frac(e[1]), frac(e[2])], abs=1e-15)
        assert w == (int(e[3]), int(e[4]))


@pytest.fixture(scope="module")
def open_grid():
    return grid_domain(41, 0, seed_id=61)


def test_linear_field_gives_a_straight_ray(open_grid):
    # one gradient everywhere: the path is the ray source - lam * c until it
    # meets the edge of the walkable region
    g = open_grid
    mesh = grid_mesh(g)
    xy = mesh.xy
    c = np.array([1.0, 0.37])
    d = xy @ c
    s = int(np.argmin(np.hypot(xy[:, 0] - 0.8, xy[:, 1] - 0.7)))
    t = int(np.argmin(d))
    pts, where, st = tp.triangle_path(mesh, d, g.adj_ptr, g.adj_idx, s, t, 10000)
    n = np.array([-c[1], c[0]]) / np.hypot(*c)
    first_slide = next(i for i in range(1, len(where)) if where[i][1] == -1)
    assert first_slide > 10
    off = np.abs((pts[:first_slide] - xy[s]) @ n)
    assert off.max() < 1e-12
    assert st == tp.REACHED and where[-1] == (t, -1)


def test_values_decrease_along_the_path(open_grid):
    g = open_grid
    mesh = grid_mesh(g)
    xy = mesh.xy
    tgt = np.array([0.3, 0.25])
    d = np.hypot(xy[:, 0] - tgt[0], xy[:, 1] - tgt[1]) ** 2
    t = int(np.argmin(d))
    for s in (0, g.N - 1, g.N // 2 + 7):
        pts, where, st = tp.triangle_path(mesh, d, g.adj_ptr, g.adj_idx, s, t, 10000)
        assert st == tp.REACHED
        # the interpolated value at each point (vertex value, or linear along the edge)
        vals = []
        for p, (a, b) in zip(pts, where):
            if b < 0:
                vals.append(d[a])
            else:
                u = np.dot(p - xy[a], xy[b] - xy[a]) / np.dot(xy[b] - xy[a], xy[b] - xy[a])
                vals.append((1 - u) * d[a] + u * d[b])
        assert np.all(np.diff(vals) < 0)
        # close to the straight segment to the target (the exact flow)
        seg = xy[t] - xy[s]
        nrm = np.array([-seg[1], seg[0]]) / np.hypot(*seg)
        assert np.abs((pts - xy[s]) @ nrm).max() < 2 * g.h


@pytest.mark.parametrize("kind", ["kl", "tv"])
def test_disk_triangle_paths_follow_geodesics_better_than_edge_paths(kind):
    # Appendix 2.2: descent paths on the disk are hyperbolic geodesics; Fig. 2:
    # triangle-based paths are smoother than edge-based ones
    inst = build_config("disk4096")
    mesh = tp.Mesh(*inst.interior_mesh())
    ts, ss = targets_sources(0, inst.N, 4)
    gap_tri, gap_edge = [], []
    for s, t in zip(ss, ts):
        s, t = int(s), int(t)
        d = dv.FIELDS[kind](inst.P, t)
        pts, where, st = tp.triangle_path(mesh, d, inst.adj_ptr, inst.adj_idx, s, t, 20000)
        assert st == tp.REACHED
        epath, est = op.steepest_descent_path(d, inst.adj_ptr, inst.adj_idx, s, t, 4000)
        assert est == op.REACHED
        zt = pts[:, 0] + 1j * pts[:, 1]
        gap_tri.append(odisk.geodesic_distance(zt, inst.z[s], inst.z[t]).mean())
        gap_edge.append(odisk.geodesic_distance(inst.z[epath], inst.z[s], inst.z[t]).mean())
    assert np.mean(gap_tri) < np.mean(gap_edge)
