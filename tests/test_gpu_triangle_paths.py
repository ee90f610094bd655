"""GPU triangle-based descent paths (Section IV, the method of the paper's
figures) against the oracle tracer: on FP32 fields, the tracer run on the same
FP32 values; on FP64 fields (every decision in FP64), the tracer run on the
oracle's own FP64 field."""

import numpy as np
import pytest

from conftest import frac, read_golden
from oracle import divergence as dv
from oracle import triangle_path as tp
from workloads import build_config, grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu

STATUS = {tp.REACHED: "reached", tp.STUCK: "stuck", tp.MAX_STEPS: "max_steps"}


def run_gpu(k, ss, ts, fields, max_steps):
    import torch
    pts, wh, lens, st = k.trace_paths_triangles(ss, ts, fields, max_steps)
    torch.cuda.synchronize()
    pts, wh, lens, st = pts.cpu().numpy(), wh.cpu().numpy(), lens.cpu().numpy(), st.cpu().numpy()
    out = []
    for i in range(len(ss)):
        n = int(lens[i])
        assert np.all(wh[i, n:] == -1)
        out.append((pts[i, :n], [tuple(int(x) for x in w) for w in wh[i, :n]],
                    {0: "reached", 1: "stuck", 2: "max_steps"}[int(st[i])]))
    return out


def check_same(got, ref, tol=1e-12):
    gp, gw, gs = got
    rp, rw, rs = ref
    assert gs == STATUS[rs]
    assert gw == rw
    assert np.abs(gp - rp).max() <= tol


@pytest.fixture(scope="module")
def grid(gpu_ctx):
    from paper_1708_02845_amd import Kernel
    g = grid_domain(97, 3, (0.1, 0.25), seed_id=31)
    P = g.poisson_kernel().astype(np.float32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx))
    faces, xy = g.interior_mesh()
    k.attach_mesh(faces, xy)
    k.P64 = P.astype(np.float64)
    yield g, k, tp.Mesh(faces, xy)
    k.free()


@pytest.mark.parametrize("kind", ["kl", "tv", "chi2", "hellinger"])
def test_grid_triangle_paths_match_oracle(grid, kind):
    g, k, mesh = grid
    ts, ss = targets_sources(36, g.N, 6)
    F, _ = k.batch_fields(ts, kind)
    res = run_gpu(k, ss, ts, F, 20000)
    Fh = F.cpu().numpy().astype(np.float64)
    n_edge_pts = 0
    for i, (s, t) in enumerate(zip(ss, ts)):
        ref = tp.triangle_path(mesh, Fh[i], g.adj_ptr, g.adj_idx, int(s), int(t), 20000)
        check_same(res[i], ref)
        n_edge_pts += sum(1 for w in res[i][1] if w[1] >= 0)
    assert n_edge_pts > 50     # the paths do cut through triangles


def test_disk_triangle_paths_match_oracle(gpu_ctx):
    from paper_1708_02845_amd import Kernel
    inst = build_config("disk4096")
    k = Kernel.load_dense(gpu_ctx, inst.P, adjacency=(inst.adj_ptr, inst.adj_idx))
    try:
        faces, xy = inst.interior_mesh()
        k.attach_mesh(faces, xy)
        mesh = tp.Mesh(faces, xy)
        ts, ss = targets_sources(0, inst.N, 8)
        for kind in ("kl", "tv"):
            F, _ = k.batch_fields(ts, kind)
            res = run_gpu(k, ss, ts, F, 20000)
            Fh = F.cpu().numpy().astype(np.float64)
            for i, (s, t) in enumerate(zip(ss, ts)):
                ref = tp.triangle_path(mesh, Fh[i], inst.adj_ptr, inst.adj_idx, int(s), int(t),
                                       20000)
                check_same(res[i], ref)
                assert res[i][2] == "reached"
    finally:
        k.free()


def test_hand_traced_square(gpu_ctx):
    import torch
    from paper_1708_02845_amd import Kernel
    rows = read_golden("triangle_path_square4.txt")
    xy = np.array([[float(r[2]), float(r[3])] for r in rows if r[0] == "vertex"])
    faces = np.array([[int(v) for v in r[1:]] for r in rows if r[0] == "face"])
    d = np.array([float(v) for v in [r for r in rows if r[0] == "value"][0][1:]], np.float32)
    src = int([r for r in rows if r[0] == "source"][0][1])
    tgt = int([r for r in rows if r[0] == "target"][0][1])
    exp = [r for r in rows if r[0] == "point"]
    adj = {0: [1, 3, 4], 1: [0, 2, 4], 2: [1, 3, 4], 3: [0, 2, 4], 4: [0, 1, 2, 3]}
    ptr = np.cumsum([0] + [len(adj[v]) for v in range(5)]).astype(np.int64)
    idx = np.concatenate([adj[v] for v in range(5)]).astype(np.int32)
    P = np.full((5, 4), 0.25, dtype=np.float32)     # any kernel: the field is given
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(ptr, idx))
    try:
        k.attach_mesh(faces, xy)
        field = torch.from_numpy(d).cuda().reshape(1, -1)
        (pts, where, st), = run_gpu(k, [src], [tgt], field, 100)
        assert st == "reached" and len(pts) == len(exp)
        for p, w, e in zip(pts, where, exp):
            assert p == pytest.approx([frac(e[1]), frac(e[2])], abs=1e-15)
            assert w == (int(e[3]), int(e[4]))
    finally:
        k.free()


def test_step_cap_and_source_equals_target(grid):
    g, k, mesh = grid
    ts = [100, 100]
    ss = [g.N - 50, 100]
    F, _ = k.batch_fields(ts, "kl")
    res = run_gpu(k, ss, ts, F, 4)
    Fh = F.cpu().numpy().astype(np.float64)
    ref = tp.triangle_path(mesh, Fh[0], g.adj_ptr, g.adj_idx, ss[0], ts[0], 4)
    check_same(res[0], ref)
    assert len(res[0][0]) == 5 and res[0][2] == "max_steps"
    assert res[1][1] == [(100, -1)] and res[1][2] == "reached"


def test_mesh_validation(gpu_ctx):
    from paper_1708_02845_amd import DDError, Kernel
    P = np.full((5, 4), 0.25, dtype=np.float32)
    ptr = np.array([0, 1, 2, 3, 4, 4], dtype=np.int64)
    idx = np.array([1, 0, 3, 2], dtype=np.int32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(ptr, idx))
    try:
        xy = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [2, 2]], dtype=np.float64)
        F = np.zeros((1, 5), dtype=np.float32)
        import torch
        with pytest.raises(DDError, match="no mesh"):
            k.trace_paths_triangles([0], [1], torch.zeros((1, 5), device="cuda"), 10)
        bad = [np.array([[0, 1, 1]]),                    # repeated vertex
               np.array([[0, 3, 4]]),                    # collinear: zero area
               np.array([[0, 1, 5]]),                    # id out of range
               np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4]])]   # edge 0-1 in three faces
        for f in bad:
            with pytest.raises(DDError, match="DD_EINVAL"):
                k.attach_mesh(f, xy)
        k.attach_mesh(np.array([[0, 2, 1], [1, 2, 3]]), xy)   # clockwise input is fine
        del F
    finally:
        k.free()


@pytest.mark.parametrize("kind", ["kl", "tv", "chi2"])
def test_exact_fields_match_oracle(grid, kind):
    g, k, mesh = grid
    ts = targets_sources(37, g.N, 5)[0]
    E = k.exact_fields(ts, kind).cpu().numpy()
    for i, t in enumerate(ts):
        ref = dv.field(k.P64, int(t), kind)
        assert E[i, t] == 0.0
        assert np.abs(E[i] - ref).max() <= 1e-13 * np.abs(ref).max(), (kind, i)


@pytest.mark.parametrize("kind", ["kl", "tv"])
def test_grid_paths_on_fp64_fields_match_oracle_field(grid, kind):
    """Every decision on FP64 values: the paths equal the oracle's tracer on the
    oracle's own FP64 field (the fields differ only in the rounding of their
    sums, which moves the points by far less than 1e-9)."""
    g, k, mesh = grid
    ts, ss = targets_sources(38, g.N, 6)
    E = k.exact_fields(ts, kind)
    res = run_gpu(k, ss, ts, E, 20000)
    for i, (s, t) in enumerate(zip(ss, ts)):
        ref = tp.triangle_path(mesh, dv.field(k.P64, int(t), kind), g.adj_ptr, g.adj_idx, int(s),
                               int(t), 20000)
        check_same(res[i], ref, tol=1e-9)


def test_disk_paths_on_fp64_fields_match_oracle_field(gpu_ctx):
    from paper_1708_02845_amd import Kernel
    inst = build_config("disk4096")
    k = Kernel.load_dense(gpu_ctx, inst.P, adjacency=(inst.adj_ptr, inst.adj_idx))
    try:
        faces, xy = inst.interior_mesh()
        k.attach_mesh(faces, xy)
        mesh = tp.Mesh(faces, xy)
        ts, ss = targets_sources(0, inst.N, 8)
        for kind in ("kl", "tv"):
            E = k.exact_fields(ts, kind)
            res = run_gpu(k, ss, ts, E, 20000)
            for i, (s, t) in enumerate(zip(ss, ts)):
                ref = tp.triangle_path(mesh, dv.field(inst.P, int(t), kind), inst.adj_ptr,
                                       inst.adj_idx, int(s), int(t), 20000)
                check_same(res[i], ref, tol=1e-9)
                assert res[i][2] == "reached"
    finally:
        k.free()
