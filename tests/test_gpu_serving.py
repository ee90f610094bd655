"""Continuous-batching service: every query answered, identical alone and in the mix."""

import numpy as np
import pytest

from workloads import build_config, grid_domain
from workloads.serving import poisson_arrivals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def domains():
    out = {}
    for name, (G, k, cid) in {"g49": (49, 2, 61), "g65": (65, 3, 62), "g81": (81, 4, 63)}.items():
        g = grid_domain(G, k, (0.1, 0.25), seed_id=cid)
        out[name] = (g.poisson_kernel().astype(np.float32), (g.adj_ptr, g.adj_idx))
    disk = build_config("disk4096", N=1500, B=128)
    out["disk"] = (disk.P, (disk.adj_ptr, disk.adj_idx))
    return out


def test_mix_equals_alone(gpu_ctx, domains):
    from paper_1708_02845_amd.serve import Server, latency_breakdown, latency_summary
    srv = Server(gpu_ctx, max_batch=16, slots_per_domain=2, max_steps=2000, keep_fields=True)
    try:
        for name, (P, adj) in domains.items():
            assert srv.add_domain(name, P, adj)
        arr = poisson_arrivals(7, [(n, srv.domains[n].kernel.N) for n in srv.domains], 4000.0, 0.1)
        assert len(arr) > 200
        qs = srv.run_open_loop(arr, timeout=300)
        assert len(srv.completed) == len(arr) == len(qs)
        assert sorted(q.qid for q in srv.completed) == list(range(len(arr)))
        assert max(srv.batch_sizes) > 1          # batching actually happened
        for q in qs:
            assert q.done >= q.arrival and q.status in ("reached", "stuck", "max_steps")
            assert q.path[0] == q.source
        s = latency_summary(qs)
        assert 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
        b = latency_breakdown(qs)
        assert b["gpu"]["p50_ms"] > 0 and b["wait"]["p50_ms"] >= 0
        assert b["gpu"]["max_ms"] <= s["max_ms"] and b["wait"]["max_ms"] <= s["max_ms"]
        # each query alone: the same field (bit for bit) and the same path
        for q in qs[::7]:
            k = srv.domains[q.domain].kernel
            alone, _ = k.batch_fields([q.target], "kl")
            assert np.array_equal(alone[0].cpu().numpy(), q.field.cpu().numpy())
            path, status, _ = k.plan_path(q.source, q.target, "kl", 2000)
            assert (q.path, q.status) == (path, status)
    finally:
        srv.close()


def test_admission_refuses_what_does_not_fit(gpu_ctx, domains):
    from paper_1708_02845_amd.serve import Server
    P, adj = domains["g65"]
    small = Server(gpu_ctx, max_batch=8, hbm_budget=1000)
    assert not small.add_domain("g65", P, adj)
    assert small.refused and not small.domains
    srv = Server(gpu_ctx, max_batch=8, hbm_budget=srv_budget(P, 1.5))
    try:
        assert srv.add_domain("a", P, adj)
        assert not srv.add_domain("b", P, adj)   # a second copy exceeds the budget
    finally:
        srv.close()


def srv_budget(P, factor):
    from paper_1708_02845_amd.serve import Server
    from paper_1708_02845_amd import Kernel
    N, B = P.shape
    need = Kernel.dense_footprint(N, B, gemm_form="f16x3") + 2 * 8 * N * 4
    return int(need * factor)
