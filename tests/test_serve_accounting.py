"""Host-side accounting of the serving loop (no GPU): what a batch holds on the
device while it runs, what a domain is admitted with, and that a batch whose
launch fails goes back to the front of its queue in order."""

import collections

from paper_1708_02845_amd.serve import (Query, Server, latency_breakdown, latency_summary,
                                        put_back, take_batch)


def test_launch_bytes_counts_fields_and_both_call_scratches():
    # 64 fields of a 1025^2 domain, the contraction's target operands and the
    # path launch's scratch
    N = 992_998
    assert Server.launch_bytes(N, 64, (8_400_000, 1_530_000_000)) == \
        64 * N * 4 + 8_400_000 + 1_530_000_000
    assert Server.launch_bytes(N, 1, (0, 0)) == N * 4


def test_domain_footprint_covers_every_slot_at_full_batches():
    srv = Server.__new__(Server)
    srv.slots_per_domain, srv.max_batch = 2, 64
    resident, N, scratch = 66_000_000_000, 992_998, (8_400_000, 1_530_000_000)
    assert srv.domain_footprint(resident, N, scratch) == \
        resident + 2 * (64 * N * 4 + scratch[0] + scratch[1])


def test_failed_launch_returns_its_queries_in_order():
    q = collections.deque(Query(i, "d", i, i + 1, 0.0) for i in range(10))
    batch = take_batch(q, 4)
    assert [x.qid for x in batch] == [0, 1, 2, 3] and len(q) == 6
    put_back(q, batch)
    assert [x.qid for x in q] == list(range(10))


def test_latency_breakdown_splits_wait_launch_and_device_time():
    qs = []
    for i in range(100):
        q = Query(i, "d", 0, 1, arrival=10.0 + i)
        q.launched = q.arrival + 0.001 * (i % 10)     # 0..9 ms queueing
        q.launch_host_ms = 0.05
        q.gpu_ms = 2.0 + (i == 99) * 18.0
        q.done = q.launched + 1e-3 * (q.launch_host_ms + q.gpu_ms) + 1e-5
        qs.append(q)
    b = latency_breakdown(qs)
    assert abs(b["wait"]["max_ms"] - 9.0) < 1e-9 and abs(b["wait"]["p50_ms"] - 4.5) < 1e-9
    assert b["launch_host"]["p99_ms"] == 0.05
    assert b["gpu"]["p50_ms"] == 2.0 and b["gpu"]["max_ms"] == 20.0
    assert abs(b["rest"]["max_ms"] - 0.01) < 1e-6
    s = latency_summary(qs)
    # a query's latency is its wait, the launch, the device time and the poll
    assert abs(s["max_ms"] - (9.0 + 0.05 + 20.0 + 0.01)) < 1e-6


def test_queue_warning_leaves_the_admitted_bytes_alone(monkeypatch):
    # add_domain's hardware-queue check must not touch the HBM accounting
    import warnings

    from paper_1708_02845_amd import serve

    class FakeKernel:
        N = 1000

        def footprint(self):
            return 5_000_000

        def call_scratch(self, n, kind):
            return (1000, 2000)

    monkeypatch.setattr(serve.Kernel, "dense_footprint", staticmethod(lambda N, B, gemm_form: 10))
    monkeypatch.setattr(serve.Kernel, "load_dense", classmethod(lambda cls, *a, **k: FakeKernel()))
    monkeypatch.setattr(serve, "_Slot", lambda *a: object())
    monkeypatch.setenv("GPU_MAX_HW_QUEUES", "1")
    srv = Server.__new__(Server)
    srv.torch, srv.ctx, srv.gemm_form = None, None, "f16x3"
    srv.max_batch, srv.slots_per_domain, srv.max_steps = 8, 1, 100
    srv.hbm_budget, srv.hbm_used, srv.domains, srv.refused = 10**9, 0, {}, []
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        assert srv.add_domain("a", _FakeP(), None)
    assert any("hardware queues" in str(x.message) for x in w)
    assert srv.hbm_used == 5_000_000 + 8 * 1000 * 4 + 1000 + 2000


class _FakeP:
    shape = (1000, 10)
