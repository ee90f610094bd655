"""Host-side accounting of the serving loop (no GPU): what a batch holds on the
device while it runs, what a domain is admitted with, and that a batch whose
launch fails goes back to the front of its queue in order."""

import collections

from paper_1708_02845_amd.serve import Query, Server, put_back, take_batch


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
