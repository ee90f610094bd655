"""One handle used from several host threads, each on a stream of its own
(the C ABI allows it): every result equals the one computed alone."""

import threading

import numpy as np
import pytest

from workloads import grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu


def test_concurrent_calls_on_one_handle(gpu_ctx):
    import torch
    from paper_1708_02845_amd import Kernel
    g = grid_domain(65, 2, (0.1, 0.25), seed_id=91)
    P = g.poisson_kernel().astype(np.float32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx), gemm_form="f16x3")
    try:
        ts, ss = targets_sources(91, g.N, 24)
        jobs = [(kind, ts[i::4], ss[i::4]) for i, kind in enumerate(("kl", "tv", "kl", "tv"))]

        def run(kind, t, s):
            f, b = k.batch_fields(t, kind)
            paths, lens, status, _ = k.trace_paths(s, t, kind, f, b, 4000)
            torch.cuda.current_stream().synchronize()
            return f.cpu().numpy(), paths.cpu().numpy(), lens.cpu().numpy()

        alone = [run(*j) for j in jobs]
        torch.cuda.synchronize()
        got = [None] * len(jobs)
        errors = []

        def worker(i):
            try:
                with torch.cuda.stream(torch.cuda.Stream()):
                    got[i] = run(*jobs[i])
            except Exception as e:   # reported below, on the main thread
                errors.append(e)

        threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(jobs))]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        assert not errors, errors
        for a, b in zip(alone, got):
            assert np.array_equal(a[0], b[0])
            assert np.array_equal(a[2], b[2])
            for i, n in enumerate(a[2]):
                assert np.array_equal(a[1][i, :n], b[1][i, :n])
    finally:
        k.free()
