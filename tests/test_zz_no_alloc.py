"""The allocation-free batch entry point (dd_batch_distance_fields_noalloc).

It runs the kernels of dd_batch_distance_fields with the call's scratch taken
from the library's fixed per-GPU buffer, so its fields and bounds must equal
that entry point's bit for bit.  Each case makes two calls in a row, the second
with fewer targets (the buffer then holds the first call's contents), for every
branch that takes scratch: the dense contraction, the floored contraction of a
truncated handle (FP32 and FP64 stored values), the many-target pass over
stored rows (FP32 and FP16 values), and the per-target streams (no scratch).
A call whose scratch exceeds the buffer is refused before anything runs.
"""

import numpy as np
import pytest

from workloads import grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grid():
    g = grid_domain(97, 3, (0.1, 0.25), seed_id=71)
    return g, g.poisson_kernel()


def _same(k, ts, kind):
    import torch
    ref, rb = k.batch_fields(ts, kind)
    out = torch.full_like(ref, float("nan"))
    got, gb = k.batch_fields_noalloc(ts, kind, out=out)
    torch.cuda.synchronize()
    assert got.data_ptr() == out.data_ptr()
    assert torch.equal(got, ref)
    assert gb == rb


CASES = [
    # (label, load kwargs, kinds, (T first, T second))
    ("dense_f16x3", dict(gemm_form="f16x3"), ("kl",), (200, 37)),
    ("dense_f32", dict(gemm_form="f32"), ("kl",), (300, 5)),
    ("dense_bf16x3", dict(gemm_form="bf16x3"), ("kl",), (64, 33)),
    ("dense_f16", dict(gemm_form="f16"), ("kl",), (100, 31)),
    ("floored_f16x3", dict(gemm_form="f16x3", tau=1e-4), ("kl",), (130, 9)),
    ("csr_f32", dict(tau=1e-5), ("tv", "kl"), (257, 40)),
    ("csr_f16", dict(tau=1e-5, csr_values="f16"), ("tv", "kl"), (200, 12)),
    ("dense_streams", dict(), ("tv", "kl", "hellinger"), (6, 3)),
]


@pytest.mark.parametrize("label,kw,kinds,sizes", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("f64", [False, True], ids=["f32in", "f64in"])
def test_noalloc_equals_batch_entry_point(gpu_ctx, grid, label, kw, kinds, sizes, f64):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P if f64 else P.astype(np.float32), **kw)
    try:
        ts = targets_sources(72, g.N, max(sizes))[0]
        for kind in kinds:
            for T in sizes:
                _same(k, ts[:T], kind)
    finally:
        k.free()


def test_noalloc_refuses_scratch_beyond_the_buffer(gpu_ctx):
    """A truncated handle from FP64 values with the contraction operand and
    16,000 kept columns needs 2 x 8.2 MB of target operands, 16.4 MB of FP32
    and 32.8 MB of FP64 expanded target rows at 256 targets: 65.5 MB, above the
    48 MiB buffer.  At 64 targets it needs 16.4 MB and runs."""
    import torch
    from paper_1708_02845_amd import DDError, Kernel, _lib
    rng = np.random.default_rng(5)
    N, B = 300, 16000
    P = rng.random((N, B)) + 0.05
    P /= P.sum(axis=1, keepdims=True)
    k = Kernel.load_dense(gpu_ctx, P, gemm_form="f16x3", tau=1e-3)
    try:
        out = torch.full((256, N), -1.0, dtype=torch.float32, device="cuda:0")
        with pytest.raises(DDError, match="DD_EINVAL.*fixed buffer holds"):
            k.batch_fields_noalloc(np.arange(256), "kl", out=out)
        torch.cuda.synchronize()
        assert bool((out == -1.0).all())
        assert _lib.DD_NOALLOC_SCRATCH_BYTES == 48 << 20
        _same(k, np.arange(64), "kl")
        _same(k, np.arange(10, 30), "kl")
    finally:
        k.free()
