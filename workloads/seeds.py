"""Seed streams: every random draw comes from SeedSequence([seed_id, stream])."""

import numpy as np

SEED_STREAMS = {
    "geometry": 0,   # disk sample points, obstacle rectangles
    "targets": 1,
    "sources": 2,
    "arrivals": 3,   # serving inter-arrival times
    "domain": 4,     # serving: which resident domain a query goes to
    "sample": 5,     # vertex sample used for spot checks at full size
}


def rng(seed_id: int, stream) -> np.random.Generator:
    """Independent generator for (config, stream); ``stream`` is a name or int."""
    sid = SEED_STREAMS[stream] if isinstance(stream, str) else int(stream)
    return np.random.default_rng(np.random.SeedSequence([int(seed_id), sid]))


def targets_sources(seed_id: int, n: int, count: int):
    """``count`` seeded (target, source) interior-vertex pairs with source != target."""
    t = rng(seed_id, "targets").integers(0, n, size=count)
    rs = rng(seed_id, "sources")
    s = rs.integers(0, n, size=count)
    for i in range(count):
        while s[i] == t[i]:
            s[i] = rs.integers(0, n)
    return t.astype(np.int64), s.astype(np.int64)
