"""Seeded open-loop arrivals for the serving workload."""

from .seeds import rng


def poisson_arrivals(seed_id, domains, qps, duration):
    """Seeded open-loop arrivals: exponential gaps at ``qps``, uniform domain, s != t.

    ``domains``: list of (name, N).
    """
    ga, gd, gs = rng(seed_id, "arrivals"), rng(seed_id, "domain"), rng(seed_id, "sources")
    out = []
    t = 0.0
    while True:
        t += ga.exponential(1.0 / qps)
        if t > duration:
            break
        name, N = domains[int(gd.integers(len(domains)))]
        tgt = int(gs.integers(N))
        src = int(gs.integers(N))
        while src == tgt:
            src = int(gs.integers(N))
        out.append((t, name, src, tgt))
    return out
