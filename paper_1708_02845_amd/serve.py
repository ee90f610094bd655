"""Continuous-batching service for path queries over several resident domains.

A query is (domain, source, target): the KL distance field of the target and
the steepest-descent path from the source.  The server keeps each domain's
kernel resident (admitted by its HBM footprint), queues queries per domain, and
whenever a domain has a free batch slot it launches the pending queries as one
batch: one KL contraction for all their targets, then one path launch for all
of them, then an asynchronous copy of the paths to pinned host memory, all on
that slot's stream.  Queries that arrive while a batch is on the GPU go into the
next batch as soon as a slot (and device memory for its fields) frees up;
batches of different domains and slots overlap on the device.  Completion is
observed by polling stream events; latency is arrival to completion on the host
clock.

The distance fields stay on the device; with ``keep_fields`` each finished
query keeps a device view of its own field (``Query.field``).
"""

import collections
import os
import time
import warnings
from dataclasses import dataclass, field

import numpy as np

from .api import Kernel

_STATUS = {0: "reached", 1: "stuck", 2: "max_steps"}


@dataclass
class Query:
    qid: int
    domain: str
    source: int
    target: int
    arrival: float                # host clock (perf_counter seconds)
    launched: float = None        # host clock when its batch was launched
    done: float = None
    gpu_ms: float = None          # its batch's time on the device (stream events)
    launch_host_ms: float = None  # host time spent enqueuing its batch
    path: list = None
    status: str = None
    rechecks: int = 0
    batch_size: int = 0
    field: object = field(default=None, repr=False)   # device view of its field

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival

    @property
    def wait(self):
        """Arrival to launch (queueing behind the domain's previous batch)."""
        return None if self.launched is None else self.launched - self.arrival


class _Slot:
    def __init__(self, torch, max_batch, max_steps):
        self.stream = torch.cuda.Stream()      # default priority
        self.busy = False
        self.queries = []
        self.event = None
        self.start = None
        self.launched = None
        self.launch_host_ms = None
        self.fields = None
        self.host_paths = torch.empty((max_batch, max_steps + 1), dtype=torch.int32,
                                      pin_memory=True)
        self.host_info = torch.empty((3, max_batch), dtype=torch.int32, pin_memory=True)


class _Domain:
    def __init__(self, name, kernel, slots):
        self.name = name
        self.kernel = kernel
        self.queue = collections.deque()
        self.slots = slots


class Server:
    """Resident domains, per-domain queues and continuous batching.

    Each slot is a stream.  HIP maps a process's streams onto a few hardware
    queues (GPU_MAX_HW_QUEUES, 4 by default, read when the runtime starts);
    streams beyond that share queues, and a batch then waits behind whatever
    another stream of its queue holds.  The default stream takes a queue too,
    so domains x slots + 1 queues give every slot one of its own
    (``queues_needed``); add_domain warns when the setting is below that.
    """

    @staticmethod
    def queues_needed(n_domains, slots_per_domain):
        return n_domains * slots_per_domain + 1


    def __init__(self, ctx, max_batch=64, slots_per_domain=1, max_steps=4000,
                 hbm_budget=None, gemm_form="f16x3", field_reserve=2, keep_fields=False):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.max_batch = int(max_batch)
        self.slots_per_domain = int(slots_per_domain)
        self.max_steps = int(max_steps)
        self.gemm_form = gemm_form
        self.field_reserve = field_reserve
        self.keep_fields = keep_fields
        free, _ = torch.cuda.mem_get_info(ctx.device)
        self.hbm_budget = int(free * 0.9) if hbm_budget is None else int(hbm_budget)
        self.hbm_used = 0
        self.domains = {}
        self.refused = []
        self.completed = []
        self.batch_sizes = collections.Counter()
        self._next_id = 0

    # ---- admission ----
    @staticmethod
    def launch_bytes(N, n, scratch):
        """Device bytes one batch of n queries holds while it runs: its fields
        (n x N FP32) and the scratch of its two calls (``scratch`` = (contraction,
        paths) bytes from Kernel.call_scratch)."""
        return n * N * 4 + scratch[0] + scratch[1]

    def domain_footprint(self, resident, N, scratch):
        """Resident bytes of a domain plus what its batch slots hold at full batches."""
        return resident + self.slots_per_domain * self.launch_bytes(N, self.max_batch, scratch)

    def add_domain(self, name, P, adjacency):
        """Load a domain if its footprint (resident bytes, and the fields and call
        scratch of full batches in every slot) fits the HBM budget; False if
        refused."""
        N, B = P.shape
        pre = Kernel.dense_footprint(N, B, gemm_form=self.gemm_form)
        if self.hbm_used + pre > self.hbm_budget:
            self.refused.append((name, pre))
            return False
        k = Kernel.load_dense(self.ctx, P, adjacency=adjacency, gemm_form=self.gemm_form)
        need = self.domain_footprint(k.footprint(), N, k.call_scratch(self.max_batch, "kl"))
        if self.hbm_used + need > self.hbm_budget:
            k.free()
            self.refused.append((name, need))
            return False
        queues = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
        wanted = self.queues_needed(len(self.domains) + 1, self.slots_per_domain)
        if wanted > queues:
            warnings.warn(f"{wanted} hardware queues would give every batch slot its own, "
                          f"GPU_MAX_HW_QUEUES is {queues}: slots share queues, and a short "
                          "batch can wait behind a long one of another domain")
        slots = [_Slot(self.torch, self.max_batch, self.max_steps)
                 for _ in range(self.slots_per_domain)]
        self.domains[name] = _Domain(name, k, slots)
        self.hbm_used += need
        return True

    def close(self):
        self.torch.cuda.synchronize()
        for d in self.domains.values():
            d.kernel.free()
        self.domains.clear()

    # ---- queries ----
    def submit(self, domain, source, target, arrival=None):
        d = self.domains[domain]
        if not (0 <= source < d.kernel.N and 0 <= target < d.kernel.N):
            raise ValueError("source/target out of range")
        q = Query(self._next_id, domain, int(source), int(target),
                  time.perf_counter() if arrival is None else arrival)
        self._next_id += 1
        d.queue.append(q)
        return q

    def pending(self):
        return sum(len(d.queue) for d in self.domains.values()) + \
            sum(1 for d in self.domains.values() for s in d.slots if s.busy)

    def _launch(self, d, slot):
        torch = self.torch
        n = min(self.max_batch, len(d.queue))
        N = d.kernel.N
        free, _ = torch.cuda.mem_get_info(self.ctx.device)
        if free < self.field_reserve * self.launch_bytes(N, n, d.kernel.call_scratch(n, "kl")):
            return False                              # wait for memory to free up
        qs = take_batch(d.queue, n)
        ts = np.array([q.target for q in qs], dtype=np.int32)
        ss = np.array([q.source for q in qs], dtype=np.int32)
        t_launch = time.perf_counter()
        try:
            with torch.cuda.stream(slot.stream):
                start = torch.cuda.Event(enable_timing=True)
                start.record(slot.stream)
                fields = torch.empty((n, N), dtype=torch.float32,
                                     device=f"cuda:{self.ctx.device}")
                _, bounds = d.kernel.batch_fields(ts, "kl", out=fields, stream=slot.stream)
                paths, lens, status, rechecks = d.kernel.trace_paths(
                    ss, ts, "kl", fields, bounds, self.max_steps, stream=slot.stream)
                slot.host_paths[:n].copy_(paths, non_blocking=True)
                slot.host_info[0, :n].copy_(lens, non_blocking=True)
                slot.host_info[1, :n].copy_(status, non_blocking=True)
                slot.host_info[2, :n].copy_(rechecks, non_blocking=True)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(slot.stream)
        except Exception:
            # the queries go back to the front of the queue, in order; with other
            # batches in flight the launch is retried once they free memory
            put_back(d.queue, qs)
            if any(s.busy for dom in self.domains.values() for s in dom.slots):
                return False
            raise
        slot.busy, slot.queries, slot.event, slot.fields = True, qs, ev, fields
        slot.start, slot.launched = start, t_launch
        slot.launch_host_ms = 1e3 * (time.perf_counter() - t_launch)
        self.batch_sizes[n] += 1
        return True

    def _finish(self, slot):
        now = time.perf_counter()
        info = slot.host_info.numpy()
        paths = slot.host_paths.numpy()
        gpu_ms = slot.start.elapsed_time(slot.event)
        for i, q in enumerate(slot.queries):
            q.path = paths[i, :info[0, i]].tolist()
            q.status = _STATUS[int(info[1, i])]
            q.rechecks = int(info[2, i])
            q.batch_size = len(slot.queries)
            q.launched, q.gpu_ms, q.launch_host_ms = slot.launched, gpu_ms, slot.launch_host_ms
            if self.keep_fields:
                q.field = slot.fields[i]
            q.done = now
            self.completed.append(q)
        slot.busy, slot.queries, slot.event = False, [], None

    def poll(self):
        """Finish completed batches, then launch into every free slot."""
        progressed = False
        for d in self.domains.values():
            for slot in d.slots:
                if slot.busy and slot.event.query():
                    self._finish(slot)
                    progressed = True
            for slot in d.slots:
                if not slot.busy and d.queue:
                    progressed |= self._launch(d, slot)
        return progressed

    def drain(self, timeout=600.0):
        t0 = time.perf_counter()
        while self.pending():
            if not self.poll():
                time.sleep(0)
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError("queries still pending")

    # ---- open-loop driver ----
    def run_open_loop(self, arrivals, timeout=600.0):
        """``arrivals``: list of (offset_s, domain, source, target), offsets ascending.

        Queries are submitted at their scheduled times (the arrival time used
        for latency is the scheduled one, so a slow loop cannot hide queueing).
        """
        t0 = time.perf_counter()
        i = 0
        out = []
        while i < len(arrivals) or self.pending():
            now = time.perf_counter()
            while i < len(arrivals) and t0 + arrivals[i][0] <= now:
                off, dom, s, t = arrivals[i]
                out.append(self.submit(dom, s, t, arrival=t0 + off))
                i += 1
            if not self.poll():
                time.sleep(0)
            if now - t0 > timeout:
                raise TimeoutError("open-loop run did not finish")
        return out


def take_batch(queue, n):
    """The first n queries of a domain queue, removed from it."""
    return [queue.popleft() for _ in range(n)]


def put_back(queue, qs):
    """Return a batch taken by take_batch to the front of its queue, in order."""
    queue.extendleft(reversed(qs))


def latency_summary(queries):
    lat = np.array([q.latency for q in queries]) * 1e3
    return {"queries": len(lat), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
            "mean_ms": float(lat.mean())}


def latency_breakdown(queries):
    """p50/p99/max (ms) of the parts of the latency: the wait from arrival to
    the launch of the query's batch, the host time of that launch, and the
    batch's time on the device (from its first to its last stream event,
    including any time its kernels wait for the device behind other streams'
    work), and the rest: the time before the batch's first event runs (behind
    earlier work in the same hardware queue) and until the host polls the
    completion."""
    out = {}
    rest = [1e3 * q.latency - 1e3 * q.wait - q.launch_host_ms - q.gpu_ms for q in queries]
    for name, vals in (("wait", [1e3 * q.wait for q in queries]),
                       ("launch_host", [q.launch_host_ms for q in queries]),
                       ("gpu", [q.gpu_ms for q in queries]), ("rest", rest)):
        v = np.array(vals, dtype=np.float64)
        out[name] = {"p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99)),
                     "max_ms": float(v.max())}
    return out
