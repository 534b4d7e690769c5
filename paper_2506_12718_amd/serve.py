"""Serving loop: continuous batching of convolution requests on one GPU.

Requests (a grid shape, a filter id and an input) arrive over time.  The
server

* admits a request when a stream slot is free and its device memory fits
  the HBM budget (input/output buffers plus, on a cache miss, the plan with
  its filter spectrum);
* keeps plans, twiddles and filter spectra resident in an LRU cache keyed by
  (shape, filter), evicting only entries no in-flight request uses;
* runs every admitted request on one of S HIP streams, so requests that
  arrive while others are on the GPU overlap with them on the device;
* detects completions with stream events and records latency
  (arrival -> completion) and throughput;
* fails a request whose preparation or launch raises, or that cannot fit
  the budget even alone, records it in ``failed`` with the error, returns
  its slot, memory reservation and cache reference, and carries on
  (``GpuExecutor`` can inject such a failure: PAFC_FAULT_INJECT=prepare:N or
  launch:N fails the N-th call).

Results do not depend on what else runs: every convolution is the same
deterministic kernel sequence on its own buffers (the plan state it shares
with concurrent requests -- twiddles and spectrum -- is only read).

The executor is pluggable: ``GpuExecutor`` drives the C ABI through the
Python binding; the tests also drive the admission and cache logic with a
host-only fake executor.
"""
from __future__ import annotations

import collections
import heapq
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Optional


@dataclass
class Request:
    rid: int
    dims: tuple
    fid: int
    x: Any = None              # device tensor (GPU executor) or opaque token
    arrival: float = 0.0       # host clock, seconds
    start: float = 0.0         # admitted to a stream
    done: float = 0.0          # completion observed
    out: Any = None
    slot: int = -1
    meta: dict = field(default_factory=dict)
    error: Optional[str] = None   # set when the request failed


class PlanCache:
    """LRU cache of (shape, filter) -> prepared plan with a byte budget."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.entries = collections.OrderedDict()   # key -> [obj, bytes, refs]
        self.bytes = 0
        self.hits = 0
        self.misses = 0
        self.evictions = 0

    def get(self, key):
        """The entry for `key` (moved to the most recently used end), or None."""
        e = self.entries.get(key)
        if e is None:
            return None
        self.entries.move_to_end(key)
        return e

    def can_fit(self, extra: int, reserved: int) -> bool:
        """Can `extra` more bytes fit, evicting unused entries if needed?
        Entries with a reference (in flight, or pinned by the admission
        being decided) are not reclaimable."""
        free = self.budget - reserved - self.bytes
        if extra <= free:
            return True
        reclaim = sum(b for (o, b, r) in self.entries.values() if r == 0)
        return extra <= free + reclaim

    def recharge(self, entry, nbytes: int):
        """Set an entry's charge to the bytes its object really holds."""
        self.bytes += int(nbytes) - entry[1]
        entry[1] = int(nbytes)

    def make_room(self, extra: int, reserved: int, release: Callable):
        for key in list(self.entries.keys()):
            if self.budget - reserved - self.bytes >= extra:
                break
            obj, b, refs = self.entries[key]
            if refs == 0:
                del self.entries[key]
                self.bytes -= b
                self.evictions += 1
                release(obj)

    def put(self, key, obj, nbytes):
        self.misses += 1
        self.entries[key] = [obj, int(nbytes), 0]
        self.bytes += int(nbytes)
        return self.entries[key]


class Server:
    """Admission, caching and continuous batching over an executor."""

    def __init__(self, executor, budget_bytes=64 << 30, slots=4, clock=time.perf_counter):
        self.ex = executor
        self.cache = PlanCache(budget_bytes)
        self.slots = slots
        self.clock = clock
        self.pending = collections.deque()
        self.inflight = {}            # slot -> request
        self.free_slots = list(range(slots))
        self.reserved = 0             # bytes of in-flight request buffers
        self.completed = []
        self.failed = []
        self.max_inflight = 0
        self.lock = threading.Lock()

    # -- admission
    def submit(self, req: Request):
        with self.lock:
            self.pending.append(req)

    def _admit_one(self) -> bool:
        if not self.pending or not self.free_slots:
            return False
        req = self.pending[0]
        key = (tuple(req.dims), req.fid)
        entry = self.cache.get(key)
        need = self.ex.request_bytes(req)
        if entry is not None:
            # pin the hit while deciding, so that it is not counted as
            # memory that eviction could free for this very request
            entry[2] += 1
            extra, total = need, need + entry[1]
        else:
            est = self.ex.plan_bytes(req)
            extra, total = need + est, need + est
        if not self.cache.can_fit(extra, self.reserved):
            if entry is not None:
                entry[2] -= 1
            if self.inflight:
                return False  # wait for completions to free memory
            # nothing in flight: every other entry could be evicted, so the
            # request alone (with its plan) exceeds the budget
            self.pending.popleft()
            self._fail(req, "request %d (%d bytes with its plan) does not fit the HBM budget"
                       % (req.rid, total))
            return True
        self.pending.popleft()
        slot = self.free_slots.pop()
        self.cache.make_room(extra, self.reserved, self.ex.release_plan)
        if entry is None:
            try:
                plan = self.ex.prepare(req, slot)
            except Exception as e:  # nothing was cached or reserved yet
                self.free_slots.append(slot)
                self._fail(req, "prepare: %s" % e)
                return True
            entry = self.cache.put(key, plan, self.ex.plan_bytes(req))
            entry[2] += 1
            # charge what the plan really holds (the estimate is an upper
            # bound), then evict again in case it was not
            held = getattr(self.ex, "held_bytes", None)
            if held is not None:
                self.cache.recharge(entry, held(plan))
                self.cache.make_room(need, self.reserved, self.ex.release_plan)
        else:
            self.cache.hits += 1
        self.reserved += need
        req.slot = slot
        req.start = self.clock()
        try:
            self.ex.launch(req, entry[0], slot)
        except Exception as e:
            entry[2] -= 1
            self.reserved -= need
            self.free_slots.append(slot)
            self._fail(req, "launch: %s" % e)
            return True
        req.meta["entry"] = entry
        self.inflight[slot] = req
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        return True

    def _fail(self, req: Request, msg: str):
        req.error = msg
        req.done = self.clock()
        req.out = None
        self.failed.append(req)

    def _reap(self) -> int:
        n = 0
        for slot, req in list(self.inflight.items()):
            if self.ex.finished(req):
                req.done = self.clock()
                entry = req.meta.pop("entry")
                entry[2] -= 1
                self.reserved -= self.ex.request_bytes(req)
                self.ex.complete(req)
                del self.inflight[slot]
                self.free_slots.append(slot)
                self.completed.append(req)
                n += 1
        return n

    def step(self) -> int:
        """One scheduling round: reap completions, admit what fits."""
        with self.lock:
            n = self._reap()
            while self._admit_one():
                pass
        return n

    def idle(self) -> bool:
        with self.lock:
            return not self.pending and not self.inflight

    def drain(self, poll=2e-5):
        while not self.idle():
            if self.step() == 0:
                time.sleep(poll)


def run_open_loop(server: Server, requests, rate_hz: float, seed: int = 5,
                  make_input: Optional[Callable] = None, poll=2e-5):
    """Offer `requests` with Poisson arrivals at `rate_hz` (exponential gaps
    from a seeded generator) and serve them; returns the completed list."""
    import numpy as np
    rng = np.random.default_rng([seed, 1])
    gaps = rng.exponential(1.0 / rate_hz, size=len(requests))
    t0 = server.clock()
    due = t0
    i = 0
    while i < len(requests) or not server.idle():
        now = server.clock()
        while i < len(requests) and due <= now:
            req = requests[i]
            req.arrival = due
            if make_input is not None:
                req.x = make_input(req)
            server.submit(req)
            due += gaps[i]
            i += 1
        if server.step() == 0:
            time.sleep(poll)
    return server.completed


def run_closed_loop(server: Server, requests, make_input=None):
    """All requests offered at once (capacity measurement)."""
    t0 = server.clock()
    for r in requests:
        r.arrival = t0
        if make_input is not None:
            r.x = make_input(r)
        server.submit(r)
    server.drain()
    return server.completed


def latency_stats(reqs):
    import numpy as np
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {"n": len(reqs), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "throughput_per_s": len(reqs) / span if span > 0 else float("inf")}


class GpuExecutor:
    """Runs requests through the permutation-avoiding convolution library.

    prepare(): plan for the request's shape, with the request's Gaussian
    filter installed as its closed-form spectrum (pafc_set_symbol GAUSSIAN:
    no filter array is formed or transformed), enqueued on the slot's
    stream.  launch(): convolve on the slot's stream into a fresh output
    buffer, ordered after the stream that produced the input and after the
    plan's preparation.  finished(): the completion event has fired.
    """

    def __init__(self, dtype=None, sigma_of=None, slots=4):
        import torch
        import paper_2506_12718_amd as pafc
        self.torch = torch
        self.pafc = pafc
        self.dtype = dtype if dtype is not None else torch.complex64
        self.elem = 8 if self.dtype == torch.complex64 else 16
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.sigma_of = sigma_of
        self.prepared = 0
        # fault injection (tests of the server's failure handling):
        # PAFC_FAULT_INJECT=prepare:N or launch:N fails the N-th such call
        import os
        spec = os.environ.get("PAFC_FAULT_INJECT", "")
        kind, _, nth = spec.partition(":")
        self.fault = (kind, int(nth)) if kind in ("prepare", "launch") and nth.isdigit() else None
        self.calls = {"prepare": 0, "launch": 0}

    def _maybe_fail(self, kind):
        self.calls[kind] += 1
        if self.fault == (kind, self.calls[kind]):
            raise RuntimeError("injected %s failure (call %d)" % (kind, self.calls[kind]))

    def request_bytes(self, req):
        n = 1
        for d in req.dims:
            n *= d
        return n * self.elem  # the output buffer (the input is the caller's)

    def plan_bytes(self, req):
        """Upper bound of a plan's device memory before it exists: the
        spectrum (at most 1.25 N elements with the padding of ragged
        tile-major tiles), one N-element staging array, and the twiddles,
        index maps, symbol tables and descriptors (below 256 KiB for every
        served grid; a GPU test checks the bound against
        pafc_plan_device_bytes)."""
        n = 1
        for d in req.dims:
            n *= d
        return (9 * n * self.elem) // 4 + (256 << 10)

    def held_bytes(self, obj):
        """Device memory a prepared plan really holds (pafc_plan_device_bytes)."""
        return obj["bytes"]

    def prepare(self, req, slot):
        self._maybe_fail("prepare")
        torch = self.torch
        s = self.streams[slot]
        plan = self.pafc.Plan(req.dims, self.dtype, stream=s)
        try:
            plan.set_symbol("gaussian", self.sigma_of(req.dims, req.fid), stream=s)
        except Exception:
            plan.close()
            raise
        ev = torch.cuda.Event()
        ev.record(s)
        self.prepared += 1
        return {"plan": plan, "ready": ev, "bytes": plan.device_bytes}

    def release_plan(self, obj):
        obj["ready"].synchronize()
        obj["plan"].close()

    def launch(self, req, obj, slot):
        self._maybe_fail("launch")
        torch = self.torch
        s = self.streams[slot]
        s.wait_event(obj["ready"])
        # the input was produced on this thread's current stream: order the
        # convolution after it, and keep the allocator from reusing the
        # input's memory before the convolution has read it
        s.wait_stream(torch.cuda.current_stream())
        req.x.record_stream(s)
        with torch.cuda.stream(s):
            out = torch.empty(req.dims, dtype=self.dtype, device="cuda")
            obj["plan"].convolve(req.x, out=out, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        req.out = out
        req.meta["ev"] = ev

    def finished(self, req):
        return req.meta["ev"].query()

    def complete(self, req):
        req.meta.pop("ev", None)
