"""Admission, caching and continuous-batching logic of the server, driven on
the CPU by a fake executor (no GPU)."""
import pytest

from paper_2506_12718_amd.serve import Request, Server, latency_stats, run_closed_loop


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-6
        return self.t


class FakeExecutor:
    """A request finishes `polls` finished() queries after launch."""

    def __init__(self, polls=3, elem=8):
        self.polls = polls
        self.elem = elem
        self.prepared = []
        self.released = []
        self.live_plans = set()
        self.max_bytes_seen = 0

    def _n(self, req):
        n = 1
        for d in req.dims:
            n *= d
        return n

    def request_bytes(self, req):
        return self._n(req) * self.elem

    def plan_bytes(self, req):
        return self._n(req) * self.elem

    def prepare(self, req, slot):
        key = (tuple(req.dims), req.fid)
        self.prepared.append(key)
        self.live_plans.add(key)
        return {"key": key}

    def release_plan(self, obj):
        self.released.append(obj["key"])
        self.live_plans.discard(obj["key"])

    def launch(self, req, obj, slot):
        assert obj["key"] in self.live_plans  # never run on an evicted plan
        req.meta["left"] = self.polls
        req.out = ("y", req.rid)

    def finished(self, req):
        req.meta["left"] -= 1
        return req.meta["left"] <= 0

    def complete(self, req):
        pass


def mk(n, dims=(64, 64), fid=0):
    return [Request(rid=i, dims=dims, fid=fid) for i in range(n)]


def test_slots_bound_inflight_and_fifo():
    ex = FakeExecutor()
    s = Server(ex, budget_bytes=1 << 40, slots=3, clock=FakeClock())
    reqs = mk(20)
    done = run_closed_loop(s, reqs)
    assert len(done) == 20
    assert s.max_inflight == 3
    assert sorted(r.rid for r in done) == list(range(20))
    starts = [r.start for r in sorted(done, key=lambda r: r.rid)]
    assert starts == sorted(starts)  # admitted in arrival order


def test_plan_cache_hits_when_budget_allows():
    ex = FakeExecutor()
    s = Server(ex, budget_bytes=1 << 40, slots=4, clock=FakeClock())
    reqs = [Request(rid=i, dims=(32, 32), fid=i % 3) for i in range(30)]
    run_closed_loop(s, reqs)
    assert len(ex.prepared) == 3
    assert s.cache.hits == 27 and s.cache.evictions == 0


def test_budget_forces_eviction_and_queueing():
    ex = FakeExecutor(polls=2)
    n = 64 * 64 * 8
    # room for two plans and two request buffers
    s = Server(ex, budget_bytes=4 * n, slots=4, clock=FakeClock())
    reqs = [Request(rid=i, dims=(64, 64), fid=i % 4) for i in range(24)]
    done = run_closed_loop(s, reqs)
    assert len(done) == 24
    assert s.cache.evictions > 0
    assert len(ex.prepared) > 4
    assert s.max_inflight <= 2
    assert s.cache.bytes + s.reserved <= 4 * n


def test_entries_in_use_are_never_evicted():
    ex = FakeExecutor(polls=5)
    n = 32 * 32 * 8
    s = Server(ex, budget_bytes=3 * n, slots=2, clock=FakeClock())
    reqs = [Request(rid=i, dims=(32, 32), fid=i % 5) for i in range(40)]
    run_closed_loop(s, reqs)  # FakeExecutor.launch asserts the plan is live
    assert len(s.completed) == 40


def test_request_larger_than_budget_fails_alone():
    """A request that cannot fit the budget even alone fails; the requests
    around it are served."""
    ex = FakeExecutor()
    s = Server(ex, budget_bytes=3 * 64 * 64 * 8, slots=2, clock=FakeClock())
    reqs = [Request(rid=0, dims=(32, 32), fid=0), Request(rid=1, dims=(256, 256), fid=1),
            Request(rid=2, dims=(32, 32), fid=0)]
    run_closed_loop(s, reqs)
    assert [r.rid for r in s.failed] == [1] and "budget" in s.failed[0].error
    assert sorted(r.rid for r in s.completed) == [0, 2]
    assert s.reserved == 0


class FailingExecutor(FakeExecutor):
    """prepare() or launch() raises on chosen requests (an allocation or a
    launch that fails)."""

    def __init__(self, fail_prepare=(), fail_launch=()):
        super().__init__()
        self.fail_prepare, self.fail_launch = set(fail_prepare), set(fail_launch)

    def prepare(self, req, slot):
        if req.rid in self.fail_prepare:
            raise RuntimeError("out of device memory")
        return super().prepare(req, slot)

    def launch(self, req, obj, slot):
        if req.rid in self.fail_launch:
            raise RuntimeError("launch failed")
        return super().launch(req, obj, slot)


def test_failed_prepare_and_launch_do_not_stop_the_server():
    ex = FailingExecutor(fail_prepare={3}, fail_launch={5, 6})
    s = Server(ex, budget_bytes=1 << 30, slots=2, clock=FakeClock())
    reqs = [Request(rid=i, dims=(16, 16 + (i % 4)), fid=i % 4) for i in range(20)]
    run_closed_loop(s, reqs)
    assert sorted(r.rid for r in s.failed) == [3, 5, 6]
    assert all(r.error for r in s.failed) and all(r.out is None for r in s.failed)
    assert sorted(r.rid for r in s.completed) == [i for i in range(20) if i not in (3, 5, 6)]
    # nothing leaked: no reservation, no reference, every slot free
    assert s.reserved == 0 and not s.inflight and sorted(s.free_slots) == [0, 1]
    assert all(e[2] == 0 for e in s.cache.entries.values())
    # the failed preparation left no cache entry behind; a later request of
    # that shape prepared its plan again
    assert ex.prepared.count(((16, 19), 3)) == 1


def test_latency_stats():
    reqs = mk(4)
    for i, r in enumerate(reqs):
        r.arrival, r.done = float(i), float(i) + 0.001 * (i + 1)
    st = latency_stats(reqs)
    assert st["n"] == 4 and abs(st["p50_ms"] - 2.5) < 1e-9


class SizedExecutor(FakeExecutor):
    """Plans charged at an estimate before planning and at what they really
    hold afterwards (held_bytes), as the GPU executor does."""

    def plan_bytes(self, req):
        return 2 * self._n(req) * self.elem

    def held_bytes(self, obj):
        n = 1
        for d in obj["key"][0]:
            n *= d
        return n * self.elem + 100


def test_budget_holds_after_every_step_with_hits():
    """reserved + cached bytes never exceed the budget: a cache hit is pinned
    while its admission is decided, so it is not counted as memory that
    evicting it could free, and hits evict other unused entries when needed.
    The sequence interleaves a small and a large grid so that hits on the
    small plan arrive while the large one is in flight."""
    import random
    for executor in (FakeExecutor, SizedExecutor):
        rnd = random.Random(3)
        ex = executor(polls=4)
        small, large = (32, 32), (64, 64)
        n_s, n_l = 32 * 32 * 8, 64 * 64 * 8
        budget = 2 * n_l + 2 * n_s + n_l // 2
        s = Server(ex, budget_bytes=budget, slots=3, clock=FakeClock())
        reqs = [Request(rid=i, dims=rnd.choice([small, large]), fid=rnd.randrange(3))
                for i in range(200)]
        for r in reqs:
            s.submit(r)
        steps = 0
        while not s.idle():
            s.step()
            steps += 1
            assert s.reserved + s.cache.bytes <= budget, (steps, s.reserved, s.cache.bytes)
            assert steps < 100000
        assert len(s.completed) + len(s.failed) == len(reqs)
        assert not s.failed
        assert s.cache.hits > 0 and s.cache.evictions > 0
        assert s.cache.hits + s.cache.misses == len(reqs)


def test_request_that_cannot_fit_alone_fails():
    ex = FakeExecutor()
    s = Server(ex, budget_bytes=64 * 64 * 8, slots=2, clock=FakeClock())
    reqs = [Request(rid=0, dims=(64, 64), fid=0), Request(rid=1, dims=(16, 16), fid=0)]
    done = run_closed_loop(s, reqs)
    assert [r.rid for r in s.failed] == [0] and "does not fit" in s.failed[0].error
    assert [r.rid for r in done] == [1]
