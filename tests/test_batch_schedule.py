"""CPU model of the persistent batched launch's claim protocol.

One launch of G blocks (possibly more than fit the device at once, so some
start only after others have left).  A block repeatedly claims the next job
with an atomic increment of a counter and runs every pass of that job itself;
past the last job it leaves, incrementing an exit counter, and the block that
finds every other block gone resets both counters for the next launch.  No
block ever waits for another, so any interleaving terminates.

The model executes the protocol step by step (one atomic operation or one
unit of work per step) under random interleavings, random job lengths and
random residency limits, and checks: every job is run exactly once per
launch, jobs are claimed in list order, both counters are zero after every
launch (so a replayed graph starts clean), and the makespan of the claim
order (largest jobs first) stays within the list-scheduling bound
total / G + largest job.
"""
import numpy as np
import pytest


def run_launch(jobs, grid, resident, ctl, rng):
    """Execute one launch; returns (claims in time order, per-block busy
    time, makespan in steps)."""
    njobs = len(jobs)
    # block state: 'wait' (not yet resident), 'claim', ('work', job, left), 'done'
    state = ["wait"] * grid
    busy = [0] * grid
    claims = []
    started = 0
    step = 0
    runs = [0] * njobs
    while True:
        active = [b for b in range(grid) if state[b] not in ("wait", "done")]
        # residency: blocks start in index order as slots free up
        while started < grid and len(active) < resident:
            state[started] = "claim"
            active.append(started)
            started += 1
        if not active:
            break
        b = active[rng.integers(0, len(active))]
        st = state[b]
        if st == "claim":
            k = ctl["next"]  # atomic fetch-add
            ctl["next"] += 1
            if k >= njobs:
                before = ctl["exited"]  # atomic fetch-add
                ctl["exited"] += 1
                if before == grid - 1:
                    ctl["next"] = 0
                    ctl["exited"] = 0
                state[b] = "done"
            else:
                claims.append(k)
                state[b] = ("work", k, jobs[k])
        else:
            _, k, left = st
            busy[b] += 1
            if left == 1:
                runs[k] += 1
                state[b] = "claim"
            else:
                state[b] = ("work", k, left - 1)
        step += 1
    assert all(s == "done" for s in state)
    return claims, busy, runs


@pytest.mark.parametrize("seed", range(12))
def test_every_job_once_in_order_and_counters_reset(seed):
    rng = np.random.default_rng(seed)
    njobs = int(rng.integers(1, 60))
    grid = int(rng.integers(1, 24))
    resident = int(rng.integers(1, grid + 1))
    jobs = sorted((int(v) for v in rng.integers(1, 30, njobs)), reverse=True)
    ctl = {"next": 0, "exited": 0}
    for launch in range(3):  # replays of one captured launch
        claims, busy, runs = run_launch(jobs, grid, resident, ctl, rng)
        assert claims == list(range(njobs))
        assert runs == [1] * njobs
        assert ctl == {"next": 0, "exited": 0}, (launch, ctl)
        assert sum(busy) == sum(jobs)


def test_blocks_beyond_the_jobs_and_beyond_residency_leave():
    rng = np.random.default_rng(1)
    ctl = {"next": 0, "exited": 0}
    claims, busy, runs = run_launch([5, 3], grid=16, resident=4, ctl=ctl, rng=rng)
    assert runs == [1, 1] and ctl == {"next": 0, "exited": 0}


def list_schedule(jobs, workers):
    """Makespan when each free worker takes the next job of the list."""
    import heapq
    free = [0] * workers
    for j in jobs:
        t = heapq.heappop(free)
        heapq.heappush(free, t + j)
    return max(free)


@pytest.mark.parametrize("seed", range(6))
def test_largest_first_claims_are_near_balanced(seed):
    """With jobs claimed largest first, the last block finishes no later
    than the average load plus the largest job (list scheduling); for the
    benchmark's size mix (18 classes, 4096 problems, ~500 resident blocks)
    that is within a few percent of perfect balance."""
    rng = np.random.default_rng(seed)
    sizes = np.array([2 ** k for k in range(8, 17)] + [3 ** k for k in range(6, 11)]
                     + [5 ** k for k in range(4, 8)])
    work = sorted((int(v) for v in rng.choice(sizes, 4096)), reverse=True)
    for workers in (256, 512):
        mk = list_schedule(work, workers)
        avg = sum(work) / workers
        assert mk <= avg + work[0]
        assert mk <= 1.05 * avg, (workers, mk / avg)
