"""Serving policy on the CPU: a fake executor with a fake clock stands in for
the GPU (admission by footprint, bypass with aging, cancellation, failures,
cross-request batches and out-of-order completion)."""
import pytest

from paper_1706_08563_amd.serve import Request, Scheduler, serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-3)


class FakeExecutor:
    """Build time and footprint come from the request; synthesis of a batch
    takes 1 ms per chunk."""

    def __init__(self, clock, fail_ids=()):
        self.clock = clock
        self.inflight = []
        self.batches = []
        self.fail_ids = set(fail_ids)
        self.live = 0
        self.max_live = 0

    def plan(self, req):
        req.chunks_total = req.info.get("chunks", 1)
        return req.info["foot"]

    def start(self, req):
        if req.rid in self.fail_ids:
            raise MemoryError("fake allocation failure")
        req.info["built_at"] = self.clock() + req.info.get("build", 0.01)
        self.live += req.footprint
        self.max_live = max(self.max_live, self.live)

    def is_built(self, req):
        return self.clock() >= req.info["built_at"]

    def chunks_left(self, req):
        return range(req.chunks_issued, req.chunks_total)

    def synthesize(self, batch):
        for req, _ in batch:
            req.chunks_issued += 1
        self.batches.append([(r.rid, c) for r, c in batch])
        self.inflight.append((self.clock() + 1e-3 * len(batch), list(batch)))

    def finished_batches(self):
        done = []
        while self.inflight and self.inflight[0][0] <= self.clock():
            done.append(self.inflight.pop(0)[1])
        return done

    def collect(self, req):
        req.result = req.rid
        self.live -= req.footprint


def _req(rid, t, foot, build=0.01, chunks=1):
    r = Request(rid, t, 256, 2, 10, (4, 4), rid)
    r.info.update(foot=foot, build=build, chunks=chunks)
    return r


def _run(reqs, capacity, **kw):
    clk = Clock()
    ex = FakeExecutor(clk, kw.pop("fail_ids", ()))
    sched = Scheduler(capacity, **kw)
    serve(reqs, ex, sched, clock=clk, sleep=clk.sleep)
    return sched, ex


def test_admission_never_exceeds_budget_and_all_complete():
    reqs = [_req(i, 0.001 * i, foot=10 + (i % 5) * 20) for i in range(40)]
    sched, ex = _run(reqs, capacity=100, max_building=3)
    assert len(sched.done) == 40 and not sched.rejected
    assert sched.peak_used <= 100 and ex.max_live <= 100
    assert sched.used == 0
    assert all(r.latency >= 0 and r.t_admit >= r.arrival for r in reqs)


def test_over_budget_request_is_rejected():
    reqs = [_req(0, 0.0, foot=50), _req(1, 0.0, foot=500), _req(2, 0.0, foot=50)]
    sched, _ = _run(reqs, capacity=100)
    assert [r.rid for r in sched.rejected] == [1] and reqs[1].state == "rejected"
    assert {r.rid for r in sched.done} == {0, 2}


def test_bypass_then_aging_prevents_starvation():
    # one large request behind a long stream of small ones that keep the budget busy
    reqs = [_req(0, 0.0, foot=60, build=0.05)]
    reqs += [_req(1, 0.0005, foot=90, build=0.02)]
    reqs += [_req(i, 0.001 + 0.002 * i, foot=30, build=0.02) for i in range(2, 60)]
    sched, _ = _run(reqs, capacity=100, max_building=8, aging=3)
    big = reqs[1]
    assert big.state == "done"
    # it was passed by some small requests, but not by all of them
    passed = [r for r in reqs[2:] if r.t_admit < big.t_admit]
    assert 0 < len(passed) < 58


def test_cancel_queued_request():
    sched = Scheduler(100)
    a, b = _req(0, 0.0, 80), _req(1, 0.0, 80)
    sched.arrive(a, 80)
    sched.arrive(b, 80)
    assert sched.admit(0.0) == [a]
    assert sched.cancel(b) and b.state == "cancelled"
    assert not sched.cancel(a)          # already admitted
    assert sched.queue == []


def test_allocation_failure_releases_budget():
    reqs = [_req(i, 0.0, foot=40) for i in range(5)]
    sched, _ = _run(reqs, capacity=100, fail_ids={1, 3})
    assert {r.rid for r in sched.done} == {0, 2, 4}
    assert {r.rid for r in sched.rejected} == {1, 3}
    assert all(r.state == "failed" and "allocation" in r.info["error"] for r in (reqs[1], reqs[3]))
    assert sched.used == 0


def test_batches_mix_requests_and_respect_max_jobs():
    reqs = [_req(i, 0.0, foot=10, chunks=3, build=0.01) for i in range(6)]
    sched, ex = _run(reqs, capacity=100, max_building=6, max_jobs=5)
    assert all(len(b) <= 5 for b in ex.batches)
    assert any(len({rid for rid, _ in b}) > 1 for b in ex.batches)
    issued = sorted(x for b in ex.batches for x in b)
    assert issued == sorted((i, c) for i in range(6) for c in range(3))


def test_out_of_order_completion():
    # a slow early request and a fast later one: the later one finishes first
    reqs = [_req(0, 0.0, foot=40, build=0.5), _req(1, 0.01, foot=40, build=0.01)]
    sched, _ = _run(reqs, capacity=100)
    assert reqs[1].t_done < reqs[0].t_done
    assert [r.rid for r in sched.done] == [1, 0]


def test_batches_take_at_most_jobs_per_request_chunks_of_one_request():
    reqs = [_req(0, 0.0, foot=10, chunks=11), _req(1, 0.0, foot=10, chunks=2)]
    sched, ex = _run(reqs, capacity=100, max_building=2, max_jobs=24, jobs_per_request=3)
    for b in ex.batches:
        for rid in {r for r, _ in b}:
            assert sum(1 for r, _ in b if r == rid) <= 3
    issued = sorted(x for b in ex.batches for x in b)
    assert issued == sorted([(0, c) for c in range(11)] + [(1, c) for c in range(2)])
    assert len(sched.done) == 2


def test_small_requests_are_batched_before_a_large_one_and_it_is_not_starved():
    """Least remaining work first: the chunks of small requests that arrive
    while a large request's chunks wait go out first, each batch's cost stays
    within batch_cost (a large chunk goes alone), and aging lets the large
    request through while small ones keep arriving."""
    big = _req(0, 0.0, foot=10, chunks=6)
    big.info["cost"] = 100.0
    small = [_req(i, 0.0005 * i, foot=10, chunks=1) for i in range(1, 40)]
    reqs = [big] + small

    class CostExecutor(FakeExecutor):
        def plan(self, req):
            req.chunk_cost = req.info.get("cost", 1.0)
            return super().plan(req)

    clk = Clock()
    ex = CostExecutor(clk)
    sched = Scheduler(1000, max_building=40, max_jobs=8, aging=4, batch_cost=100.0)
    serve(reqs, ex, sched, clock=clk, sleep=clk.sleep)
    assert len(sched.done) == 40
    for b in ex.batches:
        if any(rid == 0 for rid, _ in b):
            assert len(b) == 1                      # a large chunk fills a batch by itself
        else:
            assert len(b) <= 8
    # the first small requests finish before the large one
    assert sum(1 for r in small if r.t_done < big.t_done) > 10
    # and the large one is not left to the end: aging gives it batches while
    # small requests are still being served
    first_big = min(i for i, b in enumerate(ex.batches) if any(rid == 0 for rid, _ in b))
    last_small = max(i for i, b in enumerate(ex.batches) if any(rid != 0 for rid, _ in b))
    assert first_big < last_small


def test_request_that_cannot_start_waits_and_budget_is_released():
    """An admitted request whose device memory is not free yet goes back to
    the queue (budget released) and starts later; nothing is lost."""
    class Refusing(FakeExecutor):
        def __init__(self, clock):
            super().__init__(clock)
            self.refused = 0

        def start(self, req):
            if req.rid == 1 and self.refused < 3:
                self.refused += 1
                return False
            super().start(req)
            return True

    reqs = [_req(i, 0.0, foot=30) for i in range(4)]
    clk = Clock()
    ex = Refusing(clk)
    sched = Scheduler(100, max_building=4)
    serve(reqs, ex, sched, clock=clk, sleep=clk.sleep)
    assert ex.refused == 3
    assert {r.rid for r in sched.done} == {0, 1, 2, 3} and not sched.rejected
    assert sched.used == 0 and sched.peak_used <= 100


def test_smaller_builds_go_first_and_large_ones_are_not_held_forever():
    """A build with much more work left than the smallest one waits, until it
    has been held build_hold seconds; builds within build_ratio proceed."""
    sched = Scheduler(1000, build_ratio=4.0, build_hold=2.0)
    big, small, mid = _req(0, 0.0, 10), _req(1, 0.0, 10), _req(2, 0.0, 10)
    left = {0: 1000.0, 1: 10.0, 2: 30.0}
    sched.building = [big, small, mid]
    f = lambda r: left[r.rid]            # noqa: E731
    assert sched.may_build(small, 0.0, f) and sched.may_build(mid, 0.0, f)
    assert not sched.may_build(big, 0.0, f) and not sched.may_build(big, 1.9, f)
    assert sched.may_build(big, 2.0, f)          # held long enough
    assert not sched.may_build(big, 2.5, f)      # and held again from now on
    sched.building = [big]
    assert sched.may_build(big, 2.6, f)          # alone: nothing smaller to wait for
    left[1] = 0.0                                # a build with every part issued
    sched.building = [big, small]
    assert sched.may_build(big, 2.7, f) and sched.may_build(small, 2.7, f)


class RangedExecutor(FakeExecutor):
    """Builds in parts of 1 ms each on one serial build queue; the next part
    of a request is issued only after its previous part has finished."""

    def __init__(self, clock):
        super().__init__(clock)
        self.busy_until = 0.0

    def _issue(self, req):
        start = max(self.clock(), self.busy_until)
        self.busy_until = start + 1e-3
        req.info["part_done"] = self.busy_until
        req.info["parts_left"] -= 1

    def start(self, req):
        req.info["parts_left"] = req.info["parts"]
        self._issue(req)

    def is_built(self, req, may_issue=True):
        if self.clock() < req.info["part_done"]:
            return False
        if req.info["parts_left"]:
            if may_issue:
                self._issue(req)
            return False
        return True

    def build_left(self, req):
        return float(req.info["parts_left"])


def test_build_pacing_in_the_serving_loop():
    """With pacing, a small build admitted beside a large one is built on
    its own; without it the two interleave part by part.  Both finish."""
    def run(**kw):
        clk = Clock()
        big, small = _req(0, 0.0, 10), _req(1, 0.0055, 10)
        big.info["parts"], small.info["parts"] = 40, 3
        sched = Scheduler(1000, **kw)
        serve([big, small], RangedExecutor(clk), sched, clock=clk, sleep=clk.sleep)
        assert {r.rid for r in sched.done} == {0, 1}
        return big.t_built, small.t_built - small.t_admit
    big_free, small_free = run()
    big_paced, small_paced = run(build_ratio=4.0, build_hold=1.0)
    assert small_paced < small_free
    assert big_paced >= big_free


class _Buf:
    def __init__(self, n):
        self.n = n

    def numel(self):
        return self.n


class _Ev:
    def __init__(self, done=False):
        self.done = done

    def query(self):
        return self.done


def test_device_arena_best_fit_coalescing_and_events():
    """The arena gives disjoint aligned ranges, picks the smallest free range
    that fits, merges neighbours on release and hands the pending events of a
    released range to its next owner (completed events are dropped)."""
    from paper_1706_08563_amd.serve import DeviceArena
    A = DeviceArena.ALIGN
    ar = DeviceArena(_Buf(10 * A))
    a = ar.alloc(3 * A)
    b = ar.alloc(1)                                  # rounded up to one alignment unit
    c = ar.alloc(2 * A)
    assert [x[:2] for x in (a, b, c)] == [(0, 3 * A), (3 * A, A), (4 * A, 2 * A)]
    assert ar.alloc(5 * A) is None and ar.free_bytes == 4 * A
    pending, finished = _Ev(False), _Ev(True)
    ar.release(b[0], b[1], pending)                  # a 1-unit hole at 3A
    ar.release(a[0], a[1], finished)                 # merges with it: [0, 4A)
    assert ar.free[0][:2] == [0, 4 * A] and ar.free[0][2] == [pending]
    d = ar.alloc(4 * A)                              # two free ranges of 4A: the first is taken
    assert d[:2] == (0, 4 * A) and d[2] == [pending]
    e = ar.alloc(A)                                  # from the tail [6A, 10A)
    assert e[:2] == (6 * A, A) and e[2] == []
    for r in (c, d, e):
        ar.release(r[0], r[1])
    assert len(ar.free) == 1 and ar.free[0][:2] == [0, 10 * A]
    # best fit prefers the smaller of two holes
    x, y, z = ar.alloc(2 * A), ar.alloc(A), ar.alloc(3 * A)
    ar.release(x[0], x[1])
    ar.release(z[0], z[1])                           # holes: 2A at 0 and 7A from 3A (merged with the tail)
    assert ar.alloc(2 * A)[:2] == (0, 2 * A)


def test_device_arena_random_alloc_release_never_overlaps():
    """A seeded random sequence of allocations and releases: live ranges
    never overlap, stay inside the buffer, and live + free bytes always equal
    the buffer; after releasing everything one free range remains."""
    import random
    from paper_1706_08563_amd.serve import DeviceArena
    A = DeviceArena.ALIGN
    cap = 64 * A
    ar = DeviceArena(_Buf(cap))
    rng = random.Random(7)
    live = []
    for _ in range(2000):
        if live and (rng.random() < 0.45 or ar.free_bytes < A):
            off, n, _ = live.pop(rng.randrange(len(live)))
            ar.release(off, n, _Ev(rng.random() < 0.5))
        else:
            r = ar.alloc(rng.randint(1, 9 * A))
            if r is not None:
                off, n, evs = r
                assert off % A == 0 and n % A == 0 and 0 <= off and off + n <= cap
                assert all(not e.query() for e in evs)
                for o, m, _ in live:
                    assert off + n <= o or o + m <= off
                live.append(r)
        assert sum(n for _, n, _ in live) + ar.free_bytes == cap
        offs = [f[0] for f in ar.free]
        assert offs == sorted(offs)
        assert all(a[0] + a[1] < b[0] for a, b in zip(ar.free, ar.free[1:]))   # neighbours merged
    for off, n, _ in live:
        ar.release(off, n)
    assert len(ar.free) == 1 and ar.free[0][:2] == [0, cap]
