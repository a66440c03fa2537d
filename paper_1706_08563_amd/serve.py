"""Continuous-batching request loop for PRISM simulations on one GPU.

Requests (a cell, grid size, interpolation factor, slice count and probe
scan each) arrive over time.  The loop

* admits a request when its HBM footprint fits the free budget (the analogue
  of choosing a memory model from a device-memory estimate, "Streaming Data
  for Very Large Simulations"), first come first served with bypass: a later
  request that fits may pass a waiting one, until the waiting one has been
  passed `aging` times;
* builds each admitted request's potential and S-matrix on that request's own
  HIP stream, so builds of different requests overlap on the device; a
  build is issued one beam range at a time (about 2^30 beam-pixels each,
  `prism_build_smatrix_range`), the next range only once the previous one
  has finished, so other requests' work never queues behind a whole large
  build on a shared hardware queue;
* carves the large device buffers (S-matrices, workspaces) from one arena
  allocated once, since device memory returned to the driver and allocated
  again is cleared first (seconds for a large S-matrix);
* keeps every built S-matrix resident until its probes are done, and
  synthesises probes of all built requests together: each scheduling step
  issues one batched synthesis (prism_probe_outputs_batched) over up to
  `max_jobs` probe chunks from different requests on a synthesis stream;
* returns each request's detector outputs and records its latency from
  arrival to host-side result.

`Scheduler` holds the policy and no device state, so it is exercised on the
CPU with a fake executor; `GpuExecutor` drives the library.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------- requests --
@dataclass
class Request:
    rid: int
    arrival: float                 # seconds since the start of the stream
    n: int                         # grid side
    f: int                         # interpolation factor
    n_slices: int
    scan: tuple                    # (nx, ny)
    seed: int
    E0: float = 200e3
    alpha_max: float = 0.02
    dalpha: float = 1e-3
    pixel: float = 0.09765625      # A per pixel (cell side = n * pixel)
    # the specimen: (positions [n, 3] A, species index [n], species list) or a
    # callable returning that tuple (called when the request is admitted)
    sample: object = None
    # filled while serving
    state: str = "queued"          # queued -> building -> built -> done | rejected | cancelled
    footprint: int = 0
    skipped: int = 0
    chunks_total: int = 0
    chunks_done: int = 0
    chunks_issued: int = 0
    chunk_cost: float = 1.0        # synthesis work of one probe chunk (any unit, set by the executor)
    passed: int = 0                # batches formed without this request while it had chunks left
    held_since: float = math.nan   # when its build was first held back behind smaller builds
    t_admit: float = math.nan
    t_built: float = math.nan
    t_done: float = math.nan
    result: object = None
    info: dict = field(default_factory=dict)

    @property
    def cell(self):
        L = self.n * self.pixel
        return (L, L, 2.0 * self.n_slices)

    @property
    def n_probes(self):
        return self.scan[0] * self.scan[1]

    @property
    def latency(self):
        return self.t_done - self.arrival


# --------------------------------------------------------------- scheduler --
class Scheduler:
    """Admission, bookkeeping and batch formation; no device state."""

    def __init__(self, capacity: int, max_building: int = 4, max_jobs: int = 24, aging: int = 8,
                 jobs_per_request: int = 4, batch_cost: float | None = None, build_ratio: float = math.inf,
                 build_hold: float = 2.0):
        self.capacity = int(capacity)
        self.used = 0
        self.max_building = max_building
        self.max_jobs = max_jobs
        self.aging = aging
        # probe chunks of one request per batch (bounds a request's share of
        # the batch workspace, which its footprint accounts for)
        self.jobs_per_request = jobs_per_request
        # a batch takes further chunks only while its summed chunk_cost stays
        # within this (None: no limit)
        self.batch_cost = batch_cost
        # a build whose remaining work exceeds build_ratio x the smallest
        # remaining build issues no further part until the smaller ones are
        # done, or until it has been held build_hold seconds (inf: builds are
        # never held; on mixed streams of 256^2-2048^2 grids at load 0.8 a
        # ratio of 4 lowered the median latency but raised the 99th
        # percentile by about 2 % at the same throughput)
        self.build_ratio = build_ratio
        self.build_hold = build_hold
        self.queue: list[Request] = []
        self.building: list[Request] = []
        self.built: list[Request] = []
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.peak_used = 0

    def arrive(self, req: Request, footprint: int):
        req.footprint = int(footprint)
        if req.footprint > self.capacity:
            req.state = "rejected"
            self.rejected.append(req)
            return False
        self.queue.append(req)
        return True

    def cancel(self, req: Request) -> bool:
        """Cancel a request that has not been admitted yet."""
        if req in self.queue:
            self.queue.remove(req)
            req.state = "cancelled"
            return True
        return False

    def admit(self, now: float) -> list:
        """Requests to start now: first come first served; a later request that
        fits may pass waiting ones, each of which counts that bypass; once a
        waiting request has been passed `aging` times nobody passes it."""
        out = []
        waiting = []                    # earlier requests that did not fit
        for req in list(self.queue):
            if len(self.building) + len(out) >= self.max_building:
                break
            if self.used + req.footprint <= self.capacity:
                if any(w.skipped >= self.aging for w in waiting):
                    break
                for w in waiting:
                    w.skipped += 1
                self.queue.remove(req)
                self.used += req.footprint
                self.peak_used = max(self.peak_used, self.used)
                req.state = "building"
                req.t_admit = now
                out.append(req)
            else:
                waiting.append(req)
        self.building.extend(out)
        return out

    def defer(self, req: Request):
        """Return an admitted request whose device work could not start yet
        (device memory held elsewhere) to the queue, in arrival order."""
        if req in self.building:
            self.building.remove(req)
            self.used -= req.footprint
        req.state = "queued"
        req.t_admit = math.nan
        k = 0
        while k < len(self.queue) and self.queue[k].arrival <= req.arrival:
            k += 1
        self.queue.insert(k, req)

    def fail(self, req: Request, now: float, reason: str):
        """A request whose device work could not start (e.g. allocation failure)."""
        if req in self.building:
            self.building.remove(req)
            self.used -= req.footprint
        req.state = "failed"
        req.t_done = now
        req.info["error"] = reason
        self.rejected.append(req)

    def may_build(self, req: Request, now: float, build_left) -> bool:
        """Whether a building request may issue the next part of its build:
        smaller builds go first (`build_left(req)` is its remaining work)."""
        mine = build_left(req)
        # builds whose every part is issued hold nobody back
        smallest = min((x for x in (build_left(r) for r in self.building) if x > 0), default=0.0)
        if mine <= 0 or mine <= self.build_ratio * smallest:
            req.held_since = math.nan
            return True
        if math.isnan(req.held_since):
            req.held_since = now
        if now - req.held_since >= self.build_hold:
            req.held_since = math.nan
            return True
        return False

    def mark_built(self, req: Request, now: float):
        self.building.remove(req)
        req.state = "built"
        req.t_built = now
        self.built.append(req)

    def next_batch(self, chunks_left) -> list:
        """Up to max_jobs (request, chunk index) pairs from built requests, at
        most jobs_per_request per request.  Requests with the least remaining
        synthesis work (chunk_cost x chunks left) come first, except that a
        request passed over `aging` times goes before all others (oldest
        first); with batch_cost set, a chunk joins a non-empty batch only
        while the batch's cost stays within it, so the chunks of a large
        request form batches of their own instead of holding small requests'
        chunks back.  `chunks_left(req)` gives the chunks not yet issued."""
        ready = [r for r in self.built if len(chunks_left(r)) > 0]

        def key(r):
            starved = r.passed >= self.aging
            return (not starved, r.arrival if starved else r.chunk_cost * len(chunks_left(r)), r.arrival)

        batch, cost = [], 0.0
        for req in sorted(ready, key=key):
            for k, c in enumerate(chunks_left(req)):
                if len(batch) >= self.max_jobs or k >= self.jobs_per_request:
                    break
                if batch and self.batch_cost is not None and cost + req.chunk_cost > self.batch_cost:
                    break
                batch.append((req, c))
                cost += req.chunk_cost
        taken = {id(r) for r, _ in batch}
        for r in ready:
            r.passed = 0 if id(r) in taken else r.passed + 1
        return batch

    def chunk_done(self, req: Request, now: float) -> bool:
        req.chunks_done += 1
        if req.chunks_done == req.chunks_total:
            self.built.remove(req)
            self.used -= req.footprint
            req.state = "done"
            req.t_done = now
            self.done.append(req)
            return True
        return False

    @property
    def idle(self):
        return not (self.queue or self.building or self.built)


# --------------------------------------------------------------- GPU side --
class DeviceArena:
    """Best-fit sub-allocator over one device buffer, for the large buffers
    of the requests (S-matrices, build and synthesis workspaces).  Device
    memory that the driver takes back and hands out again is cleared first,
    seconds for the size of a large S-matrix (5.6 s for 168 GB) during which
    the GPU runs out of queued work; carving every large buffer from one
    allocation made once avoids that.  A released range keeps the events
    after which it is free; whoever is given part of it waits for them."""

    ALIGN = 1 << 21

    def __init__(self, buf):
        self.buf = buf
        self.free = [[0, buf.numel(), []]]            # [offset, size, events], by offset

    def alloc(self, nbytes: int):
        """(offset, size, events to wait for) of a range of at least nbytes, or None."""
        n = -(-max(int(nbytes), 1) // self.ALIGN) * self.ALIGN
        best = None
        for i, (_, size, _) in enumerate(self.free):
            if size >= n and (best is None or size < self.free[best][1]):
                best = i
        if best is None:
            return None
        off, size, evs = self.free[best]
        evs = [e for e in evs if not e.query()]
        if size == n:
            del self.free[best]
        else:
            self.free[best] = [off + n, size - n, list(evs)]
        return off, n, evs

    def release(self, off: int, n: int, event=None):
        """Return a range; `event` (if any) completes when its last user is done."""
        evs = [event] if event is not None else []
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        self.free.insert(i, [off, n, evs])
        # coalesce with the following and the preceding free range
        if i + 1 < len(self.free) and off + n == self.free[i + 1][0]:
            nxt = self.free.pop(i + 1)
            self.free[i][1] += nxt[1]
            self.free[i][2] += nxt[2]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            cur = self.free.pop(i)
            self.free[i - 1][1] += cur[1]
            self.free[i - 1][2] += cur[2]
        for r in self.free:
            r[2] = [e for e in r[2] if not e.query()]

    @property
    def free_bytes(self):
        return sum(size for _, size, _ in self.free)


class GpuExecutor:
    """Runs requests with libprism on the current HIP device."""

    def __init__(self, precision: int, probe_chunk_bytes: int = 1 << 30, build_ws_bytes: int = 16 << 30,
                 split_limit_bytes: int = 8 << 30, jobs_per_request: int = 4, range_pixels: int = 1 << 30,
                 reserve_bytes: int = 8 << 30, arena_bytes: int | None = None):
        import torch

        from . import api
        from ._lib import PRISM_FP32  # noqa: F401
        self.torch = torch
        self.api = api
        self.precision = precision
        self.probe_chunk_bytes = probe_chunk_bytes
        self.build_ws_bytes = build_ws_bytes
        # S-matrices whose split copy would exceed this are contracted in beam
        # chunks (prism_probe_outputs_chunked) instead of in the shared batch
        self.split_limit_bytes = split_limit_bytes
        self.jobs_per_request = jobs_per_request      # must match the scheduler's
        # beams of one build range: about range_pixels beam-pixels (n^2 each)
        self.range_pixels = range_pixels
        # device memory left free beside every request's footprint (the HIP
        # runtime's own queues, scratch and events)
        self.reserve_bytes = reserve_bytes
        # one allocation for the large buffers (DeviceArena), made by
        # reserve_arena() or at the first start: arena_bytes, or the free
        # device memory less the reserve and arena_headroom for the smaller
        # allocations (potentials, outputs, plans)
        self.arena_bytes = arena_bytes
        self.arena_headroom = 24 << 30
        self.arena = None
        self.synth_stream = torch.cuda.Stream()
        self.inflight = []              # (event, [(req, chunk)], workspace handles)

    # -- planning (host) --
    def plan(self, req: Request):
        """Descriptors, beam batch and probe chunks of a request; returns its footprint."""
        api = self.api
        g = api.prism_grid_init(req.cell, 2.0, req.n)
        d = api.prism_smatrix_plan(g, req.E0, req.alpha_max, req.f)
        per_beam = d.build_ws_bytes // max(d.n_beams, 1)
        bb = max(1, min(d.n_beams, self.build_ws_bytes // max(per_beam, 1)))
        if bb < d.n_beams:
            d = api.prism_smatrix_plan(g, req.E0, req.alpha_max, req.f, beam_batch=bb)
        nx, ny = req.scan
        xs = np.arange(nx) * (req.cell[0] / nx)
        ys = np.arange(ny) * (req.cell[1] / ny)
        yy, xx = np.meshgrid(ys, xs, indexing="ij")
        xy = np.stack([xx.ravel(), yy.ravel()], axis=1)
        per_probe = d.n_beams * 8 + d.m_win * d.m_win * (12 if d.m_win > 128 else 8)
        pc = max(1, min(len(xy), self.probe_chunk_bytes // per_probe))
        chunks = [xy[i:i + pc] for i in range(0, len(xy), pc)]
        plans = [api.prism_probe_plan_init(d, c, req.dalpha) for c in chunks]
        n_bins = plans[0].n_bins
        kb = (d.n_beams + 15) // 16
        split_bytes = d.ns * d.ns * kb * 128
        beam_chunk = 0
        if split_bytes > self.split_limit_bytes:
            # beam-chunked chunks run one after another on one shared workspace
            beam_chunk = max(16, (self.split_limit_bytes // (d.ns * d.ns * 128)) * 16)
            ws = max(_chunked_ws(d, p, beam_chunk) for p in plans)
        else:
            # a batch holds up to jobs_per_request chunks of this request, each
            # with its own coefficients and windows, plus one split S
            per_chunk = max(p.ws_bytes for p in plans) - split_bytes
            ws = split_bytes + min(self.jobs_per_request, len(plans)) * per_chunk
        foot = (g.n_slices * g.n * g.n * 4 + d.smatrix_bytes + d.build_ws_bytes
                + sum(p.plan_bytes for p in plans) + ws + len(xy) * n_bins * 4)
        req.info.update(grid=g, desc=d, chunks=chunks, n_bins=n_bins, n_beams=d.n_beams, m_win=d.m_win,
                        beam_batch=d.beam_batch or d.n_beams, beam_chunk=beam_chunk)
        req.chunks_total = len(chunks)
        # complex multiply-adds of one chunk's contraction (the synthesis's
        # dominant work), the unit of the scheduler's batch_cost
        req.chunk_cost = float(d.n_beams) * d.m_win * d.m_win * len(chunks[0])
        return int(foot)

    # -- build --
    def _fits(self, need: int) -> bool:
        """Whether `need` bytes can be allocated while the device keeps the
        reserve free: blocks the caching allocator holds are reused first,
        fresh device memory only for the rest."""
        torch = self.torch
        cached = torch.cuda.memory_reserved() - torch.cuda.memory_allocated()
        return torch.cuda.mem_get_info()[0] - max(0, need - cached) >= self.reserve_bytes

    def reserve_arena(self):
        """Allocate the arena now (else at the first request): a server's
        start-up cost, seconds when the memory was in use before."""
        torch = self.torch
        if self.arena is None:
            size = self.arena_bytes
            if size is None:
                size = torch.cuda.mem_get_info()[0] - self.reserve_bytes - self.arena_headroom
            size = (int(size) // DeviceArena.ALIGN) * DeviceArena.ALIGN
            self.arena = DeviceArena(torch.empty(max(size, DeviceArena.ALIGN), dtype=torch.uint8, device="cuda"))
        return self.arena

    def _alloc(self, nbytes: int, stream):
        """A uint8 device buffer of nbytes usable on `stream` and its handle:
        from the arena when it has room, else from the caching allocator when
        the device can hold it (None otherwise)."""
        torch = self.torch
        r = self.reserve_arena().alloc(nbytes)
        if r is not None:
            off, n, evs = r
            for e in evs:
                stream.wait_event(e)                  # the range's previous users have finished
            return self.arena.buf[off:off + nbytes], ("arena", off, n)
        if not self._fits(nbytes):
            torch.cuda.empty_cache()
            if not self._fits(nbytes):
                return None
        try:
            t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        except torch.cuda.OutOfMemoryError:
            return None
        return t, ("torch", t)

    def _release(self, handle, event=None, stream=None):
        if handle[0] == "arena":
            self.arena.release(handle[1], handle[2], event)
        elif stream is not None:
            handle[1].record_stream(stream)           # the caching allocator waits for the stream

    def start(self, req: Request):
        """Allocate and issue the request's first build range; False when the
        device cannot hold its footprint (plus the reserve).  The scheduler's
        budget counts footprints only.  The S-matrix and the build workspace
        come from the arena (DeviceArena), else from the caching allocator."""
        torch, api = self.torch, self.api
        info = req.info
        d = info["desc"]
        st = torch.cuda.Stream()
        s_bytes = d.n_beams * d.ns * d.ns * 8
        got = []
        for nb in (d.build_ws_bytes, s_bytes):
            r = self._alloc(nb, st)
            if r is None:
                for _, h in got:
                    self._release(h)
                return False
            got.append(r)
        (ws, ws_h), (sbuf, s_h) = got
        try:
            out = torch.empty((req.n_probes, info["n_bins"]), dtype=torch.float32, device="cuda")
        except torch.cuda.OutOfMemoryError:
            for _, h in got:
                self._release(h)
            return False
        info["stream"] = st
        info["handles"] = {"build_ws": ws_h, "S": s_h}
        info["build_ws"] = ws
        info["S"] = sbuf.view(torch.complex64).view(d.n_beams, d.ns, d.ns)
        info["out"] = out
        pos, sp, species = req.sample() if callable(req.sample) else req.sample
        with torch.cuda.stream(st):
            info["plans"] = [api.prism_probe_plan_upload(d, c, req.dalpha) for c in info["chunks"]]
            info["V"] = api.prism_project_potential(pos, sp, species, info["grid"])
        info["range_beams"] = max(16, min(d.beam_batch or d.n_beams, self.range_pixels // (req.n * req.n)))
        info["next_beam"] = 0
        info["built_event"] = None
        self._next_range(req)
        return True

    def _next_range(self, req: Request):
        """Issue the request's next beam range on its stream."""
        torch, api = self.torch, self.api
        info = req.info
        d, st = info["desc"], info["stream"]
        b0 = info["next_beam"]
        cnt = min(info["range_beams"], d.n_beams - b0)
        with torch.cuda.stream(st):
            api.prism_build_smatrix_range(d, info["V"], info["S"], b0, cnt, ws=info["build_ws"])
            ev = torch.cuda.Event()
            ev.record(st)
        info["next_beam"] = b0 + cnt
        info["built_event"] = ev
        if info["next_beam"] == d.n_beams:
            # the last range is queued: the potential and the workspace are
            # released, free once the stream has used them
            info["V"].record_stream(st)
            del info["V"]
            self._release(info["handles"].pop("build_ws"), ev, st)
            del info["build_ws"]

    def is_built(self, req: Request, may_issue: bool = True) -> bool:
        """True once every range has finished; issues the next range when the
        previous one has (and the scheduler lets it)."""
        info = req.info
        if not info["built_event"].query():
            return False
        if info["next_beam"] < info["desc"].n_beams:
            if may_issue:
                self._next_range(req)
            return False
        return True

    def build_left(self, req: Request) -> float:
        """Remaining build work of a request: beams not yet issued x slices x n^2."""
        info = req.info
        return float(info["desc"].n_beams - info["next_beam"]) * req.n_slices * req.n * req.n

    # -- synthesis --
    def synthesize(self, batch):
        """Issue one batched synthesis for [(req, chunk)] on the synthesis
        stream; chunks of requests marked for beam-chunked contraction are
        issued one by one on the same stream."""
        torch, api = self.torch, self.api
        items, single = [], []
        for req, c in batch:
            info = req.info
            self.synth_stream.wait_event(info["built_event"])
            p0 = sum(len(x) for x in info["chunks"][:c])
            out = info["out"][p0:p0 + len(info["chunks"][c])]
            it = (info["desc"], info["S"], info["plans"][c], out)
            (single if info.get("beam_chunk") else items).append((it, info.get("beam_chunk")))
            req.chunks_issued += 1
        keep = []

        def workspace(nbytes):
            r = self._alloc(max(int(nbytes), 1), self.synth_stream)
            if r is None:                             # as the caching allocator alone would
                t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")
                r = (t, ("torch", t))
            keep.append(r[1])
            return r[0]

        with torch.cuda.stream(self.synth_stream):
            if items:
                its = [it for it, _ in items]
                ws = workspace(api.prism_probe_batch_workspace(its))
                api.prism_probe_outputs_batched(its, self.precision, ws=ws)
            if single:
                # one workspace serves every beam-chunked item (same stream, in order)
                need = max(api.prism_probe_chunked_workspace(d, plan, bc) for (d, S, plan, out), bc in single)
                ws = workspace(need)
                for (d, S, plan, out), bc in single:
                    api.prism_probe_outputs_chunked(d, S, plan, self.precision, bc, ws=ws, out=out)
            ev = torch.cuda.Event()
            ev.record(self.synth_stream)
        self.inflight.append((ev, list(batch), keep))

    def finished_batches(self):
        """Batches whose synthesis completed (in issue order)."""
        done = []
        while self.inflight and self.inflight[0][0].query():
            ev, batch, handles = self.inflight.pop(0)
            for h in handles:
                self._release(h)                      # its synthesis has finished
            done.append(batch)
        return done

    def collect(self, req: Request):
        info = req.info
        req.result = info["out"].cpu().numpy()
        for k in ("S", "out", "plans"):
            info.pop(k, None)
        # the S-matrix's range (its syntheses have all finished)
        for h in info.pop("handles", {}).values():
            self._release(h)

    def chunks_left(self, req: Request):
        return range(req.chunks_issued, req.chunks_total)


def _chunked_ws(d, plan, beam_chunk):
    import ctypes

    from ._lib import check, lib
    need = ctypes.c_size_t()
    check(lib.prism_probe_chunked_workspace(ctypes.byref(d), ctypes.byref(plan), int(beam_chunk), ctypes.byref(need)))
    return need.value


# ---------------------------------------------------------------- the loop --
def serve(requests, executor, scheduler: Scheduler, clock=time.perf_counter, idle_sleep=2e-4, on_done=None,
          sleep=time.sleep):
    """Run the request stream to completion; returns the scheduler."""
    pending = sorted(requests, key=lambda r: r.arrival)
    t0 = clock()
    i = 0
    while i < len(pending) or not scheduler.idle or getattr(executor, "inflight", None):
        now = clock() - t0
        while i < len(pending) and pending[i].arrival <= now:
            req = pending[i]
            scheduler.arrive(req, executor.plan(req))
            i += 1
        admitted = scheduler.admit(now)
        for k, req in enumerate(admitted):
            try:
                started = executor.start(req)
            except (MemoryError, RuntimeError) as exc:    # e.g. device allocation failure
                scheduler.fail(req, clock() - t0, str(exc))
                continue
            if started is False:
                # the device cannot hold it yet: it and the requests admitted
                # after it wait in the queue
                for r in admitted[k:]:
                    scheduler.defer(r)
                break
        build_left = getattr(executor, "build_left", None) if math.isfinite(scheduler.build_ratio) else None
        for req in list(scheduler.building):
            if build_left is None:
                built = executor.is_built(req)
            else:
                built = executor.is_built(req, scheduler.may_build(req, clock() - t0, build_left))
            if built:
                scheduler.mark_built(req, clock() - t0)
        if not executor.inflight:
            batch = scheduler.next_batch(executor.chunks_left)
            if batch:
                executor.synthesize(batch)
        progressed = False
        for batch in executor.finished_batches():
            progressed = True
            for req, _ in batch:
                if scheduler.chunk_done(req, clock() - t0):
                    executor.collect(req)
                    req.t_done = clock() - t0
                    if on_done:
                        on_done(req)
        if not progressed:
            sleep(idle_sleep)
    return scheduler


def summarize(sched: Scheduler, wall: float):
    done = sched.done
    lat = np.array([r.latency for r in done]) if done else np.zeros(1)
    probes = sum(r.n_probes for r in done)
    by_grid = {}
    for n in sorted({r.n for r in done}):
        ln = np.array([r.latency for r in done if r.n == n])
        by_grid[str(n)] = {"requests": int(len(ln)), "p50_latency_s": float(np.percentile(ln, 50)),
                           "p99_latency_s": float(np.percentile(ln, 99))}
    return {"requests": len(done), "rejected": len(sched.rejected), "probes": probes,
            "wall_s": wall, "probes_per_s": probes / wall if wall > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "latency_by_grid": by_grid, "peak_hbm_reserved": sched.peak_used}
