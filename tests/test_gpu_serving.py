"""Serving on the GPU: a mixed stream of small requests through the
continuous-batching loop; each request's result equals its result alone, and
one request matches the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from gates import check_D

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _requests():
    from paper_1706_08563_amd.serve import Request
    params = [(0.000, 128, 2, 3, (6, 6)), (0.001, 256, 4, 4, (5, 7)), (0.002, 128, 4, 2, (9, 9)),
              (0.003, 256, 2, 3, (4, 4)), (0.004, 512, 8, 2, (3, 5)), (0.005, 128, 1, 2, (4, 4))]
    out = []
    for i, (t, n, f, s, sc) in enumerate(params):
        r = Request(i, t, n, f, s, sc, 1000 + i, E0=80e3, pixel=0.15625)
        r.sample = W.serving_sample(r.cell, r.seed)
        out.append(r)
    return out


def _run(reqs, prec, **kw):
    import torch
    from paper_1706_08563_amd.serve import GpuExecutor, Scheduler, serve
    ex = GpuExecutor(prec, probe_chunk_bytes=kw.pop("chunk", 1 << 30),
                     split_limit_bytes=kw.pop("split_limit", 8 << 30), range_pixels=kw.pop("range_pixels", 1 << 30))
    sched = Scheduler(int(64e9), **kw)
    serve(reqs, ex, sched)
    torch.cuda.synchronize()
    return sched


@pytest.mark.parametrize("prec", [0, 1])
def test_mix_equals_alone(prec):
    say(f"serving mix of 6 requests, precision {prec}, small probe chunks")
    mixed = _requests()
    sched = _run(mixed, prec, max_building=4, max_jobs=8, chunk=1 << 19)
    assert len(sched.done) == 6 and not sched.rejected
    assert sum(r.chunks_total for r in mixed) > 6          # several chunks per request
    for r in mixed:
        alone = [x for x in _requests() if x.rid == r.rid]
        _run(alone, prec, max_building=1, max_jobs=1, chunk=1 << 30)
        diff = np.max(np.abs(alone[0].result - r.result))
        say(f"  request {r.rid} (n={r.n}, f={r.f}): max |mix - alone| = {diff:.3e}")
        assert diff <= 1e-6 * max(np.max(np.abs(r.result)), 1e-30)


def test_served_request_matches_oracle():
    say("serving: request 1 against the oracle")
    reqs = _requests()
    _run(reqs, 0, max_building=3, max_jobs=8)
    r = reqs[1]
    pos, sp = W.nanoparticle_in_amorphous(r.cell, rng=np.random.default_rng(r.seed))
    lam, sig = O.wavelength(r.E0), O.interaction_constant(r.E0)
    L = r.cell[0]
    V = O.projected_potential(pos, sp, (W.AU, W.C), r.cell, 2.0, r.n)
    beams = O.beam_set(r.n, L, lam, r.alpha_max, r.f)
    S = O.build_smatrix(V, L, 2.0, lam, sig, beams)
    xy = W.scan_positions(r.cell, *r.scan)
    ref = O.prism_outputs(S, beams, L, r.n, lam, r.f, xy)
    check_D(r.result, ref, "served request 1")


def test_beam_chunked_requests_in_the_mix():
    """Requests whose split S-matrix exceeds the executor's limit are
    contracted in beam chunks; their results agree with the batched path to
    FP32 summation order and the others are unchanged."""
    say("serving: beam-chunked contraction for requests above the split limit")
    mixed = _requests()
    _run(mixed, 1, max_building=4, max_jobs=8, split_limit=1 << 20)
    assert all(r.info.get("beam_chunk") for r in mixed if r.n >= 256)
    ref = _requests()
    _run(ref, 1, max_building=4, max_jobs=8)
    for a, b in zip(mixed, ref):
        err = O.rel_err(a.result, b.result)
        say(f"  request {a.rid} (n={a.n}, beam chunk {a.info.get('beam_chunk')}): rel diff {err:.3e}")
        assert err <= 1e-5


def test_builds_in_beam_ranges_equal_whole_builds():
    """With builds issued a few beams at a time (every request's S-matrix in
    several ranges, interleaved with the other requests' ranges and
    syntheses) every result equals the one-range build bit for bit."""
    say("serving: builds in small beam ranges vs one range per request")
    a = _requests()
    _run(a, 1, max_building=4, max_jobs=8, range_pixels=16 * 128 * 128)
    assert max(r.info["range_beams"] for r in a) < max(r.info["n_beams"] for r in a)
    b = _requests()
    _run(b, 1, max_building=4, max_jobs=8)
    for x, y in zip(a, b):
        say(f"  request {x.rid} (n={x.n}, {x.info['n_beams']} beams, ranges of {x.info['range_beams']})")
        assert np.array_equal(x.result, y.result)


def test_paced_builds_equal_unpaced():
    """With build pacing on (larger builds hold their next range while
    smaller ones proceed) every request completes and its result equals the
    unpaced run bit for bit."""
    say("serving: build pacing on vs off, builds in small beam ranges")
    a = _requests()
    sched = _run(a, 1, max_building=4, max_jobs=8, range_pixels=16 * 128 * 128, build_ratio=2.0, build_hold=0.5)
    assert len(sched.done) == len(a) and not sched.rejected
    b = _requests()
    _run(b, 1, max_building=4, max_jobs=8, range_pixels=16 * 128 * 128)
    for x, y in zip(a, b):
        assert np.array_equal(x.result, y.result), f"request {x.rid}"
