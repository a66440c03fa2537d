"""Streaming memory model ("Streaming Data for Very Large Simulations") on
the GPU: potential and S-matrix in page-locked host memory, staged through
double-buffered device slots on copy streams.

* the streaming S-matrix build equals the single-transfer build bit for bit
  (same kernels on the same values) and both match the FP64 oracle;
* streaming multislice equals single-transfer multislice bit for bit;
* the streamed synthesis (beam chunks accumulated in FP32 windows) matches
  the single-transfer synthesis to FP32 rounding and the oracle to 1e-4, for
  3D and 4D outputs, ragged last chunks and chunk = all beams;
* the memory planner's streaming plan runs end to end within its budget.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from gates import check_D

pytestmark = pytest.mark.gpu
TOL = 1e-4


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_1706_08563_amd as P
    assert torch.cuda.is_available()
    return P


def _setup(P, n=128, f=2, seed=21, n_atoms=48, cell=(20.0, 20.0, 8.0)):
    import torch
    w, pos, sp = W.small_workload(n=n, cell=cell, n_atoms=n_atoms, f=f, seed=seed)
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    V = P.prism_project_potential(pos, sp, w.species, g)
    torch.cuda.synchronize()
    Vh = V.cpu().pin_memory()
    return w, pos, sp, g, V, Vh


@pytest.mark.parametrize("beam_batch", [0, 7])
def test_streaming_build_bitwise_and_oracle(P, beam_batch):
    import torch
    say(f"streaming S-matrix build, beam_batch={beam_batch}")
    w, pos, sp, g, V, Vh = _setup(P)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f, beam_batch=beam_batch)
    S_res = P.prism_build_smatrix(d, V)
    S_str = P.prism_build_smatrix_streaming(d, Vh)
    torch.cuda.synchronize()
    a = S_res.cpu().numpy()
    b = S_str.numpy()
    say(f"  beams {d.n_beams}, batch {d.beam_batch}: max |diff| {np.abs(a - b).max():.3e}")
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    Vref = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    L = w.cell[0]
    beams = P.prism_beam_list(d).astype(np.int64)
    t = O.transmission(Vref, d.sigma)
    Pp = O.propagator(w.n, L, d.lambda_, w.dz)
    for bi in (0, d.n_beams - 1):
        ref = O.smatrix_layer(t, Pp, int(beams[bi, 0]), int(beams[bi, 1]))
        err = np.linalg.norm(b[bi] - ref) / np.linalg.norm(ref)
        assert err <= TOL


def test_streaming_multislice_bitwise(P):
    import torch
    say("streaming multislice vs single transfer")
    w, pos, sp, g, V, Vh = _setup(P, seed=22)
    xy = W.scan_positions(w.cell, 3, 3)
    a = P.multislice_outputs(g, w.E0, w.alpha_max, V, xy, batch=4, C1=10.0)
    b = P.multislice_outputs_streaming(g, w.E0, w.alpha_max, Vh, xy, batch=4, C1=10.0)
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(a, b)
    Vref = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    ref = O.multislice_outputs(Vref, w.cell[0], w.dz, O.wavelength(w.E0), O.interaction_constant(w.E0),
                               w.alpha_max, xy, C1=10.0)
    check_D(b, ref, "streamed multislice")


@pytest.mark.parametrize("n,L,f,a,prec,chunk", [(128, 16.0, 2, 0.02, 0, 16), (256, 20.0, 2, 0.02, 1, 50),
                                                (256, 20.0, 1, 0.02, 1, 10**6), (512, 40.0, 1, 0.008, 1, 97)])
def test_streaming_synthesis(P, n, L, f, a, prec, chunk):
    import torch
    g = P.prism_grid_init((L, L, 2.0), 2.0, n)
    d = P.prism_smatrix_plan(g, 200e3, a, f)
    chunk = min(chunk, d.n_beams)
    say(f"streamed synthesis n={n} f={f} beams={d.n_beams} chunk={chunk} precision={prec}")
    rng = np.random.default_rng(51 + n)
    S = W.random_complex((d.n_beams, d.ns, d.ns), rng)
    xy = np.concatenate([W.random_positions((L, L), 9, rng), [[0.0, 0.0], [L - 1e-9, 0.5 * L]]])
    plan = P.prism_probe_plan_upload(d, xy, C1=-12.0, C3=1e5)
    Sh = torch.from_numpy(S).pin_memory()
    D_res = P.prism_probe_outputs(d, Sh.cuda(), plan, prec)
    D_str = P.prism_probe_outputs_streaming(d, Sh, plan, prec, chunk)
    I_str = P.prism_probe_outputs_streaming(d, Sh, plan, prec, chunk, diffraction=True)
    torch.cuda.synchronize()
    beams = P.prism_beam_list(d).astype(np.int64)
    ref = O.prism_outputs(S.astype(np.complex128), beams, L, n, d.lambda_, f, xy, C1=-12.0, C3=1e5)
    e_res = O.rel_err(D_str.cpu().numpy(), D_res.cpu().numpy())
    e_ref = O.rel_err(D_str.cpu().numpy(), ref)
    say(f"  streamed vs resident {e_res:.3e}, vs oracle {e_ref:.3e}")
    assert e_res <= 1e-5
    check_D(D_str.cpu().numpy(), ref, "streamed synthesis")
    ref4 = O.prism_diffraction(S.astype(np.complex128), beams, L, n, d.lambda_, f, xy, C1=-12.0, C3=1e5)
    got4 = I_str.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got4 - ref4) / np.linalg.norm(ref4) <= TOL


@pytest.mark.parametrize("prec,chunk", [(0, 37), (1, 16), (2, 100)])
def test_chunked_synthesis_device_s(P, prec, chunk):
    import torch
    n, L, f, a = 256, 20.0, 2, 0.02
    g = P.prism_grid_init((L, L, 2.0), 2.0, n)
    d = P.prism_smatrix_plan(g, 200e3, a, f)
    say(f"beam-chunked synthesis from device S: beams={d.n_beams} chunk={chunk} precision={prec}")
    rng = np.random.default_rng(61 + prec)
    S = W.random_complex((d.n_beams, d.ns, d.ns), rng)
    xy = np.concatenate([W.random_positions((L, L), 7, rng), [[0.0, 0.0]]])
    plan = P.prism_probe_plan_upload(d, xy, C1=8.0)
    Sh = torch.from_numpy(S).pin_memory()
    Sd = Sh.cuda()
    D_chk = P.prism_probe_outputs_chunked(d, Sd, plan, prec, chunk)
    D_str = P.prism_probe_outputs_streaming(d, Sh, plan, prec, chunk)
    D_res = P.prism_probe_outputs(d, Sd, plan, prec)
    I_chk = P.prism_probe_outputs_chunked(d, Sd, plan, prec, chunk, diffraction=True)
    torch.cuda.synchronize()
    a_, b_ = D_chk.cpu().numpy(), D_str.cpu().numpy()
    assert np.array_equal(a_, b_)                       # same kernels, same chunks
    assert O.rel_err(a_, D_res.cpu().numpy()) <= (1e-5 if prec < 2 else 1e-3)
    beams = P.prism_beam_list(d).astype(np.int64)
    if prec < 2:
        ref = O.prism_outputs(S.astype(np.complex128), beams, L, n, d.lambda_, f, xy, C1=8.0)
        check_D(a_, ref, "beam-chunked synthesis")
        ref4 = O.prism_diffraction(S.astype(np.complex128), beams, L, n, d.lambda_, f, xy, C1=8.0)
        got4 = I_chk.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(got4 - ref4) / np.linalg.norm(ref4) <= TOL


def test_memory_plan_streaming_end_to_end(P):
    import torch
    from paper_1706_08563_amd import memory as M
    say("memory planner: forced streaming under a tight budget, end to end")
    w, pos, sp, g, V, Vh = _setup(P, n=256, f=2, seed=23, cell=(24.0, 24.0, 8.0))
    xy = W.scan_positions(w.cell, 6, 6)
    d0 = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    mp_single = M.plan_memory(g, w.E0, w.alpha_max, w.f, xy, 1 << 40)
    assert mp_single.mode == "single"
    budget = mp_single.single_bytes // 3
    mp = M.plan_memory(g, w.E0, w.alpha_max, w.f, xy, budget, min_beam_chunk=8)
    say(f"  budget {budget} B: mode {mp.mode}, beam batch {mp.desc.beam_batch}, beam chunk {mp.beam_chunk}, "
        f"probe chunk {mp.probe_chunk}, peak {mp.peak_bytes} B (single {mp.single_bytes} B)")
    assert mp.mode == "streaming" and mp.peak_bytes <= budget
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    out = M.run_prism(mp, Vh, xy, P.PRISM_SPLIT_BF16X3)
    torch.cuda.synchronize()
    used = torch.cuda.max_memory_allocated() - before
    ref_dev = M.run_prism(mp_single, V, xy, P.PRISM_SPLIT_BF16X3)
    torch.cuda.synchronize()
    say(f"  device bytes used by the streamed run {used} (planned peak {mp.peak_bytes})")
    assert used <= mp.peak_bytes + (64 << 20)
    assert O.rel_err(out.cpu().numpy(), ref_dev.cpu().numpy()) <= 1e-5
    assert d0.n_beams == mp.desc.n_beams
