"""Parity at the full workload sizes, in the launch configuration the
benchmark times, on outputs the FP64 oracle can compute one by one:

* 1024^2 PRISM f = 4 (1245 beams, 50 slices): the whole S-matrix is built on
  the GPU; sampled layers are compared with the oracle's single-beam build.
* the same geometry's probe synthesis over the full 128 x 128 scan on a seeded
  S-matrix operand; sampled probes against the oracle (FP32 and split-BF16).
* 1024^2 multislice (50 slices): sampled probes of the 64 x 64 scan.
* 2048^2 PRISM f = 8 (1245 beams, 50 slices): sampled S-matrix layers.
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


def _potentials(P, w):
    pos, sp = W.atoms_for(w)
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    V = P.prism_project_potential(pos, sp, w.species, g)
    Vref = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    return g, V, Vref


@pytest.mark.parametrize("cfg", ["prism_f4_np_1024", "prism_f8_np_2048"])
def test_full_smatrix_sampled_layers(P, cfg):
    import torch
    w = W.WORKLOADS[cfg]
    say(f"full S-matrix {w.name}: build on GPU, sampled layers vs oracle")
    g, V, Vref = _potentials(P, w)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    S = P.prism_build_smatrix(d, V)
    torch.cuda.synchronize()
    beams = P.prism_beam_list(d)
    t = O.transmission(Vref, d.sigma)
    Pp = O.propagator(w.n, w.cell[0], d.lambda_, w.dz)
    sample = (0, 311, len(beams) // 2, len(beams) - 1) if cfg == "prism_f4_np_1024" else (0, len(beams) // 2 + 7)
    for b in sample:
        ref = O.smatrix_layer(t, Pp, int(beams[b, 0]), int(beams[b, 1]))
        got = S[b].cpu().numpy().astype(np.complex128)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        say(f"  beam {b} {tuple(beams[b])}: rel err {err:.3e}")
        assert err <= TOL


def test_full_synthesis_sampled_probes(P):
    import torch
    w = W.WORKLOADS["prism_f4_np_1024"]
    say("full synthesis 1024^2 f=4, 128x128 probes, seeded S operand")
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    rng = np.random.default_rng(202)
    Sh = W.random_complex((d.n_beams, d.ns, d.ns), rng)
    S = torch.from_numpy(Sh).cuda()
    xy = W.scan_positions(w.cell, *w.scan)
    plan = P.prism_probe_plan_upload(d, xy)
    pick = np.array([0, 1, 127, 128, 4095, 8192 + 64, 12345, 16383])
    beams = P.prism_beam_list(d).astype(np.int64)
    ref = O.prism_outputs(Sh, beams, w.cell[0], w.n, d.lambda_, w.f, xy[pick])
    for name, prec in (("fp32", P.PRISM_FP32), ("bf16x3", P.PRISM_SPLIT_BF16X3)):
        out = P.prism_probe_outputs(d, S, plan, prec).cpu().numpy()
        check_D(out[pick], ref, f"{name} on {len(pick)} sampled probes")


def test_full_synthesis_2048_sampled_probes(P):
    import torch
    w = W.WORKLOADS["prism_f8_np_2048"]
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    say(f"full synthesis 2048^2 f=8: {d.n_beams} beams x {d.ns}^2 seeded S operand, 256x256 probes")
    rng = np.random.default_rng(404)
    S = torch.empty((d.n_beams, d.ns, d.ns), dtype=torch.complex64, device="cuda")
    for b0 in range(0, d.n_beams, 64):
        S[b0:b0 + 64] = torch.from_numpy(W.random_complex((min(64, d.n_beams - b0), d.ns, d.ns), rng)).cuda()
    xy = W.scan_positions(w.cell, *w.scan)
    assert len(xy) == 65536
    plan = P.prism_probe_plan_upload(d, xy)
    pick = np.array([0, 1, 255, 256, 32768 + 128, 40000, 65535 - 256, 65535])
    say("  copying S to the host for the oracle")
    Sh = S.cpu().numpy()
    beams = P.prism_beam_list(d).astype(np.int64)
    ref = O.prism_outputs(Sh, beams, w.cell[0], w.n, d.lambda_, w.f, xy[pick])
    del Sh
    for name, prec in (("bf16x3", P.PRISM_SPLIT_BF16X3), ("fp32", P.PRISM_FP32)):
        say(f"  {name} synthesis of 65536 probes")
        out = P.prism_probe_outputs(d, S, plan, prec).cpu().numpy()
        check_D(out[pick], ref, f"{name} on {len(pick)} sampled probes")


def test_full_multislice_sampled_probes(P):
    w = W.WORKLOADS["multislice_np_1024"]
    say("full multislice 1024^2, 50 slices, sampled probes of the 64x64 scan")
    g, V, Vref = _potentials(P, w)
    xy = W.scan_positions(w.cell, *w.scan)
    pick = np.array([0, 2080, 4095])
    out = P.multislice_outputs(g, w.E0, w.alpha_max, V, xy, batch=1024).cpu().numpy()
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    ref = O.multislice_outputs(Vref, w.cell[0], w.dz, lam, sig, w.alpha_max, xy[pick])
    check_D(out[pick], ref, "multislice sampled probes")


def _fixture(name):
    """FP64 3D outputs of a workload's 16 x 16 probe subset, written by
    tests/golden/make_golden.py from the oracle alone."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_fp64_subset.npz")
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} not written (tests/golden/make_golden.py --workload {name})")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


@pytest.mark.parametrize("cfg", ["prism_f4_np_1024", "prism_f8_np_2048"])
def test_end_to_end_against_fp64_fixture(P, cfg):
    """The benchmarked path end to end: the GPU-built S-matrix of every beam of
    the aperture through every slice, synthesised at the 16 x 16 probe subset
    of the full scan in the same plan as the whole scan (so the subset's
    windows come from the launch the benchmark times), against the FP64
    oracle's streamed PRISM of the same cell; multislice on the same probes
    for the 1024^2 cell.  FP32 and split-BF16 are gated, plain BF16 reported."""
    import torch
    w = W.WORKLOADS[cfg]
    fx = _fixture(cfg)
    say(f"end to end {cfg}: GPU S-matrix + full-scan synthesis vs FP64 fixture ({len(fx['probe_xy'])} probes)")
    pos, sp = W.atoms_for(w)
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    V = P.prism_project_potential(pos, sp, w.species, g)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    assert np.array_equal(P.prism_beam_list(d), fx["beams"])
    S = P.prism_build_smatrix(d, V)
    xy = W.scan_positions(w.cell, *w.scan)
    sub = w.scan[0] // 16
    j, i = np.meshgrid(np.arange(0, w.scan[1], sub), np.arange(0, w.scan[0], sub), indexing="ij")
    idx = (j * w.scan[0] + i).ravel()
    assert np.array_equal(xy[idx], fx["probe_xy"])
    plan = P.prism_probe_plan_upload(d, xy)
    for name, prec, tol in (("bf16x3", P.PRISM_SPLIT_BF16X3, TOL), ("fp32", P.PRISM_FP32, TOL),
                            ("bf16", P.PRISM_BF16, None)):
        out = P.prism_probe_outputs(d, S, plan, prec)
        torch.cuda.synchronize()
        check_D(out[torch.from_numpy(idx).cuda()].cpu().numpy(), fx["prism"], f"{name} PRISM f={w.f}", tol=tol)
        del out
    if "multislice" in fx:
        ms = P.multislice_outputs(g, w.E0, w.alpha_max, V, fx["probe_xy"], batch=256).cpu().numpy()
        check_D(ms, fx["multislice"], "multislice")
        # the method's own approximation at this f (GPU and FP64): reported only
        check_D(fx["prism"], fx["multislice"], f"FP64 PRISM f={w.f} vs FP64 multislice", tol=None)
