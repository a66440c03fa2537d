"""prism_probe_outputs_noalloc: probe synthesis whose workspace is the
library's fixed device scratch array (no device allocation in the call).

GPU: through the C ABI, two calls in a row on the 256^2 simple-cubic PRISM
workload (all 256 probes, then a ragged 5-probe subset, so the second call
runs over the first call's leftover scratch contents), each equal bit for bit
to prism_probe_outputs with a caller workspace (same kernels, same order of
operations) and within the 1e-4 gates of the FP64 oracle.
CPU: a plan whose workspace exceeds the scratch array is refused before any
device work.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from gates import check_D


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def test_noalloc_rejects_plans_beyond_the_scratch():
    import paper_1706_08563_amd as P
    w = W.WORKLOADS["prism_f4_np_1024"]
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    plan = P.prism_probe_plan_init(d, W.scan_positions(w.cell, *w.scan))
    assert plan.ws_bytes > P.PRISM_NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(256)   # never dereferenced: the size check comes first
    rc = P.lib.prism_probe_outputs_noalloc(ctypes.byref(d), fake, ctypes.byref(plan), fake, P.PRISM_FP32, fake,
                                           None)
    assert rc == P.PRISM_E_WORKSPACE
    assert b"fixed scratch" in P.lib.prism_last_error()


@pytest.mark.gpu
@pytest.mark.parametrize("prec_name", ["fp32", "bf16x3"])
def test_noalloc_matches_caller_workspace_two_calls(prec_name):
    import torch
    import paper_1706_08563_amd as P
    prec = {"fp32": P.PRISM_FP32, "bf16x3": P.PRISM_SPLIT_BF16X3}[prec_name]
    w = W.WORKLOADS["prism_f2_sc_256"]
    say(f"noalloc {w.name} {prec_name}: build")
    pos, sp = W.atoms_for(w)
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    V = P.prism_project_potential(pos, sp, w.species, g)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    S = P.prism_build_smatrix(d, V)
    torch.cuda.synchronize()
    L = w.cell[0]
    Vref = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    beams = O.beam_set(w.n, L, d.lambda_, w.alpha_max, w.f)
    Sref = O.build_smatrix(Vref, L, w.dz, d.lambda_, d.sigma, beams)
    full = W.scan_positions(w.cell, *w.scan)
    sets = [("all 256 probes", full), ("5 probes", full[[3, 40, 77, 150, 255]] + np.array([0.37, -0.21]))]
    for label, xy in sets:
        say(f"noalloc {w.name} {prec_name}: {label}")
        plan = P.prism_probe_plan_upload(d, xy)
        assert plan.plan.ws_bytes <= P.PRISM_NOALLOC_SCRATCH_BYTES
        got = P.prism_probe_outputs_noalloc(d, S, plan, prec)
        ref_gpu = P.prism_probe_outputs(d, S, plan, prec)
        torch.cuda.synchronize()
        a, b = got.cpu().numpy(), ref_gpu.cpu().numpy()
        assert a.shape == (len(xy), plan.plan.n_bins)
        assert np.array_equal(a, b), (label, float(np.max(np.abs(a - b))))
        ref = O.prism_outputs(Sref, beams, L, w.n, d.lambda_, w.f, xy)
        check_D(a, ref, f"noalloc {prec_name} {label}")
