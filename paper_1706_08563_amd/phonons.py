"""Frozen-phonon averaging of PRISM outputs.

The paper averages its images over thermal configurations of the atoms (32
frozen phonons for the oxide comparison, 16 for the tomography study).  Each
configuration is a full simulation: potential, S-matrix, probe synthesis.  The
probe plan does not depend on the configuration and is made once; the outputs
of every configuration are accumulated on the device with weight 1/N by the
synthesis kernels themselves (prism_probe_job.out_scale / accumulate).
"""
from __future__ import annotations

from . import api


def frozen_phonon_outputs(grid, E0: float, alpha_max: float, f: int, configs, species_idx, species, xy,
                          precision: int = 0, dalpha: float = 1e-3, C1: float = 0.0, C3: float = 0.0,
                          beam_batch: int = 0):
    """Mean over `configs` (a list of [n_atoms, 3] position arrays, A) of the
    PRISM 3D outputs; returns [n_probes, n_bins] float32 on the device."""
    import torch
    d = api.prism_smatrix_plan(grid, E0, alpha_max, f, beam_batch=beam_batch)
    plan = api.prism_probe_plan_upload(d, xy, dalpha, C1=C1, C3=C3)
    ws_b = torch.empty(d.build_ws_bytes, dtype=torch.uint8, device="cuda")
    S = torch.empty((d.n_beams, d.ns, d.ns), dtype=torch.complex64, device="cuda")
    out = torch.empty((plan.plan.n_probes, plan.plan.n_bins), dtype=torch.float32, device="cuda")
    ws_p = None
    w = 1.0 / len(configs)
    for k, pos in enumerate(configs):
        V = api.prism_project_potential(pos, species_idx, species, grid)
        api.prism_build_smatrix(d, V, ws=ws_b, S=S)
        items = [(d, S, plan, out, None, w, 1 if k else 0)]
        if ws_p is None:
            ws_p = torch.empty(api.prism_probe_batch_workspace(items), dtype=torch.uint8, device="cuda")
        api.prism_probe_outputs_batched(items, precision, ws=ws_p)
    return out
