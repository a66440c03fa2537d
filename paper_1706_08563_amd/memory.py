"""Choice between the single-transfer and the streaming memory model.

The paper selects a memory model automatically from an estimate of the device
memory a simulation needs ("Streaming Data for Very Large Simulations"):
single transfer when the large arrays fit on the device, streaming otherwise.
Here the estimate is exact: every device byte of both models is a library
workspace size, so the choice is made from the library's own size queries
(host-side calls only, no device access).

Single transfer keeps V, the transmission of every slice, the S-matrix, the
probe plan, the synthesis workspace and the outputs resident.  Streaming keeps
V and S in host memory; its peak is the larger of the streaming build
workspace and the streamed synthesis (plan, workspace of one beam chunk pair,
outputs), since the two phases run one after the other.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import api


@dataclass
class MemoryPlan:
    mode: str                 # "single" or "streaming"
    desc: object              # prism_smatrix_desc (beam batch chosen to fit)
    beam_chunk: int           # beams per streamed synthesis chunk (streaming only)
    probe_chunk: int          # probes per synthesis call
    peak_bytes: int           # device bytes the chosen model needs
    single_bytes: int         # device bytes of the single-transfer model at full beam batch


def single_transfer_bytes(d, plan, n_outputs_bytes: int) -> int:
    g = d.grid
    v_bytes = g.n_slices * g.n * g.n * 4
    return int(v_bytes + d.build_ws_bytes + d.smatrix_bytes + plan.plan_bytes + plan.ws_bytes + n_outputs_bytes)


def _stream_synth_ws(d, plan, beam_chunk):
    import ctypes
    from ._lib import lib, check
    need = ctypes.c_size_t()
    check(lib.prism_probe_streaming_workspace(ctypes.byref(d), ctypes.byref(plan), int(beam_chunk),
                                              ctypes.byref(need)))
    return need.value


def _synth_peak(d, xy, dalpha, probe_chunk, beam_chunk, out_bytes):
    """Streamed synthesis peak over probe chunks: the largest chunk's plan
    and workspace, plus the whole output."""
    worst = 0
    for p0 in range(0, len(xy), probe_chunk):
        plan = api.prism_probe_plan_init(d, xy[p0:p0 + probe_chunk], dalpha)
        worst = max(worst, plan.plan_bytes + _stream_synth_ws(d, plan, beam_chunk))
    return worst + out_bytes


def plan_memory(grid, E0: float, alpha_max: float, f: int, xy, budget_bytes: int, dalpha: float = 1e-3,
                force: str | None = None, min_beam_chunk: int = 64) -> MemoryPlan:
    """Pick the memory model for a PRISM simulation that must fit in
    `budget_bytes` of device memory: single transfer when it fits, otherwise
    streaming with the largest build beam batch, then the largest probe chunk
    that fits with at least `min_beam_chunk` beams per streamed chunk, then
    the largest beam chunk.  `force` = "single" or "streaming" overrides the
    choice, as the paper lets users do.  Raises MemoryError when nothing fits."""
    import numpy as np
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    if force not in (None, "single", "streaming"):
        raise ValueError("force must be None, 'single' or 'streaming'")
    d = api.prism_smatrix_plan(grid, E0, alpha_max, f)
    plan = api.prism_probe_plan_init(d, xy, dalpha)
    out_bytes = plan.n_probes * plan.n_bins * 4
    single = single_transfer_bytes(d, plan, out_bytes)
    if force == "single" or (force is None and single <= budget_bytes):
        if single > budget_bytes:
            raise MemoryError(f"single transfer needs {single} B > budget {budget_bytes} B")
        return MemoryPlan("single", d, d.n_beams, len(xy), single, single)
    batch = d.n_beams
    while True:
        db = api.prism_smatrix_plan(grid, E0, alpha_max, f, beam_batch=batch)
        build = api.prism_streaming_build_workspace(db)
        if build <= budget_bytes or batch == 1:
            break
        batch = max(1, batch // 2)
    if build > budget_bytes:
        raise MemoryError(f"streaming build needs {build} B > budget {budget_bytes} B with one beam per batch")
    bc0 = min(min_beam_chunk, d.n_beams)
    pc = max(len(xy), 1)
    while pc > 1 and _synth_peak(db, xy, dalpha, pc, bc0, out_bytes) > budget_bytes:
        pc = (pc + 1) // 2
    if _synth_peak(db, xy, dalpha, pc, bc0, out_bytes) > budget_bytes:
        raise MemoryError("streamed synthesis does not fit even one probe at a time")
    bc = d.n_beams
    while bc > bc0 and _synth_peak(db, xy, dalpha, pc, bc, out_bytes) > budget_bytes:
        bc = max(bc0, bc // 2)
    peak = max(build, _synth_peak(db, xy, dalpha, pc, bc, out_bytes))
    return MemoryPlan("streaming", db, bc, pc, peak, single)


def run_prism(mp: MemoryPlan, V, xy, precision: int, dalpha: float = 1e-3):
    """The 3D output [n_probes, n_bins] (device) of a PRISM simulation in the
    planned memory model.  V: device float32 [S, n, n] for single transfer, or
    host (page-locked) float32 for streaming."""
    import numpy as np
    import torch
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    d = mp.desc
    if mp.mode == "single":
        S = api.prism_build_smatrix(d, V)
        plan = api.prism_probe_plan_upload(d, xy, dalpha)
        return api.prism_probe_outputs(d, S, plan, precision)
    S_host = api.prism_build_smatrix_streaming(d, V)
    torch.cuda.current_stream().synchronize()
    outs = []
    for p0 in range(0, len(xy), mp.probe_chunk):
        plan = api.prism_probe_plan_upload(d, xy[p0:p0 + mp.probe_chunk], dalpha)
        outs.append(api.prism_probe_outputs_streaming(d, S_host, plan, precision, mp.beam_chunk))
    return torch.cat(outs, 0)
