"""Python entry points with the names of the C ABI (include/prism.h).

Marshalling only: numpy host arrays become ctypes arrays, device buffers and
workspaces are torch tensors on the current HIP device, and the current torch
stream is handed to the library.  No step of the simulation is computed here.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from ._lib import (lib, check, prism_atom, prism_species, prism_grid, prism_smatrix_desc, prism_probe_plan,
                   prism_probe_job, prism_aberrations, PRISM_FP32)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes, device=None):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device or "cuda")


# ---------------------------------------------------------------- grid --
def prism_grid_init(cell, dz: float, n: int) -> prism_grid:
    g = prism_grid()
    c = (ctypes.c_double * 3)(*[float(v) for v in cell])
    check(lib.prism_grid_init(c, float(dz), int(n), ctypes.byref(g)))
    return g


# ------------------------------------------------------------ S-matrix --
def prism_smatrix_plan(grid: prism_grid, E0: float, alpha_max: float, f: int,
                       beam_batch: int = 0) -> prism_smatrix_desc:
    d = prism_smatrix_desc()
    d.grid = grid
    d.E0 = float(E0)
    d.alpha_max = float(alpha_max)
    d.f = int(f)
    d.beam_batch = int(beam_batch)
    check(lib.prism_smatrix_plan(ctypes.byref(d)))
    return d


def prism_beam_list(d: prism_smatrix_desc) -> np.ndarray:
    out = np.zeros((d.n_beams, 2), dtype=np.int32)
    check(lib.prism_beam_list(ctypes.byref(d), out.ctypes.data_as(ctypes.c_void_p), d.n_beams))
    return out


def prism_detector_bin_map(lam: float, Lw: float, alpha_aa: float, dalpha: float, n_bins: int, m: int) -> np.ndarray:
    out = np.zeros((m, m), dtype=np.int32)
    check(lib.prism_detector_bin_map(float(lam), float(Lw), float(alpha_aa), float(dalpha), int(n_bins), int(m),
                                     out.ctypes.data_as(ctypes.c_void_p)))
    return out


# ------------------------------------------------------------ potential --
def prism_detector_default_bins(grid: prism_grid, E0: float, dalpha: float = 1e-3):
    """(n_bins, alpha_aa): the default detector extent of a grid."""
    nb = ctypes.c_int32()
    a = ctypes.c_double()
    check(lib.prism_detector_default_bins(ctypes.byref(grid), float(E0), float(dalpha), ctypes.byref(nb),
                                          ctypes.byref(a)))
    return nb.value, a.value


def prism_project_potential(pos, species_idx, species, grid: prism_grid, device=None):
    """V [n_slices, n, n] float32 on the device from host atoms."""
    torch = _torch()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n_atoms = len(pos)
    atoms = (prism_atom * max(n_atoms, 1))()
    for i in range(n_atoms):
        atoms[i].x, atoms[i].y, atoms[i].z = float(pos[i, 0]), float(pos[i, 1]), float(pos[i, 2])
        atoms[i].species = int(species_idx[i])
    sp = (prism_species * len(species))()
    for i, s in enumerate(species):
        sp[i].n_gauss = len(s.amp)
        for g in range(len(s.amp)):
            sp[i].amp[g] = float(s.amp[g])
            sp[i].width[g] = float(s.width[g])
    need = ctypes.c_size_t()
    check(lib.prism_project_potential_workspace(n_atoms, ctypes.byref(need)))
    ws = _workspace(need.value, device)
    V = torch.empty((grid.n_slices, grid.n, grid.n), dtype=torch.float32, device=device or "cuda")
    check(lib.prism_project_potential(atoms, n_atoms, sp, len(species), ctypes.byref(grid), _dev(V), _dev(ws),
                                      need.value, _stream()))
    return V


def prism_build_smatrix(d: prism_smatrix_desc, V, ws=None, S=None):
    """S [n_beams, n/2, n/2] complex64 on the device."""
    torch = _torch()
    if S is None:
        S = torch.empty((d.n_beams, d.ns, d.ns), dtype=torch.complex64, device=V.device)
    if ws is None:
        ws = _workspace(d.build_ws_bytes, V.device)
    check(lib.prism_build_smatrix(ctypes.byref(d), _dev(V), _dev(S), _dev(ws), ws.numel(), _stream()))
    return S


def prism_build_smatrix_range(d: prism_smatrix_desc, V, S, first: int, count: int, ws=None):
    """Layers first .. first + count - 1 of S (the whole [n_beams, n/2, n/2] array)."""
    if ws is None:
        ws = _workspace(d.build_ws_bytes, V.device)
    check(lib.prism_build_smatrix_range(ctypes.byref(d), _dev(V), _dev(S), int(first), int(count), _dev(ws),
                                        ws.numel(), _stream()))
    return S


# -------------------------------------------------------- probe outputs --
@dataclass
class ProbePlan:
    plan: prism_probe_plan
    dev: object          # device tensor holding the plan tables
    xy: np.ndarray       # host positions the plan was made for


def _aberrations(C1, C3):
    if not C1 and not C3:
        return None
    ab = prism_aberrations()
    ab.C1, ab.C3 = float(C1), float(C3)
    return ctypes.byref(ab)


def _map(detector_map, side):
    m = np.ascontiguousarray(detector_map, dtype=np.int32)
    if m.shape != (side, side):
        raise ValueError(f"detector map must be int32 [{side}][{side}] (FFT order), got {m.shape}")
    return m


def prism_probe_plan_init(d: prism_smatrix_desc, xy, dalpha: float = 1e-3, n_bins: int = 0, C1: float = 0.0,
                          C3: float = 0.0, detector_map=None) -> prism_probe_plan:
    """detector_map: optional int32 [m_win][m_win] (FFT order) virtual
    detectors with n_bins detectors, in place of annular bins of width dalpha."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    p = prism_probe_plan()
    if detector_map is None:
        check(lib.prism_probe_plan_init(ctypes.byref(d), xy.ctypes.data_as(ctypes.c_void_p), len(xy), float(dalpha),
                                        int(n_bins), _aberrations(C1, C3), ctypes.byref(p)))
    else:
        m = _map(detector_map, d.m_win)
        check(lib.prism_probe_plan_init_map(ctypes.byref(d), xy.ctypes.data_as(ctypes.c_void_p), len(xy),
                                            m.ctypes.data_as(ctypes.c_void_p), int(n_bins), _aberrations(C1, C3),
                                            ctypes.byref(p)))
    return p


def prism_probe_plan_upload(d: prism_smatrix_desc, xy, dalpha: float = 1e-3, n_bins: int = 0,
                            device=None, C1: float = 0.0, C3: float = 0.0, detector_map=None) -> ProbePlan:
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    p = prism_probe_plan_init(d, xy, dalpha, n_bins, C1, C3, detector_map)
    dev = _workspace(p.plan_bytes, device)
    if detector_map is None:
        check(lib.prism_probe_plan_upload(ctypes.byref(d), xy.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p),
                                          _dev(dev), _stream()))
    else:
        m = _map(detector_map, d.m_win)
        check(lib.prism_probe_plan_upload_map(ctypes.byref(d), xy.ctypes.data_as(ctypes.c_void_p),
                                              m.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p), _dev(dev),
                                              _stream()))
    return ProbePlan(p, dev, xy)


def prism_probe_outputs(d: prism_smatrix_desc, S, plan: ProbePlan, precision: int = PRISM_FP32, ws=None, out=None):
    """out [n_probes, n_bins] float32 on the device."""
    torch = _torch()
    p = plan.plan
    if out is None:
        out = torch.empty((p.n_probes, p.n_bins), dtype=torch.float32, device=S.device)
    if ws is None:
        ws = _workspace(p.ws_bytes, S.device)
    check(lib.prism_probe_outputs(ctypes.byref(d), _dev(S), ctypes.byref(p), _dev(plan.dev), int(precision),
                                  _dev(out), _dev(ws), ws.numel(), _stream()))
    return out


def prism_probe_outputs_noalloc(d: prism_smatrix_desc, S, plan: ProbePlan, precision: int = PRISM_FP32, out=None):
    """prism_probe_outputs with the library's fixed device scratch as its
    workspace (no device allocation inside the call; `out` may be given)."""
    torch = _torch()
    p = plan.plan
    if out is None:
        out = torch.empty((p.n_probes, p.n_bins), dtype=torch.float32, device=S.device)
    check(lib.prism_probe_outputs_noalloc(ctypes.byref(d), _dev(S), ctypes.byref(p), _dev(plan.dev), int(precision),
                                          _dev(out), _stream()))
    return out


def prism_probe_diffraction(d: prism_smatrix_desc, S, plan: ProbePlan, precision: int = PRISM_FP32, ws=None,
                            out=None):
    """out [n_probes, m, m] float32 on the device: |FFT_M(psi_p)|^2 / M^4 (4D output)."""
    torch = _torch()
    p = plan.plan
    if out is None:
        out = torch.empty((p.n_probes, d.m_win, d.m_win), dtype=torch.float32, device=S.device)
    if ws is None:
        ws = _workspace(p.ws_bytes, S.device)
    check(lib.prism_probe_diffraction(ctypes.byref(d), _dev(S), ctypes.byref(p), _dev(plan.dev), int(precision),
                                      _dev(out), _dev(ws), ws.numel(), _stream()))
    return out


def _jobs(items):
    arr = (prism_probe_job * max(len(items), 1))()
    for k, it in enumerate(items):
        d, S, plan, out = it[:4]
        diff = it[4] if len(it) > 4 else None
        arr[k].desc = ctypes.pointer(d)
        arr[k].S = S.data_ptr()
        arr[k].plan = ctypes.pointer(plan.plan)
        arr[k].plan_dev = plan.dev.data_ptr()
        arr[k].out = out.data_ptr() if out is not None else None
        arr[k].diffraction = diff.data_ptr() if diff is not None else None
        arr[k].out_scale = float(it[5]) if len(it) > 5 else 1.0
        arr[k].accumulate = int(it[6]) if len(it) > 6 else 0
    return arr


def prism_probe_batch_workspace(items) -> int:
    """items: list of (desc, S, ProbePlan, out[, diffraction[, out_scale[, accumulate]]]) tuples."""
    need = ctypes.c_size_t()
    check(lib.prism_probe_batch_workspace(_jobs(items), len(items), ctypes.byref(need)))
    return need.value


def prism_probe_outputs_batched(items, precision: int = PRISM_FP32, ws=None):
    """Probe outputs of several (desc, S, ProbePlan, out) jobs in shared launches."""
    arr = _jobs(items)
    if ws is None:
        ws = _workspace(prism_probe_batch_workspace(items), items[0][1].device if items else None)
    check(lib.prism_probe_outputs_batched(arr, len(items), int(precision), _dev(ws), ws.numel(), _stream()))
    return [it[3] for it in items]


# ------------------------------------------------------------ multislice --
def multislice_workspace(grid: prism_grid, batch: int, n_probes: int) -> int:
    need = ctypes.c_size_t()
    check(lib.multislice_workspace(ctypes.byref(grid), int(batch), int(n_probes), ctypes.byref(need)))
    return need.value


def multislice_outputs(grid: prism_grid, E0: float, alpha_max: float, V, xy, dalpha: float = 1e-3,
                       n_bins: int = 0, batch: int = 64, ws=None, out=None, C1: float = 0.0, C3: float = 0.0,
                       detector_map=None):
    """out [n_probes, n_bins] float32 on the device.  detector_map: optional
    int32 [n][n] (FFT order) virtual detectors with n_bins detectors."""
    torch = _torch()
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    if detector_map is None and n_bins <= 0:
        n_bins = prism_detector_default_bins(grid, E0, dalpha)[0]
    if ws is None:
        ws = _workspace(multislice_workspace(grid, batch, len(xy)), V.device)
    if out is None:
        out = torch.empty((len(xy), n_bins), dtype=torch.float32, device=V.device)
    if detector_map is None:
        check(lib.multislice_outputs(ctypes.byref(grid), float(E0), float(alpha_max), _aberrations(C1, C3), _dev(V),
                                     xy.ctypes.data_as(ctypes.c_void_p), len(xy), float(dalpha), int(n_bins),
                                     int(batch), _dev(out), _dev(ws), ws.numel(), _stream()))
    else:
        m = _map(detector_map, grid.n)
        check(lib.multislice_outputs_map(ctypes.byref(grid), float(E0), float(alpha_max), _aberrations(C1, C3),
                                         _dev(V), xy.ctypes.data_as(ctypes.c_void_p), len(xy),
                                         m.ctypes.data_as(ctypes.c_void_p), int(n_bins), int(batch), _dev(out),
                                         _dev(ws), ws.numel(), _stream()))
    return out


# ------------------------------------------- streaming memory model --
def _pinned(shape, dtype):
    torch = _torch()
    return torch.empty(shape, dtype=dtype, pin_memory=True)


def _side_stream(st):
    return st if st is not None else _torch().cuda.Stream()


def prism_streaming_build_workspace(d: prism_smatrix_desc) -> int:
    need = ctypes.c_size_t()
    check(lib.prism_streaming_build_workspace(ctypes.byref(d), ctypes.byref(need)))
    return need.value


def prism_build_smatrix_streaming(d: prism_smatrix_desc, V_host, S_host=None, ws=None, h2d=None, d2h=None):
    """S-matrix into host memory (complex64 [n_beams, ns, ns], page-locked) from
    a host potential V_host (float32 [n_slices, n, n]); complete once the
    current stream has drained."""
    torch = _torch()
    assert V_host.device.type == "cpu" and V_host.dtype == torch.float32 and V_host.is_contiguous()
    if S_host is None:
        S_host = _pinned((d.n_beams, d.ns, d.ns), torch.complex64)
    if ws is None:
        ws = _workspace(prism_streaming_build_workspace(d))
    h2d, d2h = _side_stream(h2d), _side_stream(d2h)
    check(lib.prism_build_smatrix_streaming(ctypes.byref(d), _dev(V_host), _dev(S_host), _dev(ws), ws.numel(),
                                            _stream(), ctypes.c_void_p(h2d.cuda_stream),
                                            ctypes.c_void_p(d2h.cuda_stream)))
    return S_host


def prism_probe_streaming_workspace(d: prism_smatrix_desc, plan: ProbePlan, beam_chunk: int) -> int:
    need = ctypes.c_size_t()
    check(lib.prism_probe_streaming_workspace(ctypes.byref(d), ctypes.byref(plan.plan), int(beam_chunk),
                                              ctypes.byref(need)))
    return need.value


def prism_probe_outputs_streaming(d: prism_smatrix_desc, S_host, plan: ProbePlan, precision: int = PRISM_FP32,
                                  beam_chunk: int = 128, ws=None, out=None, diffraction: bool = False, h2d=None):
    """Probe outputs (or the 4D output with diffraction=True) from a host
    S-matrix streamed in beam chunks."""
    torch = _torch()
    assert S_host.device.type == "cpu" and S_host.dtype == torch.complex64 and S_host.is_contiguous()
    p = plan.plan
    if out is None:
        shape = (p.n_probes, d.m_win, d.m_win) if diffraction else (p.n_probes, p.n_bins)
        out = torch.empty(shape, dtype=torch.float32, device=plan.dev.device)
    if ws is None:
        ws = _workspace(prism_probe_streaming_workspace(d, plan, beam_chunk), plan.dev.device)
    h2d = _side_stream(h2d)
    o3, o4 = (None, _dev(out)) if diffraction else (_dev(out), None)
    check(lib.prism_probe_outputs_streaming(ctypes.byref(d), _dev(S_host), ctypes.byref(p), _dev(plan.dev),
                                            int(precision), int(beam_chunk), o3, o4, _dev(ws), ws.numel(),
                                            _stream(), ctypes.c_void_p(h2d.cuda_stream)))
    return out


def prism_probe_chunked_workspace(d: prism_smatrix_desc, plan: ProbePlan, beam_chunk: int) -> int:
    need = ctypes.c_size_t()
    check(lib.prism_probe_chunked_workspace(ctypes.byref(d), ctypes.byref(plan.plan), int(beam_chunk),
                                            ctypes.byref(need)))
    return need.value


def prism_probe_outputs_chunked(d: prism_smatrix_desc, S, plan: ProbePlan, precision: int = PRISM_FP32,
                                beam_chunk: int = 128, ws=None, out=None, diffraction: bool = False):
    """Probe outputs (or the 4D output) from a device S-matrix contracted in beam chunks."""
    torch = _torch()
    p = plan.plan
    if out is None:
        shape = (p.n_probes, d.m_win, d.m_win) if diffraction else (p.n_probes, p.n_bins)
        out = torch.empty(shape, dtype=torch.float32, device=S.device)
    if ws is None:
        ws = _workspace(prism_probe_chunked_workspace(d, plan, beam_chunk), S.device)
    o3, o4 = (None, _dev(out)) if diffraction else (_dev(out), None)
    check(lib.prism_probe_outputs_chunked(ctypes.byref(d), _dev(S), ctypes.byref(p), _dev(plan.dev), int(precision),
                                          int(beam_chunk), o3, o4, _dev(ws), ws.numel(), _stream()))
    return out


def multislice_streaming_workspace(grid: prism_grid, batch: int, n_probes: int) -> int:
    need = ctypes.c_size_t()
    check(lib.multislice_streaming_workspace(ctypes.byref(grid), int(batch), int(n_probes), ctypes.byref(need)))
    return need.value


def multislice_outputs_streaming(grid: prism_grid, E0: float, alpha_max: float, V_host, xy, dalpha: float = 1e-3,
                                 n_bins: int = 0, batch: int = 64, ws=None, out=None, C1: float = 0.0,
                                 C3: float = 0.0, h2d=None):
    """multislice_outputs with the potential in host memory, streamed a slice ahead."""
    torch = _torch()
    assert V_host.device.type == "cpu" and V_host.dtype == torch.float32 and V_host.is_contiguous()
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    if n_bins <= 0:
        n_bins = prism_detector_default_bins(grid, E0, dalpha)[0]
    if ws is None:
        ws = _workspace(multislice_streaming_workspace(grid, batch, len(xy)))
    if out is None:
        out = torch.empty((len(xy), n_bins), dtype=torch.float32, device=ws.device)
    h2d = _side_stream(h2d)
    check(lib.multislice_outputs_streaming(ctypes.byref(grid), float(E0), float(alpha_max), _aberrations(C1, C3),
                                           _dev(V_host), xy.ctypes.data_as(ctypes.c_void_p), len(xy), float(dalpha),
                                           int(n_bins), int(batch), _dev(out), _dev(ws), ws.numel(), _stream(),
                                           ctypes.c_void_p(h2d.cuda_stream)))
    return out


def prism_set_build_streams(n: int):
    """Streams of the S-matrix build, 1-4, or 0 (the default) for 4 up to
    1024^2 grids and 1 above: each beam batch is split into that many parts
    that overlap on the current stream and partner streams; 1 runs everything
    on the current stream."""
    check(lib.prism_set_build_streams(int(n)))


def prism_device_copy(src, dst):
    """Copy tensor src into dst (same byte size, multiple of 16) with the
    library's plain streaming copy kernel on the current stream."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("prism_device_copy: size mismatch")
    check(lib.prism_device_copy(_dev(src), _dev(dst), nbytes, _stream()))


# ---------------------------------------------------------------- timing --
def prism_timing_enable(enable: bool = True):
    check(lib.prism_timing_enable(1 if enable else 0))


def prism_timing_reset():
    check(lib.prism_timing_reset())


def prism_timing_read(cls: int):
    """(total device ms, launches) of kernel class `cls` since the last reset."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    check(lib.prism_timing_read(int(cls), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value
