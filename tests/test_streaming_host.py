"""Host-side checks of the streaming memory model (no GPU): workspace sizes
of the streaming entry points against the layout they document, argument
validation that happens before any device call, and the memory planner's
choices."""
import ctypes

import numpy as np
import pytest

import workloads as W


def _P():
    import paper_1706_08563_amd as P
    return P


def _desc(P, n=1024, f=4, beam_batch=0):
    w = W.WORKLOADS["prism_f4_np_1024"]
    g = P.prism_grid_init(w.cell, w.dz, n)
    return w, g, P.prism_smatrix_plan(g, w.E0, w.alpha_max, f, beam_batch=beam_batch)


def test_streaming_build_workspace_is_small_and_scales_with_batch():
    P = _P()
    w, g, d = _desc(P)
    n = g.n
    full = P.prism_streaming_build_workspace(d)
    # two potential slices, one transmission slice and its row spectrum, the
    # band wave buffer and two S staging buffers of one batch, plus small tables
    core = 2 * 4 * n * n + 2 * 8 * n * n + d.n_beams * (4 * n * n + 2 * 8 * d.ns * d.ns)
    assert core <= full <= core + (1 << 20)
    _, _, d8 = _desc(P, beam_batch=8)
    small = P.prism_streaming_build_workspace(d8)
    core8 = 2 * 4 * n * n + 2 * 8 * n * n + 8 * (4 * n * n + 2 * 8 * d.ns * d.ns)
    assert core8 <= small <= core8 + (1 << 20)
    # with batching, the resident build still holds every slice's transmission,
    # the potential and the whole S-matrix; streaming holds none of them
    resident = d8.build_ws_bytes + d8.smatrix_bytes + g.n_slices * n * n * 4
    assert small * 20 < resident


def test_streaming_synthesis_workspace_and_validation():
    P = _P()
    w, g, d = _desc(P)
    xy = W.scan_positions(w.cell, 8, 8)
    plan = P.prism_probe_plan_init(d, xy)

    class _Plan:           # the workspace query reads only the host plan
        pass
    pp = _Plan()
    pp.plan = plan
    a = P.prism_probe_streaming_workspace(d, pp, 64)
    b = P.prism_probe_streaming_workspace(d, pp, 128)
    assert b - a >= 2 * 64 * d.ns * d.ns * 8 + 64 * 64 * 8 - 4096
    for bad in (0, -3, d.n_beams + 1):
        with pytest.raises(P.PrismError) as e:
            P.prism_probe_streaming_workspace(d, pp, bad)
        assert e.value.code == P.PRISM_E_INVAL
    lib = P._lib.lib
    # NULL host S-matrix and bad precision are rejected before any device work
    rc = lib.prism_probe_outputs_streaming(ctypes.byref(d), None, ctypes.byref(plan), ctypes.c_void_p(16), 0, 64,
                                           ctypes.c_void_p(16), None, ctypes.c_void_p(16), 1 << 40, None, None)
    assert rc == P.PRISM_E_INVAL
    rc = lib.prism_probe_outputs_streaming(ctypes.byref(d), ctypes.c_void_p(16), ctypes.byref(plan),
                                           ctypes.c_void_p(16), 7, 64, ctypes.c_void_p(16), None,
                                           ctypes.c_void_p(16), 1 << 40, None, None)
    assert rc == P.PRISM_E_INVAL
    rc = lib.prism_probe_outputs_streaming(ctypes.byref(d), ctypes.c_void_p(16), ctypes.byref(plan),
                                           ctypes.c_void_p(16), 0, 64, ctypes.c_void_p(16), None,
                                           ctypes.c_void_p(16), 100, None, None)
    assert rc == P.PRISM_E_WORKSPACE


def test_streaming_build_and_multislice_validation():
    P = _P()
    w, g, d = _desc(P)
    lib = P._lib.lib
    rc = lib.prism_build_smatrix_streaming(ctypes.byref(d), None, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                           1 << 40, None, None, None)
    assert rc == P.PRISM_E_INVAL
    rc = lib.prism_build_smatrix_streaming(ctypes.byref(d), ctypes.c_void_p(16), ctypes.c_void_p(16),
                                           ctypes.c_void_p(16), 10, None, None, None)
    assert rc == P.PRISM_E_WORKSPACE
    res = P.multislice_workspace(g, 16, 100)
    st = P.multislice_streaming_workspace(g, 16, 100)
    n = g.n
    # streaming keeps one transmission slice and two potential slices instead of all slices
    assert res - st == (g.n_slices - 1) * 8 * n * n - 2 * 4 * n * n
    xy = np.zeros((4, 2))
    rc = lib.multislice_outputs_streaming(ctypes.byref(g), 80e3, 0.02, None, None,
                                          xy.ctypes.data_as(ctypes.c_void_p), 4, 1e-3, 0, 4, ctypes.c_void_p(16),
                                          ctypes.c_void_p(16), 1 << 40, None, None)
    assert rc == P.PRISM_E_INVAL


def test_memory_planner_choices():
    P = _P()
    from paper_1706_08563_amd import memory as M
    w = W.WORKLOADS["prism_f4_np_1024"]
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    xy = W.scan_positions(w.cell, 32, 32)
    big = M.plan_memory(g, w.E0, w.alpha_max, w.f, xy, 1 << 40)
    assert big.mode == "single" and big.peak_bytes == big.single_bytes
    for budget in (big.single_bytes - 1, big.single_bytes // 4, 1 << 30):
        mp = M.plan_memory(g, w.E0, w.alpha_max, w.f, xy, budget)
        assert mp.mode == "streaming" and mp.peak_bytes <= budget
        assert 1 <= mp.beam_chunk <= mp.desc.n_beams and 1 <= mp.probe_chunk <= len(xy)
    # a tighter budget never gets larger chunks
    a = M.plan_memory(g, w.E0, w.alpha_max, w.f, xy, big.single_bytes // 4)
    b = M.plan_memory(g, w.E0, w.alpha_max, w.f, xy, 1 << 30)
    assert (b.desc.beam_batch or b.desc.n_beams) <= (a.desc.beam_batch or a.desc.n_beams)
    assert b.beam_chunk * b.probe_chunk <= a.beam_chunk * a.probe_chunk
    with pytest.raises(MemoryError):
        M.plan_memory(g, w.E0, w.alpha_max, w.f, xy, 1 << 20)
    with pytest.raises(MemoryError):
        M.plan_memory(g, w.E0, w.alpha_max, w.f, xy, 1 << 30, force="single")
    forced = M.plan_memory(g, w.E0, w.alpha_max, w.f, xy, 1 << 40, force="streaming")
    assert forced.mode == "streaming"
