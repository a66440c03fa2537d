"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates its arguments, and its host-side integer planning
(beam sets, detector bin maps) equals the oracle's bit for bit."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1706_08563_amd as P
    return P


def test_library_exports_every_declared_symbol():
    P = _lib()
    hdr = open(os.path.join(ROOT, "include", "prism.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"^\s*(?:int|const char\s*\*)\s+(\w+)\s*\(", hdr, flags=re.M))
    assert declared, "no declarations parsed"
    raw = ctypes.CDLL(P.LIB_PATH)
    for name in declared:
        assert hasattr(raw, name), name
    assert declared == set(P.EXPORTED)


def test_grid_validation_codes():
    P = _lib()
    g = P.prism_grid_init((20.0, 20.0, 20.0), 2.0, 256)
    assert g.n_slices == 10
    with pytest.raises(P.PrismError) as e:
        P.prism_grid_init((20.0, 20.0, 20.0), 2.0, 250)
    assert e.value.code == P.PRISM_E_UNSUPPORTED
    with pytest.raises(P.PrismError) as e:
        P.prism_grid_init((20.0, 21.0, 20.0), 2.0, 256)
    assert e.value.code == P.PRISM_E_UNSUPPORTED
    with pytest.raises(P.PrismError) as e:
        P.prism_grid_init((20.0, 20.0, 20.0), 0.0, 256)
    assert e.value.code == P.PRISM_E_INVAL
    g = P.prism_grid_init((20.0, 20.0, 7.0), 2.0, 64)
    assert g.n_slices == 4


def test_smatrix_plan_validation_codes():
    P = _lib()
    g = P.prism_grid_init((20.0, 20.0, 20.0), 2.0, 256)
    for args, code in [((80e3, 0.2, 2), P.PRISM_E_UNSUPPORTED),   # alpha_max above alpha_AA
                       ((80e3, 0.02, 3), P.PRISM_E_UNSUPPORTED),   # f does not divide n/2
                       ((80e3, 0.02, 16), P.PRISM_E_UNSUPPORTED),  # window 8 < 16
                       ((-1.0, 0.02, 2), P.PRISM_E_INVAL),
                       ((80e3, 0.02, 0), P.PRISM_E_INVAL)]:
        with pytest.raises(P.PrismError) as e:
            P.prism_smatrix_plan(g, *args)
        assert e.value.code == code, args


@pytest.mark.parametrize("cfg", ["prism_f2_sc_256", "prism_f4_np_1024", "prism_f8_np_2048"])
def test_plan_constants_and_beams_match_oracle(cfg):
    P = _lib()
    w = W.WORKLOADS[cfg]
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    lam = O.wavelength(w.E0)
    assert abs(d.lambda_ - lam) <= 1e-15 * lam
    assert abs(d.sigma - O.interaction_constant(w.E0)) <= 1e-15 * d.sigma
    assert d.alpha_aa == O.alpha_aa(lam, w.n, w.cell[0])
    ob = O.beam_set(w.n, w.cell[0], lam, w.alpha_max, w.f)
    gb = P.prism_beam_list(d)
    assert gb.shape == ob.shape and np.array_equal(gb, ob)
    assert d.m_win == w.n // 2 // w.f


@pytest.mark.parametrize("m,f,cfg", [(64, 2, "prism_f2_sc_256"), (128, 4, "prism_f4_np_1024"),
                                      (128, 8, "prism_f8_np_2048"), (256, 1, "prism_f2_sc_256"),
                                      (1024, 1, "multislice_np_1024")])
def test_bin_map_bit_exact(m, f, cfg):
    P = _lib()
    w = W.WORKLOADS[cfg]
    L = w.cell[0]
    lam = O.wavelength(w.E0)
    a_aa = O.alpha_aa(lam, w.n, L)
    nb = O.default_n_bins(lam, w.n, L, 1e-3)
    Lw = L / f
    ref = O.bin_map(lam, m, Lw, a_aa, 1e-3, nb)
    got = P.prism_detector_bin_map(lam, Lw, a_aa, 1e-3, nb, m)
    assert np.array_equal(ref, got)


def test_bin_map_edges_and_explicit_bin_count():
    P = _lib()
    lam, Lw = 0.025, 25.0
    for m, nb in [(64, 16), (64, 5), (32, 3)]:
        a_aa = O.alpha_aa(lam, 2 * m, 2 * Lw)
        assert np.array_equal(P.prism_detector_bin_map(lam, Lw, a_aa, 1e-3, nb, m),
                              O.bin_map(lam, m, Lw, a_aa, 1e-3, nb))


@pytest.mark.parametrize("cfg", ["prism_f2_sc_256", "multislice_np_1024", "prism_f8_np_2048"])
@pytest.mark.parametrize("dalpha", [1e-3, 2.5e-3, 0.7e-3])
def test_detector_default_bins_query_matches_oracle(cfg, dalpha):
    """The library reports the default detector extent (the binding computes
    none of it): alpha_AA and ceil(alpha_AA / dalpha) equal the oracle's."""
    P = _lib()
    w = W.WORKLOADS[cfg]
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    lam = O.wavelength(w.E0)
    nb, a = P.prism_detector_default_bins(g, w.E0, dalpha)
    assert a == O.alpha_aa(lam, w.n, w.cell[0])
    assert nb == O.default_n_bins(lam, w.n, w.cell[0], dalpha)
    if dalpha == 1e-3:
        assert nb == (134 if w.n == 256 else 65)
    for bad in ((0.0, dalpha), (w.E0, 0.0), (w.E0, -1e-3)):
        with pytest.raises(P.PrismError) as e:
            P.prism_detector_default_bins(g, *bad)
        assert e.value.code == P.PRISM_E_INVAL


def test_probe_plan_work_tiles_follow_the_scan_lattice():
    """On the benchmark scans (probes every 4 S-grid pixels, 128-pixel
    windows) every window is tiled at its own phase: exactly (128/16)^2 = 64
    work tiles per probe, and every work tile holds 64 probes, one full
    workgroup of the MFMA contraction (no products outside a window, no
    partly filled probe chunk)."""
    P = _lib()
    for name in ("prism_f4_np_1024", "prism_f8_np_2048"):
        w = W.WORKLOADS[name]
        g = P.prism_grid_init(w.cell, w.dz, w.n)
        d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
        xy = W.scan_positions(w.cell, *w.scan)
        p = P.prism_probe_plan_init(d, xy)
        assert d.m_win == 128
        assert p.n_entries == 64 * len(xy), name
        assert p.max_per_tile == 64 and p.n_tiles == len(xy), name
    # irregular positions: one tiling phase per corner offset would leave the
    # 64-probe chunks nearly empty, so the plan keeps the 16-aligned grid,
    # where a window not aligned to it overlaps 9 tiles per axis
    rng = np.random.default_rng(5)
    xr = rng.uniform(0.0, w.cell[0], size=(4096, 2))
    p = P.prism_probe_plan_init(d, xr)
    assert 64 * len(xr) < p.n_entries <= 81 * len(xr)
    assert p.n_tiles <= (d.ns // 16) ** 2


def test_probe_plan_sizes():
    P = _lib()
    w = W.WORKLOADS["prism_f2_sc_256"]
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    xy = W.scan_positions(w.cell, *w.scan)
    p = P.prism_probe_plan_init(d, xy)
    assert p.n_probes == 256 and p.n_bins == 134
    # each probe window (64 px) overlaps 4 or 5 tiles of 16 px per axis
    assert 256 * 16 <= p.n_entries <= 256 * 25
    # the binned pixel count equals the oracle bin map's
    lam = O.wavelength(w.E0)
    bm = O.bin_map(lam, 64, w.cell[0] / 2, O.alpha_aa(lam, w.n, w.cell[0]), 1e-3, 134)
    assert p.n_binned == int((bm >= 0).sum())
    with pytest.raises(P.PrismError) as e:
        P.prism_probe_plan_init(d, np.array([[np.nan, 0.0]]))
    assert e.value.code == P.PRISM_E_INVAL


def test_one_hip_runtime_whatever_the_import_order():
    """The library and PyTorch share one HIP runtime even when the package is
    imported before torch (two runtimes would make torch's streams and
    memory invalid for the library)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1706_08563_amd\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read()\n"
            "libs = {l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}\n"
            "print(len(libs))\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1"


def test_build_stream_count_validation():
    import paper_1706_08563_amd as P
    for bad in (5, -1):
        with pytest.raises(P.PrismError) as e:
            P.prism_set_build_streams(bad)
        assert e.value.code == P.PRISM_E_INVAL
    for ok in (1, 3, 4, 2, 0):                        # ends on the default (by grid size)
        P.prism_set_build_streams(ok)


def test_device_copy_argument_checks():
    import ctypes
    import paper_1706_08563_amd as P
    lib = P.lib
    buf = ctypes.create_string_buffer(64)
    base = ctypes.addressof(buf)
    aligned = (base + 15) // 16 * 16
    # rejected on the host before any device work: NULL, size, alignment, overlap
    assert lib.prism_device_copy(None, ctypes.c_void_p(aligned), 16, None) == P.PRISM_E_INVAL
    assert lib.prism_device_copy(ctypes.c_void_p(aligned), ctypes.c_void_p(aligned + 16), 8, None) == P.PRISM_E_INVAL
    assert lib.prism_device_copy(ctypes.c_void_p(aligned + 4), ctypes.c_void_p(aligned + 32), 16, None) == P.PRISM_E_INVAL
    assert lib.prism_device_copy(ctypes.c_void_p(aligned), ctypes.c_void_p(aligned + 16), 32, None) == P.PRISM_E_INVAL
    assert lib.prism_device_copy(ctypes.c_void_p(aligned), ctypes.c_void_p(aligned + 16), 0, None) == P.PRISM_OK


def test_detector_map_plans_and_validation():
    """Plans with a caller's detector map: binned pixel count is the map's
    mapped pixels; entries outside [-1, n_bins) and maps of the wrong side are
    refused; annular and map plans do not upload for each other."""
    P = _lib()
    w = W.WORKLOADS["prism_f2_sc_256"]
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    xy = W.scan_positions(w.cell, 4, 4)
    M = d.m_win
    rng = np.random.default_rng(5)
    dmap = rng.integers(-1, 7, size=(M, M)).astype(np.int32)
    p = P.prism_probe_plan_init(d, xy, n_bins=7, detector_map=dmap)
    assert p.n_bins == 7 and p.dalpha == 0.0 and p.n_binned == int((dmap >= 0).sum())
    for bad, nb in ((np.where(dmap == 3, 7, dmap), 7), (np.where(dmap == 3, -2, dmap), 7), (dmap, 0)):
        with pytest.raises(P.PrismError) as e:
            P.prism_probe_plan_init(d, xy, n_bins=nb, detector_map=bad)
        assert e.value.code == P.PRISM_E_INVAL
    with pytest.raises(ValueError):
        P.prism_probe_plan_init(d, xy, n_bins=7, detector_map=dmap[:-1])
    ct = P._lib.ctypes
    pa = P.prism_probe_plan_init(d, xy)
    fake = ct.c_void_p(0x1000)           # never dereferenced: the calls fail on their arguments first
    xyc = np.ascontiguousarray(xy)
    dm = np.ascontiguousarray(dmap)
    assert P.lib.prism_probe_plan_upload_map(ct.byref(d), xyc.ctypes.data_as(ct.c_void_p),
                                             dm.ctypes.data_as(ct.c_void_p), ct.byref(pa), fake, None) \
        == P.PRISM_E_INVAL
    assert P.lib.prism_probe_plan_upload(ct.byref(d), xyc.ctypes.data_as(ct.c_void_p), ct.byref(p), fake, None) \
        == P.PRISM_E_INVAL


def test_build_range_argument_checks():
    """prism_build_smatrix_range refuses ranges outside [0, n_beams) and a
    short workspace before any device work (fake device pointers)."""
    P = _lib()
    w = W.WORKLOADS["prism_f2_sc_256"]
    g = P.prism_grid_init(w.cell, w.dz, w.n)
    d = P.prism_smatrix_plan(g, w.E0, w.alpha_max, w.f)
    ct = P._lib.ctypes
    fake = ct.c_void_p(256)
    for first, cnt in ((-1, 1), (0, -1), (0, d.n_beams + 1), (d.n_beams, 1), (d.n_beams - 3, 4)):
        rc = P.lib.prism_build_smatrix_range(ct.byref(d), fake, fake, first, cnt, fake, d.build_ws_bytes, None)
        assert rc == P.PRISM_E_INVAL, (first, cnt)
    rc = P.lib.prism_build_smatrix_range(ct.byref(d), fake, fake, 0, 1, fake, d.build_ws_bytes - 1, None)
    assert rc == P.PRISM_E_WORKSPACE
    # an empty range is accepted and does nothing
    assert P.lib.prism_build_smatrix_range(ct.byref(d), fake, fake, 5, 0, fake, d.build_ws_bytes, None) == P.PRISM_OK


def test_timing_classes_match_the_header():
    """Every timing class the binding names is readable, and the next index is
    rejected (the header's PRISM_TIMING_CLASSES)."""
    import paper_1706_08563_amd as P
    hdr = open(os.path.join(ROOT, "include", "prism.h")).read()
    n = int(re.search(r"#define PRISM_TIMING_CLASSES\s+(\d+)", hdr).group(1))
    assert sorted(P.TIMING_CLASSES.values()) == list(range(n))
    for name, cls in P.TIMING_CLASSES.items():
        assert re.search(r"#define PRISM_K_%s\s+%d\b" % (name.upper(), cls), hdr), name
        P.prism_timing_read(cls)
    with pytest.raises(P.PrismError):
        P.prism_timing_read(n)
