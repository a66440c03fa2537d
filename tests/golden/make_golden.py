"""Writes the oracle's regression fixtures in this folder.  Calls only the
oracle and the seeded input generators; run from the repository root:

    python tests/golden/make_golden.py                      # 64^2 fixture (seconds)
    python tests/golden/make_golden.py --workload prism_f4_np_1024 --processes 8
    python tests/golden/make_golden.py --workload prism_f8_np_2048 --processes 8

The full-size fixtures hold FP64 3D outputs of a benchmark workload on its
16 x 16 probe subset (every (scan/16)-th probe per axis): every beam of the
aperture through every slice, streamed into the subset's windows.  For the
1024^2 nanoparticle cell they also hold multislice on the same probes.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def tiny_prism_case():
    """A 64^2, 2-slice random cell, PRISM at f = 2 and multislice on three probes."""
    w, pos, sp = W.small_workload(n=64, cell=(10.0, 10.0, 4.0), n_atoms=8, f=2, seed=11)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    beams = O.beam_set(w.n, w.cell[0], lam, w.alpha_max, w.f)
    S = O.build_smatrix(V, w.cell[0], w.dz, lam, sig, beams)
    xy = np.array([[0.0, 0.0], [2.3, 7.9], [9.9, 4.1]])
    prism = O.prism_outputs(S, beams, w.cell[0], w.n, lam, w.f, xy)
    ms = O.multislice_outputs(V, w.cell[0], w.dz, lam, sig, w.alpha_max, xy)
    return xy, prism, ms


def write_tiny():
    xy, prism, ms = tiny_prism_case()
    with open(os.path.join(HERE, "tiny_prism_f2_64.txt"), "w") as fh:
        fh.write("# Oracle regression fixture written by tests/golden/make_golden.py (oracle only):\n")
        fh.write("# 64^2 random cell (small_workload n=64, cell 10 x 10 x 4 A, 8 atoms, seed 11), 80 keV,\n")
        fh.write("# 20 mrad; rows: probe x, y (A), then the PRISM f=2 and the multislice 3D outputs\n")
        fh.write("# (1 mrad bins) of that probe.\n")
        for p in range(len(xy)):
            fh.write(f"probe {float(xy[p, 0])!r} {float(xy[p, 1])!r}\n")
            fh.write("prism " + " ".join(repr(float(v)) for v in prism[p]) + "\n")
            fh.write("multislice " + " ".join(repr(float(v)) for v in ms[p]) + "\n")


def subset_positions(w):
    """The workload's scan restricted to a 16 x 16 probe subset."""
    return W.scan_positions(w.cell, *w.scan, sub=w.scan[0] // 16)


def fixture_path(name):
    return os.path.join(HERE, f"{name}_fp64_subset.npz")


def write_full(name, processes, with_multislice):
    w = W.WORKLOADS[name]
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    L = w.cell[0]
    t0 = time.time()
    pos, sp = W.atoms_for(w)
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    print(f"[golden] {name}: potential ({len(pos)} atoms) {time.time() - t0:.0f} s", flush=True)
    xy = subset_positions(w)
    beams = O.beam_set(w.n, L, lam, w.alpha_max, w.f)
    out = {"probe_xy": xy, "beams": beams}
    t0 = time.time()
    out["prism"] = O.prism_outputs_streamed(V, L, w.dz, lam, sig, beams, w.n, w.f, xy,
                                            processes=processes, groups=8 * processes)
    print(f"[golden] {name}: PRISM f={w.f} ({len(beams)} beams, {len(xy)} probes) {time.time() - t0:.0f} s",
          flush=True)
    if with_multislice:
        t0 = time.time()
        out["multislice"] = O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy, processes=processes)
        print(f"[golden] {name}: multislice ({len(xy)} probes) {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(fixture_path(name), **out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default=None)
    ap.add_argument("--processes", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--no-multislice", action="store_true")
    a = ap.parse_args()
    if a.workload is None:
        write_tiny()
    else:
        write_full(a.workload, a.processes, not a.no_multislice)


if __name__ == "__main__":
    main()
