"""Writes the oracle's regression fixtures in this folder.  Calls only the
oracle and the seeded input generators; run from the repository root:

    python tests/golden/make_golden.py
"""
import os
import sys

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


def main():
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


if __name__ == "__main__":
    main()
