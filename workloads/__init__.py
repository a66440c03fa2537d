"""Seeded synthetic inputs for STEM simulation workloads.

This module is shared by the FP64 oracle tests, the GPU parity tests and the
benchmark.  It only *generates inputs*: atom coordinates, species parameters,
grid/beam/scan parameters, and random arrays used as operands.  It performs no
step of the simulation itself (no potential, no propagation, no beams, no
detector arithmetic).

Structures stand in for the paper's benchmark samples (the amorphous carbon
cell of the Algorithm Comparison benchmark, the Ruddlesden-Popper oxide and the
FePt particle), none of which is reproduced here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Species:
    """Projected potential of one atomic species as a sum of 2D Gaussians.

    amp[i] is the 2D integral of Gaussian i of the projected potential (V*A^2),
    width[i] its standard deviation (A).
    """
    amp: tuple
    width: tuple


def species_for_z(z: int) -> Species:
    """Two-Gaussian species with amplitudes (20, 5) V*A^2 scaled by Z/6."""
    return Species(amp=(20.0 * z / 6.0, 5.0 * z / 6.0), width=(0.3, 0.8))


@dataclass(frozen=True)
class Workload:
    name: str
    cell: tuple            # (Lx, Ly, Lz) in A
    n: int                 # real-space grid side (pixels)
    dz: float              # slice thickness (A)
    E0: float              # beam energy (eV)
    alpha_max: float       # probe semi-angle / beam aperture (rad)
    f: int                 # PRISM interpolation factor (0: multislice only)
    scan: tuple            # (nx, ny) probe grid
    species: tuple = field(default_factory=tuple)
    seed: int = 0
    structure: str = "sc"  # "sc" simple cubic, "np" nanoparticle in amorphous matrix, "amorphous"

    @property
    def n_slices(self) -> int:
        return int(np.ceil(self.cell[2] / self.dz - 1e-12))


# ---------------------------------------------------------------------------
# Workload definitions: a small PRISM case (256^2, f = 2, simple cubic), the
# 1024^2 multislice case, the 1024^2 PRISM f = 4 case (the benchmark
# workload) and the 2048^2 PRISM f = 8 case, on the nanoparticle-in-matrix
# cell; each named by method, f, structure and grid.
# ---------------------------------------------------------------------------
AU = species_for_z(79)
C = species_for_z(6)
SC1 = Species(amp=(20.0, 5.0), width=(0.3, 0.8))

WORKLOADS = {w.name: w for w in (
    Workload("prism_f2_sc_256", (20.0, 20.0, 20.0), 256, 2.0, 80e3, 0.020, 2,
             (16, 16), (SC1,), seed=0, structure="sc"),
    Workload("multislice_np_1024", (100.0, 100.0, 100.0), 1024, 2.0, 200e3, 0.020, 0,
             (64, 64), (AU, C), seed=1, structure="np"),
    Workload("prism_f4_np_1024", (100.0, 100.0, 100.0), 1024, 2.0, 200e3, 0.020, 4,
             (128, 128), (AU, C), seed=1, structure="np"),
    Workload("prism_f8_np_2048", (200.0, 200.0, 100.0), 2048, 2.0, 200e3, 0.020, 8,
             (256, 256), (AU, C), seed=3, structure="np"),
)}


# ---------------------------------------------------------------------------
# Structure generators.
# ---------------------------------------------------------------------------
def simple_cubic(a: float, reps: int, jitter: float, rng: np.random.Generator):
    """Sites (i, j, k) * a for i, j, k in [0, reps), Gaussian jitter per coordinate."""
    g = np.arange(reps, dtype=np.float64) * a
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    return pos, np.zeros(len(pos), dtype=np.int32)


def fcc_sphere(a: float, radius: float, centre, jitter: float, rng: np.random.Generator):
    """FCC lattice (4-atom basis) sites within `radius` of `centre`."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    nmax = int(np.ceil(radius / a)) + 1
    r = np.arange(-nmax, nmax + 1, dtype=np.float64)
    i, j, k = np.meshgrid(r, r, r, indexing="ij")
    cells = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    keep = np.sum(sites * sites, axis=1) <= radius * radius
    pos = sites[keep] + np.asarray(centre, dtype=np.float64)
    pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    return pos


def nanoparticle_in_amorphous(cell, a_fcc=4.08, radius=30.0, jitter=0.08,
                              density=0.05, rng=None):
    """Z=79 FCC particle at the cell centre in a uniform-random Z=6 matrix.

    Species index 0 is the particle species, 1 the matrix species.  Matrix
    atoms inside the particle radius are removed.
    """
    rng = rng if rng is not None else np.random.default_rng(0)
    cell = np.asarray(cell, dtype=np.float64)
    centre = cell / 2.0
    radius = min(radius, 0.3 * cell[0], 0.3 * cell[1], 0.45 * cell[2])
    p = fcc_sphere(a_fcc, radius, centre, jitter, rng)
    n_matrix = int(round(density * float(np.prod(cell))))
    m = rng.uniform(0.0, 1.0, size=(n_matrix, 3)) * cell
    d = m - centre
    m = m[np.sum(d * d, axis=1) > radius * radius]
    pos = np.concatenate([p, m], axis=0)
    species = np.concatenate([np.zeros(len(p), np.int32), np.ones(len(m), np.int32)])
    return pos, species


def amorphous(cell, density, rng):
    cell = np.asarray(cell, dtype=np.float64)
    n = int(round(density * float(np.prod(cell))))
    return rng.uniform(0.0, 1.0, size=(n, 3)) * cell, np.zeros(n, np.int32)


def atoms_for(w: Workload):
    """(positions [n,3] float64 in A, species index [n] int32) for a workload."""
    rng = np.random.default_rng(w.seed)
    if w.structure == "sc":
        reps = int(round(w.cell[0] / 4.0))
        return simple_cubic(4.0, reps, 0.05, rng)
    if w.structure == "np":
        return nanoparticle_in_amorphous(w.cell, rng=rng)
    if w.structure == "amorphous":
        return amorphous(w.cell, 0.05, rng)
    raise ValueError(w.structure)


def scan_positions(cell, nx: int, ny: int, sub: int = 1):
    """Probe positions x_i = i*Lx/nx, y_j = j*Ly/ny (row-major over (j, i)).

    `sub` > 1 keeps every sub-th position per axis (a subset of the same scan).
    Returns [P, 2] float64 (x, y) in A.
    """
    xs = np.arange(0, nx, sub, dtype=np.float64) * (cell[0] / nx)
    ys = np.arange(0, ny, sub, dtype=np.float64) * (cell[1] / ny)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel()], axis=1)


def random_positions(cell, n: int, rng: np.random.Generator):
    """Uniform random probe positions inside the cell's x-y face."""
    return rng.uniform(0.0, 1.0, size=(n, 2)) * np.asarray(cell[:2], dtype=np.float64)


def random_complex(shape, rng: np.random.Generator, dtype=np.complex64):
    """Standard complex normal samples (used as a synthetic S-matrix operand)."""
    a = rng.standard_normal(shape, dtype=np.float32)
    b = rng.standard_normal(shape, dtype=np.float32)
    return (a + 1j * b).astype(dtype)


def small_workload(n=64, cell=(10.0, 10.0, 6.0), dz=2.0, E0=80e3, alpha_max=0.02, f=2,
                   scan=(4, 4), seed=0, n_atoms=12):
    """A tiny random cell for fast parity tests (several tiles, ragged scans)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * np.asarray(cell)
    species = rng.integers(0, 2, size=n_atoms).astype(np.int32)
    w = Workload(f"small_{n}", tuple(cell), n, dz, E0, alpha_max, f, scan,
                 (SC1, AU), seed=seed, structure="given")
    return w, pos, species


# ---------------------------------------------------------------------------
# Serving stream: Poisson arrivals of mixed simulations.
# ---------------------------------------------------------------------------
def serving_stream(n_requests: int, rate: float, seed: int = 4, grids=(256, 512, 1024, 2048), fs=(2, 4, 8),
                   slices=(10, 50), scan=(16, 128)):
    """Request parameters (dicts) with Poisson arrival times (rate per second).

    Grid from `grids`, interpolation factor from `fs`, slice count uniform in
    `slices`, square scan side uniform in `scan`; the cell of request i is the
    nanoparticle-in-amorphous recipe seeded with 1000 + i.
    """
    rng = np.random.default_rng(seed)
    # unit-rate gaps drawn first in every case, so the requests themselves do
    # not depend on the rate (rate 0: everything arrives at t = 0)
    gaps = rng.exponential(1.0, size=n_requests)
    t = np.cumsum(gaps) / rate if rate > 0 else np.zeros(n_requests)
    out = []
    for i in range(n_requests):
        s = int(rng.integers(scan[0], scan[1] + 1))
        out.append(dict(rid=i, arrival=float(t[i]), n=int(rng.choice(grids)), f=int(rng.choice(fs)),
                        n_slices=int(rng.integers(slices[0], slices[1] + 1)), scan=(s, s), seed=1000 + i))
    return out


def serving_sample(cell, seed: int):
    """Callable giving the specimen of a serving request: the nanoparticle in
    an amorphous matrix of the 1024^2 workloads, scaled to `cell`, seeded with `seed`."""
    def make():
        pos, sp = nanoparticle_in_amorphous(cell, rng=np.random.default_rng(seed))
        return pos, sp, (AU, C)
    return make


def thermal_configs(pos, sigma: float, n_configs: int, seed: int):
    """Frozen-phonon configurations: `pos` displaced by independent Gaussian
    offsets of standard deviation `sigma` (A) per coordinate."""
    rng = np.random.default_rng(seed)
    pos = np.asarray(pos, dtype=np.float64)
    return [pos + rng.normal(0.0, sigma, size=pos.shape) for _ in range(n_configs)]
