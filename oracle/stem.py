"""FP64 oracle: multislice and PRISM STEM simulation, step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function states the
passage of the paper it follows.  Conventions and readings of points the paper
leaves open:

* Grid.  A square cell of side L sampled by n x n pixels, dx = L/n, pixel (j, i)
  at (x, y) = (i dx, j dx); arrays are indexed [y][x].  Fourier indices k are
  integers in FFT order, q = k/L.  Forward transform sign e^{-2 pi i k.r/n},
  inverse normalised by 1/n^2 (NumPy/SciPy convention).
* Constants (the paper only names lambda and sigma, Eqs. 1-2): relativistic
  wavelength lambda = hc / sqrt(e E0 (2 m0 c^2 + e E0)) and interaction
  constant sigma = 2 pi m e lambda / h^2 with m = m0 + e E0 / c^2, CODATA 2018.
* Band limit (not mentioned in the paper): the propagator keeps |q| < 1/(4 dx),
  i.e. kx^2 + ky^2 < n^2/16 in exact integers.  With the wave band-limited to
  half Nyquist, the product with an unfiltered transmission aliases only onto
  frequencies the mask removes, and the exit wave is exactly represented on
  every second pixel (n/2 x n/2 S-matrix storage).
* Step order: in every slice, transmit (Eq. 1) then propagate (Eq. 2),
  including after the last slice.
* Probe: hard aperture (Airy disk, Fig. 1c), lambda |q| <= alpha_max inclusive,
  coefficients normalised so that sum |c|^2 = 1; optional coherent aberrations
  exp(-i chi), chi = pi lam C1 q^2 + (pi/2) C3 lam^3 q^4 (defocus C1 > 0 is
  free propagation over C1 with the Eq. (2) propagator).
* PRISM window: side M = (n/2)/f pixels of the S-matrix grid (L/f in A),
  centred on the S-grid pixel nearest the probe (round half up), starting at
  centre - M/2, periodic.
* Detector: alpha = lambda |q|; 1-mrad bins [b da, (b+1) da); pixels with
  alpha >= alpha_AA = lambda n / (4 L) belong to no bin.
"""
from __future__ import annotations

import math
import multiprocessing

import numpy as np
import scipy.fft as sfft

PLANCK = 6.62607015e-34      # J s (exact, SI 2019)
LIGHT = 299792458.0          # m/s (exact)
CHARGE = 1.602176634e-19     # C (exact)
MASS0 = 9.1093837015e-31     # kg (CODATA 2018)

WORKERS = -1                 # scipy.fft worker threads (all cores)


# ---------------------------------------------------------------------------
# Transforms (library primitive; convention pinned against direct DFTs).
# ---------------------------------------------------------------------------
def fft2(a):
    return sfft.fft2(a, workers=WORKERS)


def ifft2(a):
    return sfft.ifft2(a, workers=WORKERS)


# ---------------------------------------------------------------------------
# Constants (Eqs. 1 and 2 name sigma and lambda).
# ---------------------------------------------------------------------------
def wavelength(E0: float) -> float:
    """Relativistic electron wavelength in A for beam energy E0 in eV."""
    eE = CHARGE * E0
    return PLANCK * LIGHT / math.sqrt(eE * (2.0 * MASS0 * LIGHT * LIGHT + eE)) * 1e10


def interaction_constant(E0: float) -> float:
    """Beam-sample interaction constant sigma of Eq. (1) in rad/(V*A)."""
    lam_m = wavelength(E0) * 1e-10
    m = MASS0 + CHARGE * E0 / (LIGHT * LIGHT)
    return 2.0 * math.pi * m * CHARGE * lam_m / (PLANCK * PLANCK) * 1e-10


# ---------------------------------------------------------------------------
# Grid helpers.
# ---------------------------------------------------------------------------
def fourier_indices(n: int) -> np.ndarray:
    """Integer Fourier indices in FFT order: 0, 1, ..., n/2-1, -n/2, ..., -1."""
    return np.concatenate([np.arange(0, (n + 1) // 2), np.arange(-(n // 2), 0)]).astype(np.int64)


def band_limit_mask(n: int) -> np.ndarray:
    """[n][n] bool: |q| < 1/(4 dx), evaluated exactly as 16 (kx^2+ky^2) < n^2."""
    k = fourier_indices(n)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    return 16 * (kx * kx + ky * ky) < n * n


# ---------------------------------------------------------------------------
# Projected potential ("Calculation of the Projected Potentials"; Fig. 1a-b).
# The paper integrates Kirkland scattering factors into per-species lookup
# tables; the workloads here prescribe analytic Gaussian species instead.
# ---------------------------------------------------------------------------
def n_slices_for(Lz: float, dz: float) -> int:
    return int(math.ceil(Lz / dz - 1e-12))


def slice_index(z, dz: float, n_slices: int):
    """Slab of thickness dz that holds z: clamp(floor(z/dz), 0, S-1)."""
    return np.clip(np.floor(np.asarray(z, dtype=np.float64) / dz), 0, n_slices - 1).astype(np.int64)


def projected_potential(pos, species_idx, species, cell, dz: float, n: int) -> np.ndarray:
    """V[s][y][x] in V*A: sum over atoms in slice s of their Gaussian terms.

    Each Gaussian of amplitude A (its 2D integral) and standard deviation w
    contributes A/(2 pi w^2) exp(-d^2/(2 w^2)) at minimum-image distance d,
    truncated at d < 6 max(w) of that species.  Plain loop over atoms; each atom
    evaluates every pixel row/column through the minimum image, so no pixel is
    counted twice.
    """
    L = float(cell[0])
    assert abs(cell[0] - cell[1]) < 1e-12, "square cells only"
    S = n_slices_for(cell[2], dz)
    dx = L / n
    V = np.zeros((S, n, n), dtype=np.float64)
    grid = np.arange(n, dtype=np.float64) * dx
    sl = slice_index(np.asarray(pos)[:, 2], dz, S)
    for a in range(len(pos)):
        sp = species[int(species_idx[a])]
        rc = 6.0 * max(sp.width)
        assert 2.0 * rc < L, "cutoff must be below half the cell"
        x = float(pos[a, 0]) % L
        y = float(pos[a, 1]) % L
        ddx = grid - x
        ddx -= L * np.round(ddx / L)
        ddy = grid - y
        ddy -= L * np.round(ddy / L)
        ix = np.nonzero(np.abs(ddx) < rc)[0]
        iy = np.nonzero(np.abs(ddy) < rc)[0]
        d2 = ddy[iy][:, None] ** 2 + ddx[ix][None, :] ** 2
        inside = d2 < rc * rc
        val = np.zeros_like(d2)
        for A, w in zip(sp.amp, sp.width):
            val += A / (2.0 * math.pi * w * w) * np.exp(-d2 / (2.0 * w * w))
        val[~inside] = 0.0
        V[sl[a]][np.ix_(iy, ix)] += val
    return V


# ---------------------------------------------------------------------------
# Eq. (1): transmission.  Eq. (2): Fresnel propagator.
# ---------------------------------------------------------------------------
def transmission(V, sigma: float):
    """t = exp(i sigma V) over real-space coordinates (Eq. 1)."""
    return np.exp(1j * sigma * np.asarray(V, dtype=np.float64))


def propagator(n: int, L: float, lam: float, dz: float):
    """[n][n]: band-limit mask times exp(-i pi lambda |q|^2 dz) (Eq. 2)."""
    k = fourier_indices(n).astype(np.float64)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    q2 = (kx / L) ** 2 + (ky / L) ** 2
    return band_limit_mask(n) * np.exp(-1j * math.pi * lam * q2 * dz)


# ---------------------------------------------------------------------------
# Detector (Fig. 1e): annular ring detectors -> a 3D output [probe][bin].
# The bin map is an explicit sequence of correctly rounded float64 operations
# so that any IEEE-754 implementation reproduces it bit for bit.
# ---------------------------------------------------------------------------
def alpha_aa(lam: float, n: int, L: float) -> float:
    """Anti-aliasing angle lambda * n / (4 L) (half of the real-space Nyquist)."""
    return lam * n / (4.0 * L)


def default_n_bins(lam: float, n: int, L: float, dalpha: float) -> int:
    return int(math.ceil(alpha_aa(lam, n, L) / dalpha))


def bin_map(lam: float, m: int, Lw: float, a_aa: float, dalpha: float, n_bins: int) -> np.ndarray:
    """[m][m] int32 annular-bin index of each Fourier pixel of an m x m grid of side Lw.

    alpha = lam * sqrt(kx^2 + ky^2) / Lw; bin = floor(alpha / dalpha) when
    alpha < a_aa and that bin is below n_bins, else -1.
    """
    k = fourier_indices(m)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    k2 = (kx * kx + ky * ky).astype(np.float64)
    alpha = lam * np.sqrt(k2) / Lw
    b = np.floor(alpha / dalpha).astype(np.int64)
    b[alpha >= a_aa] = -1
    b[b >= n_bins] = -1
    return b.astype(np.int32)


def detect(I, bmap, n_bins: int):
    """Sum intensity I over pixels of each bin."""
    sel = bmap >= 0
    return np.bincount(bmap[sel].ravel(), weights=I[sel].ravel(), minlength=n_bins)[:n_bins]


# ---------------------------------------------------------------------------
# Probe and beams (Fig. 1c, Fig. 1g).
# ---------------------------------------------------------------------------
def beam_set(n: int, L: float, lam: float, alpha_max: float, f: int) -> np.ndarray:
    """[B][2] int (kx, ky): every f-th Fourier index in both axes inside the
    maximum angle, lam * sqrt(kx^2+ky^2) / L <= alpha_max.  Sorted by (ky, kx).

    f = 1 gives the full aperture of the conventional probe.
    """
    out = []
    k = sorted(fourier_indices(n).tolist())
    for ky in k:
        for kx in k:
            if kx % f or ky % f:
                continue
            if lam * math.sqrt(float(kx * kx + ky * ky)) / L <= alpha_max:
                out.append((kx, ky))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def aberration_phase(beams, L: float, lam: float, C1: float = 0.0, C3: float = 0.0) -> np.ndarray:
    """chi(q) = pi lam C1 |q|^2 + (pi/2) C3 lam^3 |q|^4 for each beam (rad).

    Coherent wave aberrations carried by the probe coefficients ("PRISM Probe
    Simulations": defocus C1 and spherical aberration C3, both in A).  With
    the propagator exp(-i pi lam |q|^2 dz) of Eq. (2), exp(-i chi) at C3 = 0
    is free propagation over C1.
    """
    q2 = (beams[:, 0].astype(np.float64) / L) ** 2 + (beams[:, 1].astype(np.float64) / L) ** 2
    return math.pi * lam * C1 * q2 + 0.5 * math.pi * C3 * lam ** 3 * q2 * q2


def probe_coefficients(beams, L: float, xy, lam: float = 0.0, C1: float = 0.0, C3: float = 0.0) -> np.ndarray:
    """c[p][b] = |B|^(-1/2) exp(-2 pi i (kx x_p + ky y_p) / L) exp(-i chi(q_b)).

    Fourier phase shifts that translate each plane wave so the summed probe is
    centred at (x_p, y_p), times the aberration phase ("PRISM Probe
    Simulations").
    """
    xy = np.atleast_2d(np.asarray(xy, dtype=np.float64))
    kx = beams[:, 0].astype(np.float64)
    ky = beams[:, 1].astype(np.float64)
    arg = (xy[:, 0:1] * kx[None, :] + xy[:, 1:2] * ky[None, :]) / L
    c = np.exp(-2j * math.pi * arg) / math.sqrt(len(beams))
    if C1 or C3:
        c = c * np.exp(-1j * aberration_phase(beams, L, lam, C1, C3))[None, :]
    return c


# ---------------------------------------------------------------------------
# Multislice (Fig. 1c-e; "Multislice Probe Simulations").
# ---------------------------------------------------------------------------
def multislice_exit_spectrum(V, L: float, dz: float, lam: float, sigma: float,
                             alpha_max: float, xy, C1: float = 0.0, C3: float = 0.0):
    """Psi(k) after the last slice for one probe at xy (Fourier space, FFT order)."""
    S, n, _ = V.shape
    t = transmission(V, sigma)
    P = propagator(n, L, lam, dz)
    ap = beam_set(n, L, lam, alpha_max, 1)
    c = probe_coefficients(ap, L, xy, lam, C1, C3)[0]
    Psi0 = np.zeros((n, n), dtype=np.complex128)
    Psi0[ap[:, 1] % n, ap[:, 0] % n] = c
    psi = n * n * ifft2(Psi0)
    Psi = None
    for s in range(S):
        psi = psi * t[s]
        Psi = fft2(psi) * P
        if s < S - 1:
            psi = ifft2(Psi)
    return Psi


def multislice_outputs(V, L: float, dz: float, lam: float, sigma: float, alpha_max: float,
                       probe_xy, dalpha: float = 1e-3, n_bins: int | None = None, C1: float = 0.0,
                       C3: float = 0.0, processes: int = 1, detector_map=None):
    """D[p][bin] = sum over bin of |Psi_exit|^2 / n^4 for each probe (3D output).

    detector_map: optional [n][n] int detector index per Fourier pixel (FFT
    order, -1 = none) with n_bins detectors, in place of annular bins (virtual
    detectors, Fig. 1e).  Probes are independent; `processes` > 1 runs them in
    forked worker processes (same arithmetic per probe)."""
    S, n, _ = V.shape
    if detector_map is not None:
        bmap = np.asarray(detector_map)
    else:
        if n_bins is None:
            n_bins = default_n_bins(lam, n, L, dalpha)
        bmap = bin_map(lam, n, L, alpha_aa(lam, n, L), dalpha, n_bins)
    probe_xy = np.atleast_2d(np.asarray(probe_xy, dtype=np.float64))

    def one(p):
        Psi = multislice_exit_spectrum(V, L, dz, lam, sigma, alpha_max, probe_xy[p], C1, C3)
        return detect(np.abs(Psi) ** 2 / float(n) ** 4, bmap, n_bins)

    rows = _fork_map(one, range(len(probe_xy)), processes)
    return np.array(rows, dtype=np.float64).reshape(len(probe_xy), n_bins)


# ---------------------------------------------------------------------------
# PRISM: compact S-matrix ("PRISM Probe Simulations"; Fig. 1h).
# ---------------------------------------------------------------------------
def smatrix_layer(t, P, kx: int, ky: int):
    """One S-matrix layer: plane wave exp(2 pi i (kx x + ky y)/n) multisliced
    through every slice and stored in real space on every second pixel."""
    S, n, _ = t.shape
    j = np.arange(n, dtype=np.float64)
    psi = np.exp(2j * math.pi * (ky * j[:, None] + kx * j[None, :]) / n)
    Psi = None
    for s in range(S):
        psi = psi * t[s]
        Psi = fft2(psi) * P
        psi = ifft2(Psi)
    return psi[::2, ::2]


def build_smatrix(V, L: float, dz: float, lam: float, sigma: float, beams):
    """S[b][my][mx] complex128 for every beam in `beams`."""
    S_, n, _ = V.shape
    t = transmission(V, sigma)
    P = propagator(n, L, lam, dz)
    out = np.empty((len(beams), n // 2, n // 2), dtype=np.complex128)
    for b, (kx, ky) in enumerate(beams):
        out[b] = smatrix_layer(t, P, int(kx), int(ky))
    return out


# ---------------------------------------------------------------------------
# PRISM probe synthesis (Fig. 1i-k; "PRISM Probe Simulations").
# ---------------------------------------------------------------------------
def window_centre(x: float, L: float, n: int) -> int:
    """Nearest S-grid pixel to coordinate x: floor(x / (2 (L/n)) + 0.5) mod n/2."""
    return int(math.floor(x / (2.0 * (L / n)) + 0.5)) % (n // 2)


def probe_window(Smat, c, cx: int, cy: int, M: int):
    """psi_w[v][u] = sum_b c_b S_b[(cy - M/2 + v) mod Ns][(cx - M/2 + u) mod Ns]."""
    Ns = Smat.shape[1]
    rows = (cy - M // 2 + np.arange(M)) % Ns
    cols = (cx - M // 2 + np.arange(M)) % Ns
    crop = Smat[:, rows][:, :, cols]
    return np.tensordot(c, crop, axes=(0, 0))


def window_detector_map(lam: float, n: int, L: float, f: int, dalpha: float, n_bins, detector_map):
    """(map, n_bins) over the M x M window grid: the caller's map, or annular
    bins of width dalpha up to alpha_AA."""
    M = (n // 2) // f
    if detector_map is not None:
        return np.asarray(detector_map), n_bins
    if n_bins is None:
        n_bins = default_n_bins(lam, n, L, dalpha)
    return bin_map(lam, M, L / f, alpha_aa(lam, n, L), dalpha, n_bins), n_bins


def prism_outputs(Smat, beams, L: float, n: int, lam: float, f: int, probe_xy,
                  dalpha: float = 1e-3, n_bins: int | None = None, C1: float = 0.0, C3: float = 0.0,
                  detector_map=None):
    """D[p][bin] for each probe from a compact S-matrix (3D output);
    detector_map: optional [M][M] detector index per window Fourier pixel (FFT
    order, -1 = none) with n_bins detectors, in place of annular bins."""
    Ns = n // 2
    M = Ns // f
    bmap, n_bins = window_detector_map(lam, n, L, f, dalpha, n_bins, detector_map)
    probe_xy = np.atleast_2d(np.asarray(probe_xy, dtype=np.float64))
    C = probe_coefficients(beams, L, probe_xy, lam, C1, C3)
    D = np.zeros((len(probe_xy), n_bins))
    for p in range(len(probe_xy)):
        cx = window_centre(probe_xy[p, 0], L, n)
        cy = window_centre(probe_xy[p, 1], L, n)
        w = probe_window(Smat, C[p], cx, cy, M)
        I = np.abs(fft2(w)) ** 2 / float(M) ** 4
        D[p] = detect(I, bmap, n_bins)
    return D


def prism_diffraction(Smat, beams, L: float, n: int, lam: float, f: int, probe_xy,
                      C1: float = 0.0, C3: float = 0.0):
    """I[p][ky][kx] = |FFT_M(psi_p)|^2 / M^4 on the window's Fourier grid (FFT
    order): the entire probe diffraction pattern of each probe, the 4D output
    of Fig. 1e/k."""
    Ns = n // 2
    M = Ns // f
    probe_xy = np.atleast_2d(np.asarray(probe_xy, dtype=np.float64))
    C = probe_coefficients(beams, L, probe_xy, lam, C1, C3)
    out = np.zeros((len(probe_xy), M, M))
    for p in range(len(probe_xy)):
        cx = window_centre(probe_xy[p, 0], L, n)
        cy = window_centre(probe_xy[p, 1], L, n)
        w = probe_window(Smat, C[p], cx, cy, M)
        out[p] = np.abs(fft2(w)) ** 2 / float(M) ** 4
    return out


def frozen_phonon_prism(configs, species_idx, species, cell, dz: float, n: int, E0: float, alpha_max: float,
                        f: int, probe_xy, C1: float = 0.0, C3: float = 0.0):
    """Mean over thermal configurations of the PRISM 3D output, each
    configuration simulated in full (frozen-phonon averaging)."""
    lam, sig = wavelength(E0), interaction_constant(E0)
    L = float(cell[0])
    beams = beam_set(n, L, lam, alpha_max, f)
    acc = None
    for pos in configs:
        V = projected_potential(pos, species_idx, species, cell, dz, n)
        D = prism_outputs(build_smatrix(V, L, dz, lam, sig, beams), beams, L, n, lam, f, probe_xy, C1=C1, C3=C3)
        acc = D if acc is None else acc + D
    return acc / len(configs)


# ---------------------------------------------------------------------------
# PRISM without storing the S-matrix.  The paper's streaming memory model
# ("Streaming Data for Very Large Simulations") keeps only the data of the
# current step on the device; applied here, each beam's layer is built, its
# contribution c_b(p) S_b is added into every probe's window, and the layer is
# dropped.  The window sum is linear in the beams, so the result equals
# build_smatrix followed by prism_outputs (up to the order of the FP64 sums)
# while holding P windows instead of |B| layers.
# ---------------------------------------------------------------------------
def smatrix_windows(t, P, beams, coeffs, centres, M: int):
    """sum over the given beams of coeffs[p][b] times beam b's layer cropped to
    probe p's window: [len(centres)][M][M] complex128."""
    acc = np.zeros((len(centres), M, M), dtype=np.complex128)
    for b, (kx, ky) in enumerate(beams):
        layer = smatrix_layer(t, P, int(kx), int(ky))[None]
        for p, (cx, cy) in enumerate(centres):
            acc[p] += probe_window(layer, coeffs[p, b:b + 1], cx, cy, M)
    return acc


def prism_outputs_streamed(V, L: float, dz: float, lam: float, sigma: float, beams, n: int, f: int, probe_xy,
                           dalpha: float = 1e-3, n_bins: int | None = None, C1: float = 0.0, C3: float = 0.0,
                           processes: int = 1, groups: int | None = None, detector_map=None):
    """D[p][bin] of prism_outputs(build_smatrix(V, ...), ...) with the beams
    streamed through window accumulators; `groups` beam groups are summed in
    `processes` forked worker processes."""
    Ns = n // 2
    M = Ns // f
    bmap, n_bins = window_detector_map(lam, n, L, f, dalpha, n_bins, detector_map)
    probe_xy = np.atleast_2d(np.asarray(probe_xy, dtype=np.float64))
    t = transmission(V, sigma)
    P = propagator(n, L, lam, dz)
    C = probe_coefficients(beams, L, probe_xy, lam, C1, C3)
    centres = [(window_centre(x, L, n), window_centre(y, L, n)) for x, y in probe_xy]
    parts = np.array_split(np.arange(len(beams)), max(1, groups or processes))

    def one(idx):
        return smatrix_windows(t, P, beams[idx], C[:, idx], centres, M)

    w = np.zeros((len(probe_xy), M, M), dtype=np.complex128)
    for part in _fork_map(one, parts, processes):
        w += part
    D = np.zeros((len(probe_xy), n_bins))
    for p in range(len(probe_xy)):
        D[p] = detect(np.abs(fft2(w[p])) ** 2 / float(M) ** 4, bmap, n_bins)
    return D


# ---------------------------------------------------------------------------
# Worker processes for the independent items above (probes of multislice,
# beam groups of the streamed PRISM).  Forked children inherit the inputs;
# each runs its transforms on one thread.
# ---------------------------------------------------------------------------
_FORK_TASK = None


def _fork_call(i):
    global WORKERS
    WORKERS = 1
    return _FORK_TASK(i)


def _fork_map(fn, items, processes: int):
    global _FORK_TASK
    items = list(items)
    if processes <= 1 or len(items) <= 1:
        return [fn(x) for x in items]
    _FORK_TASK = lambda i: fn(items[i])  # noqa: E731
    try:
        with multiprocessing.get_context("fork").Pool(min(processes, len(items))) as pool:
            return pool.map(_fork_call, range(len(items)), chunksize=1)
    finally:
        _FORK_TASK = None


# ---------------------------------------------------------------------------
# Error metrics.
# ---------------------------------------------------------------------------
def rel_err(D, Dref) -> float:
    """Frobenius-norm relative error over probes x bins."""
    D = np.asarray(D, dtype=np.float64)
    Dref = np.asarray(Dref, dtype=np.float64)
    return float(np.linalg.norm(D - Dref) / np.linalg.norm(Dref))


def adf_signal(D, dalpha: float, lo: float) -> np.ndarray:
    """Annular dark-field image value per probe: bins with b*dalpha >= lo."""
    D = np.asarray(D, dtype=np.float64)
    b = np.arange(D.shape[1])
    return D[:, b * dalpha >= lo - 1e-15].sum(axis=1)
