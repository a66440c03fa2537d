"""Pins of the FP64 oracle against facts fixed by mathematics and physics.

Each test checks the oracle against something other than itself: direct DFT
sums, textbook constants, closed forms, sum rules, exact symmetries, and the
exactness of PRISM at f = 1 (the plane-wave basis is then complete, "Description
of Algorithms").  None of these compares the oracle with the GPU path.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W


# ---------------------------------------------------------------------------
# T1: transform convention against direct O(N^2) DFT sums.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(4, 4), (8, 8), (16, 16), (6, 10)])
def test_fft_convention_matches_direct_dft(shape):
    rng = np.random.default_rng(1)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ny, nx = shape
    y = np.arange(ny)[:, None]
    x = np.arange(nx)[None, :]
    direct = np.zeros(shape, dtype=np.complex128)
    inv = np.zeros(shape, dtype=np.complex128)
    for ky in range(ny):
        for kx in range(nx):
            ph = np.exp(-2j * math.pi * (ky * y / ny + kx * x / nx))
            direct[ky, kx] = np.sum(a * ph)
            inv[ky, kx] = np.sum(a * np.conj(ph)) / (nx * ny)
    assert np.max(np.abs(O.stem.fft2(a) - direct)) < 1e-12
    assert np.max(np.abs(O.stem.ifft2(a) - inv)) < 1e-13


def test_fourier_indices_order():
    assert O.fourier_indices(8).tolist() == [0, 1, 2, 3, -4, -3, -2, -1]


# ---------------------------------------------------------------------------
# Constants: textbook tabulations of the relativistic wavelength and the
# interaction constant (Kirkland, Advanced Computing in Electron Microscopy,
# table of electron wavelength and sigma vs. accelerating voltage), and the
# independent closed form sigma = 2 pi/(lambda E0) (m0 c^2 + e E0)/(2 m0 c^2 + e E0).
# ---------------------------------------------------------------------------
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_table(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [tuple(float(x) for x in line.split()) for line in fh if line.strip() and not line.startswith("#")]


@pytest.mark.parametrize("E0,lam,sig", _golden_table("electron_wavelength_sigma.txt"))
def test_wavelength_and_sigma_textbook(E0, lam, sig):
    assert abs(O.wavelength(E0) - lam) / lam < 2e-4
    assert abs(O.interaction_constant(E0) - sig) / sig < 2e-4


@pytest.mark.parametrize("E0", [1e3, 80e3, 200e3, 1e6])
def test_sigma_kirkland_closed_form(E0):
    mc2 = O.MASS0 * O.LIGHT ** 2
    eE = O.CHARGE * E0
    lam = O.wavelength(E0)
    expected = 2 * math.pi / (lam * E0) * (mc2 + eE) / (2 * mc2 + eE)
    assert abs(O.interaction_constant(E0) - expected) / expected < 1e-12


def test_nonrelativistic_limit():
    # E0 << m0 c^2: lambda -> h / sqrt(2 m0 e E0) (1 - eps/4), sigma lambda E0 / pi -> 1 + eps/2,
    # eps = e E0 / (m0 c^2), to first order.
    E0 = 10.0
    eps = O.CHARGE * E0 / (O.MASS0 * O.LIGHT ** 2)
    lam_nr = O.PLANCK / math.sqrt(2 * O.MASS0 * O.CHARGE * E0) * 1e10
    assert abs(O.wavelength(E0) / lam_nr - (1 - eps / 4)) < 1e-10
    assert abs(O.interaction_constant(E0) * O.wavelength(E0) * E0 / math.pi - (1 + eps / 2)) < 1e-10


# ---------------------------------------------------------------------------
# Projected potential: sum rule, periodic wrap, slicing.
# ---------------------------------------------------------------------------
def test_potential_sum_rule():
    w, pos, sp = W.small_workload(n=64, n_atoms=20, seed=3)
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    dx = w.cell[0] / w.n
    total = sum(sum(w.species[s].amp) for s in sp)
    assert abs(V.sum() * dx * dx / total - 1) < 1e-7


def test_potential_slice_assignment_and_sum_per_slice():
    sp = (W.SC1,)
    cell = (12.0, 12.0, 6.0)
    pos = np.array([[1.0, 2.0, 0.5], [5.0, 5.0, 2.5], [7.0, 9.0, 5.9], [3.0, 3.0, -0.2], [4.0, 4.0, 6.3]])
    V = O.projected_potential(pos, np.zeros(5, np.int32), sp, cell, 2.0, 96)
    dx = 12.0 / 96
    per = V.sum(axis=(1, 2)) * dx * dx / 25.0
    # slice 0 gets z=0.5 and the clamped z=-0.2; slice 1 z=2.5; slice 2 z=5.9 and clamped z=6.3
    assert np.allclose(per, [2, 1, 2], atol=1e-7)


def test_potential_periodic_wrap_is_a_roll():
    sp = (W.SC1,)
    cell = (12.0, 12.0, 2.0)
    n = 96
    dx = cell[0] / n
    a = O.projected_potential(np.array([[40 * dx, 50 * dx, 1.0]]), np.zeros(1, np.int32), sp, cell, 2.0, n)
    # same atom moved across the periodic boundary by (-45, +50) pixels
    b = O.projected_potential(np.array([[(40 - 45) * dx, (50 + 50) * dx, 1.0]]), np.zeros(1, np.int32),
                              sp, cell, 2.0, n)
    assert np.max(np.abs(np.roll(a, (50, -45), axis=(1, 2)) - b)) < 1e-9 * a.max()


def test_potential_radial_profile_peak():
    # On-pixel atom: the peak pixel holds the sum of Gaussian peak heights A/(2 pi w^2).
    sp = (W.SC1,)
    n, L = 128, 16.0
    dx = L / n
    V = O.projected_potential(np.array([[64 * dx, 32 * dx, 0.3]]), np.zeros(1, np.int32), sp, (L, L, 2.0), 2.0, n)
    peak = 20 / (2 * math.pi * 0.09) + 5 / (2 * math.pi * 0.64)
    assert abs(V[0, 32, 64] - peak) < 1e-12 * peak
    assert np.unravel_index(np.argmax(V[0]), V[0].shape) == (32, 64)


# ---------------------------------------------------------------------------
# T2: norm identities of Eq. (1) and Eq. (2).
# ---------------------------------------------------------------------------
def test_transmission_is_unitary():
    rng = np.random.default_rng(0)
    V = rng.uniform(0, 50, size=(32, 32))
    psi = rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32))
    t = O.transmission(V, 1e-3)
    assert abs(np.linalg.norm(psi * t) / np.linalg.norm(psi) - 1) < 1e-14


def test_propagation_conserves_in_band_norm_and_removes_out_of_band():
    n, L = 64, 10.0
    rng = np.random.default_rng(2)
    psi = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Psi = O.stem.fft2(psi)
    mask = O.band_limit_mask(n)
    P = O.propagator(n, L, O.wavelength(80e3), 2.0)
    out = O.stem.ifft2(Psi * P)
    # Parseval: the kept energy is exactly the in-band energy of the input
    in_band = np.sum(np.abs(Psi[mask]) ** 2) / (n * n)
    assert abs(np.sum(np.abs(out) ** 2) / in_band - 1) < 1e-12
    # the mask is the disc 16 (kx^2+ky^2) < n^2 : count lattice points directly
    cnt = sum(1 for kx in range(-n // 2, n // 2) for ky in range(-n // 2, n // 2) if 16 * (kx * kx + ky * ky) < n * n)
    assert mask.sum() == cnt


# ---------------------------------------------------------------------------
# T3: free-space Fresnel spreading of a Gaussian in closed form.
# psi_0 = exp(-r^2/(2 s^2))  ->  psi_z = exp(-r^2/(2 s^2 (1+i b))) / (1+i b),
# b = lambda z / (2 pi s^2), for the propagator exp(-i pi lambda q^2 z).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("E0,z", [(80e3, 100.0), (200e3, 40.0)])
def test_free_space_gaussian_closed_form(E0, z):
    n, L, s = 256, 20.0, 1.0
    lam = O.wavelength(E0)
    dx = L / n
    c = np.arange(n) * dx - L / 2
    yy, xx = np.meshgrid(c, c, indexing="ij")
    r2 = xx ** 2 + yy ** 2
    psi0 = np.exp(-r2 / (2 * s * s))
    nsteps = int(round(z / 2.0))
    P = O.propagator(n, L, lam, 2.0)
    Psi = O.stem.fft2(psi0)
    for _ in range(nsteps):
        Psi = Psi * P
    psiz = O.stem.ifft2(Psi)
    b = lam * z / (2 * math.pi * s * s)
    expected = np.exp(-r2 / (2 * s * s * (1 + 1j * b))) / (1 + 1j * b)
    assert np.max(np.abs(psiz - expected)) < 1e-10
    # width grows as s sqrt(1 + b^2)
    I = np.abs(psiz) ** 2
    var = np.sum(I * xx ** 2) / np.sum(I)
    assert abs(math.sqrt(2 * var) / (s * math.sqrt(1 + b * b)) - 1) < 1e-9


# T4: propagator composition.
def test_propagator_composition():
    n, L = 64, 12.0
    lam = O.wavelength(200e3)
    P1 = O.propagator(n, L, lam, 2.0)
    P5 = O.propagator(n, L, lam, 10.0)
    assert np.max(np.abs(P1 ** 5 - P5)) < 1e-12


# ---------------------------------------------------------------------------
# Beams and bins.
# ---------------------------------------------------------------------------
def test_beam_counts_gauss_circle():
    # |B_f| is the number of lattice points (f m, f n) in the disc of radius alpha L / lambda.
    n, L, E0, a = 256, 20.0, 80e3, 0.02
    lam = O.wavelength(E0)
    R = a * L / lam
    for f in (1, 2, 3, 4):
        cnt = 0
        m = int(R // f) + 1
        for i in range(-m, m + 1):
            for j in range(-m, m + 1):
                if (f * i) ** 2 + (f * j) ** 2 <= R * R:
                    cnt += 1
        assert len(O.beam_set(n, L, lam, a, f)) == cnt
    assert len(O.beam_set(256, 20.0, lam, 0.02, 1)) == 293
    assert len(O.beam_set(256, 20.0, lam, 0.02, 2)) == 69


def test_beam_set_symmetry():
    lam = O.wavelength(200e3)
    B = O.beam_set(1024, 100.0, lam, 0.02, 4)
    s = set(map(tuple, B.tolist()))
    assert len(B) == 1245
    assert all((-kx, -ky) in s and (ky, -kx) in s for kx, ky in s)
    assert (0, 0) in s and all(kx % 4 == 0 and ky % 4 == 0 for kx, ky in s)


def test_bin_map_rules():
    lam, Lw, m = 0.025, 25.0, 64          # alpha = 1e-3 * |k| exactly up to rounding
    a_aa = O.alpha_aa(lam, 2 * m, 2 * Lw)
    n_bins = O.default_n_bins(lam, 2 * m, 2 * Lw, 1e-3)
    bm = O.bin_map(lam, m, Lw, a_aa, 1e-3, n_bins)
    k = O.fourier_indices(m)
    assert bm[0, 0] == 0
    assert bm[0, 1] == 1 and bm[1, 1] == 1 and bm[0, 2] == 2   # |k| = 1.414 -> bin 1
    assert bm[k.tolist().index(7), k.tolist().index(7)] == 9     # |k| = 9.899
    # corners beyond alpha_AA are excluded; all bins are in range
    assert bm[m // 2, m // 2] == -1
    assert bm.max() == n_bins - 1 and bm.min() == -1
    # cumulative pixel counts: bins 0..b hold the lattice points with |k| < b + 1
    # (points with |k| = b + 1 exactly sit on an edge and may fall either side)
    counts = np.cumsum(np.bincount(bm[bm >= 0].ravel()))
    kk = np.array([kx * kx + ky * ky for kx in k for ky in k])
    for b in range(n_bins):
        lo = np.sum(kk < (b + 1) ** 2)
        hi = np.sum(kk <= (b + 1) ** 2)
        assert lo <= counts[b] <= hi


# ---------------------------------------------------------------------------
# T5/T6: vacuum closed form, and a constant potential equals vacuum.
# D[p][bin] = #{beams of B_f falling in bin} / |B_f| for every probe.
# ---------------------------------------------------------------------------
def _vacuum_expected(lam, n, L, a, f, dalpha, n_bins):
    B = O.beam_set(n, L, lam, a, f)
    ang = np.array([lam * math.hypot(kx, ky) / L for kx, ky in B])
    nz = ang > 0
    assert np.min(np.abs(ang[nz] / dalpha - np.round(ang[nz] / dalpha))) > 1e-9   # no beam on an edge
    bins = np.floor(ang / dalpha).astype(int)
    return np.bincount(bins, minlength=n_bins)[:n_bins] / len(B)


def test_multislice_vacuum_closed_form():
    n, L, E0, a = 64, 10.0, 80e3, 0.02
    lam, sig = O.wavelength(E0), O.interaction_constant(E0)
    nb = O.default_n_bins(lam, n, L, 1e-3)
    V = np.zeros((3, n, n))
    xy = np.array([[0.0, 0.0], [3.3, 7.1], [9.9, 0.2]])
    D = O.multislice_outputs(V, L, 2.0, lam, sig, a, xy)
    exp = _vacuum_expected(lam, n, L, a, 1, 1e-3, nb)
    assert np.max(np.abs(D - exp[None, :])) < 1e-13
    Dc = O.multislice_outputs(V + 17.0, L, 2.0, lam, sig, a, xy)
    assert np.max(np.abs(Dc - D)) < 1e-13


@pytest.mark.parametrize("f", [1, 2, 4])
def test_prism_vacuum_closed_form(f):
    n, L, E0, a = 64, 10.0, 80e3, 0.02
    lam, sig = O.wavelength(E0), O.interaction_constant(E0)
    nb = O.default_n_bins(lam, n, L, 1e-3)
    V = np.zeros((2, n, n)) + 3.0
    beams = O.beam_set(n, L, lam, a, f)
    S = O.build_smatrix(V, L, 2.0, lam, sig, beams)
    xy = np.array([[0.0, 0.0], [3.3, 7.1], [9.9, 0.2], [5.0, 5.0]])
    D = O.prism_outputs(S, beams, L, n, lam, f, xy)
    exp = _vacuum_expected(lam, n, L, a, f, 1e-3, nb)
    assert np.max(np.abs(D - exp[None, :])) < 1e-13


# ---------------------------------------------------------------------------
# T7: PRISM at f = 1 reproduces multislice (complete plane-wave basis).
# ---------------------------------------------------------------------------
def test_prism_f1_equals_multislice():
    w, pos, sp = W.small_workload(n=64, n_atoms=16, seed=5)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    L = w.cell[0]
    xy = np.array([[0.0, 0.0], [2.5, 7.5], [6.1, 3.9], [9.7, 9.7]])
    Dm = O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy)
    beams = O.beam_set(w.n, L, lam, w.alpha_max, 1)
    S = O.build_smatrix(V, L, w.dz, lam, sig, beams)
    Dp = O.prism_outputs(S, beams, L, w.n, lam, 1, xy)
    assert O.rel_err(Dp, Dm) < 1e-10
    # and the specimen actually scatters (the test is not vacuous)
    assert np.sum(Dm[:, 40:]) > 1e-4


def test_prism_error_grows_with_f():
    w, pos, sp = W.small_workload(n=128, cell=(16.0, 16.0, 6.0), n_atoms=40, seed=6)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    L = w.cell[0]
    xy = W.scan_positions(w.cell, 4, 4)
    Dm = O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy)
    errs = []
    for f in (1, 2, 4):
        beams = O.beam_set(w.n, L, lam, w.alpha_max, f)
        S = O.build_smatrix(V, L, w.dz, lam, sig, beams)
        errs.append(O.rel_err(O.prism_outputs(S, beams, L, w.n, lam, f, xy), Dm))
    assert errs[0] < 1e-10 and errs[0] < errs[1] < errs[2]


# ---------------------------------------------------------------------------
# T9: translation covariance by whole S-grid pixels.
# ---------------------------------------------------------------------------
def test_translation_covariance():
    w, pos, sp = W.small_workload(n=64, n_atoms=10, seed=7)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    L = w.cell[0]
    d = np.array([2 * 3 * L / w.n, 2 * 5 * L / w.n])
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    pos2 = pos.copy()
    pos2[:, :2] += d
    V2 = O.projected_potential(pos2, sp, w.species, w.cell, w.dz, w.n)
    xy = np.array([[1.0, 2.0], [4.0, 8.0]])
    beams = O.beam_set(w.n, L, lam, w.alpha_max, 2)
    D1 = O.prism_outputs(O.build_smatrix(V, L, w.dz, lam, sig, beams), beams, L, w.n, lam, 2, xy)
    D2 = O.prism_outputs(O.build_smatrix(V2, L, w.dz, lam, sig, beams), beams, L, w.n, lam, 2, xy + d)
    assert O.rel_err(D2, D1) < 1e-10
    M1 = O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy)
    M2 = O.multislice_outputs(V2, L, w.dz, lam, sig, w.alpha_max, xy + d)
    assert O.rel_err(M2, M1) < 1e-10


def test_smatrix_storage_is_exact_decimation():
    # The exit wave is band-limited to |k| < n/4, so the n/2 grid samples it
    # without aliasing: the half-grid spectrum equals the central crop / 4.
    n, L = 64, 10.0
    lam, sig = O.wavelength(80e3), O.interaction_constant(80e3)
    rng = np.random.default_rng(4)
    V = rng.uniform(0, 30, size=(2, n, n))
    t = O.transmission(V, sig)
    P = O.propagator(n, L, lam, 2.0)
    layer = O.smatrix_layer(t, P, 2, -3)
    psi = np.exp(2j * math.pi * (-3 * np.arange(n)[:, None] + 2 * np.arange(n)[None, :]) / n)
    for s in range(2):
        psi = O.stem.ifft2(O.stem.fft2(psi * t[s]) * P)
    full = O.stem.fft2(psi)
    half = O.stem.fft2(layer)
    k = O.fourier_indices(n // 2) % n
    assert np.max(np.abs(half - full[np.ix_(k, k)] / 4)) < 1e-10 * np.abs(full).max()


# ---------------------------------------------------------------------------
# Sign of Eq. (1) relative to Eq. (2): a positive (attractive) quadratic
# potential V = -a r^2 / 2 + const acts as a converging lens.  For a Gaussian
# psi = exp(-Q r^2 / 2) the transmission gives Q -> Q + i sigma a and free
# propagation over z gives psi_z = (Q'/Q) exp(-Q' r^2 / 2) with
# 1/Q' = 1/Q + i lambda z / (2 pi).
# ---------------------------------------------------------------------------
def test_quadratic_lens_closed_form_fixes_sign_convention():
    n, L, s, E0, z = 256, 40.0, 2.0, 200e3, 100.0
    lam, sig = O.wavelength(E0), O.interaction_constant(E0)
    a = 2 * math.pi / (lam * sig * 500.0)           # focal length 500 A
    dx = L / n
    c = np.arange(n) * dx - L / 2
    yy, xx = np.meshgrid(c, c, indexing="ij")
    r2 = xx ** 2 + yy ** 2
    V = 40.0 - a * r2 / 2
    psi = np.exp(-r2 / (2 * s * s)) * O.transmission(V, sig)
    Psi = O.stem.fft2(psi) * O.propagator(n, L, lam, z)
    psiz = O.stem.ifft2(Psi)
    Q = 1 / (s * s) + 1j * sig * a
    Qp = 1 / (1 / Q + 1j * lam * z / (2 * math.pi))
    expected = np.exp(1j * sig * 40.0) * (Qp / Q) * np.exp(-Qp * r2 / 2)
    assert np.max(np.abs(psiz - expected)) < 1e-8
    # converging: the beam is narrower after z than at the entrance
    I = np.abs(psiz) ** 2
    assert np.sum(I * r2) / np.sum(I) < s * s


def test_probe_window_is_periodic_crop_at_centre_minus_half():
    # Independent formulation of the window: roll the S grid so that pixel
    # (cy - M/2, cx - M/2) comes to the origin and keep the leading M x M block.
    rng = np.random.default_rng(8)
    Ns, M, B = 16, 8, 3
    S = rng.standard_normal((B, Ns, Ns)) + 1j * rng.standard_normal((B, Ns, Ns))
    c = rng.standard_normal(B) + 1j * rng.standard_normal(B)
    for cx, cy in [(0, 0), (3, 14), (15, 1), (8, 8)]:
        rolled = np.roll(S, (-(cy - M // 2), -(cx - M // 2)), axis=(1, 2))[:, :M, :M]
        ref = np.einsum("b,byx->yx", c, rolled)
        assert np.max(np.abs(O.probe_window(S, c, cx, cy, M) - ref)) < 1e-13
    # centre: nearest S-grid pixel, halves round up
    L, n = 10.0, 64                      # S-grid pitch 2 L / n = 0.3125
    assert O.window_centre(0.0, L, n) == 0
    assert O.window_centre(0.15, L, n) == 0 and O.window_centre(0.16, L, n) == 1
    assert O.window_centre(0.3125 * 1.5, L, n) == 2
    assert O.window_centre(9.9, L, n) == 0 and O.window_centre(-0.2, L, n) == 31


# ---------------------------------------------------------------------------
# Aberrations carried by the probe coefficients.  Defocus C1 with the Eq. (2)
# propagator is free propagation over C1: a probe defocused by m dz equals the
# in-focus probe sent through m vacuum slices first.
# ---------------------------------------------------------------------------
def test_defocus_equals_vacuum_slices_in_front():
    w, pos, sp = W.small_workload(n=64, n_atoms=14, seed=9)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    L = w.cell[0]
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    m = 3
    Vpad = np.concatenate([np.zeros((m,) + V.shape[1:]), V], axis=0)
    xy = (3.7, 6.2)
    a = O.multislice_exit_spectrum(V, L, w.dz, lam, sig, w.alpha_max, xy, C1=m * w.dz)
    b = O.multislice_exit_spectrum(Vpad, L, w.dz, lam, sig, w.alpha_max, xy)
    assert np.max(np.abs(a - b)) < 1e-10 * np.max(np.abs(b))
    # and defocus changes the result (the test is not vacuous)
    c = O.multislice_exit_spectrum(V, L, w.dz, lam, sig, w.alpha_max, xy)
    assert np.max(np.abs(np.abs(a) - np.abs(c))) > 1e-3 * np.max(np.abs(c))


def test_aberrated_prism_f1_equals_aberrated_multislice():
    w, pos, sp = W.small_workload(n=64, n_atoms=16, seed=10, f=1)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    L = w.cell[0]
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    xy = np.array([[0.0, 0.0], [5.5, 2.5]])
    kw = dict(C1=-40.0, C3=2.0e5)
    Dm = O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy, **kw)
    beams = O.beam_set(w.n, L, lam, w.alpha_max, 1)
    Dp = O.prism_outputs(O.build_smatrix(V, L, w.dz, lam, sig, beams), beams, L, w.n, lam, 1, xy, **kw)
    assert O.rel_err(Dp, Dm) < 1e-10
    assert O.rel_err(Dm, O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy)) > 1e-3


def test_aberration_phase_spherical_term_as_local_defocus():
    # On a thin ring |q| ~ q0 the C3 term equals a defocus C3 lam^2 q0^2 up to
    # a constant and a second-order remainder (pi/2) C3 lam^3 (q^2 - q0^2)^2.
    lam, L = 0.025, 100.0
    beams = np.array([[40, 0], [0, 41], [29, 29], [-39, 9]])
    q2 = (beams[:, 0] / L) ** 2 + (beams[:, 1] / L) ** 2
    q0sq = 0.16
    C3 = 1.0e6
    chi = O.aberration_phase(beams, L, lam, C3=C3)
    local = O.aberration_phase(beams, L, lam, C1=C3 * lam ** 2 * q0sq) - 0.5 * math.pi * C3 * lam ** 3 * q0sq ** 2
    rem = 0.5 * math.pi * C3 * lam ** 3 * (q2 - q0sq) ** 2
    assert np.max(np.abs(chi - local - rem)) < 1e-12


# ---------------------------------------------------------------------------
# 4D output: the full diffraction pattern per probe.
# ---------------------------------------------------------------------------
def test_diffraction_vacuum_peaks_and_parseval():
    n, L, E0, a, f = 64, 10.0, 80e3, 0.02, 2
    lam, sig = O.wavelength(E0), O.interaction_constant(E0)
    beams = O.beam_set(n, L, lam, a, f)
    S = O.build_smatrix(np.zeros((2, n, n)), L, 2.0, lam, sig, beams)
    xy = np.array([[1.0, 2.0], [7.5, 0.3]])
    I = O.prism_diffraction(S, beams, L, n, lam, f, xy)
    M = n // 2 // f
    # vacuum: one peak 1/|B| at every beam's window frequency k/f, zero elsewhere
    expected = np.zeros((M, M))
    for kx, ky in beams:
        expected[(ky // f) % M, (kx // f) % M] = 1.0 / len(beams)
    assert np.max(np.abs(I - expected[None])) < 1e-14


def test_diffraction_bins_sum_to_3d_output():
    w, pos, sp = W.small_workload(n=64, n_atoms=12, seed=11)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    L = w.cell[0]
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    beams = O.beam_set(w.n, L, lam, w.alpha_max, 2)
    S = O.build_smatrix(V, L, w.dz, lam, sig, beams)
    xy = np.array([[2.0, 3.0], [9.0, 1.0]])
    I = O.prism_diffraction(S, beams, L, w.n, lam, 2, xy)
    D = O.prism_outputs(S, beams, L, w.n, lam, 2, xy)
    M = w.n // 4
    bm = O.bin_map(lam, M, L / 2, O.alpha_aa(lam, w.n, L), 1e-3, D.shape[1])
    for p in range(len(xy)):
        assert np.allclose(O.stem.detect(I[p], bm, D.shape[1]), D[p], rtol=0, atol=1e-15)
    # Parseval: total intensity equals the window's mean squared amplitude
    C = O.probe_coefficients(beams, L, xy)
    cx, cy = O.window_centre(xy[0, 0], L, w.n), O.window_centre(xy[0, 1], L, w.n)
    win = O.probe_window(S, C[0], cx, cy, M)
    assert abs(I[0].sum() - np.sum(np.abs(win) ** 2) / M ** 2) < 1e-12


def test_frozen_phonon_average_of_identical_configs_is_single_run():
    w, pos, sp = W.small_workload(n=64, n_atoms=10, seed=12)
    lam = O.wavelength(w.E0)
    xy = np.array([[1.0, 1.0], [6.0, 4.0]])
    one = O.frozen_phonon_prism([pos], sp, w.species, w.cell, w.dz, w.n, w.E0, w.alpha_max, 2, xy)
    three = O.frozen_phonon_prism([pos, pos, pos], sp, w.species, w.cell, w.dz, w.n, w.E0, w.alpha_max, 2, xy)
    assert O.rel_err(three, one) < 1e-14
    # and the mean of two different configurations is the mean of their runs
    cfgs = W.thermal_configs(pos, 0.1, 2, seed=5)
    two = O.frozen_phonon_prism(cfgs, sp, w.species, w.cell, w.dz, w.n, w.E0, w.alpha_max, 2, xy)
    singles = [O.frozen_phonon_prism([c], sp, w.species, w.cell, w.dz, w.n, w.E0, w.alpha_max, 2, xy) for c in cfgs]
    assert O.rel_err(two, 0.5 * (singles[0] + singles[1])) < 1e-14
    assert O.rel_err(singles[0], singles[1]) > 1e-4


# ---------------------------------------------------------------------------
# Regression fixture: the oracle's 3D outputs on a 64^2 random cell as written
# by tests/golden/make_golden.py (oracle only).  Guards the oracle against
# unintended changes; any intended change to its arithmetic regenerates the
# fixture in the same commit.
# ---------------------------------------------------------------------------
def read_tiny_prism_fixture():
    probes, prism, ms = [], [], []
    with open(os.path.join(GOLDEN, "tiny_prism_f2_64.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            tag, *vals = line.split()
            v = [float(x) for x in vals]
            {"probe": probes, "prism": prism, "multislice": ms}[tag].append(v)
    return np.array(probes), np.array(prism), np.array(ms)


def test_oracle_reproduces_tiny_prism_fixture():
    xy, prism_ref, ms_ref = read_tiny_prism_fixture()
    w, pos, sp = W.small_workload(n=64, cell=(10.0, 10.0, 4.0), n_atoms=8, f=2, seed=11)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    beams = O.beam_set(w.n, w.cell[0], lam, w.alpha_max, w.f)
    S = O.build_smatrix(V, w.cell[0], w.dz, lam, sig, beams)
    prism = O.prism_outputs(S, beams, w.cell[0], w.n, lam, w.f, xy)
    ms = O.multislice_outputs(V, w.cell[0], w.dz, lam, sig, w.alpha_max, xy)
    assert np.allclose(prism, prism_ref, rtol=1e-12, atol=1e-15)
    assert np.allclose(ms, ms_ref, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# Error metrics and the detector's extent, each against values fixed by hand.
# ---------------------------------------------------------------------------
def test_rel_err_known_pair():
    # difference (0, 0, 0, -4) has norm 4; the reference (1, 2, 2, 4) has norm 5
    D = np.array([[1.0, 2.0], [2.0, 0.0]])
    Dref = np.array([[1.0, 2.0], [2.0, 4.0]])
    assert O.rel_err(D, Dref) == 0.8
    assert O.rel_err(Dref, Dref) == 0.0
    # relative to the second argument, not the first
    assert O.rel_err(Dref, D) == 4.0 / 3.0


def test_adf_signal_bins_at_the_inner_angle():
    # bin b holds 2^b: the dark-field sum from 40 mrad counts bins 40..64
    # only, i.e. 2^65 - 2^40 (bin 39 = [39, 40) mrad is bright field; bins
    # 40 and 41 are in), both exact in binary
    D = np.array([2.0 ** np.arange(65), np.zeros(65)])
    D[1, 39], D[1, 40], D[1, 41] = 1.0, 10.0, 100.0
    adf = O.adf_signal(D, 1e-3, 0.04)
    assert adf[0] == 2.0 ** 65 - 2.0 ** 40
    assert adf[1] == 110.0
    # the inner angle is a bin edge whatever its rounding in binary
    assert O.adf_signal(D, 1e-3, 0.041)[1] == 100.0
    assert O.adf_signal(D, 1e-3, 0.039)[1] == 111.0


@pytest.mark.parametrize("E0,n,L,n_bins", [(80e3, 256, 20.0, 134), (200e3, 1024, 100.0, 65),
                                           (200e3, 2048, 200.0, 65)])
def test_antialias_angle_is_the_propagator_band_edge(E0, n, L, n_bins):
    """alpha_AA is the scattering angle where the propagator's band limit cuts
    off: a Fourier pixel passes the band-limit mask exactly when its angle
    lam |k| / L is below alpha_AA (checked on every pixel of the grid), and the
    default bin count is the least number of 1 mrad bins that covers every
    pixel inside the band (the values of the benchmark geometries: 134 at
    80 keV, 20 A, 256^2; 65 at 200 keV, 0.0977 A pixels)."""
    lam = O.wavelength(E0)
    a_aa = O.alpha_aa(lam, n, L)
    k = O.fourier_indices(n)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    ang = lam * np.sqrt((kx * kx + ky * ky).astype(np.float64)) / L
    mask = O.band_limit_mask(n)
    # the pixels with |k| = n/4 exactly lie on the edge (angle alpha_AA up to
    # rounding) and are outside the band; every other pixel is clear of it,
    # so there the comparison is exact
    edge = 16 * (kx * kx + ky * ky) == n * n
    assert edge.sum() == 4 and not mask[edge].any()
    assert np.max(np.abs(ang[edge] - a_aa)) <= 4e-16 * a_aa
    assert np.min(np.abs(ang[~edge] - a_aa)) > 1e-9 * a_aa
    assert np.array_equal(mask[~edge], ang[~edge] < a_aa)
    nb = O.default_n_bins(lam, n, L, 1e-3)
    assert nb == n_bins
    inside = ang[mask]
    assert np.floor(inside.max() / 1e-3) == nb - 1


# ---------------------------------------------------------------------------
# PRISM with the beams streamed through window accumulators (no stored
# S-matrix): the vacuum closed form, f = 1 against multislice, and the stored
# form on a scattering cell, with the beams split over worker processes.
# ---------------------------------------------------------------------------
def test_prism_streamed_vacuum_closed_form():
    n, L, E0, a, f = 64, 10.0, 80e3, 0.02, 2
    lam, sig = O.wavelength(E0), O.interaction_constant(E0)
    nb = O.default_n_bins(lam, n, L, 1e-3)
    beams = O.beam_set(n, L, lam, a, f)
    xy = np.array([[0.0, 0.0], [3.3, 7.1], [9.9, 0.2]])
    D = O.prism_outputs_streamed(np.zeros((2, n, n)) + 5.0, L, 2.0, lam, sig, beams, n, f, xy, groups=3)
    assert np.max(np.abs(D - _vacuum_expected(lam, n, L, a, f, 1e-3, nb)[None, :])) < 1e-13


def test_prism_streamed_f1_equals_multislice_and_stored_form():
    w, pos, sp = W.small_workload(n=64, n_atoms=16, seed=5)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    L = w.cell[0]
    xy = np.array([[0.0, 0.0], [2.5, 7.5], [6.1, 3.9], [9.7, 9.7], [-1.2, 13.3]])
    Dm = O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy)
    Dm2 = O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy, processes=2)
    assert np.array_equal(Dm, Dm2)
    b1 = O.beam_set(w.n, L, lam, w.alpha_max, 1)
    assert O.rel_err(O.prism_outputs_streamed(V, L, w.dz, lam, sig, b1, w.n, 1, xy, processes=2), Dm) < 1e-10
    b2 = O.beam_set(w.n, L, lam, w.alpha_max, 2)
    stored = O.prism_outputs(O.build_smatrix(V, L, w.dz, lam, sig, b2), b2, L, w.n, lam, 2, xy)
    streamed = O.prism_outputs_streamed(V, L, w.dz, lam, sig, b2, w.n, 2, xy, processes=2, groups=5)
    assert O.rel_err(streamed, stored) < 1e-13
    assert O.rel_err(stored, Dm) > 1e-4      # f = 2 differs from multislice: the check is not vacuous


# ---------------------------------------------------------------------------
# Virtual detectors (Fig. 1e): a caller's detector map in place of annular
# bins.  detect() against hand sums; the vacuum closed form generalised to any
# map (the beams' pixels carry 1/|B| each); the annular map given explicitly
# reproduces the default output.
# ---------------------------------------------------------------------------
def test_detect_hand_sums():
    I = (2.0 ** np.arange(16)).reshape(4, 4)
    bmap = np.array([[0, 0, 1, -1], [2, 1, 1, -1], [-1, -1, 2, 0], [3, 3, 3, 3]])
    D = O.detect(I, bmap, 5)
    assert D.tolist() == [1 + 2 + 2 ** 11, 4 + 32 + 64, 16 + 2 ** 10, 2 ** 12 + 2 ** 13 + 2 ** 14 + 2 ** 15, 0.0]


def _segment_map(m, n_rings=3):
    """Quadrant segments of rings of the m x m FFT-order grid plus an
    off-centre disc: detector 4 r + quadrant for ring r, 4 n_rings for the disc."""
    k = O.fourier_indices(m)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    r = np.sqrt(kx * kx + ky * ky)
    ring = np.floor(r / (m / (2.0 * n_rings))).astype(int)
    quad = (kx >= 0).astype(int) + 2 * (ky >= 0).astype(int)
    out = np.where(ring < n_rings, 4 * ring + quad, -1)
    disc = (kx - m // 8) ** 2 + (ky + m // 16) ** 2 <= (m // 16) ** 2
    out[disc] = 4 * n_rings
    return out.astype(np.int32), 4 * n_rings + 1


@pytest.mark.parametrize("f", [1, 2])
def test_virtual_detector_vacuum_closed_form(f):
    n, L, E0, a = 64, 10.0, 80e3, 0.02
    lam, sig = O.wavelength(E0), O.interaction_constant(E0)
    beams = O.beam_set(n, L, lam, a, f)
    M = n // 2 // f
    dmap, nb = _segment_map(M)
    xy = np.array([[0.0, 0.0], [3.3, 7.1], [9.9, 0.2]])
    S = O.build_smatrix(np.zeros((2, n, n)) + 1.5, L, 2.0, lam, sig, beams)
    D = O.prism_outputs(S, beams, L, n, lam, f, xy, detector_map=dmap, n_bins=nb)
    # each beam lands on window pixel (kx/f, ky/f) with intensity 1/|B|
    exp = np.zeros(nb)
    for kx, ky in beams:
        d = dmap[(ky // f) % M, (kx // f) % M]
        if d >= 0:
            exp[d] += 1.0 / len(beams)
    assert np.max(np.abs(D - exp[None, :])) < 1e-13
    assert exp.min() == 0.0 and np.count_nonzero(exp) >= 4     # several detectors lit, some dark
    if f == 1:
        nmap, nbm = _segment_map(n)
        Dm = O.multislice_outputs(np.zeros((2, n, n)) + 1.5, L, 2.0, lam, sig, a, xy, detector_map=nmap,
                                  n_bins=nbm)
        expm = np.zeros(nbm)
        for kx, ky in beams:
            if nmap[ky % n, kx % n] >= 0:
                expm[nmap[ky % n, kx % n]] += 1.0 / len(beams)
        assert np.max(np.abs(Dm - expm[None, :])) < 1e-13


def test_virtual_detector_annular_map_equals_default():
    w, pos, sp = W.small_workload(n=64, n_atoms=16, seed=5)
    lam, sig = O.wavelength(w.E0), O.interaction_constant(w.E0)
    V = O.projected_potential(pos, sp, w.species, w.cell, w.dz, w.n)
    L, n, f = w.cell[0], w.n, 2
    xy = np.array([[0.0, 0.0], [2.5, 7.5]])
    beams = O.beam_set(n, L, lam, w.alpha_max, f)
    S = O.build_smatrix(V, L, w.dz, lam, sig, beams)
    nb = O.default_n_bins(lam, n, L, 1e-3)
    amap = O.bin_map(lam, n // 2 // f, L / f, O.alpha_aa(lam, n, L), 1e-3, nb)
    assert np.array_equal(O.prism_outputs(S, beams, L, n, lam, f, xy, detector_map=amap, n_bins=nb),
                          O.prism_outputs(S, beams, L, n, lam, f, xy))
    nmap = O.bin_map(lam, n, L, O.alpha_aa(lam, n, L), 1e-3, nb)
    assert np.array_equal(O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy, detector_map=nmap, n_bins=nb),
                          O.multislice_outputs(V, L, w.dz, lam, sig, w.alpha_max, xy))


def test_first_slice_is_the_shifted_row_spectrum():
    """The identity the first row pass of the GPU build rests on (shift
    theorem, Eqs. 1-2 with a plane-wave input): the row transform of a plane
    wave e^{2 pi i (kx x + ky y)/n} times a transmission T equals the row
    transform of T shifted by kx and phased by e^{2 pi i ky y/n}."""
    rng = np.random.default_rng(5)
    n = 64
    T = np.exp(1j * rng.uniform(0, 2, size=(n, n)))
    y, x = np.mgrid[0:n, 0:n]
    R = np.fft.fft(T, axis=1)
    for kx, ky in ((0, 0), (3, -5), (-7, 2), (31, -32)):
        pw = np.exp(2j * np.pi * (kx * x + ky * y) / n)
        lhs = np.fft.fft(pw * T, axis=1)
        k = np.arange(n)
        rhs = np.exp(2j * np.pi * ky * np.arange(n) / n)[:, None] * R[:, (k - kx) % n]
        assert np.max(np.abs(lhs - rhs)) < 1e-10 * np.max(np.abs(lhs))
