"""FP64 CPU oracle for the PRISM and multislice STEM hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything under this package.
Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use it.

The oracle is a plain, slow, obviously-correct NumPy implementation in float64
of what the GPU path computes, written from the paper (Pryor, Ophus, Miao,
"A Streaming Multi-GPU Implementation of Image Simulation Algorithms for
Scanning Transmission Electron Microscopy", 2017):

* projected potential slices          -- "Calculation of the Projected Potentials"
* transmission                        -- Eq. (1)
* Fresnel propagation                 -- Eq. (2)
* multislice probe simulation         -- "Description of Algorithms", Fig. 1c-e;
                                         "Multislice Probe Simulations"
* PRISM beam set, compact S-matrix    -- Fig. 1f-h; "PRISM Probe Simulations"
* PRISM probe synthesis               -- Fig. 1i-k; "PRISM Probe Simulations"
* annular detector bins (3D output)   -- Fig. 1e

Where the paper is silent (relativistic constants, band limit, normalisation,
window centring, bin edges) the readings are listed in the module docstrings
of `stem.py` and in the design notes.  It shares no code with the GPU path.
"""
from .stem import (  # noqa: F401
    PLANCK, LIGHT, CHARGE, MASS0,
    wavelength, interaction_constant,
    fourier_indices, band_limit_mask,
    slice_index, projected_potential,
    transmission, propagator,
    alpha_aa, default_n_bins, bin_map,
    beam_set, probe_coefficients, aberration_phase,
    multislice_outputs, multislice_exit_spectrum,
    smatrix_layer, build_smatrix, smatrix_windows, prism_outputs_streamed,
    window_centre, probe_window, prism_outputs, prism_diffraction, frozen_phonon_prism, window_detector_map, detect,
    rel_err, adf_signal,
)
