"""Detector-output gates shared by the GPU parity tests.

A 3D output D[probe][bin] passes against the FP64 reference when
* the Frobenius relative error over probes x bins is within tol,
* the relative error of the dark-field signal (bins from 40 mrad) is within tol,
* every element satisfies |dD| <= tol |D_ref| + tol * 1e-3 * max(D_ref):
  relative per bin, with an absolute floor of 1e-3 of the brightest bin so that
  bins that are empty to rounding (window corners, far dark field) do not
  demand a relative error below the arithmetic's resolution.
Each check prints the norm-wise errors and the worst per-bin relative errors
(|dD| / max(|D_ref|, 1e-3 max D_ref), the maximum over probes, per bin).
"""
import sys

import numpy as np

import oracle as O

TOL = 1e-4
FLOOR = 1e-3


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def per_bin_max(got, ref):
    """Worst relative error of each bin over probes, with the floor above."""
    got = np.atleast_2d(np.asarray(got, dtype=np.float64))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    scale = np.maximum(np.abs(ref), FLOOR * np.max(np.abs(ref)))
    return np.max(np.abs(got - ref) / scale, axis=0)


def check_D(got, ref, label, tol=TOL, adf_from=0.04, dalpha=1e-3):
    """Gate (tol not None) or only report (tol None) a 3D output against its
    reference.  adf_from=None: the outputs are not annular bins (virtual
    detectors), so there is no dark-field signal to gate."""
    got = np.atleast_2d(np.asarray(got, dtype=np.float64))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    assert got.shape == ref.shape, (got.shape, ref.shape)
    e_all = O.rel_err(got, ref)
    if adf_from is None:
        e_adf = 0.0
    else:
        assert ref.shape[1] * dalpha > adf_from, (label, "no bin reaches the dark-field range")
        e_adf = O.rel_err(O.adf_signal(got, dalpha, adf_from), O.adf_signal(ref, dalpha, adf_from))
    pb = per_bin_max(got, ref)
    worst = np.argsort(pb)[::-1][:3]
    say(f"  {label}: rel_all={e_all:.3e} rel_adf={e_adf:.3e} per-bin max={pb.max():.3e} "
        f"(bins {', '.join(f'{int(b)}:{pb[b]:.2e}' for b in worst)})")
    if tol is not None:
        bound = tol * np.abs(ref) + tol * FLOOR * np.max(np.abs(ref))
        bad = np.abs(got - ref) > bound
        assert e_all <= tol and e_adf <= tol, (label, e_all, e_adf)
        assert not bad.any(), (label, "element-wise", np.argwhere(bad)[:5].tolist())
    return e_all, e_adf, float(pb.max())
