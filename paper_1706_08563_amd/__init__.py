"""MI355X (gfx950) PRISM / multislice STEM simulation.

Thin Python layer over libprism.so (HIP kernels + C ABI, include/prism.h).
PyTorch only provides device memory and the HIP stream; every step of the
simulation runs in the library's kernels.  Importing this package fails if
the library has not been built.
"""
from ._lib import (  # noqa: F401
    PRISM_OK, PRISM_E_INVAL, PRISM_E_UNSUPPORTED, PRISM_E_NOMEM, PRISM_E_DEVICE, PRISM_E_WORKSPACE,
    PRISM_FP32, PRISM_SPLIT_BF16X3, PRISM_BF16, PRISM_NOALLOC_SCRATCH_BYTES, PrismError, EXPORTED, LIB_PATH,
    prism_atom, prism_species, prism_grid, prism_smatrix_desc, prism_probe_plan, prism_probe_job, TIMING_CLASSES,
)
from .api import (  # noqa: F401
    lib, prism_grid_init, prism_smatrix_plan, prism_beam_list, prism_detector_bin_map, prism_detector_default_bins,
    prism_project_potential, prism_build_smatrix, prism_build_smatrix_range, prism_probe_plan_init, prism_probe_plan_upload,
    prism_probe_outputs, multislice_outputs, multislice_workspace, ProbePlan,
    prism_timing_enable, prism_timing_reset, prism_timing_read,
    prism_probe_batch_workspace, prism_probe_outputs_batched, prism_probe_diffraction,
    prism_streaming_build_workspace, prism_build_smatrix_streaming, prism_probe_streaming_workspace,
    prism_probe_outputs_streaming, multislice_streaming_workspace, multislice_outputs_streaming,
    prism_probe_chunked_workspace, prism_probe_outputs_chunked, prism_set_build_streams,
    prism_device_copy, prism_probe_outputs_noalloc,
)
from . import _lib  # noqa: F401
