"""ctypes view of libprism.so: the structures and functions of include/prism.h.

Argument marshalling only.  Every computation happens in the HIP library; if
the library has not been built this module raises on import.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p, c_char_p

_HERE = os.path.dirname(os.path.abspath(__file__))
# PRISM_LIBRARY selects another build of the same library (A/B comparisons).
LIB_PATH = os.environ.get("PRISM_LIBRARY") or os.path.join(_HERE, "libprism.so")

PRISM_OK = 0
PRISM_E_INVAL = -1
PRISM_E_UNSUPPORTED = -2
PRISM_E_NOMEM = -3
PRISM_E_DEVICE = -4
PRISM_E_WORKSPACE = -5

PRISM_FP32 = 0
PRISM_SPLIT_BF16X3 = 1
PRISM_BF16 = 2

PRISM_NOALLOC_SCRATCH_BYTES = 64 << 20   # fixed scratch of prism_probe_outputs_noalloc


class prism_atom(ctypes.Structure):
    _fields_ = [("x", c_double), ("y", c_double), ("z", c_double), ("species", c_int32), ("pad", c_int32)]


class prism_species(ctypes.Structure):
    _fields_ = [("n_gauss", c_int32), ("pad", c_int32), ("amp", c_double * 4), ("width", c_double * 4)]


class prism_grid(ctypes.Structure):
    _fields_ = [("n", c_int32), ("n_slices", c_int32), ("cell", c_double * 3), ("dz", c_double)]


class prism_smatrix_desc(ctypes.Structure):
    _fields_ = [("grid", prism_grid), ("E0", c_double), ("alpha_max", c_double), ("f", c_int32),
                ("beam_batch", c_int32), ("n_beams", c_int32), ("ns", c_int32), ("m_win", c_int32),
                ("pad", c_int32), ("lambda_", c_double), ("sigma", c_double), ("alpha_aa", c_double),
                ("smatrix_bytes", c_size_t), ("build_ws_bytes", c_size_t)]


class prism_aberrations(ctypes.Structure):
    _fields_ = [("C1", c_double), ("C3", c_double)]


class prism_probe_plan(ctypes.Structure):
    _fields_ = [("n_probes", c_int64), ("n_bins", c_int32), ("n_tiles", c_int32), ("n_entries", c_int64),
                ("max_per_tile", c_int32), ("n_binned", c_int32), ("dalpha", c_double),
                ("plan_bytes", c_size_t), ("ws_bytes", c_size_t), ("C1", c_double), ("C3", c_double),
                ("off", c_size_t * 10)]


class prism_probe_job(ctypes.Structure):
    _fields_ = [("desc", POINTER(prism_smatrix_desc)), ("S", c_void_p), ("plan", POINTER(prism_probe_plan)),
                ("plan_dev", c_void_p), ("out", c_void_p), ("diffraction", c_void_p), ("out_scale", ctypes.c_float),
                ("accumulate", c_int32)]


class PrismError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libprism error {code}: {msg}")
        self.code = code


_SIGNATURES = {
    "prism_last_error": ([], c_char_p),
    "prism_grid_init": ([POINTER(c_double), c_double, c_int32, POINTER(prism_grid)], c_int32),
    "prism_project_potential_workspace": ([c_int64, POINTER(c_size_t)], c_int32),
    "prism_project_potential": ([POINTER(prism_atom), c_int64, POINTER(prism_species), c_int32,
                                 POINTER(prism_grid), c_void_p, c_void_p, c_size_t, c_void_p], c_int32),
    "prism_smatrix_plan": ([POINTER(prism_smatrix_desc)], c_int32),
    "prism_beam_list": ([POINTER(prism_smatrix_desc), c_void_p, c_int32], c_int32),
    "prism_build_smatrix": ([POINTER(prism_smatrix_desc), c_void_p, c_void_p, c_void_p, c_size_t, c_void_p],
                            c_int32),
    "prism_build_smatrix_range": ([POINTER(prism_smatrix_desc), c_void_p, c_void_p, c_int32, c_int32, c_void_p,
                                   c_size_t, c_void_p], c_int32),
    "prism_probe_plan_init": ([POINTER(prism_smatrix_desc), c_void_p, c_int64, c_double, c_int32,
                               POINTER(prism_aberrations), POINTER(prism_probe_plan)], c_int32),
    "prism_probe_plan_upload": ([POINTER(prism_smatrix_desc), c_void_p, POINTER(prism_probe_plan), c_void_p,
                                 c_void_p], c_int32),
    "prism_probe_plan_init_map": ([POINTER(prism_smatrix_desc), c_void_p, c_int64, c_void_p, c_int32,
                                   POINTER(prism_aberrations), POINTER(prism_probe_plan)], c_int32),
    "prism_probe_plan_upload_map": ([POINTER(prism_smatrix_desc), c_void_p, c_void_p, POINTER(prism_probe_plan),
                                     c_void_p, c_void_p], c_int32),
    "multislice_outputs_map": ([POINTER(prism_grid), c_double, c_double, POINTER(prism_aberrations), c_void_p,
                                c_void_p, c_int64, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_size_t,
                                c_void_p], c_int32),
    "prism_probe_outputs": ([POINTER(prism_smatrix_desc), c_void_p, POINTER(prism_probe_plan), c_void_p, c_int32,
                             c_void_p, c_void_p, c_size_t, c_void_p], c_int32),
    "prism_probe_outputs_noalloc": ([POINTER(prism_smatrix_desc), c_void_p, POINTER(prism_probe_plan), c_void_p,
                                     c_int32, c_void_p, c_void_p], c_int32),
    "prism_probe_diffraction": ([POINTER(prism_smatrix_desc), c_void_p, POINTER(prism_probe_plan), c_void_p, c_int32,
                                 c_void_p, c_void_p, c_size_t, c_void_p], c_int32),
    "prism_probe_batch_workspace": ([POINTER(prism_probe_job), c_int32, POINTER(c_size_t)], c_int32),
    "prism_probe_outputs_batched": ([POINTER(prism_probe_job), c_int32, c_int32, c_void_p, c_size_t, c_void_p],
                                    c_int32),
    "multislice_workspace": ([POINTER(prism_grid), c_int32, c_int64, POINTER(c_size_t)], c_int32),
    "multislice_outputs": ([POINTER(prism_grid), c_double, c_double, POINTER(prism_aberrations), c_void_p, c_void_p,
                            c_int64, c_double, c_int32, c_int32, c_void_p, c_void_p, c_size_t, c_void_p], c_int32),
    "prism_streaming_build_workspace": ([POINTER(prism_smatrix_desc), POINTER(c_size_t)], c_int32),
    "prism_build_smatrix_streaming": ([POINTER(prism_smatrix_desc), c_void_p, c_void_p, c_void_p, c_size_t,
                                       c_void_p, c_void_p, c_void_p], c_int32),
    "prism_probe_streaming_workspace": ([POINTER(prism_smatrix_desc), POINTER(prism_probe_plan), c_int32,
                                         POINTER(c_size_t)], c_int32),
    "prism_probe_outputs_streaming": ([POINTER(prism_smatrix_desc), c_void_p, POINTER(prism_probe_plan), c_void_p,
                                       c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p,
                                       c_void_p], c_int32),
    "prism_probe_chunked_workspace": ([POINTER(prism_smatrix_desc), POINTER(prism_probe_plan), c_int32,
                                       POINTER(c_size_t)], c_int32),
    "prism_probe_outputs_chunked": ([POINTER(prism_smatrix_desc), c_void_p, POINTER(prism_probe_plan), c_void_p,
                                     c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p], c_int32),
    "multislice_streaming_workspace": ([POINTER(prism_grid), c_int32, c_int64, POINTER(c_size_t)], c_int32),
    "multislice_outputs_streaming": ([POINTER(prism_grid), c_double, c_double, POINTER(prism_aberrations), c_void_p,
                                      c_void_p, c_int64, c_double, c_int32, c_int32, c_void_p, c_void_p, c_size_t,
                                      c_void_p, c_void_p], c_int32),
    "prism_detector_bin_map": ([c_double, c_double, c_double, c_double, c_int32, c_int32, c_void_p], c_int32),
    "prism_detector_default_bins": ([POINTER(prism_grid), c_double, c_double, POINTER(c_int32), POINTER(c_double)],
                                    c_int32),
    "prism_set_build_streams": ([c_int32], c_int32),
    "prism_device_copy": ([c_void_p, c_void_p, c_size_t, c_void_p], c_int32),
    "prism_timing_enable": ([c_int32], c_int32),
    "prism_timing_reset": ([], c_int32),
    "prism_timing_read": ([c_int32, POINTER(c_double), POINTER(c_int64)], c_int32),
}

TIMING_CLASSES = {"pass_a": 0, "pass_b": 1, "final": 2, "transmission": 3, "coefficients": 4, "contract": 5,
                  "window": 6, "potential": 7, "bin_reduce": 8, "split": 9, "first": 10}

EXPORTED = tuple(_SIGNATURES)


def load():
    # The library and PyTorch must share one HIP runtime (streams and device
    # memory cross between them).  PyTorch's HIP libraries find their runtime
    # under an unversioned name next to themselves; loading this library
    # first would bind the system runtime to the versioned name and leave
    # PyTorch to load a second copy.  Import torch first so that this
    # library binds to the runtime PyTorch already loaded.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
                          " (hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = load()


def check(rc):
    if rc != PRISM_OK:
        raise PrismError(rc, lib.prism_last_error().decode())
    return rc
