"""MI355X (gfx950) explicit finite-difference acoustic propagator.

The library libwavefd.so (HIP kernels + C ABI, include/wavefd.h) does all the
numerical work; this package is its Python binding:

* `_abi`        - ctypes binding with the C names (wf_forward, wf_adjoint, ...)
* `propagator`  - `Propagator` (one device-resident model) and
                  `ModelingFunction` (torch.autograd.Function: m -> shot record)
* `serve`       - the continuous-batching serving front-end

Importing the package loads the library and fails if it is not built.
"""
from . import _abi
from ._abi import WaveFDError, make_geom
from .propagator import ModelingFunction, Propagator, model_data, pad_replicate, slowness_sq

__all__ = ["_abi", "WaveFDError", "make_geom", "Propagator", "ModelingFunction", "model_data",
           "pad_replicate", "slowness_sq"]
