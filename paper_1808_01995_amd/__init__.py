"""MI355X (gfx950) explicit finite-difference acoustic propagator.

The library libwavefd.so (HIP kernels + C ABI, include/wavefd.h) does all the
numerical work; this package is its Python binding:

* `_abi`        - ctypes binding with the C names (wf_forward, wf_adjoint, ...)
* `propagator`  - `Propagator` (one device-resident model),
                  `ModelingFunction` (torch.autograd.Function: m -> shot record)
                  and `FWIObjective` (m -> multi-shot misfit, gradient formed
                  in the forward pass)
* `serve`       - the continuous-batching serving front-end

Importing the package loads the library and fails if it is not built.
"""
from . import _abi
from ._abi import WaveFDError, make_geom
from .propagator import (FWIObjective, ModelingFunction, Propagator, fwi_objective, model_data,
                         pad_replicate, slowness_sq)

__all__ = ["_abi", "WaveFDError", "make_geom", "Propagator", "ModelingFunction", "model_data",
           "FWIObjective", "fwi_objective",
           "pad_replicate", "slowness_sq"]
