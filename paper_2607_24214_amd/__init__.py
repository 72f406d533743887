"""MI355X-native quasistatic particle-in-cell hot path (HIP, gfx950).

The compute lives in libqsa.so (C ABI in include/qsa.h); this package is its
thin Python binding.  Importing the binding does not need a GPU; creating a
Sim does, and fails loudly if the library has not been built.
"""
from ._lib import FIELD_IDS, QSAError, QSAParams, lib  # noqa: F401
from .sim import (Batch, FieldEnergy, Sim, batch_sweep_static, dirichlet_solve, linear_model,  # noqa: F401
                  make_params, params_from_workload)

__all__ = ["Sim", "Batch", "FieldEnergy", "batch_sweep_static", "dirichlet_solve", "linear_model", "make_params",
           "params_from_workload", "QSAError", "QSAParams", "lib", "FIELD_IDS"]
