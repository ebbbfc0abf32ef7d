"""MI355X-native AAHRT: GFST forward/adjoint operators and sparse (FISTA) inversion.

The computation lives in the HIP library libaahrt.so (C ABI in include/aahrt.h);
this package only marshals arguments.  Importing it does not load the library;
the first Plan() does, and raises if the library has not been built.
"""
from .api import Axes, Plan, plan_from_workload
from .autograd import AAHRTFunction, aahrt

__all__ = ['Axes', 'Plan', 'plan_from_workload', 'AAHRTFunction', 'aahrt']
