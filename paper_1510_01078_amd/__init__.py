"""MI355X (gfx950) NEDNER-NUFFT planar photoacoustic reconstruction.

The compute path is the HIP library libpatnufft.so (C ABI in
include/pat_nufft.h); `Plan` is its Python binding. `inputs` holds the
seeded synthetic workloads.
"""
__version__ = "0.1.0"


def __getattr__(name):
    if name == "Plan":
        from .plan import Plan
        return Plan
    raise AttributeError(name)
