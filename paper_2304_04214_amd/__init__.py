"""MI355X (gfx950) implementation of the synthetic-turbulence-generator inlet
for the wall-modelled MRT lattice Boltzmann channel (arXiv 2304.04214).

The compute path is the HIP library ``liblbm.so`` (C ABI in include/lbm.h);
this package only marshals arguments.  Importing it does not load the
library; the first call that needs it does, and fails loudly if it has not
been built.
"""
__all__ = ["Channel", "copy_probe", "lattice_tables", "synthetic", "build"]


def __getattr__(name):
    if name in ("Channel", "copy_probe", "lattice_tables"):
        from . import channel
        return getattr(channel, name)
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
