"""MI355X (gfx950) lattice Boltzmann library for natural convection of a
power-law fluid in a porous square cavity (arXiv:2011.15073).

The update runs in hand-written HIP kernels behind the C ABI of
``include/pmlbm.h`` (``libpmlbm.so``); this package is its Python binding:
``Cavity`` (one simulation), ``Sweep`` / ``tune`` (many cavities advanced
together), ``Adjoint`` / ``nusselt`` / ``vjp_step`` (gradients of the Nusselt
number).  PyTorch supplies device memory and streams only.
"""
from ._lib import (PM_CLAMP_GAMMA, PM_CLAMP_NU, PM_FP32, PM_FP64, PmError, lattice_of,
                   make_params, workspace_bytes)
from .cavity import Cavity, copy_probe
from .sweep import Sweep, tune
from .adjoint import Adjoint, nusselt, vjp_step

__all__ = ["Cavity", "Sweep", "tune", "Adjoint", "nusselt", "vjp_step", "copy_probe", "PmError",
           "make_params", "lattice_of", "workspace_bytes", "PM_FP32", "PM_FP64", "PM_CLAMP_NU",
           "PM_CLAMP_GAMMA"]
