"""MI355X (gfx950) lattice Boltzmann library for natural convection of a
power-law fluid in a porous square cavity (arXiv:2011.15073).

The update runs in hand-written HIP kernels behind the C ABI of
``include/pmlbm.h`` (``libpmlbm.so``); this package is its Python binding:
``Cavity`` (one simulation), ``Sweep`` / ``tune`` (many cavities advanced
together), ``Adjoint`` / ``nusselt`` / ``vjp_step`` (gradients of the Nusselt
number).  PyTorch supplies device memory and streams only.

The binding is loaded on first use of any of these names (the first access
loads ``libpmlbm.so`` and raises if it is missing: there is no fallback), so
that ``paper_2011_15073_amd.inputs`` -- the seeded input generators, which
hold none of the method's arithmetic -- can be imported without the library.
"""
import importlib

_EXPORTS = {
    "Cavity": ".cavity", "copy_probe": ".cavity",
    "Sweep": ".sweep", "tune": ".sweep",
    "Adjoint": ".adjoint", "nusselt": ".adjoint", "vjp_step": ".adjoint",
    "PmError": "._lib", "make_params": "._lib", "lattice_of": "._lib", "workspace_bytes": "._lib",
    "PM_FP32": "._lib", "PM_FP64": "._lib", "PM_FP16": "._lib", "PM_CLAMP_NU": "._lib", "PM_CLAMP_GAMMA": "._lib",
}

__all__ = list(_EXPORTS)


_SUBMODULES = ("cavity", "sweep", "adjoint", "_lib", "inputs")


def __getattr__(name):
    if name in _SUBMODULES:
        return importlib.import_module("." + name, __name__)
    mod = _EXPORTS.get(name)
    if mod is None:
        raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
    value = getattr(importlib.import_module(mod, __name__), name)
    globals()[name] = value
    return value


def __dir__():
    return sorted(set(globals()) | set(_EXPORTS))
