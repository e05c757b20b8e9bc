"""FP64 CPU oracle for the power-law / porous MRT lattice Boltzmann update.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It is a thin ctypes
wrapper over ``libpmoracle.so`` (built from ``pmoracle.c`` by ``build.py``)
and shares no code with the GPU library.

The oracle follows the update step by step as the paper states it
(Eqs. (12)-(24); readings where the paper is silent are documented in
``pmoracle.c``): collide every node with explicit matrix products, then
stream with bounce-back / anti-bounce-back walls.
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class Physics(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
                ("n", C.c_double), ("Da", C.c_double), ("Ra", C.c_double),
                ("Pr", C.c_double), ("eps", C.c_double), ("mach", C.c_double),
                ("nu_lo", C.c_double), ("nu_hi", C.c_double),
                ("clamp_mode", C.c_int32), ("forchheimer", C.c_int32),
                ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
                ("sT_e", C.c_double), ("sT_nu", C.c_double),
                ("gx", C.c_double), ("gy", C.c_double), ("T_init", C.c_double)]


class Lattice(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
                ("nu0", C.c_double), ("npow", C.c_double),
                ("nu_min", C.c_double), ("nu_max", C.c_double),
                ("gamma_scale", C.c_double), ("eps", C.c_double),
                ("K", C.c_double), ("K_scale", C.c_double),
                ("Feps", C.c_double), ("gbeta", C.c_double), ("T_m", C.c_double),
                ("gx", C.c_double), ("gy", C.c_double), ("alpha", C.c_double),
                ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
                ("sT_e", C.c_double), ("sT_nu", C.c_double),
                ("T_hot", C.c_double), ("T_cold", C.c_double),
                ("T_init", C.c_double), ("U_lb", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_DP = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(HERE, "libpmoracle.so")
    src = os.path.join(HERE, "pmoracle.c")
    if (not os.path.exists(path)) or os.path.getmtime(path) < os.path.getmtime(src):
        _build.build()
    L = C.CDLL(path)
    L.orc_map_physics.argtypes = [C.POINTER(Physics), C.POINTER(Lattice)]
    L.orc_map_physics.restype = C.c_int
    L.orc_new.argtypes = [C.POINTER(Lattice)]
    L.orc_new.restype = C.c_void_p
    L.orc_free.argtypes = [C.c_void_p]
    L.orc_last_error.restype = C.c_char_p
    L.orc_set_logda.argtypes = [C.c_void_p, C.c_void_p]
    L.orc_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_steps_done.argtypes = [C.c_void_p]
    L.orc_steps_done.restype = C.c_int64
    L.orc_step.argtypes = [C.c_void_p, C.c_int64]
    L.orc_macros.argtypes = [C.c_void_p] + [C.c_void_p] * 5
    L.orc_nu_bar.argtypes = [C.c_void_p]
    L.orc_nu_bar.restype = C.c_double
    L.orc_run_to_steady.argtypes = [C.c_void_p, C.c_double, C.c_int64, C.c_int64,
                                    C.POINTER(C.c_int64)]
    L.orc_run_to_steady.restype = C.c_double
    L.orc_collide_node.argtypes = [C.POINTER(Lattice), C.c_double, _DP, _DP, _DP, _DP,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]
    L.orc_feq.argtypes = [C.c_double] * 4 + [_DP]
    L.orc_forcing.argtypes = [C.c_double] * 6 + [_DP]
    L.orc_geq.argtypes = [C.c_double] * 3 + [_DP]
    L.orc_matrices.argtypes = [_DP] * 4
    L.orc_shear_sq.argtypes = [C.POINTER(Lattice), _DP, C.c_double, C.c_double,
                               C.c_double, C.c_double]
    L.orc_shear_sq.restype = C.c_double
    L.orc_viscosity.argtypes = [C.POINTER(Lattice), _DP, C.c_double, C.c_double,
                                C.c_double]
    L.orc_viscosity.restype = C.c_double
    _LIB = L
    return L


def physics(nx, ny=None, *, n=1.0, Da=math.inf, Ra=1e3, Pr=10.0, eps=1.0, mach=0.1,
            nu_lo=0.1, nu_hi=10.0, clamp_mode=0, forchheimer=1, s_e=0.0, s_eps=0.0,
            s_q=0.0, sT_e=0.0, sT_nu=0.0, gx=0.0, gy=0.0, T_init=0.5,
            periodic_x=0, periodic_y=0) -> Physics:
    """Physical parameters (0 for a rate selects its default)."""
    return Physics(nx, nx if ny is None else ny, periodic_x, periodic_y, n, Da, Ra, Pr,
                   eps, mach, nu_lo, nu_hi, clamp_mode, forchheimer, s_e, s_eps, s_q,
                   sT_e, sT_nu, gx, gy, T_init)


def map_physics(p: Physics) -> Lattice:
    lat = Lattice()
    if lib().orc_map_physics(C.byref(p), C.byref(lat)) != 0:
        raise ValueError(lib().orc_last_error().decode())
    return lat


def lattice(nx, ny=None, **kw) -> Lattice:
    """Lattice parameters with test-friendly defaults, overridable by keyword."""
    lat = Lattice()
    d = dict(nx=nx, ny=nx if ny is None else ny, periodic_x=0, periodic_y=0,
             nu0=0.1, npow=1.0, nu_min=0.01, nu_max=1.0, gamma_scale=1.0, eps=1.0,
             K=math.inf, K_scale=float(nx * nx), Feps=0.0, gbeta=0.0, T_m=0.5,
             gx=0.0, gy=0.0, alpha=0.1, s_e=1.4, s_eps=1.4, s_q=1.2, sT_e=1.0,
             sT_nu=1.0, T_hot=1.0, T_cold=0.0, T_init=0.5, U_lb=0.1 / math.sqrt(3.0))
    d.update(kw)
    for k, v in d.items():
        setattr(lat, k, v)
    return lat


class Oracle:
    """One oracle simulation state (pre-collision populations, FP64)."""

    def __init__(self, lat: Lattice, logda=None):
        self.lat = lat
        self._h = lib().orc_new(C.byref(lat))
        if not self._h:
            raise ValueError(lib().orc_last_error().decode())
        self.nx, self.ny = lat.nx, lat.ny
        if logda is not None:
            self.set_logda(logda)

    @classmethod
    def from_physics(cls, p: Physics, logda=None):
        return cls(map_physics(p), logda)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _LIB is not None:
            try:
                _LIB.orc_free(h)
            except Exception:
                pass
            self._h = None

    def set_logda(self, logda):
        a = np.ascontiguousarray(logda, dtype=np.float64).reshape(self.ny, self.nx)
        self._logda = a
        lib().orc_set_logda(self._h, a.ctypes.data)

    def step(self, k: int):
        lib().orc_step(self._h, int(k))
        return self

    @property
    def steps(self) -> int:
        return lib().orc_steps_done(self._h)

    def state(self):
        f = np.empty((9, self.ny, self.nx))
        g = np.empty((5, self.ny, self.nx))
        lib().orc_get_state(self._h, f.ctypes.data, g.ctypes.data)
        return f, g

    def set_state(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert f.size == 9 * self.nx * self.ny and g.size == 5 * self.nx * self.ny
        lib().orc_set_state(self._h, f.ctypes.data, g.ctypes.data)

    def macros(self):
        """dict of rho, ux, uy (lattice units), T, nu, each [ny, nx]."""
        out = {k: np.empty((self.ny, self.nx)) for k in ("rho", "ux", "uy", "T", "nu")}
        lib().orc_macros(self._h, *(out[k].ctypes.data for k in ("rho", "ux", "uy", "T", "nu")))
        return out

    def fields(self):
        """Nondimensional U, V (u / U_lb) and theta, each [ny, nx]."""
        m = self.macros()
        U = self.lat.U_lb
        th = (m["T"] - self.lat.T_cold) / (self.lat.T_hot - self.lat.T_cold)
        return m["ux"] / U, m["uy"] / U, th

    def nu_bar(self) -> float:
        return lib().orc_nu_bar(self._h)

    def run_to_steady(self, tol=1e-8, check_every=1000, max_steps=2_000_000):
        steps = C.c_int64(0)
        r = lib().orc_run_to_steady(self._h, tol, int(check_every), int(max_steps),
                                    C.byref(steps))
        return r, steps.value


def matrices():
    M = np.empty((9, 9)); Mi = np.empty((9, 9)); N = np.empty((5, 5)); Ni = np.empty((5, 5))
    lib().orc_matrices(M, Mi, N, Ni)
    return M, Mi, N, Ni


def feq(eps, rho, ux, uy):
    out = np.empty(9)
    lib().orc_feq(eps, rho, ux, uy, out)
    return out


def forcing(eps, rho, ux, uy, Fx, Fy):
    out = np.empty(9)
    lib().orc_forcing(eps, rho, ux, uy, Fx, Fy, out)
    return out


def geq(T, ux, uy):
    out = np.empty(5)
    lib().orc_geq(T, ux, uy, out)
    return out


def collide_node(lat: Lattice, K, f, g):
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    fo = np.empty(9); go = np.empty(5)
    vals = [C.c_double() for _ in range(5)]
    lib().orc_collide_node(C.byref(lat), K, f, g, fo, go, *(C.byref(v) for v in vals))
    rho, ux, uy, T, nu = (v.value for v in vals)
    return fo, go, dict(rho=rho, ux=ux, uy=uy, T=T, nu=nu)


def shear_sq(lat: Lattice, f, rho, vx, vy, s_nu):
    return lib().orc_shear_sq(C.byref(lat), np.ascontiguousarray(f, dtype=np.float64),
                              rho, vx, vy, s_nu)


def viscosity(lat: Lattice, f, rho, vx, vy):
    return lib().orc_viscosity(C.byref(lat), np.ascontiguousarray(f, dtype=np.float64),
                               rho, vx, vy)
