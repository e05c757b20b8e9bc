"""ctypes binding of libpmlbm.so (the C ABI declared in include/pmlbm.h).

Argument marshalling only: every step of the update runs in the HIP kernels
of the shared library.  If the library is missing this module raises at
import time -- there is no fallback implementation.
"""
import ctypes as C
import math
import os

# torch must load its HIP runtime before libpmlbm.so resolves libamdhip64:
# the library then binds to the same runtime as the device memory and streams
# it is handed (a second runtime in the process would see no device).
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmlbm.so")

PM_OK, PM_EINVAL, PM_EDEVICE, PM_EDIVERGED, PM_ESTATE = 0, -1, -2, -3, -4
PM_FP32, PM_FP64, PM_FP16 = 0, 1, 2
PM_CLAMP_NU, PM_CLAMP_GAMMA = 0, 1
PM_ROUND_NEAREST, PM_ROUND_STOCHASTIC, PM_ROUND_AUTO = 0, 1, 2

# every symbol the header declares, in declaration order
EXPORTS = [
    "pm_params_default", "pm_lattice_of", "pm_workspace_bytes", "pm_init", "pm_destroy",
    "pm_set_logda", "pm_step", "pm_steps_done", "pm_nu", "pm_residual", "pm_run_to_steady",
    "pm_fields", "pm_stream_function", "pm_viscosity", "pm_get_populations", "pm_set_populations",
    "pm_state_bytes", "pm_save_state", "pm_load_state", "pm_copy_probe",
    "pm_sweep_workspace_bytes", "pm_sweep_create", "pm_sweep_set_order", "pm_sweep_set_tile", "pm_sweep_run",
    "pm_sweep_advance", "pm_sweep_status",
    "pm_sweep_step", "pm_sweep_case", "pm_sweep_destroy", "pm_sweep_last_error",
    "pm_adjoint_workspace_bytes", "pm_adjoint_create", "pm_adjoint_forward",
    "pm_adjoint_backward", "pm_adjoint_set_shear_floor", "pm_adjoint_set_lambda_dtype", "pm_adjoint_destroy",
    "pm_adjoint_last_error",
    "pm_adjoint_vjp_scratch_bytes", "pm_adjoint_vjp", "pm_adjoint_vjp_noalloc",
    "pm_strerror", "pm_last_error",
]

PM_ORDER_CASE, PM_ORDER_LARGEST, PM_ORDER_INTERLEAVE = 0, 1, 2


class PmParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
                ("n", C.c_double), ("Da", C.c_double), ("Ra", C.c_double), ("Pr", C.c_double),
                ("eps", C.c_double), ("mach", C.c_double),
                ("nu_lo", C.c_double), ("nu_hi", C.c_double),
                ("clamp_mode", C.c_int32), ("dtype", C.c_int32), ("forchheimer", C.c_int32),
                ("has_logda", C.c_int32),
                ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double),
                ("sT_e", C.c_double), ("sT_nu", C.c_double),
                ("gx", C.c_double), ("gy", C.c_double), ("T_init", C.c_double),
                ("step_kernel", C.c_int32), ("rounding", C.c_int32)]


class PmLattice(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "U_lb", "nu0", "nu_min", "nu_max", "gamma_scale", "eps", "K", "Feps", "gbeta", "T_m",
        "alpha", "tau0", "tau_min", "tau_max", "tau_g", "s_e", "s_eps", "s_q", "sT_e", "sT_nu")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python paper_2011_15073_amd/build.py` first")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_size_t, C.c_double
    P = C.POINTER
    sig = {
        "pm_params_default": ([P(PmParams)], i32),
        "pm_lattice_of": ([P(PmParams), P(PmLattice)], i32),
        "pm_workspace_bytes": ([P(PmParams), P(sz)], i32),
        "pm_init": ([P(PmParams), vp, sz, vp, P(vp)], i32),
        "pm_destroy": ([vp], None),
        "pm_set_logda": ([vp, vp, i32], i32),
        "pm_step": ([vp, i64], i32),
        "pm_steps_done": ([vp, P(i64)], i32),
        "pm_nu": ([vp, P(dbl)], i32),
        "pm_residual": ([vp, P(dbl), P(i64)], i32),
        "pm_run_to_steady": ([vp, dbl, i64, i64, P(i64), P(dbl)], i32),
        "pm_fields": ([vp, vp, vp, vp, i32], i32),
        "pm_viscosity": ([vp, vp, i32], i32),
        "pm_stream_function": ([vp, vp, i32], i32),
        "pm_get_populations": ([vp, vp, vp, i32], i32),
        "pm_set_populations": ([vp, vp, vp, i32], i32),
        "pm_state_bytes": ([vp, P(sz)], i32),
        "pm_save_state": ([vp, vp, sz], i32),
        "pm_load_state": ([vp, vp, sz], i32),
        "pm_copy_probe": ([vp, vp, sz, vp], i32),
        "pm_sweep_workspace_bytes": ([P(PmParams), i32, P(sz)], i32),
        "pm_sweep_create": ([P(PmParams), i32, vp, sz, vp, P(vp)], i32),
        "pm_sweep_set_order": ([vp, i32], i32),
        "pm_sweep_set_tile": ([vp, i32, i32], i32),
        "pm_sweep_run": ([vp, dbl, i64, i64, P(i64), P(dbl)], i32),
        "pm_sweep_step": ([vp, i64], i32),
        "pm_sweep_advance": ([vp, dbl, i64, i64, i64, P(i32)], i32),
        "pm_sweep_status": ([vp, P(i64), P(dbl)], i32),
        "pm_sweep_case": ([vp, i32, P(vp)], i32),
        "pm_sweep_destroy": ([vp], None),
        "pm_sweep_last_error": ([vp], C.c_char_p),
        "pm_adjoint_workspace_bytes": ([P(PmParams), i64, i64, P(sz)], i32),
        "pm_adjoint_create": ([vp, i64, i64, vp, sz, P(vp)], i32),
        "pm_adjoint_forward": ([vp, P(dbl)], i32),
        "pm_adjoint_backward": ([vp, dbl, vp, P(dbl), P(dbl)], i32),
        "pm_adjoint_set_shear_floor": ([vp, dbl], i32),
        "pm_adjoint_set_lambda_dtype": ([vp, i32], i32),
        "pm_adjoint_destroy": ([vp], None),
        "pm_adjoint_last_error": ([vp], C.c_char_p),
        "pm_adjoint_vjp_scratch_bytes": ([vp], sz),
        "pm_adjoint_vjp": ([vp, vp, vp, vp, vp, sz, P(dbl)], i32),
        "pm_adjoint_vjp_noalloc": ([vp, vp, vp, vp, P(dbl)], i32),
        "pm_strerror": ([i32], C.c_char_p),
        "pm_last_error": ([vp], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        try:
            fn = getattr(L, name)
        except AttributeError:
            raise ImportError(f"{LIB_PATH} does not export {name} (a stale build?); rebuild it with "
                              "`python paper_2011_15073_amd/build.py`") from None
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def check(rc, ctx=None, errfn=None):
    if rc != PM_OK:
        msg = (errfn or lib.pm_last_error)(ctx).decode(errors="replace")
        raise PmError(rc, f"{lib.pm_strerror(rc).decode()}: {msg}")
    return rc


def make_params(nx, ny=None, *, n=1.0, Da=math.inf, Ra=1e3, Pr=10.0, eps=1.0, mach=0.1,
                nu_lo=0.1, nu_hi=10.0, clamp_mode=PM_CLAMP_NU, dtype="fp32", forchheimer=1,
                has_logda=0, s_e=0.0, s_eps=0.0, s_q=0.0, sT_e=0.0, sT_nu=0.0, gx=0.0, gy=0.0,
                T_init=0.5, periodic_x=0, periodic_y=0, step_kernel=0, rounding="auto") -> PmParams:
    p = PmParams()
    check(lib.pm_params_default(C.byref(p)))
    p.nx, p.ny = int(nx), int(nx if ny is None else ny)
    p.periodic_x, p.periodic_y = int(periodic_x), int(periodic_y)
    p.n, p.Da, p.Ra, p.Pr, p.eps, p.mach = n, Da, Ra, Pr, eps, mach
    p.nu_lo, p.nu_hi, p.clamp_mode = nu_lo, nu_hi, int(clamp_mode)
    p.dtype = {"fp32": PM_FP32, "fp64": PM_FP64, "fp16": PM_FP16, PM_FP32: PM_FP32, PM_FP64: PM_FP64,
               PM_FP16: PM_FP16}[dtype]
    p.forchheimer, p.has_logda = int(forchheimer), int(has_logda)
    p.s_e, p.s_eps, p.s_q, p.sT_e, p.sT_nu = s_e, s_eps, s_q, sT_e, sT_nu
    p.gx, p.gy, p.T_init = gx, gy, T_init
    p.step_kernel = {"auto": 0, "single": 1, "pair": 2, 0: 0, 1: 1, 2: 2}[step_kernel]
    p.rounding = {"nearest": PM_ROUND_NEAREST, "stochastic": PM_ROUND_STOCHASTIC, "auto": PM_ROUND_AUTO,
                  PM_ROUND_NEAREST: PM_ROUND_NEAREST, PM_ROUND_STOCHASTIC: PM_ROUND_STOCHASTIC,
                  PM_ROUND_AUTO: PM_ROUND_AUTO}[rounding]
    return p


def lattice_of(p: PmParams) -> PmLattice:
    out = PmLattice()
    check(lib.pm_lattice_of(C.byref(p), C.byref(out)))
    return out


def workspace_bytes(p: PmParams) -> int:
    n = C.c_size_t()
    check(lib.pm_workspace_bytes(C.byref(p), C.byref(n)))
    return n.value
