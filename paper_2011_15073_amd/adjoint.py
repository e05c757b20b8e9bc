"""Gradients of the hot-wall Nusselt number through the discrete adjoint of
the update (pm_adjoint_* of the C ABI), exposed as a torch.autograd.Function.

``nusselt(logda, n, Ra, ...)`` runs T steps of the cavity from rest (FP32 or
FP64 state) and returns Nu_bar (Eq. 24) as a 0-d tensor; backward gives
dNu/d(logda field), dNu/dn and dNu/dRa.  Memory: checkpoints every C steps
(default C = ceil(sqrt(T))), each segment replayed before its adjoint steps.
All arithmetic runs in the library's kernels; torch only holds memory.
"""
import ctypes as C
import math

import torch

from ._lib import PM_FP32, check, lib
from .cavity import Cavity


class Adjoint:
    """Forward run with checkpoints + backward sweep for one cavity.

    ``lambda_dtype="fp32"`` (FP32 cavities only) stores the adjoint state in
    FP32 between steps, halving its memory traffic; the arithmetic stays FP64.
    """

    def __init__(self, cavity: Cavity, T: int, C_every: int = None, shear_floor: float = 0.0,
                 lambda_dtype: str = "fp64"):
        self.cav = cavity
        self.T = int(T)
        self.C = int(C_every or math.ceil(math.sqrt(T)))
        nb = C.c_size_t()
        check(lib.pm_adjoint_workspace_bytes(C.byref(cavity.params), self.T, self.C, C.byref(nb)))
        align = 1 << 21
        self.ws = torch.empty(nb.value + align, dtype=torch.uint8, device=cavity.device)
        base = (self.ws.data_ptr() + align - 1) // align * align
        h = C.c_void_p()
        check(lib.pm_adjoint_create(cavity._h, self.T, self.C, C.c_void_p(base), nb, C.byref(h)))
        self._h = h
        if shear_floor:
            self._check(lib.pm_adjoint_set_shear_floor(self._h, float(shear_floor)))
        if lambda_dtype not in ("fp64", "fp32"):
            raise ValueError(f"lambda_dtype must be 'fp64' or 'fp32', not {lambda_dtype!r}")
        if lambda_dtype == "fp32":
            self._check(lib.pm_adjoint_set_lambda_dtype(self._h, PM_FP32))

    def _check(self, rc):
        return check(rc, self._h, lib.pm_adjoint_last_error)

    def forward(self):
        J = C.c_double()
        self._check(lib.pm_adjoint_forward(self._h, C.byref(J)))
        return J.value

    def backward(self, seed=1.0):
        cav = self.cav
        g_ld = None
        ptr = None
        if cav.params.has_logda:
            g_ld = torch.empty((cav.ny, cav.nx), dtype=torch.float64, device=cav.device)
            ptr = C.c_void_p(g_ld.data_ptr())
        gn, gRa = C.c_double(), C.c_double()
        self._check(lib.pm_adjoint_backward(self._h, float(seed), ptr, C.byref(gn), C.byref(gRa)))
        return g_ld, gn.value, gRa.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.pm_adjoint_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NuFn(torch.autograd.Function):
    """J = Nu_bar after T steps; inputs: logda [N, N] (float64), n, Ra (0-d)."""

    @staticmethod
    def forward(ctx, logda, n, Ra, T, C_every, kw):
        N = logda.shape[-1]
        cav = Cavity(N, logda=logda.detach(), n=float(n), Ra=float(Ra), **kw)
        adj = Adjoint(cav, T, C_every)
        J = adj.forward()
        ctx.adj = adj
        ctx.devices = (logda.device, n.device if torch.is_tensor(n) else None,
                       Ra.device if torch.is_tensor(Ra) else None)
        return torch.tensor(J, dtype=torch.float64, device=logda.device)

    @staticmethod
    def backward(ctx, gJ):
        g_ld, gn, gRa = ctx.adj.backward(seed=float(gJ))
        ctx.adj.close()
        dl, dn, dR = ctx.devices
        return (g_ld.to(device=dl, dtype=torch.float64), torch.tensor(gn, dtype=torch.float64, device=dn),
                torch.tensor(gRa, dtype=torch.float64, device=dR), None, None, None)


def nusselt(logda, n, Ra, T=5000, C_every=None, **kw):
    """Differentiable Nu_bar after T steps from rest; ``kw``: the other
    ``make_params`` keywords (Pr, eps, dtype, ...)."""
    return NuFn.apply(logda, n, Ra, int(T), C_every, kw)


def vjp_step(cavity: Cavity, lam_next):
    """One adjoint step at the cavity's current state: returns (lam,
    grad_logda or None, dL/dn, dL/dRa) for L = <lam_next, S_{k+1}>."""
    lam_next = lam_next.to(device=cavity.device, dtype=torch.float64).contiguous()
    lam = torch.empty_like(lam_next)
    g_ld = (torch.zeros((cavity.ny, cavity.nx), dtype=torch.float64, device=cavity.device)
            if cavity.params.has_logda else None)
    nbytes = lib.pm_adjoint_vjp_scratch_bytes(cavity._h)
    scratch = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=cavity.device)
    gs = (C.c_double * 2)()
    check(lib.pm_adjoint_vjp(cavity._h, C.c_void_p(lam_next.data_ptr()), C.c_void_p(lam.data_ptr()),
                             C.c_void_p(g_ld.data_ptr()) if g_ld is not None else None,
                             C.c_void_p(scratch.data_ptr()), nbytes, gs), cavity._h)
    return lam, g_ld, gs[0], gs[1]


def vjp_step_noalloc(cavity: Cavity, lam_next, lam=None, grad_logda=None):
    """``vjp_step`` through the allocation-free entry point: the library keeps
    the partial sums in its own static device array, so no scratch buffer is
    passed (and none is allocated if ``lam`` and ``grad_logda`` are given)."""
    if lam is None:
        lam = torch.empty_like(lam_next)
    if grad_logda is None and cavity.params.has_logda:
        grad_logda = torch.zeros((cavity.ny, cavity.nx), dtype=torch.float64, device=cavity.device)
    gs = (C.c_double * 2)()
    check(lib.pm_adjoint_vjp_noalloc(cavity._h, C.c_void_p(lam_next.data_ptr()), C.c_void_p(lam.data_ptr()),
                                     C.c_void_p(grad_logda.data_ptr()) if grad_logda is not None else None,
                                     gs), cavity._h)
    return lam, grad_logda, gs[0], gs[1]
