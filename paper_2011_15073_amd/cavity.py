"""Python front end of the C ABI: a cavity simulation whose device memory and
stream come from PyTorch.

torch is used only for memory and streams: the workspace is a uint8 tensor,
outputs are tensors allocated here, and the library enqueues on the current
torch stream of the device.  All arithmetic runs in the library's kernels.
"""
import ctypes as C

import torch

from . import _lib
from ._lib import PM_FP32, PM_FP64, check, lib

_TORCH_DT = {PM_FP32: torch.float32, PM_FP64: torch.float64}


def _dt_code(dtype):
    if dtype in (torch.float32, "fp32", PM_FP32):
        return PM_FP32
    if dtype in (torch.float64, "fp64", PM_FP64):
        return PM_FP64
    raise ValueError(f"unsupported dtype {dtype}")


class Cavity:
    """One simulation context (``pm_init`` ... ``pm_destroy``).

    Parameters follow ``pm_params`` (pmlbm.h); ``dtype`` is ``"fp32"``,
    ``"fp64"`` or ``"fp16"`` (half-precision population storage with FP32
    arithmetic; fields and populations are still returned as FP32/FP64).  The context is bound to ``torch.cuda.current_stream(device)``
    at construction time.
    """

    def __init__(self, nx, ny=None, *, device="cuda:0", logda=None, **kw):
        if not torch.cuda.is_available():
            raise RuntimeError("Cavity needs a ROCm GPU (torch.cuda.is_available() is False)")
        if logda is not None:
            kw["has_logda"] = 1
        self.params = _lib.make_params(nx, ny, **kw)
        self.lattice = _lib.lattice_of(self.params)
        self.device = torch.device(device)
        self.nx, self.ny = self.params.nx, self.params.ny
        self.dtype_code = self.params.dtype
        nbytes = _lib.workspace_bytes(self.params)
        with torch.cuda.device(self.device):
            # 2 MiB-aligned base: the population region starts on a large-page
            # boundary (measured ~3% faster at 4096^2 than 256 B alignment)
            align = 1 << 21
            self.ws = torch.empty(nbytes + align, dtype=torch.uint8, device=self.device)
            self._base = (self.ws.data_ptr() + align - 1) // align * align
            self.stream = torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            check(lib.pm_init(C.byref(self.params), C.c_void_p(self._base), C.c_size_t(nbytes),
                              C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self._nbytes = nbytes
        if logda is not None:
            self.set_logda(logda)

    # -- lifetime --
    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.pm_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        return check(rc, self._h)

    # -- stepping --
    def step(self, k: int = 1):
        self._check(lib.pm_step(self._h, int(k)))
        return self

    @property
    def steps(self) -> int:
        v = C.c_int64()
        self._check(lib.pm_steps_done(self._h, C.byref(v)))
        return v.value

    def nu(self) -> float:
        v = C.c_double()
        self._check(lib.pm_nu(self._h, C.byref(v)))
        return v.value

    def residual(self, with_step=False):
        """max |theta - theta_snapshot| since the last call (then snapshot :=
        theta); with_step: also the step count at which it was taken."""
        v, at = C.c_double(), C.c_int64()
        self._check(lib.pm_residual(self._h, C.byref(v), C.byref(at)))
        return (v.value, at.value) if with_step else v.value

    def run_to_steady(self, tol=1e-8, check_every=1000, max_steps=10_000_000, history=None):
        """Advance until the residual taken every check_every steps is below
        tol, or max_steps steps; returns (last residual, steps taken).  With
        ``history`` (a list), the same chunks and stopping rule are driven
        from here and (step count, residual, Nu) is appended after every
        check: the residual and Nu histories of the run."""
        if history is not None and check_every > 0 and max_steps >= 0:
            done, r = 0, float("inf")
            while done < max_steps:
                k = min(int(check_every), int(max_steps) - done)
                self.step(k)
                done += k
                r, at = self.residual(with_step=True)
                history.append((at, r, self.nu()))
                if r < tol:
                    break
            return r, done
        steps, r = C.c_int64(), C.c_double()
        self._check(lib.pm_run_to_steady(self._h, float(tol), int(check_every), int(max_steps),
                                         C.byref(steps), C.byref(r)))
        return r.value, steps.value

    # -- fields and state --
    def fields(self, dtype=torch.float64):
        """Nondimensional (U, V, theta), each a [ny, nx] tensor."""
        code = _dt_code(dtype)
        out = [torch.empty((self.ny, self.nx), dtype=_TORCH_DT[code], device=self.device)
               for _ in range(3)]
        self._check(lib.pm_fields(self._h, *(C.c_void_p(t.data_ptr()) for t in out), code))
        return tuple(out)

    def stream_function(self, dtype=torch.float64, out=None):
        """Nondimensional stream function psi [ny, nx] (psi = 0 on the bottom
        wall; U = d psi / dY, V = -d psi / dX), into ``out`` if given (a
        contiguous [ny, nx] tensor of this device, float32 or float64)."""
        if out is None:
            code = _dt_code(dtype)
            out = torch.empty((self.ny, self.nx), dtype=_TORCH_DT[code], device=self.device)
        else:
            code = _dt_code(out.dtype)
            assert out.is_contiguous() and tuple(out.shape) == (self.ny, self.nx) and out.device == self.device
        self._check(lib.pm_stream_function(self._h, C.c_void_p(out.data_ptr()), code))
        return out

    def viscosity(self, dtype=torch.float64):
        code = _dt_code(dtype)
        out = torch.empty((self.ny, self.nx), dtype=_TORCH_DT[code], device=self.device)
        self._check(lib.pm_viscosity(self._h, C.c_void_p(out.data_ptr()), code))
        return out

    def populations(self, dtype=torch.float64):
        code = _dt_code(dtype)
        f = torch.empty((9, self.ny, self.nx), dtype=_TORCH_DT[code], device=self.device)
        g = torch.empty((5, self.ny, self.nx), dtype=_TORCH_DT[code], device=self.device)
        self._check(lib.pm_get_populations(self._h, C.c_void_p(f.data_ptr()),
                                           C.c_void_p(g.data_ptr()), code))
        return f, g

    def set_populations(self, f, g):
        f = torch.as_tensor(f, device=self.device).contiguous()
        g = torch.as_tensor(g, device=self.device).contiguous()
        if f.dtype != g.dtype:
            g = g.to(f.dtype)
        assert f.numel() == 9 * self.nx * self.ny and g.numel() == 5 * self.nx * self.ny
        self._keep = (f, g)
        self._check(lib.pm_set_populations(self._h, C.c_void_p(f.data_ptr()),
                                           C.c_void_p(g.data_ptr()), _dt_code(f.dtype)))

    def set_logda(self, logda):
        t = torch.as_tensor(logda, device=self.device).contiguous()
        assert t.numel() == self.nx * self.ny
        self._logda = t
        self._check(lib.pm_set_logda(self._h, C.c_void_p(t.data_ptr()), _dt_code(t.dtype)))

    def state_bytes(self) -> int:
        n = C.c_size_t()
        self._check(lib.pm_state_bytes(self._h, C.byref(n)))
        return n.value

    def save_state(self):
        buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        self._check(lib.pm_save_state(self._h, C.c_void_p(buf.data_ptr()), buf.numel()))
        return buf

    def load_state(self, buf):
        self._check(lib.pm_load_state(self._h, C.c_void_p(buf.data_ptr()), buf.numel()))


def copy_probe(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """Streaming copy kernel of the library (read + write bandwidth probe)."""
    nbytes = min(src.numel() * src.element_size(), dst.numel() * dst.element_size())
    nbytes -= nbytes % 16
    s = stream or torch.cuda.current_stream(src.device)
    check(lib.pm_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                            C.c_size_t(nbytes), C.c_void_p(s.cuda_stream)))
