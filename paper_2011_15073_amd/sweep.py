"""Batched parameter sweep (pm_sweep_* of the C ABI) and its schedule tuner.

A sweep advances many independent cavities together -- e.g. the (n, Da, Ra)
grid of the paper's parametric study with uneven grid sides -- with one
launch per time step over all live cases and one HIP-graph replay per chunk
of steps plus the per-case stopping test.  Each case ends bitwise equal to
the same case run alone with ``Cavity.run_to_steady``.

The tuner times every tile order (PM_ORDER_*) with every tile shape (tile_w
columns by tile_h rows per workgroup) on a scratch sweep of the same case set
and caches the fastest in a JSON file keyed by the device and the case shapes
(``$PMLBM_TUNE_CACHE``, default ``~/.cache/pmlbm/sweep.json``).  Results do
not depend on the schedule: every choice gives bitwise the same cases.
"""
import ctypes as C
import hashlib
import json
import os

import torch

from . import _lib
from ._lib import check, lib
from .cavity import _TORCH_DT

ORDERS = {"case": _lib.PM_ORDER_CASE, "largest": _lib.PM_ORDER_LARGEST,
          "interleave": _lib.PM_ORDER_INTERLEAVE}
# tile shapes (columns, rows) the sweep kernels take
TILES = [(256, 1), (128, 2), (64, 4), (128, 1), (64, 2), (64, 1)]


class _CaseView:
    """Read-only view of one case of a sweep (a borrowed pm_ctx)."""

    def __init__(self, sweep, i):
        self._sweep = sweep
        h = C.c_void_p()
        sweep._check(lib.pm_sweep_case(sweep._h, i, C.byref(h)))
        self._h = h
        p = sweep.params[i]
        self.nx, self.ny, self.device = p.nx, p.ny, sweep.device
        self.lattice = _lib.lattice_of(p)

    def _c(self, rc):
        return check(rc, self._h)

    def fields(self, dtype=torch.float64):
        code = _lib.PM_FP64 if dtype == torch.float64 else _lib.PM_FP32
        out = [torch.empty((self.ny, self.nx), dtype=_TORCH_DT[code], device=self.device)
               for _ in range(3)]
        self._c(lib.pm_fields(self._h, *(C.c_void_p(t.data_ptr()) for t in out), code))
        return tuple(out)

    def nu(self):
        v = C.c_double()
        self._c(lib.pm_nu(self._h, C.byref(v)))
        return v.value

    def populations(self, dtype=torch.float32):
        code = _lib.PM_FP64 if dtype == torch.float64 else _lib.PM_FP32
        f = torch.empty((9, self.ny, self.nx), dtype=_TORCH_DT[code], device=self.device)
        g = torch.empty((5, self.ny, self.nx), dtype=_TORCH_DT[code], device=self.device)
        self._c(lib.pm_get_populations(self._h, C.c_void_p(f.data_ptr()),
                                       C.c_void_p(g.data_ptr()), code))
        return f, g

    @property
    def steps(self):
        v = C.c_int64()
        self._c(lib.pm_steps_done(self._h, C.byref(v)))
        return v.value


class Sweep:
    """``cases``: list of dicts of ``make_params`` keywords, each with ``nx``
    (and optionally ``ny``)."""

    def __init__(self, cases, *, device="cuda:0", order="case", tile=(256, 1)):
        self.device = torch.device(device)
        n = len(cases)
        arr = (_lib.PmParams * n)()
        for i, kw in enumerate(cases):
            kw = dict(kw)
            nx = kw.pop("nx")
            ny = kw.pop("ny", None)
            arr[i] = _lib.make_params(nx, ny, **kw)
        self.params = arr
        self.ncases = n
        nb = C.c_size_t()
        check(lib.pm_sweep_workspace_bytes(arr, n, C.byref(nb)))
        align = 1 << 21
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nb.value + align, dtype=torch.uint8, device=self.device)
            base = (self.ws.data_ptr() + align - 1) // align * align
            self.stream = torch.cuda.current_stream(self.device)
            h = C.c_void_p()
            check(lib.pm_sweep_create(arr, n, C.c_void_p(base), nb, C.c_void_p(self.stream.cuda_stream),
                                      C.byref(h)))
        self._h = h
        self.set_order(order)
        self.set_tile(*tile)

    def _check(self, rc):
        return check(rc, self._h, lib.pm_sweep_last_error)

    def set_order(self, order):
        self.order = order
        self._check(lib.pm_sweep_set_order(self._h, ORDERS[order]))

    def set_tile(self, tile_w, tile_h=1):
        self.tile = (int(tile_w), int(tile_h))
        self._check(lib.pm_sweep_set_tile(self._h, int(tile_w), int(tile_h)))

    def step(self, k):
        self._check(lib.pm_sweep_step(self._h, int(k)))

    def run(self, tol=1e-8, check_every=1000, max_steps=10_000_000, progress=None,
            chunks_per_call=50):
        """Run every case to its stopping test; ``progress(nlive, steps)`` is
        called every ``chunks_per_call`` chunks.  Returns (steps, residuals)."""
        steps = (C.c_int64 * self.ncases)()
        res = (C.c_double * self.ncases)()
        nlive = C.c_int(1)
        while nlive.value:
            self._check(lib.pm_sweep_advance(self._h, float(tol), int(check_every), int(max_steps),
                                             int(chunks_per_call), C.byref(nlive)))
            if progress is not None:
                lib.pm_sweep_status(self._h, steps, res)
                progress(nlive.value, list(steps))
        self._check(lib.pm_sweep_status(self._h, steps, res))
        return list(steps), list(res)

    def case(self, i):
        return _CaseView(self, i)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.pm_sweep_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _cache_path():
    return os.environ.get("PMLBM_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pmlbm", "sweep.json"))


def _key(cases, device):
    name = torch.cuda.get_device_properties(device).name
    shapes = sorted((c["nx"], c.get("ny", c["nx"]), c.get("dtype", "fp32"), float(c.get("n", 1.0)) != 1.0)
                    for c in cases)
    return name + ":" + hashlib.sha256(repr(shapes).encode()).hexdigest()[:16]


def tune(cases, *, device="cuda:0", steps=200, use_cache=True):
    """Fastest schedule for this case set: cached, else timed on a scratch
    sweep (``steps`` steps per tile order and tile shape, after a warm-up).
    Returns ({"order": ..., "tile": (tile_w, tile_h)}, {"order WxH": us/step})."""
    key = _key(cases, torch.device(device))
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        hit = cache.get(key)
        if hit and "tile" in hit:
            return {"order": hit["order"], "tile": tuple(hit["tile"])}, hit["us_per_step"]
    scratch = Sweep(cases, device=device)
    times, best, best_t = {}, None, float("inf")
    for tile in TILES:
        scratch.set_tile(*tile)
        for name in ORDERS:
            scratch.set_order(name)
            scratch.step(20)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(scratch.stream)
            scratch.step(steps)
            e1.record(scratch.stream)
            e1.synchronize()
            t = e0.elapsed_time(e1) * 1e3 / steps
            times[f"{name} {tile[0]}x{tile[1]}"] = t
            if t < best_t:
                best, best_t = {"order": name, "tile": tile}, t
    scratch.close()
    del scratch
    if use_cache:
        cache[key] = {"order": best["order"], "tile": list(best["tile"]), "us_per_step": times}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return best, times
