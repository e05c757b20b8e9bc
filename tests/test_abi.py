"""CPU-side checks of the C ABI: the shared library loads, exports every
symbol include/pmlbm.h declares, validates parameters, and its host-side
parameter mapping agrees with the oracle's independent implementation of the
same mapping.  No GPU calls."""
import math
import os
import re

import pytest

import oracle as O
import paper_2011_15073_amd as P
from paper_2011_15073_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "pmlbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(_lib.lib, s), f"{s} declared in pmlbm.h but not exported"
    assert sorted(_lib.EXPORTS) == syms


def test_params_struct_layout_matches_header():
    # the ctypes mirror must have the same field order as the C struct
    text = open(os.path.join(ROOT, "include", "pmlbm.h")).read()
    body = text[text.index("typedef struct {\n  int32_t nx, ny;"):text.index("} pm_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl or decl.startswith("typedef"):
            decl = decl.split("{", 1)[-1].strip()
        if not decl:
            continue
        parts = decl.split(None, 1)
        names += [n.strip() for n in parts[1].split(",")]
    assert names == [f for f, _ in _lib.PmParams._fields_]


@pytest.mark.parametrize("case", [
    dict(N=64, n=1.0, Da=0.1, Ra=1e3, Pr=10.0, eps=0.6),
    dict(N=256, n=0.6, Da=1e-3, Ra=1e5, Pr=10.0, eps=0.6),
    dict(N=4096, n=0.8, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6),
    dict(N=160, n=1.4, Da=math.inf, Ra=1e5, Pr=100.0, eps=1.0, forchheimer=0),
    dict(N=48, n=0.7, Da=1e-2, Ra=1e4, Pr=6.2, eps=0.6, clamp_mode=1, nu_lo=0.01, nu_hi=1e6),
])
def test_host_mapping_matches_oracle(case):
    case = dict(case)
    N = case.pop("N")
    p = P.make_params(N, **case)
    L = P.lattice_of(p)
    o = O.map_physics(O.physics(N, **case))
    for k in ("U_lb", "nu0", "nu_min", "nu_max", "gamma_scale", "eps", "Feps", "gbeta",
              "alpha", "s_e", "s_eps", "s_q", "sT_e", "sT_nu"):
        a, b = getattr(L, k), getattr(o, k)
        assert a == pytest.approx(b, rel=1e-14, abs=0.0), k
    assert (math.isinf(L.K) and math.isinf(o.K)) or L.K == pytest.approx(o.K, rel=1e-15)
    assert L.tau_g == pytest.approx(3 * o.alpha + 0.5, rel=1e-15)


@pytest.mark.parametrize("bad", [
    dict(nx=1), dict(eps=0.0), dict(eps=1.2), dict(n=0.0), dict(Ra=-1.0), dict(Da=0.0),
    dict(mach=0.0), dict(nu_lo=2.0), dict(nu_lo=0.5, nu_hi=0.4), dict(dtype=7),
    dict(s_q=2.5), dict(rounding=3), dict(rounding=1, dtype=1),
])
def test_invalid_parameters_are_rejected(bad):
    p = P.make_params(32)
    for k, v in bad.items():
        setattr(p, k, v)
    with pytest.raises(P.PmError) as e:
        P.lattice_of(p)
    assert e.value.code == _lib.PM_EINVAL
    assert _lib.lib.pm_last_error(None).decode()


def test_workspace_size_covers_planes():
    p = P.make_params(4096, 4096, dtype="fp32")
    assert P.workspace_bytes(p) >= 15 * 4096 * 4096 * 4
    p64 = P.make_params(33, 17, dtype="fp64", has_logda=1)
    assert P.workspace_bytes(p64) >= 16 * 33 * 17 * 8
    assert P.workspace_bytes(p64) % 256 == 0


def test_strerror_codes():
    for code in (0, -1, -2, -3, -4):
        assert _lib.lib.pm_strerror(code)


def test_step_kernel_choice():
    """PM_STEP_PAIR needs FP32 and cavity walls on both axes; the automatic
    choice takes the two-step kernel (and its second population region) only
    on grids large enough to fill the GPU."""
    kw = dict(n=1.0, Da=0.1, Ra=1e3, Pr=10.0, eps=0.6)
    with pytest.raises(P.PmError):
        P.workspace_bytes(P.make_params(64, dtype="fp64", step_kernel="pair", **kw))
    with pytest.raises(P.PmError):
        P.workspace_bytes(P.make_params(64, dtype="fp32", step_kernel="pair", periodic_x=1, **kw))
    auto = P.workspace_bytes(P.make_params(256, dtype="fp32", **kw))
    single = P.workspace_bytes(P.make_params(256, dtype="fp32", step_kernel="single", **kw))
    pair = P.workspace_bytes(P.make_params(256, dtype="fp32", step_kernel="pair", **kw))
    assert auto == single < pair
    # the two-step kernel's row groups are a launch's y dimension (<= 65535)
    tall = dict(nx=300, ny=24 * 65535 + 1, dtype="fp32", **kw)
    with pytest.raises(P.PmError):
        P.workspace_bytes(P.make_params(step_kernel="pair", **tall))
    assert P.workspace_bytes(P.make_params(**tall)) == P.workspace_bytes(P.make_params(step_kernel="single", **tall))
    big_auto = P.workspace_bytes(P.make_params(4096, dtype="fp32", **kw))
    big_single = P.workspace_bytes(P.make_params(4096, dtype="fp32", step_kernel="single", **kw))
    assert big_auto >= big_single + 14 * 4096 * 4096 * 4


def _sweep_ws(cases):
    """pm_sweep_workspace_bytes on a list of pm_params: (status, bytes)."""
    import ctypes as C
    arr = (_lib.PmParams * max(1, len(cases)))(*cases)
    nb = C.c_size_t(0)
    return _lib.lib.pm_sweep_workspace_bytes(arr, len(cases), C.byref(nb)), nb.value


def test_sweep_case_lists_are_validated():
    """The sweep's host checks (no device needed): 1..4096 cases, one dtype
    for all, no per-cell log-Da planes, every case valid on its own; the
    workspace holds every case's own workspace."""
    kw = dict(n=0.8, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.6)
    a = P.make_params(128, dtype="fp64", **kw)
    b = P.make_params(200, 96, dtype="fp64", **kw)
    rc, one = _sweep_ws([a])
    assert rc == 0 and one >= P.workspace_bytes(a)
    rc, two = _sweep_ws([a, b])
    assert rc == 0 and two >= P.workspace_bytes(a) + P.workspace_bytes(b) and two > one
    assert _sweep_ws([])[0] == _lib.PM_EINVAL
    assert _sweep_ws([a] * 4097)[0] == _lib.PM_EINVAL
    assert _sweep_ws([a, P.make_params(64, dtype="fp32", **kw)])[0] == _lib.PM_EINVAL
    assert _sweep_ws([a, P.make_params(64, dtype="fp64", has_logda=1, **kw)])[0] == _lib.PM_EINVAL
    bad = P.make_params(64, dtype="fp64", **kw)
    bad.eps = 0.0
    assert _sweep_ws([a, bad])[0] == _lib.PM_EINVAL
    assert _lib.lib.pm_last_error(None).decode()


def test_adjoint_workspace_checks():
    """pm_adjoint_workspace_bytes (no device needed): the workspace holds
    ceil(T / C) state checkpoints, the replay slots and two FP64 adjoint
    states; T >= 1, 1 <= C <= T, cavity walls, the nu clamp and no extra body
    force are required."""
    import ctypes as C

    def ws(p, T, Cc):
        nb = C.c_size_t(0)
        return _lib.lib.pm_adjoint_workspace_bytes(C.byref(p), T, Cc, C.byref(nb)), nb.value

    kw = dict(n=0.8, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.6, dtype="fp32", has_logda=1)
    p = P.make_params(48, 40, **kw)
    rc, nb = ws(p, 100, 10)
    assert rc == 0 and nb >= 2 * 14 * 48 * 40 * 8 + 10 * 14 * 48 * 40 * 4
    assert ws(p, 100, 10)[1] < ws(p, 100, 1)[1]  # 100 checkpoints against 10
    for T, Cc in ((0, 1), (10, 0), (10, 11)):
        assert ws(p, T, Cc)[0] == _lib.PM_EINVAL
    for bad in (dict(periodic_x=1), dict(clamp_mode=1), dict(gx=1e-6), dict(dtype="fp16")):
        assert ws(P.make_params(48, 40, **dict(kw, **bad)), 100, 10)[0] == _lib.PM_EINVAL
    assert _lib.lib.pm_last_error(None).decode()
    # the adjoint's setters reject a missing adjoint before touching anything
    assert _lib.lib.pm_adjoint_set_lambda_dtype(None, _lib.PM_FP32) == _lib.PM_EINVAL
    assert _lib.lib.pm_adjoint_set_shear_floor(None, 0.1) == _lib.PM_EINVAL


def test_fp16_storage_parameters():
    """PM_FP16: half the population bytes of FP32, FP32 per-cell planes, the
    single-step kernel only (PM_STEP_PAIR refused, PM_STEP_AUTO takes no second
    region), stochastic or nearest rounding, not in a sweep."""
    kw = dict(n=0.8, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6)
    n = 4096 * 4096
    f16 = P.workspace_bytes(P.make_params(4096, dtype="fp16", **kw))
    f32 = P.workspace_bytes(P.make_params(4096, dtype="fp32", step_kernel="single", **kw))
    assert 14 * n * 2 <= f16 < f32 and f32 - f16 >= 14 * n * 2
    assert P.workspace_bytes(P.make_params(4096, dtype="fp16", step_kernel="single", **kw)) == f16
    with pytest.raises(P.PmError):
        P.workspace_bytes(P.make_params(4096, dtype="fp16", step_kernel="pair", **kw))
    for r in ("auto", "stochastic", "nearest"):
        P.lattice_of(P.make_params(64, dtype="fp16", rounding=r, **kw))
    assert _sweep_ws([P.make_params(64, dtype="fp16", **kw)])[0] == _lib.PM_EINVAL
    assert "FP16" in _lib.lib.pm_last_error(None).decode()
