"""GPU: the batched parameter sweep against the same cases run alone.

Each case of a sweep must stop at the same step and end bitwise equal to the
single-case run (same kernel body, same arithmetic), whatever the tile
schedule; one case of the sweep is also checked against the oracle."""
import numpy as np
import pytest
import torch

import paper_2011_15073_amd as P
from pairs import compare_fields, oracle_for

pytestmark = pytest.mark.gpu

CASES = [
    dict(nx=40, n=0.6, Da=1e-3, Ra=1e4, Pr=10.0, eps=0.6),
    dict(nx=64, n=1.0, Da=1e-2, Ra=1e3, Pr=10.0, eps=0.6),
    dict(nx=96, ny=70, n=0.8, Da=1e-1, Ra=1e4, Pr=10.0, eps=0.6),
    dict(nx=33, n=0.8, Da=1e-2, Ra=1e5, Pr=10.0, eps=0.6),
    dict(nx=130, n=1.0, Da=1e-3, Ra=1e4, Pr=10.0, eps=0.6),
    dict(nx=72, n=0.6, Da=1e-1, Ra=1e3, Pr=10.0, eps=0.6),
]
TOL, CHECK, CAP = 1e-5, 500, 12000


def run_alone(kw, dtype):
    kw = dict(kw)
    nx = kw.pop("nx")
    ny = kw.pop("ny", None)
    c = P.Cavity(nx, ny, dtype=dtype, **kw)
    r, steps = c.run_to_steady(tol=TOL, check_every=CHECK, max_steps=CAP)
    return c, steps, r


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
@pytest.mark.parametrize("order", ["case", "largest", "interleave"])
def test_sweep_equals_cases_run_alone(dtype, order):
    cases = [dict(c, dtype=dtype) for c in CASES]
    sw = P.Sweep(cases, order=order)
    steps, res = sw.run(tol=TOL, check_every=CHECK, max_steps=CAP)
    print("sweep steps", steps, flush=True)
    for i, kw in enumerate(CASES):
        alone, s_alone, r_alone = run_alone(kw, dtype)
        assert steps[i] == s_alone, (i, steps[i], s_alone)
        assert res[i] == r_alone
        view = sw.case(i)
        assert view.steps == s_alone
        dt = torch.float64 if dtype == "fp64" else torch.float32
        fa, ga = alone.populations(dt)
        fb, gb = view.populations(dt)
        assert torch.equal(fa, fb) and torch.equal(ga, gb), i
        assert view.nu() == alone.nu()


def test_sweep_stops_cases_at_their_own_steps():
    cases = [dict(c, dtype="fp32") for c in CASES]
    sw = P.Sweep(cases)
    steps, res = sw.run(tol=1e-3, check_every=CHECK, max_steps=CAP)
    for s, r in zip(steps, res):
        assert s % CHECK == 0 and 0 < s <= CAP
        assert r < 1e-3 or s == CAP
    # a second run continues nothing: every case has stopped
    steps2, _ = sw.run(tol=1e-3, check_every=CHECK, max_steps=CAP)
    assert steps2 == steps


def test_sweep_case_matches_oracle():
    """A well-conditioned case (tau >= 0.6 everywhere) of a two-case FP64
    sweep against the oracle after 1500 steps."""
    good = dict(nx=48, n=0.8, Da=1e-2, Ra=1e3, Pr=6.2, eps=0.6, nu_lo=0.5, nu_hi=2.0)
    sw = P.Sweep([dict(good, dtype="fp64"), dict(CASES[1], dtype="fp64")])
    sw.step(1500)
    view = sw.case(0)
    phys = {k: v for k, v in good.items() if k not in ("nx", "ny")}
    orc = oracle_for(good["nx"], **phys).step(1500)
    Ug, Vg, Tg = (t.cpu().numpy() for t in view.fields())
    Ur, Vr, Tr = orc.fields()
    for a, b in ((Ug, Ur), (Vg, Vr), (Tg, Tr)):
        assert np.abs(a - b).max() / np.abs(b).max() <= 1e-11
    assert abs(view.nu() - orc.nu_bar()) / orc.nu_bar() <= 1e-11


def test_tuner_returns_a_valid_order(tmp_path, monkeypatch):
    monkeypatch.setenv("PMLBM_TUNE_CACHE", str(tmp_path / "tune.json"))
    cases = [dict(c, dtype="fp32") for c in CASES]
    order, times = P.tune(cases, steps=50)
    assert order in ("case", "largest", "interleave")
    assert all(t > 0 for t in times.values())
    order2, _ = P.tune(cases, steps=50)  # served from the cache
    assert order2 == order
