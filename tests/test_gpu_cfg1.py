"""GPU: the 256 x 256 power-law porous cavity run to steady state against the
stored FP64 oracle result (tests/golden/cfg1_256_oracle.npz, written by
tests/golden/make_cfg1_golden.py, which calls only the oracle).

Workload: n = 0.6 with the viscosity clamped to [0.1, 10] nu0, Da = 1e-3,
Ra = 1e5, Pr = 10, eps = 0.6, from rest, stopped at the first 1000-step
check with max |dT| < 1e-8 (the oracle stops at S* = 331 000)."""
import os

import numpy as np
import pytest
import torch

import paper_2011_15073_amd as P
from paper_2011_15073_amd import inputs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
PHYS = dict(n=0.6, Da=1e-3, Ra=1e5, Pr=10.0, eps=0.6, nu_lo=0.1, nu_hi=10.0)
N = 256


@pytest.fixture(scope="module")
def gold():
    return dict(np.load(os.path.join(HERE, "golden", "cfg1_256_oracle.npz")))


def errors(cav, g):
    """Max error over every node relative to the oracle's full-field
    maxima, per field; Nu."""
    U, V, T = (t.cpu().numpy() for t in cav.fields(torch.float64))
    out = {}
    for name, a, ref, scale in (("U", U, "U", "maxU"), ("V", V, "V", "maxV"), ("theta", T, "T", "maxT")):
        out[name] = float(np.abs(a - g[ref]).max() / g[scale])
    out["Nu"] = abs(cav.nu() - float(g["nu_bar"])) / float(g["nu_bar"])
    return out


def all_nodes(cav):
    return [t.cpu().numpy() for t in cav.fields(torch.float64)], cav.nu()


@pytest.fixture(scope="module")
def fp64_runs(gold):
    """The FP64 run to steady state, and the same physics from a rest state
    perturbed by 6e-8 relative, stepped to the same step count: how well the
    stopping state itself is determined (the run stops while the slow mode
    still drifts ~1e-8 per 1000 steps)."""
    cav = P.Cavity(N, dtype="fp64", **PHYS)
    r, steps = cav.run_to_steady(tol=1e-8, check_every=1000, max_steps=2_000_000)
    pert = P.Cavity(N, dtype="fp64", **PHYS)
    f0, g0 = inputs.random_state(N, N, seed=5, amp=6e-8, T0=0.5, amp_T=3e-8)
    pert.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
    pert.step(steps)
    (a, nu_a), (b, nu_b) = all_nodes(cav), all_nodes(pert)
    scales = (float(gold["maxU"]), float(gold["maxV"]), float(gold["maxT"]))
    spread = max([float(np.abs(x - y).max()) / sc for x, y, sc in zip(a, b, scales)] + [abs(nu_a - nu_b) / nu_a])
    return cav, r, steps, spread


def test_fp64_stops_at_the_oracle_step_with_the_oracle_state(gold, fp64_runs):
    """Same stopping step as the oracle; state within 1e-11, or within three
    times the FP64 run's own spread under a 6e-8 initial perturbation where
    that is larger (after 331 000 steps the stopping state is determined to
    ~1e-9 only)."""
    cav, r, steps, spread = fp64_runs
    e = errors(cav, gold)
    print(f"FP64: {steps} steps (oracle {int(gold['steps'])}), r {r:.4e} (oracle {float(gold['residual']):.4e}), "
          f"errors {e}, own spread {spread:.2e}", flush=True)
    assert steps == int(gold["steps"])
    assert r == pytest.approx(float(gold["residual"]), rel=1e-2)
    assert max(e.values()) <= max(1e-11, 3 * spread)


def test_fp32_at_the_oracle_step(gold):
    """FP32 storage and arithmetic with round-to-nearest updates
    (PM_ROUND_NEAREST), run for exactly S* steps (the FP64 stopping step).
    Measured: U 4.8e-4, V 2.0e-4, theta 2.4e-4, Nu 2.4e-4 -- above the 1e-4
    FP32 bar: near the steady flow the same state rounds the same way every
    step and the slowly decaying low-shear power-law mode sums that fixed
    pattern into a bias (FP64 arithmetic on FP32-rounded populations gives
    3.2e-4).  Bounded here at 1e-3 as a regression check; the default
    stochastic rounding below meets the bar."""
    cav = P.Cavity(N, dtype="fp32", rounding="nearest", **PHYS)
    cav.step(int(gold["steps"]))
    e32 = errors(cav, gold)
    print(f"FP32 round-to-nearest at S*: {e32}", flush=True)
    assert max(e32.values()) <= 1e-3


def test_fp32_stochastic_rounding_meets_the_bar(gold):
    """FP32 storage and arithmetic with the default rounding (PM_ROUND_AUTO:
    stochastically rounded population updates with FP32 storage), run for
    exactly S* steps: the bias that round-to-nearest storage accumulates in
    the slow modes is gone, and every field and Nu meet the 1e-4 FP32 bar."""
    cav = P.Cavity(N, dtype="fp32", **PHYS)
    assert cav.params.rounding == 2
    cav.step(int(gold["steps"]))
    e = errors(cav, gold)
    print(f"FP32 stochastic rounding (default) at S*: {e}", flush=True)
    assert max(e.values()) <= 1e-4
