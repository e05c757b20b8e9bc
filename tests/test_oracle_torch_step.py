"""CPU: the differentiable torch re-implementation of the update (the adjoint's
autograd reference) pinned to the C oracle, and its autograd gradients pinned
to finite differences of itself."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import torch_step as TS
from paper_2011_15073_amd import inputs

PHYS = dict(Pr=10.0, eps=0.6)


@pytest.mark.parametrize("n", [0.7, 1.0, 1.4])
def test_one_step_matches_c_oracle(n):
    nx, ny, Ra = 21, 13, 1e4
    f0, g0 = inputs.random_state(nx, ny, seed=7, amp=0.03, amp_T=0.2)
    ld = inputs.logda_field(max(nx, ny), seed=3)[:ny, :nx].copy()
    orc = O.Oracle.from_physics(O.physics(nx, ny, n=n, Ra=Ra, **PHYS), logda=ld)
    orc.set_state(f0, g0)
    orc.step(1)
    fr, gr = orc.state()
    Pm = TS.Params(nx, ny, n=n, Ra=Ra, **PHYS)
    f, g = TS.step(Pm, torch.from_numpy(f0), torch.from_numpy(g0), torch.from_numpy(ld))
    assert np.abs(f.numpy() - fr).max() <= 1e-14
    assert np.abs(g.numpy() - gr).max() <= 1e-14


def test_trajectory_from_rest_matches_c_oracle():
    N, T, n, Ra = 12, 30, 0.7, 1e4
    ld = inputs.logda_field(N, seed=5)
    orc = O.Oracle.from_physics(O.physics(N, n=n, Ra=Ra, **PHYS), logda=ld)
    orc.step(T)
    Pm = TS.Params(N, N, n=n, Ra=Ra, **PHYS)
    f, g = TS.rest_state(Pm)
    for _ in range(T):
        f, g = TS.step(Pm, f, g, torch.from_numpy(ld))
    fr, gr = orc.state()
    assert np.abs(f.numpy() - fr).max() <= 1e-13
    assert np.abs(g.numpy() - gr).max() <= 1e-13
    assert TS.nu_bar(Pm, g).item() == pytest.approx(orc.nu_bar(), rel=1e-12)


def test_autograd_matches_central_differences():
    """Gradient of a few-step Nu_bar with respect to the log10 Da field, n and
    Ra, from a random (unclamped-viscosity) state, against central
    differences of the same function (torch.autograd.gradcheck)."""
    nx, ny, steps = 6, 5, 3
    f0, g0 = inputs.random_state(nx, ny, seed=2, amp=0.03, amp_T=0.2)
    ld0 = inputs.logda_field(max(nx, ny), seed=4)[:ny, :nx].copy()

    def J(ld, n, Ra):
        Pm = TS.Params(nx, ny, n=n, Ra=Ra, **PHYS)
        f, g = torch.from_numpy(f0), torch.from_numpy(g0)
        for _ in range(steps):
            f, g = TS.step(Pm, f, g, ld)
        return TS.nu_bar(Pm, g)

    args = (torch.tensor(ld0, requires_grad=True), torch.tensor(0.8, dtype=torch.float64, requires_grad=True),
            torch.tensor(1e4, dtype=torch.float64, requires_grad=True))
    assert torch.autograd.gradcheck(J, args, eps=1e-6, atol=1e-8, rtol=1e-5)
