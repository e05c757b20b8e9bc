"""GPU: the allocation-free adjoint step (pm_adjoint_vjp_noalloc) against the
scratch-buffer one (pm_adjoint_vjp), both called through the C ABI: the
adjoint state, the log-Da gradient and dL/dn, dL/dRa must be bitwise equal.
Two calls in a row share the library's static scratch, the second on a
smaller grid (its partials must not see the first call's); a grid whose
workgroups exceed the static array is rejected before any launch."""
import numpy as np
import pytest
import torch

import paper_2011_15073_amd as P
from paper_2011_15073_amd import inputs
from paper_2011_15073_amd.adjoint import vjp_step_noalloc

pytestmark = pytest.mark.gpu

PHYS = dict(Pr=10.0, eps=0.6, Ra=1e4)


def one_case(nx, ny, n, dtype, pre_steps, seed):
    f0, g0 = inputs.random_state(nx, ny, seed=seed, amp=0.03, amp_T=0.2)
    ld = inputs.logda_field(max(nx, ny), seed=seed + 1)[:ny, :nx].copy()
    lam_next = torch.from_numpy(np.random.default_rng(seed + 2).standard_normal((14, ny, nx))).cuda()
    cav = P.Cavity(nx, ny, dtype=dtype, logda=torch.from_numpy(ld), n=n, **PHYS)
    cav.set_populations(torch.from_numpy(f0), torch.from_numpy(g0))
    cav.step(pre_steps)
    ref = P.vjp_step(cav, lam_next)
    got = vjp_step_noalloc(cav, lam_next)
    torch.cuda.synchronize()
    print(f"{nx}x{ny} n={n} {dtype} pre={pre_steps}: dn {got[2]:.6e} / {ref[2]:.6e}, "
          f"dRa {got[3]:.6e} / {ref[3]:.6e}", flush=True)
    assert torch.equal(got[0], ref[0])
    assert torch.equal(got[1], ref[1])
    assert got[2] == ref[2] and got[3] == ref[3]
    assert torch.isfinite(got[0]).all() and abs(got[2]) > 0


@pytest.mark.parametrize("n,dtype", [(0.7, "fp64"), (1.4, "fp32")])
def test_noalloc_vjp_equals_scratch_vjp_twice(n, dtype):
    one_case(300, 41, n, dtype, pre_steps=1, seed=11)   # 2 x 41 workgroups
    one_case(21, 13, n, dtype, pre_steps=0, seed=23)    # then a smaller grid


def test_noalloc_vjp_rejects_grids_beyond_the_static_scratch():
    # ceil(257 / 256) * 32769 = 65538 workgroups > 65536: rejected before any launch
    cav = P.Cavity(257, 32769, dtype="fp32", n=1.0, **PHYS)
    dummy = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    with pytest.raises(P.PmError, match="static scratch"):
        vjp_step_noalloc(cav, dummy, lam=dummy)
