"""The oracle's steady-state loop (orc_run_to_steady) against its definition.

The 256 x 256 power-law cavity is run "until max |dT| per 1000 steps
< 1e-8".  The loop: take a snapshot of T at the start; advance in chunks of
check_every steps (the last chunk shortened so that no more than max_steps
are taken); after each chunk r = max over nodes of |T - snapshot| and the
snapshot becomes T; stop at the first chunk with r < tol, or with a NaN
anywhere (reported as r = NaN), or at max_steps.  Recomputed here from
single steps and the oracle's temperature field, so an off-by-one chunk, a
snapshot taken at the wrong time or a wrong cap would fail.
"""
import math

import numpy as np
import pytest

import oracle as O

PHYS = dict(n=0.8, Da=1e-2, Ra=1e4, Pr=10.0, eps=0.6)


def reference_loop(orc, tol, check_every, max_steps):
    prev = orc.macros()["T"]
    done, r = 0, math.inf
    while done < max_steps:
        k = min(check_every, max_steps - done)
        orc.step(k)
        done += k
        cur = orc.macros()["T"]
        d = np.abs(cur - prev)
        r = math.nan if np.isnan(d).any() else float(d.max())
        prev = cur
        if r < tol or math.isnan(r):
            break
    return r, done


@pytest.mark.parametrize("check_every,max_steps", [(40, 2000), (40, 1000), (35, 150)])
def test_run_to_steady_stops_at_first_check_below_tol(check_every, max_steps):
    N = 12
    a = O.Oracle.from_physics(O.physics(N, **PHYS))
    b = O.Oracle.from_physics(O.physics(N, **PHYS))
    # a tolerance the residual crosses at the sixth check (rs[i]: check i + 1)
    probe = O.Oracle.from_physics(O.physics(N, **PHYS))
    rs = [reference_loop(probe, -1.0, check_every, check_every)[0] for _ in range(12)]
    tol = math.sqrt(rs[4] * rs[5])
    r_ref, s_ref = reference_loop(a, tol, check_every, max_steps)
    r, s = b.run_to_steady(tol=tol, check_every=check_every, max_steps=max_steps)
    assert (r, s) == (r_ref, s_ref)
    if max_steps >= 6 * check_every:
        assert s == 6 * check_every and r < tol          # stopped by the tolerance
    else:
        assert s == max_steps                            # stopped by the cap (here not a multiple of the chunk)
    fa, ga = a.state()
    fb, gb = b.state()
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb)


def test_run_to_steady_in_slices_stops_at_the_same_step():
    """Calls of a multiple of check_every steps each continue the same loop:
    every call takes its first snapshot where the previous one took its last."""
    N, check = 12, 40
    one = O.Oracle.from_physics(O.physics(N, **PHYS))
    probe = O.Oracle.from_physics(O.physics(N, **PHYS))
    rs = [reference_loop(probe, -1.0, check, check)[0] for _ in range(12)]
    tol = math.sqrt(rs[6] * rs[7])
    r1, s1 = one.run_to_steady(tol=tol, check_every=check, max_steps=10 ** 6)
    sliced = O.Oracle.from_physics(O.physics(N, **PHYS))
    total, r = 0, math.inf
    while True:
        r, done = sliced.run_to_steady(tol=tol, check_every=check, max_steps=3 * check)
        total += done
        if r < tol or done < 3 * check:
            break
    assert (r, total) == (r1, s1) == (r1, 8 * check)


def test_run_to_steady_reports_nan():
    N = 8
    o = O.Oracle.from_physics(O.physics(N, **PHYS))
    f, g = o.state()
    g[0, 3, 4] = np.nan
    o.set_state(f, g)
    r, s = o.run_to_steady(tol=1e-8, check_every=10, max_steps=1000)
    assert math.isnan(r) and s == 10
